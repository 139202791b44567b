// Optimal warping path of one pair (paper, "Mathematical background" and
// Fig. 1: the cumulative-cost matrix of Eq. (c) and the path of matched
// cells through it from (1,1) to (n,m)).  The distance matrix never needs
// the whole matrix; the path of a chosen pair does.
//
// k_cost_matrix sweeps the pair like the wavefront strip kernels -- one
// workgroup of G wavefronts, lane l of wavefront g owning rows
// [(64g+l)H, (64g+l)H+H) of the shorter series, column s - l - g(64+kLag) at
// step s, the strip's bottom cell passed down by DPP and between wavefronts
// through an LDS ring -- and stores, for every cell, either its cost or the
// move the walk back takes from it.  The store layout follows the sweep, not
// the matrix: at step s wavefront g writes one contiguous block per lane,
// lane l's H values at ((s*G + g)*64 + l)*H + h (costs, 16-byte vector
// stores) or its H 2-bit moves in ceil(H/16) words at ((s*G + g)*64 + l)*W2
// + h/16 (moves).  When the caller asks for the cost matrix the sweep stores
// costs, k_backtrack decides the moves from them and k_row_major rewrites
// them row-major; otherwise it stores the moves (2 bits a cell, a sixteenth
// of the memory) and k_backtrack_moves follows them.
#include "dtw_device.h"
#include "dtwmi.h"

#include <cstdio>
#include <mutex>

namespace dtwmi {
namespace {

constexpr int kLag = 16;   // steps each wavefront trails the one above; also the barrier period
constexpr int kPRing = 64; // LDS ring slots per wavefront boundary

// Geometry of the sweep and of its buffer Z.
struct PathGeom {
    int H, G, logH;  // rows per lane (a power of two), wavefronts
    int na, nb;      // rows spread over the lanes (shorter series) and columns (longer one)
    int steps;       // steps of the sweep: nb + 63 + (G-1)(64+kLag)
    int swap;        // 1: the sweep rows are the columns j of C (x is the longer series)
};

__device__ __forceinline__ int64_t zindex(const PathGeom &g, int r, int c) {
    const int L = r >> g.logH, h = r & (g.H - 1);
    const int wave = L >> 6, lane = L & 63;
    const int64_t s = (int64_t)c + lane + wave * (64 + kLag);
    return ((s * g.G + wave) * 64 + lane) * g.H + h;
}

// Word and bit offset of the 2-bit move of sweep cell (r, c) (W2 words per
// lane and step).
__device__ __forceinline__ int64_t mindex(const PathGeom &g, int r, int c) {
    const int L = r >> g.logH, h = r & (g.H - 1);
    const int wave = L >> 6, lane = L & 63;
    const int64_t s = (int64_t)c + lane + wave * (64 + kLag);
    const int W2 = (g.H + 15) >> 4;
    return ((s * g.G + wave) * 64 + lane) * W2 + (h >> 4);
}
__device__ __forceinline__ int mshift(const PathGeom &g, int r) { return 2 * (r & (g.H - 1) & 15); }

// c(i+1, j+1) of Eq. (c) for 0-based (i, j) in the caller's orientation (i
// over x, j over y), +inf for i < 0 or j < 0 (the border of the recurrence).
__device__ __forceinline__ float cell_at(const float *__restrict__ Z, const PathGeom &g, int i, int j) {
    if (i < 0 || j < 0) return kInf;
    return Z[g.swap ? zindex(g, j, i) : zindex(g, i, j)];
}

// The walk's move out of a cell in the caller's orientation: 3 to (i-1, j-1),
// 1 to (i-1, j), 2 to (i, j-1) -- the predecessor of smallest cumulative cost,
// ties in that order.
__device__ __forceinline__ unsigned move_code(float diag, float cu, float cl) {
    return (diag <= cu && diag <= cl) ? 3u : (cu <= cl ? 1u : 2u);
}

// MODE 0: store costs in Z.  MODE 1, 2: store the 2-bit moves in M (1: the
// sweep rows are the caller's i, 2: they are its j) and c(n, m) in *cost.
template <int H, int G, bool BANDED, int MODE>
__global__ __launch_bounds__(64 * G) void k_cost_matrix(const float *__restrict__ a, const float *__restrict__ b,
                                                        const PathGeom geo, int band, float *__restrict__ Z,
                                                        unsigned *__restrict__ M, float *__restrict__ cost) {
    constexpr int W2 = (H + 15) / 16;  // move words per lane and step
    __shared__ float ring[G > 1 ? G - 1 : 1][kPRing];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int na = geo.na, nb = geo.nb;
    const int rbase = (wave * 64 + lane) * H;
    const int skew = lane + wave * (64 + kLag);  // column = s - skew
    const int col0 = -wave * (64 + kLag);        // column of lane 0 at step 0

    float x[H], A[H], B[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int r = rbase + h;
        x[h] = r < na ? a[r] : 0.0f;  // rows past na never feed a row below na
        A[h] = kInf;
    }
    if constexpr (G > 1) {
        for (int k = threadIdx.x; k < (G - 1) * kPRing; k += 64 * G) ring[k / kPRing][k % kPRing] = kInf;
        __syncthreads();
    }
    // y travels down the lanes with the anti-diagonal: lane l at step s uses
    // the y lane l-1 used at step s-1, and lane 0 takes y[s + col0] from a
    // 64-value block loaded one block ahead (lane q holds y[s0 + q + col0]).
    // Columns outside 0..nb-1 read the nearest end value: cells of columns
    // before 0 see only +inf neighbours, cells past nb-1 are never read back
    // and never feed a column below nb.
    auto yblock = [&](int s0) {
        const int c = s0 + lane + col0;
        return b[c < 0 ? 0 : (c >= nb ? nb - 1 : c)];
    };
    float ynext = yblock(0), yv = 0.0f;
    float up_in = kInf;
    float diag_in = (lane == 0 && wave == 0) ? 0.0f : kInf;  // c(0,0) of the 1-based recurrence
    // sweep-order store: lane-major within a step, H contiguous floats (or
    // W2 move words) per lane
    float *__restrict__ zl = MODE == 0 ? Z + ((int64_t)wave * 64 + lane) * H : nullptr;
    const int64_t zstep = (int64_t)G * 64 * H;
    unsigned *__restrict__ ml = MODE != 0 ? M + ((int64_t)wave * 64 + lane) * W2 : nullptr;
    const int64_t mstep = (int64_t)G * 64 * W2;
    const int rlast = geo.na - 1 - rbase;  // the row of c(n, m) in this lane (if 0 <= rlast < H)

    // One step: column s - skew of this lane's H rows, from the previous
    // column Oi into Oo (two steps per iteration ping-pong the arrays).
    auto step = [&](int s, float ycur, int qs, const float (&Oi)[H], float (&Oo)[H]) {
        // lane 0's up neighbour for step s+1: column s+1 - wave(64+kLag) of
        // the wavefront above, written by it at the end of step s+1-kLag (a
        // barrier lies between); read early so the LDS latency overlaps the step
        float fill = kInf;
        if constexpr (G > 1) {
            if (wave > 0) fill = ring[wave - 1][(s + 1 - wave * (64 + kLag)) & (kPRing - 1)];
        }
        yv = lane_shift_down(yv, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ycur), qs)));
        const int c = s - skew;
        float diag = diag_in, up = up_in;
        const int off = rbase - c;
        unsigned mw[W2];
#pragma unroll
        for (int k = 0; k < W2; ++k) mw[k] = 0u;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            float xe = x[h];
            if constexpr (BANDED) xe = (unsigned)(off + h + band) > (unsigned)(2 * band) ? kBig : xe;
            const float d = xe - yv;
            const float mn = min3f(diag, up, Oi[h]);
            const float v = fmaf(d, d, mn);
            // the move from the minimum already at hand: the diagonal if it is
            // the minimum, else (i-1, j) if that is, else (i, j-1) -- the order
            // of move_code's ties
            if constexpr (MODE == 1) mw[h / 16] |= (mn == diag ? 3u : (mn == up ? 1u : 2u)) << (2 * (h % 16));
            if constexpr (MODE == 2) mw[h / 16] |= (mn == diag ? 3u : (mn == Oi[h] ? 1u : 2u)) << (2 * (h % 16));
            diag = Oi[h];
            up = v;
            Oo[h] = v;
        }
        if constexpr (MODE == 0) {
            if constexpr (H % 4 == 0) {
#pragma unroll
                for (int h = 0; h < H; h += 4)
                    *reinterpret_cast<float4 *>(zl + h) = make_float4(Oo[h], Oo[h + 1], Oo[h + 2], Oo[h + 3]);
            } else {
#pragma unroll
                for (int h = 0; h < H; ++h) zl[h] = Oo[h];
            }
            zl += zstep;
        } else {
            if constexpr (W2 == 1) {
                ml[0] = mw[0];
            } else if constexpr (W2 == 2) {
                *reinterpret_cast<uint2 *>(ml) = make_uint2(mw[0], mw[1]);
            } else {
#pragma unroll
                for (int k = 0; k < W2; k += 4)
                    *reinterpret_cast<uint4 *>(ml + k) = make_uint4(mw[k], mw[k + 1], mw[k + 2], mw[k + 3]);
            }
            ml += mstep;
            if (c == geo.nb - 1 && static_cast<unsigned>(rlast) < static_cast<unsigned>(H)) {
                float v = Oo[0];
#pragma unroll
                for (int h = 1; h < H; ++h) v = rlast == h ? Oo[h] : v;
                *cost = v;
            }
        }
        const float bottom = Oo[H - 1];
        if constexpr (G > 1) {
            if (lane == 63 && wave < G - 1) ring[wave][c & (kPRing - 1)] = bottom;
        }
        const float recv = lane_shift_down(bottom, fill);
        diag_in = up_in;
        up_in = recv;
        if constexpr (G > 1) {
            if ((s + 1) % kLag == 0) __syncthreads();
        }
    };

    // Blocks of 64 steps: the y block is consumed in registers while the next
    // one loads (a value loaded in the inner loop would make every step wait
    // for all earlier stores, which share the vector memory counter).
    for (int s0 = 0; s0 < geo.steps; s0 += 64) {
        const float ycur = ynext;
        ynext = yblock(s0 + 64);
        const int s1 = s0 + 64 < geo.steps ? s0 + 64 : geo.steps;
        int s = s0;
        for (; s + 1 < s1; s += 2) {
            step(s, ycur, s - s0, A, B);
            step(s + 1, ycur, s + 1 - s0, B, A);
        }
        if (s < s1) {  // odd step count: only in the last block
            step(s, ycur, s - s0, A, B);
#pragma unroll
            for (int h = 0; h < H; ++h) A[h] = B[h];
        }
    }
}

// One wavefront walks back from (n-1, m-1) to (0, 0): from each cell to the
// predecessor with the smallest cumulative cost, ties in the order diagonal,
// (i-1, j), (i, j-1); on the first row or column only one predecessor exists
// (the others are the +inf border) and the walk takes it outright, which also
// keeps it inside the matrix when costs overflow or are NaN.
//
// The walk runs on 64x64 tiles of C with the current cell at the bottom-right
// corner; each tile allows at least 63 moves.  Lane t loads tile row t (64
// independent loads in flight) and the wavefront decides every cell's move in
// parallel (the row above arrives by DPP): 2 bits per cell, bit 0 "row - 1",
// bit 1 "column - 1", 0 where the walk must leave the tile (its first row or
// column, where the move would need cells outside it) or has reached the
// origin; 16 cells per register, 4 registers per lane.  A move is then a
// register-indexed read, a lane read and a few scalar operations, no memory
// access.  Lane (k mod 64) of two registers keeps the k-th cell of the path;
// every 64 cells the wavefront stores them with one write.  The path is
// produced backwards and reversed in place at the end.
typedef unsigned MoveWords __attribute__((ext_vector_type(16)));  // register-indexed reads need >= 16 elements

// The walk itself: tile_moves(i0, j0, mw) fills the moves of the tile with
// bottom-right corner (i0+63, j0+63) (row i0 + lane in each lane); returns
// the path length.
template <class TileMoves>
__device__ __forceinline__ int64_t walk_back(int n, int m, int *__restrict__ path, TileMoves tile_moves) {
    const int lane = threadIdx.x;
    int i = n - 1, j = m - 1;  // current cell (wave-uniform)
    int pi = i, pj = j;        // lane kk holds cell kbase + kk until the flush
    int64_t kbase = 0;
    int kk = 1;
    while (i > 0 || j > 0) {
        const int i0 = i - 63, j0 = j - 63;
        MoveWords mw = {};
        tile_moves(i0, j0, mw);
        int ta = 63, tb = 63;
        for (;;) {
            const unsigned word = mw[tb >> 4];
            const unsigned code =
                (static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(word), ta)) >> (2 * (tb & 15))) & 3u;
            if (code == 0u) break;
            ta -= static_cast<int>(code & 1u);
            tb -= static_cast<int>(code >> 1);
            const bool mine = lane == kk;
            pi = mine ? i0 + ta : pi;
            pj = mine ? j0 + tb : pj;
            if (++kk == 64) {
                path[2 * (kbase + lane)] = pi;
                path[2 * (kbase + lane) + 1] = pj;
                kbase += 64;
                kk = 0;
            }
        }
        i = i0 + ta;
        j = j0 + tb;
    }
    if (lane < kk) {
        path[2 * (kbase + lane)] = pi;
        path[2 * (kbase + lane) + 1] = pj;
    }
    const int64_t k = kbase + kk;
    __syncthreads();  // the stores above are visible to every lane of the workgroup
    for (int64_t p = lane; p < k / 2; p += 64) {
        const int64_t q = k - 1 - p;
        const int a0 = path[2 * p], a1 = path[2 * p + 1];
        const int b0 = path[2 * q], b1 = path[2 * q + 1];
        path[2 * p] = b0;
        path[2 * p + 1] = b1;
        path[2 * q] = a0;
        path[2 * q + 1] = a1;
    }
    return k;
}

// A move with the walk's edge rules: on C's first row only (i, j-1) and on
// its first column only (i-1, j) exist (the others are the +inf border; the
// rule also keeps the walk inside the matrix when costs overflow or are NaN);
// 0 (leave the tile) on the tile's first row and at the origin.
__device__ __forceinline__ unsigned edge_rules(unsigned code, int r, int jc) {
    code = r == 0 ? (jc == 0 ? 0u : 2u) : (jc == 0 ? 1u : code);
    return threadIdx.x == 0 ? 0u : code;
}

// Walk from stored costs: the wavefront decides every cell's move of the tile
// in parallel (the row above arrives by DPP).
__global__ __launch_bounds__(64) void k_backtrack(const float *__restrict__ Z, const PathGeom geo, int n, int m,
                                                  int *__restrict__ path, int64_t *__restrict__ out_len,
                                                  float *__restrict__ out_cost) {
    const int lane = threadIdx.x;
    const int64_t k = walk_back(n, m, path, [&](int i0, int j0, MoveWords &mw) {
        const int r = i0 + lane;
        const int rc = r < 0 ? 0 : r;
        // zindex(rr, cc) = zindex(rr, 0) + cc*S: a per-lane base plus a
        // wave-uniform offset per tile column, whichever series the rows are
        const int64_t S = (int64_t)geo.G * 64 * geo.H;
        const float *__restrict__ zr = Z + (geo.swap ? rc * S : zindex(geo, rc, 0));
        float v[64];
        if (geo.swap) {
#pragma unroll
            for (int q = 0; q < 64; ++q) v[q] = zr[zindex(geo, j0 + q < 0 ? 0 : j0 + q, 0)];
        } else {
#pragma unroll
            for (int q = 0; q < 64; ++q) v[q] = zr[(j0 + q < 0 ? 0 : j0 + q) * S];
        }
#pragma unroll
        for (int q = 0; q < 64; ++q) v[q] = (r < 0 || j0 + q < 0) ? kInf : v[q];
        float diag = lane_shift_down(v[0], kInf);
#pragma unroll
        for (int q = 1; q < 64; ++q) {
            const float up = lane_shift_down(v[q], kInf), left = v[q - 1];
            mw[q >> 4] |= edge_rules(move_code(diag, up, left), r, j0 + q) << (2 * (q & 15));
            diag = up;
        }
    });
    if (lane == 0) {
        *out_len = k;
        *out_cost = cell_at(Z, geo, n - 1, m - 1);
    }
}

// Walk from the moves the sweep stored (2 bits per cell in its layout).
__global__ __launch_bounds__(64) void k_backtrack_moves(const unsigned *__restrict__ M, const PathGeom geo, int n,
                                                        int m, int *__restrict__ path, int64_t *__restrict__ out_len) {
    const int lane = threadIdx.x;
    const int64_t k = walk_back(n, m, path, [&](int i0, int j0, MoveWords &mw) {
        const int r = i0 + lane;
        const int rc = r < 0 ? 0 : r;
        // mindex(rr, cc) = mindex(rr, 0) + cc*S2, as for the costs
        const int64_t S2 = (int64_t)geo.G * 64 * ((geo.H + 15) >> 4);
        unsigned w[64];
        if (geo.swap) {  // caller row i0 + lane is sweep column rc; column j0 + q is sweep row j0 + q
#pragma unroll
            for (int q = 0; q < 64; ++q) {
                const int rr = j0 + q < 0 ? 0 : j0 + q;
                w[q] = M[mindex(geo, rr, 0) + rc * S2] >> mshift(geo, rr);
            }
        } else {
            const unsigned *__restrict__ mr = M + mindex(geo, rc, 0);
            const int sh = mshift(geo, rc);
#pragma unroll
            for (int q = 0; q < 64; ++q) w[q] = mr[(j0 + q < 0 ? 0 : j0 + q) * S2] >> sh;
        }
#pragma unroll
        for (int q = 1; q < 64; ++q) mw[q >> 4] |= edge_rules(w[q] & 3u, r, j0 + q) << (2 * (q & 15));
    });
    if (lane == 0) *out_len = k;
}

// C[i*m + j] = c(i+1, j+1): one thread per element, stores coalesced.
__global__ __launch_bounds__(256) void k_row_major(const float *__restrict__ Z, const PathGeom geo, int n, int m,
                                                   float *__restrict__ C) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)n * m) return;
    const int i = static_cast<int>(e / m), j = static_cast<int>(e - (int64_t)i * m);
    C[e] = cell_at(Z, geo, i, j);
}

template <int H, int G, int MODE>
void launch_cost_mode(bool banded, const float *a, const float *b, const PathGeom &g, int band, float *Z,
                      unsigned *M, float *cost, hipStream_t s) {
    if (banded)
        hipLaunchKernelGGL((k_cost_matrix<H, G, true, MODE>), dim3(1), dim3(64 * G), 0, s, a, b, g, band, Z, M, cost);
    else
        hipLaunchKernelGGL((k_cost_matrix<H, G, false, MODE>), dim3(1), dim3(64 * G), 0, s, a, b, g, band, Z, M,
                           cost);
}

// Z != nullptr: store costs; else the moves into M and c(n, m) into *cost.
template <int H, int G>
void launch_cost_matrix(bool banded, const float *a, const float *b, const PathGeom &g, int band, float *Z,
                        unsigned *M, float *cost, hipStream_t s) {
    if (Z)
        launch_cost_mode<H, G, 0>(banded, a, b, g, band, Z, M, cost, s);
    else if (g.swap)
        launch_cost_mode<H, G, 2>(banded, a, b, g, band, Z, M, cost, s);
    else
        launch_cost_mode<H, G, 1>(banded, a, b, g, band, Z, M, cost, s);
}

using CostFn = void (*)(bool, const float *, const float *, const PathGeom &, int, float *, unsigned *, float *,
                        hipStream_t);
struct PathShape {
    int H, G;
    CostFn fn;
};
// In increasing row capacity 64*H*G; wide pairs use up to 8 wavefronts (two per SIMD).
const PathShape kPathShapes[] = {
    {1, 1, &launch_cost_matrix<1, 1>},   {2, 1, &launch_cost_matrix<2, 1>},   {4, 1, &launch_cost_matrix<4, 1>},
    {8, 1, &launch_cost_matrix<8, 1>},   {8, 2, &launch_cost_matrix<8, 2>},   {8, 4, &launch_cost_matrix<8, 4>},
    {8, 8, &launch_cost_matrix<8, 8>},   {16, 8, &launch_cost_matrix<16, 8>}, {32, 8, &launch_cost_matrix<32, 8>},
    {64, 8, &launch_cost_matrix<64, 8>},
};
constexpr int kPathMaxRows = 64 * 64 * 8;

int path_err(int code, const char *msg, hipError_t e = hipSuccess) {
    char buf[256];
    if (e != hipSuccess)
        snprintf(buf, sizeof buf, "dtw_path: %s: %s", msg, hipGetErrorString(e));
    else
        snprintf(buf, sizeof buf, "dtw_path: %s", msg);
    return set_error(code, buf);
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

// Move buffers kept between calls, one per device, grown to the largest pair
// so far up to kPathKeepBytes (larger ones are allocated for the call and
// freed); a call holds the lock of the cache until its stream has finished.
constexpr size_t kPathKeepBytes = size_t(1) << 30;
constexpr int kPathDevices = 64;
struct PathCache {
    std::mutex lock;
    void *p[kPathDevices] = {};
    size_t bytes[kPathDevices] = {};
};
PathCache &path_cache() {
    static PathCache c;
    return c;
}

}  // namespace
}  // namespace dtwmi

using namespace dtwmi;

extern "C" int dtw_path(const float *x, int32_t n, const float *y, int32_t m, int32_t window, int32_t *path,
                        int64_t *path_len, float *cost, float *C, void *stream) {
    clear_error();
    if (!x || !y || !path || !path_len || !cost) return path_err(DTW_ERR_INVALID_ARG, "x, y, path, path_len or cost is NULL");
    if (n < 1 || m < 1) return path_err(DTW_ERR_INVALID_ARG, "series lengths must be >= 1");
    PathGeom g{};
    g.swap = n > m;
    g.na = g.swap ? m : n;
    g.nb = g.swap ? n : m;
    if (g.na > kPathMaxRows) return path_err(DTW_ERR_UNSUPPORTED, "the shorter series has more than 32768 points");
    const PathShape *shape = nullptr;
    for (const PathShape &p : kPathShapes)
        if (64 * p.H * p.G >= g.na) {
            shape = &p;
            break;
        }
    g.H = shape->H;
    g.G = shape->G;
    g.logH = __builtin_ctz(static_cast<unsigned>(g.H));
    const int64_t steps = (int64_t)g.nb + 63 + (int64_t)(g.G - 1) * (64 + kLag);
    if (steps > INT32_MAX) return path_err(DTW_ERR_UNSUPPORTED, "series too long");
    g.steps = static_cast<int>(steps);
    const int diff = g.nb - g.na;
    const int band = window < 0 ? -1 : (window > diff ? window : diff);
    const bool banded = band >= 0 && band < g.nb - 1;  // a wider band admits every cell
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (!C) {
        // moves only: 2 bits a cell in a kept buffer, the length and cost after them
        const size_t mbytes = ((size_t)steps * g.G * 64 * ((g.H + 15) / 16) * sizeof(unsigned) + 255) / 256 * 256;
        const size_t need = mbytes + 256;
        int dev = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return path_err(DTW_ERR_HIP, "hipGetDevice", e);
        if (dev < 0 || dev >= kPathDevices) return path_err(DTW_ERR_UNSUPPORTED, "device index out of range");
        PathCache &pc = path_cache();
        std::lock_guard<std::mutex> guard(pc.lock);
        DevBuf once;
        char *buf = nullptr;
        if (need > kPathKeepBytes) {
            if ((e = hipMalloc(&once.p, need)) != hipSuccess)
                return path_err(DTW_ERR_OUT_OF_MEMORY, "move buffer allocation", e);
            buf = static_cast<char *>(once.p);
        } else {
            if (pc.bytes[dev] < need) {
                if (pc.p[dev]) (void)hipFree(pc.p[dev]);  // the previous call's stream has finished
                pc.p[dev] = nullptr;
                pc.bytes[dev] = 0;
                if ((e = hipMalloc(&pc.p[dev], need)) != hipSuccess)
                    return path_err(DTW_ERR_OUT_OF_MEMORY, "move buffer allocation", e);
                pc.bytes[dev] = need;
            }
            buf = static_cast<char *>(pc.p[dev]);
        }
        unsigned *M = reinterpret_cast<unsigned *>(buf);
        int64_t *d_len = reinterpret_cast<int64_t *>(buf + mbytes);
        float *d_cost = reinterpret_cast<float *>(buf + mbytes + 64);
        // on a failure after a launch, wait for the stream before the buffer is released
        auto failed = [&](const char *what) {
            const int rc = path_err(DTW_ERR_HIP, what, e);
            (void)hipStreamSynchronize(s);
            return rc;
        };
        shape->fn(banded, g.swap ? y : x, g.swap ? x : y, g, band, nullptr, M, d_cost, s);
        if ((e = hipGetLastError()) != hipSuccess) return failed("cost-matrix kernel launch");
        hipLaunchKernelGGL(k_backtrack_moves, dim3(1), dim3(64), 0, s, M, g, n, m, path, d_len);
        if ((e = hipGetLastError()) != hipSuccess) return failed("backtrack kernel launch");
        e = hipMemcpyAsync(path_len, d_len, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(cost, d_cost, sizeof(float), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return failed("path result");
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return path_err(DTW_ERR_HIP, "path result", e);
        return DTW_OK;
    }

    // the cost matrix asked for: keep every cell's cost, decide the moves from them
    const int64_t zbytes = steps * g.G * g.H * 64 * (int64_t)sizeof(float);
    DevBuf z, small;
    e = hipMalloc(&z.p, static_cast<size_t>(zbytes));
    if (e != hipSuccess) return path_err(DTW_ERR_OUT_OF_MEMORY, "cost matrix allocation", e);
    if ((e = hipMalloc(&small.p, 256)) != hipSuccess) return path_err(DTW_ERR_OUT_OF_MEMORY, "allocation", e);
    float *Z = static_cast<float *>(z.p);
    int64_t *d_len = static_cast<int64_t *>(small.p);
    float *d_cost = reinterpret_cast<float *>(static_cast<char *>(small.p) + 64);

    shape->fn(banded, g.swap ? y : x, g.swap ? x : y, g, band, Z, nullptr, nullptr, s);
    if ((e = hipGetLastError()) != hipSuccess) return path_err(DTW_ERR_HIP, "cost-matrix kernel launch", e);
    hipLaunchKernelGGL(k_backtrack, dim3(1), dim3(64), 0, s, Z, g, n, m, path, d_len, d_cost);
    if ((e = hipGetLastError()) != hipSuccess) return path_err(DTW_ERR_HIP, "backtrack kernel launch", e);
    {
        const int64_t blocks = ((int64_t)n * m + 255) / 256;
        if (blocks > INT32_MAX) return path_err(DTW_ERR_UNSUPPORTED, "cost matrix too large for C");
        hipLaunchKernelGGL(k_row_major, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, Z, g, n, m, C);
        if ((e = hipGetLastError()) != hipSuccess) return path_err(DTW_ERR_HIP, "row-major kernel launch", e);
    }
    e = hipMemcpyAsync(path_len, d_len, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(cost, d_cost, sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return path_err(DTW_ERR_HIP, "path result", e);
    return DTW_OK;
}
