// Optimal warping path of one pair (paper, "Mathematical background" and
// Fig. 1: the cumulative-cost matrix of Eq. (c) and the path of matched
// cells through it from (1,1) to (n,m)).  The distance matrix never needs
// the whole matrix; the path of a chosen pair does.
//
// k_cost_matrix sweeps the pair like the wavefront strip kernels -- one
// workgroup of G wavefronts, lane l of wavefront g owning rows
// [(64g+l)H, (64g+l)H+H) of the shorter series, column s - l - g(64+kLag) at
// step s, the strip's bottom cell passed down by DPP and between wavefronts
// through an LDS ring -- and stores every cell.  The store layout follows the
// sweep, not the matrix: at step s wavefront g writes one contiguous block of
// 64*H floats, lane l's H cells at Z[((s*G + g)*64 + l)*H + h], as 16-byte
// vector stores.  k_backtrack reads that layout through zindex(); k_row_major
// rewrites it as the row-major matrix when the caller asks for it.
#include "dtw_device.h"
#include "dtwmi.h"

#include <cstdio>

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

// c(i+1, j+1) of Eq. (c) for 0-based (i, j) in the caller's orientation (i
// over x, j over y), +inf for i < 0 or j < 0 (the border of the recurrence).
__device__ __forceinline__ float cell_at(const float *__restrict__ Z, const PathGeom &g, int i, int j) {
    if (i < 0 || j < 0) return kInf;
    return Z[g.swap ? zindex(g, j, i) : zindex(g, i, j)];
}

template <int H, int G, bool BANDED>
__global__ __launch_bounds__(64 * G) void k_cost_matrix(const float *__restrict__ a, const float *__restrict__ b,
                                                        const PathGeom geo, int band, float *__restrict__ Z) {
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
    // sweep-order store: lane-major within a step, H contiguous floats per lane
    float *__restrict__ zl = Z + ((int64_t)wave * 64 + lane) * H;
    const int64_t zstep = (int64_t)G * 64 * H;

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
#pragma unroll
        for (int h = 0; h < H; ++h) {
            float xe = x[h];
            if constexpr (BANDED) xe = (unsigned)(off + h + band) > (unsigned)(2 * band) ? kBig : xe;
            const float d = xe - yv;
            const float v = fmaf(d, d, min3f(diag, up, Oi[h]));
            diag = Oi[h];
            up = v;
            Oo[h] = v;
        }
        if constexpr (H % 4 == 0) {
#pragma unroll
            for (int h = 0; h < H; h += 4)
                *reinterpret_cast<float4 *>(zl + h) = make_float4(Oo[h], Oo[h + 1], Oo[h + 2], Oo[h + 3]);
        } else {
#pragma unroll
            for (int h = 0; h < H; ++h) zl[h] = Oo[h];
        }
        zl += zstep;
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

__global__ __launch_bounds__(64) void k_backtrack(const float *__restrict__ Z, const PathGeom geo, int n, int m,
                                                  int *__restrict__ path, int64_t *__restrict__ out_len,
                                                  float *__restrict__ out_cost) {
    const int lane = threadIdx.x;
    int i = n - 1, j = m - 1;  // current cell (wave-uniform)
    int pi = i, pj = j;        // lane kk holds cell kbase + kk until the flush
    int64_t kbase = 0;
    int kk = 1;
    while (i > 0 || j > 0) {
        const int i0 = i - 63, j0 = j - 63;
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
        MoveWords mw = {};
        float diag = lane_shift_down(v[0], kInf);
#pragma unroll
        for (int q = 1; q < 64; ++q) {
            const float up = lane_shift_down(v[q], kInf), left = v[q - 1];
            unsigned code = (diag <= up && diag <= left) ? 3u : (up <= left ? 1u : 2u);
            code = r == 0 ? (j0 + q == 0 ? 0u : 2u) : (j0 + q == 0 ? 1u : code);  // C's first row / column
            code = lane == 0 ? 0u : code;                                         // the tile's first row
            mw[q >> 4] |= code << (2 * (q & 15));
            diag = up;
        }
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
    if (lane == 0) {
        *out_len = k;
        *out_cost = cell_at(Z, geo, n - 1, m - 1);
    }
}

// C[i*m + j] = c(i+1, j+1): one thread per element, stores coalesced.
__global__ __launch_bounds__(256) void k_row_major(const float *__restrict__ Z, const PathGeom geo, int n, int m,
                                                   float *__restrict__ C) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)n * m) return;
    const int i = static_cast<int>(e / m), j = static_cast<int>(e - (int64_t)i * m);
    C[e] = cell_at(Z, geo, i, j);
}

template <int H, int G>
void launch_cost_matrix(bool banded, const float *a, const float *b, const PathGeom &g, int band, float *Z,
                        hipStream_t s) {
    if (banded)
        hipLaunchKernelGGL((k_cost_matrix<H, G, true>), dim3(1), dim3(64 * G), 0, s, a, b, g, band, Z);
    else
        hipLaunchKernelGGL((k_cost_matrix<H, G, false>), dim3(1), dim3(64 * G), 0, s, a, b, g, band, Z);
}

using CostFn = void (*)(bool, const float *, const float *, const PathGeom &, int, float *, hipStream_t);
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
    const int64_t zbytes = steps * g.G * g.H * 64 * (int64_t)sizeof(float);

    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf z, small;
    hipError_t e = hipMalloc(&z.p, static_cast<size_t>(zbytes));
    if (e != hipSuccess) return path_err(DTW_ERR_OUT_OF_MEMORY, "cost matrix allocation", e);
    if ((e = hipMalloc(&small.p, 256)) != hipSuccess) return path_err(DTW_ERR_OUT_OF_MEMORY, "allocation", e);
    float *Z = static_cast<float *>(z.p);
    int64_t *d_len = static_cast<int64_t *>(small.p);
    float *d_cost = reinterpret_cast<float *>(static_cast<char *>(small.p) + 64);

    shape->fn(banded, g.swap ? y : x, g.swap ? x : y, g, band, Z, s);
    if ((e = hipGetLastError()) != hipSuccess) return path_err(DTW_ERR_HIP, "cost-matrix kernel launch", e);
    hipLaunchKernelGGL(k_backtrack, dim3(1), dim3(64), 0, s, Z, g, n, m, path, d_len, d_cost);
    if ((e = hipGetLastError()) != hipSuccess) return path_err(DTW_ERR_HIP, "backtrack kernel launch", e);
    if (C) {
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
