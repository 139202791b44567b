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
// sweep, not the matrix: at step s wavefront g writes its H rows as H
// contiguous 64-lane runs, Z[((s*G + g)*H + h)*64 + l], so every store is one
// coalesced 256-byte line.  k_backtrack reads that layout through zindex();
// k_row_major rewrites it as the row-major matrix when the caller asks for it.
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
    return ((s * g.G + wave) * g.H + h) * 64 + lane;
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

    float x[H], O[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int r = rbase + h;
        x[h] = r < na ? a[r] : 0.0f;  // rows past na never feed a row below na
        O[h] = kInf;
    }
    if constexpr (G > 1) {
        for (int k = threadIdx.x; k < (G - 1) * kPRing; k += 64 * G) ring[k / kPRing][k % kPRing] = kInf;
        __syncthreads();
    }
    float up_in = kInf;
    float diag_in = (lane == 0 && wave == 0) ? 0.0f : kInf;  // c(0,0) of the 1-based recurrence
    float *__restrict__ zw = Z + (int64_t)wave * H * 64 + lane;
    const int64_t zstep = (int64_t)G * H * 64;

    for (int s = 0; s < geo.steps; ++s) {
        const int c = s - skew;
        // columns before 0 only ever see +inf neighbours; columns past nb are
        // never read back and never feed a column below nb
        const float yv = b[c < 0 ? 0 : (c >= nb ? nb - 1 : c)];
        float diag = diag_in, up = up_in;
        const int off = rbase - c;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            float xe = x[h];
            if constexpr (BANDED) xe = (unsigned)(off + h + band) > (unsigned)(2 * band) ? kBig : xe;
            const float d = xe - yv;
            const float v = fmaf(d, d, min3f(diag, up, O[h]));
            diag = O[h];
            up = v;
            O[h] = v;
            zw[h * 64] = v;
        }
        zw += zstep;
        const float bottom = O[H - 1];
        float fill = kInf;
        if constexpr (G > 1) {
            if (lane == 63 && wave < G - 1) ring[wave][c & (kPRing - 1)] = bottom;
            // lane 0's up neighbour for step s+1: column s+1 - wave(64+kLag) of the
            // wavefront above, written by it kLag steps ago (a barrier lies between)
            if (wave > 0) fill = ring[wave - 1][(s + 1 - wave * (64 + kLag)) & (kPRing - 1)];
        }
        const float recv = lane_shift_down(bottom, fill);
        diag_in = up_in;
        up_in = recv;
        if constexpr (G > 1) {
            if ((s + 1) % kLag == 0) __syncthreads();
        }
    }
}

// One wavefront walks back from (n-1, m-1) to (0, 0): from each cell to the
// predecessor with the smallest cumulative cost, ties in the order diagonal,
// (i-1, j), (i, j-1).  The walk runs on 64x64 tiles of C staged in LDS with
// the current cell at the tile's bottom-right corner; every tile allows at
// least 63 steps.  Lane 0 walks and writes the path backwards; the wavefront
// then reverses it in place.
__global__ __launch_bounds__(64) void k_backtrack(const float *__restrict__ Z, const PathGeom geo, int n, int m,
                                                  int *__restrict__ path, int64_t *__restrict__ out_len,
                                                  float *__restrict__ out_cost) {
    __shared__ float tile[64][65];
    __shared__ int64_t st[3];
    const int lane = threadIdx.x;
    int i = n - 1, j = m - 1;
    int64_t k = 1;
    if (lane == 0) {
        path[0] = i;
        path[1] = j;
    }
    while (i > 0 || j > 0) {
        const int i0 = i - 63, j0 = j - 63;
        for (int q = 0; q < 64; ++q) tile[lane][q] = cell_at(Z, geo, i0 + lane, j0 + q);
        __syncthreads();
        if (lane == 0) {
            int ta = 63, tb = 63;
            while (ta > 0 && tb > 0 && (i > 0 || j > 0)) {
                const float d = tile[ta - 1][tb - 1], u = tile[ta - 1][tb], l = tile[ta][tb - 1];
                // on the first row or column only one predecessor exists (the
                // others are the +inf border); taking it outright keeps the walk
                // inside the matrix even when costs overflow or are NaN
                if (i == 0) {
                    --tb;
                } else if (j == 0) {
                    --ta;
                } else if (d <= u && d <= l) {
                    --ta;
                    --tb;
                } else if (u <= l) {
                    --ta;
                } else {
                    --tb;
                }
                i = i0 + ta;
                j = j0 + tb;
                path[2 * k] = i;
                path[2 * k + 1] = j;
                ++k;
            }
            st[0] = i;
            st[1] = j;
            st[2] = k;
        }
        __syncthreads();
        i = static_cast<int>(st[0]);
        j = static_cast<int>(st[1]);
        k = st[2];
        __syncthreads();  // st is read by every lane before lane 0 writes it again
    }
    for (int64_t p = lane; p < k / 2; p += 64) {
        const int64_t q = k - 1 - p;
        const int pi = path[2 * p], pj = path[2 * p + 1];
        const int qi = path[2 * q], qj = path[2 * q + 1];
        path[2 * p] = qi;
        path[2 * p + 1] = qj;
        path[2 * q] = pi;
        path[2 * q + 1] = pj;
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
