// HIP kernels (gfx950) for the all-pairs DTW distance matrix.
//
// Every kernel evaluates the recurrence of Eq. (c) of the paper
// ("Mathematical background"):
//     c(i,j) = (x_i - y_j)^2 + min{ c(i-1,j-1), c(i-1,j), c(i,j-1) }
// keeping only O(row) state in registers -- the GPU form of the paper's
// "preceding vector" scheme -- and writes c(n,m) into the condensed distance
// matrix D (same section).  The window rule |i-j| <= max(w,|n-m|) follows the
// paper's Introduction.  The recurrence is a min-plus scan, so all work is
// FP32 (or FP64) VALU: v_sub, v_min3, v_fma per cell; no matrix cores.
//
// This header: the lane-band kernel (one pair per lane, equal lengths, narrow
// band), used for datasets of equal-length series.  dtw_lane.hip instantiates
// it for plain FP32 sums and dtw_lane_rb.hip for rebased sums (two sources,
// so that the 128 instances compile in parallel).
#pragma once

#include "dtw_device.h"

#include <array>
#include <utility>

namespace dtwmi {
namespace {

// ---------------------------------------------------------------------------
// Lane-band kernel.
//
// Row i of the band holds cells k = 0..W-1 (column i-B+k), updated in place:
//   new[k] = (x_i - y_{i-B+k})^2 + min3(old[k], old[k+1], new[k-1]).
// R consecutive rows are swept together, row i+r lagging 2 cells behind row
// i+r-1: at step t row i+r updates cell t-2r, which only reads cells row
// i+r-1 finished at steps t-2 and t-1, so the R updates of a step are
// independent (R chains of instruction-level parallelism per lane) and all
// still happen in place.  Step t of row i+r uses y[i-B+t-r]: a window of
// C+R-1 wave-uniform values per chunk of C steps, fetched into SGPRs with
// scalar loads one chunk ahead; a scheduling barrier keeps the compiler from
// hoisting the loads of a whole row (which would exceed the SGPR file).
// A chunk whose columns all lie outside [0, L) is skipped with a wave-uniform
// branch: cells left of column 0 are +inf and stay +inf, and cells right of
// column L-1 are never read by an admissible cell.  For bands of up to
// kLaneEdgeMaxW cells, row groups whose band reaches past column 0 or L-1 (the
// first and last ~B rows) sweep in chunks of kLaneEdgeChunk steps, so that
// fewer cells outside the matrix share a chunk with cells inside it (at
// W = 51, L = 256: 0.8% more cells than the admissible ones instead of 2.5%);
// the others in chunks of kLaneChunk.
#ifndef DTWMI_LANE_ROWS
#define DTWMI_LANE_ROWS 4
#endif
#ifndef DTWMI_LANE_CHUNK
#define DTWMI_LANE_CHUNK 16
#endif
#ifndef DTWMI_LANE_EDGE_CHUNK
#define DTWMI_LANE_EDGE_CHUNK 4
#endif
constexpr int kLaneRows = DTWMI_LANE_ROWS;
constexpr int kLaneChunk = DTWMI_LANE_CHUNK;
constexpr int kLaneEdgeChunk = DTWMI_LANE_EDGE_CHUNK;
constexpr int kLaneEdgeMaxW = 63;

template <int W>
__device__ __forceinline__ void lane_cell(float (&st)[W], int k, float xi, float yk) {
    const float d = xi - yk;
    float t;
    if (W == 1) {
        t = st[0];
    } else if (k == 0) {
        t = fminf(st[0], st[1]);  // left of the band is +inf
    } else if (k == W - 1) {
        t = fminf(st[W - 1], st[W - 2]);  // up is outside the band
    } else {
        t = min3f(st[k], st[k + 1], st[k - 1]);
    }
    st[k] = fmaf(d, d, t);
}

// One chunk (steps CH*C .. CH*C+C-1) of a group of R rows starting at row i,
// then the following chunks.  ybase[v] = y[i-B-(R-1)+v]; ycur holds this
// chunk's window on entry and the first window of the next group (read from
// ynext) on exit.  col0 = i-B is the column of cell 0 of row i.
template <int W, int R, int C, int CH>
__device__ __forceinline__ void lane_group(float (&st)[W], const float (&x)[R], const float *__restrict__ ybase,
                                           const float *__restrict__ ynext, float (&ycur)[C + R - 1], int col0,
                                           int L) {
    constexpr int T = W + 2 * (R - 1), NY = C + R - 1, NCH = (T + C - 1) / C, T0 = CH * C;
    float ynxt[NY];
#pragma unroll
    for (int u = 0; u < NY; ++u) ynxt[u] = (CH + 1 < NCH) ? ybase[T0 + C + u] : ynext[u];
    __builtin_amdgcn_sched_barrier(0);
    const bool live = (col0 + T0 + C - 1 >= 0) && (col0 + T0 - (R - 1) < L);
    if (live) {
#pragma unroll
        for (int u = 0; u < C; ++u) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int p = T0 + u - 2 * r;
                if (p >= 0 && p < W) lane_cell<W>(st, p, x[r], ycur[u + R - 1 - r]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NY; ++u) ycur[u] = ynxt[u];
    if constexpr (CH + 1 < NCH) lane_group<W, R, C, CH + 1>(st, x, ybase, ynext, ycur, col0, L);
}

// Rebased accumulation (RB): every lane keeps its band row relative to a
// running base (true value = stored + base) and every kLaneRebaseRows rows
// subtracts the row's smallest value from it, so that the rounding of each
// fused add is relative to the small stored values instead of the whole
// cumulative cost (long warping paths keep about the accuracy of compensated
// sums at the cost of plain ones).  One lane is one pair, so no value crosses
// lanes and the base needs no conversion.
constexpr int kLaneRebaseRows = 32;

// Row groups i .. iend-1 (iend - i a multiple of R) in chunks of C steps; the
// y window and x of the first group are read here, those of the following
// groups one group ahead.
template <int W, int R, int C, bool RB>
__device__ __forceinline__ void lane_rows(float (&st)[W], float &base, const float *__restrict__ ycol,
                                          const float *__restrict__ xrow, int &i, int iend, int B, int L) {
    if (i >= iend) return;
    float ycur[C + R - 1];
#pragma unroll
    for (int u = 0; u < C + R - 1; ++u) ycur[u] = ycol[i + u - (R - 1)];
    float x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = xrow[i + r];
    for (; i < iend; i += R) {
        float xn[R];  // next group's x, requested one group ahead (stays inside the pad)
#pragma unroll
        for (int r = 0; r < R; ++r) xn[r] = xrow[i + R + r];
        lane_group<W, R, C, 0>(st, x, ycol + i - (R - 1), ycol + i + 1, ycur, i - B, L);
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = xn[r];
        if constexpr (RB) {
            static_assert(kLaneRebaseRows % R == 0, "renormalise between row groups");
            if ((i + R) % kLaneRebaseRows == 0) {  // every row of the group is complete here
                float mn = st[0];
#pragma unroll
                for (int k = 1; k < W; ++k) mn = fminf(mn, st[k]);
                const float nb = base + (mn < kInf ? mn : 0.0f);
                const float d = nb - base;
#pragma unroll
                for (int k = 0; k < W; ++k) st[k] -= d;
                base = nb;
            }
        }
    }
}

// Lane-band items have equal cost, so the kernel takes one item per workgroup
// (hardware dispatch); an item loop would only add registers to this kernel.
// Workgroups go to the 8 XCDs of the device in turn, so workgroup w takes item
// (w mod 8) * ceil(n/8) + w / 8: each XCD works through one contiguous eighth
// of the item list, whose tiles share row series in that XCD's L2 (any order
// is correct; this one only keeps the reads local).
template <int W, bool RB>
__global__ __launch_bounds__(64) void k_lane(const float *__restrict__ ws, const SeriesInfo *__restrict__ ser,
                                             const DatasetInfo *__restrict__ dsi,
                                             const LaneItem *__restrict__ items,
                                             const LanePartner *__restrict__ partners, unsigned n_items) {
    constexpr int B = (W - 1) / 2, R = kLaneRows, C = kLaneChunk;
    const unsigned per_xcd = (n_items + 7) / 8;
    const unsigned idx = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (idx >= n_items) return;
    const LaneItem it = items[idx];
    const DatasetInfo D = dsi[it.ds];
    const int lane = threadIdx.x;
    const bool valid = lane < it.cnt;
    int bl;
    int64_t slot;
    if (it.list < 0) {  // all pairs: partner (a + d0 + lane) mod N, condensed output
        bl = it.a + it.d0 + lane;
        bl = bl >= D.N ? bl - D.N : bl;
        const int a = it.a < bl ? it.a : bl, b = it.a < bl ? bl : it.a;
        slot = condensed_index(a, b, D.N);
    } else {  // explicit pair list
        const LanePartner P = partners[it.list + (valid ? lane : 0)];
        bl = P.b;
        slot = P.slot;
    }
    if (!valid) bl = it.a;  // idle lanes recompute a valid pair and store nothing
    const float *__restrict__ ycol = ws + ser[D.series_base + it.a].pstart - B;  // ycol[v] = y[v-B]
    const float *__restrict__ xrow = ws + ser[D.series_base + bl].pstart;
    const int L = D.L;

    float st[W];
#pragma unroll
    for (int k = 0; k < W; ++k) st[k] = kInf;
    st[B] = 0.0f;  // c(0,0) of the 1-based recurrence, seen as the diagonal of cell (1,1)

    float base = 0.0f;  // rebased form only
    int i = 0;
    if (L >= R) {
        // A group starting at row i sweeps columns i-B (its first row's cell
        // 0) to i+R-1+B (its last row's cell W-1): groups at i < itop reach
        // left of column 0, groups at i >= ibot right of column L-1; both
        // sweep in chunks of kLaneEdgeChunk steps for bands up to
        // kLaneEdgeMaxW cells (wider bands hold fewer wavefronts per SIMD,
        // which then wait longer for the y values of the more numerous
        // chunks than the skipped cells save).
        constexpr int CE = (W <= kLaneEdgeMaxW && kLaneEdgeChunk < C) ? kLaneEdgeChunk : C;
        const int Lr = L - L % R;
        if constexpr (CE == C) {
            lane_rows<W, R, C, RB>(st, base, ycol, xrow, i, Lr, B, L);
        } else {
            const int itop = min(Lr, R * ((B + R - 1) / R));
            const int ibot = max(itop, min(Lr, R * ((L - B - R + 1 + R - 1) / R)));
            lane_rows<W, R, CE, RB>(st, base, ycol, xrow, i, itop, B, L);
            lane_rows<W, R, C, RB>(st, base, ycol, xrow, i, ibot, B, L);
            lane_rows<W, R, CE, RB>(st, base, ycol, xrow, i, Lr, B, L);
        }
    }
    if constexpr (R > 1) {
        for (; i < L; ++i) {  // rows left over when R does not divide L
            float ycur[C];
#pragma unroll
            for (int u = 0; u < C; ++u) ycur[u] = ycol[i + u];
            const float x1[1] = {xrow[i]};
            lane_group<W, 1, C, 0>(st, x1, ycol + i, ycol + i + 1, ycur, i - B, L);
        }
    }

    if (valid) D.out[slot] = RB ? st[B] + base : st[B];
}

using LaneFn = hipError_t (*)(const float *, const SeriesInfo *, const DatasetInfo *, const LaneItem *,
                              const LanePartner *, unsigned, hipStream_t);

template <bool RB, int I>
hipError_t lane_launcher(const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi, const LaneItem *items,
                         const LanePartner *partners, unsigned n, hipStream_t st) {
    hipLaunchKernelGGL((k_lane<2 * I + 1, RB>), dim3(8 * ((n + 7) / 8)), dim3(64), 0, st, ws, ser, dsi, items,
                       partners, n);
    return hipGetLastError();
}

template <bool RB, size_t... I>
constexpr std::array<LaneFn, sizeof...(I)> make_lane_table(std::index_sequence<I...>) {
    return {{&lane_launcher<RB, static_cast<int>(I)>...}};
}

}  // namespace
}  // namespace dtwmi
