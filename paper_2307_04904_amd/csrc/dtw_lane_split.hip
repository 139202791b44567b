// Split lane-band kernel for the all-pairs DTW matrix: the band row of a pair
// spread over P lanes, 64/P pairs per wavefront (integer division; with P = 12
// the last 4 lanes idle).  Evaluates Eq. (c) of the
// paper ("Mathematical background") under the window rule of the
// Introduction, for equal-length series, in plain FP32 sums: each cell with
// the same operations as the one-pair-per-lane kernel (dtw_lane.h), so the
// results are bit for bit the same.
//
// The one-pair-per-lane kernel needs 64 pairs per wavefront and one lane
// sweeps a whole pair: a pair list of a few thousand pairs (a k-medoids step:
// every series against a few medoids) makes too few wavefronts to fill the
// device, and each takes as long as the whole step.  Spreading a pair over P
// lanes gives P times the wavefronts, each about P times shorter.
#include "dtw_device.h"

#include <algorithm>
#include <array>
#include <utility>

namespace dtwmi {
namespace {

// ---------------------------------------------------------------------------
// Band row of W = 2B+1 cells (cell k of row i is column i-B+k, as in the
// one-pair-per-lane kernel) cut into P pieces: lane p of a pair's group owns
// cells [K_p, K_p + c_p), c_p = w = ceil(W/P) for the first P - s lanes and
// w - 1 for the last s = P*w - W ("short" lanes; their last register is
// padding).  Lane p sweeps row r = t - p at step t:
//   new[u] = (x_r - y_{r-B+K_p+u})^2 + min3(old[u], old[u+1], new[u-1]);
// the left value of its first cell is the last cell of row r of lane p-1,
// computed one step earlier and received by a DPP shift right at the end of
// that step; the up value of its last cell is cell K_{p+1} of row r-1, which
// lane p+1 computes first in this same step and hands over by a DPP shift left
// right after.  Lane 0's left and lane P-1's up are outside the band (+inf):
// each move raises the value a group-edge lane receives to +inf.  Row -1 is
// the initial register contents (+inf but for c(0,0), the diagonal of cell (0,0)), and a
// lane that has not started (r < 0) or has finished (r >= L) keeps its
// registers, so a lane that starts reads row -1 from its right neighbour and
// the final row stays in place.
//
// Steps go in iterations of U, the series values of an iteration in registers
// (x of the U rows, y of the U + w - 1 columns), double-buffered and loaded
// one iteration ahead.  Iterations in which every lane of every group is on a
// row of [0, L) run without the per-cell keep/commit selects.
// U: 16 steps, 8 for lanes of more than 8 cells (fewer buffered series values)
template <int w>
constexpr int split_steps() { return w <= 8 ? 16 : 8; }

// Lane l gets lane l-1's v (from_left) or lane l+1's (from_right): row_shr:1 /
// row_shl:1 within rows of 16 lanes when groups tile those rows (P = 4, 8,
// 16), wave_shr:1 / wave_shl:1 across the wavefront otherwise (P = 12, 32).
// The value received is raised to `pen`, the bits of +inf on the lanes at a
// group edge (which must see +inf from outside the band) and 0 elsewhere: an
// integer max on the bit patterns, exact for the values of the sweep (each
// non-negative or +inf, whose patterns order as the values do).  A lane
// without a source reads 0 and so gets `pen`.  The compiler folds the move
// and the max into one v_max_i32 with the DPP shift on its first operand.
template <int P>
__device__ __forceinline__ float from_left(float v, int pen) {
    constexpr int ctrl = 16 % P == 0 ? 0x111 : 0x138;
    return __int_as_float(max(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, true), pen));
}
template <int P>
__device__ __forceinline__ float from_right(float v, int pen) {
    constexpr int ctrl = 16 % P == 0 ? 0x101 : 0x130;
    return __int_as_float(max(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, true), pen));
}

// Lane constants of a split group.
struct SplitLane {
    int p;          // lane within the group
    int pen_first;  // p == 0 (no band cell to the left): the bits of +inf, else 0
    int pen_last;   // p == P-1 (no band cell to the right): the bits of +inf, else 0
    bool shrt;      // holds w-1 cells
};

// One step of one lane: row r of its cells.  MASK: commit only when `act`.
// left_in carries the left value of the first cell into the next step; both
// it and up_dpp are +inf on the lanes at a group edge.
template <int P, int w, bool MASK>
__device__ __forceinline__ void split_step(float (&st)[w], float &left_in, float &up_dpp, const SplitLane &ln,
                                           float x, const float *yv, bool act) {
    float nw[w];
#pragma unroll
    for (int u = 0; u < w; ++u) {
        const float d = x - yv[u];
        const float left = u == 0 ? left_in : nw[u - 1];
        float up;
        if (u < w - 2) {
            up = st[u + 1];
        } else if (u == w - 2) {
            up = ln.shrt ? up_dpp : st[u + 1];  // a short lane's last cell takes the neighbour's
        } else {
            up = up_dpp;
        }
        float v = fmaf(d, d, min3f(st[u], up, left));
        if constexpr (MASK) v = act ? v : st[u];
        nw[u] = v;
        if (u == 0) {
            // cell K_{p+1} of row r-1 from the lane to the right (its first cell of this step)
            up_dpp = from_right<P>(v, ln.pen_last);
        }
    }
#pragma unroll
    for (int u = 0; u < w; ++u) st[u] = nw[u];
    const float send = ln.shrt ? st[w - 2] : st[w - 1];  // the lane's last band cell
    left_in = from_left<P>(send, ln.pen_first);
}

template <int P, int w, int U, bool MASK>
__device__ __forceinline__ void split_iter(float (&st)[w], float &left_in, float &up_dpp, const SplitLane &ln,
                                           const float (&xb)[U], const float (&yb)[U + w - 1], int t0, int L) {
#pragma unroll
    for (int s = 0; s < U; ++s) {
        const bool act = static_cast<unsigned>(t0 + s - ln.p) < static_cast<unsigned>(L);
        float x = xb[s];
        // the masked and the unmasked bodies would otherwise share their
        // differences, which the compiler then computes for a whole
        // iteration ahead of the branch (all of them live at once)
        if constexpr (MASK) asm volatile("" : "+v"(x));
        split_step<P, w, MASK>(st, left_in, up_dpp, ln, x, yb + s, act);
        // one step at a time: without this the scheduler hoists the
        // differences of later steps and runs out of registers
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int U, int NY>
__device__ __forceinline__ void split_load(float (&xb)[U], float (&yb)[NY], const float *__restrict__ xl,
                                           const float *__restrict__ yl, int t0) {
#pragma unroll
    for (int s = 0; s < U; ++s) xb[s] = xl[t0 + s];
#pragma unroll
    for (int v = 0; v < NY; ++v) yb[v] = yl[t0 + v];
}

// Items as for the one-pair-per-lane kernel, with at most 64/P partners each
// (group g of the wavefront takes partner g); hardware dispatch with the same
// XCD-aware item map.
template <int P, int w>
__global__ __launch_bounds__(64) void k_lane_split(const float *__restrict__ ws, const SeriesInfo *__restrict__ ser,
                                                   const DatasetInfo *__restrict__ dsi,
                                                   const LaneItem *__restrict__ items,
                                                   const LanePartner *__restrict__ partners, unsigned n_items, int W) {
    constexpr int U = split_steps<w>(), NY = U + w - 1;
    const unsigned per_xcd = (n_items + 7) / 8;
    const unsigned idx = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (idx >= n_items) return;
    const LaneItem it = items[idx];
    const DatasetInfo D = dsi[it.ds];
    const int lane = threadIdx.x;
    const int grp = lane / P;
    SplitLane ln;
    ln.p = lane % P;
    ln.pen_first = ln.p == 0 ? 0x7f800000 : 0;  // the bits of +inf
    ln.pen_last = ln.p == P - 1 ? 0x7f800000 : 0;
    const bool valid = grp < it.cnt;
    int bl;
    int64_t slot;
    if (it.list < 0) {  // partner a + d0 + grp (mod N): all pairs or a row range of the condensed matrix
        bl = it.a + it.d0 + grp;
        bl = bl >= D.N ? bl - D.N : bl;
        const int a = it.a < bl ? it.a : bl, b = it.a < bl ? bl : it.a;
        slot = condensed_index(a, b, D.N);
    } else {  // explicit pair list
        const LanePartner Pn = partners[it.list + (valid ? grp : 0)];
        bl = Pn.b;
        slot = Pn.slot;
    }
    if (!valid) bl = it.a;  // idle groups recompute a valid pair and store nothing
    const int B = (W - 1) / 2, L = D.L;
    const int nshort = P * w - W;
    ln.shrt = ln.p >= P - nshort;
    const int K = ln.p * w - max(0, ln.p - (P - nshort));  // first band cell of this lane
    const int cnt = ln.shrt ? w - 1 : w;
    // x of row t - p at step t; y of cell u at step t: column t - p - B + K + u
    const float *__restrict__ xl = ws + ser[D.series_base + bl].pstart - ln.p;
    const float *__restrict__ yl = ws + ser[D.series_base + it.a].pstart - ln.p - B + K;

    float st[w];
#pragma unroll
    for (int u = 0; u < w; ++u) st[u] = (K + u == B) ? 0.0f : kInf;  // row -1
    float left_in = kInf, up_dpp = kInf;

    const int T = L + P - 1;  // steps: lane p sweeps rows 0..L-1 at steps p..L-1+p
    float xa[U], xb[U], ya[NY], yb[NY];
    split_load<U, NY>(xa, ya, xl, yl, 0);
    for (int t0 = 0; t0 < T; t0 += 2 * U) {
        split_load<U, NY>(xb, yb, xl, yl, t0 + U);
        if (t0 >= P - 1 && t0 + U <= L)
            split_iter<P, w, U, false>(st, left_in, up_dpp, ln, xa, ya, t0, L);
        else
            split_iter<P, w, U, true>(st, left_in, up_dpp, ln, xa, ya, t0, L);
        if (t0 + U >= T) break;
        split_load<U, NY>(xa, ya, xl, yl, t0 + 2 * U);
        if (t0 + U >= P - 1 && t0 + 2 * U <= L)
            split_iter<P, w, U, false>(st, left_in, up_dpp, ln, xb, yb, t0 + U, L);
        else
            split_iter<P, w, U, true>(st, left_in, up_dpp, ln, xb, yb, t0 + U, L);
    }
    if (valid && B >= K && B < K + cnt) D.out[slot] = pick<w>(st, B - K);
}

using SplitFn = hipError_t (*)(const float *, const SeriesInfo *, const DatasetInfo *, const LaneItem *,
                               const LanePartner *, unsigned, int, hipStream_t);

template <int P, int w>
hipError_t split_launcher(const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi, const LaneItem *items,
                          const LanePartner *partners, unsigned n, int W, hipStream_t st) {
    hipLaunchKernelGGL((k_lane_split<P, w>), dim3(8 * ((n + 7) / 8)), dim3(64), 0, st, ws, ser, dsi, items, partners,
                       n, W);
    return hipGetLastError();
}

// Cells per lane w = kSplitMinW .. kSplitMaxW
constexpr int kSplitMinW = 3, kSplitMaxW = 16;

template <int P, size_t... I>
constexpr std::array<SplitFn, sizeof...(I)> make_split_table(std::index_sequence<I...>) {
    return {{&split_launcher<P, kSplitMinW + static_cast<int>(I)>...}};
}

constexpr int kSplitWidths = kSplitMaxW - kSplitMinW + 1;
const std::array<SplitFn, kSplitWidths> kSplit4 = make_split_table<4>(std::make_index_sequence<kSplitWidths>{});
const std::array<SplitFn, kSplitWidths> kSplit8 = make_split_table<8>(std::make_index_sequence<kSplitWidths>{});
// W <= 127 needs w <= 11 for P = 12, w <= 8 for P = 16 and w <= 4 for P = 32
const std::array<SplitFn, 11 - kSplitMinW + 1> kSplit12 = make_split_table<12>(std::make_index_sequence<11 - kSplitMinW + 1>{});
const std::array<SplitFn, 8 - kSplitMinW + 1> kSplit16 = make_split_table<16>(std::make_index_sequence<8 - kSplitMinW + 1>{});
const std::array<SplitFn, 4 - kSplitMinW + 1> kSplit32 = make_split_table<32>(std::make_index_sequence<4 - kSplitMinW + 1>{});

}  // namespace

int split_max_cells(int P) { return P == 32 ? 4 : (P == 16 ? 8 : (P == 12 ? 11 : kSplitMaxW)); }

bool lane_split_supported(int P, int W) {
    if (!lane_width_supported(W)) return false;
    if (P != 4 && P != 8 && P != 12 && P != 16 && P != 32) return false;
    const int w = (W + P - 1) / P;
    return w >= kSplitMinW && w <= split_max_cells(P);
}

hipError_t launch_lane_split(int P, int W, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                             const LaneItem *items, const LanePartner *partners, unsigned n_items,
                             hipStream_t stream) {
    if (!lane_split_supported(P, W)) return hipErrorInvalidValue;
    if (n_items == 0) return hipSuccess;
    const int i = (W + P - 1) / P - kSplitMinW;
    const SplitFn f = P == 4    ? kSplit4[i]
                      : P == 8  ? kSplit8[i]
                      : P == 12 ? kSplit12[i]
                      : P == 16 ? kSplit16[i]
                                : kSplit32[i];
    return f(ws, ser, dsi, items, partners, n_items, W, stream);
}

}  // namespace dtwmi
