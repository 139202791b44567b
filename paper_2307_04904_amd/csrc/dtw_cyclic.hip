// Cyclic banded kernel for the all-pairs DTW matrix: one pair per wavefront,
// blocks of rows of the longer series cycling over the 64 lanes, each block
// visiting only the columns its window admits.  Evaluates Eq. (c) of the
// paper ("Mathematical background") under the window rule of the
// Introduction, in FP32 (plain, or rebased: every lane keeps its values
// relative to a running base of its own, see below).
#include "dtw_device.h"

namespace dtwmi {
namespace {

// ---------------------------------------------------------------------------
// Cyclic banded strips: one pair per wavefront, row blocks cycling over the
// lanes.  Block g (rows [gH, gH+H)) runs on lane g mod 64 and processes column
// c at step c + g, but only over its window columns [max(0, gH-b),
// min(m-1, gH+H-1+b)]; when its window ends the lane takes block g+64.  With
// 64(H+1) >= 2b+H a lane's next block never starts before its current one
// ends, so the one-step skew between consecutive blocks holds everywhere and
// the boundary row still moves by one DPP rotation (lane 63 -> lane 0) per
// step.  Idle lanes sweep only while blocks are active instead of the whole
// rectangle, which is what matters when the window is much narrower than the
// pair: the in-window cells are a diagonal strip of the rectangle.
//
// The window needs no masking of whole rows.  An admissible cell (i,j) reads
// two cells that can lie outside the window: its left neighbour (i,j-1) when
// i-j = b and its upper neighbour (i-1,j) when j-i = b; every other cell
// outside the window feeds only cells outside it.  So the kernel computes the
// cells of a block's rows before they enter the window with their real x
// values (the results are never read), and only
//  * at the entry of row i (column i-b) sets that row's left value to +inf;
//  * at the exit of row i (column i+b+1) sets x_i to kBig, so that the row's
//    cells from there on overflow to +inf and the row below reads +inf;
//  * replaces a received boundary value by +inf past the previous block's
//    window (its last row exits there; its lane may already work on another
//    block).

// Register vector of a block's H rows (x, and the two column buffers), with a
// wave-uniform runtime index turned into one indexed register move
// (s_set_gpr_idx): the compiler does that for vectors of more than 8 elements
// and expands smaller ones into a compare and a select per element, so small
// blocks get 9 elements.
template <int H>
struct CycVec {
    static constexpr int W = H <= 8 ? 9 : (H <= 12 ? H : (H <= 16 ? 16 : H));
    typedef float T __attribute__((ext_vector_type(W)));
};

template <int H>
struct CycLane {  // the block a lane of a cyclic strip works on
    int g;     // block index
    int gend;  // last step of block g, or INT_MAX when no block g+64 follows it
    int tphi;  // from step tphi+1 on, the boundary row received lies past its window
    int E, emax;  // row h <= emax of the block enters the window at step E + h
    int X, xmax;  // row h <= xmax leaves it at step X + h (x becomes kBig)
    const float *__restrict__ yl;  // y column of step s: yl[s]
};

// Load block c.g into this lane: x of its rows (rows past n read the +inf pad
// after the series; their cells never feed row n-1), the step its window ends,
// the masking step of its boundary row and its y pointer.  y is read at
// columns s - g without a clamp: every lane reads between column -63 (a block
// starts at most 63 steps before its first column) and m+66 (no lane holds a
// block more than 63 below the last one, which ends at step m-1+Qf), inside
// the +inf pads of the staged series.
template <int H>
__device__ __forceinline__ void cyc_block(CycLane<H> &c, typename CycVec<H>::T &x, const float *__restrict__ xp,
                                          const float *__restrict__ yp, int n, int m, int b, int Qf) {
    const int r0 = c.g * H;
    const float *__restrict__ xb = xp + (r0 < n ? r0 : n);
#pragma unroll
    for (int h = 0; h < H; ++h) x[h] = xb[h];
    const bool live = r0 < n;
    c.gend = (live && c.g + 64 <= Qf) ? min(m - 1, r0 + H - 1 + b) + c.g : 0x7fffffff;
    c.tphi = ((c.g > 0 && live) ? min(m - 1, r0 - 1 + b) : -1) + c.g;
    c.yl = yp - c.g;
    // Row r0+h enters at column r0+h-b, i.e. step g(H+1)+h-b, for rows before
    // n (rows past n never feed row n-1); it leaves after column r0+h+b, at
    // step g(H+1)+h+b+1, for h <= H-2 (the last row is masked by the next
    // block) and a column before m (later exits are not needed).  A block
    // without events gets a start far past every step.
    const int emax = min(H - 1, n - 1 - r0), xmax = min(H - 2, m - 2 - r0 - b);
    c.E = emax >= 0 ? c.g * (H + 1) - b : 0x40000000;
    c.emax = max(emax, 0);
    c.X = xmax >= 0 ? c.g * (H + 1) + b + 1 : 0x40000000;
    c.xmax = max(xmax, 0);
}

// Window events of step s, detected per lane from its own block: the lane
// whose row h = s - E enters sets that row's left value to +inf, the lane
// whose row h = s - X leaves sets x_h to kBig.  Consecutive blocks' events lie
// H+1 steps apart and each block has at most H of each kind, so at most one
// lane has an entry and one an exit at any step; its row index, read from the
// first active lane, is wave-uniform and each event is one indexed register
// move on one lane (the empty asm statements keep each a one-lane branch:
// without them the compiler turns it into a select of the whole register
// vector).  A lane takes block g+64 no later than that block's first entry
// (with 64(H+1) = 2b+H on the same step, the switch first), and exits come
// before its block ends, so every event finds its block on its lane.
template <int H>
__device__ __forceinline__ void cyc_events(int s, const CycLane<H> &c, typename CycVec<H>::T &x,
                                           typename CycVec<H>::T &O) {
    const int he = s - c.E;
    if (static_cast<unsigned>(he) <= static_cast<unsigned>(c.emax)) {
        asm volatile("");
        O[__builtin_amdgcn_readfirstlane(he)] = kInf;
    }
    const int hx = s - c.X;
    if (static_cast<unsigned>(hx) <= static_cast<unsigned>(c.xmax)) {
        asm volatile("");
        x[__builtin_amdgcn_readfirstlane(hx)] = kBig;
    }
}

// Rebased accumulation (RB): the wavefront stores its values relative to a
// base it shares (true value = stored + base), and every kCycRebaseSteps steps
// the base moves up to the smallest value on its frontier: every lane's H
// cells and the boundary values it holds (which carry the last row of a block
// that has already left its window).  Every path to a cell computed later
// passes through that frontier and local costs are never negative, so stored
// values stay between 0 and the true cost and each fused add rounds relative
// to them instead of the whole cumulative cost: never more than plain sums,
// on long paths typically an order of magnitude less.  Rows not yet admitted
// hold values of a wider window, which are no larger than the true ones; they
// can only lower the minimum, so the base stays a lower bound.
constexpr int kCycRebaseSteps = 32;  // a multiple of the 4 steps of one loop iteration

// One step.  y0..y3 hold (or are loading) y at this lane's columns of steps
// s..s+3; a block switch moves the columns by -64, so it reloads them.
template <int H, bool RB>
__device__ __forceinline__ void cyc_step(int s, CycLane<H> &c, typename CycVec<H>::T &x, typename CycVec<H>::T &O,
                                         typename CycVec<H>::T &N, float &up_in, float &diag_in, float &raw_up,
                                         float &raw_diag, float &y0, float &y1, float &y2, float &y3,
                                         const float *__restrict__ xp, const float *__restrict__ yp, int n, int m,
                                         int b, int Qf) {
    if (s > c.gend) {  // this lane's block left the window: take block g+64
        c.g += 64;
        cyc_block<H>(c, x, xp, yp, n, m, b, Qf);
        y0 = c.yl[s];
        y1 = c.yl[s + 1];
        y2 = c.yl[s + 2];
        y3 = c.yl[s + 3];
        // Wait for these loads here (vmcnt 0): x is read in this step, and
        // without the wait the compiler, merging this rare path with the
        // common one, would wait for every load in flight at every step.
        __builtin_amdgcn_s_waitcnt(0x0F70);
        // Row 0 may be admitted at this very step (when 64(H+1) = 2b+H), so
        // its left neighbour must be +inf now; the other rows get theirs at
        // their entries.
        O[0] = kInf;
        // The neighbour lane already holds block g-1 (g the new block), so the
        // values it sent in the last two steps are row gH-1 at this step's
        // column and at the one before; keep those that row's window admits (a
        // path along the band edge runs through them when the switch comes one
        // step before the new block's first admissible column).
        up_in = s > c.tphi ? kInf : raw_up;
        diag_in = s - 1 > c.tphi ? kInf : raw_diag;
    }
    cyc_events<H>(s, c, x, O);
    const float yv = y0;
    float diag = diag_in, up = up_in;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const float d = x[h] - yv;
        const float v = fmaf(d, d, min3f(diag, up, O[h]));
        diag = O[h];
        up = v;
        N[h] = v;
    }
    // DPP wave_ror:1: lane l receives lane l-1, lane 0 receives lane 63 (every
    // lane has a source, so no old value is needed)
    const float recv = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(N[H - 1]), 0x13C, 0xF, 0xF, true));
    raw_diag = raw_up;
    raw_up = recv;
    diag_in = up_in;
    up_in = s < c.tphi ? recv : kInf;  // past the previous block's window
}

// Renormalise the rebased form: the base moves up by the smallest of every
// lane's rows 0..H-1 and `held`; returns the shift subtracted from every
// stored value (the difference of the new and the old base as computed).
template <int H>
__device__ __forceinline__ float cyc_rebase(typename CycVec<H>::T &A, float held, float &base) {
    float mn = held;
#pragma unroll
    for (int h = 0; h < H; ++h) mn = fminf(mn, A[h]);
    mn = wave_min(mn);
    const float nb = base + (mn < kInf ? mn : 0.0f);
    const float d = nb - base;
#pragma unroll
    for (int h = 0; h < H; ++h) A[h] -= d;
    base = nb;
    return d;
}

template <int H, bool RB>
__device__ __forceinline__ void cyc_item(const WaveItem it, const float *__restrict__ ws,
                                         const SeriesInfo *__restrict__ ser, const DatasetInfo *__restrict__ dsi) {
    typedef typename CycVec<H>::T xvec;
    const int lane = item_lane(it.ds);
    const DatasetInfo DI = dsi[it.ds];
    const SeriesInfo sr = ser[DI.series_base + it.rows];
    const SeriesInfo sc = ser[DI.series_base + it.cols];
    const int n = sr.len, m = sc.len, b = it.band;
    const float *__restrict__ xp = ws + sr.pstart;
    const float *__restrict__ yp = ws + sc.pstart;
    const int Qf = (n - 1) / H, hf = (n - 1) - Qf * H;
    const int sfinal = (m - 1) + Qf;

    CycLane<H> c;
    c.g = lane;
    xvec x, A, Bv;
    cyc_block<H>(c, x, xp, yp, n, m, b, Qf);
#pragma unroll
    for (int h = 0; h < CycVec<H>::W; ++h) {
        A[h] = kInf;
        Bv[h] = kInf;
    }
    float up_in = kInf;
    float diag_in = lane == 0 ? 0.0f : kInf;
    float raw_up = kInf, raw_diag = kInf;  // unmasked values received in the last two steps
    float base = 0.0f;                     // rebased form only: the wavefront's base

    // Four steps per iteration, so that the y prefetch registers rotate by
    // name instead of by copies.
    int s = 0;
    float q0 = c.yl[0], q1 = c.yl[1], q2, q3;
    __builtin_amdgcn_s_waitcnt(0x0F70);  // x in place before the loop (see the block switch)
    for (; s + 3 <= sfinal; s += 4) {
        q2 = c.yl[s + 2];
        q3 = c.yl[s + 3];
        cyc_step<H, RB>(s, c, x, A, Bv, up_in, diag_in, raw_up, raw_diag, q0, q1, q2, q3, xp, yp, n, m, b, Qf);
        cyc_step<H, RB>(s + 1, c, x, Bv, A, up_in, diag_in, raw_up, raw_diag, q1, q2, q3, q0, xp, yp, n, m,
                    b, Qf);
        q0 = c.yl[s + 4];
        q1 = c.yl[s + 5];
        cyc_step<H, RB>(s + 2, c, x, A, Bv, up_in, diag_in, raw_up, raw_diag, q2, q3, q0, q1, xp, yp, n, m,
                    b, Qf);
        cyc_step<H, RB>(s + 3, c, x, Bv, A, up_in, diag_in, raw_up, raw_diag, q3, q0, q1, q2, xp, yp, n, m,
                    b, Qf);
        if constexpr (RB) {
            if ((s + 4) % kCycRebaseSteps == 0) {
                const float d = cyc_rebase<H>(A, fminf(fminf(up_in, diag_in), fminf(raw_up, raw_diag)), base);
                up_in -= d;
                diag_in -= d;
                raw_up -= d;
                raw_diag -= d;
            }
        }
    }
    const int rem = sfinal + 1 - s;  // 0..3 steps left
    if (rem >= 1) {
        q2 = c.yl[s + 2];
        q3 = c.yl[s + 3];
        cyc_step<H, RB>(s, c, x, A, Bv, up_in, diag_in, raw_up, raw_diag, q0, q1, q2, q3, xp, yp, n, m, b, Qf);
    }
    if (rem >= 2)
        cyc_step<H, RB>(s + 1, c, x, Bv, A, up_in, diag_in, raw_up, raw_diag, q1, q2, q3, q0, xp, yp, n, m,
                    b, Qf);
    if (rem >= 3)
        cyc_step<H, RB>(s + 2, c, x, A, Bv, up_in, diag_in, raw_up, raw_diag, q2, q3, q0, q1, xp, yp, n, m,
                    b, Qf);
    const float res = (rem & 1) ? Bv[hf] : A[hf];
    if (lane == (Qf & 63)) DI.out[it.slot] = RB ? res + base : res;
}

// Waves per SIMD the register allocation aims for: plain H = 28 fits 4 (126
// VGPRs, no scratch) instead of 3 when asked; H = 20, 24 and 32, and the
// rebased H = 28 (two more registers), would spill.
template <int H, bool RB>
constexpr int cyc_min_waves() { return H == 28 && !RB ? 4 : 1; }

template <int H, bool RB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(cyc_min_waves<H, RB>()))) void k_strip_cyc(const float *__restrict__ ws, const SeriesInfo *__restrict__ ser,
                                                  const DatasetInfo *__restrict__ dsi,
                                                  const WaveItem *__restrict__ items, unsigned *__restrict__ queue,
                                                  unsigned n_items) {
    unsigned idx = blockIdx.x;
    for (;;) {
        if (queue) idx = next_item<1>(queue, nullptr);
        if (idx >= n_items) break;
        cyc_item<H, RB>(items[idx], ws, ser, dsi);
        if (!queue) break;
    }
}

template <int H>
hipError_t cyc_launch(bool rb, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi, const WaveItem *items,
                      unsigned n, unsigned *queue, unsigned grid, hipStream_t st) {
    if (rb)
        hipLaunchKernelGGL((k_strip_cyc<H, true>), dim3(grid), dim3(64), 0, st, ws, ser, dsi, items, queue, n);
    else
        hipLaunchKernelGGL((k_strip_cyc<H, false>), dim3(grid), dim3(64), 0, st, ws, ser, dsi, items, queue, n);
    return hipGetLastError();
}

template <int H>
int cyc_slots(bool rb) {
    return rb ? resident_blocks(reinterpret_cast<const void *>(&k_strip_cyc<H, true>), 64)
              : resident_blocks(reinterpret_cast<const void *>(&k_strip_cyc<H, false>), 64);
}

using SlotsFn = int (*)(bool);
using CycFn = hipError_t (*)(bool, const float *, const SeriesInfo *, const DatasetInfo *, const WaveItem *, unsigned,
                             unsigned *, unsigned, hipStream_t);
struct CycEntry {
    int H;
    CycFn fn;
    SlotsFn slots;
};
#define DTWMI_CYC(H) {H, &cyc_launch<H>, &cyc_slots<H>}
const CycEntry kCyclic[] = {DTWMI_CYC(1),  DTWMI_CYC(2),  DTWMI_CYC(3),  DTWMI_CYC(4),  DTWMI_CYC(6),
                            DTWMI_CYC(8),  DTWMI_CYC(10), DTWMI_CYC(12), DTWMI_CYC(16), DTWMI_CYC(20),
                            DTWMI_CYC(24), DTWMI_CYC(28), DTWMI_CYC(32)};
#undef DTWMI_CYC

// Grid of a launch: one workgroup per item, or with a queue the resident
// workgroups (at most one per item).
unsigned grid_for(unsigned n, unsigned *queue, int slots) {
    if (!queue || slots <= 0) return n;
    return n < static_cast<unsigned>(slots) ? n : static_cast<unsigned>(slots);
}

}  // namespace

int cyclic_shapes(int *H_out, int max_out) {
    int k = 0;
    for (const CycEntry &e : kCyclic) {
        if (H_out && k < max_out) H_out[k] = e.H;
        ++k;
    }
    return k;
}

int cyclic_resident(int H, bool rebased) {
    for (const CycEntry &e : kCyclic)
        if (e.H == H) return e.slots(rebased);
    return 0;
}

hipError_t launch_cyclic(int H, bool rebased, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                         const WaveItem *items, unsigned n_items, unsigned *queue, int slots, hipStream_t stream) {
    if (n_items == 0) return hipSuccess;
    for (const CycEntry &e : kCyclic)
        if (e.H == H)
            return e.fn(rebased, ws, ser, dsi, items, n_items, queue, grid_for(n_items, queue, slots), stream);
    return hipErrorInvalidValue;
}

}  // namespace dtwmi
