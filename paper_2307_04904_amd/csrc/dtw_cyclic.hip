// Cyclic banded kernel for the all-pairs DTW matrix: one pair per wavefront,
// blocks of rows of the longer series cycling over the 64 lanes, each block
// visiting only the columns its window admits.  Evaluates Eq. (c) of the
// paper ("Mathematical background") under the window rule of the
// Introduction, in FP32.
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
// A received boundary value is replaced by +inf past the previous block's
// window (its lane may already work on another block); window edges inside a
// block use the row events above (exit events of a block's last row are not
// needed: that row leaves the window when the block ends).
template <int H>
struct CycLane {  // the block a lane of a cyclic strip works on
    int g, gend, phi;
    int yb;  // y column of step s is s - yb: g, or far to the left once no block is left
};

// Load block c.g of the pair into this lane (rows past n get x = 1e30).
template <int H>
__device__ __forceinline__ void cyc_setup(CycLane<H> &c, typename XVec<H>::T &xr, typename XVec<H>::T &x,
                                          const float *__restrict__ xp, int n, int m, int b) {
    const int r0 = c.g * H;
    // rows [r0, r0+H) read from min(r0, n): at most H-1 < kPad past the end
    const float *__restrict__ xb = xp + (r0 < n ? r0 : n);
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int r = r0 + h;
        const float v = xb[h];
        xr[h] = r < n ? v : 0.0f;
        x[h] = (r < n && r - b <= 0) ? v : kBig;
    }
    c.gend = r0 < n ? min(m - 1, r0 + H - 1 + b) + c.g : 0x7fffffff;
    c.yb = r0 < n ? c.g : (1 << 29);
    c.phi = (c.g > 0 && r0 < n) ? min(m - 1, r0 - 1 + b) : -1;
}

// Move this lane to block c.g + 64 at a block switch.  Its rows start past
// the window (r > b for every block g >= 64 when 64(H+1) >= 2b+H), so x is
// kBig and the entry events admit them; rows past n read the +inf pad after
// the series, whose cells never feed row n-1.
template <int H>
__device__ __forceinline__ void cyc_next_block(CycLane<H> &c, typename XVec<H>::T &xr, typename XVec<H>::T &x,
                                               const float *__restrict__ xp, int n, int m, int b) {
    c.g += 64;
    const int r0 = c.g * H;
    const float *__restrict__ xb = xp + (r0 < n ? r0 : n);
#pragma unroll
    for (int h = 0; h < H; ++h) {
        xr[h] = xb[h];
        x[h] = kBig;
    }
    c.gend = r0 < n ? min(m - 1, r0 + H - 1 + b) + c.g : 0x7fffffff;
    c.yb = r0 < n ? c.g : (1 << 29);
    c.phi = r0 < n ? min(m - 1, r0 - 1 + b) : -1;
}

// Row events of step s (wave-uniform: one lane per event).  Entry of row
// qH+h at column qH+h-b, exit after column qH+h+b.  Only two tests are needed:
//  * entries stop after row n-1 (s_last): in a pair with at most 64 blocks the
//    band may be wide, and an entry of a block past n would land on the lane
//    still holding block q-64;
//  * exits need q >= 0 (q & 63 of a negative q names a lane with a live block).
// Other spurious events are harmless: entries at columns <= 0 repeat what the
// block set-up did (only blocks q < 64 have such rows when 64(H+1) >= 2b+H);
// rows past n never feed row n-1; an exit that comes after its lane moved to
// block q+64 precedes the entry of the same row there by at least one step.
template <int H>
__device__ __forceinline__ void cyc_events(int s, RowCounter &en, RowCounter &ex, typename XVec<H>::T &x,
                                           const typename XVec<H>::T &xr, int lane, int s_last) {
    // The empty asm statements keep each move a one-lane branch: without them
    // the compiler turns it into a select of the whole register vector.
    if (en.h < H && s <= s_last) {
        if (lane == (en.q & 63)) {
            asm volatile("");
            x[en.h] = xr[en.h];
        }
    }
    en.advance<H>();
    if (ex.h <= H - 2 && ex.q >= 0) {
        if (lane == (ex.q & 63)) {
            asm volatile("");
            x[ex.h] = kBig;
        }
    }
    ex.advance<H>();
}

// y at column col, read from the +inf pad at -1 for columns left of the series.
// No upper clamp: a lane reads at most 4 columns past m (steps prefetched
// beyond its block's last step), well inside the pad, and a lane without a
// block reads with yb far to the right of s.
__device__ __forceinline__ float cyc_y(const float *__restrict__ yp, int col) {
    return yp[col < -1 ? -1 : col];
}

// One step.  y0..y3 hold (or are loading) y at this lane's columns of steps
// s..s+3; a block switch moves the columns by -64, so it reloads them.
template <int H>
__device__ __forceinline__ void cyc_step(int s, CycLane<H> &c, typename XVec<H>::T &xr, typename XVec<H>::T &x,
                                         float (&O)[H], float (&N)[H], float &up_in, float &diag_in,
                                         float &raw_up, float &raw_diag, RowCounter &en, RowCounter &ex,
                                         float &y0, float &y1, float &y2, float &y3,
                                         const float *__restrict__ xp, const float *__restrict__ yp, int lane,
                                         int n, int m, int b, int s_last) {
    if (s > c.gend) {  // this lane's block left the window: take block g+64
        cyc_next_block<H>(c, xr, x, xp, n, m, b);
        y0 = cyc_y(yp, s - c.yb);
        y1 = cyc_y(yp, s + 1 - c.yb);
        y2 = cyc_y(yp, s + 2 - c.yb);
        y3 = cyc_y(yp, s + 3 - c.yb);
        // Row 0 may be admitted at this very step (when 64(H+1) = 2b+H), so
        // its left neighbour must be +inf now; rows below are admitted at
        // least one step later and their kBig cells of the steps before are +inf.
        O[0] = kInf;
        // The neighbour lane already holds block g-1 (g the new block), so the
        // values it sent in the last two steps are row gH-1 at this step's
        // column and at the one before; keep those that row's window admits (a
        // path along the band edge runs through them when the switch comes one
        // step before the new block's first admissible column).
        const int col0 = s - c.g;
        up_in = col0 > c.phi ? kInf : raw_up;
        diag_in = col0 - 1 > c.phi ? kInf : raw_diag;
    }
    cyc_events<H>(s, en, ex, x, xr, lane, s_last);
    const int col = s - c.g;
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
    // DPP wave_ror:1: lane l receives lane l-1, lane 0 receives lane 63
    const float recv = __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(kInf), __float_as_int(N[H - 1]), 0x13C, 0xF, 0xF, false));
    raw_diag = raw_up;
    raw_up = recv;
    diag_in = up_in;
    up_in = (col + 1 > c.phi) ? kInf : recv;  // past the previous block's window
}

template <int H>
__device__ __forceinline__ void cyc_item(const WaveItem it, const float *__restrict__ ws,
                                         const SeriesInfo *__restrict__ ser, const DatasetInfo *__restrict__ dsi) {
    typedef typename XVec<H>::T xvec;
    const int lane = item_lane(it.ds);
    const DatasetInfo DI = dsi[it.ds];
    const SeriesInfo sr = ser[DI.series_base + it.rows];
    const SeriesInfo sc = ser[DI.series_base + it.cols];
    const int n = sr.len, m = sc.len, b = it.band;
    const float *__restrict__ xp = ws + sr.pstart;
    const float *__restrict__ yp = ws + sc.pstart;
    const int Qf = (n - 1) / H, hf = (n - 1) - Qf * H;
    const int sfinal = (m - 1) + Qf;
    const int s_last = Qf * (H + 1) + hf - b;  // entry step of row n-1

    CycLane<H> c;
    c.g = lane;
    xvec xr, x;
    cyc_setup<H>(c, xr, x, xp, n, m, b);
    float A[H], Bv[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        A[h] = kInf;
        Bv[h] = kInf;
    }
    float up_in = kInf;
    float diag_in = lane == 0 ? 0.0f : kInf;
    float raw_up = kInf, raw_diag = kInf;  // unmasked values received in the last two steps
    RowCounter en, ex;
    en.init<H>(b);
    ex.init<H>(-b - 1);

    int s = 0;
    float y0 = cyc_y(yp, -c.yb), y1 = cyc_y(yp, 1 - c.yb), y2, y3, y4;
    for (; s + 2 <= sfinal + 1; s += 2) {
        // loads for the next two steps go out before this pair of steps
        y2 = cyc_y(yp, s + 2 - c.yb);
        y3 = cyc_y(yp, s + 3 - c.yb);
        cyc_step<H>(s, c, xr, x, A, Bv, up_in, diag_in, raw_up, raw_diag, en, ex, y0, y1, y2, y3, xp, yp, lane, n,
                    m, b, s_last);
        cyc_step<H>(s + 1, c, xr, x, Bv, A, up_in, diag_in, raw_up, raw_diag, en, ex, y1, y2, y3, y4, xp, yp, lane,
                    n, m, b, s_last);
        y0 = y2;
        y1 = y3;
    }
    float res;
    if (s <= sfinal) {
        cyc_step<H>(s, c, xr, x, A, Bv, up_in, diag_in, raw_up, raw_diag, en, ex, y0, y1, y2, y3, xp, yp, lane, n,
                    m, b, s_last);
        res = pick<H>(Bv, hf);
    } else {
        res = pick<H>(A, hf);
    }
    if (lane == (Qf & 63)) DI.out[it.slot] = res;
}

template <int H>
__global__ __launch_bounds__(64) void k_strip_cyc(const float *__restrict__ ws, const SeriesInfo *__restrict__ ser,
                                                  const DatasetInfo *__restrict__ dsi,
                                                  const WaveItem *__restrict__ items, unsigned *__restrict__ queue,
                                                  unsigned n_items) {
    unsigned idx = blockIdx.x;
    for (;;) {
        if (queue) idx = next_item<1>(queue, nullptr);
        if (idx >= n_items) break;
        cyc_item<H>(items[idx], ws, ser, dsi);
        if (!queue) break;
    }
}

template <int H>
hipError_t cyc_launch(const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi, const WaveItem *items,
                      unsigned n, unsigned *queue, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((k_strip_cyc<H>), dim3(grid), dim3(64), 0, st, ws, ser, dsi, items, queue, n);
    return hipGetLastError();
}

template <int H>
int cyc_slots() {
    return resident_blocks(reinterpret_cast<const void *>(&k_strip_cyc<H>), 64);
}

using SlotsFn = int (*)();
using CycFn = hipError_t (*)(const float *, const SeriesInfo *, const DatasetInfo *, const WaveItem *, unsigned,
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

int cyclic_resident(int H) {
    for (const CycEntry &e : kCyclic)
        if (e.H == H) return e.slots();
    return 0;
}

hipError_t launch_cyclic(int H, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                         const WaveItem *items, unsigned n_items, unsigned *queue, int slots, hipStream_t stream) {
    if (n_items == 0) return hipSuccess;
    for (const CycEntry &e : kCyclic)
        if (e.H == H) return e.fn(ws, ser, dsi, items, n_items, queue, grid_for(n_items, queue, slots), stream);
    return hipErrorInvalidValue;
}

}  // namespace dtwmi
