// Wavefront strip kernels for the all-pairs DTW matrix: one pair per
// workgroup of 1..16 wavefronts, each lane owning a strip of rows of the
// shorter series; plain, rebased or Kahan-compensated FP32, or FP64
// accumulation.  Evaluates Eq. (c) of the paper ("Mathematical background")
// under the window rule of the Introduction.
//
// This header holds the kernel templates; dtw_strip.hip instantiates the FP32
// forms and dtw_strip_f64.hip the FP64 ones, built without signalling-NaN
// handling: the FP64 recurrence produces no NaN, and in IEEE mode every min
// operand of unknown origin costs an extra quieting instruction.
#pragma once

#include "dtw_device.h"

#include <type_traits>

namespace dtwmi {
namespace {

// ---------------------------------------------------------------------------
// Wavefront strip kernels: one pair per workgroup of G wavefronts.
//
// Lane l of wavefront g owns rows [(64g+l)H, (64g+l)H+H) of the row series
// and at step s processes column s - l - g(64+D) (anti-diagonal skew).  Each
// step updates a whole strip column: H cells in order, each cell's "up" being
// the cell just computed above it.  The bottom cell goes to lane l+1 with a
// DPP wave_shr:1 move; the previous step's received value is the diagonal.
// Between wavefronts of one workgroup the bottom row of lane 63 is handed
// over through an LDS ring: wavefront g lags wavefront g-1 by D = K extra
// steps and the workgroup meets at a barrier every K steps, so a value is
// always read at least one barrier after it was written.  State per lane is
// 2H cells, ping-ponged over two unrolled steps.

// Accumulation policies: cell(x, y, diag, up, left) evaluates Eq. (c).
struct AccPlain {  // FP32: sub, min3, fused multiply-add
    using T = float;
    __device__ static T inf() { return kInf; }
    __device__ static T zero() { return 0.0f; }
    __device__ static T cell(float xe, float yv, T diag, T up, T left) {
        const float d = xe - yv;
        return fmaf(d, d, min3f(diag, up, left));
    }
    __device__ static float result(T v) { return v; }
};

// Rebased FP32: the cells of AccPlain, with the values of a wavefront stored
// relative to a base it shares (true value = stored value + base).  Every few
// steps the base moves up to the smallest value on the wavefront's current
// frontier -- its lanes' current cells, the boundary values they hold and,
// for a wavefront after the first, every value of the LDS ring from the
// wavefront above and the floor that one last posted (its base, or +inf once
// its whole frontier has left the window: without that, a wavefront below
// would stay capped at a base frozen when the window moved past the rows
// above, and its sums would round like plain ones); in a row pass after the
// first, the first wavefront also holds the smallest value of the row above
// the pass.  Every path to a cell
// computed later passes through that frontier and local costs are never
// negative, so the base stays below every value computed afterwards: stored
// values lie between 0 and the true cost, and each fused add rounds relative
// to the stored value -- the distance of the path above the frontier's
// cheapest cell plus what it gained since the last renormalisation -- instead
// of the whole cumulative cost.  The rounding is never larger than that of
// plain sums and on long paths typically an order of magnitude smaller.
// Values between lanes need no conversion (one base); values handed between
// wavefronts through LDS travel as absolute values.
struct AccRebased : AccPlain {};

template <class ACC>
constexpr bool kRebased = std::is_same<ACC, AccRebased>::value;

// Steps between renormalisations (one-column and two-column sweeps).
constexpr int kRebaseSteps = 32;
constexpr int kRebaseSteps2 = 16;

// Renormalise a wavefront: the base moves up by the smallest of the H cells of
// every lane and `held` (the lane's other frontier values, relative to the
// base); returns the shift applied (the difference of the new and the old base
// as computed, subtracted from every stored value).  All +inf: no shift, and
// `floor` (the absolute lower bound of every value the wavefront computes from
// now on, which it posts for the wavefront below) becomes +inf -- a frontier
// of +inf only ever produces +inf -- else it is the new base.
template <int H>
__device__ __forceinline__ float rebase_wave(float (&A)[H], float held, float &base, float &floor) {
    float mn = held;
#pragma unroll
    for (int h = 0; h < H; ++h) mn = fminf(mn, A[h]);
    mn = wave_min(mn);
    const bool live = mn < kInf;
    const float nb = base + (live ? mn : 0.0f);
    const float d = nb - base;
#pragma unroll
    for (int h = 0; h < H; ++h) A[h] -= d;
    base = nb;
    floor = live ? nb : kInf;
    return d;
}

// Kahan-compensated FP32: each cell carries (s, c) with the true value close to
// s - c and |c| about half an ulp of s at most.  The predecessor is the
// smallest (s, -c) in lexicographic order: the smallest running sum s and,
// among equal sums, the largest compensation, i.e. the smallest true value
// (sums differing by an ulp or more are ordered by s alone).  Ties of s are
// common where local costs fall below an ulp of the cumulative cost and are
// absorbed into c, so taking the first tied predecessor would add up to an ulp
// per such cell, a bias that grows with the path.  The local cost is then added
// with Kahan's compensated step.  An unreachable cell (s = +inf) gets c = NaN
// from inf - inf; that is harmless: a reachable cell has a finite predecessor,
// whose s is the minimum, so the c of an unreachable one is masked out.
struct KahanCell {
    float s, c;
};
struct AccKahan {
    using T = KahanCell;
    __device__ static T inf() { return {kInf, 0.0f}; }
    __device__ static T zero() { return {0.0f, 0.0f}; }
    __device__ static T cell(float xe, float yv, T diag, T up, T left) {
        const float d = xe - yv;
        const float q = d * d;
        const float p = min3f(diag.s, up.s, left.s);
        const float cd = (p == diag.s) ? diag.c : -kInf;
        const float cu = (p == up.s) ? up.c : -kInf;
        const float cl = (p == left.s) ? left.c : -kInf;
        const float cs = fmaxf(fmaxf(cd, cu), cl);
        const float yk = q - cs;
        const float t = p + yk;
        return {t, (t - p) - yk};
    }
    __device__ static float result(T v) { return v.s < kInf ? v.s - v.c : v.s; }
};

// FP64: the operations of an IEEE double evaluation of Eq. (c) -- difference,
// product, min of three, sum -- in that order, so the result equals the FP64
// reference rounded once to FP32.  (An inadmissible cell's 1e30 x gives a
// cost of ~1e60 instead of +inf; every admissible cell has an admissible
// finite predecessor, so such values are never the minimum of one.)
struct AccF64 {
    using T = double;
    __device__ static T inf() { return kInfD; }
    __device__ static T zero() { return 0.0; }
    __device__ static T cell(float xe, float yv, T diag, T up, T left) {
        const double d = static_cast<double>(xe) - static_cast<double>(yv);
        const double t = fmin(fmin(diag, up), left);
        return d * d + t;
    }
    __device__ static float result(T v) { return static_cast<float>(v); }
};

__device__ __forceinline__ KahanCell lane_shift_down(KahanCell v, KahanCell fill) {
    return {lane_shift_down(v.s, fill.s), lane_shift_down(v.c, fill.c)};
}

// Window edges by row events.  With the skew of this wavefront, row h of
// lane l (strip rows rbase..rbase+H-1, column s - skew at step s) enters the
// window (column r-b) at step E + h and leaves it (column r+b+1) at step X + h,
// E = rbase + skew - b, X = rbase + skew + b + 1.  Consecutive lanes' events
// lie H+1 steps apart and each lane has H of each kind, so at most one lane of
// a wavefront enters and one leaves per step; each lane detects its own
// events, and the row index, read from the single active lane, is
// wave-uniform.  A row outside the window has its x replaced by 1e30 (its
// local cost overflows), so the cell loop itself carries no test.  Entries at
// columns <= 0 repeat the start-up value; events of rows past n touch cells
// that never feed row n-1.  Each move is a one-lane branch; the empty asm
// statement keeps the compiler from turning it into a select of the whole
// register vector.
struct BandEvents {
    int E, X;

    __device__ __forceinline__ void init(int rbase, int skew, int band) {
        E = rbase + skew - band;
        X = rbase + skew + band + 1;
    }

    template <int H>
    __device__ __forceinline__ void step(int s, typename XVec<H>::T &xe, const typename XVec<H>::T &xr) {
        const int he = s - E;
        if (static_cast<unsigned>(he) < static_cast<unsigned>(H)) {
            asm volatile("");
            const int h = __builtin_amdgcn_readfirstlane(he);
            xe[h] = xr[h];
        }
        const int hx = s - X;
        if (static_cast<unsigned>(hx) < static_cast<unsigned>(H)) {
            asm volatile("");
            xe[__builtin_amdgcn_readfirstlane(hx)] = kBig;
        }
    }
};

// True iff row rbase+h and column c are outside the window (off = rbase - c).
__device__ __forceinline__ bool outside(int off, int h, int band) {
    const int o = off + h;
    return o > band || o < -band;
}

constexpr int kEpoch = 16;     // steps between workgroup barriers (multi-wavefront strips)
constexpr int kRing = 64;      // LDS ring slots per wavefront boundary (>= 2*kEpoch + 2)

template <class ACC, int H, bool PERCELL, typename XT>
__device__ __forceinline__ void strip_step(int c, float yv, const XT &x, const typename ACC::T (&O)[H],
                                           typename ACC::T (&N)[H], typename ACC::T &up_in,
                                           typename ACC::T &diag_in, int rbase, int band) {
    using T = typename ACC::T;
    T diag = diag_in, up = up_in;
    const int off = rbase - c;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        float xe = x[h];
        if constexpr (PERCELL) xe = outside(off, h, band) ? kBig : xe;
        const T v = ACC::cell(xe, yv, diag, up, O[h]);
        diag = O[h];
        up = v;
        N[h] = v;
    }
}

// A value of the pass buffer as another wavefront of the workgroup last wrote
// it: an agent-scope atomic load, served by L2 (no stale cache line of an
// earlier pass, and never a scalar load).
__device__ __forceinline__ float pass_load(const float *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double pass_load(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ KahanCell pass_load(const KahanCell *p) {
    const unsigned long long v = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
    return {__uint_as_float(static_cast<unsigned>(v)), __uint_as_float(static_cast<unsigned>(v >> 32))};
}

// Pairs whose shorter series has more rows than the workgroup holds (n >
// 64HG) are swept in row passes of 64HG rows: pass p covers rows [pR, pR+R)
// over every column, with lane 0 of wavefront 0 reading the row above, pR-1,
// from a global buffer of the workgroup (m values) that the last lane of the
// last wavefront of pass p-1 wrote, and writing its own last row over it.  At
// every column the read comes dozens of steps before the write (the skew of
// the workgroup's lanes), in program order for one wavefront and across
// barriers for several; between passes a fence and a barrier make the row
// visible.  Values in the buffer are absolute (plus the base, for rebased
// sums).  PASSES = false instantiates the single-pass sweep alone (no buffer;
// every pair fits), which needs fewer registers.
template <class ACC, int H, int G, bool BANDED, bool PASSES>
__device__ __forceinline__ void strip_item(const WaveItem it, const float *__restrict__ ws,
                                           const SeriesInfo *__restrict__ ser, const DatasetInfo *__restrict__ dsi,
                                           typename ACC::T (*ring)[kRing], float *bound,
                                           typename ACC::T *__restrict__ pbuf) {
    using T = typename ACC::T;
    constexpr bool EVENTS = BANDED && H <= 32;  // wider strips test every cell
    constexpr bool PERCELL = BANDED && !EVENTS;
    constexpr int D = G > 1 ? kEpoch : 0;
    constexpr int CAP = 64 * H * G;  // rows of one pass
    typedef typename XVec<H>::T xvec;

    const int lane = item_lane(it.ds) & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform within a wavefront
    const DatasetInfo DI = dsi[it.ds];
    const SeriesInfo sr = ser[DI.series_base + it.rows];
    const SeriesInfo sc = ser[DI.series_base + it.cols];
    const int n = sr.len, m = sc.len, band = it.band;
    const float *__restrict__ xp = ws + sr.pstart;
    const float *__restrict__ yp = ws + sc.pstart;
    const int skew = lane + wave * (64 + D);  // column = s - skew
    const int npass = PASSES ? (n + CAP - 1) / CAP : 1;

    for (int pass = 0; pass < npass; ++pass) {
        const int P = pass * CAP;  // first row of the pass
        const bool last = !PASSES || pass == npass - 1;
        const bool top = PASSES && pass > 0 && wave == 0;  // lane 0 reads the row above from pbuf
        const int rbase = P + (wave * 64 + lane) * H;
        const int rl = (last ? n - 1 : P + CAP - 1) - P;  // the pass's last row, local
        const int Lf = rl / H, wf = Lf >> 6, lf = Lf & 63, hf = rl - Lf * H;
        const int sfinal = (m - 1) + lf + wf * (64 + D);  // step computing (last row, m-1)

        float xa[H];
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int r = rbase + h;
            const float v = xp[r < n ? r : n - 1];
            xa[h] = r < n ? v : 0.0f;  // rows past n never feed row n-1
        }
        xvec xr, x;
        T A[H], Bv[H];
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int r = rbase + h;
            xr[h] = xa[h];
            x[h] = (!EVENTS || (r < n && r - band <= 0)) ? xa[h] : kBig;
            A[h] = ACC::inf();
            Bv[h] = ACC::inf();
        }
        BandEvents ev;
        if constexpr (EVENTS) ev.init(rbase, skew, band);
        if constexpr (G > 1) {
            for (int k = threadIdx.x; k < (G - 1) * kRing; k += 64 * G) ring[k / kRing][k % kRing] = ACC::inf();
            if constexpr (kRebased<ACC>) {
                if (threadIdx.x < G) bound[threadIdx.x] = 0.0f;  // the trivial lower bound
            }
            __syncthreads();
        }
        float base = 0.0f;     // rebased accumulation only: the wavefront's base
        float top_min = kInf;  // rebased passes after the first: the smallest value of the row above
        if constexpr (kRebased<ACC>) {
            if (top) {
                for (int c = lane; c < m; c += 64) top_min = fminf(top_min, pass_load(pbuf + c));
                top_min = wave_min(top_min);
            }
        }
        // value of the row above at column c (lane 0 of wavefront 0, passes after the first)
        auto top_at = [&](int c) -> T {
            if constexpr (PASSES) {
                if (c < 0 || c >= m) return ACC::inf();
                if constexpr (kRebased<ACC>) return pass_load(pbuf + c) - base;
                return pass_load(pbuf + c);
            }
            return ACC::inf();
        };
        T up_in = ACC::inf();
        if (top) up_in = lane == 0 ? top_at(0) : ACC::inf();
        T diag_in = (lane == 0 && wave == 0 && pass == 0) ? ACC::zero() : ACC::inf();  // c(0,0), 1-based

        // y of column s - skew; the +inf pads cover the columns a single wavefront
        // reads ([-63, m+64]), later wavefronts clamp into [-1, m]
        auto yat = [&](int s) {
            const int c = s - skew;
            if constexpr (G == 1) return yp[c];
            return yp[c < -1 ? -1 : (c > m ? m : c)];
        };
        // value handed to lane 0 of this wavefront: the LDS ring for wavefronts after
        // the first, the row above from pbuf for the first wavefront of a later pass
        // (column s for its lane 0, whose skew is 0)
        auto boundary = [&](int s) -> T {
            if constexpr (G > 1) {
                if (wave > 0) {
                    if constexpr (kRebased<ACC>) return ring[wave - 1][(s - skew) & (kRing - 1)] - base;
                    return ring[wave - 1][(s - skew) & (kRing - 1)];
                }
            }
            if (top) return top_at(s);
            return ACC::inf();
        };
        auto publish = [&](int s, const T &bottom) {
            if constexpr (G > 1) {
                if (lane == 63 && wave < G - 1) {
                    if constexpr (kRebased<ACC>)
                        ring[wave][(s - skew) & (kRing - 1)] = bottom + base;
                    else
                        ring[wave][(s - skew) & (kRing - 1)] = bottom;
                }
            }
            if (PASSES && !last && lane == 63 && wave == G - 1) {  // the pass's last row, for the next pass
                const int c = s - skew;
                if (c >= 0 && c < m) {
                    if constexpr (kRebased<ACC>)
                        pbuf[c] = bottom + base;
                    else
                        pbuf[c] = bottom;
                }
            }
        };

        // Every wavefront of the workgroup runs steps 0..sfinal (a uniform count,
        // so all reach the same barriers); the result is read after the last step.
        float y0 = yat(0), y1 = yat(1);
        int s = 0;
        for (; s + 2 <= sfinal + 1; s += 2) {
            const float y2 = yat(s + 2), y3 = yat(s + 3);
            const T b1 = boundary(s + 1), b2 = boundary(s + 2);
            if constexpr (EVENTS) ev.step<H>(s, x, xr);
            strip_step<ACC, H, PERCELL>(s - skew, y0, x, A, Bv, up_in, diag_in, rbase, band);
            {
                const T recv = lane_shift_down(Bv[H - 1], b1);
                publish(s, Bv[H - 1]);
                diag_in = up_in;
                up_in = recv;
            }
            if constexpr (EVENTS) ev.step<H>(s + 1, x, xr);
            strip_step<ACC, H, PERCELL>(s + 1 - skew, y1, x, Bv, A, up_in, diag_in, rbase, band);
            {
                const T recv = lane_shift_down(A[H - 1], b2);
                publish(s + 1, A[H - 1]);
                diag_in = up_in;
                up_in = recv;
            }
            if constexpr (kRebased<ACC>) {
                if ((s + 2) % kRebaseSteps == 0) {
                    float held = fminf(up_in, diag_in);
                    if constexpr (G > 1) {
                        if (wave > 0) held = fminf(held, fminf(ring[wave - 1][lane], bound[wave - 1]) - base);
                    }
                    if (top) held = fminf(held, top_min - base);
                    float floor;
                    const float d = rebase_wave<H>(A, held, base, floor);
                    up_in -= d;
                    diag_in -= d;
                    if constexpr (G > 1) {
                        if (lane == 0) bound[wave] = floor;
                    }
                }
            }
            y0 = y2;
            y1 = y3;
            if constexpr (G > 1) {
                if ((s + 2) % kEpoch == 0) __syncthreads();
            }
        }
        T res;
        if (s <= sfinal) {  // one step left (s == sfinal)
            if constexpr (EVENTS) ev.step<H>(s, x, xr);
            strip_step<ACC, H, PERCELL>(s - skew, y0, x, A, Bv, up_in, diag_in, rbase, band);
            publish(s, Bv[H - 1]);
            res = pick<H>(Bv, hf);
        } else {
            res = pick<H>(A, hf);
        }
        if (PASSES && !last) {
            // the row is written: make it visible to every wavefront before the next pass
            __threadfence();
            __syncthreads();
            continue;
        }
        if (wave == wf && lane == lf) {
            if constexpr (kRebased<ACC>)
                DI.out[it.slot] = res + base;
            else
                DI.out[it.slot] = ACC::result(res);
        }
    }
}

// Unwindowed strips, two columns per step.  Lane l of wavefront g handles
// columns c0 = 2u - (m & 1) and c0 + 1, u = t - l - g(64+D), at step t (the
// pairing puts the last column m-1 second in its pair; a column -1 reads the
// +inf pad and stays +inf).  Within the step the two columns are evaluated
// interleaved with a one-row lag -- cell (h, c0), then (h-1, c0+1) -- so each
// lane runs two independent dependency chains, and the second column is
// written over the first one's predecessor in place: the state is H cells
// plus three, not 2H.  Both bottom cells go down one lane per step (two DPP
// moves); between wavefronts both go through the LDS ring.
template <class ACC, int H, int G>
__device__ __forceinline__ void strip2_item(const WaveItem it, const float *__restrict__ ws,
                                            const SeriesInfo *__restrict__ ser, const DatasetInfo *__restrict__ dsi,
                                            typename ACC::T (*ring)[kRing], float *bound) {
    using T = typename ACC::T;
    constexpr int D = G > 1 ? kEpoch : 0;

    const int lane = item_lane(it.ds) & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const DatasetInfo DI = dsi[it.ds];
    const SeriesInfo sr = ser[DI.series_base + it.rows];
    const SeriesInfo sc = ser[DI.series_base + it.cols];
    const int n = sr.len, m = sc.len;
    const float *__restrict__ xp = ws + sr.pstart;
    const float *__restrict__ yp = ws + sc.pstart;
    const int rbase = (wave * 64 + lane) * H;
    const int shift = m & 1;
    const int skew = lane + wave * (64 + D);  // u = t - skew
    const int Lf = (n - 1) / H, wf = Lf >> 6, lf = Lf & 63, hf = (n - 1) - Lf * H;
    const int tfinal = (m - 2 + shift) / 2 + lf + wf * (64 + D);  // step whose second column is m-1

    float x[H];
    T A[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int r = rbase + h;
        const float v = xp[r < n ? r : n - 1];
        x[h] = r < n ? v : 0.0f;  // rows past n never feed row n-1
        A[h] = ACC::inf();
    }
    if constexpr (G > 1) {
        for (int k = threadIdx.x; k < (G - 1) * kRing; k += 64 * G) ring[k / kRing][k % kRing] = ACC::inf();
        if constexpr (kRebased<ACC>) {
            if (threadIdx.x < G) bound[threadIdx.x] = 0.0f;  // the trivial lower bound
        }
        __syncthreads();
    }
    // Row -1 as seen by lane 0 of wavefront 0: +inf, except c(0,0) = 0 of the
    // 1-based recurrence, the diagonal of column 0.
    const bool corner = lane == 0 && wave == 0;
    T recv0 = (corner && shift) ? ACC::zero() : ACC::inf();   // bottom of column c0 from the lane above
    T recv1 = ACC::inf();                                     // bottom of column c0 + 1
    T prev1 = (corner && !shift) ? ACC::zero() : ACC::inf();  // bottom of column c0 - 1
    float base = 0.0f;  // rebased accumulation only: the wavefront's base

    auto col_of = [&](int t) { return 2 * (t - skew) - shift; };  // first column of step t
    // y of column c: a single wavefront reads columns [-127, m+127] (inside
    // the +inf pads); later wavefronts clamp into [-1, m]
    auto yv = [&](int c) -> float {
        if constexpr (G == 1) return yp[c];
        return yp[c < -1 ? -1 : (c > m ? m : c)];
    };
    auto boundary = [&](int t, int k) -> T {  // lane 0's up value for column k of step t
        if constexpr (G > 1) {
            if (wave > 0) {
                if constexpr (kRebased<ACC>) return ring[wave - 1][(col_of(t) + k) & (kRing - 1)] - base;
                return ring[wave - 1][(col_of(t) + k) & (kRing - 1)];
            }
        }
        return ACC::inf();
    };
    auto publish = [&](int t, const T &b0, const T &b1) {
        if constexpr (G > 1) {
            if (lane == 63 && wave < G - 1) {
                const int c = col_of(t);
                if constexpr (kRebased<ACC>) {
                    ring[wave][c & (kRing - 1)] = b0 + base;
                    ring[wave][(c + 1) & (kRing - 1)] = b1 + base;
                } else {
                    ring[wave][c & (kRing - 1)] = b0;
                    ring[wave][(c + 1) & (kRing - 1)] = b1;
                }
            }
        }
    };

    const int c = col_of(0);
    float y0 = yv(c), y1 = yv(c + 1);
    for (int t = 0; t <= tfinal; ++t) {
        const int cn = col_of(t + 1);
        const float n0 = yv(cn), n1 = yv(cn + 1);
        // column c0: diag = prev1 (row -1 of column c0-1), up = recv0; column c0+1: diag = recv0, up = recv1
        T bm1 = ACC::inf(), bm2 = ACC::inf();
#pragma unroll
        for (int h = 0; h <= H; ++h) {
            T bh = ACC::inf();
            if (h < H) bh = ACC::cell(x[h], y0, h == 0 ? prev1 : A[h - 1], h == 0 ? recv0 : bm1, A[h]);
            if (h >= 1) {
                const int g = h - 1;
                A[g] = ACC::cell(x[g], y1, g == 0 ? recv0 : bm2, g == 0 ? recv1 : A[g - 1 < 0 ? 0 : g - 1], bm1);
            }
            if (h < H) {
                bm2 = bm1;
                bm1 = bh;
            }
        }
        // bm1 = column c0 row H-1, A[H-1] = column c0+1 row H-1
        publish(t, bm1, A[H - 1]);
        prev1 = recv1;
        recv0 = lane_shift_down(bm1, boundary(t + 1, 0));
        recv1 = lane_shift_down(A[H - 1], boundary(t + 1, 1));
        if constexpr (kRebased<ACC>) {
            if ((t + 1) % kRebaseSteps2 == 0) {
                float held = fminf(fminf(recv0, recv1), prev1);
                if constexpr (G > 1) {
                    if (wave > 0) held = fminf(held, fminf(ring[wave - 1][lane], bound[wave - 1]) - base);
                }
                float floor;
                const float d = rebase_wave<H>(A, held, base, floor);
                recv0 -= d;
                recv1 -= d;
                prev1 -= d;
                if constexpr (G > 1) {
                    if (lane == 0) bound[wave] = floor;
                }
            }
        }
        y0 = n0;
        y1 = n1;
        if constexpr (G > 1) {
            if ((t + 1) % kEpoch == 0) __syncthreads();
        }
    }
    if (wave == wf && lane == lf) {
        if constexpr (kRebased<ACC>)
            DI.out[it.slot] = pick<H>(A, hf) + base;
        else
            DI.out[it.slot] = ACC::result(pick<H>(A, hf));
    }
}

// PASSES: pairs with more rows than 64*H*G may occur, swept in row passes
// through pass_buf, pass_stride values of ACC::T per workgroup (blockIdx.x).
template <class ACC, int H, int G, bool BANDED, bool PASSES>
__global__ __launch_bounds__(64 * G) void k_strip(const float *__restrict__ ws, const SeriesInfo *__restrict__ ser,
                                                  const DatasetInfo *__restrict__ dsi,
                                                  const WaveItem *__restrict__ items, unsigned *__restrict__ queue,
                                                  unsigned n_items, void *pass_buf, int64_t pass_stride) {
    __shared__ typename ACC::T ring[G > 1 ? G - 1 : 1][kRing];
    __shared__ float bound[G];  // rebased multi-wavefront strips: each wavefront's last base
    __shared__ unsigned slot;
    unsigned idx = blockIdx.x;
    for (;;) {
        if (queue) idx = next_item<G>(queue, &slot);
        if (idx >= n_items) break;
        // unwindowed plain FP32 strips take two columns per step; the
        // compensated and FP64 cells already hold enough independent work
        // per cell (measured slower in the two-column form)
        typename ACC::T *pbuf =
            PASSES ? static_cast<typename ACC::T *>(pass_buf) + (int64_t)blockIdx.x * pass_stride : nullptr;
        if constexpr (!BANDED && (std::is_same<ACC, AccPlain>::value || kRebased<ACC>)) {
            if (!PASSES || ser[dsi[items[idx].ds].series_base + items[idx].rows].len <= 64 * H * G)
                strip2_item<ACC, H, G>(items[idx], ws, ser, dsi, ring, bound);
            else  // several row passes: the one-column sweep
                strip_item<ACC, H, G, BANDED, PASSES>(items[idx], ws, ser, dsi, ring, bound, pbuf);
        } else {
            strip_item<ACC, H, G, BANDED, PASSES>(items[idx], ws, ser, dsi, ring, bound, pbuf);
        }
        if (!queue) break;
    }
}

template <class ACC, int H, int G>
hipError_t strip_launch(bool banded, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                        const WaveItem *items, unsigned n, unsigned *queue, unsigned grid, void *pass_buf,
                        int64_t pass_stride, hipStream_t st) {
    const dim3 g(grid), block(64 * G);
    if (banded && pass_buf)
        hipLaunchKernelGGL((k_strip<ACC, H, G, true, true>), g, block, 0, st, ws, ser, dsi, items, queue, n,
                           pass_buf, pass_stride);
    else if (banded)
        hipLaunchKernelGGL((k_strip<ACC, H, G, true, false>), g, block, 0, st, ws, ser, dsi, items, queue, n,
                           nullptr, 0);
    else if (pass_buf)
        hipLaunchKernelGGL((k_strip<ACC, H, G, false, true>), g, block, 0, st, ws, ser, dsi, items, queue, n,
                           pass_buf, pass_stride);
    else
        hipLaunchKernelGGL((k_strip<ACC, H, G, false, false>), g, block, 0, st, ws, ser, dsi, items, queue, n,
                           nullptr, 0);
    return hipGetLastError();
}

template <class ACC, int H, int G>
int strip_slots(bool banded, bool passes) {
    const void *k = banded ? (passes ? reinterpret_cast<const void *>(&k_strip<ACC, H, G, true, true>)
                                     : reinterpret_cast<const void *>(&k_strip<ACC, H, G, true, false>))
                           : (passes ? reinterpret_cast<const void *>(&k_strip<ACC, H, G, false, true>)
                                     : reinterpret_cast<const void *>(&k_strip<ACC, H, G, false, false>));
    return resident_blocks(k, 64 * G);
}

}  // namespace

using StripFn = hipError_t (*)(bool, const float *, const SeriesInfo *, const DatasetInfo *, const WaveItem *,
                               unsigned, unsigned *, unsigned, void *, int64_t, hipStream_t);
using StripSlotsFn = int (*)(bool, bool);
struct StripEntry {  // one instantiated strip shape of an accumulation mode (AccMode)
    int accum, H, G;
    StripFn fn;
    StripSlotsFn slots;
};

#define DTWMI_STRIP(A, ACC, H, G) {A, H, G, &strip_launch<ACC, H, G>, &strip_slots<ACC, H, G>}

// The FP64 shapes (dtw_strip_f64.hip): sets *out and returns their number.
int strip_f64_entries(const StripEntry **out);

}  // namespace dtwmi
