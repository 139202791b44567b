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
// Two kernel families:
//  * lane-band (k_lane): one pair per lane.  All 64 lanes of a wavefront share
//    the column series y (wave-uniform, read with scalar loads) and each lane
//    has its own row series x.  The DP is swept row by row in band
//    coordinates k = j - i + B, so the 2B+1 band cells of a row live in
//    registers and are updated in place:  new[k] = cost + min3(old[k] (diag),
//    old[k+1] (up), new[k-1] (left)).  Columns outside [0,m) read +inf pads.
//  * wavefront (k_wave_*): one pair per wavefront.  Lane l owns rows
//    [l*H, l*H+H) and at step s processes column s-l (anti-diagonal skew), so
//    a whole strip column is updated per step with the boundary row passed to
//    the next lane by a DPP wave_shr:1 move.  State is 2H registers (ping-pong
//    over two steps, FP32) or H registers updated in place (FP64, Kahan).
#include "dtw_internal.h"

#include <array>
#include <utility>

namespace dtwmi {
namespace {

constexpr float kInf = __builtin_huge_valf();
constexpr float kBig = 1.0e30f;    // x value of an inadmissible cell: (kBig - y)^2 overflows to +inf
constexpr double kInfD = __builtin_huge_val();
constexpr double kBigD = 1.0e300;  // same for FP64

__device__ __forceinline__ float min3f(float a, float b, float c) { return fminf(fminf(a, b), c); }

// Lane i receives v from lane i-1; lane 0 receives `fill` (DPP wave_shr:1, bound_ctrl off).
__device__ __forceinline__ float lane_shift_down(float v, float fill) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v),
                                                      0x138, 0xF, 0xF, false));
}

__device__ __forceinline__ double lane_shift_down(double v, double fill) {
    const long long vb = __double_as_longlong(v), fb = __double_as_longlong(fill);
    const int lo = __builtin_amdgcn_update_dpp((int)(fb & 0xffffffff), (int)(vb & 0xffffffff), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(fb >> 32), (int)(vb >> 32), 0x138, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int64_t condensed_index(int i, int j, int N) {
    // i < j
    return (int64_t)i * N - (int64_t)i * (i + 1) / 2 + (j - i - 1);
}

// ---------------------------------------------------------------------------
// Staging: copy every series into its padded FP32 slot, widening 16-bit types
// exactly, with +inf in the pads.
// ---------------------------------------------------------------------------
// Work distribution.  Without a queue a workgroup takes item blockIdx.x and
// exits.  With a queue (a counter zeroed by k_zero before the launch) a grid
// of resident workgroups pulls item indices with one atomic add each, in the
// order the planner sorted the items (decreasing cost), until the counter
// passes n_items.  The index is made wave-uniform so the item's fields stay
// in scalar registers.
template <int G>
__device__ __forceinline__ unsigned next_item(unsigned *__restrict__ queue, unsigned *s_slot) {
    if constexpr (G == 1) {
        unsigned v = 0;
        if (threadIdx.x == 0) v = atomicAdd(queue, 1u);
        return __builtin_amdgcn_readfirstlane(v);
    } else {
        if (threadIdx.x == 0) *s_slot = atomicAdd(queue, 1u);
        __syncthreads();
        const unsigned v = __builtin_amdgcn_readfirstlane(*s_slot);
        __syncthreads();  // every wavefront has read the slot before it is written again
        return v;
    }
}

// threadIdx.x as a value the compiler cannot see to be the same for every
// item (it.ds >= 0, so the min is 0): keeps lane-derived per-row constants
// inside the item loop instead of holding them in registers across items.
__device__ __forceinline__ int item_lane(int ds) { return static_cast<int>(threadIdx.x) + min(ds, 0); }

__global__ __launch_bounds__(64) void k_zero(unsigned *__restrict__ p, int n) {
    for (int i = threadIdx.x; i < n; i += 64) p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_stage(const SeriesSrc *__restrict__ src,
                                               const SeriesInfo *__restrict__ ser,
                                               float *__restrict__ ws) {
    const int g = blockIdx.x;
    const SeriesSrc s = src[g];
    const SeriesInfo si = ser[g];
    float *dst = ws + si.pstart - kPad;
    const int total = (si.len + 2 * kPad + 3) & ~3;
    for (int p = threadIdx.x; p < total; p += blockDim.x) {
        const int t = p - kPad;
        float v = kInf;
        if (t >= 0 && t < s.len) {
            if (s.dtype == 0) {
                v = static_cast<const float *>(s.base)[s.off + t];
            } else if (s.dtype == 1) {
                const unsigned short b = static_cast<const unsigned short *>(s.base)[s.off + t];
                v = __uint_as_float(static_cast<unsigned int>(b) << 16);
            } else {
                v = static_cast<float>(static_cast<const _Float16 *>(s.base)[s.off + t]);
            }
        }
        dst[p] = v;
    }
}

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
// column L-1 are never read by an admissible cell.
#ifndef DTWMI_LANE_ROWS
#define DTWMI_LANE_ROWS 4
#endif
#ifndef DTWMI_LANE_CHUNK
#define DTWMI_LANE_CHUNK 16
#endif
constexpr int kLaneRows = DTWMI_LANE_ROWS;
constexpr int kLaneChunk = DTWMI_LANE_CHUNK;

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

// Lane-band items have equal cost, so the kernel takes one item per workgroup
// (hardware dispatch); an item loop would only add registers to this kernel.
template <int W>
__global__ __launch_bounds__(64) void k_lane(const float *__restrict__ ws, const SeriesInfo *__restrict__ ser,
                                             const DatasetInfo *__restrict__ dsi,
                                             const LaneItem *__restrict__ items) {
    constexpr int B = (W - 1) / 2, R = kLaneRows, C = kLaneChunk;
    const LaneItem it = items[blockIdx.x];
    const DatasetInfo D = dsi[it.ds];
    const int lane = threadIdx.x;
    const bool valid = lane < it.cnt;
    int bl = it.a + it.d0 + lane;
    bl = bl >= D.N ? bl - D.N : bl;
    if (!valid) bl = it.a;  // idle lanes recompute a valid pair and store nothing
    const float *__restrict__ ycol = ws + ser[D.series_base + it.a].pstart - B;  // ycol[v] = y[v-B]
    const float *__restrict__ xrow = ws + ser[D.series_base + bl].pstart;
    const int L = D.L;

    float st[W];
#pragma unroll
    for (int k = 0; k < W; ++k) st[k] = kInf;
    st[B] = 0.0f;  // c(0,0) of the 1-based recurrence, seen as the diagonal of cell (1,1)

    int i = 0;
    if (L >= R) {
        float ycur[C + R - 1];
#pragma unroll
        for (int u = 0; u < C + R - 1; ++u) ycur[u] = ycol[u - (R - 1)];
        float x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = xrow[r];
        for (; i + R <= L; i += R) {
            float xn[R];  // next group's x, requested one group ahead (stays inside the pad)
#pragma unroll
            for (int r = 0; r < R; ++r) xn[r] = xrow[i + R + r];
            lane_group<W, R, C, 0>(st, x, ycol + i - (R - 1), ycol + i + 1, ycur, i - B, L);
#pragma unroll
            for (int r = 0; r < R; ++r) x[r] = xn[r];
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

    if (valid) {
        const int a = it.a < bl ? it.a : bl, b = it.a < bl ? bl : it.a;
        D.out[condensed_index(a, b, D.N)] = st[B];
    }
}


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

// v[h] for a wave-uniform runtime h, as a tree of selects on the bits of h
// (a plain indexed read would push the whole register array to scratch).
template <int H, typename T>
__device__ __forceinline__ T pick(const T (&v)[H], int h) {
    constexpr int P = H <= 1 ? 1 : (H <= 2 ? 2 : (H <= 4 ? 4 : (H <= 8 ? 8 : (H <= 16 ? 16 : (H <= 32 ? 32 : 64)))));
    T t[P];
#pragma unroll
    for (int k = 0; k < P; ++k) t[k] = v[k < H ? k : H - 1];
#pragma unroll
    for (int width = P / 2, bit = 0; width >= 1; width /= 2, ++bit) {
        const bool hi = (h >> bit) & 1;
#pragma unroll
        for (int k = 0; k < width; ++k) t[k] = hi ? t[2 * k + 1] : t[2 * k];
    }
    return t[0];
}

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

// Kahan-compensated FP32: each cell carries (s, c) with the true value close
// to s - c.  The min compares the running sums s (ties prefer diag, then up,
// then left) and takes the compensation of the chosen predecessor; the local
// cost is then added with Kahan's compensated step.  An unreachable cell (s =
// +inf) gets c = NaN from inf - inf; that is harmless: a reachable cell has a
// finite predecessor, fminf ignores quiet NaNs and NaN never compares equal,
// so such a c is never selected.
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
        const float c1 = (p == up.s) ? up.c : left.c;
        const float cs = (p == diag.s) ? diag.c : c1;
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

// Window edges by row events.  With the skew of this wavefront, a row of the
// strip enters the window (column r-b) at step l(H+1)+h-be and leaves it
// (column r+b+1) at step l(H+1)+h+bx+1, where l, h are the wave-local lane and
// strip row and be, bx are the band shifted by the wavefront's offset: at most
// one row enters and one row leaves per step, and the lane and strip row of
// each event are wave-uniform.  A row outside the window has its x replaced
// by 1e30 (its local cost overflows), so the cell loop itself carries no test.
// x lives in a register vector so that an event's uniform row index becomes
// one indexed register move (s_set_gpr_idx) instead of a test per cell.
// (At least 16 elements: the compiler turns an indexed move into a chain of
// compares and selects for smaller vectors.)
template <int H>
struct XVec {
    typedef float T __attribute__((ext_vector_type(H < 16 ? 16 : H)));
};

struct RowCounter {  // t = s + off written as q(H+1) + h with 0 <= h <= H (q < 0 before the first event)
    int q, h;
    template <int H>
    __device__ __forceinline__ void init(int off) {
        q = off >= 0 ? off / (H + 1) : -((-off + H) / (H + 1));
        h = off - q * (H + 1);
    }
    template <int H>
    __device__ __forceinline__ void advance() {
        if (++h == H + 1) {
            h = 0;
            ++q;
        }
    }
};

struct BandEvents {
    RowCounter en, ex;
    int nloc, col_shift;  // rows of the pair from this wavefront's first row; column = s - l - col_shift

    template <int H>
    __device__ __forceinline__ void init(int band, int n_rows, int wave, int D) {
        const int row0 = wave * 64 * H;
        nloc = n_rows - row0;
        col_shift = wave * (64 + D);
        const int shift = row0 + col_shift;
        en.init<H>(band - shift);       // entry at step s: s + b - shift = l(H+1) + h
        ex.init<H>(-band - shift - 1);  // exit at step s:  s - b - shift - 1 = l(H+1) + h
    }

    // Apply the events of step s (counters are at step s on entry), then advance.
    template <int H>
    __device__ __forceinline__ void step(int s, typename XVec<H>::T &xe, const typename XVec<H>::T &xr, int lane) {
        if (en.h < H && en.q >= 0 && en.q < 64 && en.q * H + en.h < nloc && s - en.q - col_shift > 0) {
            const float cur = xe[en.h];
            const float v = xr[en.h];
            xe[en.h] = lane == en.q ? v : cur;
        }
        en.advance<H>();
        if (ex.h < H && ex.q >= 0 && ex.q < 64 && ex.q * H + ex.h < nloc) {
            const float cur = xe[ex.h];
            xe[ex.h] = lane == ex.q ? kBig : cur;
        }
        ex.advance<H>();
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

template <class ACC, int H, int G, bool BANDED>
__device__ __forceinline__ void strip_item(const WaveItem it, const float *__restrict__ ws,
                                           const SeriesInfo *__restrict__ ser, const DatasetInfo *__restrict__ dsi,
                                           typename ACC::T (*ring)[kRing]) {
    using T = typename ACC::T;
    constexpr bool EVENTS = BANDED && H <= 32;  // wider strips test every cell
    constexpr bool PERCELL = BANDED && !EVENTS;
    constexpr int D = G > 1 ? kEpoch : 0;
    typedef typename XVec<H>::T xvec;

    const int lane = item_lane(it.ds) & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform within a wavefront
    const DatasetInfo DI = dsi[it.ds];
    const SeriesInfo sr = ser[DI.series_base + it.rows];
    const SeriesInfo sc = ser[DI.series_base + it.cols];
    const int n = sr.len, m = sc.len, band = it.band;
    const float *__restrict__ xp = ws + sr.pstart;
    const float *__restrict__ yp = ws + sc.pstart;
    const int rbase = (wave * 64 + lane) * H;
    const int skew = lane + wave * (64 + D);  // column = s - skew
    const int Lf = (n - 1) / H, wf = Lf >> 6, lf = Lf & 63, hf = (n - 1) - Lf * H;
    const int sfinal = (m - 1) + lf + wf * (64 + D);  // step computing cell (n-1, m-1)

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
    if constexpr (EVENTS) ev.init<H>(band, n, wave, D);
    if constexpr (G > 1) {
        for (int k = threadIdx.x; k < (G - 1) * kRing; k += 64 * G) ring[k / kRing][k % kRing] = ACC::inf();
        __syncthreads();
    }
    T up_in = ACC::inf();
    T diag_in = (lane == 0 && wave == 0) ? ACC::zero() : ACC::inf();  // c(0,0) of the 1-based recurrence

    // y of column s - skew; the +inf pads cover the columns a single wavefront
    // reads ([-63, m+64]), later wavefronts clamp into [-1, m]
    auto yat = [&](int s) {
        const int c = s - skew;
        if constexpr (G == 1) return yp[c];
        return yp[c < -1 ? -1 : (c > m ? m : c)];
    };
    // value handed to lane 0 of this wavefront (LDS ring for wavefronts after the first)
    auto boundary = [&](int s) -> T {
        if constexpr (G > 1) {
            if (wave > 0) return ring[wave - 1][(s - skew) & (kRing - 1)];
        }
        return ACC::inf();
    };
    auto publish = [&](int s, const T &bottom) {
        if constexpr (G > 1) {
            if (lane == 63 && wave < G - 1) ring[wave][(s - skew) & (kRing - 1)] = bottom;
        }
    };

    // Every wavefront of the workgroup runs steps 0..sfinal (a uniform count,
    // so all reach the same barriers); the result is read after the last step.
    float y0 = yat(0), y1 = yat(1);
    int s = 0;
    for (; s + 2 <= sfinal + 1; s += 2) {
        const float y2 = yat(s + 2), y3 = yat(s + 3);
        if constexpr (EVENTS) ev.step<H>(s, x, xr, lane);
        strip_step<ACC, H, PERCELL>(s - skew, y0, x, A, Bv, up_in, diag_in, rbase, band);
        {
            const T recv = lane_shift_down(Bv[H - 1], boundary(s + 1));
            publish(s, Bv[H - 1]);
            diag_in = up_in;
            up_in = recv;
        }
        if constexpr (EVENTS) ev.step<H>(s + 1, x, xr, lane);
        strip_step<ACC, H, PERCELL>(s + 1 - skew, y1, x, Bv, A, up_in, diag_in, rbase, band);
        {
            const T recv = lane_shift_down(A[H - 1], boundary(s + 2));
            publish(s + 1, A[H - 1]);
            diag_in = up_in;
            up_in = recv;
        }
        y0 = y2;
        y1 = y3;
        if constexpr (G > 1) {
            if ((s + 2) % kEpoch == 0) __syncthreads();
        }
    }
    T res;
    if (s <= sfinal) {  // one step left (s == sfinal)
        if constexpr (EVENTS) ev.step<H>(s, x, xr, lane);
        strip_step<ACC, H, PERCELL>(s - skew, y0, x, A, Bv, up_in, diag_in, rbase, band);
        res = pick<H>(Bv, hf);
    } else {
        res = pick<H>(A, hf);
    }
    if (wave == wf && lane == lf) {
        const int a = it.rows < it.cols ? it.rows : it.cols;
        const int b = it.rows < it.cols ? it.cols : it.rows;
        DI.out[condensed_index(a, b, DI.N)] = ACC::result(res);
    }
}

template <class ACC, int H, int G, bool BANDED>
__global__ __launch_bounds__(64 * G) void k_strip(const float *__restrict__ ws, const SeriesInfo *__restrict__ ser,
                                                  const DatasetInfo *__restrict__ dsi,
                                                  const WaveItem *__restrict__ items, unsigned *__restrict__ queue,
                                                  unsigned n_items) {
    __shared__ typename ACC::T ring[G > 1 ? G - 1 : 1][kRing];
    __shared__ unsigned slot;
    unsigned idx = blockIdx.x;
    for (;;) {
        if (queue) idx = next_item<G>(queue, &slot);
        if (idx >= n_items) break;
        strip_item<ACC, H, G, BANDED>(items[idx], ws, ser, dsi, ring);
        if (!queue) break;
    }
}

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
        c.g += 64;
        cyc_setup<H>(c, xr, x, xp, n, m, b);
        y0 = cyc_y(yp, s - c.yb);
        y1 = cyc_y(yp, s + 1 - c.yb);
        y2 = cyc_y(yp, s + 2 - c.yb);
        y3 = cyc_y(yp, s + 3 - c.yb);
#pragma unroll
        for (int h = 0; h < H; ++h) O[h] = kInf;
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
    if (lane == (Qf & 63)) {
        const int a = it.rows < it.cols ? it.rows : it.cols;
        const int bb = it.rows < it.cols ? it.cols : it.rows;
        DI.out[condensed_index(a, bb, DI.N)] = res;
    }
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

// ---------------------------------------------------------------------------
// Launch tables.  Every DP launcher takes the item count, the queue counter
// (nullptr: one workgroup per item) and the grid size; its resident function
// gives the workgroups of that kernel the device holds at once.
int resident_blocks(const void *fn, int block) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, block, 0) != hipSuccess) return 0;
    return cus * per;
}

using LaneFn = hipError_t (*)(const float *, const SeriesInfo *, const DatasetInfo *, const LaneItem *, unsigned,
                              hipStream_t);
using SlotsFn = int (*)();

template <int I>
hipError_t lane_launcher(const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi, const LaneItem *items,
                         unsigned n, hipStream_t st) {
    hipLaunchKernelGGL(k_lane<2 * I + 1>, dim3(n), dim3(64), 0, st, ws, ser, dsi, items);
    return hipGetLastError();
}

template <size_t... I>
constexpr std::array<LaneFn, sizeof...(I)> make_lane_table(std::index_sequence<I...>) {
    return {{&lane_launcher<static_cast<int>(I)>...}};
}

const std::array<LaneFn, (kLaneMaxW + 1) / 2> kLaneTable =
    make_lane_table(std::make_index_sequence<(kLaneMaxW + 1) / 2>{});

template <class ACC, int H, int G>
hipError_t strip_launch(bool banded, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                        const WaveItem *items, unsigned n, unsigned *queue, unsigned grid, hipStream_t st) {
    const dim3 g(grid), block(64 * G);
    if (banded)
        hipLaunchKernelGGL((k_strip<ACC, H, G, true>), g, block, 0, st, ws, ser, dsi, items, queue, n);
    else
        hipLaunchKernelGGL((k_strip<ACC, H, G, false>), g, block, 0, st, ws, ser, dsi, items, queue, n);
    return hipGetLastError();
}

template <class ACC, int H, int G>
int strip_slots(bool banded) {
    return banded ? resident_blocks(reinterpret_cast<const void *>(&k_strip<ACC, H, G, true>), 64 * G)
                  : resident_blocks(reinterpret_cast<const void *>(&k_strip<ACC, H, G, false>), 64 * G);
}

using StripFn = hipError_t (*)(bool, const float *, const SeriesInfo *, const DatasetInfo *, const WaveItem *,
                               unsigned, unsigned *, unsigned, hipStream_t);
using StripSlotsFn = int (*)(bool);
struct StripEntry {
    int accum, H, G;
    StripFn fn;
    StripSlotsFn slots;
};

#define DTWMI_STRIP(A, ACC, H, G) {A, H, G, &strip_launch<ACC, H, G>, &strip_slots<ACC, H, G>}
// Instantiated shapes, per accumulation mode in increasing row capacity 64*H*G.
const StripEntry kStrips[] = {
    DTWMI_STRIP(0, AccPlain, 1, 1),  DTWMI_STRIP(0, AccPlain, 2, 1),  DTWMI_STRIP(0, AccPlain, 4, 1),
    DTWMI_STRIP(0, AccPlain, 8, 1),  DTWMI_STRIP(0, AccPlain, 12, 1), DTWMI_STRIP(0, AccPlain, 16, 1),
    DTWMI_STRIP(0, AccPlain, 24, 1), DTWMI_STRIP(0, AccPlain, 32, 1), DTWMI_STRIP(0, AccPlain, 16, 2),
    DTWMI_STRIP(0, AccPlain, 48, 1), DTWMI_STRIP(0, AccPlain, 24, 2), DTWMI_STRIP(0, AccPlain, 64, 1),
    DTWMI_STRIP(0, AccPlain, 32, 2), DTWMI_STRIP(0, AccPlain, 32, 4), DTWMI_STRIP(0, AccPlain, 32, 8),
    DTWMI_STRIP(0, AccPlain, 64, 8),
    DTWMI_STRIP(1, AccKahan, 1, 1),  DTWMI_STRIP(1, AccKahan, 2, 1),  DTWMI_STRIP(1, AccKahan, 4, 1),
    DTWMI_STRIP(1, AccKahan, 8, 1),  DTWMI_STRIP(1, AccKahan, 16, 1), DTWMI_STRIP(1, AccKahan, 16, 2),
    DTWMI_STRIP(1, AccKahan, 16, 4), DTWMI_STRIP(1, AccKahan, 16, 8), DTWMI_STRIP(1, AccKahan, 16, 16),
    DTWMI_STRIP(2, AccF64, 1, 1),    DTWMI_STRIP(2, AccF64, 2, 1),    DTWMI_STRIP(2, AccF64, 4, 1),
    DTWMI_STRIP(2, AccF64, 8, 1),    DTWMI_STRIP(2, AccF64, 16, 1),   DTWMI_STRIP(2, AccF64, 16, 2),
    DTWMI_STRIP(2, AccF64, 16, 4),   DTWMI_STRIP(2, AccF64, 16, 8),   DTWMI_STRIP(2, AccF64, 16, 16),
};
#undef DTWMI_STRIP

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

using CycFn = hipError_t (*)(const float *, const SeriesInfo *, const DatasetInfo *, const WaveItem *, unsigned,
                             unsigned *, unsigned, hipStream_t);
struct CycEntry {
    int H;
    CycFn fn;
    SlotsFn slots;
};
const CycEntry kCyclic[] = {{1, &cyc_launch<1>, &cyc_slots<1>},    {2, &cyc_launch<2>, &cyc_slots<2>},
                            {4, &cyc_launch<4>, &cyc_slots<4>},    {8, &cyc_launch<8>, &cyc_slots<8>},
                            {12, &cyc_launch<12>, &cyc_slots<12>}, {16, &cyc_launch<16>, &cyc_slots<16>},
                            {24, &cyc_launch<24>, &cyc_slots<24>}, {32, &cyc_launch<32>, &cyc_slots<32>}};

// Grid of a launch: one workgroup per item, or with a queue the resident
// workgroups (at most one per item).
unsigned grid_for(unsigned n, unsigned *queue, int slots) {
    if (!queue || slots <= 0) return n;
    return n < static_cast<unsigned>(slots) ? n : static_cast<unsigned>(slots);
}

}  // namespace

hipError_t launch_stage(const SeriesSrc *src, const SeriesInfo *ser, float *ws, int32_t nseries,
                        hipStream_t stream) {
    if (nseries <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stage, dim3(nseries), dim3(256), 0, stream, src, ser, ws);
    return hipGetLastError();
}

hipError_t launch_zero(unsigned *p, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, stream, p, n);
    return hipGetLastError();
}

bool lane_width_supported(int W) { return W >= 1 && W <= kLaneMaxW && (W & 1); }

hipError_t launch_lane(int W, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                       const LaneItem *items, unsigned n_items, hipStream_t stream) {
    if (!lane_width_supported(W)) return hipErrorInvalidValue;
    if (n_items == 0) return hipSuccess;
    return kLaneTable[(W - 1) / 2](ws, ser, dsi, items, n_items, stream);
}

int strip_shapes(int accum, StripShape *out, int max_out) {
    int k = 0;
    for (const StripEntry &e : kStrips)
        if (e.accum == accum) {
            if (out && k < max_out) out[k] = StripShape{e.H, e.G};
            ++k;
        }
    return k;
}

int strip_resident(int accum, StripShape shape, bool banded) {
    for (const StripEntry &e : kStrips)
        if (e.accum == accum && e.H == shape.H && e.G == shape.G) return e.slots(banded);
    return 0;
}

hipError_t launch_strip(int accum, StripShape shape, bool banded, const float *ws, const SeriesInfo *ser,
                        const DatasetInfo *dsi, const WaveItem *items, unsigned n_items, unsigned *queue, int slots,
                        hipStream_t stream) {
    if (n_items == 0) return hipSuccess;
    for (const StripEntry &e : kStrips)
        if (e.accum == accum && e.H == shape.H && e.G == shape.G)
            return e.fn(banded, ws, ser, dsi, items, n_items, queue, grid_for(n_items, queue, slots), stream);
    return hipErrorInvalidValue;
}

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
