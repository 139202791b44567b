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
// Wavefront kernels.
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

// True iff row rbase+h and column c are outside the window (off = rbase - c).
__device__ __forceinline__ bool outside(int off, int h, int band) {
    const int o = off + h;
    return o > band || o < -band;
}

struct WaveSetup {
    const float *xp;
    const float *yp;  // yp[s] = y[s - lane]
    int n, m, lstar, S, hstar, band, rbase;
    float *out_at;
};

__device__ __forceinline__ WaveSetup wave_setup(int H, const float *__restrict__ ws,
                                                const SeriesInfo *__restrict__ ser,
                                                const DatasetInfo *__restrict__ dsi,
                                                const WaveItem &it, int lane) {
    const DatasetInfo D = dsi[it.ds];
    const SeriesInfo sr = ser[D.series_base + it.rows];
    const SeriesInfo sc = ser[D.series_base + it.cols];
    WaveSetup w;
    w.n = sr.len;
    w.m = sc.len;
    w.xp = ws + sr.pstart;
    w.yp = ws + sc.pstart - lane;
    w.lstar = (w.n - 1) / H;
    w.S = w.m + w.lstar;
    w.hstar = (w.n - 1) - w.lstar * H;
    w.band = it.band;
    w.rbase = lane * H;
    const int a = it.rows < it.cols ? it.rows : it.cols;
    const int b = it.rows < it.cols ? it.cols : it.rows;
    w.out_at = D.out + condensed_index(a, b, D.N);
    return w;
}

template <int H>
__device__ __forceinline__ void load_rows(float (&x)[H], const WaveSetup &w) {
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int r = w.rbase + h;
        const float v = w.xp[r < w.n ? r : w.n - 1];
        x[h] = r < w.n ? v : 0.0f;  // rows past n are never read back into row n-1
    }
}

template <int H, bool BANDED, typename XT>
__device__ __forceinline__ void wave_step_f32(int s, float yv, const XT &x, const float (&O)[H], float (&N)[H],
                                              float &up_in, float &diag_in, const WaveSetup &w, int lane) {
    float diag = diag_in, up = up_in;
    const int off = w.rbase - (s - lane);
#pragma unroll
    for (int h = 0; h < H; ++h) {
        float xe = x[h];
        if constexpr (BANDED) xe = outside(off, h, w.band) ? kBig : xe;
        const float d = xe - yv;
        const float t = min3f(diag, up, O[h]);
        const float v = fmaf(d, d, t);
        diag = O[h];
        up = v;
        N[h] = v;
    }
    const float recv = lane_shift_down(N[H - 1], kInf);
    diag_in = up_in;
    up_in = recv;
}

// Window edges by row events.  With the skew "lane l at step s is at column
// s-l", row r = l*H+h enters the window (column r-b) at step l(H+1)+h-b and
// leaves it (column r+b+1) at step l(H+1)+h+b+1: at most one row enters and
// one row leaves per step, and both the lane and the strip row of each event
// are wave-uniform.  A row outside the window has its x replaced by 1e30 (its
// local cost overflows to +inf), so the cell loop itself carries no test.
// The x values live in a register vector so that the uniform row index of an
// event becomes one indexed register move (s_set_gpr_idx) instead of a test
// per cell.
template <int H>
struct XVec {
    typedef float T __attribute__((ext_vector_type(H)));
};

struct BandEvents {
    int le, he;  // next entry: lane, strip row (he == H: no entry this step)
    int lx, hx;  // next exit
    int b, n;

    template <int H>
    __device__ __forceinline__ void init(int band, int n_rows) {
        b = band;
        n = n_rows;
        le = band / (H + 1);
        he = band - le * (H + 1);
        lx = 0;
        hx = 0;
    }

    // Apply the events of step s, then advance to step s+1.
    template <int H>
    __device__ __forceinline__ void step(int s, typename XVec<H>::T &xe, const typename XVec<H>::T &xr, int lane) {
        if (he < H && le < 64 && le * H + he < n && s - le > 0) {
            const float cur = xe[he];
            const float v = xr[he];
            xe[he] = lane == le ? v : cur;
        }
        if (++he == H + 1) {
            he = 0;
            ++le;
        }
        if (s > b) {
            if (hx < H && lx < 64 && lx * H + hx < n) {
                const float cur = xe[hx];
                xe[hx] = lane == lx ? kBig : cur;
            }
            if (++hx == H + 1) {
                hx = 0;
                ++lx;
            }
        }
    }
};

template <int H, bool BANDED>
__global__ __launch_bounds__(64) void k_wave_plain(const float *__restrict__ ws,
                                                   const SeriesInfo *__restrict__ ser,
                                                   const DatasetInfo *__restrict__ dsi,
                                                   const WaveItem *__restrict__ items) {
    // window edges by row events up to 32 rows per lane; wider strips test every cell
    constexpr bool EVENTS = BANDED && H <= 32;
    constexpr bool PERCELL = BANDED && !EVENTS;
    typedef typename XVec<H>::T xvec;
    const int lane = threadIdx.x;
    const WaveItem it = items[blockIdx.x];
    const WaveSetup w = wave_setup(H, ws, ser, dsi, it, lane);
    float xa[H], A[H], Bv[H];
    load_rows<H>(xa, w);
    xvec xr, x;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int r = w.rbase + h;
        xr[h] = xa[h];
        x[h] = (!EVENTS || (r < w.n && r - w.band <= 0)) ? xa[h] : kBig;
        A[h] = kInf;
        Bv[h] = kInf;
    }
    BandEvents ev;
    if constexpr (EVENTS) ev.init<H>(w.band, w.n);
    float up_in = kInf;
    float diag_in = lane == 0 ? 0.0f : kInf;
    float y0 = w.yp[0], y1 = w.yp[1];
    int s = 0;
    for (; s + 2 <= w.S; s += 2) {
        const float y2 = w.yp[s + 2], y3 = w.yp[s + 3];
        if constexpr (EVENTS) ev.step<H>(s, x, xr, lane);
        wave_step_f32<H, PERCELL>(s, y0, x, A, Bv, up_in, diag_in, w, lane);
        if constexpr (EVENTS) ev.step<H>(s + 1, x, xr, lane);
        wave_step_f32<H, PERCELL>(s + 1, y1, x, Bv, A, up_in, diag_in, w, lane);
        y0 = y2;
        y1 = y3;
    }
    float res;
    if (s < w.S) {
        if constexpr (EVENTS) ev.step<H>(s, x, xr, lane);
        wave_step_f32<H, PERCELL>(s, y0, x, A, Bv, up_in, diag_in, w, lane);
        res = pick<H>(Bv, w.hstar);
    } else {
        res = pick<H>(A, w.hstar);
    }
    if (lane == w.lstar) *w.out_at = res;
}

// FP64 accumulation: the same operations as an IEEE double evaluation of
// Eq. (c) -- difference, product, min of three, sum -- in that order.
template <int H, bool BANDED>
__global__ __launch_bounds__(64) void k_wave_fp64(const float *__restrict__ ws,
                                                  const SeriesInfo *__restrict__ ser,
                                                  const DatasetInfo *__restrict__ dsi,
                                                  const WaveItem *__restrict__ items) {
    const int lane = threadIdx.x;
    const WaveItem it = items[blockIdx.x];
    const WaveSetup w = wave_setup(H, ws, ser, dsi, it, lane);
    float x[H];
    double st[H];
    load_rows<H>(x, w);
#pragma unroll
    for (int h = 0; h < H; ++h) st[h] = kInfD;
    double up_in = kInfD;
    double diag_in = lane == 0 ? 0.0 : kInfD;
    float ynext = w.yp[0];
    for (int s = 0; s < w.S; ++s) {
        const double yv = static_cast<double>(ynext);
        ynext = w.yp[s + 1];
        double diag = diag_in, up = up_in;
        const int off = w.rbase - (s - lane);
#pragma unroll
        for (int h = 0; h < H; ++h) {
            double xe = static_cast<double>(x[h]);
            if constexpr (BANDED) xe = outside(off, h, w.band) ? kBigD : xe;
            const double d = xe - yv;
            const double t = fmin(fmin(diag, up), st[h]);
            const double v = d * d + t;
            diag = st[h];
            st[h] = v;
            up = v;
        }
        const double recv = lane_shift_down(st[H - 1], kInfD);
        diag_in = up_in;
        up_in = recv;
    }
    const double res = pick<H>(st, w.hstar);
    if (lane == w.lstar) *w.out_at = static_cast<float>(res);
}

// Kahan-compensated FP32: each cell carries (s, c) with the true value close
// to s - c.  The min compares the running sums s (ties prefer diag, then up,
// then left) and takes the compensation of the chosen predecessor; the local
// cost is then added with Kahan's compensated step.  Unreachable (+inf) cells
// carry c = 0.
template <int H, bool BANDED>
__global__ __launch_bounds__(64) void k_wave_kahan(const float *__restrict__ ws,
                                                   const SeriesInfo *__restrict__ ser,
                                                   const DatasetInfo *__restrict__ dsi,
                                                   const WaveItem *__restrict__ items) {
    const int lane = threadIdx.x;
    const WaveItem it = items[blockIdx.x];
    const WaveSetup w = wave_setup(H, ws, ser, dsi, it, lane);
    float x[H], ss[H], cc[H];
    load_rows<H>(x, w);
#pragma unroll
    for (int h = 0; h < H; ++h) {
        ss[h] = kInf;
        cc[h] = 0.0f;
    }
    float up_s = kInf, up_c = 0.0f;
    float diag_s = lane == 0 ? 0.0f : kInf, diag_c = 0.0f;
    float ynext = w.yp[0];
    for (int s = 0; s < w.S; ++s) {
        const float yv = ynext;
        ynext = w.yp[s + 1];
        float ds = diag_s, dc = diag_c, us = up_s, uc = up_c;
        const int off = w.rbase - (s - lane);
#pragma unroll
        for (int h = 0; h < H; ++h) {
            float xe = x[h];
            if constexpr (BANDED) xe = outside(off, h, w.band) ? kBig : xe;
            const float d = xe - yv;
            const float q = d * d;
            const float p = min3f(ds, us, ss[h]);
            const float csel = (p == ds) ? dc : ((p == us) ? uc : cc[h]);
            const float yk = q - csel;
            const float t = p + yk;
            float cn = (t - p) - yk;
            cn = (t < kInf) ? cn : 0.0f;
            ds = ss[h];
            dc = cc[h];
            ss[h] = t;
            cc[h] = cn;
            us = t;
            uc = cn;
        }
        const float rs = lane_shift_down(ss[H - 1], kInf);
        const float rc = lane_shift_down(cc[H - 1], 0.0f);
        diag_s = up_s;
        diag_c = up_c;
        up_s = rs;
        up_c = rc;
    }
    float rs = pick<H>(ss, w.hstar), rc = pick<H>(cc, w.hstar);
    const float res = (rs < kInf) ? rs - rc : rs;
    if (lane == w.lstar) *w.out_at = res;
}

// ---------------------------------------------------------------------------
// Launch tables.
using LaneFn = hipError_t (*)(const float *, const SeriesInfo *, const DatasetInfo *, const LaneItem *,
                              int64_t, hipStream_t);

template <int I>
hipError_t lane_launcher(const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                         const LaneItem *items, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_lane<2 * I + 1>, dim3(static_cast<unsigned>(n)), dim3(64), 0, st, ws, ser, dsi,
                       items);
    return hipGetLastError();
}

template <size_t... I>
constexpr std::array<LaneFn, sizeof...(I)> make_lane_table(std::index_sequence<I...>) {
    return {{&lane_launcher<static_cast<int>(I)>...}};
}

const std::array<LaneFn, (kLaneMaxW + 1) / 2> kLaneTable =
    make_lane_table(std::make_index_sequence<(kLaneMaxW + 1) / 2>{});

template <int H, bool BANDED>
hipError_t wave_launch_h(int accum, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                         const WaveItem *items, int64_t n, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>(n)), block(64);
    switch (accum) {
        case 0: hipLaunchKernelGGL((k_wave_plain<H, BANDED>), grid, block, 0, st, ws, ser, dsi, items); break;
        case 1: hipLaunchKernelGGL((k_wave_kahan<H, BANDED>), grid, block, 0, st, ws, ser, dsi, items); break;
        case 2: hipLaunchKernelGGL((k_wave_fp64<H, BANDED>), grid, block, 0, st, ws, ser, dsi, items); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

constexpr int kWaveH[] = {1, 2, 4, 8, 12, 16, 24, 32, 48, 64};

}  // namespace

hipError_t launch_stage(const SeriesSrc *src, const SeriesInfo *ser, float *ws, int32_t nseries,
                        hipStream_t stream) {
    if (nseries <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stage, dim3(nseries), dim3(256), 0, stream, src, ser, ws);
    return hipGetLastError();
}

bool lane_width_supported(int W) { return W >= 1 && W <= kLaneMaxW && (W & 1); }

hipError_t launch_lane(int W, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                       const LaneItem *items, int64_t n_items, hipStream_t stream) {
    if (!lane_width_supported(W)) return hipErrorInvalidValue;
    if (n_items <= 0) return hipSuccess;
    return kLaneTable[(W - 1) / 2](ws, ser, dsi, items, n_items, stream);
}

int wave_rows_per_lane(int n) {
    for (int H : kWaveH)
        if (64 * H >= n) return H;
    return 0;
}

hipError_t launch_wave(int H, bool banded, int accum, const float *ws, const SeriesInfo *ser,
                       const DatasetInfo *dsi, const WaveItem *items, int64_t n_items, hipStream_t stream) {
    if (n_items <= 0) return hipSuccess;
#define DTWMI_WAVE_CASE(HV)                                                                  \
    case HV:                                                                                 \
        return banded ? wave_launch_h<HV, true>(accum, ws, ser, dsi, items, n_items, stream) \
                      : wave_launch_h<HV, false>(accum, ws, ser, dsi, items, n_items, stream);
    switch (H) {
        DTWMI_WAVE_CASE(1)
        DTWMI_WAVE_CASE(2)
        DTWMI_WAVE_CASE(4)
        DTWMI_WAVE_CASE(8)
        DTWMI_WAVE_CASE(12)
        DTWMI_WAVE_CASE(16)
        DTWMI_WAVE_CASE(24)
        DTWMI_WAVE_CASE(32)
        DTWMI_WAVE_CASE(48)
        DTWMI_WAVE_CASE(64)
        default: return hipErrorInvalidValue;
    }
#undef DTWMI_WAVE_CASE
}

}  // namespace dtwmi
