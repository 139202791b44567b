// Host side of the C ABI: validation, pair enumeration and tiling, workspace
// layout, plan execution.  See include/dtwmi.h for the contract.
//
// Pair enumeration.  The paper computes all p(p-1)/2 pairwise distances
// ("Mathematical background") and fills the symmetric matrix D.  This library
// writes each unordered pair once into the condensed upper triangle.
//  * lane-band datasets (all series of equal length, narrow band, plain or
//    rebased sums): tiles of up to 64 pairs at consecutive cyclic distances
//    from one series (lane_cyclic_tiles).
//  * wavefront datasets: one item per pair (i<j).  Each pair goes either to a
//    strip kernel (the shorter series spread over the lanes, every column
//    swept) or, with PLAIN accumulation and a window, to the cyclic kernel
//    (blocks of the longer series cycling over the lanes, each block visiting
//    only its window), whichever a step-count cost model finds cheaper.
//    Items are grouped by kernel instance and each group is sorted by
//    decreasing cost, so the longest pairs start first.
//  * accumulation: AUTO gives each pair plain FP32 sums when its longest
//    warping path (n+m-1 cells) has at most 2048 cells, beyond that rebased
//    FP32 sums when the pair has a window or the path has at most 4096
//    cells, and FP64 sums otherwise (pair_acc).
//  * strip pairs whose shorter series exceeds the rows of the largest
//    workgroup shape are swept in row passes through a per-workgroup buffer
//    that the plan allocates.
//  * a condensed sub-range [k_begin, k_end) restricts a plan to those output
//    entries: lane-band datasets are then tiled by rows of the condensed
//    matrix (runs of up to 64 consecutive partners j of one series i), the
//    others enumerate only the pairs of the range.
#include "dtw_internal.h"
#include "dtwmi.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <new>
#include <string>
#include <tuple>
#include <vector>

using namespace dtwmi;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace

// Error reporting shared with the other host sources of the library.
namespace dtwmi {
int set_error(int code, const char *msg) {
    g_err = msg;
    return code;
}
void clear_error() { g_err.clear(); }
}  // namespace dtwmi

namespace {

int hip_fail(hipError_t e, const char *what) {
    return fail(DTW_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Admissible cells of an n x m problem with band b (b < 0: none).  Closed
// form of sum_i |{j : |i-j| <= b, 0 <= j < m}|, valid because b >= |n-m|.
int64_t band_cells(int64_t n, int64_t m, int64_t b) {
    if (n <= 0 || m <= 0) return 0;
    if (b < 0 || b >= std::max(n, m) - 1) return n * m;
    // sum over i of (min(m-1, i+b) + 1) - max(0, i-b)
    int64_t upper = 0;
    const int64_t i_split = std::min(n - 1, m - b - 1);  // rows with i+b+1 <= m
    if (i_split >= 0) upper += (i_split + 1) * (b + 1) + i_split * (i_split + 1) / 2;
    const int64_t rest = (n - 1) - std::max<int64_t>(i_split, -1);
    upper += rest * m;
    int64_t lower = 0;
    if (n - 1 > b) {
        const int64_t t = n - 1 - b;
        lower = t * (t + 1) / 2;
    }
    return upper - lower;
}

// Condensed index of the unordered pair {i, j}, i != j.
int64_t condensed_host(int32_t i, int32_t j, int32_t N) {
    const int64_t a = std::min(i, j), b = std::max(i, j);
    return a * N - a * (a + 1) / 2 + (b - a - 1);
}

// Accumulation of one pair (AccMode) under the public mode; b is the pair's
// effective band (-1: none).  AUTO: plain sums up to 2048-cell warping paths;
// beyond, rebased sums for pairs with a window (the frontier stays near the
// path: measured ~10x below plain sums at 8,191-cell paths) and for
// unwindowed paths up to 4096 cells; unwindowed longer paths, where the
// cheapest frontier cell can lie far below the path and rebased sums gain
// less, run in FP64 (the oracle's operations, rounded once).
constexpr int64_t kAutoPlainMaxPath = 2048;
constexpr int64_t kAutoRebasedMaxPathNoWindow = 4096;
int pair_acc(int accum, int64_t n, int64_t m, int64_t b) {
    switch (accum) {
        case DTW_ACC_PLAIN: return kAccPlain;
        case DTW_ACC_KAHAN: return kAccKahan;
        case DTW_ACC_FP64: return kAccF64;
        case DTW_ACC_REBASED: return kAccRebased;
        default: {
            const int64_t path = n + m - 1;
            if (path <= kAutoPlainMaxPath) return kAccPlain;
            if (b >= 0 || path <= kAutoRebasedMaxPathNoWindow) return kAccRebased;
            return kAccF64;
        }
    }
}
// Modes with the plain FP32 cell, which the lane-band and cyclic kernels run.
bool plain_cell(int acc) { return acc == kAccPlain || acc == kAccRebased; }
const char *acc_name(int acc) {
    switch (acc) {
        case kAccKahan: return "kahan";
        case kAccF64: return "fp64";
        case kAccRebased: return "rebased";
        default: return "plain";
    }
}

int64_t effective_band(int32_t w, int32_t n, int32_t m) {
    if (w < 0) return -1;
    const int64_t d = n > m ? (int64_t)n - m : (int64_t)m - n;
    const int64_t b = std::max<int64_t>(w, d);
    return b >= std::max(n, m) - 1 ? -1 : b;
}

// Lane-band tiles of all pairs of an N-series dataset: series a is paired
// with the series at cyclic distances 1..h_a, (a + d) mod N, h_a =
// floor((N-1)/2), plus the pair at distance N/2 for a < N/2 when N is even,
// so that every unordered pair appears once and every series has the same
// number of partners (tiles of 64 partners, almost all full).  The tiles are
// emitted distance-run by distance-run (first partner distance d0 = 1, 65,
// 129, ...), every series within a run: consecutive tiles (a, d0) and
// (a+1, d0) share 63 of their 64 row series, which keeps a wavefront's reads
// in the L2 of its XCD (the kernel hands each XCD a contiguous range of
// tiles).  Calls emit(a, d0, cnt) for the partners (a + d0 + lane) mod N,
// lane < cnt.
template <class F>
void lane_cyclic_tiles(int32_t N, F emit) {
    const int32_t hmax = N / 2;  // the most partners of one series
    for (int32_t d0 = 1; d0 <= hmax; d0 += 64)
        for (int32_t a = 0; a < N; ++a) {
            const int32_t h = (N % 2 == 0 && a < N / 2) ? N / 2 : (N - 1) / 2;
            if (d0 <= h) emit(a, d0, std::min(64, h - d0 + 1));
        }
}

struct LaneGroup {
    int W;
    bool rebased;
    int64_t begin, count;
    int P = 1;  // lanes per pair: 1 (64 pairs per wavefront) or 4, 8, 16, 32 (the split kernel)
    int64_t cap = 0;  // item slots reserved for the group (autotuning: the most any split needs)
    int model_P = 1;  // the choice before autotuning
    std::vector<std::pair<int, float>> tuned_ms;  // autotuning: (P, ms per launch)
};

// The items of 64/P pairs of a list of 64-pair lane-band tiles (P > 1), or
// the tiles themselves (P = 1), appended to `out`.
void split_lane_items(const std::vector<LaneItem> &tiles, int P, std::vector<LaneItem> &out) {
    for (const LaneItem &it : tiles) {
        if (P == 1) {
            out.push_back(it);
            continue;
        }
        const int per = 64 / P;  // pairs per split item: partners q*per .. q*per+per-1 of the tile
        for (int q = 0; q * per < it.cnt; ++q) {
            LaneItem sub = it;
            sub.cnt = std::min(per, it.cnt - q * per);
            if (it.list < 0)
                sub.d0 += q * per;
            else
                sub.list += q * per;
            out.push_back(sub);
        }
    }
}

// Candidate splits of a lane-band group: 1 and every supported P (plain sums).
std::vector<int> lane_split_candidates(int W, bool rebased) {
    std::vector<int> c{1};
    if (!rebased)
        for (int P : {4, 8, 12, 16, 32})
            if (lane_split_supported(P, W)) c.push_back(P);
    return c;
}

// Lanes per pair of a lane-band group of 64-pair items over series of up to
// L points: one (64 pairs per wavefront) when the items give every SIMD at
// least two wavefronts; else the split (P = 4, 8, 12, 16 or 32 lanes per
// pair, items of 64/P pairs) of the smallest estimated time.  The estimate: L + P - 1
// steps, each the longer of the dependent chain through a lane (two
// operations per cell of its w = ceil(W/P) and five for the hand-overs, ~10
// cycles each) and the issue of the 3w + 6 instructions of every wavefront
// sharing its SIMD (~3.3 cycles each), all wavefronts resident at once --
// constants fitted to the 10,000 pairs of 512 points, band 103, where 8,
// 16 and 32 lanes per pair measured 0.078, 0.069 and 0.087 ms (4 lanes would
// hold 26 cells, past the instances); 12 lanes, added later, 0.059 against
// 0.064 with 16 and 0.073 with 8 on one device (2,000 wavefronts: at most two
// per SIMD instead of three).
int lane_split_choice(int W, bool rebased, int L, const std::vector<LaneItem> &items, int simds) {
    if (rebased || (int64_t)items.size() >= 2LL * simds) return 1;
    int best = 1;
    double best_t = 0.0;
    for (int P : {4, 8, 12, 16, 32}) {
        if (!lane_split_supported(P, W)) continue;
        int64_t waves = 0;
        for (const LaneItem &it : items) waves += (it.cnt + 64 / P - 1) / (64 / P);
        const int w = (W + P - 1) / P;
        const double per_simd = std::ceil((double)waves / simds);
        const double t = (double)(L + P - 1) * std::max(10.0 * (2 * w + 5), 3.3 * (3 * w + 6) * per_simd);
        if (best == 1 || t < best_t) {
            best = P;
            best_t = t;
        }
    }
    return best;
}

struct WaveGroup {
    StripShape shape;  // G == 0: cyclic kernel with H = shape.H
    bool banded;
    int acc;           // AccMode
    int64_t begin, count;
    int slots = 0;           // resident workgroups of the kernel (queue mode)
    int64_t band_cells = 0;  // admissible cells of the group's pairs
    int64_t swept_cells = 0; // cells its kernel sweeps, padding included
    int64_t max_rows = 0, max_cols = 0;  // longest series spread over the lanes / swept
    void *pass_buf = nullptr;            // row-pass buffer of a strip group with pairs over 64*H*G rows
    int64_t pass_stride = 0;             // its values per workgroup
};


// Cost model of the wavefront families, in VALU instructions of one
// wavefront.  Strips: wavefront-steps times instructions per step (3 per cell
// row plus loop overhead per step, from the instruction mix of the compiled
// loops), times a measured factor per instance: the median time per modelled
// instruction that DTW_FLAG_AUTOTUNE found for that instance over the buckets
// of the 64-dataset batched workload on MI355X, relative to the unwindowed
// 12-row strip (the factors carry the scalar work and waits of the window
// events and the occupancy of each register budget).  Cyclic kernel: the
// instruction count of its compiled loop (3 per cell row plus 13 per step:
// y address, block-switch test, the two window-event tests and moves, the
// boundary rotation and its mask) and ~45 per block switch, at the strips'
// issue rate: with its window events detected per lane the cyclic kernel
// issues VALU as fast as a strip (0.43-0.48 per wave-cycle at 20-32 rows).
// On the batched workload this plain count chose better than the calibrated
// factors (11,150 against 11,070 GCUPS on one box; 1.15x the count 11,145,
// 1.3x 10,920).
constexpr int kMaxQueues = 128;  // queue counters of a plan (one per wavefront kernel group)
constexpr int64_t kStripStepOverhead = 15;
constexpr int64_t kCyclicStepOverhead = 13;
constexpr int64_t kCyclicSwitchCost = 45;

struct CalEntry {
    int H;
    int strip_plain, strip_banded;  // x100
};
const CalEntry kCal[] = {{1, 100, 300},  {2, 100, 304},  {4, 87, 236},   {8, 95, 197},   {12, 103, 150},
                         {16, 108, 151}, {24, 112, 163}, {32, 118, 171}, {48, 125, 180}, {64, 130, 190}};

int64_t cal_factor(int H, bool banded) {
    for (const CalEntry &c : kCal)
        if (c.H >= H) return banded ? c.strip_banded : c.strip_plain;
    return banded ? 190 : 130;
}

// Steps a strip workgroup takes on an n x m pair (n = rows spread over lanes),
// over all its row passes of 64*H*G rows.
int64_t strip_steps(StripShape sh, int64_t n, int64_t m) {
    const int64_t cap = (int64_t)64 * sh.H * sh.G;
    int64_t steps = 0;
    for (int64_t P = 0; P < n; P += cap) {
        const int64_t lanes = (std::min(cap, n - P) - 1) / sh.H;  // last lane holding a row
        steps += m + lanes % 64 + (lanes / 64) * (64 + (sh.G > 1 ? 16 : 0));
    }
    return steps;
}

// Workgroups of several wavefronts also pay the LDS hand-over and barriers
// (measured: x1.2 for G = 2 against the same rows on one wavefront).
constexpr int64_t kMultiWaveFactor = 120;

int64_t strip_cost(StripShape sh, int64_t n, int64_t m, bool banded) {
    const int64_t c = sh.G * strip_steps(sh, n, m) * (3 * sh.H + kStripStepOverhead) * cal_factor(sh.H, banded) / 100;
    return sh.G > 1 ? c * kMultiWaveFactor / 100 : c;
}

// Cyclic kernel, rows = the longer series (n points), cols = the shorter (m),
// band b >= 0.  Blocks of H rows; block q sweeps columns at steps q + c.  A
// lane may take block q+64 only after block q has left its window, which holds
// when there are at most 64 blocks or 64(H+1) >= 2b+H.
bool cyclic_fits(int H, int64_t n, int64_t b) {
    const int64_t Q = (n + H - 1) / H;
    return Q <= 64 || 64 * (int64_t)(H + 1) >= 2 * b + H;
}

int64_t cyclic_steps(int H, int64_t n, int64_t m) { return m + (n - 1) / H; }

int64_t cyclic_cost(int H, int64_t n, int64_t m) {
    const int64_t blocks = (n + H - 1) / H;
    const int64_t switches = blocks > 64 ? blocks - 64 : 0;
    return cyclic_steps(H, n, m) * (3 * H + kCyclicStepOverhead) + switches * kCyclicSwitchCost;
}

// Strip shape for a pair whose shorter series has n points: of the two
// instantiated shapes of smallest row capacity 64*H*G >= n (restricted to
// H == force_h when force_h > 0), the cheaper by the cost model; when no
// shape holds n rows, the largest one, swept in row passes ({0,0} if force_h
// matches no shape).
StripShape pick_strip(int accum, int n, int m, bool banded, int force_h) {
    StripShape shapes[64];
    const int k = strip_shapes(accum, shapes, 64);
    StripShape best{0, 0}, largest{0, 0};
    int64_t best_cost = 0;
    int taken = 0;
    for (int i = 0; i < k && i < 64; ++i) {
        if (force_h > 0 && shapes[i].H != force_h) continue;
        largest = shapes[i];  // shapes come in increasing capacity
        if (taken < 2 && 64 * shapes[i].H * shapes[i].G >= n) {
            const int64_t c = strip_cost(shapes[i], n, m, banded);
            if (!best.H || c < best_cost) {
                best = shapes[i];
                best_cost = c;
            }
            ++taken;
        }
    }
    return best.H ? best : largest;
}

// Cheapest instantiated cyclic block height for the pair (0 if none fits);
// force_h > 0 restricts the choice to that height.
int pick_cyclic(int64_t n, int64_t m, int64_t b, int force_h, int64_t *cost) {
    int hs[32];
    const int k = cyclic_shapes(hs, 32);
    int best = 0;
    int64_t best_cost = 0;
    for (int i = 0; i < k && i < 32; ++i) {
        const int H = hs[i];
        if ((force_h > 0 && H != force_h) || !cyclic_fits(H, n, b)) continue;
        const int64_t c = cyclic_cost(H, n, m);
        if (!best || c < best_cost) {
            best = H;
            best_cost = c;
        }
    }
    *cost = best_cost;
    return best;
}

// A pair for the wavefront families: `shorter` has n points, `longer` m >= n.
struct WavePair {
    int32_t d, shorter, longer, n, m;
    int32_t b;     // effective band, -1 = none
    int64_t slot;  // output index in the dataset's output
    int32_t acc;   // AccMode of the pair
};

// Kernel instance of a wavefront pair: a strip shape, or (G == 0) the cyclic
// kernel with H rows per block.
struct Choice {
    int H = 0, G = 0;
    bool cyclic() const { return G == 0 && H > 0; }
    bool operator==(const Choice &o) const { return H == o.H && G == o.G; }
    bool operator<(const Choice &o) const { return H != o.H ? H < o.H : G < o.G; }
};

int64_t choice_cost(Choice c, const WavePair &w) {
    return c.cyclic() ? cyclic_cost(c.H, w.m, w.n) : strip_cost(StripShape{c.H, c.G}, w.n, w.m, w.b >= 0);
}

int64_t choice_steps_cells(Choice c, const WavePair &w) {  // cells swept, padding included
    return c.cyclic() ? (int64_t)64 * c.H * cyclic_steps(c.H, w.m, w.n)
                      : (int64_t)64 * c.G * c.H * strip_steps(StripShape{c.H, c.G}, w.n, w.m);
}

// The cost model's choice for a pair (H == 0 if no instance fits), for the
// pair's accumulation (rebased instances cost the same as plain ones within a
// few per cent, so one model serves both).
Choice model_choice(int kernel, int force_h, const WavePair &w) {
    int64_t cyc_cost = 0;
    const int cyc_h = (plain_cell(w.acc) && w.b >= 0 && kernel != DTW_KERNEL_WAVE)
                          ? pick_cyclic(w.m, w.n, w.b, force_h, &cyc_cost)
                          : 0;
    const StripShape sh =
        kernel == DTW_KERNEL_CYCLIC && cyc_h ? StripShape{0, 0} : pick_strip(w.acc, w.n, w.m, w.b >= 0, force_h);
    if (cyc_h && (!sh.H || cyc_cost < strip_cost(sh, w.n, w.m, w.b >= 0))) return Choice{cyc_h, 0};
    return Choice{sh.H, sh.G};
}

// Work item of a pair for its kernel: strips spread the shorter series over
// the lanes, the cyclic kernel the longer one.
WaveItem make_item(Choice c, const WavePair &w) {
    return c.cyclic() ? WaveItem{w.d, w.longer, w.shorter, w.b, w.slot}
                      : WaveItem{w.d, w.shorter, w.longer, w.b, w.slot};
}

// Half-octave bucket of a positive length: 2*floor(log2 v) + (v >= 1.5 * 2^floor(log2 v)).
int half_octave(int64_t v) {
    int k = 0;
    while ((v >> (k + 1)) > 0) ++k;
    return 2 * k + (v >= (int64_t(3) << k) / 2 ? 1 : 0);
}
int64_t half_octave_lo(int h) { return h & 1 ? (int64_t(3) << (h / 2)) / 2 : int64_t(1) << (h / 2); }

// Autotuning record of one (shorter length, longer length, band) bucket.
struct TunedBucket {
    int n_ho, m_ho, b_ho;  // half-octave buckets (b_ho of b+1; -1 = no window)
    int acc;               // AccMode of the bucket's pairs
    int64_t pairs;
    Choice model, chosen;  // chosen: the fastest measured on the bucket's own sample
    std::vector<std::pair<Choice, float>> us_per_pair;  // measured candidates
    std::vector<int64_t> idx;  // the bucket's wavefront pairs
    bool applied = false;      // chosen kept by the whole-plan trials
};

struct PlanTrial {  // one whole-plan timing of the autotuner
    int switched;   // buckets given their measured choice (the rest: the model's)
    float ms;       // execute time, median of the timed executes
};

}  // namespace

struct dtw_plan_s {
    int device = 0;
    int dtype = 0, accum = 0, kernel = 0, flags = 0;  // accum: the public dtw_accum
    int32_t nseries = 0;
    void *dev_block = nullptr;  // one allocation holding everything below
    void *pass_block = nullptr; // row-pass buffers of strip groups with very long pairs
    size_t dev_bytes = 0;
    float *ws = nullptr;
    SeriesSrc *d_src = nullptr;
    SeriesInfo *d_ser = nullptr;
    DatasetInfo *d_ds = nullptr;
    LaneItem *d_lane = nullptr;
    LanePartner *d_partner = nullptr;
    WaveItem *d_wave = nullptr;
    unsigned *d_queue = nullptr;  // one counter per wavefront group, zeroed by every execute
    int n_queue = 0;
    std::vector<LaneGroup> lane_groups;
    std::vector<WaveGroup> wave_groups;
    dtw_plan_stats stats{};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed_once = false;
    std::vector<TunedBucket> tuned;
    std::vector<PlanTrial> trials;
    // 64-pair tiles of each lane-band group, kept for autotuning its split
    std::vector<std::vector<LaneItem>> lane_tiles;
    // Wavefront groups run on up to kAuxStreams streams of the plan, forked
    // from and joined back to the caller's stream, so that one group's last
    // workgroups overlap the next group's first.
    int n_aux = 0;
    hipStream_t aux[4] = {};
    hipEvent_t fork_ev = nullptr, join_ev[4] = {};
};
constexpr int kAuxStreams = 4;

namespace {

int validate_options(const dtw_options *opt) {
    if (!opt) return DTW_OK;
    if (opt->dtype < DTW_F32 || opt->dtype > DTW_F16) return fail(DTW_ERR_INVALID_ARG, "unknown dtype %d", opt->dtype);
    if (opt->accum < DTW_ACC_AUTO || opt->accum > DTW_ACC_REBASED)
        return fail(DTW_ERR_INVALID_ARG, "unknown accumulation mode %d", opt->accum);
    if (opt->kernel < DTW_KERNEL_AUTO || opt->kernel > DTW_KERNEL_CYCLIC)
        return fail(DTW_ERR_INVALID_ARG, "unknown kernel family %d", opt->kernel);
    if (opt->rows_per_lane < 0 || opt->rows_per_lane > 64)
        return fail(DTW_ERR_INVALID_ARG, "rows_per_lane=%d outside 0..64", opt->rows_per_lane);
    if (opt->pairs_per_wave != 0 && opt->pairs_per_wave != 2 && opt->pairs_per_wave != 4 &&
        opt->pairs_per_wave != 5 && opt->pairs_per_wave != 8 && opt->pairs_per_wave != 16 &&
        opt->pairs_per_wave != 64)
        return fail(DTW_ERR_INVALID_ARG, "pairs_per_wave=%d is not 0, 2, 4, 5, 8, 16 or 64", opt->pairs_per_wave);
    if ((opt->kernel == DTW_KERNEL_CYCLIC || opt->kernel == DTW_KERNEL_LANE) &&
        (opt->accum == DTW_ACC_KAHAN || opt->accum == DTW_ACC_FP64))
        return fail(DTW_ERR_UNSUPPORTED, "the %s kernel needs AUTO, PLAIN or REBASED accumulation",
                    opt->kernel == DTW_KERNEL_CYCLIC ? "cyclic" : "lane-band");
    if (opt->k_begin < 0 || (opt->k_end > 0 && opt->k_end < opt->k_begin))
        return fail(DTW_ERR_INVALID_ARG, "output range [%lld, %lld) is invalid", (long long)opt->k_begin,
                    (long long)opt->k_end);
    if (opt->flags & ~(DTW_FLAG_TIMING | DTW_FLAG_NO_QUEUE | DTW_FLAG_AUTOTUNE))
        return fail(DTW_ERR_INVALID_ARG, "unknown flags 0x%x", opt->flags);
    return DTW_OK;
}

// need_all: the dataset is evaluated for all its pairs (N >= 2 needs series
// and out_condensed); otherwise for a pair list (N >= 1 needs series).
// Series lengths stay below 2^28 points so that every step and column count of
// a kernel fits an int.
constexpr int32_t kMaxSeriesLen = 1 << 28;
int validate_dataset(const dtw_dataset &d, int idx, bool need_all = true) {
    if (d.N < 0) return fail(DTW_ERR_INVALID_ARG, "dataset %d: N=%d < 0", idx, d.N);
    if (d.N < (need_all ? 2 : 1)) return DTW_OK;
    if (!d.series) return fail(DTW_ERR_INVALID_ARG, "dataset %d: series is NULL", idx);
    if (need_all && !d.out_condensed) return fail(DTW_ERR_INVALID_ARG, "dataset %d: out_condensed is NULL", idx);
    if (!d.lengths || !d.offsets) return fail(DTW_ERR_INVALID_ARG, "dataset %d: lengths/offsets is NULL", idx);
    for (int32_t s = 0; s < d.N; ++s) {
        if (d.lengths[s] < 1) return fail(DTW_ERR_INVALID_ARG, "dataset %d: lengths[%d]=%d < 1", idx, s, d.lengths[s]);
        if (d.lengths[s] > kMaxSeriesLen)
            return fail(DTW_ERR_UNSUPPORTED, "dataset %d: lengths[%d]=%d exceeds %d points", idx, s, d.lengths[s],
                        kMaxSeriesLen);
        if (d.offsets[s] < 0) return fail(DTW_ERR_INVALID_ARG, "dataset %d: offsets[%d] < 0", idx, s);
    }
    return DTW_OK;
}

void destroy_plan(dtw_plan p) {
    if (!p) return;
    if (p->dev_block) (void)hipFree(p->dev_block);
    if (p->pass_block) (void)hipFree(p->pass_block);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
    for (int a = 0; a < kAuxStreams; ++a) {
        if (p->join_ev[a]) (void)hipEventDestroy(p->join_ev[a]);
        if (p->aux[a]) (void)hipStreamDestroy(p->aux[a]);
    }
    delete p;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---- autotuning (DTW_FLAG_AUTOTUNE) ----
constexpr int kTuneSample = 32;      // distinct pairs timed per bucket
constexpr int kTuneCandidates = 4;   // instances timed per bucket, best by the cost model first
constexpr int kTuneMaxItems = 16384;  // items of one timing launch (sample repeated to fill the device)

// Instances that can run every pair of a bucket: the cyclic heights that fit
// all of them and the two smallest strip shapes that hold the longest shorter
// series (strips only when the plan's kernel family allows them).
std::vector<Choice> bucket_candidates(int acc, int kernel, int force_h, const std::vector<WavePair> &wp,
                                      const std::vector<int64_t> &idx) {
    int max_n = 0;
    bool all_banded = true;
    for (int64_t k : idx) {
        max_n = std::max(max_n, wp[k].n);
        all_banded = all_banded && wp[k].b >= 0;
    }
    std::vector<Choice> out;
    if (plain_cell(acc) && all_banded && kernel != DTW_KERNEL_WAVE) {
        int hs[32];
        const int kc = cyclic_shapes(hs, 32);
        for (int i = 0; i < kc && i < 32; ++i) {
            if (force_h > 0 && hs[i] != force_h) continue;
            bool fits = true;
            for (int64_t k : idx) fits = fits && cyclic_fits(hs[i], wp[k].m, wp[k].b);
            if (fits) out.push_back(Choice{hs[i], 0});
        }
    }
    if (!(kernel == DTW_KERNEL_CYCLIC && !out.empty())) {
        StripShape shapes[64];
        const int ks = strip_shapes(acc, shapes, 64);
        int taken = 0;
        for (int i = 0; i < ks && i < 64 && taken < 2; ++i)
            if (64 * shapes[i].H * shapes[i].G >= max_n && (force_h <= 0 || shapes[i].H == force_h)) {
                out.push_back(Choice{shapes[i].H, shapes[i].G});
                ++taken;
            }
    }
    return out;
}

// Time the candidate instances of every (shorter length, longer length, band)
// bucket on the plan's own data and give each bucket's pairs the fastest.
// Each timing launch repeats a sample of the bucket's pairs until it fills
// the device once (its resident workgroups), so it measures throughput, not
// the latency of a few pairs.  The kernels write the sampled pairs' results
// into the outputs, which every execute overwrites.
int autotune(dtw_plan p, const std::vector<WavePair> &wp, std::vector<Choice> &choice, int kernel, int force_h) {
    std::map<std::tuple<int, int, int, int>, std::vector<int64_t>> buckets;
    for (size_t k = 0; k < wp.size(); ++k)
        buckets[std::make_tuple(half_octave(wp[k].n), half_octave(wp[k].m),
                                wp[k].b < 0 ? -1 : half_octave((int64_t)wp[k].b + 1), wp[k].acc)]
            .push_back((int64_t)k);

    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    WaveItem *d_items = nullptr;
    std::vector<WaveItem> host(kTuneMaxItems);
    std::set<std::pair<Choice, bool>> warmed;
    int rc = DTW_OK;
    hipError_t e = launch_stage(p->d_src, p->d_ser, p->ws, p->nseries, s);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMalloc(&d_items, kTuneMaxItems * sizeof(WaveItem));
    if (e != hipSuccess) rc = hip_fail(e, "autotune set-up");

    for (auto it = buckets.begin(); rc == DTW_OK && it != buckets.end(); ++it) {
        const std::vector<int64_t> &idx = it->second;
        const int acc = std::get<3>(it->first);
        std::vector<Choice> cands = bucket_candidates(acc, kernel, force_h, wp, idx);
        if (cands.size() < 2) continue;  // nothing to choose
        std::vector<int64_t> sample;
        const int64_t ns = std::min<int64_t>(kTuneSample, (int64_t)idx.size());
        for (int64_t t = 0; t < ns; ++t) sample.push_back(idx[(size_t)(t * (int64_t)idx.size() / ns)]);
        std::vector<std::pair<int64_t, Choice>> ranked;
        for (const Choice &c : cands) {
            int64_t cost = 0;
            for (int64_t k : sample) cost += choice_cost(c, wp[k]);
            ranked.push_back({cost, c});
        }
        std::stable_sort(ranked.begin(), ranked.end(),
                         [](const std::pair<int64_t, Choice> &a, const std::pair<int64_t, Choice> &b) {
                             return a.first < b.first;
                         });
        if (ranked.size() > (size_t)kTuneCandidates) ranked.resize(kTuneCandidates);
        const bool banded = std::get<2>(it->first) >= 0;
        TunedBucket tb{std::get<0>(it->first), std::get<1>(it->first), std::get<2>(it->first), acc,
                       (int64_t)idx.size(), ranked[0].second, ranked[0].second, {}};
        float best = 0.0f;
        for (const auto &rc_pair : ranked) {
            const Choice c = rc_pair.second;
            const int slots = c.cyclic() ? cyclic_resident(c.H, acc == kAccRebased)
                                         : strip_resident(acc, StripShape{c.H, c.G}, banded, false);
            const int64_t T = std::min<int64_t>(kTuneMaxItems, std::max<int64_t>((int64_t)sample.size(), slots));
            for (int64_t t = 0; t < T; ++t) host[(size_t)t] = make_item(c, wp[sample[(size_t)(t % ns)]]);
            e = hipMemcpy(d_items, host.data(), (size_t)T * sizeof(WaveItem), hipMemcpyHostToDevice);
            auto run = [&]() {
                return c.cyclic() ? launch_cyclic(c.H, acc == kAccRebased, p->ws, p->d_ser, p->d_ds, d_items,
                                                  (unsigned)T, nullptr, 0, s)
                                  : launch_strip(acc, StripShape{c.H, c.G}, banded, p->ws, p->d_ser, p->d_ds,
                                                 d_items, (unsigned)T, nullptr, 0, nullptr, 0, s);
            };
            if (e == hipSuccess && !warmed.count({c, banded})) {  // first launch of an instance loads its code
                e = run();
                warmed.insert({c, banded});
            }
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            if (e == hipSuccess) e = run();
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = hip_fail(e, "autotune timing launch");
                break;
            }
            const float us = 1000.0f * ms / (float)T;
            tb.us_per_pair.push_back({c, us});
            if (tb.us_per_pair.size() == 1 || us < best) {
                best = us;
                tb.chosen = c;
            }
        }
        if (rc != DTW_OK) break;
        for (int64_t k : idx) choice[(size_t)k] = tb.chosen;
        tb.idx = idx;
        p->tuned.push_back(tb);
    }
    if (d_items) (void)hipFree(d_items);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

hipError_t launch_lane_group(const dtw_plan p, const LaneGroup &g, hipStream_t s) {
    return g.P > 1 ? launch_lane_split(g.P, g.W, p->ws, p->d_ser, p->d_ds, p->d_lane + g.begin, p->d_partner,
                                       (unsigned)g.count, s)
                   : launch_lane(g.W, g.rebased, p->ws, p->d_ser, p->d_ds, p->d_lane + g.begin, p->d_partner,
                                 (unsigned)g.count, s);
}

// Median of `reps` timed runs of `run` (after one untimed), in ms.
template <class Run>
int time_median(Run run, int reps, float *ms_out) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    std::vector<float> ms;
    int rc = e == hipSuccess ? run() : hip_fail(e, "hipEventCreate");
    if (rc == DTW_OK && (e = hipDeviceSynchronize()) != hipSuccess) rc = hip_fail(e, "autotune timing");
    for (int r = 0; rc == DTW_OK && r < reps; ++r) {
        if ((e = hipEventRecord(e0, nullptr)) != hipSuccess) {
            rc = hip_fail(e, "hipEventRecord");
            break;
        }
        if ((rc = run()) != DTW_OK) break;
        float t = 0.0f;
        if ((e = hipEventRecord(e1, nullptr)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) {
            rc = hip_fail(e, "autotune timing");
            break;
        }
        ms.push_back(t);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc == DTW_OK) {
        std::sort(ms.begin(), ms.end());
        *ms_out = ms[ms.size() / 2];
    }
    return rc;
}

// Pairs per wavefront of every lane-band group, measured: each candidate
// split of the group's tiles is uploaded and its launch timed on its own
// (lane-band groups run one after the other on the caller's stream, so a
// launch alone is what an execute sees); the fastest stays.
int autotune_lanes(dtw_plan p) {
    hipError_t e = launch_stage(p->d_src, p->d_ser, p->ws, p->nseries, nullptr);
    if (e != hipSuccess) return hip_fail(e, "staging kernel launch");
    for (size_t gi = 0; gi < p->lane_groups.size(); ++gi) {
        LaneGroup &g = p->lane_groups[gi];
        const std::vector<LaneItem> &tiles = p->lane_tiles[gi];
        const std::vector<int> cands = lane_split_candidates(g.W, g.rebased);
        if (tiles.empty() || cands.size() < 2) continue;
        int best = g.P;
        float best_ms = 0.0f;
        for (int P : cands) {
            std::vector<LaneItem> items;
            split_lane_items(tiles, P, items);
            if ((int64_t)items.size() > g.cap) continue;  // not reserved (cannot happen: cap is the most)
            if ((e = hipMemcpy(p->d_lane + g.begin, items.data(), items.size() * sizeof(LaneItem),
                               hipMemcpyHostToDevice)) != hipSuccess)
                return hip_fail(e, "hipMemcpy (autotune)");
            g.P = P;
            g.count = (int64_t)items.size();
            float ms = 0.0f;
            const int rc = time_median(
                [&]() {
                    const hipError_t el = launch_lane_group(p, g, nullptr);
                    return el == hipSuccess ? DTW_OK : hip_fail(el, "lane-band kernel launch");
                },
                3, &ms);
            if (rc) return rc;
            g.tuned_ms.push_back({P, ms});
            if (g.tuned_ms.size() == 1 || ms < best_ms) {
                best = P;
                best_ms = ms;
            }
        }
        std::vector<LaneItem> items;
        split_lane_items(tiles, best, items);
        if ((e = hipMemcpy(p->d_lane + g.begin, items.data(), items.size() * sizeof(LaneItem),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "hipMemcpy (autotune)");
        g.P = best;
        g.count = (int64_t)items.size();
    }
    return DTW_OK;
}

// Whole-plan trials of the measured bucket choices: each bucket's winner was
// measured on the bucket's sample alone, at the full occupancy of one
// instance, while an execute runs many instances side by side on several
// streams -- so a winner alone is not always a winner in the plan.  The
// buckets whose winner differs from the model are ranked by the measured
// gain (time per pair saved x pairs); the plan is built and timed (median of
// three executes) with the model's choices and with the top quarter, half,
// three quarters and all of them switched, and the fastest of those stays.
// The model's plan is one of the trials, so tuning never ends slower than
// the model on the measured runs.
template <class Assign>
int autotune_plan(dtw_plan p, const std::vector<WavePair> &wp, const std::vector<Choice> &model, Assign &assign) {
    std::vector<size_t> cand;
    for (size_t b = 0; b < p->tuned.size(); ++b)
        if (!(p->tuned[b].chosen == p->tuned[b].model)) cand.push_back(b);
    auto gain = [&](size_t b) {
        const TunedBucket &t = p->tuned[b];
        double um = 0.0, uc = 0.0;
        for (const auto &x : t.us_per_pair) {
            if (x.first == t.model) um = x.second;
            if (x.first == t.chosen) uc = x.second;
        }
        return (um - uc) * (double)t.pairs;
    };
    std::stable_sort(cand.begin(), cand.end(), [&](size_t a, size_t b) { return gain(a) > gain(b); });
    std::vector<int> ks;
    for (int q = 0; q <= 4; ++q) {
        const int k = (int)((cand.size() * q + 3) / 4);
        if (ks.empty() || ks.back() != k) ks.push_back(k);
    }
    auto choices = [&](int k) {
        std::vector<Choice> c = model;
        for (int i = 0; i < k; ++i)
            for (int64_t idx : p->tuned[cand[(size_t)i]].idx) c[(size_t)idx] = p->tuned[cand[(size_t)i]].chosen;
        return c;
    };
    int best_k = 0;
    float best_ms = 0.0f;
    for (int k : ks) {
        int rc = assign(choices(k));
        float ms = 0.0f;
        if (rc == DTW_OK) rc = time_median([&]() { return dtw_plan_execute(p, nullptr); }, 3, &ms);
        if (rc) return rc;
        p->trials.push_back(PlanTrial{k, ms});
        if (p->trials.size() == 1 || ms < best_ms) {
            best_k = k;
            best_ms = ms;
        }
    }
    for (int i = 0; i < best_k; ++i) p->tuned[cand[(size_t)i]].applied = true;
    return assign(choices(best_k));
}

std::string choice_name(Choice c) {
    char buf[48];
    if (c.cyclic())
        snprintf(buf, sizeof buf, "cyclic:%d", c.H);
    else
        snprintf(buf, sizeof buf, "strip:%dx%d", c.H, c.G);
    return buf;
}

}  // namespace

extern "C" {

const char *dtw_last_error(void) { return g_err.c_str(); }

int32_t dtw_version(void) { return 100; }

int dtw_band_cells(int32_t n, int32_t m, int32_t window, int64_t *cells) {
    if (!cells) return fail(DTW_ERR_INVALID_ARG, "cells is NULL");
    if (n < 0 || m < 0) return fail(DTW_ERR_INVALID_ARG, "negative length");
    *cells = band_cells(n, m, effective_band(window, n, m));
    return DTW_OK;
}

}  // extern "C"

namespace {

// An explicit pair list for dataset 0 (dtw_plan_create_pairs).
struct PairRequest {
    const dtw_pair *pairs;
    int64_t n;
    float *out;
};

// Plan for all pairs of every dataset (req == nullptr) or for the listed
// pairs of dataset 0.  Arguments are validated by the callers.
int plan_build(dtw_plan *plan_out, const dtw_dataset *ds, int32_t n_datasets, const dtw_options *opt,
               const PairRequest *req) {
    int rc = DTW_OK;

    const int dtype = opt ? opt->dtype : DTW_F32;
    const int accum = opt ? opt->accum : DTW_ACC_AUTO;
    const int kernel = opt ? opt->kernel : DTW_KERNEL_AUTO;
    const int flags = opt ? opt->flags : 0;
    const int force_h = opt ? opt->rows_per_lane : 0;
    const int force_ppw = opt ? opt->pairs_per_wave : 0;
    const int64_t k_begin = opt ? opt->k_begin : 0;
    const int64_t k_end_opt = opt ? opt->k_end : 0;

    // ---- host-side planning (no HIP calls) ----
    std::vector<SeriesSrc> src;
    std::vector<SeriesInfo> ser;
    std::vector<DatasetInfo> dsi;
    std::vector<LaneItem> lane_items;
    std::vector<LanePartner> partners;  // explicit partners of pair-list lane items
    std::map<std::pair<int, bool>, std::vector<LaneItem>> lane_by_w;  // (W, rebased)
    std::vector<WavePair> wpairs;
    dtw_plan_stats st{};
    size_t ws_floats = 0;

    for (int32_t d = 0; d < n_datasets; ++d) {
        const dtw_dataset &D = ds[d];
        DatasetInfo info{};
        info.out = req ? req->out : D.out_condensed;
        info.N = D.N;
        info.window = D.window;
        info.series_base = static_cast<int32_t>(ser.size());
        // output entries [k0, k1) of this dataset
        const int64_t n_out = req ? req->n : (D.N >= 2 ? (int64_t)D.N * (D.N - 1) / 2 : 0);
        const int64_t k1 = k_end_opt > 0 ? std::min(k_end_opt, n_out) : n_out;
        const int64_t k0 = std::min(k_begin, k1);
        if (D.N < (req ? 1 : 2) || k1 <= k0) {
            info.L = -1;
            dsi.push_back(info);
            continue;
        }
        bool uniform = true;
        for (int32_t s = 0; s < D.N; ++s) {
            uniform = uniform && D.lengths[s] == D.lengths[0];
            SeriesSrc ss{D.series, D.offsets[s], D.lengths[s], dtype};
            SeriesInfo si{};
            si.len = D.lengths[s];
            si.pstart = static_cast<int64_t>(ws_floats) + kPad;
            ws_floats += align_up(static_cast<size_t>(D.lengths[s]) + 2 * kPad, 4);
            src.push_back(ss);
            ser.push_back(si);
        }
        info.L = uniform ? D.lengths[0] : -1;
        dsi.push_back(info);
        const int64_t npairs = k1 - k0;
        const bool full = k0 == 0 && k1 == n_out;
        st.pairs += npairs;

        // Kernel family for this dataset.
        int lane_w = 0;
        const int lane_acc =
            uniform ? pair_acc(accum, D.lengths[0], D.lengths[0], effective_band(D.window, D.lengths[0], D.lengths[0]))
                    : kAccPlain;
        if (uniform && plain_cell(lane_acc)) {
            const int32_t L = D.lengths[0];
            const int32_t b = (D.window < 0 || D.window >= L - 1) ? L - 1 : D.window;
            if (lane_width_supported(2 * b + 1)) lane_w = 2 * b + 1;
        }
        if (kernel == DTW_KERNEL_LANE && !lane_w)
            return fail(DTW_ERR_UNSUPPORTED,
                        "dataset %d: the lane-band kernel needs equal lengths, PLAIN or REBASED accumulation and "
                        "2*w+1 <= %d",
                        d, kLaneMaxW);
        if (kernel == DTW_KERNEL_WAVE || kernel == DTW_KERNEL_CYCLIC) lane_w = 0;
        const auto lane_key = std::make_pair(lane_w, lane_acc == kAccRebased);

        if (lane_w && req) {
            // Each listed pair goes to the tile of whichever of its series is
            // named more often in the list (the shared column series of a
            // wavefront), in runs of 64 partners: every series against a few
            // medoids makes full tiles around each medoid.
            const int32_t L = D.lengths[0], b = (lane_w - 1) / 2;
            st.band_cells += npairs * band_cells(L, L, b >= L - 1 ? -1 : b);
            std::vector<int64_t> count(D.N, 0);
            for (int64_t k = k0; k < k1; ++k) {
                ++count[req->pairs[k].i];
                ++count[req->pairs[k].j];
            }
            std::map<int32_t, std::vector<LanePartner>> by_a;
            for (int64_t k = k0; k < k1; ++k) {
                const int32_t i = req->pairs[k].i, j = req->pairs[k].j;
                const bool on_i = count[i] > count[j] || (count[i] == count[j] && i <= j);
                by_a[on_i ? i : j].push_back(LanePartner{on_i ? j : i, 0, k});
            }
            for (auto &kv : by_a)
                for (size_t s0 = 0; s0 < kv.second.size(); s0 += 64) {
                    const int32_t cnt = (int32_t)std::min<size_t>(64, kv.second.size() - s0);
                    lane_by_w[lane_key].push_back(LaneItem{d, kv.first, 0, cnt, (int64_t)partners.size()});
                    partners.insert(partners.end(), kv.second.begin() + s0, kv.second.begin() + s0 + cnt);
                    st.computed_cells += (int64_t)64 * L * lane_w;
                }
        } else if (lane_w && full) {
            const int32_t L = D.lengths[0], b = (lane_w - 1) / 2;
            st.band_cells += npairs * band_cells(L, L, b >= L - 1 ? -1 : b);
            std::vector<LaneItem> &items = lane_by_w[lane_key];
            lane_cyclic_tiles(D.N, [&](int32_t a, int32_t d0, int32_t cnt) {
                items.push_back(LaneItem{d, a, d0, cnt, -1});
                st.computed_cells += (int64_t)64 * L * lane_w;
            });
        } else if (lane_w) {
            // a part of the condensed matrix: runs of up to 64 consecutive
            // partners j > i of one series i (partner a + d0 + lane, no wrap)
            const int32_t N = D.N, L = D.lengths[0], b = (lane_w - 1) / 2;
            st.band_cells += npairs * band_cells(L, L, b >= L - 1 ? -1 : b);
            int64_t row0 = 0;  // condensed index of pair (i, i+1)
            for (int32_t i = 0; i < N - 1 && row0 < k1; row0 += N - 1 - i, ++i) {
                const int64_t lo = std::max(k0, row0), hi = std::min(k1, row0 + (N - 1 - i));
                for (int64_t k = lo; k < hi; k += 64) {
                    const int32_t cnt = (int32_t)std::min<int64_t>(64, hi - k);
                    lane_by_w[lane_key].push_back(LaneItem{d, i, (int32_t)(k - row0 + 1), cnt, -1});
                    st.computed_cells += (int64_t)64 * L * lane_w;
                }
            }
        } else {
            // pairs of the range: list positions, or condensed indices walked row by row
            int64_t i = 0, j = 1, row0 = 0;
            if (!req) {
                while (row0 + (D.N - 1 - i) <= k0) {
                    row0 += D.N - 1 - i;
                    ++i;
                }
                j = i + 1 + (k0 - row0);
            }
            for (int64_t k = k0; k < k1; ++k) {
                if (req) {
                    i = req->pairs[k].i;
                    j = req->pairs[k].j;
                }
                {
                    const int32_t ni = D.lengths[i], nj = D.lengths[j];
                    const bool swap = nj < ni;
                    WavePair w{d, (int32_t)(swap ? j : i), (int32_t)(swap ? i : j), std::min(ni, nj),
                               std::max(ni, nj), 0, 0, 0};
                    w.slot = k;
                    w.b = static_cast<int32_t>(effective_band(D.window, w.n, w.m));
                    w.acc = pair_acc(accum, w.n, w.m, w.b);
                    st.band_cells += band_cells(w.n, w.m, w.b);
                    if (!model_choice(kernel, force_h, w).H) {
                        if (force_h > 0)
                            return fail(DTW_ERR_UNSUPPORTED,
                                        "dataset %d: pair (%d,%d) (%d x %d points, band %d): no kernel with "
                                        "rows_per_lane=%d fits it",
                                        d, (int)i, (int)j, w.n, w.m, w.b, force_h);
                        return fail(DTW_ERR_UNSUPPORTED, "dataset %d: pair (%d,%d): no kernel instance fits it", d,
                                    (int)i, (int)j);
                    }
                    wpairs.push_back(w);
                }
                if (!req && ++j == D.N) {
                    ++i;
                    j = i + 1;
                }
            }
        }
    }

    dtw_plan p = new (std::nothrow) dtw_plan_s;
    if (!p) return fail(DTW_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->dtype = dtype;
    p->accum = accum;
    p->kernel = kernel;
    p->flags = flags;
    p->nseries = static_cast<int32_t>(ser.size());
    // Pairs per wavefront of each lane-band group (the SIMD count from the
    // device; 1,024 when it cannot be queried)
    int simds = 1024;
    if (!lane_by_w.empty()) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            simds = 4 * cus;
        else
            (void)hipGetLastError();
    }
    for (auto &kv : lane_by_w) {
        const int W = kv.first.first;
        const bool rebased = kv.first.second;
        int Lmax = 1;
        for (const LaneItem &it : kv.second) Lmax = std::max(Lmax, dsi[it.ds].L);
        int P = force_ppw ? 64 / force_ppw : lane_split_choice(W, rebased, Lmax, kv.second, simds);
        if (P > 1 && (rebased || !lane_split_supported(P, W))) {
            delete p;
            return fail(DTW_ERR_UNSUPPORTED,
                        "pairs_per_wave=%d: no split lane-band kernel for band width %d with %s sums (it needs "
                        "PLAIN sums and 3 to %d band cells per lane)",
                        force_ppw, W, rebased ? "rebased" : "plain", split_max_cells(P));
        }
        LaneGroup g{W, rebased, (int64_t)lane_items.size(), 0, P};
        g.model_P = P;
        split_lane_items(kv.second, P, lane_items);
        g.count = (int64_t)lane_items.size() - g.begin;
        g.cap = g.count;
        if ((flags & DTW_FLAG_AUTOTUNE) && !force_ppw) {
            // room for the split with the most items, which the tuner may try
            int64_t most = g.count;
            for (int c : lane_split_candidates(W, rebased)) {
                int64_t n = 0;
                for (const LaneItem &it : kv.second) n += c == 1 ? 1 : (it.cnt + 64 / c - 1) / (64 / c);
                most = std::max(most, n);
            }
            g.cap = most;
            lane_items.resize((size_t)(g.begin + g.cap));  // the extra slots stay unused until a trial fills them
            p->lane_tiles.push_back(kv.second);
        } else {
            p->lane_tiles.emplace_back();
        }
        p->lane_groups.push_back(g);
    }
    st.n_lane_items = 0;
    for (const LaneGroup &g : p->lane_groups) st.n_lane_items += static_cast<int32_t>(g.count);
    st.n_wave_items = static_cast<int64_t>(wpairs.size());

    // ---- device allocation and upload of everything but the wavefront items ----
    ws_floats += 256;  // slack past the last slot
    size_t off = 0;
    const size_t o_ws = off;
    off = align_up(off + ws_floats * sizeof(float), 256);
    const size_t o_src = off;
    off = align_up(off + src.size() * sizeof(SeriesSrc), 256);
    const size_t o_ser = off;
    off = align_up(off + ser.size() * sizeof(SeriesInfo), 256);
    const size_t o_ds = off;
    off = align_up(off + dsi.size() * sizeof(DatasetInfo), 256);
    const size_t o_lane = off;
    off = align_up(off + lane_items.size() * sizeof(LaneItem), 256);
    const size_t o_partner = off;
    off = align_up(off + partners.size() * sizeof(LanePartner), 256);
    const size_t o_wave = off;
    off = align_up(off + wpairs.size() * sizeof(WaveItem), 256);
    const size_t o_queue = off;
    off = align_up(off + kMaxQueues * sizeof(unsigned), 256);
    p->dev_bytes = off;
    st.workspace_bytes = static_cast<int64_t>(off);

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        destroy_plan(p);
        return hip_fail(e, "hipGetDevice");
    }
    e = hipMalloc(&p->dev_block, p->dev_bytes);
    if (e != hipSuccess) {
        destroy_plan(p);
        return fail(DTW_ERR_OUT_OF_MEMORY, "hipMalloc(%zu bytes): %s", p->dev_bytes, hipGetErrorString(e));
    }
    char *base = static_cast<char *>(p->dev_block);
    p->ws = reinterpret_cast<float *>(base + o_ws);
    p->d_src = reinterpret_cast<SeriesSrc *>(base + o_src);
    p->d_ser = reinterpret_cast<SeriesInfo *>(base + o_ser);
    p->d_ds = reinterpret_cast<DatasetInfo *>(base + o_ds);
    p->d_lane = reinterpret_cast<LaneItem *>(base + o_lane);
    p->d_partner = reinterpret_cast<LanePartner *>(base + o_partner);
    p->d_wave = reinterpret_cast<WaveItem *>(base + o_wave);
    struct Up {
        void *dst;
        const void *src;
        size_t bytes;
    } ups[] = {{p->d_src, src.data(), src.size() * sizeof(SeriesSrc)},
               {p->d_ser, ser.data(), ser.size() * sizeof(SeriesInfo)},
               {p->d_ds, dsi.data(), dsi.size() * sizeof(DatasetInfo)},
               {p->d_lane, lane_items.data(), lane_items.size() * sizeof(LaneItem)},
               {p->d_partner, partners.data(), partners.size() * sizeof(LanePartner)}};
    for (const Up &u : ups) {
        if (!u.bytes) continue;
        e = hipMemcpy(u.dst, u.src, u.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            destroy_plan(p);
            return hip_fail(e, "hipMemcpy (plan upload)");
        }
    }

    // ---- kernel instance of every wavefront pair: cost model, or measured ----
    std::vector<Choice> model(wpairs.size());
    for (size_t k = 0; k < wpairs.size(); ++k) model[k] = model_choice(kernel, force_h, wpairs[k]);
    const int64_t lane_cells = st.computed_cells;  // the lane-band tiles' share
    const bool use_queue = !(flags & DTW_FLAG_NO_QUEUE) && !wpairs.empty();

    // Group the wavefront pairs by kernel instance (H, G, banded, accumulation);
    // inside a group costlier pairs first, groups in decreasing order of their
    // costliest pair; upload the items, size the launches and the row-pass
    // buffers.  Called again by the autotuner for each whole-plan trial.
    auto assign = [&](const std::vector<Choice> &choice) -> int {
        p->wave_groups.clear();
        if (p->pass_block) {
            (void)hipFree(p->pass_block);
            p->pass_block = nullptr;
        }
        st.computed_cells = lane_cells;
        st.n_cyclic_items = 0;
        st.n_lane_items = 0;
        for (const LaneGroup &g : p->lane_groups) st.n_lane_items += static_cast<int32_t>(g.count);
        st.workspace_bytes = static_cast<int64_t>(p->dev_bytes);
        using Kind = std::tuple<int, int, bool, int>;  // H, G, banded, AccMode
        std::map<Kind, std::vector<std::pair<int64_t, WaveItem>>> wave_by_kind;
        std::map<Kind, std::pair<int64_t, int64_t>> cells_by_kind;   // admissible, swept
        std::map<Kind, std::pair<int64_t, int64_t>> extent_by_kind;  // longest rows, cols
        for (size_t k = 0; k < wpairs.size(); ++k) {
            const Choice c = choice[k];
            const WavePair &w = wpairs[k];
            const int64_t swept = choice_steps_cells(c, w);
            st.computed_cells += swept;
            st.n_cyclic_items += c.cyclic() ? 1 : 0;
            const Kind kind = std::make_tuple(c.H, c.G, c.cyclic() || w.b >= 0, (int)w.acc);
            wave_by_kind[kind].push_back({choice_cost(c, w), make_item(c, w)});
            auto &cells = cells_by_kind[kind];
            cells.first += band_cells(w.n, w.m, w.b);
            cells.second += swept;
            auto &ext = extent_by_kind[kind];
            ext.first = std::max<int64_t>(ext.first, c.cyclic() ? w.m : w.n);
            ext.second = std::max<int64_t>(ext.second, c.cyclic() ? w.n : w.m);
        }
        std::vector<typename decltype(wave_by_kind)::iterator> order;
        for (auto it = wave_by_kind.begin(); it != wave_by_kind.end(); ++it) {
            std::stable_sort(it->second.begin(), it->second.end(),
                             [](const std::pair<int64_t, WaveItem> &x, const std::pair<int64_t, WaveItem> &y) {
                                 return x.first > y.first;
                             });
            order.push_back(it);
        }
        std::stable_sort(order.begin(), order.end(),
                         [](const auto &x, const auto &y) { return x->second[0].first > y->second[0].first; });
        std::vector<WaveItem> wave_items;
        wave_items.reserve(wpairs.size());
        for (auto it : order) {
            auto &v = it->second;
            if (v.size() > 0x7fffffff) return fail(DTW_ERR_UNSUPPORTED, "more than 2^31-1 work items for one kernel");
            const StripShape sh{std::get<0>(it->first), std::get<1>(it->first)};
            const auto &cells = cells_by_kind[it->first];
            const auto &ext = extent_by_kind[it->first];
            p->wave_groups.push_back(WaveGroup{sh, std::get<2>(it->first), std::get<3>(it->first),
                                               (int64_t)wave_items.size(), (int64_t)v.size(), 0, cells.first,
                                               cells.second, ext.first, ext.second});
            for (auto &e2 : v) wave_items.push_back(e2.second);
        }
        if (p->wave_groups.size() > (size_t)kMaxQueues)
            return fail(DTW_ERR_UNSUPPORTED, "more than %d wavefront kernel groups", kMaxQueues);
        hipError_t e2 = hipSuccess;
        if (!wave_items.empty() &&
            (e2 = hipMemcpy(p->d_wave, wave_items.data(), wave_items.size() * sizeof(WaveItem),
                            hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e2, "hipMemcpy (plan upload)");
        p->n_queue = use_queue ? (int)p->wave_groups.size() : 0;
        p->d_queue = p->n_queue ? reinterpret_cast<unsigned *>(base + o_queue) : nullptr;
        auto needs_passes = [](const WaveGroup &g) {
            return g.shape.G > 0 && g.max_rows > (int64_t)64 * g.shape.H * g.shape.G;
        };
        if (use_queue)  // grid of each launch: the workgroups the device holds at once
            for (WaveGroup &g : p->wave_groups)
                g.slots = g.shape.G == 0 ? cyclic_resident(g.shape.H, g.acc == kAccRebased)
                                         : strip_resident(g.acc, g.shape, g.banded, needs_passes(g));
        // Row-pass buffers: one row of the longest swept series per workgroup of
        // every strip group holding a pair of more than 64*H*G rows.
        size_t pass_bytes = 0;
        std::vector<size_t> pass_off(p->wave_groups.size(), 0);
        for (size_t k = 0; k < p->wave_groups.size(); ++k) {
            const WaveGroup &g = p->wave_groups[k];
            if (!needs_passes(g)) continue;
            const int grid = strip_grid((unsigned)g.count, use_queue ? p->d_queue : nullptr, g.slots);
            pass_off[k] = pass_bytes + 1;  // 0 = none
            pass_bytes = align_up(pass_bytes + (size_t)grid * (size_t)g.max_cols * strip_cell_bytes(g.acc), 256);
        }
        if (pass_bytes) {
            if ((e2 = hipMalloc(&p->pass_block, pass_bytes)) != hipSuccess)
                return fail(DTW_ERR_OUT_OF_MEMORY, "hipMalloc(%zu bytes) for row passes: %s", pass_bytes,
                            hipGetErrorString(e2));
            for (size_t k = 0; k < p->wave_groups.size(); ++k)
                if (pass_off[k]) {
                    p->wave_groups[k].pass_buf = static_cast<char *>(p->pass_block) + (pass_off[k] - 1);
                    p->wave_groups[k].pass_stride = p->wave_groups[k].max_cols;
                }
            st.workspace_bytes += (int64_t)pass_bytes;
        }
        st.n_launches = (p->nseries > 0 ? 1 : 0) + (use_queue ? 1 : 0) +
                        (int32_t)(p->lane_groups.size() + p->wave_groups.size());
        p->stats = st;
        return DTW_OK;
    };

    auto plan_streams = [&](size_t groups) -> int {  // default-priority streams, events without timing
        if (p->n_aux || groups <= 1) return DTW_OK;
        p->n_aux = std::min<int>(kAuxStreams, (int)groups);
        hipError_t e2 = hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming);
        for (int a = 0; a < p->n_aux && e2 == hipSuccess; ++a) {
            e2 = hipStreamCreateWithFlags(&p->aux[a], hipStreamNonBlocking);
            if (e2 == hipSuccess) e2 = hipEventCreateWithFlags(&p->join_ev[a], hipEventDisableTiming);
        }
        return e2 == hipSuccess ? DTW_OK : hip_fail(e2, "plan stream set-up");
    };

    if (flags & DTW_FLAG_TIMING) {
        if ((e = hipEventCreate(&p->ev0)) != hipSuccess || (e = hipEventCreate(&p->ev1)) != hipSuccess) {
            destroy_plan(p);
            return hip_fail(e, "hipEventCreate");
        }
    }
    if (flags & DTW_FLAG_AUTOTUNE) {
        rc = autotune_lanes(p);
        std::vector<Choice> iso = model;
        if (rc == DTW_OK && wpairs.empty()) rc = assign(model);
        if (rc == DTW_OK && !wpairs.empty()) rc = autotune(p, wpairs, iso, kernel, force_h);
        if (rc == DTW_OK && !wpairs.empty()) rc = plan_streams(kAuxStreams);
        if (rc == DTW_OK && !wpairs.empty()) rc = autotune_plan(p, wpairs, model, assign);
        if (rc) {
            destroy_plan(p);
            return rc;
        }
        st.n_tuned_buckets = static_cast<int32_t>(p->tuned.size());
        for (const TunedBucket &t : p->tuned) st.n_tuned_changed += t.applied && !(t.chosen == t.model) ? 1 : 0;
        p->stats.n_tuned_buckets = st.n_tuned_buckets;
        p->stats.n_tuned_changed = st.n_tuned_changed;
    } else {
        rc = assign(model);
        if (rc == DTW_OK) rc = plan_streams(p->wave_groups.size());
        if (rc) {
            destroy_plan(p);
            return rc;
        }
    }
    *plan_out = p;
    return DTW_OK;
}

int validate_pairs(const dtw_dataset *ds, const dtw_pair *pairs, int64_t n_pairs, const float *out) {
    if (!ds) return fail(DTW_ERR_INVALID_ARG, "dataset is NULL");
    if (n_pairs < 0) return fail(DTW_ERR_INVALID_ARG, "n_pairs=%lld < 0", (long long)n_pairs);
    if (n_pairs == 0) return DTW_OK;
    if (!pairs || !out) return fail(DTW_ERR_INVALID_ARG, "pairs or out is NULL");
    int rc = validate_dataset(*ds, 0, false);
    if (rc) return rc;
    for (int64_t k = 0; k < n_pairs; ++k)
        if (pairs[k].i < 0 || pairs[k].i >= ds->N || pairs[k].j < 0 || pairs[k].j >= ds->N)
            return fail(DTW_ERR_INVALID_ARG, "pairs[%lld] = (%d, %d) outside 0..%d", (long long)k, pairs[k].i,
                        pairs[k].j, ds->N - 1);
    return DTW_OK;
}

// ---- plan cache of the short forms (dtw_pairwise, dtw_pairwise_ex, dtw_pairs) ----
// A cached plan is keyed by everything that shapes it except the buffers:
// device, stream, options, N, window, lengths, offsets (and the pair list).
// A hit re-points the plan at the call's series and output (k_rebind) and
// launches it: no allocation, upload or synchronisation.  Enqueueing happens
// under the cache lock, so the rebind and launches of one call are never
// interleaved with another call's on the same plan.
struct CacheKey {
    int device = 0;
    void *stream = nullptr;
    int32_t dtype = 0, accum = 0, kernel = 0, flags = 0, rows = 0, ppw = 0;
    int64_t k_begin = 0, k_end = 0;
    int32_t N = 0, window = 0;
    bool list = false;
    std::vector<int32_t> lengths;
    std::vector<int64_t> offsets;
    std::vector<int32_t> pairs;  // i, j interleaved

    bool operator==(const CacheKey &o) const {
        return device == o.device && stream == o.stream && dtype == o.dtype && accum == o.accum &&
               kernel == o.kernel && flags == o.flags && rows == o.rows && ppw == o.ppw && k_begin == o.k_begin &&
               k_end == o.k_end && N == o.N && window == o.window && list == o.list && lengths == o.lengths &&
               offsets == o.offsets && pairs == o.pairs;
    }
};

struct CacheEntry {
    CacheKey key;
    dtw_plan plan = nullptr;
    hipEvent_t done = nullptr;  // recorded after the plan's last launch
    uint64_t used = 0;
};

constexpr size_t kCacheSize = 8;
std::mutex g_cache_mu;
std::vector<CacheEntry> g_cache;
uint64_t g_cache_tick = 0;

void drop_entry(CacheEntry &c) {
    if (c.done) {
        (void)hipEventSynchronize(c.done);  // the plan's last launch has finished
        (void)hipEventDestroy(c.done);
    }
    destroy_plan(c.plan);
    c.plan = nullptr;
    c.done = nullptr;
}

int cached_run(const dtw_dataset &d, const dtw_options *opt, const PairRequest *req) {
    dtw_options o{};
    if (opt) o = *opt;
    o.flags &= DTW_FLAG_NO_QUEUE | DTW_FLAG_AUTOTUNE;  // timing needs the plan API
    CacheKey key;
    // Without a device the lookup misses and plan_build reports the request's
    // host-side errors first (all arguments are checked before any HIP work),
    // then the failing HIP call.
    hipError_t e = hipGetDevice(&key.device);
    if (e != hipSuccess) key.device = -1;
    key.stream = o.stream;
    key.dtype = o.dtype;
    key.accum = o.accum;
    key.kernel = o.kernel;
    key.flags = o.flags;
    key.rows = o.rows_per_lane;
    key.ppw = o.pairs_per_wave;
    key.k_begin = o.k_begin;
    key.k_end = o.k_end;
    key.N = d.N;
    key.window = d.window;
    key.list = req != nullptr;
    key.lengths.assign(d.lengths, d.lengths + d.N);
    key.offsets.assign(d.offsets, d.offsets + d.N);
    if (req) {
        key.pairs.resize(2 * (size_t)req->n);
        for (int64_t k = 0; k < req->n; ++k) {
            key.pairs[2 * (size_t)k] = req->pairs[k].i;
            key.pairs[2 * (size_t)k + 1] = req->pairs[k].j;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    float *out = req ? req->out : d.out_condensed;

    std::lock_guard<std::mutex> lock(g_cache_mu);
    CacheEntry *hit = nullptr;
    for (CacheEntry &c : g_cache)
        if (c.key == key) hit = &c;
    if (!hit) {
        dtw_plan p = nullptr;
        const int rc = plan_build(&p, &d, 1, &o, req);
        if (rc) return rc;
        hipEvent_t done = nullptr;
        if ((e = hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess) {
            destroy_plan(p);
            return hip_fail(e, "hipEventCreate");
        }
        if (g_cache.size() >= kCacheSize) {  // replace the least recently used plan
            size_t lru = 0;
            for (size_t c = 1; c < g_cache.size(); ++c)
                if (g_cache[c].used < g_cache[lru].used) lru = c;
            drop_entry(g_cache[lru]);
            g_cache.erase(g_cache.begin() + (long)lru);
        }
        g_cache.push_back(CacheEntry{std::move(key), p, done, 0});
        hit = &g_cache.back();
    } else if ((e = launch_rebind(hit->plan->d_src, hit->plan->nseries, d.series, hit->plan->d_ds, out, s)) !=
               hipSuccess) {
        return hip_fail(e, "rebind kernel launch");
    }
    hit->used = ++g_cache_tick;
    const int rc = dtw_plan_execute(hit->plan, s);
    if (rc) return rc;
    if ((e = hipEventRecord(hit->done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    return DTW_OK;
}

// ---- allocation-free evaluation (dtw_pairwise_noalloc) ----
// The whole device workspace of one call -- padded FP32 copy of the series,
// series and dataset tables, work items, queue counters -- lives in this
// file-scope array, one copy per device the library runs on, held until the
// process ends.  Its address on the current device comes from
// hipGetSymbolAddress (the array's name is only a host-side stand-in); the
// tables are built in a static host buffer of the same role and copied in.
// Calls share the array and the host buffer: a lock serialises the host part,
// and calls on different streams of one device race on the device part.
constexpr size_t kScratchBytes = size_t(32) << 20;   // device workspace of one call
constexpr size_t kHostStageBytes = size_t(64) << 20; // tables plus the planner's sort records
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
alignas(256) unsigned char g_host_stage[kHostStageBytes];
std::mutex g_noalloc_mu;
void *g_scratch_ptr[kMaxScratchDevices];  // device address of `scratch` per device, set once

// Sort record of a wavefront pair: its kernel instance and cost.
struct NoAllocRec {
    uint32_t kind;  // (((H * 32 + G) * 2 + banded) * 4 + acc)
    int64_t cost;
    WaveItem item;
};

int noalloc_run(const dtw_dataset &d, const dtw_options &o) {
    if (o.flags & DTW_FLAG_AUTOTUNE)
        return fail(DTW_ERR_UNSUPPORTED, "DTW_FLAG_AUTOTUNE allocates; the allocation-free entry point refuses it");
    if (o.k_begin != 0 || o.k_end != 0)
        return fail(DTW_ERR_UNSUPPORTED, "the allocation-free entry point evaluates every pair (k_begin = k_end = 0)");
    const int32_t N = d.N;
    const bool use_queue = !(o.flags & DTW_FLAG_NO_QUEUE);

    // ---- sizes (no HIP calls yet) ----
    size_t ws_floats = 0;
    bool uniform = true;
    for (int32_t s = 0; s < N; ++s) {
        ws_floats += align_up(static_cast<size_t>(d.lengths[s]) + 2 * kPad, 4);
        uniform = uniform && d.lengths[s] == d.lengths[0];
    }
    ws_floats += 256;
    int lane_w = 0;
    const int lane_acc =
        uniform ? pair_acc(o.accum, d.lengths[0], d.lengths[0], effective_band(d.window, d.lengths[0], d.lengths[0]))
                : kAccPlain;
    if (uniform && plain_cell(lane_acc) && o.kernel != DTW_KERNEL_WAVE && o.kernel != DTW_KERNEL_CYCLIC) {
        const int32_t L = d.lengths[0];
        const int32_t b = (d.window < 0 || d.window >= L - 1) ? L - 1 : d.window;
        if (lane_width_supported(2 * b + 1)) lane_w = 2 * b + 1;
    }
    if (o.kernel == DTW_KERNEL_LANE && !lane_w)
        return fail(DTW_ERR_UNSUPPORTED,
                    "the lane-band kernel needs equal lengths, PLAIN or REBASED accumulation and 2*w+1 <= %d",
                    kLaneMaxW);
    int64_t n_lane = 0;
    const int64_t n_pairs = (int64_t)N * (N - 1) / 2;
    if (lane_w) lane_cyclic_tiles(N, [&](int32_t, int32_t, int32_t) { ++n_lane; });
    const size_t o_ws = 0;
    size_t off = align_up(ws_floats * sizeof(float), 256);
    const size_t o_src = off;
    off = align_up(off + N * sizeof(SeriesSrc), 256);
    const size_t o_ser = off;
    off = align_up(off + N * sizeof(SeriesInfo), 256);
    const size_t o_ds = off;
    off = align_up(off + sizeof(DatasetInfo), 256);
    const size_t o_items = off;
    off = align_up(off + (lane_w ? n_lane * sizeof(LaneItem) : n_pairs * sizeof(WaveItem)), 256);
    const size_t o_queue = off;
    off = align_up(off + kMaxQueues * sizeof(unsigned), 256);
    const size_t need = off;
    const size_t o_sort = align_up(o_queue - o_src, 256);  // host staging: tables, then sort records
    const size_t host_need = o_sort + (lane_w ? 0 : n_pairs * sizeof(NoAllocRec));
    if (need > kScratchBytes || host_need > kHostStageBytes)
        return fail(DTW_ERR_UNSUPPORTED,
                    "the allocation-free entry point holds %zu bytes of device workspace (and %zu of host tables); "
                    "this dataset needs %zu (%zu)",
                    kScratchBytes, kHostStageBytes, need, host_need);

    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    // ---- tables, built in the host staging buffer at their device offsets minus o_src ----
    unsigned char *h = g_host_stage;
    SeriesSrc *hsrc = reinterpret_cast<SeriesSrc *>(h + (o_src - o_src));
    SeriesInfo *hser = reinterpret_cast<SeriesInfo *>(h + (o_ser - o_src));
    DatasetInfo *hds = reinterpret_cast<DatasetInfo *>(h + (o_ds - o_src));
    size_t wsf = 0;
    for (int32_t s = 0; s < N; ++s) {
        hsrc[s] = SeriesSrc{d.series, d.offsets[s], d.lengths[s], o.dtype};
        hser[s] = SeriesInfo{static_cast<int64_t>(wsf) + kPad, d.lengths[s], 0};
        wsf += align_up(static_cast<size_t>(d.lengths[s]) + 2 * kPad, 4);
    }
    *hds = DatasetInfo{d.out_condensed, N, d.window, uniform ? d.lengths[0] : -1, 0};
    struct Group {
        uint32_t kind;
        int64_t begin, count;
    } groups[kMaxQueues];
    int n_groups = 0;
    if (lane_w) {
        LaneItem *it = reinterpret_cast<LaneItem *>(h + (o_items - o_src));
        int64_t k = 0;
        lane_cyclic_tiles(N, [&](int32_t a, int32_t d0, int32_t cnt) { it[k++] = LaneItem{0, a, d0, cnt, -1}; });
    } else {
        NoAllocRec *rec = reinterpret_cast<NoAllocRec *>(h + o_sort);
        int64_t k = 0;
        for (int32_t i = 0; i < N - 1; ++i)
            for (int32_t j = i + 1; j < N; ++j, ++k) {
                const int32_t ni = d.lengths[i], nj = d.lengths[j];
                const bool swap = nj < ni;
                WavePair w{0, swap ? j : i, swap ? i : j, std::min(ni, nj), std::max(ni, nj), 0, k, 0};
                w.b = static_cast<int32_t>(effective_band(d.window, w.n, w.m));
                w.acc = pair_acc(o.accum, w.n, w.m, w.b);
                const Choice c = model_choice(o.kernel, o.rows_per_lane, w);
                if (!c.H)
                    return fail(DTW_ERR_UNSUPPORTED, "pair (%d,%d) (%d x %d points, band %d): no kernel fits it", i,
                                j, w.n, w.m, w.b);
                if (!c.cyclic() && w.n > 64 * c.H * c.G)
                    return fail(DTW_ERR_UNSUPPORTED,
                                "pair (%d,%d): a shorter series of %d points is swept in row passes, whose buffer "
                                "the allocation-free entry point does not hold",
                                i, j, w.n);
                const uint32_t banded = (c.cyclic() || w.b >= 0) ? 1u : 0u;
                rec[k] = NoAllocRec{(((uint32_t)c.H * 32u + (uint32_t)c.G) * 2u + banded) * 4u + (uint32_t)w.acc,
                                    choice_cost(c, w), make_item(c, w)};
            }
        // group by instance, costliest pairs first (in place: no allocation)
        std::sort(rec, rec + n_pairs, [](const NoAllocRec &a, const NoAllocRec &b) {
            return a.kind != b.kind ? a.kind < b.kind : a.cost > b.cost;
        });
        WaveItem *it = reinterpret_cast<WaveItem *>(h + (o_items - o_src));
        for (int64_t q = 0; q < n_pairs; ++q) {
            if (q == 0 || rec[q].kind != rec[q - 1].kind) {
                if (n_groups == kMaxQueues) return fail(DTW_ERR_UNSUPPORTED, "more than %d kernel groups", kMaxQueues);
                groups[n_groups++] = Group{rec[q].kind, q, 0};
            }
            ++groups[n_groups - 1].count;
            it[q] = rec[q].item;
        }
    }

    // ---- device part: scratch address, one table copy, launches ----
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(DTW_ERR_UNSUPPORTED, "device %d out of range", dev);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    unsigned char *base = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    hipStream_t st = static_cast<hipStream_t>(o.stream);
    // synchronous copy: the host buffer is free again when it returns
    if ((e = hipMemcpyWithStream(base + o_src, h, o_queue - o_src, hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail(e, "table copy into the scratch array");
    float *ws = reinterpret_cast<float *>(base + o_ws);
    SeriesSrc *dsrc = reinterpret_cast<SeriesSrc *>(base + o_src);
    SeriesInfo *dser = reinterpret_cast<SeriesInfo *>(base + o_ser);
    DatasetInfo *dds = reinterpret_cast<DatasetInfo *>(base + o_ds);
    unsigned *dq = reinterpret_cast<unsigned *>(base + o_queue);
    if ((e = launch_stage(dsrc, dser, ws, N, st)) != hipSuccess) return hip_fail(e, "staging kernel launch");
    if (lane_w) {
        if ((e = launch_lane(lane_w, lane_acc == kAccRebased, ws, dser, dds,
                             reinterpret_cast<LaneItem *>(base + o_items), nullptr, (unsigned)n_lane, st)) != hipSuccess)
            return hip_fail(e, "lane-band kernel launch");
        return DTW_OK;
    }
    if (use_queue && (e = launch_zero(dq, n_groups, st)) != hipSuccess)  // counters start at zero every call
        return hip_fail(e, "queue reset kernel launch");
    const WaveItem *ditems = reinterpret_cast<const WaveItem *>(base + o_items);
    for (int g = 0; g < n_groups; ++g) {
        const uint32_t kind = groups[g].kind;
        const int acc = (int)(kind % 4u), banded = (int)((kind / 4u) % 2u);
        const int G = (int)((kind / 8u) % 32u), H = (int)(kind / 256u);
        unsigned *queue = use_queue ? dq + g : nullptr;
        if (G == 0)
            e = launch_cyclic(H, acc == kAccRebased, ws, dser, dds, ditems + groups[g].begin,
                              (unsigned)groups[g].count, queue, use_queue ? cyclic_resident(H, acc == kAccRebased) : 0,
                              st);
        else
            e = launch_strip(acc, StripShape{H, G}, banded != 0, ws, dser, dds, ditems + groups[g].begin,
                             (unsigned)groups[g].count, queue,
                             use_queue ? strip_resident(acc, StripShape{H, G}, banded != 0, false) : 0, nullptr, 0,
                             st);
        if (e != hipSuccess) return hip_fail(e, "wavefront kernel launch");
    }
    return DTW_OK;
}

}  // namespace

extern "C" {

int dtw_plan_create(dtw_plan *plan_out, const dtw_dataset *ds, int32_t n_datasets, const dtw_options *opt) {
    g_err.clear();
    if (!plan_out) return fail(DTW_ERR_INVALID_ARG, "plan is NULL");
    *plan_out = nullptr;
    if (n_datasets < 0) return fail(DTW_ERR_INVALID_ARG, "n_datasets=%d < 0", n_datasets);
    if (n_datasets > 0 && !ds) return fail(DTW_ERR_INVALID_ARG, "datasets is NULL");
    int rc = validate_options(opt);
    if (rc) return rc;
    for (int32_t d = 0; d < n_datasets; ++d)
        if ((rc = validate_dataset(ds[d], d))) return rc;
    return plan_build(plan_out, ds, n_datasets, opt, nullptr);
}

int dtw_plan_create_pairs(dtw_plan *plan_out, const dtw_dataset *ds, const dtw_pair *pairs, int64_t n_pairs,
                          float *out, const dtw_options *opt) {
    g_err.clear();
    if (!plan_out) return fail(DTW_ERR_INVALID_ARG, "plan is NULL");
    *plan_out = nullptr;
    int rc = validate_options(opt);
    if (rc || (rc = validate_pairs(ds, pairs, n_pairs, out))) return rc;
    const PairRequest req{pairs, n_pairs, out};
    return plan_build(plan_out, ds, 1, opt, &req);
}

int dtw_plan_execute(dtw_plan p, void *stream) {
    if (!p) return fail(DTW_ERR_INVALID_ARG, "plan is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_stage(p->d_src, p->d_ser, p->ws, p->nseries, s);
    if (e != hipSuccess) return hip_fail(e, "staging kernel launch");
    if (p->ev0 && (e = hipEventRecord(p->ev0, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if (p->n_queue && (e = launch_zero(p->d_queue, p->n_queue, s)) != hipSuccess)
        return hip_fail(e, "queue reset kernel launch");
    int q = 0;  // queue counter of the next group
    for (const LaneGroup &g : p->lane_groups)
        if ((e = launch_lane_group(p, g, s)) != hipSuccess) return hip_fail(e, "lane-band kernel launch");
    // Wavefront groups: forked over the plan's streams (round robin, costliest
    // group first), then joined back into `s` -- also after a failed launch,
    // so that `s` never returns (or ends a capture) with work of the plan's
    // streams outstanding.
    if (p->n_aux && (e = hipEventRecord(p->fork_ev, s)) != hipSuccess) return hip_fail(e, "hipEventRecord (fork)");
    int forked = 0;
    for (; forked < p->n_aux; ++forked)
        if ((e = hipStreamWaitEvent(p->aux[forked], p->fork_ev, 0)) != hipSuccess) break;
    const char *what = e != hipSuccess ? "hipStreamWaitEvent (fork)" : nullptr;
    int k = 0;
    for (size_t gi = 0; !what && gi < p->wave_groups.size(); ++gi) {
        const WaveGroup &g = p->wave_groups[gi];
        unsigned *queue = p->d_queue ? p->d_queue + q++ : nullptr;
        hipStream_t gs = p->n_aux ? p->aux[k++ % p->n_aux] : s;
        if (g.shape.G == 0)
            e = launch_cyclic(g.shape.H, g.acc == kAccRebased, p->ws, p->d_ser, p->d_ds, p->d_wave + g.begin,
                              (unsigned)g.count, queue, g.slots, gs);
        else
            e = launch_strip(g.acc, g.shape, g.banded, p->ws, p->d_ser, p->d_ds, p->d_wave + g.begin,
                             (unsigned)g.count, queue, g.slots, g.pass_buf, g.pass_stride, gs);
        if (e != hipSuccess) what = "wavefront kernel launch";
    }
    const hipError_t e_launch = e;
    for (int a = 0; a < forked; ++a) {  // join every stream that took the fork
        hipError_t ej = hipEventRecord(p->join_ev[a], p->aux[a]);
        if (ej == hipSuccess) ej = hipStreamWaitEvent(s, p->join_ev[a], 0);
        if (ej != hipSuccess && !what) {
            what = "join of the plan's streams";
            e = ej;
        }
    }
    if (what) return hip_fail(e_launch != hipSuccess ? e_launch : e, what);
    if (p->ev1) {
        if ((e = hipEventRecord(p->ev1, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        p->timed_once = true;
    }
    return DTW_OK;
}

int dtw_plan_last_kernel_ms(dtw_plan p, float *ms) {
    if (!p || !ms) return fail(DTW_ERR_INVALID_ARG, "plan or ms is NULL");
    if (!p->ev1 || !p->timed_once) return fail(DTW_ERR_INVALID_ARG, "plan was not created with DTW_FLAG_TIMING or never executed");
    hipError_t e = hipEventSynchronize(p->ev1);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    e = hipEventElapsedTime(ms, p->ev0, p->ev1);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    return DTW_OK;
}

int dtw_plan_info(dtw_plan p, dtw_plan_stats *stats) {
    if (!p || !stats) return fail(DTW_ERR_INVALID_ARG, "plan or stats is NULL");
    *stats = p->stats;
    return DTW_OK;
}

int dtw_plan_describe(dtw_plan p, char *buf, int64_t size, int64_t *needed) {
    if (!p || !needed) return fail(DTW_ERR_INVALID_ARG, "plan or needed is NULL");
    if (size > 0 && !buf) return fail(DTW_ERR_INVALID_ARG, "buf is NULL with size > 0");
    std::string j = "{\"lane_groups\": [";
    char t[256];
    for (size_t k = 0; k < p->lane_groups.size(); ++k) {
        const LaneGroup &g = p->lane_groups[k];
        snprintf(t, sizeof t,
                 "%s{\"W\": %d, \"accum\": \"%s\", \"items\": %lld, \"pairs_per_wave\": %d, "
                 "\"model_pairs_per_wave\": %d, \"tuned_ms\": {",
                 k ? ", " : "", g.W, g.rebased ? "rebased" : "plain", (long long)g.count, 64 / g.P, 64 / g.model_P);
        j += t;
        for (size_t c = 0; c < g.tuned_ms.size(); ++c) {  // measured launch time per pairs-per-wavefront value
            snprintf(t, sizeof t, "%s\"%d\": %.4g", c ? ", " : "", 64 / g.tuned_ms[c].first,
                     (double)g.tuned_ms[c].second);
            j += t;
        }
        j += "}}";
    }
    j += "], \"wave_groups\": [";
    for (size_t k = 0; k < p->wave_groups.size(); ++k) {
        const WaveGroup &g = p->wave_groups[k];
        snprintf(t, sizeof t,
                 "%s{\"kernel\": \"%s\", \"accum\": \"%s\", \"banded\": %s, \"items\": %lld, \"grid\": %lld, "
                 "\"band_cells\": %lld, \"swept_cells\": %lld, \"max_row_passes\": %lld}",
                 k ? ", " : "", choice_name(Choice{g.shape.H, g.shape.G}).c_str(), acc_name(g.acc),
                 g.banded ? "true" : "false",
                 (long long)g.count, (long long)(p->n_queue && g.slots > 0 ? std::min<int64_t>(g.slots, g.count) : g.count),
                 (long long)g.band_cells, (long long)g.swept_cells,
                 (long long)(g.shape.G ? (g.max_rows + 64LL * g.shape.H * g.shape.G - 1) / (64LL * g.shape.H * g.shape.G)
                                       : 1));
        j += t;
    }
    j += "], \"tuned\": [";
    for (size_t k = 0; k < p->tuned.size(); ++k) {
        const TunedBucket &b = p->tuned[k];
        snprintf(t, sizeof t,
                 "%s{\"n\": [%lld, %lld], \"m\": [%lld, %lld], \"band\": %s, \"accum\": \"%s\", \"pairs\": %lld, "
                 "\"model\": \"%s\", \"chosen\": \"%s\", \"applied\": %s, \"us_per_pair\": {",
                 k ? ", " : "", (long long)half_octave_lo(b.n_ho), (long long)half_octave_lo(b.n_ho + 1) - 1,
                 (long long)half_octave_lo(b.m_ho), (long long)half_octave_lo(b.m_ho + 1) - 1,
                 b.b_ho < 0 ? "null" : "[]", acc_name(b.acc), (long long)b.pairs, choice_name(b.model).c_str(),
                 choice_name(b.chosen).c_str(), b.applied ? "true" : "false");
        std::string entry = t;
        if (b.b_ho >= 0) {  // band range of the bucket: b + 1 in [lo, hi]
            snprintf(t, sizeof t, "[%lld, %lld]", (long long)half_octave_lo(b.b_ho) - 1,
                     (long long)half_octave_lo(b.b_ho + 1) - 2);
            entry.replace(entry.find("[]"), 2, t);
        }
        j += entry;
        for (size_t c = 0; c < b.us_per_pair.size(); ++c) {
            snprintf(t, sizeof t, "%s\"%s\": %.4g", c ? ", " : "", choice_name(b.us_per_pair[c].first).c_str(),
                     (double)b.us_per_pair[c].second);
            j += t;
        }
        j += "}}";
    }
    j += "], \"plan_trials\": [";  // whole-plan timings of the autotuner: buckets switched, ms per execute
    for (size_t k = 0; k < p->trials.size(); ++k) {
        snprintf(t, sizeof t, "%s{\"switched\": %d, \"ms\": %.4g}", k ? ", " : "", p->trials[k].switched,
                 (double)p->trials[k].ms);
        j += t;
    }
    j += "]}";
    *needed = (int64_t)j.size() + 1;
    if (size < *needed) {
        if (size > 0) buf[0] = '\0';
        return size > 0 ? fail(DTW_ERR_INVALID_ARG, "buffer of %lld bytes, %lld needed", (long long)size,
                               (long long)*needed)
                        : DTW_OK;
    }
    memcpy(buf, j.c_str(), j.size() + 1);
    return DTW_OK;
}

int dtw_plan_destroy(dtw_plan p) {
    if (!p) return fail(DTW_ERR_INVALID_ARG, "plan is NULL");
    destroy_plan(p);
    return DTW_OK;
}

int dtw_pairwise_ex(const dtw_dataset *ds, const dtw_options *opt) {
    g_err.clear();
    if (!ds) return fail(DTW_ERR_INVALID_ARG, "dataset is NULL");
    int rc = validate_options(opt);
    if (rc) return rc;
    if ((rc = validate_dataset(*ds, 0))) return rc;
    if (ds->N < 2) return DTW_OK;  // nothing to write, no HIP call
    return cached_run(*ds, opt, nullptr);
}

int dtw_pairs(const dtw_dataset *ds, const dtw_pair *pairs, int64_t n_pairs, float *out, const dtw_options *opt) {
    g_err.clear();
    int rc = validate_options(opt);
    if (rc || (rc = validate_pairs(ds, pairs, n_pairs, out))) return rc;
    if (n_pairs == 0) return DTW_OK;  // nothing to write, no HIP call
    const PairRequest req{pairs, n_pairs, out};
    return cached_run(*ds, opt, &req);
}

int dtw_pairwise_noalloc(const dtw_dataset *ds, const dtw_options *opt) {
    g_err.clear();
    if (!ds) return fail(DTW_ERR_INVALID_ARG, "dataset is NULL");
    int rc = validate_options(opt);
    if (rc) return rc;
    if ((rc = validate_dataset(*ds, 0))) return rc;
    if (ds->N < 2) return DTW_OK;  // nothing to write, no HIP call
    dtw_options o{};
    if (opt) o = *opt;
    return noalloc_run(*ds, o);
}

int dtw_pairwise(const float *series, const int32_t *lengths, const int64_t *offsets, int32_t N, int32_t window,
                 float *out_condensed) {
    dtw_dataset d{series, lengths, offsets, N, window, out_condensed};
    return dtw_pairwise_ex(&d, nullptr);
}

}  // extern "C"
