// Host side of the C ABI: validation, pair enumeration and tiling, workspace
// layout, plan execution.  See include/dtwmi.h for the contract.
//
// Pair enumeration.  The paper computes all p(p-1)/2 pairwise distances
// ("Mathematical background") and fills the symmetric matrix D.  This library
// writes each unordered pair once into the condensed upper triangle.
//  * lane-band datasets (all series of equal length, narrow band, PLAIN):
//    series a is paired with the series at cyclic distances 1..h_a
//    ((a+d) mod N), h_a = floor((N-1)/2), plus the pair at distance N/2 for
//    a < N/2 when N is even.  Every unordered pair appears exactly once and
//    every series gets the same number of partners, so the 64-pair work items
//    are almost all full.
//  * wavefront datasets: one item per pair (i<j).  Each pair goes either to a
//    strip kernel (the shorter series spread over the lanes, every column
//    swept) or, with PLAIN accumulation and a window, to the cyclic kernel
//    (blocks of the longer series cycling over the lanes, each block visiting
//    only its window), whichever a step-count cost model finds cheaper.
//    Items are grouped by kernel instance and each group is sorted by
//    decreasing cost, so the longest pairs start first.
#include "dtw_internal.h"
#include "dtwmi.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
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

int64_t effective_band(int32_t w, int32_t n, int32_t m) {
    if (w < 0) return -1;
    const int64_t d = n > m ? (int64_t)n - m : (int64_t)m - n;
    const int64_t b = std::max<int64_t>(w, d);
    return b >= std::max(n, m) - 1 ? -1 : b;
}

struct LaneGroup {
    int W;
    int64_t begin, count;
};

struct WaveGroup {
    StripShape shape;  // G == 0: cyclic kernel with H = shape.H
    bool banded;
    int64_t begin, count;
    int slots = 0;  // resident workgroups of the kernel (queue mode)
};

// Strip shape for a pair whose shorter series has n points: the instantiated
// shape of smallest row capacity 64*H*G >= n, restricted to H == force_h when
// force_h > 0 ({0,0} if none fits).
StripShape pick_strip(int accum, int n, int force_h) {
    StripShape shapes[64];
    const int k = strip_shapes(accum, shapes, 64);
    for (int i = 0; i < k && i < 64; ++i)
        if (64 * shapes[i].H * shapes[i].G >= n && (force_h <= 0 || shapes[i].H == force_h)) return shapes[i];
    return StripShape{0, 0};
}

// Cost model shared by both wavefront families: wavefront-steps times VALU
// instructions per step (3 per cell row plus loop overhead per step), from
// the instruction mix of the compiled loops.
constexpr int64_t kStripStepOverhead = 15;
constexpr int64_t kCyclicStepOverhead = 20;

// Steps a strip workgroup takes on an n x m pair (n = rows spread over lanes).
int64_t strip_steps(StripShape sh, int64_t n, int64_t m) {
    const int64_t lanes = (n - 1) / sh.H;  // last lane holding a row
    return m + lanes % 64 + (lanes / 64) * (64 + (sh.G > 1 ? 16 : 0));
}

int64_t strip_cost(StripShape sh, int64_t n, int64_t m) {
    return sh.G * strip_steps(sh, n, m) * (3 * sh.H + kStripStepOverhead);
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
    return cyclic_steps(H, n, m) * (3 * H + kCyclicStepOverhead);
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

int max_strip_rows(int accum) {
    StripShape shapes[64];
    const int k = strip_shapes(accum, shapes, 64);
    int best = 0;
    for (int i = 0; i < k && i < 64; ++i) best = std::max(best, 64 * shapes[i].H * shapes[i].G);
    return best;
}

}  // namespace

struct dtw_plan_s {
    int device = 0;
    int dtype = 0, accum = 0, kernel = 0, flags = 0;
    int32_t nseries = 0;
    void *dev_block = nullptr;  // one allocation holding everything below
    size_t dev_bytes = 0;
    float *ws = nullptr;
    SeriesSrc *d_src = nullptr;
    SeriesInfo *d_ser = nullptr;
    DatasetInfo *d_ds = nullptr;
    LaneItem *d_lane = nullptr;
    WaveItem *d_wave = nullptr;
    unsigned *d_queue = nullptr;  // one counter per wavefront group, zeroed by every execute
    int n_queue = 0;
    std::vector<LaneGroup> lane_groups;
    std::vector<WaveGroup> wave_groups;
    dtw_plan_stats stats{};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed_once = false;
};

namespace {

int validate_options(const dtw_options *opt) {
    if (!opt) return DTW_OK;
    if (opt->dtype < DTW_F32 || opt->dtype > DTW_F16) return fail(DTW_ERR_INVALID_ARG, "unknown dtype %d", opt->dtype);
    if (opt->accum < DTW_ACC_PLAIN || opt->accum > DTW_ACC_FP64)
        return fail(DTW_ERR_INVALID_ARG, "unknown accumulation mode %d", opt->accum);
    if (opt->kernel < DTW_KERNEL_AUTO || opt->kernel > DTW_KERNEL_CYCLIC)
        return fail(DTW_ERR_INVALID_ARG, "unknown kernel family %d", opt->kernel);
    if (opt->rows_per_lane < 0 || opt->rows_per_lane > 64)
        return fail(DTW_ERR_INVALID_ARG, "rows_per_lane=%d outside 0..64", opt->rows_per_lane);
    if (opt->kernel == DTW_KERNEL_CYCLIC && opt->accum != DTW_ACC_PLAIN)
        return fail(DTW_ERR_UNSUPPORTED, "the cyclic kernel needs PLAIN accumulation");
    if (opt->flags & ~(DTW_FLAG_TIMING | DTW_FLAG_NO_QUEUE))
        return fail(DTW_ERR_INVALID_ARG, "unknown flags 0x%x", opt->flags);
    return DTW_OK;
}

int validate_dataset(const dtw_dataset &d, int idx) {
    if (d.N < 0) return fail(DTW_ERR_INVALID_ARG, "dataset %d: N=%d < 0", idx, d.N);
    if (d.N < 2) return DTW_OK;
    if (!d.series) return fail(DTW_ERR_INVALID_ARG, "dataset %d: series is NULL", idx);
    if (!d.out_condensed) return fail(DTW_ERR_INVALID_ARG, "dataset %d: out_condensed is NULL", idx);
    if (!d.lengths || !d.offsets) return fail(DTW_ERR_INVALID_ARG, "dataset %d: lengths/offsets is NULL", idx);
    for (int32_t s = 0; s < d.N; ++s) {
        if (d.lengths[s] < 1) return fail(DTW_ERR_INVALID_ARG, "dataset %d: lengths[%d]=%d < 1", idx, s, d.lengths[s]);
        if (d.offsets[s] < 0) return fail(DTW_ERR_INVALID_ARG, "dataset %d: offsets[%d] < 0", idx, s);
    }
    return DTW_OK;
}

void destroy_plan(dtw_plan p) {
    if (!p) return;
    if (p->dev_block) (void)hipFree(p->dev_block);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    delete p;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

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

    const int dtype = opt ? opt->dtype : DTW_F32;
    const int accum = opt ? opt->accum : DTW_ACC_PLAIN;
    const int kernel = opt ? opt->kernel : DTW_KERNEL_AUTO;
    const int flags = opt ? opt->flags : 0;
    const int force_h = opt ? opt->rows_per_lane : 0;

    // ---- host-side planning (no HIP calls) ----
    std::vector<SeriesSrc> src;
    std::vector<SeriesInfo> ser;
    std::vector<DatasetInfo> dsi;
    std::vector<LaneItem> lane_items;
    std::map<int, std::vector<LaneItem>> lane_by_w;
    // wave items by kernel instance (H, G, banded); G == 0 is the cyclic kernel
    std::map<std::tuple<int, int, bool>, std::vector<std::pair<int64_t, WaveItem>>> wave_by_kind;
    dtw_plan_stats st{};
    size_t ws_floats = 0;
    const size_t elem = dtype == DTW_F32 ? 4 : 2;

    for (int32_t d = 0; d < n_datasets; ++d) {
        const dtw_dataset &D = ds[d];
        DatasetInfo info{};
        info.out = D.out_condensed;
        info.N = D.N;
        info.window = D.window;
        info.series_base = static_cast<int32_t>(ser.size());
        if (D.N < 2) {
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
        (void)elem;
        info.L = uniform ? D.lengths[0] : -1;
        dsi.push_back(info);
        const int64_t npairs = (int64_t)D.N * (D.N - 1) / 2;
        st.pairs += npairs;

        // Kernel family for this dataset.
        int lane_w = 0;
        if (uniform && accum == DTW_ACC_PLAIN) {
            const int32_t L = D.lengths[0];
            const int32_t b = (D.window < 0 || D.window >= L - 1) ? L - 1 : D.window;
            if (lane_width_supported(2 * b + 1)) lane_w = 2 * b + 1;
        }
        if (kernel == DTW_KERNEL_LANE && !lane_w)
            return fail(DTW_ERR_UNSUPPORTED,
                        "dataset %d: the lane-band kernel needs equal lengths, PLAIN accumulation and 2*w+1 <= %d",
                        d, kLaneMaxW);
        if (kernel == DTW_KERNEL_WAVE || kernel == DTW_KERNEL_CYCLIC) lane_w = 0;

        if (lane_w) {
            const int32_t N = D.N, L = D.lengths[0], b = (lane_w - 1) / 2;
            st.band_cells += npairs * band_cells(L, L, b >= L - 1 ? -1 : b);
            for (int32_t a = 0; a < N; ++a) {
                int32_t h = (N - 1) / 2;
                if (N % 2 == 0 && a < N / 2) h = N / 2;
                for (int32_t d0 = 1; d0 <= h; d0 += 64) {
                    const int32_t cnt = std::min(64, h - d0 + 1);
                    lane_by_w[lane_w].push_back(LaneItem{d, a, d0, cnt});
                    st.computed_cells += (int64_t)64 * L * lane_w;
                }
            }
        } else {
            for (int32_t i = 0; i < D.N; ++i) {
                for (int32_t j = i + 1; j < D.N; ++j) {
                    const int32_t ni = D.lengths[i], nj = D.lengths[j];
                    const bool swap = nj < ni;
                    const int32_t shorter = swap ? j : i, longer = swap ? i : j;
                    const int32_t n = std::min(ni, nj), m = std::max(ni, nj);
                    const int64_t b = effective_band(D.window, n, m);
                    const int64_t cells = band_cells(n, m, b);
                    st.band_cells += cells;
                    // cyclic candidate: PLAIN, a window, rows = the longer series
                    int64_t cyc_cost = 0;
                    const int cyc_h = (accum == DTW_ACC_PLAIN && b >= 0 && kernel != DTW_KERNEL_WAVE)
                                          ? pick_cyclic(m, n, b, force_h, &cyc_cost)
                                          : 0;
                    const StripShape sh = kernel == DTW_KERNEL_CYCLIC && cyc_h ? StripShape{0, 0}
                                                                               : pick_strip(accum, n, force_h);
                    if (!sh.H && !cyc_h) {
                        if (force_h > 0)
                            return fail(DTW_ERR_UNSUPPORTED,
                                        "dataset %d: pair (%d,%d) (%d x %d points, band %lld): no kernel with "
                                        "rows_per_lane=%d fits it",
                                        d, i, j, n, m, (long long)b, force_h);
                        return fail(DTW_ERR_UNSUPPORTED,
                                    "dataset %d: pair (%d,%d) has both series longer than %d points", d, i, j,
                                    max_strip_rows(accum));
                    }
                    const int64_t s_cost = sh.H ? strip_cost(sh, n, m) : 0;
                    if (cyc_h && (!sh.H || cyc_cost < s_cost)) {
                        st.computed_cells += (int64_t)64 * cyc_h * cyclic_steps(cyc_h, m, n);
                        ++st.n_cyclic_items;
                        wave_by_kind[std::make_tuple(cyc_h, 0, true)].push_back(
                            {cyc_cost, WaveItem{d, longer, shorter, (int32_t)b}});
                    } else {
                        st.computed_cells += (int64_t)64 * sh.G * sh.H * strip_steps(sh, n, m);
                        wave_by_kind[std::make_tuple(sh.H, sh.G, b >= 0)].push_back(
                            {s_cost, WaveItem{d, shorter, longer, (int32_t)b}});
                    }
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

    std::vector<WaveItem> wave_items;
    for (auto &kv : lane_by_w) {
        p->lane_groups.push_back(LaneGroup{kv.first, (int64_t)lane_items.size(), (int64_t)kv.second.size()});
        lane_items.insert(lane_items.end(), kv.second.begin(), kv.second.end());
    }
    // Inside a group, costlier pairs first; groups in decreasing order of their
    // costliest pair.
    std::vector<decltype(wave_by_kind)::iterator> order;
    for (auto it = wave_by_kind.begin(); it != wave_by_kind.end(); ++it) {
        std::stable_sort(it->second.begin(), it->second.end(),
                         [](const std::pair<int64_t, WaveItem> &a, const std::pair<int64_t, WaveItem> &b) {
                             return a.first > b.first;
                         });
        order.push_back(it);
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const auto &a, const auto &b) { return a->second[0].first > b->second[0].first; });
    for (auto it : order) {
        auto &v = it->second;
        const StripShape sh{std::get<0>(it->first), std::get<1>(it->first)};
        p->wave_groups.push_back(
            WaveGroup{sh, std::get<2>(it->first), (int64_t)wave_items.size(), (int64_t)v.size(), 0});
        for (auto &e : v) wave_items.push_back(e.second);
    }
    st.n_lane_items = static_cast<int32_t>(lane_items.size());
    st.n_wave_items = static_cast<int64_t>(wave_items.size());
    const int n_groups = (int)(p->lane_groups.size() + p->wave_groups.size());
    for (const LaneGroup &g : p->lane_groups)
        if (g.count > 0x7fffffff) {
            delete p;
            return fail(DTW_ERR_UNSUPPORTED, "more than 2^31-1 work items for one kernel");
        }
    for (const WaveGroup &g : p->wave_groups)
        if (g.count > 0x7fffffff) {
            delete p;
            return fail(DTW_ERR_UNSUPPORTED, "more than 2^31-1 work items for one kernel");
        }
    const bool use_queue = !(flags & DTW_FLAG_NO_QUEUE) && !p->wave_groups.empty();
    p->n_queue = use_queue ? (int)p->wave_groups.size() : 0;
    st.n_launches = (p->nseries > 0 ? 1 : 0) + (use_queue ? 1 : 0) + n_groups;

    // ---- device allocation and upload ----
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
    const size_t o_wave = off;
    off = align_up(off + wave_items.size() * sizeof(WaveItem), 256);
    const size_t o_queue = off;
    off = align_up(off + p->n_queue * sizeof(unsigned), 256);
    p->dev_bytes = off;
    st.workspace_bytes = static_cast<int64_t>(off);
    p->stats = st;

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
    p->d_wave = reinterpret_cast<WaveItem *>(base + o_wave);
    p->d_queue = p->n_queue ? reinterpret_cast<unsigned *>(base + o_queue) : nullptr;
    if (use_queue) {  // grid of each launch: the workgroups the device holds at once
        for (WaveGroup &g : p->wave_groups)
            g.slots = g.shape.G == 0 ? cyclic_resident(g.shape.H) : strip_resident(accum, g.shape, g.banded);
    }
    struct Up {
        void *dst;
        const void *src;
        size_t bytes;
    } ups[] = {{p->d_src, src.data(), src.size() * sizeof(SeriesSrc)},
               {p->d_ser, ser.data(), ser.size() * sizeof(SeriesInfo)},
               {p->d_ds, dsi.data(), dsi.size() * sizeof(DatasetInfo)},
               {p->d_lane, lane_items.data(), lane_items.size() * sizeof(LaneItem)},
               {p->d_wave, wave_items.data(), wave_items.size() * sizeof(WaveItem)}};
    for (const Up &u : ups) {
        if (!u.bytes) continue;
        e = hipMemcpy(u.dst, u.src, u.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            destroy_plan(p);
            return hip_fail(e, "hipMemcpy (plan upload)");
        }
    }
    if (flags & DTW_FLAG_TIMING) {
        if ((e = hipEventCreate(&p->ev0)) != hipSuccess || (e = hipEventCreate(&p->ev1)) != hipSuccess) {
            destroy_plan(p);
            return hip_fail(e, "hipEventCreate");
        }
    }
    *plan_out = p;
    return DTW_OK;
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
    for (const LaneGroup &g : p->lane_groups) {
        e = launch_lane(g.W, p->ws, p->d_ser, p->d_ds, p->d_lane + g.begin, (unsigned)g.count, s);
        if (e != hipSuccess) return hip_fail(e, "lane-band kernel launch");
    }
    for (const WaveGroup &g : p->wave_groups) {
        unsigned *queue = p->d_queue ? p->d_queue + q++ : nullptr;
        if (g.shape.G == 0)
            e = launch_cyclic(g.shape.H, p->ws, p->d_ser, p->d_ds, p->d_wave + g.begin, (unsigned)g.count, queue,
                              g.slots, s);
        else
            e = launch_strip(p->accum, g.shape, g.banded, p->ws, p->d_ser, p->d_ds, p->d_wave + g.begin,
                             (unsigned)g.count, queue, g.slots, s);
        if (e != hipSuccess) return hip_fail(e, "wavefront kernel launch");
    }
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
    dtw_options o{};
    if (opt) o = *opt;
    o.flags &= DTW_FLAG_NO_QUEUE;  // timing needs the plan API
    dtw_plan p = nullptr;
    rc = dtw_plan_create(&p, ds, 1, &o);
    if (rc) return rc;
    rc = dtw_plan_execute(p, o.stream);
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(o.stream));
    destroy_plan(p);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return DTW_OK;
}

int dtw_pairwise(const float *series, const int32_t *lengths, const int64_t *offsets, int32_t N, int32_t window,
                 float *out_condensed) {
    dtw_dataset d{series, lengths, offsets, N, window, out_condensed};
    return dtw_pairwise_ex(&d, nullptr);
}

}  // extern "C"
