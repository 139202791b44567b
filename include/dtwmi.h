/*
 * dtwmi.h -- C ABI of the MI355X (gfx950) all-pairs dynamic time warping library.
 *
 * What is computed (paper "Fast dynamic time warping and clustering in C++",
 * section "Mathematical background"):
 *   - for two series x (length n) and y (length m), the cumulative cost of
 *     Eq. (c):  c(i,j) = (x_i - y_j)^2 + min{c(i-1,j-1), c(i-1,j), c(i,j-1)},
 *     c(0,0) = 0, c(i,0) = c(0,j) = +inf (1-based), result c(n,m).  No square
 *     root is taken.
 *   - a warping window w (paper, Introduction: a window of 99 lets the first
 *     point reach at most the hundredth point of the other series): cell
 *     (i,j) is admissible iff |i-j| <= max(w, |n-m|); w < 0 means no window.
 *     Inadmissible cells are +inf.
 *   - the symmetric distance matrix D with d(i,j) = cost of the pair (i,j)
 *     (same section, figure "c_to_d"), stored as its condensed upper
 *     triangle: entry k(i,j) = i*N - i*(i+1)/2 + (j-i-1) for 0 <= i < j < N,
 *     row-major, N*(N-1)/2 floats.  The zero diagonal is not stored.
 *
 * Conventions common to every entry point:
 *   - Every function returns a dtw_status.  Nothing aborts, throws or prints.
 *     On failure dtw_last_error() returns a message for the calling thread.
 *   - "device" pointers are HIP device memory (hipMalloc or a torch tensor on
 *     the GPU); "host" pointers are ordinary CPU memory.  The caller owns every
 *     buffer it passes in.
 *   - All arguments are validated on the host before any HIP call.
 *   - Series values must be finite; results for NaN or inf inputs are
 *     unspecified.  The output is always FP32.
 *   - Series may have any length from 1 to 2^28 points (longer returns
 *     DTW_ERR_UNSUPPORTED).  A pair whose shorter series has more rows than one
 *     workgroup holds (32768 points with PLAIN or REBASED sums, 16384 with
 *     KAHAN or FP64) is swept in row passes through a device buffer the plan
 *     allocates (one row of the longer series per resident workgroup);
 *     dtw_pairwise_noalloc rejects such pairs.  dtw_path has its own limit.
 */
#ifndef DTWMI_H
#define DTWMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DTW_OK = 0,
    DTW_ERR_INVALID_ARG = 1,   /* bad pointer, count, length, enum value */
    DTW_ERR_UNSUPPORTED = 2,   /* valid request outside what the kernels cover */
    DTW_ERR_OUT_OF_MEMORY = 3, /* device or host allocation failed */
    DTW_ERR_HIP = 4            /* a HIP runtime call or kernel launch failed */
} dtw_status;

/* Storage type of the input series (all accumulate in FP32 or FP64). */
typedef enum { DTW_F32 = 0, DTW_BF16 = 1, DTW_F16 = 2 } dtw_dtype;

/* Accumulation of the cumulative cost.  The paper fixes no precision; the
 * accuracy target here is a relative error of at most 1e-5 against an exact
 * (FP64) evaluation of Eq. (c) for FP32 inputs.
 *   AUTO:    (the default, 0) per pair: PLAIN when the longest warping path,
 *            n+m-1 cells, has at most 2048 cells; beyond, REBASED when the
 *            pair has a window (max(w, |n-m|) < max(n,m)-1) or the path has
 *            at most 4096 cells; longer unwindowed paths FP64.
 *   PLAIN:   FP32 sub, min, fused multiply-add per cell.  Each add rounds
 *            relative to the whole cumulative cost, so the error grows with
 *            the path length: within 1e-5 up to paths of 2048 cells, about
 *            1e-5 at 8191 (4096-point series), within 1e-4 beyond.
 *   KAHAN:   FP32 with a compensation term carried per cell and a compensated
 *            add of every local cost (the min takes the smallest running sum
 *            and, among equal sums, the largest compensation).
 *   FP64:    the whole recurrence in FP64, the final cost rounded once to FP32.
 *   REBASED: the PLAIN cell on values stored relative to a base that each
 *            wavefront (each lane, in the lane-band kernel) moves up every few
 *            steps to a lower bound of every value it computes later, so each
 *            add rounds relative to the stored value instead of the whole
 *            cost: never less accurate than PLAIN, typically several times
 *            more (about 10x with a window), at 1-3% above its cost. */
typedef enum {
    DTW_ACC_AUTO = 0,
    DTW_ACC_PLAIN = 1,
    DTW_ACC_KAHAN = 2,
    DTW_ACC_FP64 = 3,
    DTW_ACC_REBASED = 4
} dtw_accum;

/* Kernel family; AUTO picks per dataset and per pair.  The others exist for
 * tests and benchmarks.
 *   LANE:   one pair per lane, the band row kept in registers (all series of
 *           the dataset of equal length, 2*w+1 <= 127; AUTO, PLAIN or REBASED).
 *   WAVE:   one pair per workgroup of 1..16 wavefronts sweeping anti-diagonals,
 *           each lane owning a strip of rows (any lengths, any window, any
 *           accumulation).
 *   CYCLIC: one pair per wavefront; blocks of rows of the longer series cycle
 *           over the 64 lanes and each block only visits the columns its window
 *           admits (AUTO, PLAIN or REBASED).  Pairs without a window, or whose
 *           window is too wide for any instantiated block height, use WAVE. */
typedef enum { DTW_KERNEL_AUTO = 0, DTW_KERNEL_LANE = 1, DTW_KERNEL_WAVE = 2, DTW_KERNEL_CYCLIC = 3 } dtw_kernel;

/* One dataset: N series concatenated in one device buffer. */
typedef struct dtw_dataset {
    const void *series;     /* device: values of all series, element type given by dtw_options.dtype */
    const int32_t *lengths; /* host: N lengths, each >= 1 */
    const int64_t *offsets; /* host: N element offsets of each series inside `series`, >= 0 */
    int32_t N;              /* number of series, >= 0; N < 2 writes nothing */
    int32_t window;         /* Sakoe-Chiba window w; < 0 = no window */
    float *out_condensed;   /* device: N*(N-1)/2 floats, written in condensed order */
} dtw_dataset;

/* Options; a zero-initialised struct means FP32 storage, AUTO accumulation,
 * AUTO kernel, no flags, the default stream and every pair. */
typedef struct dtw_options {
    int32_t dtype;  /* dtw_dtype */
    int32_t accum;  /* dtw_accum (0 = AUTO) */
    int32_t kernel; /* dtw_kernel (0 = AUTO) */
    int32_t flags;  /* DTW_FLAG_* bits: TIMING (plan API only), NO_QUEUE, AUTOTUNE */
    int32_t rows_per_lane; /* 0 = automatic.  Else the rows each lane holds in the WAVE and
                              CYCLIC kernels (1..64); a value with no instantiated kernel for a
                              pair returns DTW_ERR_UNSUPPORTED.  Ignored by LANE. */
    int32_t pairs_per_wave; /* LANE kernel: pairs per wavefront.  0 = automatic: 64 (one pair
                              per lane) when that gives every SIMD of the device at least two
                              wavefronts, else 16, 8, 5, 4 or 2 by an estimate of the time (each
                              pair's band row spread over 4, 8, 12, 16 or 32 lanes; with 12 the
                              last 4 lanes idle; PLAIN sums only; same results bit for bit).
                              64, 16, 8, 5, 4 or 2 forces it; a split the band width has no
                              instance for (3 to 16 band cells per lane, at most 11 with 5 pairs
                              per wavefront, 8 with 4 and 4 with 2) or REBASED sums returns
                              DTW_ERR_UNSUPPORTED.  Other values are DTW_ERR_INVALID_ARG.
                              Ignored by WAVE and CYCLIC and by dtw_pairwise_noalloc (which
                              runs 64). */
    void *stream;   /* hipStream_t used by dtw_pairwise_ex and dtw_pairs; NULL = default stream */
    /* Output sub-range: only the entries k with k_begin <= k < k_end of every
     * dataset's output are evaluated and written (the condensed index k(i,j)
     * for all-pairs plans, the list position for pair lists); the other
     * entries are left untouched.  k_end <= 0 means the end of the output;
     * 0, 0 is every pair.  k_begin < 0, or 0 < k_end < k_begin, is
     * DTW_ERR_INVALID_ARG; a range past a dataset's output is clipped to it.
     * Splitting [0, N(N-1)/2) into ranges splits the work of a matrix into
     * independent parts (one per device or per call) with no exchange. */
    int64_t k_begin, k_end;
} dtw_options;

#define DTW_FLAG_TIMING 1
/* Launch one workgroup per work item (hardware dispatch order) instead of the
 * default: a grid of resident workgroups pulling cost-sorted items from a
 * device counter that every execute resets with a small kernel. */
#define DTW_FLAG_NO_QUEUE 2
/* Plan creation measures, for every bucket of wavefront pairs with similar
 * shorter length, longer length and window (half-octave ranges), up to four
 * kernel instances that can run all of them (strip shapes and cyclic block
 * heights, best by the cost model first) and gives the bucket the fastest.
 * Timing launches run on the default stream, repeat a sample of the bucket's
 * pairs until they fill the device, and write those pairs' results into the
 * outputs (every execute overwrites them).  dtw_plan_describe reports the
 * measurements.  Without it the cost model alone picks. */
#define DTW_FLAG_AUTOTUNE 4

typedef struct dtw_plan_s *dtw_plan;

/* Statistics of a plan (host values, filled by dtw_plan_info). */
typedef struct dtw_plan_stats {
    int64_t pairs;           /* number of pairs (condensed entries) written per execute */
    int64_t band_cells;      /* admissible DP cells summed over all pairs */
    int64_t computed_cells;  /* cells the kernels sweep, padding included */
    int64_t workspace_bytes; /* device memory owned by the plan */
    int32_t n_launches;      /* kernel launches per execute, staging included */
    int32_t n_lane_items;    /* LANE work items (64 pairs each) */
    int64_t n_wave_items;    /* WAVE and CYCLIC work items (one pair each) */
    int64_t n_cyclic_items;  /* the CYCLIC ones among them */
    int32_t n_tuned_buckets; /* buckets timed by DTW_FLAG_AUTOTUNE */
    int32_t n_tuned_changed; /* of which the measurement overruled the cost model */
} dtw_plan_stats;

/*
 * Short form: FP32 input, AUTO accumulation, default stream, automatic kernel.
 * series: device; lengths, offsets: host; out_condensed: device.
 * Enqueues the evaluation on the default stream and returns; the result is
 * valid after that stream is synchronised.  The short forms (this one,
 * dtw_pairwise_ex, dtw_pairs) keep the plans they build in a cache of the
 * library, keyed by device, stream, options and the dataset's shape (N,
 * window, lengths, offsets, and the pair list for dtw_pairs), not by the
 * buffers: a call whose key is cached re-points the plan at its own series
 * and output buffers with one small kernel and launches it, without any
 * allocation, upload or synchronisation.  A call whose key is new builds a
 * plan (device allocation and upload of its tables, which block the host)
 * first.  The cache holds up to 8 plans per process; replacing the least
 * recently used one waits for that plan's last launch to finish.  Calls that
 * share a key must be made from one host thread at a time (the cache itself is
 * thread-safe).
 */
int dtw_pairwise(const float *series, const int32_t *lengths, const int64_t *offsets,
                 int32_t N, int32_t window, float *out_condensed);

/* One dataset with explicit options (NULL = all zero), enqueued on opt->stream
 * like dtw_pairwise.  DTW_FLAG_TIMING is ignored (it needs the plan API). */
int dtw_pairwise_ex(const dtw_dataset *ds, const dtw_options *opt);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as dtw_pairwise_ex, with every device workspace -- the padded
 * FP32 copy of the series, the series, dataset and work-item tables and the
 * queue counters -- in a static device array of 32 MiB that the library holds
 * on each device it runs on until the process ends.  It calls no allocating
 * routine: the tables are built in a static host buffer and copied into that
 * array with a synchronous copy on opt->stream (which waits for earlier work
 * on that stream), then the kernels are enqueued and the call returns; the
 * result is valid after the stream is synchronised.  The queue counters are
 * cleared by a kernel on every call.  All calls on one device share the
 * array: a call overwrites what the previous one left there, so calls whose
 * work overlaps on one device (different streams, or threads without
 * ordering) race and must not be made.
 * Returns DTW_ERR_UNSUPPORTED when the dataset needs more than the array
 * holds (the padded series take 4*(length + 256) bytes each, plus 24 bytes
 * per work item: up to ~28 MB of series and items together), with
 * DTW_FLAG_AUTOTUNE (it allocates), with an output range other than 0, 0 and
 * for a pair swept in row passes (see the length rule above: the pass buffer
 * would not fit the array); otherwise it accepts and rejects what dtw_pairwise_ex does.  Kernel choice follows the cost
 * model (no plan-wide grouping across calls); results equal those of
 * dtw_pairwise_ex for the same options up to the rounding of rebased sums.
 */
int dtw_pairwise_noalloc(const dtw_dataset *ds, const dtw_options *opt);

/*
 * Plans: validate, enumerate and tile all pairs of n_datasets datasets once,
 * allocate the device workspace and upload the tile lists.  The plan keeps
 * the dataset device pointers (series, out_condensed) and the caller keeps
 * them alive, with unchanged lengths, until dtw_plan_destroy.  Host arrays
 * are copied and may be freed after dtw_plan_create returns.
 */
int dtw_plan_create(dtw_plan *plan, const dtw_dataset *ds, int32_t n_datasets,
                    const dtw_options *opt);

/*
 * Enqueue one full evaluation (staging of the inputs into the padded FP32
 * workspace, then every DP kernel) on `stream` (hipStream_t, NULL = default).
 * Allocates nothing and never synchronises, so it may be captured into a HIP
 * graph: kernel groups of different instances run concurrently on up to four
 * streams the plan owns, forked from `stream` and joined back into it by
 * events.  Results are valid after the stream is synchronised.  Executions of
 * one plan on different streams must not overlap (they share the workspace).
 */
int dtw_plan_execute(dtw_plan plan, void *stream);

/* Milliseconds spent in the DP kernels by the last execute (DTW_FLAG_TIMING plans only); synchronises on the end event. */
int dtw_plan_last_kernel_ms(dtw_plan plan, float *ms);

int dtw_plan_info(dtw_plan plan, dtw_plan_stats *stats);

/*
 * JSON text describing the plan: kernel groups (instance, items, grid) and,
 * with DTW_FLAG_AUTOTUNE, every timed bucket (length and band ranges, pairs,
 * the cost model's pick, the chosen instance, microseconds per pair of each
 * candidate).  Writes at most `size` bytes including the terminating NUL into
 * buf (host) and the bytes needed into *needed; size 0 only queries *needed.
 * A buffer that is too small gets an empty string and DTW_ERR_INVALID_ARG.
 */
int dtw_plan_describe(dtw_plan plan, char *buf, int64_t size, int64_t *needed);

int dtw_plan_destroy(dtw_plan plan);

/*
 * Pair subsets.  Some uses need only some distances: k-medoids evaluates each
 * series against the current medoids, not every pair (the paper's clustering
 * section).  A pair list names series of one dataset; i == j is allowed (its
 * cost is 0) and a pair may appear several times.
 */
typedef struct dtw_pair {
    int32_t i, j; /* series indices, 0 <= i, j < N */
} dtw_pair;

/*
 * Plan for a pair list of one dataset: out (device, n_pairs floats) receives
 * out[k] = DTW(series pairs[k].i, series pairs[k].j) at every execute.
 * ds->out_condensed is ignored (may be NULL).  pairs (host) is copied and may
 * be freed after the call; ds->series and out stay owned by the caller and
 * must stay alive until dtw_plan_destroy.  Pairs of an equal-length dataset
 * with 2*w+1 <= 127 (PLAIN) run on the lane-band kernel in tiles of 64 pairs
 * that share a series (the series named most often in the list); all others
 * on the wavefront kernels.  Indices outside 0..N-1 return DTW_ERR_INVALID_ARG.
 */
int dtw_plan_create_pairs(dtw_plan *plan, const dtw_dataset *ds, const dtw_pair *pairs, int64_t n_pairs,
                          float *out, const dtw_options *opt);

/* Short form of a pair-list plan, enqueued on opt->stream with the plan cache
 * of dtw_pairwise (the list is part of the key; series and out are not). */
int dtw_pairs(const dtw_dataset *ds, const dtw_pair *pairs, int64_t n_pairs, float *out, const dtw_options *opt);

/*
 * Clustering scores from a condensed distance matrix D (device, N(N-1)/2
 * floats in the order above, e.g. the output of a plan).  The paper's method,
 * after D, clusters the series around centroid series and reports the
 * clustering cost -- the sum of the distances between every series and its
 * cluster's centroid -- and a silhouette score to choose the number of
 * clusters (Introduction, list of the method's steps).  The silhouette is
 * Rousseeuw's: a(i) = mean distance to the other members of i's cluster,
 * b(i) = smallest mean distance to another non-empty cluster,
 * s(i) = (b-a)/max(a,b) (0 when both are 0), 0 for a one-member cluster.
 * All sums are FP64 in a fixed order (the same result on every run).
 * labels (device int32[N], values 0..K-1) and centroids (device int32[K],
 * series indices) are copied to the host and range-checked first
 * (DTW_ERR_INVALID_ARG).  These calls allocate a device workspace, run on
 * `stream` (hipStream_t, NULL = default) and synchronise it before
 * returning; host outputs are valid on return.
 */

/* s (device float[N], may be NULL): s(i); *mean (host): the mean of s.
 * 2 <= K <= 64; at least two clusters must be non-empty. */
int dtw_silhouette(const float *D, int32_t N, const int32_t *labels, int32_t K, float *s, double *mean,
                   void *stream);

/* Clustering cost of a labelling: *total (host) = sum of D(i, centroids[labels[i]]);
 * per_cluster (host double[K], may be NULL): the same sum per cluster.  1 <= K <= N. */
int dtw_cluster_cost(const float *D, int32_t N, const int32_t *labels, const int32_t *centroids, int32_t K,
                     double *per_cluster, double *total, void *stream);

/* k-medoids assignment step: labels_out (device int32[N]) = index of the nearest
 * centroid (lowest index on ties); *total and per_cluster as for dtw_cluster_cost. */
int dtw_assign(const float *D, int32_t N, const int32_t *centroids, int32_t K, int32_t *labels_out,
               double *per_cluster, double *total, void *stream);

/*
 * Optimal warping path of one pair (paper, "Mathematical background" and
 * Fig. 1): the cells (i, j) matched by the cheapest alignment of x and y, from
 * (0, 0) to (n-1, m-1) (0-based), found by walking back through the cumulative
 * cost matrix of Eq. (c) from its last cell, each time to the predecessor with
 * the smallest cumulative cost; ties go to the diagonal (i-1, j-1), then
 * (i-1, j), then (i, j-1).  The window rule is the one above.  PLAIN FP32
 * accumulation: *cost equals the distance-matrix entry of the pair.
 *   x (device, n floats), y (device, m floats): the two series, n, m >= 1;
 *     the shorter may have up to 32768 points (else DTW_ERR_UNSUPPORTED).
 *   path (device int32[2*(n+m-1)]): the path as (i, j) pairs in order from
 *     (0, 0); *path_len (host) receives its number of cells (n+m-1 at most).
 *   *cost (host): c(n, m).
 *   C (device float[n*m], may be NULL): the cumulative cost matrix, row-major,
 *     C[i*m + j] = c(i+1, j+1), +inf at inadmissible cells.
 * If c(n, m) is not finite (FP32 overflow) the path is admissible but not meaningful.
 * Workspace: with C == NULL the sweep stores only each cell's move (2 bits a
 * cell, about n*m/4 bytes plus padding) in a device buffer that the library
 * keeps between calls, one per device, grown to the largest pair so far up
 * to 1 GiB (larger ones are allocated for the call); calls on one device
 * take turns on it (a lock held until the call's stream has finished).  With
 * C the sweep keeps every cost, about 4 bytes a cell, allocated for the call.
 * Runs on `stream` (hipStream_t, NULL = default) and synchronises it before
 * returning.
 */
int dtw_path(const float *x, int32_t n, const float *y, int32_t m, int32_t window, int32_t *path,
             int64_t *path_len, float *cost, float *C, void *stream);

/* Admissible cells of one n x m problem under window w (host arithmetic only). */
int dtw_band_cells(int32_t n, int32_t m, int32_t window, int64_t *cells);

/* Message describing the last failure on the calling thread ("" if none). */
const char *dtw_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int32_t dtw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DTWMI_H */
