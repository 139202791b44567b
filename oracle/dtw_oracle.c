/*
 * Plain FP64 CPU oracle for dynamic time warping (DTW).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * GPU library.
 *
 * What it computes (paper: "Mathematical background", Eq. (c)):
 *   c(i,j) = (x_i - y_j)^2 + min{ c(i-1,j-1), c(i-1,j), c(i,j-1) }
 * with c(0,0) = 0 and c(i,0) = c(0,j) = +inf in 1-based indexing; the DTW
 * cost of the pair is c(n,m).  Only the previous row is kept ("preceding
 * vector", same section), which gives exactly the same numbers as the full
 * matrix because every cell is evaluated with the same operations in the
 * same order.
 *
 * Warping window (paper, Introduction: a window of 99 lets point 1 reach at
 * most point 100 of the other series): a cell is admissible iff
 * |i - j| <= w_eff, with w_eff = max(w, |n - m|) so that (n,m) is always
 * reachable for unequal lengths, and w < 0 meaning "no window".  Cells
 * outside the window are +inf.
 *
 * Arithmetic: IEEE double, round-to-nearest-even, no fast-math.  The local
 * cost is the squared difference written as d*d; the sum is a plain add.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

static int64_t band_of(int32_t w, int32_t n, int32_t m)
{
    if (w < 0) return (int64_t)1 << 40; /* no window */
    int64_t d = (int64_t)n - (int64_t)m;
    if (d < 0) d = -d;
    return (int64_t)w > d ? (int64_t)w : d;
}

/* Number of admissible cells of one n x m problem under window w. */
int64_t oracle_band_cells(int32_t n, int32_t m, int32_t w)
{
    int64_t b = band_of(w, n, m), total = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t lo = i - b, hi = i + b;
        if (lo < 0) lo = 0;
        if (hi > m - 1) hi = m - 1;
        if (hi >= lo) total += hi - lo + 1;
    }
    return total;
}

/*
 * DTW of one pair with the two-row scheme.  work must hold 2*(m+1) doubles.
 * Returns +inf if n or m is zero.
 */
double oracle_dtw_pair(const double *x, int32_t n, const double *y, int32_t m,
                       int32_t w, double *work)
{
    if (n <= 0 || m <= 0) return INFINITY;
    int64_t b = band_of(w, n, m);
    double *prev = work, *cur = work + (m + 1);
    /* Row 0 of the 1-based matrix: c(0,0) = 0, c(0,j) = +inf. */
    prev[0] = 0.0;
    for (int32_t j = 1; j <= m; ++j) prev[j] = INFINITY;
    for (int32_t i = 1; i <= n; ++i) {
        cur[0] = INFINITY;
        for (int32_t j = 1; j <= m; ++j) {
            int64_t off = (int64_t)i - (int64_t)j;
            if (off < 0) off = -off;
            if (off > b) {
                cur[j] = INFINITY;
                continue;
            }
            double best = prev[j - 1];
            if (prev[j] < best) best = prev[j];
            if (cur[j - 1] < best) best = cur[j - 1];
            double d = x[i - 1] - y[j - 1];
            cur[j] = d * d + best;
        }
        double *t = prev;
        prev = cur;
        cur = t;
    }
    return prev[m];
}

/*
 * Same recurrence with the whole (n+1) x (m+1) matrix stored row-major in C.
 * Used only to cross-check the two-row version and to expose the matrix of
 * small examples.  Returns C[n][m].
 */
double oracle_dtw_full(const double *x, int32_t n, const double *y, int32_t m,
                       int32_t w, double *C)
{
    if (n <= 0 || m <= 0) return INFINITY;
    int64_t b = band_of(w, n, m);
    int64_t ld = (int64_t)m + 1;
    C[0] = 0.0;
    for (int32_t j = 1; j <= m; ++j) C[j] = INFINITY;
    for (int32_t i = 1; i <= n; ++i) {
        C[i * ld] = INFINITY;
        for (int32_t j = 1; j <= m; ++j) {
            int64_t off = (int64_t)i - (int64_t)j;
            if (off < 0) off = -off;
            if (off > b) {
                C[i * ld + j] = INFINITY;
                continue;
            }
            double best = C[(i - 1) * ld + (j - 1)];
            if (C[(i - 1) * ld + j] < best) best = C[(i - 1) * ld + j];
            if (C[i * ld + (j - 1)] < best) best = C[i * ld + (j - 1)];
            double d = x[i - 1] - y[j - 1];
            C[i * ld + j] = d * d + best;
        }
    }
    return C[(int64_t)n * ld + m];
}

/* ------------------------------------------------------------------ */
/* Many pairs on all host cores: static chunks of an explicit pair list. */

typedef struct {
    const double *series;
    const int64_t *offsets;
    const int32_t *lengths;
    const int32_t *pi, *pj; /* pair list */
    const int32_t *window;  /* per pair */
    double *out;
    int64_t begin, end;
    int32_t max_len;
    int status;
} job_t;

static void *run_job(void *arg)
{
    job_t *jb = (job_t *)arg;
    double *work = (double *)malloc(sizeof(double) * 2 * ((size_t)jb->max_len + 1));
    if (!work) {
        jb->status = -1;
        return NULL;
    }
    for (int64_t p = jb->begin; p < jb->end; ++p) {
        int32_t a = jb->pi[p], b = jb->pj[p];
        jb->out[p] = oracle_dtw_pair(jb->series + jb->offsets[a], jb->lengths[a],
                                     jb->series + jb->offsets[b], jb->lengths[b],
                                     jb->window[p], work);
    }
    free(work);
    jb->status = 0;
    return NULL;
}

int32_t oracle_host_threads(void)
{
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int32_t)c : 1;
}

/*
 * out[p] = DTW(series[pi[p]], series[pj[p]]) under window[p], for p < P.
 * threads <= 0 means one thread per online core.  Returns the number of
 * threads used, or a negative value on allocation failure.
 */
int32_t oracle_dtw_pairs(const double *series, const int64_t *offsets,
                         const int32_t *lengths, int32_t N, const int32_t *pi,
                         const int32_t *pj, const int32_t *window, int64_t P,
                         double *out, int32_t threads)
{
    int32_t max_len = 1;
    for (int32_t s = 0; s < N; ++s)
        if (lengths[s] > max_len) max_len = lengths[s];
    if (threads <= 0) threads = oracle_host_threads();
    if (P < threads) threads = P > 0 ? (int32_t)P : 1;
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    job_t *jobs = (job_t *)calloc((size_t)threads, sizeof(job_t));
    if (!tid || !jobs) {
        free(tid);
        free(jobs);
        return -1;
    }
    int64_t chunk = (P + threads - 1) / threads;
    for (int32_t t = 0; t < threads; ++t) {
        job_t *jb = &jobs[t];
        jb->series = series;
        jb->offsets = offsets;
        jb->lengths = lengths;
        jb->pi = pi;
        jb->pj = pj;
        jb->window = window;
        jb->out = out;
        jb->max_len = max_len;
        jb->begin = t * chunk < P ? t * chunk : P;
        jb->end = (t + 1) * chunk < P ? (t + 1) * chunk : P;
        jb->status = 0;
        pthread_create(&tid[t], NULL, run_job, jb);
    }
    int bad = 0;
    for (int32_t t = 0; t < threads; ++t) {
        pthread_join(tid[t], NULL);
        if (jobs[t].status) bad = 1;
    }
    free(tid);
    free(jobs);
    return bad ? -1 : threads;
}
