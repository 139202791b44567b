// Clustering scores from the condensed DTW matrix D (the method's steps after
// D, paper Introduction: the clustering cost -- sum of the distances between
// every series and its cluster's centroid -- and the silhouette score used to
// choose the number of clusters; the k-medoids assignment of each series to
// its nearest centroid).  The silhouette follows Rousseeuw's definition:
// a(i) = mean distance to the other members of i's cluster, b(i) = smallest
// mean distance to another non-empty cluster, s(i) = (b-a)/max(a,b) (0 when
// both are 0), 0 for a singleton; the score is the mean of s(i).
//
// These kernels read D, N(N-1)/2 floats; the row-sum kernel is bound by HBM
// bandwidth.  All sums are FP64 and every reduction has a fixed order, so
// results do not change from run to run.
#include "dtw_device.h"
#include "dtwmi.h"

#include <algorithm>
#include <cstdio>
#include <vector>

namespace dtwmi {
namespace {

constexpr int kRowBlock = 64;   // rows of D per workgroup (one row per lane)
constexpr int kReduce = 256;    // threads of the reduction kernels

__device__ __forceinline__ float dist(const float *__restrict__ D, int i, int j, int N) {
    return i == j ? 0.0f : D[i < j ? condensed_index(i, j, N) : condensed_index(j, i, N)];
}

// P[split][i][J] = sum of D(i, j) over the columns j of this split's column
// tiles with j != i and labels[j] == J.  Workgroup (row block, split) of one
// wavefront: thread t owns row i0 + t and K <= 16 NV accumulators in registers.
// A column's label is the same for every lane (one column per step of the
// accumulation loop), so acc[label] is a register-indexed read-modify-write
// on a wave-uniform index (s_set_gpr_idx); labels come in by scalar loads.
// Each tile's values are loaded CH columns at a time, all in flight at once:
//  * left of the diagonal, D(j, i) for a column j is 64 consecutive entries of
//    row j of the condensed triangle, one coalesced load per column;
//  * right of it, D(i, j) for a row i is 64 consecutive entries of row i:
//    the wavefront first copies the tile row by row (one coalesced load per
//    row, lane = column) into LDS and reads it back transposed (lane = row);
//  * the diagonal tile reads entry by entry.
// Entries outside the matrix or on the diagonal contribute 0.  Additions run
// in column order, so the result does not depend on the schedule.
typedef double Acc16 __attribute__((ext_vector_type(16)));  // register-indexed access needs <= 16 doubles

// acc[l] += x for a wave-uniform l < 16 NV, over NV vectors of 16 accumulators.
template <int NV>
__device__ __forceinline__ void acc_add(Acc16 (&acc)[NV], int l, double x) {
    if constexpr (NV == 1) {
        acc[0][l] += x;
    } else {
        if (l < 16) {
            acc[0][l] += x;
        } else if (NV == 2 || l < 32) {
            acc[1][l - 16] += x;
        } else if (NV == 3 || l < 48) {
            acc[NV > 2 ? 2 : 0][l - 32] += x;
        } else {
            acc[NV > 3 ? 3 : 0][l - 48] += x;
        }
    }
}

template <int NV, int CH>
__global__ __launch_bounds__(kRowBlock) void k_row_cluster_sums(const float *__restrict__ D, int N,
                                                                const int *__restrict__ labels, int K,
                                                                int tiles_per_split, double *__restrict__ P) {
    __shared__ float tile[kRowBlock][kRowBlock + 1];
    Acc16 acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = Acc16{};
    const int t = threadIdx.x;
    const int i0 = blockIdx.x * kRowBlock, i = i0 + t;
    const int split = blockIdx.y;
    const int n_tiles = (N + kRowBlock - 1) / kRowBlock;
    const int jt0 = split * tiles_per_split, jt1 = min(n_tiles, jt0 + tiles_per_split);
    for (int jt = jt0; jt < jt1; ++jt) {
        const int j0 = jt * kRowBlock;
        const bool left = j0 + kRowBlock <= i0, right = j0 >= i0 + kRowBlock;
        if (right) {
            const int j = j0 + t;
            __builtin_amdgcn_wave_barrier();  // the previous tile's reads of `tile` are done
            for (int r0 = 0; r0 < kRowBlock; r0 += 16) {
                float w[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int ir = i0 + r0 + r;  // wave-uniform row
                    w[r] = (ir < N && j < N) ? D[condensed_index(ir, j0, N) + t] : 0.0f;
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) tile[r0 + r][t] = w[r];
            }
            __builtin_amdgcn_wave_barrier();
        }
        for (int c0 = 0; c0 < kRowBlock; c0 += CH) {
            float v[CH];
            if (left) {  // D(j, i), consecutive in i
#pragma unroll
                for (int c = 0; c < CH; ++c) v[c] = i < N ? D[condensed_index(j0 + c0 + c, i, N)] : 0.0f;
            } else if (right) {
#pragma unroll
                for (int c = 0; c < CH; ++c) v[c] = tile[t][c0 + c];
            } else {  // the diagonal tile
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int jc = j0 + c0 + c;
                    v[c] = (i < N && jc < N) ? dist(D, i, jc, N) : 0.0f;
                }
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int jc = j0 + c0 + c;
                const int lc = jc < N ? labels[jc] : 0;  // wave-uniform
                acc_add<NV>(acc, lc, (double)v[c]);
            }
        }
    }
    if (i < N)
#pragma unroll
        for (int J = 0; J < 16 * NV; ++J)
            if (J < K) P[((int64_t)split * N + i) * K + J] = acc[J / 16][J % 16];
}

// Each entry of D once: workgroup (SC, SR) of kSilR wavefronts covers rows
// [512 SR, 512 SR + 512) (wavefront w: row block I = 8 SR + w, 64 rows) and
// columns [512 SC, 512 SC + 512) (kSilT column tiles); a tile (I, J) is
// processed only for J >= I, and on the diagonal (J == I) only for i < j, so
// every condensed entry D(i, j), i < j, is read by exactly one wavefront.  It
// adds D(i, j) both to row i's sum for cluster labels[j] and to row j's sum
// for cluster labels[i]:
//  * lane = column j: the tile is loaded row by row (coalesced: 64
//    consecutive entries of row i of the condensed triangle) into registers,
//    and each lane adds its column's values over the tile's rows (label of
//    the row wave-uniform); the eight wavefronts' column sums of the tile are
//    then added in wavefront order through LDS and written to
//    Pcol[SR][J][j] (per super-row SR);
//  * lane = row i: the tile goes through LDS to be read transposed, and each
//    lane adds its row's values over the tile's columns, in registers across
//    the kSilT tiles, written once to Prow[SC][J][i] (per super-column SC).
// (Cluster-major partials: the per-series kernel reads each cluster's sums
// of consecutive series as one coalesced run.)
// The per-series sums then add the Prow and Pcol partials in a fixed order,
// so D is read once from HBM and the results repeat bit for bit.  K <= 16.
constexpr int kSilR = 8;  // row blocks (wavefronts) per workgroup
constexpr int kSilT = 8;  // column tiles per workgroup
constexpr int kSilRows = kSilR * kRowBlock, kSilCols = kSilT * kRowBlock;
// the super-tiles (SR, SC) holding a tile on or above the diagonal: SC >= sil_first_sc(SR)
__host__ __device__ constexpr int sil_first_sc(int SR) { return kSilRows * SR / kSilCols; }
__host__ __device__ constexpr int sil_last_sr(int SC) { return (kSilCols * SC + kSilCols - 1) / kSilRows; }
// Super-tiles of an n_sr x n_sc grid on or above the diagonal
__host__ __device__ inline int sil_count(int n_sr, int n_sc) {
    int n = 0;
    for (int SR = 0; SR < n_sr; ++SR) n += max(0, n_sc - sil_first_sc(SR));
    return n;
}

// One workgroup per super-tile on or above the diagonal, numbered row by row;
// workgroup b takes super-tile (b mod 8) * ceil(n/8) + b / 8, so that the
// hardware's round-robin over the 8 XCDs gives each XCD a run of neighbouring
// super-tiles, which share the cache lines at their column boundaries in that
// XCD's L2.
__global__ __launch_bounds__(64 * kSilR) void k_cluster_sums_once(const float *__restrict__ D, int N,
                                                                  const int *__restrict__ labels, int K,
                                                                  double *__restrict__ Prow,
                                                                  double *__restrict__ Pcol, int n_sr, int n_sc,
                                                                  int n_st) {
    __shared__ float tile[kSilR][kRowBlock][kRowBlock + 1];  // a wavefront's tile; reused for its column sums
    int t = (blockIdx.x % 8) * ((n_st + 7) / 8) + blockIdx.x / 8;
    if (t >= n_st) return;  // uniform per workgroup
    int SR = 0;
    for (; SR < n_sr - 1; ++SR) {  // the super-row holding super-tile t (uniform)
        const int cnt = n_sc - sil_first_sc(SR);
        if (t < cnt) break;
        t -= cnt;
    }
    const int SC = sil_first_sc(SR) + t;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;  // w: wave-uniform
    const int I = kSilR * SR + w, i0 = I * kRowBlock;
    Acc16 accr[1] = {Acc16{}};
#pragma unroll 1
    for (int t = 0; t < kSilT; ++t) {
        const int J = kSilT * SC + t, j0 = J * kRowBlock;
        const bool valid = J >= I && i0 < N && j0 < N;  // wave-uniform
        Acc16 accc[1] = {Acc16{}};
        const int j = j0 + lane;
        if (valid) {
            float v[kRowBlock];  // all 64 rows of the tile in flight at once
#pragma unroll
            for (int r = 0; r < kRowBlock; ++r) {
                const int ir = i0 + r;
                v[r] = (ir < j && j < N) ? D[condensed_index(ir, j, N)] : 0.0f;
            }
#pragma unroll
            for (int r = 0; r < kRowBlock; ++r) {
                const int ir = i0 + r;
                acc_add<1>(accc, ir < N ? labels[ir] : 0, (double)v[r]);  // wave-uniform label
                tile[w][r][lane] = v[r];
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll 8
            for (int c = 0; c < kRowBlock; ++c) {
                const int jc = j0 + c;
                acc_add<1>(accr, jc < N ? labels[jc] : 0, (double)tile[w][lane][c]);
            }
            __builtin_amdgcn_wave_barrier();  // the transposed reads are done before the tile is reused
        }
        // column sums of the tile: this wavefront's into its LDS region, then added in wavefront order
        double *red = reinterpret_cast<double *>(&tile[w][0][0]);  // [16][64]
#pragma unroll
        for (int k = 0; k < 16; ++k) red[k * kRowBlock + lane] = accc[0][k];
        __syncthreads();
        if (j0 < N) {
            for (int k = w; k < K; k += kSilR) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < kSilR; ++q) s += reinterpret_cast<const double *>(&tile[q][0][0])[k * kRowBlock + lane];
                if (j < N) Pcol[((int64_t)SR * K + k) * N + j] = s;
            }
        }
        __syncthreads();  // the sums are read before the next tile overwrites the regions
    }
    const int i = i0 + lane;
    if (i < N)
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (k < K) Prow[((int64_t)SC * K + k) * N + i] = accr[0][k];
}

// Fixed-order tree sum of one workgroup's values into out.
__device__ __forceinline__ void block_sum(double v, double *red, double *out) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kReduce / 2; w > 0; w /= 2) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// s(i) from the cluster sums; per-workgroup partial sums of s.  P holds
// `splits` row-sum partials per series (k_row_cluster_sums); or, with Pcol,
// the partials of k_cluster_sums_once: the row sums of every super-column
// from sil_first_sc on (the super-tiles on or above the diagonal) in P, then
// the column sums of super-rows 0 .. sil_last_sr in Pcol.
__global__ __launch_bounds__(kReduce) void k_silhouette_rows(const double *__restrict__ P, int splits, int N, int K,
                                                             const int *__restrict__ labels,
                                                             const int *__restrict__ sizes, float *__restrict__ s_out,
                                                             double *__restrict__ partial,
                                                             const double *__restrict__ Pcol, int n_sr) {
    __shared__ double red[kReduce];
    const int i = blockIdx.x * kReduce + threadIdx.x;
    double s = 0.0;
    if (i < N) {
        const int A = labels[i];
        if (sizes[A] > 1) {
            double a = 0.0, b = __builtin_huge_val();
            const int sp0 = Pcol ? sil_first_sc(i / kSilRows) : 0;
            const int sr1 = Pcol ? min(n_sr - 1, sil_last_sr(i / kSilCols)) : -1;
            for (int J = 0; J < K; ++J) {
                double sum = 0.0;
                if (Pcol) {  // unrolled so that the loads of several partials are in flight together
#pragma unroll 8
                    for (int sp = sp0; sp < splits; ++sp) sum += P[((int64_t)sp * K + J) * N + i];
#pragma unroll 8
                    for (int sr = 0; sr <= sr1; ++sr) sum += Pcol[((int64_t)sr * K + J) * N + i];
                } else {
                    for (int sp = 0; sp < splits; ++sp) sum += P[((int64_t)sp * N + i) * K + J];
                }
                if (J == A)
                    a = sum / (double)(sizes[A] - 1);
                else if (sizes[J] > 0)
                    b = fmin(b, sum / (double)sizes[J]);
            }
            const double m = fmax(a, b);
            s = m == 0.0 ? 0.0 : (b - a) / m;
        }
        if (s_out) s_out[i] = (float)s;
    }
    block_sum(s, red, partial + blockIdx.x);
}

// Distance of each series to its own centroid (cost) or to its nearest
// centroid (assignment, lowest cluster index on ties).
__global__ __launch_bounds__(kReduce) void k_centroid_dist(const float *__restrict__ D, int N,
                                                           const int *__restrict__ labels,
                                                           const int *__restrict__ centroids, int K,
                                                           int *__restrict__ labels_out, double *__restrict__ v) {
    const int i = blockIdx.x * kReduce + threadIdx.x;
    if (i >= N) return;
    if (labels) {
        v[i] = (double)dist(D, i, centroids[labels[i]], N);
        return;
    }
    float best = __builtin_huge_valf();
    int lab = 0;
    for (int c = 0; c < K; ++c) {
        const float d = dist(D, i, centroids[c], N);
        if (d < best) {
            best = d;
            lab = c;
        }
    }
    labels_out[i] = lab;
    v[i] = (double)best;
}

// One workgroup: out[J] = sum of v[i] over the series with key[i] == J (key ==
// nullptr: all series into out[0]), each thread over i = t, t+256, ... then a
// tree, J after J.
__global__ __launch_bounds__(kReduce) void k_sum_by_key(const double *__restrict__ v, int n,
                                                        const int *__restrict__ key, int K, double *__restrict__ out) {
    __shared__ double red[kReduce];
    for (int J = 0; J < K; ++J) {
        double s = 0.0;
        for (int i = threadIdx.x; i < n; i += kReduce)
            if (!key || key[i] == J) s += v[i];
        block_sum(s, red, out + J);
        __syncthreads();
    }
}

// ---- host side ----
int fail_msg(int code, const char *fmt, long long a = 0, long long b = 0, long long c = 0) {
    char buf[256];
    snprintf(buf, sizeof buf, fmt, a, b, c);
    return set_error(code, buf);
}

int hip_err(hipError_t e, const char *what) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return set_error(DTW_ERR_HIP, buf);
}

// Device labels or centroids copied to the host and range-checked.
int fetch_indices(const int32_t *dev, int64_t n, int32_t limit, const char *what, std::vector<int32_t> &host,
                  hipStream_t s) {
    host.resize((size_t)n);
    hipError_t e = hipMemcpyAsync(host.data(), dev, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(e, "hipMemcpy (indices)");
    for (int64_t k = 0; k < n; ++k)
        if (host[(size_t)k] < 0 || host[(size_t)k] >= limit) {
            char buf[160];
            snprintf(buf, sizeof buf, "%s[%lld] = %d outside 0..%d", what, (long long)k, host[(size_t)k], limit - 1);
            return set_error(DTW_ERR_INVALID_ARG, buf);
        }
    return DTW_OK;
}

// Owns the device workspace of one call.
struct Scratch {
    void *p = nullptr;
    ~Scratch() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace
}  // namespace dtwmi

using namespace dtwmi;

extern "C" {

int dtw_silhouette(const float *D, int32_t N, const int32_t *labels, int32_t K, float *s_out, double *mean,
                   void *stream) {
    clear_error();
    if (!D || !labels || !mean) return set_error(DTW_ERR_INVALID_ARG, "D, labels or mean is NULL");
    if (N < 2) return fail_msg(DTW_ERR_INVALID_ARG, "N=%lld < 2", N);
    if (K < 2 || K > kSilhouetteMaxK)
        return fail_msg(K < 2 ? DTW_ERR_INVALID_ARG : DTW_ERR_UNSUPPORTED, "K=%lld outside 2..%lld", K,
                        kSilhouetteMaxK);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int32_t> lab;
    int rc = fetch_indices(labels, N, K, "labels", lab, s);
    if (rc) return rc;
    std::vector<int32_t> sizes(K, 0);
    for (int32_t l : lab) ++sizes[l];
    if (std::count_if(sizes.begin(), sizes.end(), [](int32_t z) { return z > 0; }) < 2)
        return set_error(DTW_ERR_INVALID_ARG, "the silhouette needs at least two non-empty clusters");

    // K <= 16: each entry of D read once (k_cluster_sums_once; partials per
    // super-column and super-row).  More clusters: every entry read for both
    // its rows, the column tiles split so that there are ~2048 workgroups of
    // one wavefront, each with at least one tile (more splits cost more in the
    // per-series reduction of the partial sums than they gain here).
    const bool once = K <= 16;
    const int row_blocks = (N + kRowBlock - 1) / kRowBlock;
    const int n_tiles = row_blocks;
    const int target_groups = 2048;
    const int n_sc = (N + kSilCols - 1) / kSilCols, n_sr = (N + kSilRows - 1) / kSilRows;
    const int splits = once ? n_sc : std::max(1, std::min(n_tiles, (target_groups + row_blocks - 1) / row_blocks));
    const int tiles_per_split = (n_tiles + splits - 1) / splits;
    const int red_blocks = (N + kReduce - 1) / kReduce;
    const size_t o_sizes = 0, o_P = 256, bytes_P = (size_t)splits * N * K * sizeof(double);
    const size_t bytes_Pc = once ? (size_t)n_sr * N * K * sizeof(double) : 0;
    const size_t o_Pc = o_P + ((bytes_P + 255) / 256) * 256;
    const size_t o_part = o_Pc + ((bytes_Pc + 255) / 256) * 256;
    const size_t o_out = o_part + ((red_blocks * sizeof(double) + 255) / 256) * 256;
    Scratch w;
    hipError_t e = hipMalloc(&w.p, o_out + 256);
    if (e != hipSuccess) return set_error(DTW_ERR_OUT_OF_MEMORY, "workspace allocation failed");
    char *base = static_cast<char *>(w.p);
    int *d_sizes = reinterpret_cast<int *>(base + o_sizes);
    double *d_P = reinterpret_cast<double *>(base + o_P);
    double *d_Pc = once ? reinterpret_cast<double *>(base + o_Pc) : nullptr;
    double *d_part = reinterpret_cast<double *>(base + o_part);
    double *d_out = reinterpret_cast<double *>(base + o_out);
    e = hipMemcpyAsync(d_sizes, sizes.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_err(e, "hipMemcpy (cluster sizes)");
    static_assert(kSilhouetteMaxK <= 64, "four vectors of 16 accumulators");
    if (once) {
        const int n_st = sil_count(n_sr, n_sc);
        hipLaunchKernelGGL(k_cluster_sums_once, dim3(8 * ((n_st + 7) / 8)), dim3(64 * kSilR), 0, s, D, N, labels, K,
                           d_P, d_Pc, n_sr, n_sc, n_st);
    } else {
        hipLaunchKernelGGL((k_row_cluster_sums<4, 16>), dim3(row_blocks, splits), dim3(kRowBlock), 0, s, D, N, labels,
                           K, tiles_per_split, d_P);
    }
    if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "row-sum kernel launch");
    hipLaunchKernelGGL(k_silhouette_rows, dim3(red_blocks), dim3(kReduce), 0, s, d_P, splits, N, K, labels, d_sizes,
                       s_out, d_part, d_Pc, n_sr);
    if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "silhouette kernel launch");
    hipLaunchKernelGGL(k_sum_by_key, dim3(1), dim3(kReduce), 0, s, d_part, red_blocks, nullptr, 1, d_out);
    if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "reduction kernel launch");
    double total = 0.0;
    e = hipMemcpyAsync(&total, d_out, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(e, "silhouette result");
    *mean = total / (double)N;
    return DTW_OK;
}

// Shared body of the cost and assignment entry points.
static int centroid_scores(const float *D, int32_t N, const int32_t *labels, const int32_t *centroids, int32_t K,
                           int32_t *labels_out, double *per_cluster, double *total, void *stream) {
    clear_error();
    if (!D || !centroids || !total) return set_error(DTW_ERR_INVALID_ARG, "D, centroids or total is NULL");
    if (!labels && !labels_out) return set_error(DTW_ERR_INVALID_ARG, "labels_out is NULL");
    if (N < 2) return fail_msg(DTW_ERR_INVALID_ARG, "N=%lld < 2", N);
    if (K < 1 || K > N) return fail_msg(DTW_ERR_INVALID_ARG, "K=%lld outside 1..%lld", K, N);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int32_t> host;
    int rc = fetch_indices(centroids, K, N, "centroids", host, s);
    if (!rc && labels) rc = fetch_indices(labels, N, K, "labels", host, s);
    if (rc) return rc;
    const int blocks = (N + kReduce - 1) / kReduce;
    const size_t o_v = 0, o_out = (((size_t)N * sizeof(double) + 255) / 256) * 256;
    Scratch w;
    hipError_t e = hipMalloc(&w.p, o_out + (size_t)(K + 1) * sizeof(double));
    if (e != hipSuccess) return set_error(DTW_ERR_OUT_OF_MEMORY, "workspace allocation failed");
    double *d_v = reinterpret_cast<double *>(static_cast<char *>(w.p) + o_v);
    double *d_out = reinterpret_cast<double *>(static_cast<char *>(w.p) + o_out);
    hipLaunchKernelGGL(k_centroid_dist, dim3(blocks), dim3(kReduce), 0, s, D, N, labels, centroids, K, labels_out, d_v);
    if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "centroid kernel launch");
    hipLaunchKernelGGL(k_sum_by_key, dim3(1), dim3(kReduce), 0, s, d_v, N, nullptr, 1, d_out + K);
    if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "reduction kernel launch");
    if (per_cluster) {
        hipLaunchKernelGGL(k_sum_by_key, dim3(1), dim3(kReduce), 0, s, d_v, N, labels ? labels : labels_out, K, d_out);
        if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "reduction kernel launch");
    }
    std::vector<double> res(K + 1);
    e = hipMemcpyAsync(res.data(), d_out, (K + 1) * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(e, "cluster cost result");
    *total = res[K];
    if (per_cluster) std::copy(res.begin(), res.begin() + K, per_cluster);
    return DTW_OK;
}

int dtw_cluster_cost(const float *D, int32_t N, const int32_t *labels, const int32_t *centroids, int32_t K,
                     double *per_cluster, double *total, void *stream) {
    if (!labels) {
        clear_error();
        return set_error(DTW_ERR_INVALID_ARG, "labels is NULL");
    }
    return centroid_scores(D, N, labels, centroids, K, nullptr, per_cluster, total, stream);
}

int dtw_assign(const float *D, int32_t N, const int32_t *centroids, int32_t K, int32_t *labels_out,
               double *per_cluster, double *total, void *stream) {
    return centroid_scores(D, N, nullptr, centroids, K, labels_out, per_cluster, total, stream);
}

}  // extern "C"
