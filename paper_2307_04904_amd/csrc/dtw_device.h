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
// Kernel families, one source each: dtw_lane.hip (one pair per lane, equal
// lengths, narrow band), dtw_strip.hip (one pair per workgroup, rows of the
// shorter series in lane strips), dtw_cyclic.hip (one pair per wavefront,
// blocks of the longer series cycling over the lanes); dtw_stage.hip stages
// the inputs; dtw_path.hip keeps the whole matrix of one pair for its warping
// path and dtw_cluster.hip scores clusterings from D.  This header holds the
// device helpers they share.  Not part of the public ABI.
#pragma once

#include "dtw_internal.h"

#include <type_traits>

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

// Minimum of v over the 64 lanes of the wavefront, returned to every lane:
// butterflies within each row of 16 lanes by DPP (quad swaps, then rotations
// by 4 and 8), then the four row minima read from lanes 0, 16, 32 and 48.
// Every lane must be active.
__device__ __forceinline__ float wave_min(float v) {
    auto dpp = [](float a, auto ctrl) {
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(a), decltype(ctrl)::value, 0xF, 0xF, true));
    };
    v = fminf(v, dpp(v, std::integral_constant<int, 0xB1>{}));   // quad_perm [1,0,3,2]
    v = fminf(v, dpp(v, std::integral_constant<int, 0x4E>{}));   // quad_perm [2,3,0,1]
    v = fminf(v, dpp(v, std::integral_constant<int, 0x124>{}));  // row_ror:4
    v = fminf(v, dpp(v, std::integral_constant<int, 0x128>{}));  // row_ror:8
    const int b = __float_as_int(v);
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(b, 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(b, 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(b, 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(b, 48));
    return fminf(fminf(r0, r1), fminf(r2, r3));
}

__device__ __forceinline__ int64_t condensed_index(int i, int j, int N) {
    // i < j
    return (int64_t)i * N - (int64_t)i * (i + 1) / 2 + (j - i - 1);
}

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

// Row series values of a strip in a register vector, so that a window event's
// wave-uniform row index becomes one indexed register move (s_set_gpr_idx)
// instead of a test per cell.  At least 16 elements: the compiler turns an
// indexed move into a chain of compares and selects for smaller vectors.
template <int H>
struct XVec {
    typedef float T __attribute__((ext_vector_type(H < 16 ? 16 : H)));
};

}  // namespace
}  // namespace dtwmi
