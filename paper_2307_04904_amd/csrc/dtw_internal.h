// Internal layout shared by the host planner (dtw_api.hip) and the kernel
// sources (dtw_stage.hip, dtw_lane.hip, dtw_strip.hip, dtw_cyclic.hip,
// dtw_cluster.hip, dtw_path.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dtwmi {

// Padding (in FP32 elements) written before and after every staged series.
// Pad cells hold +inf, so a read of y outside [0, m) yields an inadmissible
// (+inf) local cost without any branch.  Kernels rely on:
//   lane-band kernel: reads y[i-B .. i+B] with B <= 63, x[0 .. L+7];
//   wavefront kernels: clamp column reads into [-1, m].
constexpr int kPad = 128;
constexpr int kLaneMaxW = 127;   // widest band (2*B+1) of the lane-band kernel

// Accumulation of a kernel instance (the public dtw_accum AUTO resolves to
// kAccPlain or kAccRebased per pair):
//   kAccPlain:   FP32 sub, min3, fused multiply-add per cell;
//   kAccKahan:   FP32 with a compensation term carried per cell;
//   kAccF64:     the recurrence in FP64, rounded once at the end;
//   kAccRebased: the plain FP32 cell, every lane keeping its values relative
//                to a running base of its own that it renormalises every few
//                steps (rounding relative to the small stored values).
enum AccMode { kAccPlain = 0, kAccKahan = 1, kAccF64 = 2, kAccRebased = 3 };


struct SeriesSrc {     // where a series lives in the caller's buffer
    const void *base;  // device pointer of the dataset buffer
    int64_t off;       // element offset
    int32_t len;
    int32_t dtype;     // dtw_dtype
};

struct SeriesInfo {    // where a series lives in the staged FP32 workspace
    int64_t pstart;    // index of element 0 (16-byte aligned); pads at [-kPad, 0) and [len, len+kPad)
    int32_t len;
    int32_t pad_;
};

struct DatasetInfo {
    float *out;        // condensed output of this dataset
    int32_t N;
    int32_t window;    // as given (< 0 = none)
    int32_t L;         // common length if all series are equal, else -1
    int32_t series_base;  // global index of the dataset's first series
};

// Lane-band work item: one wavefront evaluates, for lane < cnt, the pair of
// series a and partner b written to output slot k:
//   list < 0:  b = (a + d0 + lane) mod N, k = condensed index of (a, b);
//   list >= 0: (b, k) = partners[list + lane] (explicit pair lists).
// All series of the dataset have length L.
struct LaneItem {
    int32_t ds, a, d0, cnt;
    int64_t list;
};
struct LanePartner {
    int32_t b, pad_;
    int64_t slot;
};

// Wavefront work item: one pair; `rows` is the series spread over the lanes,
// `cols` the one swept step by step; the result goes to out[slot] of the
// dataset (the condensed index for all-pairs plans).
struct WaveItem {
    int32_t ds, rows, cols, band;  // band = max(w, |n-m|), or -1 for none
    int64_t slot;
};

// Kernel launchers (one kernel source each).  All asynchronous on `stream`.
// Wavefront launchers take the item count and a queue counter: with queue == nullptr
// the grid has one workgroup per item; otherwise min(items, slots) resident
// workgroups pull items from the counter, which must be zero at launch
// (launch_zero).  `slots` comes from the matching *_resident function
// (workgroups the device holds at once; 0 if it cannot be queried).
hipError_t launch_stage(const SeriesSrc *src, const SeriesInfo *ser, float *ws, int32_t nseries,
                        hipStream_t stream);
hipError_t launch_zero(unsigned *p, int n, hipStream_t stream);
// Set every SeriesSrc.base of a one-dataset plan to `series` and its output to `out`.
hipError_t launch_rebind(SeriesSrc *src, int32_t nseries, const void *series, DatasetInfo *dsi, float *out,
                         hipStream_t stream);
// Workgroups of `block` threads of kernel `fn` the current device holds at
// once (CUs x occupancy per CU; 0 if it cannot be queried).
int resident_blocks(const void *fn, int block);
bool lane_width_supported(int W);
// Lane-band items all cost the same: one workgroup per item, no queue.
// rebased: kAccRebased sums instead of kAccPlain.
hipError_t launch_lane(int W, bool rebased, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                       const LaneItem *items, const LanePartner *partners, unsigned n_items, hipStream_t stream);
// Strip shapes of the wavefront kernels: H rows per lane, G wavefronts per pair
// (a workgroup of 64*G lanes covers up to 64*H*G rows of the shorter series).
struct StripShape {
    int H, G;
};
// Instantiated shapes for an accumulation mode (AccMode), in increasing row capacity;
// returns their number (writes at most max_out of them).
int strip_shapes(int accum, StripShape *out, int max_out);
int strip_resident(int accum, StripShape shape, bool banded);
hipError_t launch_strip(int accum, StripShape shape, bool banded, const float *ws, const SeriesInfo *ser,
                        const DatasetInfo *dsi, const WaveItem *items, unsigned n_items, unsigned *queue, int slots,
                        hipStream_t stream);
// Cyclic banded strips (kAccPlain or, with rebased, kAccRebased; window
// required): H rows per block, blocks cycling over the 64 lanes of one
// wavefront; needs 64(H+1) >= 2b+H whenever the pair has more than 64 blocks.
int cyclic_shapes(int *H_out, int max_out);
int cyclic_resident(int H, bool rebased);
hipError_t launch_cyclic(int H, bool rebased, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                         const WaveItem *items, unsigned n_items, unsigned *queue, int slots, hipStream_t stream);

// Last-error message of the calling thread (dtw_last_error), for every host
// source of the library: set_error stores msg and returns code.
int set_error(int code, const char *msg);
void clear_error();

// Clustering scores from a condensed distance matrix (dtw_cluster.hip).
constexpr int kSilhouetteMaxK = 64;  // clusters held in LDS by the row-sum kernel

}  // namespace dtwmi
