// Kernel launchers shared by the host planner (dtw_api.hip) and the kernel
// sources (dtw_stage.hip, dtw_lane.hip, dtw_strip.hip, dtw_cyclic.hip,
// dtw_cluster.hip, dtw_path.hip); the data layout is in dtw_layout.h.  Not
// part of the public ABI.
#pragma once

#include "dtw_layout.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dtwmi {

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
// The split lane-band kernel (dtw_lane_split.hip): P = 4, 8, 12, 16 or 32
// lanes per pair, 64/P pairs per wavefront (integer division: 12 lanes give 5
// and leave 4 lanes idle), plain FP32 sums; items of at most 64/P partners,
// one workgroup each; 3 to split_max_cells(P) band cells per lane.
int split_max_cells(int P);
bool lane_split_supported(int P, int W);
hipError_t launch_lane_split(int P, int W, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                             const LaneItem *items, const LanePartner *partners, unsigned n_items,
                             hipStream_t stream);
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
// Workgroups of an instance the device holds at once (passes: the row-pass form).
int strip_resident(int accum, StripShape shape, bool banded, bool passes);
// Pairs whose shorter series exceeds 64*H*G rows are swept in row passes; they
// need pass_buf: pass_stride (>= the longest swept series) values of the
// mode's cell type (strip_cell_bytes) per workgroup of the launch
// (strip_grid workgroups), else nullptr.
hipError_t launch_strip(int accum, StripShape shape, bool banded, const float *ws, const SeriesInfo *ser,
                        const DatasetInfo *dsi, const WaveItem *items, unsigned n_items, unsigned *queue, int slots,
                        void *pass_buf, int64_t pass_stride, hipStream_t stream);
int strip_grid(unsigned n_items, unsigned *queue, int slots);  // workgroups of a strip launch
constexpr int strip_cell_bytes(int accum) { return accum == kAccF64 || accum == kAccKahan ? 8 : 4; }
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
