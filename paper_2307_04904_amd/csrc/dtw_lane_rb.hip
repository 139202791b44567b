// Lane-band kernel instances with rebased FP32 sums (the kernel: dtw_lane.h).
#include "dtw_lane.h"

namespace dtwmi {
namespace {

const std::array<LaneFn, (kLaneMaxW + 1) / 2> kLaneTableRb =
    make_lane_table<true>(std::make_index_sequence<(kLaneMaxW + 1) / 2>{});

}  // namespace

// Called by launch_lane (dtw_lane.hip) after its argument checks.
hipError_t launch_lane_rebased(int W, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                               const LaneItem *items, const LanePartner *partners, unsigned n_items,
                               hipStream_t stream) {
    return kLaneTableRb[(W - 1) / 2](ws, ser, dsi, items, partners, n_items, stream);
}

}  // namespace dtwmi
