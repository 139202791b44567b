// Lane-band kernel instances with plain FP32 sums (the kernel: dtw_lane.h).
#include "dtw_lane.h"

namespace dtwmi {
namespace {

const std::array<LaneFn, (kLaneMaxW + 1) / 2> kLaneTable =
    make_lane_table<false>(std::make_index_sequence<(kLaneMaxW + 1) / 2>{});

}  // namespace

bool lane_width_supported(int W) { return W >= 1 && W <= kLaneMaxW && (W & 1); }

hipError_t launch_lane_rebased(int W, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                               const LaneItem *items, const LanePartner *partners, unsigned n_items,
                               hipStream_t stream);

hipError_t launch_lane(int W, bool rebased, const float *ws, const SeriesInfo *ser, const DatasetInfo *dsi,
                       const LaneItem *items, const LanePartner *partners, unsigned n_items, hipStream_t stream) {
    if (!lane_width_supported(W)) return hipErrorInvalidValue;
    if (n_items == 0) return hipSuccess;
    if (rebased) return launch_lane_rebased(W, ws, ser, dsi, items, partners, n_items, stream);
    return kLaneTable[(W - 1) / 2](ws, ser, dsi, items, partners, n_items, stream);
}

}  // namespace dtwmi
