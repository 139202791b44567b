// Strip kernel instances with FP64 cells (the kernels: dtw_strip.h).  This
// source is built without signalling-NaN handling (-fno-honor-nans,
// -mno-amdgpu-ieee): the FP64 recurrence never produces a NaN (inadmissible
// cells get a finite 1e30 row value or a +inf pad, never inf - inf), and in
// IEEE mode every v_min_f64 operand of unknown origin would first be quieted
// by an extra v_max_f64.
#include "dtw_strip.h"

namespace dtwmi {
namespace {

const StripEntry kStripsF64[] = {
    DTWMI_STRIP(kAccF64, AccF64, 1, 1),    DTWMI_STRIP(kAccF64, AccF64, 2, 1),    DTWMI_STRIP(kAccF64, AccF64, 4, 1),
    DTWMI_STRIP(kAccF64, AccF64, 8, 1),    DTWMI_STRIP(kAccF64, AccF64, 16, 1),   DTWMI_STRIP(kAccF64, AccF64, 16, 2),
    DTWMI_STRIP(kAccF64, AccF64, 16, 4),   DTWMI_STRIP(kAccF64, AccF64, 16, 8),   DTWMI_STRIP(kAccF64, AccF64, 16, 16),
};

}  // namespace

int strip_f64_entries(const StripEntry **out) {
    *out = kStripsF64;
    return (int)(sizeof(kStripsF64) / sizeof(kStripsF64[0]));
}

}  // namespace dtwmi
