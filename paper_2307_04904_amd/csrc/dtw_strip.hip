// Strip kernel instances with FP32 cells (plain, rebased, Kahan-compensated);
// the kernels are in dtw_strip.h, the FP64 instances in dtw_strip_f64.hip.
#include "dtw_strip.h"

namespace dtwmi {
namespace {

// Instantiated shapes, per accumulation mode in increasing row capacity 64*H*G.
const StripEntry kStrips[] = {
    // plain FP32: every height up to 8, then steps of 2 to 16, of 4 to 32, of 8 to 64,
    // so that a series of n points fills at least ~85% of its lanes' rows
    DTWMI_STRIP(kAccPlain, AccPlain, 1, 1),  DTWMI_STRIP(kAccPlain, AccPlain, 2, 1),  DTWMI_STRIP(kAccPlain, AccPlain, 3, 1),
    DTWMI_STRIP(kAccPlain, AccPlain, 4, 1),  DTWMI_STRIP(kAccPlain, AccPlain, 5, 1),  DTWMI_STRIP(kAccPlain, AccPlain, 6, 1),
    DTWMI_STRIP(kAccPlain, AccPlain, 7, 1),  DTWMI_STRIP(kAccPlain, AccPlain, 8, 1),  DTWMI_STRIP(kAccPlain, AccPlain, 10, 1),
    DTWMI_STRIP(kAccPlain, AccPlain, 12, 1), DTWMI_STRIP(kAccPlain, AccPlain, 14, 1), DTWMI_STRIP(kAccPlain, AccPlain, 16, 1),
    DTWMI_STRIP(kAccPlain, AccPlain, 20, 1), DTWMI_STRIP(kAccPlain, AccPlain, 24, 1), DTWMI_STRIP(kAccPlain, AccPlain, 28, 1),
    DTWMI_STRIP(kAccPlain, AccPlain, 32, 1), DTWMI_STRIP(kAccPlain, AccPlain, 16, 2), DTWMI_STRIP(kAccPlain, AccPlain, 40, 1),
    DTWMI_STRIP(kAccPlain, AccPlain, 48, 1), DTWMI_STRIP(kAccPlain, AccPlain, 24, 2), DTWMI_STRIP(kAccPlain, AccPlain, 56, 1),
    DTWMI_STRIP(kAccPlain, AccPlain, 64, 1), DTWMI_STRIP(kAccPlain, AccPlain, 32, 2), DTWMI_STRIP(kAccPlain, AccPlain, 32, 4),
    DTWMI_STRIP(kAccPlain, AccPlain, 32, 8), DTWMI_STRIP(kAccPlain, AccPlain, 64, 8),
    // rebased FP32: the same shapes
    DTWMI_STRIP(kAccRebased, AccRebased, 1, 1),  DTWMI_STRIP(kAccRebased, AccRebased, 2, 1),  DTWMI_STRIP(kAccRebased, AccRebased, 3, 1),
    DTWMI_STRIP(kAccRebased, AccRebased, 4, 1),  DTWMI_STRIP(kAccRebased, AccRebased, 5, 1),  DTWMI_STRIP(kAccRebased, AccRebased, 6, 1),
    DTWMI_STRIP(kAccRebased, AccRebased, 7, 1),  DTWMI_STRIP(kAccRebased, AccRebased, 8, 1),  DTWMI_STRIP(kAccRebased, AccRebased, 10, 1),
    DTWMI_STRIP(kAccRebased, AccRebased, 12, 1), DTWMI_STRIP(kAccRebased, AccRebased, 14, 1), DTWMI_STRIP(kAccRebased, AccRebased, 16, 1),
    DTWMI_STRIP(kAccRebased, AccRebased, 20, 1), DTWMI_STRIP(kAccRebased, AccRebased, 24, 1), DTWMI_STRIP(kAccRebased, AccRebased, 28, 1),
    DTWMI_STRIP(kAccRebased, AccRebased, 32, 1), DTWMI_STRIP(kAccRebased, AccRebased, 16, 2), DTWMI_STRIP(kAccRebased, AccRebased, 40, 1),
    DTWMI_STRIP(kAccRebased, AccRebased, 48, 1), DTWMI_STRIP(kAccRebased, AccRebased, 24, 2), DTWMI_STRIP(kAccRebased, AccRebased, 56, 1),
    DTWMI_STRIP(kAccRebased, AccRebased, 64, 1), DTWMI_STRIP(kAccRebased, AccRebased, 32, 2), DTWMI_STRIP(kAccRebased, AccRebased, 32, 4),
    DTWMI_STRIP(kAccRebased, AccRebased, 32, 8), DTWMI_STRIP(kAccRebased, AccRebased, 64, 8),
    DTWMI_STRIP(kAccKahan, AccKahan, 1, 1),  DTWMI_STRIP(kAccKahan, AccKahan, 2, 1),  DTWMI_STRIP(kAccKahan, AccKahan, 4, 1),
    DTWMI_STRIP(kAccKahan, AccKahan, 8, 1),  DTWMI_STRIP(kAccKahan, AccKahan, 16, 1), DTWMI_STRIP(kAccKahan, AccKahan, 16, 2),
    DTWMI_STRIP(kAccKahan, AccKahan, 16, 4), DTWMI_STRIP(kAccKahan, AccKahan, 16, 8), DTWMI_STRIP(kAccKahan, AccKahan, 16, 16),
};

// Grid of a launch: one workgroup per item, or with a queue the resident
// workgroups (at most one per item).
unsigned grid_for(unsigned n, unsigned *queue, int slots) {
    if (!queue || slots <= 0) return n;
    return n < static_cast<unsigned>(slots) ? n : static_cast<unsigned>(slots);
}

// The entry of an instance (nullptr if none).
const StripEntry *find_strip(int accum, StripShape shape) {
    const StripEntry *f64 = nullptr;
    const int nf = strip_f64_entries(&f64);
    const StripEntry *tab = accum == kAccF64 ? f64 : kStrips;
    const int n = accum == kAccF64 ? nf : (int)(sizeof(kStrips) / sizeof(kStrips[0]));
    for (int i = 0; i < n; ++i)
        if (tab[i].accum == accum && tab[i].H == shape.H && tab[i].G == shape.G) return &tab[i];
    return nullptr;
}

}  // namespace

int strip_shapes(int accum, StripShape *out, int max_out) {
    const StripEntry *f64 = nullptr;
    const int nf = strip_f64_entries(&f64);
    const StripEntry *tab = accum == kAccF64 ? f64 : kStrips;
    const int n = accum == kAccF64 ? nf : (int)(sizeof(kStrips) / sizeof(kStrips[0]));
    int k = 0;
    for (int i = 0; i < n; ++i)
        if (tab[i].accum == accum) {
            if (out && k < max_out) out[k] = StripShape{tab[i].H, tab[i].G};
            ++k;
        }
    return k;
}

int strip_resident(int accum, StripShape shape, bool banded, bool passes) {
    const StripEntry *e = find_strip(accum, shape);
    return e ? e->slots(banded, passes) : 0;
}

hipError_t launch_strip(int accum, StripShape shape, bool banded, const float *ws, const SeriesInfo *ser,
                        const DatasetInfo *dsi, const WaveItem *items, unsigned n_items, unsigned *queue, int slots,
                        void *pass_buf, int64_t pass_stride, hipStream_t stream) {
    if (n_items == 0) return hipSuccess;
    const StripEntry *e = find_strip(accum, shape);
    if (!e) return hipErrorInvalidValue;
    return e->fn(banded, ws, ser, dsi, items, n_items, queue, grid_for(n_items, queue, slots), pass_buf, pass_stride,
                 stream);
}

int strip_grid(unsigned n_items, unsigned *queue, int slots) { return (int)grid_for(n_items, queue, slots); }

}  // namespace dtwmi
