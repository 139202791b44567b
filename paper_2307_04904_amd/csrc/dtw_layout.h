// Data layout shared by the host planner and the kernels: the staged series,
// the per-dataset records and the work items.  Not part of the public ABI.
#pragma once

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
//   kAccRebased: the plain FP32 cell, with stored values relative to a base
//                that moves up every few steps to a lower bound of every
//                value still to come (rounding relative to the small stored
//                values).
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

}  // namespace dtwmi
