// Staging of the inputs into the padded FP32 workspace, the queue reset
// kernel, and the occupancy query the wavefront launchers share.
#include "dtw_device.h"

namespace dtwmi {
namespace {

// ---------------------------------------------------------------------------
// Staging: copy every series into its padded FP32 slot, widening 16-bit types
// exactly, with +inf in the pads.
__global__ __launch_bounds__(256) void k_stage(const SeriesSrc *__restrict__ src,
                                               const SeriesInfo *__restrict__ ser,
                                               float *__restrict__ ws) {
    const int g = blockIdx.x;
    const SeriesSrc s = src[g];
    const SeriesInfo si = ser[g];
    float *dst = ws + si.pstart - kPad;
    const int total = (si.len + 2 * kPad + 3) & ~3;
    for (int p = threadIdx.x; p < total; p += blockDim.x) {
        const int t = p - kPad;
        float v = kInf;
        if (t >= 0 && t < s.len) {
            if (s.dtype == 0) {
                v = static_cast<const float *>(s.base)[s.off + t];
            } else if (s.dtype == 1) {
                const unsigned short b = static_cast<const unsigned short *>(s.base)[s.off + t];
                v = __uint_as_float(static_cast<unsigned int>(b) << 16);
            } else {
                v = static_cast<float>(static_cast<const _Float16 *>(s.base)[s.off + t]);
            }
        }
        dst[p] = v;
    }
}

__global__ __launch_bounds__(64) void k_zero(unsigned *__restrict__ p, int n) {
    for (int i = threadIdx.x; i < n; i += 64) p[i] = 0u;
}

// Re-point a one-dataset plan at other buffers of the same shape: every
// series' source buffer and the dataset's output.
__global__ __launch_bounds__(256) void k_rebind(SeriesSrc *__restrict__ src, int nseries, const void *series,
                                                DatasetInfo *__restrict__ dsi, float *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nseries) src[i].base = series;
    if (i == 0) dsi[0].out = out;
}

}  // namespace

int resident_blocks(const void *fn, int block) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, block, 0) != hipSuccess) return 0;
    return cus * per;
}

hipError_t launch_stage(const SeriesSrc *src, const SeriesInfo *ser, float *ws, int32_t nseries,
                        hipStream_t stream) {
    if (nseries <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stage, dim3(nseries), dim3(256), 0, stream, src, ser, ws);
    return hipGetLastError();
}

hipError_t launch_rebind(SeriesSrc *src, int32_t nseries, const void *series, DatasetInfo *dsi, float *out,
                         hipStream_t stream) {
    hipLaunchKernelGGL(k_rebind, dim3((nseries + 255) / 256 > 0 ? (nseries + 255) / 256 : 1), dim3(256), 0, stream,
                       src, nseries, series, dsi, out);
    return hipGetLastError();
}

hipError_t launch_zero(unsigned *p, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, stream, p, n);
    return hipGetLastError();
}

}  // namespace dtwmi
