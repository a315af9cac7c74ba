// Measurement probes: the streaming-read ceiling of HBM and the cost of the
// x gather alone, used to place the SpMV kernels on a roofline.
#include "lb_device.h"
#include "lb_internal.h"

namespace lbk {
using namespace lb;

typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void probe_stream_kernel(const f32x4 *__restrict__ p, int64_t n4,
                                                           float *__restrict__ out) {
    float a = 0.f;
    for (int64_t i : grid_stride_range(0, n4)) {
        const f32x4 v = __builtin_nontemporal_load(p + i);
        a += (v.x + v.y) + (v.z + v.w);
    }
    out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = a;
}

__global__ __launch_bounds__(256) void probe_gather_kernel(const int32_t *__restrict__ idx, int64_t n,
                                                           const float *__restrict__ x, float *__restrict__ out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const int32_t c0 = ld_stream(idx + i), c1 = ld_stream(idx + i + stride);
        const int32_t c2 = ld_stream(idx + i + 2 * stride), c3 = ld_stream(idx + i + 3 * stride);
        a0 += x[c0];
        a1 += x[c1];
        a2 += x[c2];
        a3 += x[c3];
    }
    for (; i < n; i += stride) a0 += x[ld_stream(idx + i)];
    out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = (a0 + a1) + (a2 + a3);
}

__global__ __launch_bounds__(256) void probe_copy_kernel(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst,
                                                         int64_t n4) {
    for (int64_t i : grid_stride_range(0, n4)) dst[i] = src[i];
}

hipError_t probe_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const int64_t n4 = static_cast<int64_t>(bytes / 16);
    int64_t grid = (n4 + 255) / 256;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(probe_copy_kernel, dim3(static_cast<uint32_t>(grid)), dim3(256), 0, s,
                       static_cast<const f32x4 *>(src), static_cast<f32x4 *>(dst), n4);
    return hipGetLastError();
}

hipError_t probe_stream_read(const void *buf, size_t bytes, float *out, int grid, hipStream_t s) {
    prof_scope p(s, "probe_stream");
    hipLaunchKernelGGL(probe_stream_kernel, dim3(grid), dim3(256), 0, s, static_cast<const f32x4 *>(buf),
                       static_cast<int64_t>(bytes / 16), out);
    return hipGetLastError();
}

// The banded gather (as in the x_bands = 2 merge path, generalised to
// BANDS in {2, 4, 8}): block b serves band (b mod 8) mod BANDS of the chunks
// slot, slot + grid / BANDS, ... with slot = (b / 8) * (8 / BANDS) +
// (b mod 8) / BANDS, so the bands of a chunk run on different XCDs and XCD
// x only gathers from band x mod BANDS of x (columns [band * cb, (band + 1)
// * cb)); grid is a multiple of 8.
constexpr int kBandChunk = 256 * 8;

template <int BANDS>
__global__ __launch_bounds__(256) void probe_gather_banded_kernel(const int32_t *__restrict__ idx, int64_t n,
                                                                  int32_t cb, const float *__restrict__ x,
                                                                  float *__restrict__ out) {
    const int xcd = static_cast<int>(blockIdx.x % kXcds);
    const int band = xcd % BANDS;
    const int64_t slots = gridDim.x / BANDS;
    float a = 0.f;
    for (int64_t u = static_cast<int64_t>(blockIdx.x / kXcds) * (kXcds / BANDS) + xcd / BANDS; u * kBandChunk < n;
         u += slots) {
        const int64_t base = u * kBandChunk + threadIdx.x;
        int32_t c[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) c[k] = base + k * 256 < n ? idx[base + k * 256] : -1;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (c[k] >= 0 && c[k] / cb == band) a += x[c[k]];
    }
    out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = a;
}

hipError_t probe_gather(const int32_t *idx, int64_t n, const float *x, int32_t cb, float *out, int grid, int bands,
                        hipStream_t s) {
    prof_scope p(s, "probe_gather");
    if (bands == 2)
        hipLaunchKernelGGL(probe_gather_banded_kernel<2>, dim3(grid), dim3(256), 0, s, idx, n, cb, x, out);
    else if (bands == 4)
        hipLaunchKernelGGL(probe_gather_banded_kernel<4>, dim3(grid), dim3(256), 0, s, idx, n, cb, x, out);
    else if (bands == 8)
        hipLaunchKernelGGL(probe_gather_banded_kernel<8>, dim3(grid), dim3(256), 0, s, idx, n, cb, x, out);
    else
        hipLaunchKernelGGL(probe_gather_kernel, dim3(grid), dim3(256), 0, s, idx, n, x, out);
    return hipGetLastError();
}

}  // namespace lbk
