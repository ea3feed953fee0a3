// Accumulation of the binned image splats of one step launch (the records
// step_binned_kernel left in the per-band buckets): each band is summed in
// an LDS tile by SPLAT_SLICES workgroups, whose partial tiles are then added
// to the image in slice order.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "launch.h"

namespace restore {

// Per band b and slice: the slice's share of band b's records summed into a
// 2^SPLAT_BAND_SHIFT-pixel LDS tile, written to partial[slice][band pixels].
__global__ __launch_bounds__(1024) void splat_accumulate_kernel(SplatArgs s) {
    extern __shared__ float tile[];
    constexpr int BAND = 1 << SPLAT_BAND_SHIFT;
    const int b = blockIdx.y, sl = blockIdx.x, t = threadIdx.x;
    const uint32_t reserved = s.count[b * SPLAT_COUNTER_STRIDE];
    const uint32_t n = reserved < (uint32_t)s.cap ? reserved : (uint32_t)s.cap;
    for (int j = t; j < BAND; j += blockDim.x) tile[j] = 0.0f;
    __syncthreads();
    const uint32_t per = (n + SPLAT_SLICES - 1) / SPLAT_SLICES;
    const uint32_t lo = (uint32_t)sl * per;
    const uint32_t hi = lo + per < n ? lo + per : n;
    const uint32_t *pix = s.pix + (size_t)b * (size_t)s.cap;
    const float *val = s.val + (size_t)b * (size_t)s.cap;
    const uint32_t off = (uint32_t)b << SPLAT_BAND_SHIFT;
    // eight records in flight per thread, then their LDS additions
    const uint32_t nt = blockDim.x;
    uint32_t i = lo + t;
    for (; i + 7 * nt < hi; i += 8 * nt) {
        uint32_t q[8];
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            q[k] = pix[i + k * nt];
            v[k] = val[i + k * nt];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) atomicAdd(&tile[q[k] - off], v[k]);
    }
    for (; i < hi; i += nt) atomicAdd(&tile[pix[i] - off], val[i]);
    __syncthreads();
    float *out = s.partial + (size_t)sl * ((size_t)s.n_bins << SPLAT_BAND_SHIFT) + off;
    for (int j = t; j < BAND; j += blockDim.x) out[j] = tile[j];
}

// image[px] += sum over slices (in slice order) of partial[slice][px]; block 0
// also clears the band counters for the next step launch.
__global__ __launch_bounds__(256) void splat_reduce_kernel(SplatArgs s) {
    const int64_t px = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < s.n_bins) s.count[threadIdx.x * SPLAT_COUNTER_STRIDE] = 0u;
    if (px >= s.n_pix) return;
    const size_t stride = (size_t)s.n_bins << SPLAT_BAND_SHIFT;
    float v = 0.0f;
#pragma unroll
    for (int sl = 0; sl < SPLAT_SLICES; ++sl) v += s.partial[(size_t)sl * stride + px];
    if (v != 0.0f) s.image[px] += v;
}

hipError_t launch_splat_accumulate(const SplatArgs &s, hipStream_t stream) {
    hipLaunchKernelGGL(splat_accumulate_kernel, dim3(SPLAT_SLICES, s.n_bins), dim3(1024),
                       (1 << SPLAT_BAND_SHIFT) * sizeof(float), stream, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(splat_reduce_kernel, dim3((unsigned)((s.n_pix + 255) / 256)), dim3(256), 0, stream, s);
    return hipGetLastError();
}

}  // namespace restore
