// Accumulation of the binned image splats of one step launch (the records
// step_binned_kernel left in the per-band buckets): each band is summed in
// an LDS tile by n_slices workgroups, whose partial tiles are then added to
// the image in slice order; and the per-pixel estimate of the image
// integrand with its batch-means standard error.
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
    const uint32_t per = (n + s.n_slices - 1) / s.n_slices;
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
    if (blockIdx.x == 0)
        for (int b = threadIdx.x; b < s.n_bins; b += blockDim.x) s.count[b * SPLAT_COUNTER_STRIDE] = 0u;
    if (px >= s.n_pix) return;
    const size_t stride = (size_t)s.n_bins << SPLAT_BAND_SHIFT;
    float v = 0.0f;
    for (int sl = 0; sl < s.n_slices; ++sl) v += s.partial[(size_t)sl * stride + px];
    if (v != 0.0f) s.image[px] += v;
}

hipError_t launch_splat_accumulate(const SplatArgs &s, hipStream_t stream) {
    hipLaunchKernelGGL(splat_accumulate_kernel, dim3(s.n_slices, s.n_bins), dim3(1024),
                       (1 << SPLAT_BAND_SHIFT) * sizeof(float), stream, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(splat_reduce_kernel, dim3((unsigned)((s.n_pix + 255) / 256)), dim3(256), 0, stream, s);
    return hipGetLastError();
}
// Completed tours of each image batch, in a fixed order: block b sums
// n_done over the chains c with floor(c batches / C) = b, i.e. c in
// [ceil(b C / batches), ceil((b + 1) C / batches)), skipping chains whose
// sums are not finite (as the run estimate does).  In tile-stratified runs
// block (b, t) does the same within tile t's chain range, whose batches
// split the tile's chains.
constexpr int IMG_THREADS = 256;
__global__ __launch_bounds__(IMG_THREADS) void image_batch_tours_kernel(ImageEstimateArgs a) {
    __shared__ double sh[IMG_THREADS];
    const int b = blockIdx.x, t = threadIdx.x;
    const int64_t B = a.batches, T = a.n_tiles > 0 ? a.n_tiles : 1, tile = blockIdx.y;
    const int64_t first = (tile * a.n_chains + T - 1) / T;
    const int64_t C = (tile + 1 == T ? a.n_chains : ((tile + 1) * a.n_chains + T - 1) / T) - first;
    const int64_t lo = first + ((int64_t)b * C + B - 1) / B, hi = first + ((int64_t)(b + 1) * C + B - 1) / B;
    double v = 0.0;
    for (int64_t c = lo + t; c < hi; c += IMG_THREADS)
        if (isfinite(a.t_done[c]) && isfinite(a.a_done[c])) v += (double)a.n_done[c];
    sh[t] = v;
    __syncthreads();
    for (int w = IMG_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) a.tours[tile * B + b] = sh[0];
}

// Per pixel j, with S_b the batch images and N_b the batches' tours: the
// ratio estimate c_tilde sum S_b / sum N_b (= the image estimate of the
// whole run) and its delta-method standard error over batches,
//   c_tilde sqrt(sum_b (S_b - R N_b)^2 / ((B - 1) B)) / mean N_b,
// the chain-level formula of the run estimate with batches as units
// (NaN for a single batch).  In tile-stratified runs the pixel's tile t
// supplies the tours N_b of its batches and the factor c_tilde A_t (A_t the
// tile's share of the box) in place of c_tilde.
__global__ __launch_bounds__(256) void image_estimate_kernel(ImageEstimateArgs a) {
    const int64_t px = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (px >= a.n_pix) return;
    const int B = a.batches;
    const double *tours = a.tours;
    double scale = a.c_tilde;
    if (a.n_tiles > 0) {
        const int x = (int)(px % a.image_w), y = (int)(px / a.image_w);
        const int tx = x / a.tile_px, ty = y / a.tile_px;
        tours += (int64_t)(ty * a.tiles_x + tx) * B;
        const int w = min(a.tile_px, a.image_w - tx * a.tile_px), h = min(a.tile_px, a.image_h - ty * a.tile_px);
        scale *= (double)w * h / ((double)a.image_w * a.image_h);
    }
    // batch image b at this pixel (exact from the fixed-point sums if any)
    auto S_b = [&](int b) {
        const int64_t i = (int64_t)b * a.n_pix + px;
        return a.image_fx ? (double)a.image_fx[i] * 0x1p-32 : (double)a.image[i];
    };
    double sS = 0.0, sN = 0.0;
    for (int b = 0; b < B; ++b) {
        sS += S_b(b);
        sN += tours[b];
    }
    const double R = sN > 0.0 ? sS / sN : 0.0;
    double ss = 0.0;
    for (int b = 0; b < B; ++b) {
        const double e = S_b(b) - R * tours[b];
        ss += e * e;
    }
    a.mean[px] = (float)(scale * R);
    a.se[px] = B > 1 && sN > 0.0 ? (float)(scale * sqrt(ss / ((double)(B - 1) * B)) / (sN / B)) : NAN;
}

hipError_t launch_image_estimate(const ImageEstimateArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL(image_batch_tours_kernel, dim3(a.batches, a.n_tiles > 0 ? a.n_tiles : 1), dim3(IMG_THREADS), 0,
                       stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(image_estimate_kernel, dim3((unsigned)((a.n_pix + 255) / 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

__global__ void image_from_fixed_kernel(const unsigned long long *fx, float *image, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) image[i] = (float)((double)fx[i] * 0x1p-32);
}

hipError_t launch_image_from_fixed(const unsigned long long *fx, float *image, int64_t n, hipStream_t stream) {
    hipLaunchKernelGGL(image_from_fixed_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, fx, image,
                       n);
    return hipGetLastError();
}

}  // namespace restore
