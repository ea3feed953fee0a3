// Kernel handles shared between the kernel translation units and the host
// runtime of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "restore_internal.h"

namespace restore {

// One instantiation of the chain kernels for a (target, dimension, local
// kernel, mu) combination; null members mean "not built".
struct KernelSet {
    const void *init = nullptr;
    const void *refresh = nullptr;
    const void *step = nullptr;
    const void *step_lds = nullptr;
    const void *drain = nullptr;
    const void *drain_lds = nullptr;
    const void *step_binned = nullptr;       // image integrand: binned splats
    const void *step_binned_lds = nullptr;
    const void *step_mh = nullptr;           // the MH reference chain M^l (c_tilde = 0)
    const void *step_tiled = nullptr;        // image integrand, tile-stratified
    const void *drain_tiled = nullptr;
    // small populations with the uniform mu: a chip-wide pre-pass of every
    // step's state-independent random inputs, and the step kernel that
    // reads them instead of drawing them on its own serial path
    const void *rand_prepass = nullptr;
    const void *step_pre = nullptr;    // also runs the next chunk's pre-pass
    const void *drain_pre = nullptr;
};

// Binned splats of one step launch into the image: per-band LDS
// accumulation of the bucketed records into per-slice partial tiles, then a
// fixed-order sum of the slices into the image; clears the band counters.
struct SplatArgs {
    const uint32_t *pix;
    const float *val;
    uint32_t *count;
    float *partial;    // [n_slices][n_bins << SPLAT_BAND_SHIFT]
    float *image;      // [image_batches][image_h][image_w]
    int32_t cap, n_bins, n_slices;
    int64_t n_pix;     // pixels of all batch images
};
hipError_t launch_splat_accumulate(const SplatArgs &s, hipStream_t stream);

// Per-pixel estimate and batch-means standard error of the image integrand
// (restore_image_estimate).
struct ImageEstimateArgs {
    const float *image;      // [batches][n_pix]
    const unsigned long long *image_fx;  // the same in units of 2^-32, or nullptr
    const uint32_t *n_done;  // per chain
    const double *t_done, *a_done;
    int64_t n_chains;
    int32_t batches;
    int64_t n_pix;
    double c_tilde;
    double *tours;           // [max(1, n_tiles)][batches] scratch: completed tours per batch
    float *mean, *se;        // [n_pix]
    // tile-stratified runs (n_tiles > 0): tile edge, tiles per row, image size
    int32_t tile_px, tiles_x, n_tiles, image_w, image_h;
};
hipError_t launch_image_estimate(const ImageEstimateArgs &a, hipStream_t stream);
// image[i] = fx[i] 2^-32 rounded to float32, i < n (fixed-point image runs).
hipError_t launch_image_from_fixed(const unsigned long long *fx, float *image, int64_t n, hipStream_t stream);

KernelSet find_kernels(int tgt, int d, int loc, int mu);
KernelSet find_kernels_hmc(int tgt, int d, int mu);   // loc = LOC_HMC
KernelSet find_kernels_rwu(int tgt, int d, int mu);   // loc = LOC_RWU

// Float64 reduction of the per-chain tour sums (see reduce_kernels.hip).
struct ReduceArgs {
    const double *a_done, *t_done;
    const uint32_t *n_done, *status;
    const float *t_cur;
    int64_t n_chains;
    double *partials;   // [n_blocks][RED_SLOTS]
    double *results;    // [RED_SLOTS]
    int32_t n_blocks;
};

enum ReduceSlot : int {
    RED_N = 0, RED_T, RED_A, RED_CENS, RED_CENS_T, RED_NONFINITE,
    RED_SS_T_N, RED_SS_A_N, RED_SS_A_T,
    RED_SLOTS = 16
};

hipError_t launch_reduce(const ReduceArgs &r, hipStream_t stream);

// Per-tile float64 reduction of tile-stratified runs: for tile t (chains
// [ceil(t C / T), ceil((t + 1) C / T))), results[t][TR_*].
enum TileReduceSlot : int {
    TR_N = 0, TR_T, TR_A, TR_CENS, TR_CENS_T, TR_NONFINITE, TR_SS_TT, TR_SS_AA, TR_SS_TA, TR_CHAINS,
    TR_SLOTS = 16
};
struct TileReduceArgs {
    const double *a_done, *t_done;
    const uint32_t *n_done, *status;
    const float *t_cur;
    int64_t n_chains;
    int32_t n_tiles;
    double *results;    // [n_tiles][TR_SLOTS]
};
hipError_t launch_tile_reduce(const TileReduceArgs &r, hipStream_t stream);

}  // namespace restore
