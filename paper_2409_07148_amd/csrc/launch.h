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
};

KernelSet find_kernels(int tgt, int d, int loc, int mu);

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

}  // namespace restore
