// Structures of the batched path: many independent targets of uneven
// dimension and chain count advanced by one persistent, work-queue kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace restore {

// One target of the batch (device copy).
struct BatchTarget {
    int32_t d, K;
    float log_c;          // ln c_tilde
    int32_t no_kill;      // c_tilde == 0
    float step;           // random-walk sigma
    uint32_t target_id;   // Philox counter word 2
    uint32_t key0, key1;  // Philox key (seed)
    int64_t chain_offset; // first global chain of this target
    int32_t n_chains;
    int32_t param_offset; // floats into the concatenated slab
    int32_t n_steps;      // budget B
    int32_t drain_cap;
    int32_t integrand_p;
    int32_t mu_kind;      // MU_UNIFORM or MU_GMM (the learned-mu form)
    int32_t mu_comp;      // MU_GMM: components
    float mu_beta;        // MU_GMM: defensive uniform share
    int32_t mu_offset;    // MU_GMM: floats into the slab (layout of the learned-mu slab)
    uint32_t chain0;      // global id of the target's chain 0 (Philox counter word 1)
};

// Queue heads: one per bucket (dimension range and mu kind), plus one.
constexpr int BATCH_HEADS = 16;

// A tile of chains of one target: one lane per chain.
struct WorkItem {
    int32_t target;
    int32_t first;   // first local chain
    int32_t count;   // chains in the tile (<= block size)
    int32_t pad;
};

// Per-target slots of the reduction results.
enum BatchSlot : int {
    BS_N = 0, BS_T, BS_A, BS_CENS, BS_CENS_T, BS_NONFINITE, BS_SS_T_N, BS_SS_A_N, BS_SS_A_T, BS_SLOTS = 16
};
enum BatchCounter : int { BC_TRANSITIONS = 0, BC_ACCEPTS, BC_KILLS, BC_SLOTS = 4 };

struct BatchArgs {
    const BatchTarget *targets;
    const WorkItem *items;
    int32_t n_items;
    int32_t n_targets;
    int32_t *queue_head;
    const float *params;
    // per-chain outputs, indexed by chain_offset + local chain
    uint32_t *n_done;
    double *t_done;
    double *a_done;
    uint32_t *status;
    float *t_cur;
    unsigned long long *counters;  // [n_targets][BC_SLOTS]
    double *results;               // [n_targets][BS_SLOTS]
};

// Kernels for items whose dimension lies in [dlo, dhi] and whose target's
// regeneration distribution is of kind mu.
struct BatchKernels {
    const void *persistent = nullptr;
    const void *per_target = nullptr;
};
BatchKernels find_batch_kernels(int dlo, int dhi, int mu);

hipError_t launch_batch_zero(const BatchArgs &b, hipStream_t s);
hipError_t launch_batch_reduce(const BatchArgs &b, hipStream_t s);

}  // namespace restore
