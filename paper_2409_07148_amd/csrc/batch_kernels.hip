// gfx950 kernels of the batched path: many independent full-covariance
// mixture targets (uneven dimension, component count and chain count) in
// one persistent launch.
//
// A work item is a tile of chains of one target, one chain per lane.  A
// persistent workgroup pops items from a queue (one atomic per item) in the
// order the host chose (longest-processing-time first by default) and runs
// the whole hot path of its tile in registers: x_0 ~ mu, B steps of Alg. 2
// with regeneration, the drain of the tour in flight, and one store of the
// chain's tour sums.  The per-lane step is the same code as the
// single-target kernels, so a target's chains reproduce a single-target run
// with the same target id bit for bit.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "chain_step.h"

namespace restore {

// LDS floats of the largest learned-mu copy: component blocks and
// cumulative weights of RESTORE_MAX_COMP components at RESTORE_MAX_DIM.
constexpr int MU_LDS_FLOATS = RESTORE_MAX_COMP * (MuGmm<RESTORE_MAX_DIM>::STRIDE + 1);

template <int D, int MU>
__device__ __forceinline__ void run_item(const BatchArgs &b, const BatchTarget &t, const WorkItem &w,
                                         float *mu_sh) {
    constexpr int NB = NBlocks<D>::value;
    StepArgs a{};
    a.n_chains = t.n_chains;
    a.n_comp = t.K;
    a.log_c = t.log_c;
    // the step keeps these in scalar registers: the item (and so its target)
    // is the same for every lane of the workgroup
    a.no_kill = __builtin_amdgcn_readfirstlane(t.no_kill);
    a.step = t.step;
    a.key0 = __builtin_amdgcn_readfirstlane(t.key0);
    a.key1 = __builtin_amdgcn_readfirstlane(t.key1);
    a.target_id = __builtin_amdgcn_readfirstlane(t.target_id);
    a.chain0 = t.chain0;
    a.integrand_p = __builtin_amdgcn_readfirstlane(t.integrand_p);
    a.image = nullptr;
    if (MU == MU_GMM) {
        a.mu_params = b.params + t.mu_offset;
        a.mu_comp = t.mu_comp;
        a.mu_beta = t.mu_beta;
    }
    const const_fptr P = (const_fptr)(b.params + t.param_offset);
    // a learned mu is read from the workgroup's LDS copy for this item, as
    // in the single-target kernels (the same arithmetic, the same chains);
    // every thread of the workgroup copies and meets the barrier
    const auto MR = stage_mu<D, MU>(a, mu_sh);
    using RT = decltype(MR);
    if ((int)threadIdx.x >= w.count) return;
    const uint32_t chain = (uint32_t)(w.first + (int)threadIdx.x);

    // x_0 ~ mu, cached log p and log u; zero sums
    Chain<D, LOC_RWMH> ch;
    {
        float head[4], cand[4 * NB];
        draw_step<NB>(0u, t.chain0 + chain, t.target_id, PURPOSE_INIT, t.key0, t.key1, head, cand);
        sample_mu<D, MU, 4 * NB, RT>(a, head[3], cand, ch.x, MR);
        ch.lp = log_target<D, TGT_FULL, false>(P, t.K, ch.x, ch.g);
        ch.lu = log_mu<D, MU, RT>(a, ch.x, MR);
        ch.a_cur = ch.t_cur = 0.0f;
        ch.a_done = ch.t_done = 0.0;
        ch.n_done = 0u;
        ch.status = ST_ALIVE;
        ch.last_dt = 0.0f;
        ch.splat_pix = -1;
        ch.splat_acc = 0.0f;
        ch.splat_fx = 0ull;
    }
    unsigned long long n_t = 0, n_acc = 0, n_kill = 0;
    bool kill = false, accept = false;
    for (int s = 0; s < t.n_steps; ++s) {
        step_once<D, TGT_FULL, LOC_RWMH, MU, false, const_fptr, false, false, false, false, RT>(
            a, P, (uint32_t)s, chain, ch, kill, accept, nullptr, MR);
        n_acc += __popcll(__ballot(accept));
        n_kill += __popcll(__ballot(kill));
    }
    n_t += __popcll(__ballot(1)) * (unsigned long long)t.n_steps;
    // drain: the tour in flight runs on without regeneration
    bool alive = true;
    for (int s = t.n_steps; s < t.n_steps + t.drain_cap; ++s) {
        const unsigned long long live = __ballot(alive);
        if (live == 0ull) break;
        n_t += __popcll(live);
        bool k = false, ac = false;
        if (alive) {
            step_once<D, TGT_FULL, LOC_RWMH, MU, true, const_fptr, false, false, false, false, RT>(
                a, P, (uint32_t)s, chain, ch, k, ac, nullptr, MR);
            alive = !k;
        }
        n_acc += __popcll(__ballot(ac));
        n_kill += __popcll(__ballot(k));
    }
    const int64_t g = t.chain_offset + chain;
    b.n_done[g] = ch.n_done;
    b.t_done[g] = ch.t_done;
    b.a_done[g] = ch.a_done;
    b.status[g] = alive ? (ST_ALIVE | ST_CENSORED) : 0u;
    b.t_cur[g] = ch.t_cur;
    const unsigned long long active = __ballot(1);
    if ((unsigned)__lane_id() == (unsigned)(__ffsll((long long)active) - 1)) {
        unsigned long long *c = b.counters + (size_t)w.target * BC_SLOTS;
        atomicAdd(c + BC_TRANSITIONS, n_t);
        atomicAdd(c + BC_ACCEPTS, n_acc);
        atomicAdd(c + BC_KILLS, n_kill);
    }
}

template <int DLO, int DHI, int MU>
__device__ __forceinline__ void run_item_dispatch(const BatchArgs &b, const BatchTarget &t, const WorkItem &w,
                                                  float *mu_sh) {
#define RESTORE_BATCH_CASE(D) \
    case D: if constexpr (D >= DLO && D <= DHI) run_item<D, MU>(b, t, w, mu_sh); break;
    switch (t.d) {
        RESTORE_BATCH_CASE(1) RESTORE_BATCH_CASE(2) RESTORE_BATCH_CASE(3) RESTORE_BATCH_CASE(4)
        RESTORE_BATCH_CASE(5) RESTORE_BATCH_CASE(6) RESTORE_BATCH_CASE(7) RESTORE_BATCH_CASE(8)
        RESTORE_BATCH_CASE(9) RESTORE_BATCH_CASE(10) RESTORE_BATCH_CASE(11) RESTORE_BATCH_CASE(12)
        RESTORE_BATCH_CASE(13) RESTORE_BATCH_CASE(14) RESTORE_BATCH_CASE(15) RESTORE_BATCH_CASE(16)
        default: break;
    }
#undef RESTORE_BATCH_CASE
}

// Persistent: every workgroup pops items until the queue is empty, so every
// wave reaches the exit once all items are taken.
template <int DLO, int DHI, int MU>
__global__ __launch_bounds__(256) void batch_persistent_kernel(BatchArgs b) {
    __shared__ int32_t item_sh;
    __shared__ float mu_sh[MU == MU_GMM ? MU_LDS_FLOATS : 1];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) item_sh = atomicAdd(b.queue_head, 1);
        __syncthreads();
        const int32_t item = item_sh;
        if (item >= b.n_items) break;
        const WorkItem w = b.items[item];
        const BatchTarget t = b.targets[w.target];
        run_item_dispatch<DLO, DHI, MU>(b, t, w, mu_sh);
    }
}

// One launch per target (the comparison mode): block i takes the i-th tile.
template <int DLO, int DHI, int MU>
__global__ __launch_bounds__(256) void batch_target_kernel(BatchArgs b, int32_t target) {
    __shared__ float mu_sh[MU == MU_GMM ? MU_LDS_FLOATS : 1];
    const BatchTarget t = b.targets[target];
    WorkItem w;
    w.target = target;
    w.first = (int32_t)(blockIdx.x * blockDim.x);
    w.count = min((int32_t)blockDim.x, t.n_chains - w.first);
    w.pad = 0;
    if (w.count <= 0) return;
    run_item_dispatch<DLO, DHI, MU>(b, t, w, mu_sh);
}

__global__ void batch_zero_kernel(BatchArgs b) {
    // queue_head points at the first of the bucket queue heads
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < BATCH_HEADS) b.queue_head[i] = 0;
    if (i < b.n_targets * BC_SLOTS) b.counters[i] = 0ull;
}

// Per-target float64 sums and residual sums of squares, two passes inside
// one workgroup per target with fixed-order trees (bit-reproducible).
constexpr int BR_THREADS = 256;

__device__ __forceinline__ void br_sum(double *sh, double *v, int nv) {
    const int t = threadIdx.x;
    for (int s = 0; s < nv; ++s) sh[s * BR_THREADS + t] = v[s];
    __syncthreads();
    for (int w = BR_THREADS / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int s = 0; s < nv; ++s) sh[s * BR_THREADS + t] += sh[s * BR_THREADS + t + w];
        __syncthreads();
    }
    for (int s = 0; s < nv; ++s) v[s] = sh[s * BR_THREADS];
    __syncthreads();
}

__global__ __launch_bounds__(BR_THREADS) void batch_reduce_kernel(BatchArgs b) {
    __shared__ double sh[6 * BR_THREADS];
    const BatchTarget t = b.targets[blockIdx.x];
    const int64_t o = t.chain_offset;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int c = threadIdx.x; c < t.n_chains; c += BR_THREADS) {
        const double td = b.t_done[o + c], ad = b.a_done[o + c];
        if (!isfinite(td) || !isfinite(ad)) { v[5] += 1.0; continue; }
        v[0] += (double)b.n_done[o + c];
        v[1] += td;
        v[2] += ad;
        if (b.status[o + c] & ST_CENSORED) { v[3] += 1.0; v[4] += (double)b.t_cur[o + c]; }
    }
    br_sum(sh, v, 6);
    const double N = v[0], T = v[1], A = v[2];
    const double R_tn = N > 0 ? T / N : 0.0, R_an = N > 0 ? A / N : 0.0, R_at = T > 0 ? A / T : 0.0;
    double r[3] = {0, 0, 0};
    for (int c = threadIdx.x; c < t.n_chains; c += BR_THREADS) {
        const double td = b.t_done[o + c], ad = b.a_done[o + c];
        if (!isfinite(td) || !isfinite(ad)) continue;
        const double n = (double)b.n_done[o + c];
        const double e1 = td - R_tn * n, e2 = ad - R_an * n, e3 = ad - R_at * td;
        r[0] += e1 * e1;
        r[1] += e2 * e2;
        r[2] += e3 * e3;
    }
    br_sum(sh, r, 3);
    if (threadIdx.x == 0) {
        double *out = b.results + (size_t)blockIdx.x * BS_SLOTS;
        for (int s = 0; s < 6; ++s) out[s] = v[s];
        out[BS_SS_T_N] = r[0];
        out[BS_SS_A_N] = r[1];
        out[BS_SS_A_T] = r[2];
    }
}

hipError_t launch_batch_zero(const BatchArgs &b, hipStream_t s) {
    const int n = b.n_targets * BC_SLOTS + BATCH_HEADS;
    hipLaunchKernelGGL(batch_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_reduce(const BatchArgs &b, hipStream_t s) {
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(b.n_targets), dim3(BR_THREADS), 0, s, b);
    return hipGetLastError();
}

BatchKernels find_batch_kernels(int dlo, int dhi, int mu) {
    BatchKernels k;
#define RESTORE_BATCH_RANGE(LO, HI)                                                                       \
    if (dlo == LO && dhi == HI) {                                                                         \
        k.persistent = mu == MU_GMM ? (const void *)batch_persistent_kernel<LO, HI, MU_GMM>               \
                                    : (const void *)batch_persistent_kernel<LO, HI, MU_UNIFORM>;          \
        k.per_target = mu == MU_GMM ? (const void *)batch_target_kernel<LO, HI, MU_GMM>                   \
                                    : (const void *)batch_target_kernel<LO, HI, MU_UNIFORM>;              \
        return k;                                                                                         \
    }
    RESTORE_BATCH_RANGE(1, 16)
    RESTORE_BATCH_RANGE(1, 4)
    RESTORE_BATCH_RANGE(5, 8)
    RESTORE_BATCH_RANGE(9, 12)
    RESTORE_BATCH_RANGE(13, 16)
#undef RESTORE_BATCH_RANGE
    return k;
}

}  // namespace restore
