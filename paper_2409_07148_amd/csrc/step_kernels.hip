// gfx950 kernels of the Jump Restore chain population.
//
// One chain per lane.  A launch loads the chain's state into registers once,
// runs n_steps steps of Alg. 2 entirely in registers and stores the state
// once, so the only HBM traffic per launch is the state itself (the
// parameters are a few KiB read through the scalar cache or LDS).
//
// Every step of Alg. 2 (Jump Restore):
//   t1 ~ Exp(1) (holding time), t2 ~ Exp(k(x)) with k = c_tilde u / p
//   (Sec. 6.2, eq. (killing-rate-simplified)); dt = min(t1, t2);
//   the time integral gains dt f(x_{i-1}) (Sec. 7.4, eq. (approx));
//   t1 < t2: one MH update (Alg. 1) with the small-step kernel;
//   otherwise: the tour ends and x is regenerated from mu.
// Both branches cost one proposal and one density evaluation, so lanes of a
// wave do the same work whichever clock fired.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "restore_internal.h"
#include "targets.h"
#include "launch.h"

namespace restore {

template <int D>
struct NBlocks { static constexpr int value = (D + 3) / 4; };

// Parameters of the target in LDS (broadcast reads) or read through the
// constant address space (wave-uniform addresses -> scalar loads).
template <bool LDS>
struct ParamPtr { using type = const_fptr; };
template <>
struct ParamPtr<true> { using type = const float *; };

template <bool LDS>
__device__ __forceinline__ typename ParamPtr<LDS>::type stage_params(const float *params, int n_floats,
                                                                    float *smem) {
    if constexpr (LDS) {
        for (int i = threadIdx.x; i < n_floats; i += blockDim.x) smem[i] = params[i];
        __syncthreads();
        return smem;
    } else {
        (void)n_floats; (void)smem;
        return (const_fptr)params;
    }
}

template <int D, int MU>
__device__ __forceinline__ float log_mu(const StepArgs &a, const float y[D]) {
    // uniform mu on the box: u = 1 there; regeneration never leaves the box
    (void)a;
    return in_unit_box<D>(y) ? 0.0f : -INFINITY;
}

template <int D, int MU, int NC>
__device__ __forceinline__ void sample_mu(const StepArgs &a, float u_cat, const float cand[NC], float y[D]) {
    (void)a; (void)u_cat;
#pragma unroll
    for (int i = 0; i < D; ++i) y[i] = cand[i];
}

// Per-lane register state of one chain.
template <int D, int LOC>
struct Chain {
    float x[D];
    float g[D];
    float lp, lu;
    float a_cur, t_cur;
    double a_done, t_done;
    uint32_t n_done;
    uint32_t status;
    float last_dt;
    // pixel splats of this lane not yet added to the image: consecutive
    // steps in the same pixel (rejected moves) are combined in registers
    int32_t splat_pix;
    float splat_acc;
};

__device__ __forceinline__ void flush_splat(const StepArgs &a, int32_t pix, float acc) {
    if (pix >= 0) atomicAdd(a.image + pix, acc);
}

template <int D, int LOC>
__device__ __forceinline__ void load_chain(const StepArgs &a, uint32_t c, Chain<D, LOC> &ch) {
    const int64_t C = a.n_chains;
#pragma unroll
    for (int i = 0; i < D; ++i) ch.x[i] = a.x[i * C + c];
    if (LOC == LOC_MALA) {
#pragma unroll
        for (int i = 0; i < D; ++i) ch.g[i] = a.grad[i * C + c];
    }
    ch.lp = a.logp[c];
    ch.lu = a.logu[c];
    ch.a_cur = a.a_cur[c];
    ch.t_cur = a.t_cur[c];
    ch.a_done = a.a_done[c];
    ch.t_done = a.t_done[c];
    ch.n_done = a.n_done[c];
    ch.status = a.status[c];
    ch.last_dt = a.last_dt[c];
    ch.splat_pix = -1;
    ch.splat_acc = 0.0f;
}

template <int D, int LOC>
__device__ __forceinline__ void store_chain(const StepArgs &a, uint32_t c, const Chain<D, LOC> &ch) {
    const int64_t C = a.n_chains;
#pragma unroll
    for (int i = 0; i < D; ++i) a.x[i * C + c] = ch.x[i];
    if (LOC == LOC_MALA) {
#pragma unroll
        for (int i = 0; i < D; ++i) a.grad[i * C + c] = ch.g[i];
    }
    a.logp[c] = ch.lp;
    a.logu[c] = ch.lu;
    a.a_cur[c] = ch.a_cur;
    a.t_cur[c] = ch.t_cur;
    a.a_done[c] = ch.a_done;
    a.t_done[c] = ch.t_done;
    a.n_done[c] = ch.n_done;
    a.status[c] = ch.status;
    a.last_dt[c] = ch.last_dt;
}

// One transition of Alg. 2 for one lane.  Returns kill / accept through the
// flags.  In the drain (RETIRE) a terminated chain is not regenerated.
template <int D, int TGT, int LOC, int MU, bool RETIRE, class PT>
__device__ __forceinline__ void step_once(const StepArgs &a, PT P, uint32_t s,
                                          uint32_t chain, Chain<D, LOC> &ch, bool &kill, bool &accept) {
    constexpr int NB = NBlocks<D>::value;
    if constexpr (std::is_same<PT, const_fptr>::value) {
        // keep the scalar parameter loads inside the step: hoisted out of the
        // step loop, a large slab overflows the SGPRs and spills to VGPR lanes
        uint64_t pv = (uint64_t)P;
        asm volatile("" : "+s"(pv));
        P = (PT)pv;
    }
    float head[4], cand[4 * NB];
    draw_step<NB>(s, chain, a.target_id, PURPOSE_STEP, a.key0, a.key1, head, cand);

    // the two exponential clocks
    const float t1 = -logf(head[0]);
    const float e2 = -logf(head[1]);
    float t2 = INFINITY;
    kill = false;
    if (!a.no_kill) {
        // t2 = E2 / k = E2 exp(log p - log u - ln c_tilde); p = 0 gives t2 = 0
        t2 = e2 * expf(ch.lp - ch.lu - a.log_c);
        kill = !(t1 < t2);
    }
    const float dt = kill ? t2 : t1;

    // accumulate dt f(x_{i-1}) into the tour in flight
    ch.t_cur += dt;
    if (a.integrand_p) ch.a_cur = fmaf(dt, expf(ch.lp), ch.a_cur);
    if (TGT == TGT_PSS && a.image) {
        // f = 1_pixel(x0, x1) at the pre-transition state (p = 0 off the box)
        const float u0 = ch.x[0], u1 = ch.x[1];
        int32_t pix = -1;
        if (u0 >= 0.0f && u0 <= 1.0f && u1 >= 0.0f && u1 <= 1.0f) {
            const int px = min(max((int)(u0 * (float)a.image_w), 0), a.image_w - 1);
            const int py = min(max((int)(u1 * (float)a.image_h), 0), a.image_h - 1);
            pix = py * a.image_w + px;
        }
        if (pix != ch.splat_pix) {
            flush_splat(a, ch.splat_pix, ch.splat_acc);
            ch.splat_pix = pix;
            ch.splat_acc = 0.0f;
        }
        ch.splat_acc += dt;
    }
    ch.last_dt = dt;
    if (kill) {
        ch.a_done += (double)ch.a_cur;
        ch.t_done += (double)ch.t_cur;
        ch.n_done += 1u;
        ch.a_cur = 0.0f;
        ch.t_cur = 0.0f;
    }
    if (RETIRE && kill) {
        accept = false;
        return;
    }

    // candidate: mu sample if killed, small-step proposal otherwise.  A
    // regenerated chain gets its gradient only when it first survives a
    // step, so waves whose lanes were all killed skip that work.
    float y[D];
    float zz = 0.0f;
    const float h = 0.5f * a.step * a.step;
    if (kill) {
        sample_mu<D, MU, 4 * NB>(a, head[3], cand, y);
    } else {
        if (LOC == LOC_MALA && !(ch.status & ST_GRAD_VALID)) {
            (void)log_target<D, TGT, true>(P, a.n_comp, ch.x, ch.g);
            ch.status |= ST_GRAD_VALID;
        }
        float z[D];
        box_muller<D, 4 * NB>(cand, z);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            float delta = a.step * z[i];
            if (LOC == LOC_MALA) {
                delta = fmaf(h, ch.g[i], delta);
                zz = fmaf(z[i], z[i], zz);
            }
            y[i] = ch.x[i] + delta;
        }
    }

    float gy[D];
    const float lpy = log_target<D, TGT, LOC == LOC_MALA>(P, a.n_comp, y, gy, !kill);
    const float luy = log_mu<D, MU>(a, y);

    accept = false;
    if (!kill) {
        if (ch.lp == -INFINITY) {
            accept = true;  // alpha = 1 where p(x) q(x, y) = 0
        } else {
            float lr = lpy - ch.lp;
            if (LOC == LOC_MALA) {
                // ln q(x->y) = -|z|^2 / 2 ;  ln q(y->x) = -|x - y - h g(y)|^2 / (2 eps^2);
                // x - y is exact in float32 for neighbouring states (Sterbenz)
                float rr = 0.0f;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const float r = fmaf(-h, gy[i], ch.x[i] - y[i]);
                    rr = fmaf(r, r, rr);
                }
                lr += 0.5f * zz - rr / (2.0f * a.step * a.step);
            }
            accept = logf(head[2]) < lr;
        }
    }
    if (kill || accept) {
#pragma unroll
        for (int i = 0; i < D; ++i) ch.x[i] = y[i];
        if (LOC == LOC_MALA) {
            if (accept) {
#pragma unroll
                for (int i = 0; i < D; ++i) ch.g[i] = gy[i];
                ch.status |= ST_GRAD_VALID;
            } else {
                ch.status &= ~ST_GRAD_VALID;
            }
        }
        ch.lp = lpy;
        ch.lu = luy;
    }
}

__device__ __forceinline__ void add_counters(unsigned long long *counters, unsigned long long t,
                                             unsigned long long acc, unsigned long long kil) {
    // one lane per wave publishes the wave's ballot counts
    const unsigned long long active = __ballot(1);
    if ((unsigned)lane_id() == (unsigned)(__ffsll((long long)active) - 1)) {
        atomicAdd(counters + CNT_TRANSITIONS, t);
        atomicAdd(counters + CNT_ACCEPTS, acc);
        atomicAdd(counters + CNT_KILLS, kil);
    }
}

// Steps with regeneration for every chain.
template <int D, int TGT, int LOC, int MU, bool LDS>
__global__ __launch_bounds__(256) void step_kernel(StepArgs a, int n_param_floats) {
    extern __shared__ float smem[];
    const auto P = stage_params<LDS>(a.params, n_param_floats, smem);
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_chains) return;
    Chain<D, LOC> ch;
    load_chain(a, (uint32_t)c, ch);
    unsigned long long n_acc = 0, n_kill = 0;
    bool kill = false, accept = false;
    for (int it = 0; it < a.n_steps; ++it) {
        step_once<D, TGT, LOC, MU, false>(a, P, a.s0 + (uint32_t)it, (uint32_t)c, ch, kill, accept);
        n_acc += __popcll(__ballot(accept));
        n_kill += __popcll(__ballot(kill));
    }
    ch.status = (ch.status & ~(ST_LAST_KILL | ST_LAST_ACCEPT)) | (kill ? ST_LAST_KILL : 0u) |
                (accept ? ST_LAST_ACCEPT : 0u);
    if (TGT == TGT_PSS && a.image) flush_splat(a, ch.splat_pix, ch.splat_acc);
    store_chain(a, (uint32_t)c, ch);
    const unsigned long long lanes = __popcll(__ballot(1));
    add_counters(a.counters, lanes * (unsigned long long)a.n_steps, n_acc, n_kill);
}

// Drain: the chains of the input list run on without regeneration until
// their tour in flight is killed.  Survivors of this chunk are compacted
// into the output list with one ballot and one atomic per wave; on the last
// chunk they are marked censored instead.
template <int D, int TGT, int LOC, int MU, bool LDS>
__global__ __launch_bounds__(256) void drain_kernel(StepArgs a, int n_param_floats, uint32_t *list_out,
                                                     uint32_t *count_out, uint32_t *count_zero,
                                                     int last_chunk) {
    extern __shared__ float smem[];
    const auto P = stage_params<LDS>(a.params, n_param_floats, smem);
    if (blockIdx.x == 0 && threadIdx.x == 0) *count_zero = 0u;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_in = a.list ? (int64_t)*a.list_count : a.n_chains;
    if (idx >= n_in) return;
    const uint32_t c = a.list ? a.list[idx] : (uint32_t)idx;
    Chain<D, LOC> ch;
    load_chain(a, c, ch);
    bool alive = (ch.status & ST_ALIVE) != 0u;
    unsigned long long n_t = 0, n_acc = 0, n_kill = 0;
    bool stepped = false, kill_last = false, acc_last = false;
    for (int it = 0; it < a.n_steps; ++it) {
        const unsigned long long live = __ballot(alive);
        if (live == 0ull) break;
        n_t += __popcll(live);
        bool kill = false, accept = false;
        if (alive) {
            step_once<D, TGT, LOC, MU, true>(a, P, a.s0 + (uint32_t)it, c, ch, kill, accept);
            stepped = true;
            kill_last = kill;
            acc_last = accept;
            alive = !kill;
        }
        n_acc += __popcll(__ballot(accept));
        n_kill += __popcll(__ballot(kill));
    }
    if (stepped) {
        ch.status = (ch.status & ~(ST_LAST_KILL | ST_LAST_ACCEPT | ST_ALIVE)) | (alive ? ST_ALIVE : 0u) |
                    (kill_last ? ST_LAST_KILL : 0u) | (acc_last ? ST_LAST_ACCEPT : 0u);
    }
    if (alive && last_chunk) ch.status |= ST_CENSORED;
    if (TGT == TGT_PSS && a.image) flush_splat(a, ch.splat_pix, ch.splat_acc);
    store_chain(a, c, ch);
    add_counters(a.counters, n_t, n_acc, n_kill);
    if (!last_chunk) {
        const unsigned long long keep = __ballot(alive);
        if (keep) {
            const int leader = __ffsll((long long)keep) - 1;
            uint32_t base = 0;
            if (lane_id() == leader) base = atomicAdd(count_out, (uint32_t)__popcll(keep));
            base = __shfl(base, leader);
            if (alive) {
                const uint32_t below = (uint32_t)__popcll(keep & ((1ull << lane_id()) - 1ull));
                list_out[base + below] = c;
            }
        }
    }
}

// x_0 ~ mu (purpose INIT, step 0), cached log p / log u / grad, zero sums.
template <int D, int TGT, int LOC, int MU>
__global__ __launch_bounds__(256) void init_kernel(StepArgs a) {
    constexpr int NB = NBlocks<D>::value;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_chains) return;
    float head[4], cand[4 * NB];
    draw_step<NB>(0u, (uint32_t)c, a.target_id, PURPOSE_INIT, a.key0, a.key1, head, cand);
    Chain<D, LOC> ch;
    sample_mu<D, MU, 4 * NB>(a, head[3], cand, ch.x);
    ch.lp = log_target<D, TGT, LOC == LOC_MALA>((const_fptr)a.params, a.n_comp, ch.x, ch.g);
    ch.lu = log_mu<D, MU>(a, ch.x);
    ch.a_cur = ch.t_cur = 0.0f;
    ch.a_done = ch.t_done = 0.0;
    ch.n_done = 0u;
    ch.status = ST_ALIVE | (LOC == LOC_MALA ? ST_GRAD_VALID : 0u);
    ch.last_dt = 0.0f;
    store_chain(a, (uint32_t)c, ch);
}

// Recompute the cached log p, log u and grad log p from x.
template <int D, int TGT, int LOC, int MU>
__global__ __launch_bounds__(256) void refresh_kernel(StepArgs a) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_chains) return;
    const int64_t C = a.n_chains;
    float x[D], g[D];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = a.x[i * C + c];
    a.logp[c] = log_target<D, TGT, LOC == LOC_MALA>((const_fptr)a.params, a.n_comp, x, g);
    a.logu[c] = log_mu<D, MU>(a, x);
    if (LOC == LOC_MALA) {
#pragma unroll
        for (int i = 0; i < D; ++i) a.grad[i * C + c] = g[i];
        a.status[c] |= ST_GRAD_VALID;
    }
}

// ---------------------------------------------------------------------------
// dispatch table
// ---------------------------------------------------------------------------

template <int D, int TGT, int LOC, int MU>
static KernelSet make_set() {
    KernelSet k;
    k.init = (const void *)init_kernel<D, TGT, LOC, MU>;
    k.refresh = (const void *)refresh_kernel<D, TGT, LOC, MU>;
    k.step = (const void *)step_kernel<D, TGT, LOC, MU, false>;
    k.step_lds = (const void *)step_kernel<D, TGT, LOC, MU, true>;
    k.drain = (const void *)drain_kernel<D, TGT, LOC, MU, false>;
    k.drain_lds = (const void *)drain_kernel<D, TGT, LOC, MU, true>;
    return k;
}

#define RESTORE_SETS_FOR(TGT, LOC, MU)                                                                \
    case 1: return make_set<1, TGT, LOC, MU>();   case 2: return make_set<2, TGT, LOC, MU>();           \
    case 3: return make_set<3, TGT, LOC, MU>();   case 4: return make_set<4, TGT, LOC, MU>();           \
    case 5: return make_set<5, TGT, LOC, MU>();   case 6: return make_set<6, TGT, LOC, MU>();           \
    case 7: return make_set<7, TGT, LOC, MU>();   case 8: return make_set<8, TGT, LOC, MU>();           \
    case 9: return make_set<9, TGT, LOC, MU>();   case 10: return make_set<10, TGT, LOC, MU>();         \
    case 11: return make_set<11, TGT, LOC, MU>(); case 12: return make_set<12, TGT, LOC, MU>();         \
    case 13: return make_set<13, TGT, LOC, MU>(); case 14: return make_set<14, TGT, LOC, MU>();         \
    case 15: return make_set<15, TGT, LOC, MU>(); case 16: return make_set<16, TGT, LOC, MU>();

KernelSet find_kernels(int tgt, int d, int loc, int mu) {
    if (mu != MU_UNIFORM) return KernelSet{};
    if (tgt == TGT_PSS) {
        if (d == 12 && loc == LOC_RWMH) return make_set<12, TGT_PSS, LOC_RWMH, MU_UNIFORM>();
        return KernelSet{};
    }
    if (tgt == TGT_ISO && loc == LOC_RWMH) {
        switch (d) { RESTORE_SETS_FOR(TGT_ISO, LOC_RWMH, MU_UNIFORM) default: break; }
    } else if (tgt == TGT_ISO && loc == LOC_MALA) {
        switch (d) { RESTORE_SETS_FOR(TGT_ISO, LOC_MALA, MU_UNIFORM) default: break; }
    } else if (tgt == TGT_FULL && loc == LOC_RWMH) {
        switch (d) { RESTORE_SETS_FOR(TGT_FULL, LOC_RWMH, MU_UNIFORM) default: break; }
    } else if (tgt == TGT_FULL && loc == LOC_MALA) {
        switch (d) { RESTORE_SETS_FOR(TGT_FULL, LOC_MALA, MU_UNIFORM) default: break; }
    }
    return KernelSet{};
}

}  // namespace restore
