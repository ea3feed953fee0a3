// Per-lane machinery of one Jump Restore chain, shared by the single-target
// kernels and the batched persistent kernel so that both run exactly the
// same arithmetic for a given (seed, chain, target id).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "restore_internal.h"
#include "targets.h"

namespace restore {

template <int D>
struct NBlocks { static constexpr int value = (D + 3) / 4; };

// Most components per log-sum-exp block of the target density: the HMC
// kernels keep the leapfrog state besides the chain's, and blocks of one
// component keep their scalar registers from spilling (measured faster
// there; the other kernels gain from blocks).
template <int LOC>
struct DensityBlock { static constexpr int value = LOC == LOC_HMC ? 1 : 4; };

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

// The learned mu's component blocks and cumulative weights in LDS, for
// kernels that evaluate log u and sample mu at every step (see MuGmm); the
// other kernels read them through the scalar cache, with the same
// arithmetic and so the same results.
template <int D, int MU>
__device__ __forceinline__ auto stage_mu(const StepArgs &a, float *smem) {
    if constexpr (MU == MU_GMM) {
        const int n = a.mu_comp * (MuGmm<D>::STRIDE + 1);
        const float *src = a.mu_params + 4;
        for (int i = threadIdx.x; i < n; i += blockDim.x) smem[i] = src[i];
        __syncthreads();
        return (lds_fptr)smem;
    } else {
        (void)a; (void)smem;
        return (const_fptr) nullptr;
    }
}

template <int D, int MU, class RT = const_fptr>
__device__ __forceinline__ float log_mu(const StepArgs &a, const float y[D], RT R = RT()) {
    if constexpr (MU == MU_GMM) {
        const auto P = (const_fptr)a.mu_params;
        if constexpr (std::is_same<typename std::remove_cv<RT>::type, lds_fptr>::value) {
            return MuGmm<D>::log_u(P, R, a.mu_comp, y);
        } else {
            (void)R;
            return MuGmm<D>::log_u(P, P + 4, a.mu_comp, y);
        }
    } else {
        (void)R;
        // uniform mu on the box: u = 1 there
        (void)a;
        return in_unit_box<D>(y) ? 0.0f : -INFINITY;
    }
}

// The second cached density of a state.  For the pi-invariant local
// kernels it is log u, and k = c_tilde u / p (Sec. 6.2, eq.
// (killing-rate-simplified)).  For the unadjusted random-walk jump process
// it is log u_eff with u_eff = u + (Q^T p - p) / c_tilde, so that the same
// k = c_tilde u_eff / p is the rate (c_tilde u + L* p) / p of Sec. 6.2,
// eq. (killing-rate) (L* p = Q^T p - p).  Where u_eff < 0 (c_tilde below
// sup (p - Q^T p) / u) the value is NaN: the step's holding time is then
// NaN and the chain's sums are reported as non-finite.  Off the box (p = 0,
// k = inf) it is not used and set to 0.
template <int D, int TGT, int LOC, int MU, class PT, class RT = const_fptr>
__device__ __forceinline__ float log_u_state(const StepArgs &a, PT P, const float y[D], float lp, RT R = RT()) {
    const float lu = log_mu<D, MU>(a, y, R);
    if constexpr (LOC == LOC_RWU && TGT == TGT_ISO) {
        if (lp == -INFINITY) return 0.0f;
        const float lq = GmmIsoInflow<D>::log_inflow(P, a.n_comp, y) - a.log_c;
        const float M = fmaxf(lu, lq);
        const float v = expf(lu - M) + expf(lq - M) - expf((lp - a.log_c) - M);
        return v >= 0.0f ? M + logf(v) : NAN;
    } else {
        (void)P; (void)lp;
        return lu;
    }
}

template <int D, int MU, int NC, class RT = const_fptr>
__device__ __forceinline__ void sample_mu(const StepArgs &a, float u_cat, const float cand[NC], float y[D],
                                          RT R = RT()) {
    if constexpr (MU == MU_GMM) {
        MuGmm<D>::template sample<const_fptr, NC, RT>((const_fptr)a.mu_params, a.mu_params, a.mu_comp, u_cat, cand,
                                                      y, R);
    } else {
        (void)a; (void)u_cat; (void)R;
#pragma unroll
        for (int i = 0; i < D; ++i) y[i] = cand[i];
    }
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
    unsigned long long splat_fx;   // the same in fixed point (image_fx runs)
    // binned splats: the record this step closed (pixel -1: none)
    int32_t out_pix;
    float out_acc;
    // first pixel of this chain's batch image
    int32_t img_base;
    // tile-stratified runs: the chain's tile (first pixel column and row,
    // width and height in pixels)
    int32_t tpx0, tpy0, tw, th;
};

__device__ __forceinline__ void flush_splat(const StepArgs &a, int32_t pix, float acc, unsigned long long fx) {
    if (pix < 0) return;
    if (a.image_fx) atomicAdd(a.image_fx + pix, fx);
    else atomicAdd(a.image + pix, acc);
}

// A holding time in units of 2^-32 (dt < 2^5, so below 2^37): integer sums
// of these are exact, hence independent of the order of the atomics.
__device__ __forceinline__ unsigned long long dt_fixed(float dt) {
    return (unsigned long long)__float2ull_rn(dt * 0x1p32f);
}

// image index of a tile-local splat index (row stride tile_px); -1 stays -1
__device__ __forceinline__ int32_t tile_to_image(const StepArgs &a, int32_t px0, int32_t py0, int32_t base,
                                                 int32_t local) {
    if (local < 0) return -1;
    const int32_t ly = local / a.tile_px;
    return base + (py0 + ly) * a.image_w + px0 + (local - ly * a.tile_px);
}

// Tile-stratified runs: chain c of C works on tile t = floor(c T / C) (tiles
// row by row); the chains of tile t are [ceil(t C / T), ceil((t + 1) C / T)).
struct TileOf {
    int32_t px0, py0, w, h;
    int64_t first, count;   // the tile's chain range
};
__device__ __forceinline__ TileOf tile_of_chain(const StepArgs &a, int64_t c) {
    const int64_t T = a.n_tiles, C = a.n_chains;
    const int64_t t = c * T / C;
    TileOf r;
    r.first = (t * C + T - 1) / T;
    r.count = ((t + 1) * C + T - 1) / T - r.first;
    r.px0 = (int32_t)(t % a.tiles_x) * a.tile_px;
    r.py0 = (int32_t)(t / a.tiles_x) * a.tile_px;
    r.w = min(a.tile_px, a.image_w - r.px0);
    r.h = min(a.tile_px, a.image_h - r.py0);
    return r;
}

// a chain's tile and the first pixel of its batch image in tile-stratified
// runs: the batch images split each tile's chains (local index c') into
// image_batches ranges, c' in floor(c' B / C_t)
struct TileSlot {
    int32_t px0, py0, w, h, img_base;
};
__device__ __forceinline__ TileSlot tile_slot(const StepArgs &a, int64_t c) {
    const TileOf t = tile_of_chain(a, c);
    TileSlot r;
    r.px0 = t.px0;
    r.py0 = t.py0;
    r.w = t.w;
    r.h = t.h;
    r.img_base = a.image_batches > 1 ? (int32_t)((c - t.first) * a.image_batches / t.count) * a.image_pixels : 0;
    return r;
}

// pixel column and row of (x0, x1) as the splats compute them; false off
// the box
__device__ __forceinline__ bool pixel_of(const StepArgs &a, float u0, float u1, int &px, int &py) {
    if (!(u0 >= 0.0f && u0 <= 1.0f && u1 >= 0.0f && u1 <= 1.0f)) return false;
    px = min(max((int)(u0 * (float)a.image_w), 0), a.image_w - 1);
    py = min(max((int)(u1 * (float)a.image_h), 0), a.image_h - 1);
    return true;
}

// is y in the tile (px0, py0, w, h)?
__device__ __forceinline__ bool in_tile(const StepArgs &a, const float *y, int32_t px0, int32_t py0, int32_t w,
                                        int32_t h) {
    int px, py;
    return pixel_of(a, y[0], y[1], px, py) && px >= px0 && px < px0 + w && py >= py0 && py < py0 + h;
}

// the tile-uniform mu: (x0, x1) = ((px0 + w u0) / W, (py0 + h u1) / H) in
// float32 (one fused multiply-add and a correctly rounded division each)
__device__ __forceinline__ void tile_sample(const StepArgs &a, int32_t px0, int32_t py0, int32_t w, int32_t h,
                                            const float *cand, float *y) {
    y[0] = __fdiv_rn(fmaf((float)w, cand[0], (float)px0), (float)a.image_w);
    y[1] = __fdiv_rn(fmaf((float)h, cand[1], (float)py0), (float)a.image_h);
}

template <int D, int LOC>
__device__ __forceinline__ void load_chain(const StepArgs &a, uint32_t c, Chain<D, LOC> &ch) {
    const int64_t C = a.n_chains;
#pragma unroll
    for (int i = 0; i < D; ++i) ch.x[i] = a.x[i * C + c];
    if (uses_grad(LOC)) {
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
    ch.splat_fx = 0ull;
    ch.out_pix = -1;
    ch.out_acc = 0.0f;
    ch.tpx0 = ch.tpy0 = ch.tw = ch.th = 0;
    if (a.tile_px > 0) {
        const TileSlot t = tile_slot(a, c);
        ch.tpx0 = t.px0;
        ch.tpy0 = t.py0;
        ch.tw = t.w;
        ch.th = t.h;
        ch.img_base = t.img_base;
        return;
    }
    // chains are split into image_batches contiguous ranges: c in batch
    // floor(c batches / C)
    ch.img_base = a.image_batches > 1
                      ? (int32_t)((int64_t)c * a.image_batches / a.n_chains) * a.image_pixels
                      : 0;
}

template <int D, int LOC>
__device__ __forceinline__ void store_chain(const StepArgs &a, uint32_t c, const Chain<D, LOC> &ch) {
    const int64_t C = a.n_chains;
#pragma unroll
    for (int i = 0; i < D; ++i) a.x[i * C + c] = ch.x[i];
    if (uses_grad(LOC)) {
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

// The state-independent random inputs of one step of one chain, as a
// pre-pass computes them for small populations (uniform mu): the holding
// and termination exponentials t1 = -ln u_E1 and e2 = -ln u_E2, ln u_acc,
// the candidate uniforms (the regeneration's state) and their Box-Muller
// normals (the local move's noise).  The same device code computes them
// inline otherwise, so both paths give the same chains bit for bit.
template <int D>
struct StepRand {
    float t1, e2, lacc;
    float cand[D];
    float z[D];
};

// One transition of Alg. 2 for one lane.  Returns kill / accept through the
// flags.  In the drain (RETIRE) a terminated chain is not regenerated.
// With BIN, a splat closed by this step is returned in ch.out_pix /
// ch.out_acc instead of being added to the image.
//
// With MH the lane runs the Metropolis-Hastings reference chain M^l instead
// (Sec. 5, eq. (mixture-proposal-kernel); Sec. 8): no killing clock; with
// probability l (its own uniform, purpose LARGE) the update proposes y ~ mu
// and accepts with the independence ratio p(y) u(x) / (p(x) u(y)) (the
// large-step kernel K_1 of Theorem B in the supplement), otherwise it is the
// small-step update; dt f(x_{i-1}) goes straight to the float64 chain sums,
// as the chain has no tours.  ST_LAST_LARGE reports the large-step choice.
template <int D, int TGT, int LOC, int MU, bool RETIRE, class PT, bool BIN = false, bool MH = false,
          bool TILED = false, bool PRE = false, class RT = const_fptr>
__device__ __forceinline__ void step_once(const StepArgs &a, PT P, uint32_t s,
                                          uint32_t chain, Chain<D, LOC> &ch, bool &kill, bool &accept,
                                          const StepRand<D> *pr = nullptr, RT mu_r = RT()) {
    static_assert(!PRE || (MU == MU_UNIFORM && !MH && !TILED), "precomputed inputs: uniform mu, restore only");
    constexpr int NB = NBlocks<D>::value;
    if constexpr (std::is_same<PT, const_fptr>::value) {
        // keep the scalar parameter loads inside the step: hoisted out of the
        // step loop, a large slab overflows the SGPRs and spills to VGPR lanes
        uint64_t pv = (uint64_t)P;
        asm volatile("" : "+s"(pv));
        P = (PT)pv;
    }
    // per-step copies of the launch's scalars: the Philox key schedule, the
    // target's counter word and the flags are then recomputed every step on
    // the scalar unit; hoisted out of the step loop they outlive the
    // density's parameter loads, spill to VGPR lanes and every step reads
    // them back with VALU instructions.  (The Metropolis-Hastings chain's
    // kernels and the image integrand's schedule better with the hoisted
    // values: measured.)
    uint32_t k0 = a.key0, k1 = a.key1, tid = a.target_id;
    int32_t no_kill = a.no_kill, rb_dt = a.rb_dt, f_p = a.integrand_p;
    if constexpr (!MH && TGT != TGT_PSS) asm volatile("" : "+s"(k0), "+s"(k1), "+s"(tid), "+s"(no_kill), "+s"(rb_dt), "+s"(f_p));
    float head[4], cand[4 * NB];
    float t1, e2;
    if constexpr (PRE) {
        t1 = pr->t1;
        e2 = pr->e2;
    } else {
        draw_step<NB>(s, a.chain0 + chain, tid, PURPOSE_STEP, k0, k1, head, cand);
        // the two exponential clocks
        t1 = -ln_u01(head[0]);
        e2 = -ln_u01(head[1]);
    }
    float t2 = INFINITY;
    float inv_k = INFINITY;
    kill = false;
    if (!MH && !no_kill) {
        // t2 = E2 / k = E2 exp(log p - log u - ln c_tilde); p = 0 gives t2 = 0
        // (hardware 2^x: |x| 2^-24 relative, far inside the decision margins)
        inv_k = exp_rel(ch.lp - ch.lu - a.log_c);
        t2 = e2 * inv_k;
        kill = !(t1 < t2);
    }
    // the holding time dt = min(t1, t2) ~ Exp(1 + k) whichever clock fires;
    // with rb_dt its conditional mean 1 / (1 + k) is accumulated instead
    float dt = kill ? t2 : t1;
    if (rb_dt) dt = inv_k > 1e30f ? 1.0f : inv_k / (1.0f + inv_k);

    bool large = false;
    if constexpr (MH) {
        if (a.large_prob > 0.0f) {
            uint32_t r[4];
            Philox::block(s, a.chain0 + chain, tid, PURPOSE_LARGE << 16, k0, k1, r);
            large = u01(r[0]) < a.large_prob;
        }
        ch.status = large ? (ch.status | ST_LAST_LARGE) : (ch.status & ~ST_LAST_LARGE);
        // no tours: dt f(x_{i-1}) goes to the chain sums
        ch.t_done += (double)dt;
        if (f_p) ch.a_done = fma((double)dt, (double)exp_rel(ch.lp), ch.a_done);
    } else {
        // accumulate dt f(x_{i-1}) into the tour in flight
        ch.t_cur += dt;
        if (f_p) ch.a_cur = fmaf(dt, exp_rel(ch.lp), ch.a_cur);
    }
    if (TGT == TGT_PSS && a.image) {
        // f = 1_pixel(x0, x1) at the pre-transition state (p = 0 off the box)
        int32_t pix = -1;
        int px, py;
        if (pixel_of(a, ch.x[0], ch.x[1], px, py)) {
            if constexpr (TILED) {
                // the index within the chain's tile (row stride tile_px);
                // a state outside the tile has p = 0 and dt = 0: no splat
                const int lx = px - ch.tpx0, ly = py - ch.tpy0;
                pix = (lx >= 0 && lx < ch.tw && ly >= 0 && ly < ch.th) ? ly * a.tile_px + lx : -1;
            } else {
                pix = ch.img_base + py * a.image_w + px;
            }
        }
        if (BIN) ch.out_pix = -1;
        if (pix != ch.splat_pix) {
            if (BIN) {
                ch.out_pix = ch.splat_pix;
                ch.out_acc = ch.splat_acc;
            } else {
                flush_splat(a, TILED ? tile_to_image(a, ch.tpx0, ch.tpy0, ch.img_base, ch.splat_pix) : ch.splat_pix,
                            ch.splat_acc, ch.splat_fx);
            }
            ch.splat_pix = pix;
            ch.splat_acc = 0.0f;
            ch.splat_fx = 0ull;
        }
        if (a.image_fx) ch.splat_fx += dt_fixed(dt);
        else ch.splat_acc += dt;
    }
    ch.last_dt = dt;
    // random-walk kinds with precomputed inputs run branch-free (selects):
    // the same arithmetic, fewer exec-mask switches on the serial step path
    constexpr bool FLAT = PRE && !uses_grad(LOC) && LOC != LOC_HMC;
    if constexpr (FLAT) {
        ch.a_done += kill ? (double)ch.a_cur : 0.0;
        ch.t_done += kill ? (double)ch.t_cur : 0.0;
        ch.n_done += kill ? 1u : 0u;
        ch.a_cur = kill ? 0.0f : ch.a_cur;
        ch.t_cur = kill ? 0.0f : ch.t_cur;
    } else if (kill) {
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

    // candidate: mu sample if killed (or a large step), small-step proposal
    // otherwise.  A regenerated chain gets its gradient only when it first
    // survives a step, so waves whose lanes were all killed skip that work.
    float y[D];
    float zz = 0.0f;
    const float h = 0.5f * a.step * a.step;
    float rho[D];          // HMC: momentum before the closing half step
    bool inside = true;    // HMC: every leapfrog point has p > 0
    if constexpr (FLAT) {
        // regeneration: the candidate uniforms; local move: x + step z
#pragma unroll
        for (int i = 0; i < D; ++i) y[i] = kill ? pr->cand[i] : fmaf(a.step, pr->z[i], ch.x[i]);
    } else if (kill || large) {
        if constexpr (PRE) {
#pragma unroll
            for (int i = 0; i < D; ++i) y[i] = pr->cand[i];
        } else {
            sample_mu<D, MU, 4 * NB, RT>(a, head[3], cand, y, mu_r);
            if constexpr (TILED) tile_sample(a, ch.tpx0, ch.tpy0, ch.tw, ch.th, cand, y);
        }
    } else {
        if (uses_grad(LOC) && !(ch.status & ST_GRAD_VALID)) {
            (void)log_target<D, TGT, true, DensityBlock<LOC>::value>(P, a.n_comp, ch.x, ch.g);
            ch.status |= ST_GRAD_VALID;
        }
        float z[D];
        if constexpr (PRE) {
#pragma unroll
            for (int i = 0; i < D; ++i) z[i] = pr->z[i];
        } else {
            box_muller<D, 4 * NB>(cand, z);
        }
        if constexpr (LOC == LOC_HMC) {
            // leapfrog with unit mass from (x, rho_0 = z): half a momentum
            // step, n position steps separated by full momentum steps; the
            // closing half step uses grad log p(y) of the final evaluation
            const float e = a.step;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                zz = fmaf(z[i], z[i], zz);
                rho[i] = fmaf(0.5f * e, ch.g[i], z[i]);
                y[i] = ch.x[i];
            }
            for (int l = 1; l < a.n_leapfrog; ++l) {
                float gq[D];
#pragma unroll
                for (int i = 0; i < D; ++i) y[i] = fmaf(e, rho[i], y[i]);
                const float lq = log_target<D, TGT, true, DensityBlock<LOC>::value>(P, a.n_comp, y, gq);
                inside = inside && lq > -INFINITY;
#pragma unroll
                for (int i = 0; i < D; ++i) rho[i] = fmaf(e, gq[i], rho[i]);
            }
#pragma unroll
            for (int i = 0; i < D; ++i) y[i] = fmaf(e, rho[i], y[i]);
        } else {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                if (LOC == LOC_MALA) {
                    const float delta = fmaf(h, ch.g[i], a.step * z[i]);
                    zz = fmaf(z[i], z[i], zz);
                    y[i] = ch.x[i] + delta;
                } else {
                    y[i] = fmaf(a.step, z[i], ch.x[i]);
                }
            }
        }
    }

    float gy[D];
    float lpy = log_target<D, TGT, uses_grad(LOC), DensityBlock<LOC>::value>(P, a.n_comp, y, gy, !kill);
    if constexpr (TILED) {
        // the chain's target is p restricted to its tile
        if (!in_tile(a, y, ch.tpx0, ch.tpy0, ch.tw, ch.th)) lpy = -INFINITY;
    }
    const float luy = (MH && large) ? log_mu<D, MU>(a, y, mu_r) : log_u_state<D, TGT, LOC, MU>(a, P, y, lpy, mu_r);

    accept = false;
    if (!kill) {
        if (ch.lp == -INFINITY || LOC == LOC_RWU) {
            accept = true;  // alpha = 1 where p(x) q(x, y) = 0; the unadjusted jump is always taken
        } else {
            float lr = lpy - ch.lp;
            if (MH && large) {
                // independence proposal: q(x, y) = u(y)
                lr += ch.lu - luy;
            } else if (LOC == LOC_MALA) {
                // ln q(x->y) = -|z|^2 / 2 ;  ln q(y->x) = -|x - y - h g(y)|^2 / (2 eps^2);
                // x - y is exact in float32 for neighbouring states (Sterbenz)
                float rr = 0.0f;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const float r = fmaf(-h, gy[i], ch.x[i] - y[i]);
                    rr = fmaf(r, r, rr);
                }
                lr += 0.5f * zz - rr / (2.0f * a.step * a.step);
            } else if (LOC == LOC_HMC) {
                // H = -log p + |rho|^2 / 2; the leapfrog map is volume-
                // preserving and reversible, so alpha = exp(-dH)
                float kk = 0.0f;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const float r = fmaf(0.5f * a.step, gy[i], rho[i]);
                    kk = fmaf(r, r, kk);
                }
                lr = inside ? lr + 0.5f * (zz - kk) : -INFINITY;
            }
            if constexpr (PRE) {
                accept = pr->lacc < lr;
            } else {
                accept = ln_u01(head[2]) < lr;
            }
        }
    }
    if constexpr (FLAT) {
        const bool take = kill || accept;
#pragma unroll
        for (int i = 0; i < D; ++i) ch.x[i] = take ? y[i] : ch.x[i];
        ch.lp = take ? lpy : ch.lp;
        ch.lu = take ? luy : ch.lu;
    } else if (kill || accept) {
#pragma unroll
        for (int i = 0; i < D; ++i) ch.x[i] = y[i];
        if (uses_grad(LOC)) {
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
                                             unsigned long long acc, unsigned long long kil,
                                             unsigned long long large = 0, unsigned long long large_acc = 0) {
    // one lane per wave publishes the wave's ballot counts
    const unsigned long long active = __ballot(1);
    if ((unsigned)lane_id() == (unsigned)(__ffsll((long long)active) - 1)) {
        unsigned long long *line = counters + (size_t)(blockIdx.x % CNT_SPREAD) * CNT_LINE;
        atomicAdd(line + CNT_TRANSITIONS, t);
        atomicAdd(line + CNT_ACCEPTS, acc);
        atomicAdd(line + CNT_KILLS, kil);
        if (large) atomicAdd(line + CNT_LARGE, large);
        if (large_acc) atomicAdd(line + CNT_LARGE_ACCEPTS, large_acc);
    }
}

}  // namespace restore
