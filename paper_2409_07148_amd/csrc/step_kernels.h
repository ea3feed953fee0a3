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
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "chain_step.h"
#include "launch.h"

namespace restore {

// Steps with regeneration for every chain.  With MH: steps of the
// Metropolis-Hastings reference chain M^l (no killing, large steps from mu
// with probability l; see step_once).
template <int D, int TGT, int LOC, int MU, bool LDS, bool MH = false>
__global__ __launch_bounds__(256) void step_kernel(StepArgs a, int n_param_floats) {
    extern __shared__ float smem[];
    const auto P = stage_params<LDS>(a.params, n_param_floats, smem);
    const auto MR = stage_mu<D, MU>(a, smem + mu_lds_offset(LDS, n_param_floats));
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_chains) return;
    Chain<D, LOC> ch;
    load_chain(a, (uint32_t)c, ch);
    unsigned long long n_acc = 0, n_kill = 0, n_large = 0, n_large_acc = 0;
    bool kill = false, accept = false;
    const bool rec = a.rec_x != nullptr && c < a.rec_chains;
    for (int it = 0; it < a.n_steps; ++it) {
        if (rec) {
            float *xo = a.rec_x + ((int64_t)it * a.rec_chains + c) * D;
#pragma unroll
            for (int i = 0; i < D; ++i) xo[i] = ch.x[i];
        }
        step_once<D, TGT, LOC, MU, false, decltype(P), false, MH, false, false, decltype(MR)>(
            a, P, a.s0 + (uint32_t)it, (uint32_t)c, ch, kill, accept, nullptr, MR);
        if (rec) a.rec_w[(int64_t)it * a.rec_chains + c] = ch.last_dt;
        n_acc += __popcll(__ballot(accept));
        n_kill += __popcll(__ballot(kill));
        if constexpr (MH) {
            const bool large = (ch.status & ST_LAST_LARGE) != 0u;
            n_large += __popcll(__ballot(large));
            n_large_acc += __popcll(__ballot(large && accept));
        }
    }
    ch.status = (ch.status & ~(ST_LAST_KILL | ST_LAST_ACCEPT)) | (kill ? ST_LAST_KILL : 0u) |
                (accept ? ST_LAST_ACCEPT : 0u);
    if (TGT == TGT_PSS && a.image) flush_splat(a, ch.splat_pix, ch.splat_acc, ch.splat_fx);
    store_chain(a, (uint32_t)c, ch);
    const unsigned long long lanes = __popcll(__ballot(1));
    add_counters(a.counters, lanes * (unsigned long long)a.n_steps, n_acc, n_kill, n_large, n_large_acc);
}

// Pre-pass of a chunk of steps for a small population (uniform mu): thread
// (chain c, step j of the chunk) draws step s0 + j of chain c and writes its
// StepRand fields to out[f][j][c] (field f of rand_fields(D); a field is
// chunk x C floats).  Chip-wide, so the Philox blocks and the
// transcendental mappings of every step run on all compute units instead of
// on the few waves of the population's serial step loop.
template <int D>
__device__ __forceinline__ void prepass_one(const StepArgs &a, uint32_t s0, int64_t c, int j, float *out,
                                            int chunk) {
    constexpr int NB = NBlocks<D>::value;
    float head[4], cand[4 * NB];
    draw_step<NB>(s0 + (uint32_t)j, a.chain0 + (uint32_t)c, a.target_id, PURPOSE_STEP, a.key0, a.key1, head, cand);
    const int64_t C = a.n_chains, fs = (int64_t)chunk * C;
    float *o = out + (int64_t)j * C + c;
    o[0] = -ln_u01(head[0]);
    o[fs] = -ln_u01(head[1]);
    o[2 * fs] = ln_u01(head[2]);
    float z[D];
    box_muller<D, 4 * NB>(cand, z);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        o[(3 + i) * fs] = cand[i];
        o[(3 + D + i) * fs] = z[i];
    }
}

template <int D>
__global__ __launch_bounds__(256) void rand_prepass_kernel(StepArgs a, float *out, int chunk) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (c >= a.n_chains || j >= a.n_steps) return;
    prepass_one<D>(a, a.s0, c, j, out, chunk);
}

// The pre-pass of the following chunk, run by extra workgroups of a step
// launch (on the compute units its few step waves leave idle): workgroup
// step_blocks + g covers the threads' chains for PRE_GEN_STEPS steps.
template <int D>
__device__ __forceinline__ void pregen_block(const StepArgs &a, const PreGen &g, int chunk) {
    const int64_t cb = ((int64_t)a.n_chains + blockDim.x - 1) / blockDim.x;
    const int64_t gb = (int64_t)blockIdx.x - g.step_blocks;
    const int64_t c = (gb % cb) * blockDim.x + threadIdx.x;
    const int j0 = (int)(gb / cb) * PRE_GEN_STEPS;
    if (c >= a.n_chains) return;
    const int j1 = min(j0 + PRE_GEN_STEPS, g.n_steps);
    for (int j = j0; j < j1; ++j) prepass_one<D>(a, g.s0, c, j, g.out, chunk);
}

// Register double buffer of precomputed step inputs: PF steps per buffer,
// loaded from pre (chunk stride) one buffer ahead of the steps that use it.
// The loads are unconditional (a step past `last` re-reads step `last`,
// which the buffer holds): straight-line code, so the compiler waits for
// the older buffer only (a count of outstanding loads) instead of for
// every load in flight.
template <int D>
struct PreFetch {
    static constexpr int F = rand_fields(D);
    static constexpr int PF = F <= 8 ? 4 : (F <= 16 ? 2 : 1);
    const char *pb;
    uint32_t C4, fs4, lane4;
    int last;
    __device__ __forceinline__ PreFetch(const float *pre, int64_t n_chains, int chunk, int64_t c, int last_)
        : pb(reinterpret_cast<const char *>(pre)), C4(4u * (uint32_t)n_chains),
          fs4((uint32_t)chunk * 4u * (uint32_t)n_chains), lane4(4u * (uint32_t)c), last(last_) {}
    __device__ __forceinline__ float ld(uint32_t off) const { return *reinterpret_cast<const float *>(pb + off); }
    __device__ __forceinline__ void fetch(StepRand<D> &r, int it) const {
        const uint32_t o = (uint32_t)it * C4 + lane4;
        r.t1 = ld(o);
        r.e2 = ld(o + fs4);
        r.lacc = ld(o + 2 * fs4);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            r.cand[i] = ld(o + (3 + i) * fs4);
            r.z[i] = ld(o + (3 + D + i) * fs4);
        }
    }
    __device__ __forceinline__ void load(StepRand<D> (&r)[PF], int it0) const {
#pragma unroll
        for (int j = 0; j < PF; ++j) fetch(r[j], min(it0 + j, last));
    }
};

// Steps with regeneration whose random inputs come from the pre-pass (a
// chunk of at most `chunk` steps; step it of the launch reads field f at
// pre[(f chunk + it) C + c]).  Two register buffers of PF steps alternate:
// one is loaded while the other's steps run.  The same chains as
// step_kernel, bit for bit.
template <int D, int TGT, int LOC>
__global__ __launch_bounds__(256) void step_pre_kernel(StepArgs a, const float *pre, int chunk, PreGen g) {
    if ((int64_t)blockIdx.x >= g.step_blocks) {
        pregen_block<D>(a, g, chunk);
        return;
    }
    using PFT = PreFetch<D>;
    constexpr int PF = PFT::PF;
    const const_fptr P = (const_fptr)a.params;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_chains) return;
    Chain<D, LOC> ch;
    load_chain(a, (uint32_t)c, ch);
    // the buffer base is wave-uniform and every byte offset fits in 32 bits
    // (at most 32 MiB per half), so the loads take the scalar-base mode
    const PFT pf(pre, a.n_chains, chunk, c, a.n_steps - 1);
    unsigned long long n_acc = 0, n_kill = 0;
    bool kill = false, accept = false;
    auto run = [&](const StepRand<D> (&r)[PF], int it0) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            if (it0 + j < a.n_steps) {
                step_once<D, TGT, LOC, MU_UNIFORM, false, const_fptr, false, false, false, true>(
                    a, P, a.s0 + (uint32_t)(it0 + j), (uint32_t)c, ch, kill, accept, &r[j]);
                n_acc += __popcll(__ballot(accept));
                n_kill += __popcll(__ballot(kill));
            }
        }
    };
    StepRand<D> A[PF], B[PF];
    pf.load(A, 0);
    for (int it0 = 0; it0 < a.n_steps; it0 += 2 * PF) {
        pf.load(B, it0 + PF);
        run(A, it0);
        pf.load(A, it0 + 2 * PF);
        run(B, it0 + PF);
    }
    ch.status = (ch.status & ~(ST_LAST_KILL | ST_LAST_ACCEPT)) | (kill ? ST_LAST_KILL : 0u) |
                (accept ? ST_LAST_ACCEPT : 0u);
    store_chain(a, (uint32_t)c, ch);
    const unsigned long long lanes = __popcll(__ballot(1));
    add_counters(a.counters, lanes * (unsigned long long)a.n_steps, n_acc, n_kill);
}

// The drain of a small population in one launch (no chain list): the first
// n_pre steps take their random inputs from the pre-pass, later ones draw
// them inline.  A wave ends when its last lane's tour is killed; survivors
// of all a.n_steps steps are censored.  The same chains as drain_kernel.
template <int D, int TGT, int LOC>
__global__ __launch_bounds__(256) void drain_pre_kernel(StepArgs a, const float *pre, int chunk, int n_pre) {
    using PFT = PreFetch<D>;
    constexpr int PF = PFT::PF;
    const const_fptr P = (const_fptr)a.params;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_chains) return;
    Chain<D, LOC> ch;
    load_chain(a, (uint32_t)c, ch);
    bool alive = (ch.status & ST_ALIVE) != 0u;
    unsigned long long n_t = 0, n_acc = 0, n_kill = 0;
    bool stepped = false, kill_last = false, acc_last = false;
    // one drain step; false once no lane of the wave is alive
    auto step = [&](int it, const StepRand<D> *r) {
        const unsigned long long live = __ballot(alive);
        if (live == 0ull) return false;
        n_t += __popcll(live);
        bool kill = false, accept = false;
        if (alive) {
            if (r)
                step_once<D, TGT, LOC, MU_UNIFORM, true, const_fptr, false, false, false, true>(
                    a, P, a.s0 + (uint32_t)it, (uint32_t)c, ch, kill, accept, r);
            else
                step_once<D, TGT, LOC, MU_UNIFORM, true, const_fptr>(a, P, a.s0 + (uint32_t)it, (uint32_t)c, ch,
                                                                     kill, accept);
            stepped = true;
            kill_last = kill;
            acc_last = accept;
            alive = !kill;
        }
        n_acc += __popcll(__ballot(accept));
        n_kill += __popcll(__ballot(kill));
        return true;
    };
    n_pre = min(n_pre, a.n_steps);
    bool more = true;
    int it = 0;
    if (n_pre > 0) {
        const PFT pf(pre, a.n_chains, chunk, c, n_pre - 1);
        auto run = [&](const StepRand<D> (&r)[PF], int it0) {
#pragma unroll
            for (int j = 0; j < PF; ++j)
                if (more && it0 + j < n_pre) more = step(it0 + j, &r[j]);
        };
        StepRand<D> A[PF], B[PF];
        pf.load(A, 0);
        for (int it0 = 0; more && it0 < n_pre; it0 += 2 * PF) {
            pf.load(B, it0 + PF);
            run(A, it0);
            pf.load(A, it0 + 2 * PF);
            run(B, it0 + PF);
        }
        it = n_pre;
    }
    for (; more && it < a.n_steps; ++it) more = step(it, nullptr);
    if (stepped) {
        ch.status = (ch.status & ~(ST_LAST_KILL | ST_LAST_ACCEPT | ST_ALIVE)) | (alive ? ST_ALIVE : 0u) |
                    (kill_last ? ST_LAST_KILL : 0u) | (acc_last ? ST_LAST_ACCEPT : 0u);
    }
    if (alive) ch.status |= ST_CENSORED;
    store_chain(a, (uint32_t)c, ch);
    add_counters(a.counters, n_t, n_acc, n_kill);
}

// Binning of the records staged in LDS: rows [0, rows) of this thread's
// column.  Counts per band (LDS atomics), one global reservation per band
// and workgroup, then each record goes to its band's bucket at the reserved
// base plus its rank (or straight to the image if the bucket is full).
// Every thread of the workgroup calls it the same number of times.
__device__ __forceinline__ void splat_flush(const StepArgs &a, uint32_t (*rp)[256], float (*rv)[256], uint32_t *cnt,
                                            uint32_t *base, int rows) {
    const int t = threadIdx.x;
    __syncthreads();
    for (int r = 0; r < rows; ++r) {
        const uint32_t p = rp[r][t];
        if (p != SPLAT_NO_PIX) atomicAdd(&cnt[p >> SPLAT_BAND_SHIFT], 1u);
    }
    __syncthreads();
    for (int b = t; b < a.n_bins; b += blockDim.x) {
        const uint32_t k = cnt[b];
        base[b] = k ? atomicAdd(a.bin_count + b * SPLAT_COUNTER_STRIDE, k) : 0u;
        cnt[b] = 0u;
    }
    __syncthreads();
    for (int r = 0; r < rows; ++r) {
        const uint32_t p = rp[r][t];
        if (p != SPLAT_NO_PIX) {
            const uint32_t b = p >> SPLAT_BAND_SHIFT;
            const uint32_t pos = base[b] + atomicAdd(&cnt[b], 1u);
            const float v = rv[r][t];
            if (pos < (uint32_t)a.bin_cap) {
                const size_t o = (size_t)b * (size_t)a.bin_cap + pos;
                a.bin_pix[o] = p;
                a.bin_val[o] = v;
            } else {
                atomicAdd(a.image + p, v);
            }
        }
    }
    __syncthreads();
    for (int b = t; b < a.n_bins; b += blockDim.x) cnt[b] = 0u;
}

// Steps with regeneration for the image integrand, with binned splats.
// Every lane stages the record (pixel, dt) its step closed, if any, in its
// LDS column; every SPLAT_ROWS steps, and once more at the end with the
// splat still open, the workgroup bins its records (splat_flush).  Lanes
// past the last chain take part in the barriers only.
template <int D, int TGT, int LOC, int MU, bool LDS>
__global__ __launch_bounds__(256) void step_binned_kernel(StepArgs a, int n_param_floats) {
    extern __shared__ float smem[];
    __shared__ uint32_t rec_pix[SPLAT_ROWS + 1][256];
    __shared__ float rec_val[SPLAT_ROWS + 1][256];
    __shared__ uint32_t cnt[SPLAT_MAX_BANDS], base[SPLAT_MAX_BANDS];
    const auto P = stage_params<LDS>(a.params, n_param_floats, smem);
    const auto MR = stage_mu<D, MU>(a, smem + mu_lds_offset(LDS, n_param_floats));
    const int t = threadIdx.x;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + t;
    const bool active = c < a.n_chains;
    for (int b = t; b < SPLAT_MAX_BANDS; b += blockDim.x) cnt[b] = 0u;
    Chain<D, LOC> ch;
    if (active) load_chain(a, (uint32_t)c, ch);
    unsigned long long n_acc = 0, n_kill = 0;
    bool kill = false, accept = false;
    const bool rec = active && a.rec_x != nullptr && c < a.rec_chains;
    int row = 0;
    for (int it = 0; it < a.n_steps; ++it) {
        uint32_t rp = SPLAT_NO_PIX;
        float rv = 0.0f;
        if (active) {
            if (rec) {
                float *xo = a.rec_x + ((int64_t)it * a.rec_chains + c) * D;
#pragma unroll
                for (int i = 0; i < D; ++i) xo[i] = ch.x[i];
            }
            step_once<D, TGT, LOC, MU, false, decltype(P), true, false, false, false, decltype(MR)>(
                a, P, a.s0 + (uint32_t)it, (uint32_t)c, ch, kill, accept, nullptr, MR);
            if (rec) a.rec_w[(int64_t)it * a.rec_chains + c] = ch.last_dt;
            if (ch.out_pix >= 0) {
                rp = (uint32_t)ch.out_pix;
                rv = ch.out_acc;
            }
        }
        rec_pix[row][t] = rp;
        rec_val[row][t] = rv;
        n_acc += __popcll(__ballot(accept));
        n_kill += __popcll(__ballot(kill));
        if (++row == SPLAT_ROWS) {
            splat_flush(a, rec_pix, rec_val, cnt, base, SPLAT_ROWS);
            row = 0;
        }
    }
    // the splat still open at the end of the launch
    rec_pix[row][t] = (active && ch.splat_pix >= 0) ? (uint32_t)ch.splat_pix : SPLAT_NO_PIX;
    rec_val[row][t] = active ? ch.splat_acc : 0.0f;
    splat_flush(a, rec_pix, rec_val, cnt, base, row + 1);
    if (active) {
        ch.status = (ch.status & ~(ST_LAST_KILL | ST_LAST_ACCEPT)) | (kill ? ST_LAST_KILL : 0u) |
                    (accept ? ST_LAST_ACCEPT : 0u);
        store_chain(a, (uint32_t)c, ch);
    }
    const unsigned long long lanes = __popcll(__ballot(active));
    if (lanes) add_counters(a.counters, lanes * (unsigned long long)a.n_steps, n_acc, n_kill);
}

// Steps with regeneration of tile-stratified runs (the image integrand):
// chain c works on its own tile (p restricted to the tile, mu uniform on
// it).  The workgroup accumulates the splats of its lanes that share the
// (tile, batch image) of its first chain in an LDS copy of that tile (LDS
// float atomics), and adds the copy to the image at the end of the launch;
// other lanes (a workgroup that straddles two tiles or batches) add their
// splats to the image directly.  Lanes past the last chain take part in
// the barriers only.
template <int D, int TGT, int LOC, int MU>
__global__ __launch_bounds__(256) void step_tiled_kernel(StepArgs a, int n_param_floats) {
    extern __shared__ float acc[];   // [tile_px * tile_px]
    (void)n_param_floats;
    const auto P = (const_fptr)a.params;
    const int t = threadIdx.x;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + t;
    const bool active = c < a.n_chains;
    const int n_acc_px = a.tile_px * a.tile_px;
    for (int i = t; i < n_acc_px; i += blockDim.x) acc[i] = 0.0f;
    // the workgroup's tile and batch image: those of its first chain
    const TileSlot first = tile_slot(a, (int64_t)blockIdx.x * blockDim.x);
    __syncthreads();
    Chain<D, LOC> ch;
    unsigned long long n_acc = 0, n_kill = 0;
    bool kill = false, accept = false;
    if (active) {
        load_chain(a, (uint32_t)c, ch);
        const bool mine = ch.tpx0 == first.px0 && ch.tpy0 == first.py0 && ch.img_base == first.img_base;
        for (int it = 0; it < a.n_steps; ++it) {
            step_once<D, TGT, LOC, MU, false, const_fptr, true, false, true>(a, P, a.s0 + (uint32_t)it,
                                                                            (uint32_t)c, ch, kill, accept);
            if (ch.out_pix >= 0) {
                if (mine) atomicAdd(acc + ch.out_pix, ch.out_acc);
                else atomicAdd(a.image + tile_to_image(a, ch.tpx0, ch.tpy0, ch.img_base, ch.out_pix), ch.out_acc);
            }
            n_acc += __popcll(__ballot(accept));
            n_kill += __popcll(__ballot(kill));
        }
        // the splat still open at the end of the launch
        if (ch.splat_pix >= 0) {
            if (mine) atomicAdd(acc + ch.splat_pix, ch.splat_acc);
            else atomicAdd(a.image + tile_to_image(a, ch.tpx0, ch.tpy0, ch.img_base, ch.splat_pix), ch.splat_acc);
        }
        ch.status = (ch.status & ~(ST_LAST_KILL | ST_LAST_ACCEPT)) | (kill ? ST_LAST_KILL : 0u) |
                    (accept ? ST_LAST_ACCEPT : 0u);
        store_chain(a, (uint32_t)c, ch);
    }
    const unsigned long long lanes = __popcll(__ballot(active));
    if (lanes) add_counters(a.counters, lanes * (unsigned long long)a.n_steps, n_acc, n_kill);
    __syncthreads();
    // the tile copy into the image (zero entries skipped)
    for (int i = t; i < n_acc_px; i += blockDim.x) {
        const float v = acc[i];
        const int ly = i / a.tile_px, lx = i - ly * a.tile_px;
        if (v != 0.0f && lx < first.w && ly < first.h)
            atomicAdd(a.image + first.img_base + (first.py0 + ly) * a.image_w + first.px0 + lx, v);
    }
}

// Drain: the chains of the input list run on without regeneration until
// their tour in flight is killed.  Survivors of this chunk are compacted
// into the output list with one ballot and one atomic per wave; on the last
// chunk they are marked censored instead.
template <int D, int TGT, int LOC, int MU, bool LDS, bool TILED = false>
__global__ __launch_bounds__(256) void drain_kernel(StepArgs a, int n_param_floats, uint32_t *list_out,
                                                     uint32_t *count_out, uint32_t *count_zero,
                                                     int last_chunk) {
    extern __shared__ float smem[];
    const auto P = stage_params<LDS>(a.params, n_param_floats, smem);
    // (tile-stratified runs have the uniform mu)
    const auto MR = stage_mu<D, TILED ? MU_UNIFORM : MU>(a, smem + mu_lds_offset(LDS, n_param_floats));
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
            step_once<D, TGT, LOC, MU, true, decltype(P), false, false, TILED, false, decltype(MR)>(
                a, P, a.s0 + (uint32_t)it, c, ch, kill, accept, nullptr, MR);
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
    if (TGT == TGT_PSS && a.image)
        flush_splat(a, TILED ? tile_to_image(a, ch.tpx0, ch.tpy0, ch.img_base, ch.splat_pix) : ch.splat_pix,
                    ch.splat_acc, ch.splat_fx);
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
    draw_step<NB>(0u, a.chain0 + (uint32_t)c, a.target_id, PURPOSE_INIT, a.key0, a.key1, head, cand);
    Chain<D, LOC> ch;
    sample_mu<D, MU, 4 * NB>(a, head[3], cand, ch.x);
    TileOf tile{};
    if (TGT == TGT_PSS && a.tile_px > 0) {
        // tile-stratified: x_0 from the uniform mu of the chain's tile
        tile = tile_of_chain(a, c);
        tile_sample(a, tile.px0, tile.py0, tile.w, tile.h, cand, ch.x);
    }
    ch.lp = log_target<D, TGT, uses_grad(LOC)>((const_fptr)a.params, a.n_comp, ch.x, ch.g);
    if (TGT == TGT_PSS && a.tile_px > 0 && !in_tile(a, ch.x, tile.px0, tile.py0, tile.w, tile.h))
        ch.lp = -INFINITY;
    ch.lu = log_u_state<D, TGT, LOC, MU>(a, (const_fptr)a.params, ch.x, ch.lp);
    ch.a_cur = ch.t_cur = 0.0f;
    ch.a_done = ch.t_done = 0.0;
    ch.n_done = 0u;
    ch.status = ST_ALIVE | (uses_grad(LOC) ? ST_GRAD_VALID : 0u);
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
    float lp = log_target<D, TGT, uses_grad(LOC)>((const_fptr)a.params, a.n_comp, x, g);
    if (TGT == TGT_PSS && a.tile_px > 0) {
        const TileOf t = tile_of_chain(a, c);
        if (!in_tile(a, x, t.px0, t.py0, t.w, t.h)) lp = -INFINITY;
    }
    a.logp[c] = lp;
    a.logu[c] = log_u_state<D, TGT, LOC, MU>(a, (const_fptr)a.params, x, lp);
    if (uses_grad(LOC)) {
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
    k.step_mh = (const void *)step_kernel<D, TGT, LOC, MU, false, true>;
    k.drain = (const void *)drain_kernel<D, TGT, LOC, MU, false>;
    k.drain_lds = (const void *)drain_kernel<D, TGT, LOC, MU, true>;
    if constexpr (TGT != TGT_PSS && MU == MU_UNIFORM) {
        k.rand_prepass = (const void *)rand_prepass_kernel<D>;
        k.step_pre = (const void *)step_pre_kernel<D, TGT, LOC>;
        k.drain_pre = (const void *)drain_pre_kernel<D, TGT, LOC>;
    }
    if constexpr (TGT == TGT_PSS) {
        k.step_binned = (const void *)step_binned_kernel<D, TGT, LOC, MU, false>;
        k.step_binned_lds = (const void *)step_binned_kernel<D, TGT, LOC, MU, true>;
        k.step_tiled = (const void *)step_tiled_kernel<D, TGT, LOC, MU>;
        k.drain_tiled = (const void *)drain_kernel<D, TGT, LOC, MU, false, true>;
    }
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

}  // namespace restore
