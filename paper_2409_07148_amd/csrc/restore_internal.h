// Internal structures shared by the host runtime and the gfx950 kernels.
#pragma once

#include <stdint.h>

namespace restore {

enum TargetKind : int { TGT_ISO = 0, TGT_FULL = 1, TGT_PSS = 2 };
// LOC_RWU: the unadjusted random-walk jump process (every jump taken, not
// pi-invariant; its killing rate carries the adjoint generator term)
enum LocalKind : int { LOC_RWMH = 0, LOC_MALA = 1, LOC_HMC = 2, LOC_RWU = 3 };
// the local kernels that use grad log p (cached per chain in the state)
__host__ __device__ constexpr bool uses_grad(int loc) { return loc == LOC_MALA || loc == LOC_HMC; }
enum MuKind : int { MU_UNIFORM = 0, MU_GMM = 1 };
enum Purpose : uint32_t { PURPOSE_INIT = 0, PURPOSE_STEP = 1, PURPOSE_LARGE = 2 };

enum StatusBits : uint32_t {
    ST_ALIVE = 1u,       // tour in flight
    ST_CENSORED = 2u,    // tour still alive at the drain cap
    ST_LAST_KILL = 4u,   // last executed step was a termination
    ST_LAST_ACCEPT = 8u, // last executed step accepted a local move
    ST_GRAD_VALID = 16u, // the cached grad log p(x) belongs to x (MALA)
    ST_LAST_LARGE = 32u, // MH chain: the last step proposed a large step
};

enum CounterSlot : int {
    CNT_TRANSITIONS = 0, CNT_ACCEPTS = 1, CNT_KILLS = 2, CNT_LARGE = 3, CNT_LARGE_ACCEPTS = 4, CNT_SLOTS = 8
};
// The run counters are spread over CNT_SPREAD copies, one per 256-byte line
// (CNT_LINE 64-bit words apart), chosen by workgroup: the waves of a launch
// then add into many lines instead of queueing on one.  Readers sum the
// copies.
constexpr int CNT_SPREAD = 64;
constexpr int CNT_LINE = 32;

// Number of float32 values per mixture component in the packed slab.  The
// log-weights and quadratic forms are in base 2 (scaled by log2 e), and a
// log-weight of -inf (w_k = 0) is stored as -2^100:
//   ISO : [ c_k | m_k (d) | h_k ]       c_k = log2 e (ln w_k - d/2 ln(2 pi s_k^2)),
//                                       h_k = log2 e / (2 s_k^2)
//   FULL: [ c_k | m_k (d) | W_k lower-tri rows (d(d+1)/2) ]
//         W_k = sqrt(log2 e / 2) L_k^-1 (S_k = L_k L_k^T),
//         c_k = log2 e (ln w_k - d/2 ln 2pi - sum ln L_k,ii)
// rounded up to a multiple of 4 floats.
__host__ __device__ constexpr int comp_stride(int kind, int d) {
    return kind == TGT_ISO ? ((2 + d + 3) / 4) * 4 : ((1 + d + d * (d + 1) / 2 + 3) / 4) * 4;
}
// ISO with the unadjusted random-walk jump process (jump N(0, sigma^2 I)):
// after the K components, K groups of INFLOW_STRIDE floats for Q^T p,
//   [ c'_k | 1/(s_k^2 + sigma^2) | alpha_k | beta_k ],
//   c'_k = ln w_k - d/2 ln(2 pi (s_k^2 + sigma^2)),  alpha_k = s_k^2 / (s_k^2 + sigma^2),
//   beta_k = 1 / sqrt(2 alpha_k sigma^2).
constexpr int INFLOW_STRIDE = 4;

// Rendering-shaped integrand slab (float32):
//   [0,16)  texture A frequencies (8 x 2)      [16,24) amplitudes / 8   [24,32) phases / (2 pi)
//   [32,80) texture B frequencies (8 x 6)      [80,88) amplitudes / 8   [88,96) phases / (2 pi)
//   [96,105) lobe directions (3 x 3)           [105,108) kappa          [108,111) log of
//   4 pi w_l kappa_l / (2 pi (1 - e^{-2 kappa_l}))                      [111] b
constexpr int PSS_SLAB = 112;

// Learned regeneration distribution slab (float32, factorised on the host
// in float64 from the caller's logits / means / log standard deviations):
//   [0]                 log2 beta (-inf when beta = 0)
//   [4 + k * S, ...)    component k: [ r_k (d) | n_k (d) | c_k ], in base 2 as the
//                       mixture targets: r_ki = sqrt(log2 e / 2) / s_ki, n_ki = -m_ki r_ki
//                       (the scaled score is fma(y_i, r_ki, n_ki)),
//                       c_k = log2 e (ln(1 - beta) + ln pi_k - d/2 ln 2 pi - sum_i ln s_ki),
//                       floored at -2^100
//   [4 + K * S, ...)    cumulative weights q_0 = beta, q_j = beta + (1 - beta) sum_{k<j} pi_k
//   [4 + K * S + K, ...) per component [ m_k (d) | s_k (d) ] for the sampler
__host__ __device__ constexpr int mu_stride(int d) { return ((1 + 2 * d + 3) / 4) * 4; }
__host__ __device__ constexpr int mu_slab_floats(int d, int K) { return 4 + K * mu_stride(d) + K + K * 2 * d; }
// Dynamic LDS of the step and drain kernels: the target parameters when
// they are staged (RESTORE_FLAG_PARAMS_LDS), rounded up to 4 floats, then
// the learned mu's K * mu_stride(d) component floats and K cumulative
// weights (slab floats [4, 4 + K (mu_stride(d) + 1))).
__host__ __device__ constexpr int mu_lds_offset(bool params_lds, int n_param_floats) {
    return params_lds ? (n_param_floats + 3) / 4 * 4 : 0;
}

// Fields of the precomputed random inputs of one step (StepRand: t1, e2,
// ln u_acc, d candidate uniforms, d Box-Muller normals).
__host__ __device__ constexpr int rand_fields(int D) { return 3 + 2 * D; }

// The pre-pass of the following chunk, run by extra workgroups of a step
// launch: workgroup step_blocks + g covers its threads' chains for
// PRE_GEN_STEPS steps of that chunk.
constexpr int PRE_GEN_STEPS = 8;
struct PreGen {
    float *out;           // the buffer half it fills
    uint32_t s0;          // first step it draws
    int32_t n_steps;      // steps it draws (<= chunk; 0: none)
    int32_t step_blocks;  // workgroups of the step launch proper
};

// Per-launch arguments of the step kernels.
struct StepArgs {
    // chain state (structure of arrays, C chains)
    float *x;          // [D][C]
    float *logp;       // [C]
    float *logu;       // [C]
    float *grad;       // [D][C] (MALA)
    float *a_cur;      // [C]
    float *t_cur;      // [C]
    float *last_dt;    // [C]
    double *a_done;    // [C]
    double *t_done;    // [C]
    uint32_t *n_done;  // [C]
    uint32_t *status;  // [C]
    unsigned long long *counters;  // [CNT_SLOTS]
    const float *params;           // packed target slab
    const float *mu_params;        // learned mu slab (inside the state buffer)
    float *image;                  // pixel splats or nullptr
    unsigned long long *image_fx;  // fixed-point pixel sums (dt 2^32 each) or nullptr
    const uint32_t *list;          // drain: chains to run, or nullptr (all)
    const uint32_t *list_count;    // drain: number of entries in list
    int64_t n_chains;
    int32_t n_comp;
    int32_t mu_comp;
    float mu_beta;
    float log_c;       // ln c_tilde
    int32_t no_kill;   // c_tilde == 0
    float step;        // sigma or epsilon
    int32_t n_leapfrog;  // HMC: leapfrog steps per update
    float large_prob;  // MH chain: large-step probability l
    uint32_t key0, key1;
    uint32_t target_id;
    uint32_t chain0;   // global id of chain 0 (Philox counter word 1 = chain0 + c)
    uint32_t s0;       // first step index of this launch
    int32_t n_steps;   // steps in this launch
    int32_t integrand_p;
    int32_t rb_dt;     // accumulate E[dt | x] = 1 / (1 + k) instead of dt
    int32_t image_w, image_h;
    int32_t image_batches;  // chains split into contiguous ranges, one image each (>= 1)
    int32_t image_pixels;   // image_w * image_h
    int32_t tile_px;        // tile-stratified runs: tile edge in pixels (0: off)
    int32_t tiles_x;        // tiles per image row
    int32_t n_tiles;        // tiles in the image
    // sample recording (restore_step_record): (x_{i-1}, dt_i) of chains < rec_chains
    float *rec_x;      // [n_steps][rec_chains][D]
    float *rec_w;      // [n_steps][rec_chains]
    int64_t rec_chains;
    // binned pixel splats (step launches of the image integrand): records
    // (pixel, dt) go to per-band buckets instead of scattered image atomics
    uint32_t *bin_pix;     // [n_bins][bin_cap] or nullptr
    float *bin_val;        // [n_bins][bin_cap]
    uint32_t *bin_count;   // entries reserved in band b at [b * SPLAT_COUNTER_STRIDE]
    int32_t bin_cap;
    int32_t n_bins;
};

// Binned splats: the image is cut into bands of 2^SPLAT_BAND_SHIFT pixels
// (one LDS tile of the accumulation kernel); a workgroup stages SPLAT_ROWS
// steps of records in LDS before binning them, and a step launch runs at
// most SPLAT_LAUNCH_STEPS steps before its records are accumulated.
constexpr int SPLAT_BAND_SHIFT = 14;
constexpr int SPLAT_MAX_BANDS = 256;
constexpr int SPLAT_ROWS = 16;
constexpr int SPLAT_LAUNCH_STEPS = 64;
constexpr int SPLAT_MAX_SLICES = 16;      // accumulation workgroups per band (at most)
constexpr int SPLAT_COUNTER_STRIDE = 64;  // one 256-byte line per band counter
constexpr uint32_t SPLAT_NO_PIX = 0xffffffffu;

}  // namespace restore
