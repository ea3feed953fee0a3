/*
 * restore.h -- C ABI of the MI355X (gfx950) Jump Restore chain engine.
 *
 * The library advances a large population of independent Jump Restore
 * chains (Holl, Singh, Seidel, "Jump Restore Light Transport", Sec. 7,
 * Alg. 2).  One chain lives in one GPU lane.  Every step of a chain
 *   1. draws a holding time t1 ~ Exp(1) and a termination time
 *      t2 ~ Exp(k(x)), with the killing rate of Sec. 6.2,
 *      eq. (killing-rate-simplified): k = c_tilde * u(x) / p(x);
 *   2. if t1 < t2, holds x for dt = t1 and makes one Metropolis-Hastings
 *      update with the small-step kernel (Alg. 1, acceptance function of
 *      eq. (optimal-acceptance-function)); otherwise holds x for dt = t2 and
 *      regenerates x ~ mu (the tour ends, Sec. 6, eq. (concatenation));
 *   3. adds dt * f(x_{i-1}) to the running tour integral (Sec. 7.4,
 *      eq. (approx); Sec. 6.3).
 * restore_estimate() turns the per-chain tour sums into the estimates of
 * Sec. 6.3: p_lambda ~ (c_tilde / j) sum tau_i, lambda(p f) ~ (c_tilde / j)
 * int f dt, and pi f ~ sum dt f / sum dt (Sec. 7.4).
 *
 * With c_tilde = 0 the same calls run the paper's reference method instead
 * (Sec. 8, practical setup): the Metropolis-Hastings chain M^l whose
 * proposal mixes a large step from mu (probability l) with the small-step
 * kernel, eq. (mixture-proposal-kernel).  It has no tours; its estimate is
 * the ergodic average pi f ~ sum dt f / sum dt after a burn-in
 * (restore_reset_sums).
 *
 * Conventions
 *   - Every function returns a restore_status: 0 on success, < 0 on error.
 *     The message of the last error on the calling thread is available from
 *     restore_last_error().  No C++ exception crosses this boundary.
 *   - Device buffers are owned by the caller (allocated e.g. as torch
 *     tensors); the library owns only the opaque restore_ctx host object.
 *     Device pointers must stay valid until restore_destroy().
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     All calls are asynchronous on that stream except restore_estimate(),
 *     which synchronises it.  Asynchronous HIP errors surface at the next
 *     synchronising call.
 *   - Random numbers: Philox4x32-10 with key (seed lo, seed hi) and counter
 *     (step, chain, target_id, purpose << 16 | block); a chain's trajectory
 *     is a function of (seed, chain, target_id) only, so it does not depend
 *     on how steps are split across calls or how chains are mapped to lanes.
 *   - The support of every target is the unit box [0,1]^d; p = 0 outside.
 *   - Tracing: with RESTORE_TRACE=1 in the environment at the first call,
 *     the compute entry points (init, step, step_record, drain, the
 *     estimates, the batch calls, the MLP, NLL and Adam calls) each open a
 *     roctx range named after the function (rocprofv3 --marker-trace); the
 *     range covers the host call, i.e. the enqueueing of its launches.
 */
#ifndef RESTORE_H
#define RESTORE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t restore_status;

#define RESTORE_OK                  0
#define RESTORE_E_INVALID_ARG      -1   /* a descriptor field or pointer is invalid   */
#define RESTORE_E_UNSUPPORTED      -2   /* valid, but not built (dimension, kind, ...) */
#define RESTORE_E_HIP              -3   /* a HIP runtime call failed                   */
#define RESTORE_E_NONFINITE        -4   /* NaN or Inf in the parameters                */
#define RESTORE_E_BAD_STATE        -5   /* call out of order (e.g. step after drain)   */
#define RESTORE_E_BUFFER_TOO_SMALL -6   /* state buffer smaller than restore_state_bytes */

#define RESTORE_MAX_DIM   16
#define RESTORE_MAX_COMP  64

/* ---- target density p (Sec. 4, eq. (targetdensity-assumption-1)) ------- */
#define RESTORE_TARGET_GMM_ISO    0
#define RESTORE_TARGET_GMM_FULL   1
#define RESTORE_TARGET_PSS        2

/* Target p on [0,1]^d.  `params` are float64 on the host, copied at init.
 *  GMM_ISO  (dim d, n_comp K): p(x) = sum_k w_k N(x; m_k, s_k^2 I) 1_box(x)
 *           params = [ w (K) | m (K*d, row-major) | s (K) ]
 *  GMM_FULL (dim d, n_comp K): p(x) = sum_k w_k N(x; m_k, S_k) 1_box(x)
 *           params = [ w (K) | m (K*d) | S (K*d*d, row-major, SPD) ]
 *  PSS      (dim 12, n_comp 0): rendering-shaped primary-sample-space
 *           integrand g(x) = tA(x0,x1) tB(x6..x11) [b + sum_l w_l h_l]
 *           with textures t(y) = 1 + (1/8) sum_{m<8} a_m sin(2 pi n_m.y + phi_m)
 *           and lobes h_l(u,v) = 4 pi vMF_kappa_l(omega(u,v); dir_l),
 *           omega = (sqrt(1-z^2) cos 2 pi v, sqrt(1-z^2) sin 2 pi v, z),
 *           z = 1 - 2u, on coordinate pairs (x0,x1), (x2,x3), (x4,x5).
 *           params = [ nA (8*2) | aA (8) | phiA (8) | nB (8*6) | aB (8) |
 *                      phiB (8) | dir (3*3) | kappa (3) | w (3) | b (1) ]  */
typedef struct {
    int32_t kind;
    int32_t dim;
    int32_t n_comp;
    int32_t reserved;
    const double *params;     /* host pointer, copied by restore_init */
    int64_t params_count;     /* number of doubles in params          */
} restore_target;

/* ---- regeneration distribution mu with density u (Sec. 6.2) ----------- */
#define RESTORE_MU_UNIFORM_BOX     0
#define RESTORE_MU_GMM_DIAG        1

/*  UNIFORM_BOX: u = 1 on [0,1]^d.
 *  GMM_DIAG:    u(y) = beta 1_box(y) + (1 - beta) sum_k pi_k N(y; m_k, diag(s_k^2)),
 *               pi = softmax(logits), s = exp(log_std).  `params_dev` is a
 *               caller-owned device float32 buffer [ logits (K) | m (K*d) |
 *               log_std (K*d) ], read once by restore_init and factorised
 *               in float64: mu stays frozen for the run (it must not depend
 *               on the state for k = c_tilde u / p to hold, Sec. 6.2).
 *               Sampling: one uniform picks the uniform share (u < beta) or
 *               a component by the cumulative weights; the component draw
 *               is m_k + s_k z with the step's Box-Muller normals.         */
typedef struct {
    int32_t kind;
    int32_t n_comp;
    float beta;
    int32_t reserved;
    const float *params_dev;
} restore_mu;

/* ---- local dynamics: the small-step kernel zeta of Alg. 1 -------------
 * The three diffusion-derived kernels of the paper's study (Sec. 9), all
 * pi-invariant MH updates, and one local process that is not
 * pi-invariant (the general restore process of Sec. 6.2). */
#define RESTORE_LOCAL_RWMH   0    /* y = x + step z                              */
#define RESTORE_LOCAL_MALA   1    /* y = x + (step^2 / 2) grad log p(x) + step z  */
#define RESTORE_LOCAL_HMC    2    /* Hamiltonian Monte Carlo: momentum rho_0 = z,
                                     n_leapfrog leapfrog steps of size `step` of
                                     dq/dt = rho, drho/dt = grad log p(q) (unit
                                     mass; half momentum steps at both ends),
                                     accepted with exp(-H(y, rho_n) + H(x, rho_0)),
                                     H = -log p + |rho|^2 / 2; a trajectory that
                                     visits a point with p = 0 is rejected.  One
                                     leapfrog step is the MALA proposal.  Built
                                     for the mixture targets with uniform mu. */
#define RESTORE_LOCAL_RW_UNADJUSTED 3 /* local dynamics that are NOT pi-invariant
                                     (Sec. 6.2): the unadjusted random-walk jump
                                     process, every holding-clock firing jumps
                                     y = x + step z with no acceptance test.  The
                                     killing rate is then the general one of eq.
                                     (killing-rate), k = (c_tilde u + L* p) / p
                                     with L* p = Q^T p - p and (Q^T p)(x) =
                                     int p(y) N(x; y, step^2 I) dy over the box
                                     (closed form with erf for the isotropic
                                     mixture).  Needs c_tilde >= sup (p - Q^T p)
                                     / u for k >= 0; a chain that reaches a
                                     state where k < 0 gets NaN sums and is
                                     counted in `nonfinite`.  A jump off the box
                                     lands where p = 0 and is killed at the next
                                     step with dt = 0.  The state's log u slot
                                     holds log u_eff, u_eff = u + L* p / c_tilde.
                                     Built for GMM_ISO with the uniform mu;
                                     c_tilde > 0 (INVALID_ARG otherwise). */

typedef struct {
    int32_t kind;
    float step;              /* random-walk or jump sigma, MALA or HMC epsilon
                                (>= 0; > 0 except for RWMH)                  */
    float large_step_prob;   /* l in [0,1] of eq. (mixture-proposal-kernel).
                                The restore process (c_tilde > 0) uses the
                                pure small-step chain M^0 (Sec. 8), so l must
                                be 0 there (UNSUPPORTED otherwise).  With
                                c_tilde = 0, each update of the MH chain M^l
                                is a large step with probability l (decided by
                                the first uniform of the step's Philox block
                                with purpose 2, block 0, against l as float32):
                                y ~ mu (drawn as a regeneration would be),
                                accepted iff u_acc < p(y) u(x) / (p(x) u(y))
                                (the kernel K_1 of Theorem B in the
                                supplement); otherwise the small-step update */
    int32_t n_leapfrog;      /* HMC: leapfrog steps per update, 1..64; 0 for
                                the other kernels                            */
} restore_local_kernel;

/* ---- run configuration ------------------------------------------------- */
#define RESTORE_INTEGRAND_ONE    1   /* f = 1: tour lifetimes (p_lambda)     */
#define RESTORE_INTEGRAND_P      2   /* f = p: lambda(p^2), pi p             */
#define RESTORE_INTEGRAND_PIXEL  4   /* f = 1_pixel(x0, x1): image splats
                                        (built for the PSS target)        */

#define RESTORE_FLAG_PARAMS_LDS  1   /* stage mixture parameters through LDS
                                        instead of the scalar cache          */
#define RESTORE_FLAG_SPLAT_DIRECT 2  /* PIXEL: add every splat to the image
                                        with a scattered atomic (smaller
                                        state, slower) instead of binning   */
#define RESTORE_FLAG_SPLAT_TIGHT 4   /* PIXEL: 64-fold smaller splat buckets,
                                        so that overflowing records take the
                                        direct path (exercises that path)   */
#define RESTORE_FLAG_INLINE_RNG  16  /* draw every step's random numbers in the
                                        step kernel also for populations below
                                        2^16 chains, which by default take
                                        them from a chip-wide pre-pass (the
                                        chains are the same either way)      */
#define RESTORE_FLAG_IMAGE_FIXED 32  /* PIXEL, untiled runs only (else
                                        UNSUPPORTED): every splat adds its
                                        dt rounded to a multiple of 2^-32
                                        to a 64-bit integer per pixel in the
                                        state buffer (exact integer sums, so
                                        the image is the same bit for bit
                                        whatever the order of the atomics,
                                        the block size or the launch
                                        split); after each restore_step and
                                        restore_drain the caller's float
                                        image receives the sums rounded to
                                        float32, and restore_image_estimate
                                        reads the integers.  A pixel holds
                                        up to 2^32 units of time            */
#define RESTORE_FLAG_RB_DT       8   /* accumulate the conditional mean
                                        E[dt | x] = 1 / (1 + k(x)) of the
                                        holding time in place of the sampled
                                        dt (both clocks still decide kill or
                                        move; unbiased because dt ~
                                        Exp(1 + k) is independent of which
                                        clock fires, Alg. 2)                 */

typedef struct {
    uint64_t seed;           /* Philox key                                   */
    int64_t n_chains;        /* C >= 1, at most 2^31 - 1                      */
    int32_t target_id;       /* Philox counter word 2 (batched targets)      */
    int32_t integrands;      /* RESTORE_INTEGRAND_* bitmask (ONE is implied) */
    double c_tilde;          /* > 0: restore; 0: the MH chain M^l (no killing,
                                no tours, every step adds to the chain sums) */
    int32_t drain_cap;       /* max extra steps to finish tours in flight    */
    int32_t image_w, image_h;/* pixel grid on (x0, x1) if PIXEL is set      */
    int32_t flags;           /* RESTORE_FLAG_*                               */
    int32_t block_size;      /* threads per workgroup (64..256, multiple of
                                64); 0 = library default: 256, or 64 below
                                2^16 chains (spreads a small population's
                                waves over more compute units)              */
    int32_t image_batches;   /* PIXEL: chains split into this many contiguous
                                ranges (chain c in batch floor(c B / C)),
                                each splatting into its own image, for the
                                per-pixel standard error; 0 or 1 = one image;
                                with tile_px > 0 the ranges split each
                                tile's chains instead                         */
    int32_t tile_px;         /* PIXEL: 0, or 1..64 for tile-stratified restore:
                                the image is cut into tiles of tile_px x
                                tile_px pixels (ragged at the right and bottom)
                                numbered row by row; chain c of C works on tile
                                floor(c T / C) only, as its own restore problem
                                (Sec. 6) with target p restricted to the
                                tile's points (the pixel of (x0, x1) in the
                                tile) and mu uniform on them (x0 = (px0 + w u0)
                                / W, x1 = (py0 + h u1) / H in float32), and the
                                killing constant c_tilde A_t (A_t the tile's
                                share of the box), so the killing rate stays
                                c_tilde / p.  The estimates add the tiles'
                                tour ratios with the factor c_tilde A_t.  Each
                                workgroup accumulates its tile's splats in
                                LDS.  Needs the uniform mu, c_tilde > 0 and at
                                least max(1, image_batches) chains per tile  */
    int32_t first_chain;     /* global id of this run's chain 0 (>= 0; first_chain
                                + n_chains <= 2^32): chain c draws its random
                                numbers with Philox counter word 1 = first_chain
                                + c, so runs over the ranges [c0, c1) of one
                                chain population follow exactly the
                                trajectories of one run over all of them (tours
                                spawned from mu are independent, Sec. 1: a
                                population can be split across launches or
                                devices with no start-up bias).  The image-batch
                                map is over the run's own chains; UNSUPPORTED
                                with tile_px > 0, whose chain-to-tile map
                                depends on the whole population                */
} restore_config;

/* ---- estimates (Sec. 6.3, Sec. 7.4) ----------------------------------- */
typedef struct {
    double p_lambda, p_lambda_se;    /* c_tilde * sum T / sum N          */
    double lam_pf, lam_pf_se;        /* c_tilde * sum A / sum N  (f = p) */
    double pi_f, pi_f_se;            /* sum A / sum T            (f = p) */
    int64_t tours_done;              /* j: completed tours               */
    int64_t tours_censored;          /* tours still alive at the cap     */
    int64_t transitions;             /* steps executed, drain included   */
    int64_t accepts, kills;
    int64_t nonfinite;               /* chains whose sums are not finite */
    double censored_time_frac;       /* censored lifetime / total time   */
    double accept_rate, kill_rate;   /* per transition                   */
    double image_scale;              /* c_tilde / j: multiplies the image sums
                                        (NaN for tile-stratified runs: per
                                        tile c_tilde A_t / j_t)            */
    int64_t large_steps;             /* MH chain: large-step proposals     */
    int64_t large_accepts;           /* MH chain: accepted large steps     */
} restore_estimate_out;

typedef struct restore_ctx restore_ctx;

/* Bytes of device memory the state buffer must provide for this problem:
 * the per-chain state of Alg. 2 (x, the cached log p, log u and grad log p,
 * the running and completed tour sums of Sec. 6.3) in structure-of-arrays
 * layout, the packed parameters, reduction and drain scratch, the splat
 * buckets of the image integrand (or its 64-bit fixed-point sums with
 * RESTORE_FLAG_IMAGE_FIXED), and for populations below 2^16 chains
 * with the uniform mu the two halves (at most 32 MiB each) of the
 * random-input pre-pass buffer of restore_step and restore_drain.  Pure host computation; the same
 * validation as restore_init (INVALID_ARG, UNSUPPORTED, NONFINITE). */
restore_status restore_state_bytes(const restore_target *target, const restore_mu *mu,
                                   const restore_local_kernel *local,
                                   const restore_config *cfg, size_t *bytes_out);

/* Validate the descriptors, pack the target parameters into the state
 * buffer (float32, each component's Cholesky factor derived here in
 * float64) and draw x_0 ~ mu for every chain (Alg. 2 input; tours are
 * spawned from mu so that chains are unbiased in parallel, Sec. 1).
 * `state_dev` (>= restore_state_bytes, 256-byte aligned) and `image_dev`
 * (float32 [image_batches][image_h][image_w], zeroed by the caller; NULL
 * unless PIXEL) are
 * caller-owned device memory.  On success *out receives a new context. */
restore_status restore_init(restore_ctx **out, const restore_target *target,
                            const restore_mu *mu, const restore_local_kernel *local,
                            const restore_config *cfg, void *state_dev,
                            size_t state_bytes, float *image_dev, void *stream);

/* Advance every chain by n_steps steps of Alg. 2 with regeneration
 * (steps s .. s + n_steps - 1, s = steps already taken).  Enqueue only.
 * With c_tilde = 0: n_steps updates of the MH chain M^l, each adding dt
 * f(x_{i-1}) to the chain's float64 sums (dt = 1 with RESTORE_FLAG_RB_DT,
 * the discrete-time average; else the Exp(1) holding time of the
 * continuous-time chain with generator K_l - id).
 * With the PIXEL integrand (unless RESTORE_FLAG_SPLAT_DIRECT or
 * RESTORE_FLAG_IMAGE_FIXED) the steps run
 * as launches of at most 64 steps whose splat records are binned by image
 * band in the state buffer and summed into the image after each launch.
 * Populations below 2^16 chains with the uniform mu (restore, no image, no
 * LDS staging, no RESTORE_FLAG_INLINE_RNG) run chunks of steps whose
 * state-independent random inputs (the Philox blocks, the clocks'
 * exponentials, ln u_acc, the candidate uniforms and their Box-Muller
 * normals) come from a chip-wide pre-pass: each step launch reads one half
 * of the buffer while extra workgroups of the same launch draw the next
 * chunk into the other half (only the first chunk of a context, or of a
 * call that follows restore_step_record, takes a pre-pass launch of its
 * own).  The chains are the same either way. */
restore_status restore_step(restore_ctx *ctx, int32_t n_steps, void *stream);

/* End of the budget (the estimators of Sec. 7.4 assume a run that ends at
 * a tour completion): run every chain on, without regeneration, until its
 * tour in flight is killed (it then retires) or drain_cap further steps
 * have passed (the tour is censored: excluded from the estimates, counted
 * and reported).  Retired chains are compacted out of the launches with
 * wavefront ballots (launches of 1, 2, 4, ... steps; below 2^16 chains one
 * launch over the whole cap, whose first steps take their random inputs
 * from the pre-pass buffer when restore_step uses it); the chains are the
 * same either way.  After
 * restore_drain no further restore_step.  For the MH chain (c_tilde = 0)
 * there is nothing to finish: no launch. */
restore_status restore_drain(restore_ctx *ctx, void *stream);

/* Burn-in of the MH chain (c_tilde = 0; the paper's MH baselines discard
 * their first 10,000 iterations, Sec. 9): zero every chain's sums, the run
 * counters and the image (if any), keeping the chain states, so that the
 * estimate covers the steps after this call only.  RESTORE_E_BAD_STATE for
 * the restore process (c_tilde > 0: a tour in flight would lose its start
 * and bias the estimates) or after restore_drain.  Enqueue only. */
restore_status restore_reset_sums(restore_ctx *ctx, void *stream);

/* Reduce the per-chain tour sums in float64 and fill *out (host memory,
 * caller-owned): p_lambda = c_tilde sum T / sum N and lam_pf = c_tilde
 * sum A / sum N over completed tours (Sec. 6.3, the tour decomposition),
 * pi_f = sum A / sum T (Sec. 7.4, eq. (approx)), each with the
 * delta-method standard error over chains; censored tours are excluded and
 * reported, chains with non-finite sums excluded and counted (nonfinite).
 * With c_tilde = 0 only pi_f exists (the others are NaN).  Synchronises
 * `stream`; HIP_ERROR reports a failure of the enqueued work. */
restore_status restore_estimate(restore_ctx *ctx, restore_estimate_out *out, void *stream);

/* Per-pixel estimate of the image integrand, lambda(p h_j) = c_tilde
 * (sum of the dt splatted into pixel j) / j (Sec. 7.4, eq. (approx) with
 * f = the pixel indicator, Sec. 6.3), into mean_dev[image_h][image_w], and
 * its delta-method standard error over the image batches into
 * se_dev[image_h][image_w] (NaN with one batch): with S_b the batch images
 * and N_b the tours completed by the batch's chains,
 * se = c_tilde sqrt(sum_b (S_b - R N_b)^2 / ((B - 1) B)) / mean N_b,
 * R = sum S_b / sum N_b.  Splats of a tour censored at the drain cap stay
 * in the image (their share of the time is censored_time_frac).  Device
 * float32 outputs, caller-owned; enqueue only (after the drain). */
restore_status restore_image_estimate(restore_ctx *ctx, float *mean_dev, float *se_dev, void *stream);

/* Device addresses of the chain state arrays, for tests and checkpointing.
 * Layout: x float32 [d][C]; logp, logu float32 [C]; grad float32 [d][C]
 * (MALA and HMC, else NULL); a_cur, t_cur float32 [C]; a_done, t_done float64
 * [C]; n_done uint32 [C]; status uint32 [C] (bit0 alive, bit1 censored,
 * bit2 last step killed, bit3 last step accepted); last_dt float32 [C]. */
typedef struct {
    float *x, *logp, *logu, *grad, *a_cur, *t_cur, *last_dt;
    double *a_done, *t_done;
    uint32_t *n_done, *status;
    int64_t n_chains;
    int32_t dim;
    int32_t steps_taken;     /* steps with regeneration so far            */
} restore_state_view;

/* Fill *view (host struct) with the device addresses above and the step
 * count; no device work.  Library bookkeeping, no passage of the paper. */
restore_status restore_get_state_view(const restore_ctx *ctx, restore_state_view *view);

/* Recompute the cached values of Alg. 2's state (log p, log u -- log u_eff
 * for the unadjusted jump process -- and grad log p) from x for every chain
 * (after a caller has written x, e.g. to restore a checkpoint or to set up
 * a parity test).  `status` bits are not touched.  Enqueue only. */
restore_status restore_refresh_cache(restore_ctx *ctx, void *stream);

/* Release the context (device buffers stay the caller's); NULL is a
 * no-op.  Library bookkeeping, no passage of the paper. */
restore_status restore_destroy(restore_ctx *ctx);

/* ---- batched targets ---------------------------------------------------
 * Many independent targets (full-covariance mixtures of uneven dimension,
 * component count and chain count; random-walk MH local moves; each with
 * the uniform mu or its own regeneration distribution of the learned form)
 * advanced together.  Each target is its own restore problem exactly as
 * above (Alg. 2 with the killing rate of eq. (killing-rate-simplified));
 * target i uses Philox target id cfgs[i].target_id, so its chains follow
 * the same trajectories as a single-target run with that id.
 * One pass = x_0 ~ mu, n_steps steps with regeneration, the drain of the
 * tours in flight (cfgs[i].drain_cap) and the per-target reduction.  The
 * work is split into tiles of block_size chains of one target; persistent
 * workgroups pop tiles from a queue in longest-processing-time-first or
 * target order, optionally one queue per dimension range; targets with the
 * uniform and with the learned-form mu take separate queues. */
#define RESTORE_BATCH_ORDER_LPT      0
#define RESTORE_BATCH_ORDER_TARGET   1
#define RESTORE_BATCH_BUCKETS_ONE    0   /* one persistent kernel for every dimension   */
#define RESTORE_BATCH_BUCKETS_DIM4   1   /* one per dimension range 1-4, 5-8, 9-12, 13-16 */
#define RESTORE_BATCH_MODE_GRAPH      0  /* replay of a captured hipGraph of the pass  */
#define RESTORE_BATCH_MODE_PERSISTENT 1  /* the same launches without the graph        */
#define RESTORE_BATCH_MODE_SEPARATE   2  /* one launch per target (for comparison)     */

typedef struct {
    int32_t block_size;   /* chains per tile = threads per workgroup: 64, 128, 256 */
    int32_t order;        /* RESTORE_BATCH_ORDER_*                                 */
    int32_t buckets;      /* RESTORE_BATCH_BUCKETS_*                               */
    int32_t reserved;
} restore_batch_tiling;

/* Device pointers to one target's per-chain results (float64 tour sums). */
typedef struct {
    uint32_t *n_done;
    double *t_done, *a_done;
    uint32_t *status;      /* bit0 alive, bit1 censored                 */
    float *t_cur;          /* lifetime so far of a censored tour        */
    int64_t n_chains;
} restore_chain_sums;

typedef struct restore_batch restore_batch;

/* Bytes of caller-owned device memory for the batch (targets table, work
 * queue, parameter slabs, per-chain results). */
restore_status restore_batch_state_bytes(int32_t n_targets, const restore_target *targets,
                                         const restore_local_kernel *locals, const restore_config *cfgs,
                                         const restore_mu *mus, size_t *bytes_out);
/* Validate, factorise every target's parameters in float64, upload, and
 * build the work queue for the default tiling (256, LPT, one kernel).
 * Arrays have n_targets entries; cfgs[i].n_chains, c_tilde, seed,
 * target_id, integrands and drain_cap are used per target.  `mus` is NULL
 * (every target regenerates from the uniform mu) or n_targets descriptors
 * as for restore_init: a GMM_DIAG entry's caller-owned device row is read
 * once here and factorised in float64, so that target's chains follow a
 * single-target run with the same mu bit for bit. */
restore_status restore_batch_init(restore_batch **out, int32_t n_targets, const restore_target *targets,
                                  const restore_local_kernel *locals, const restore_config *cfgs,
                                  const restore_mu *mus, int32_t n_steps, void *state_dev, size_t state_bytes,
                                  void *stream);
/* Change the tiling (rebuilds the queue, synchronous; results are
 * independent of the tiling). */
restore_status restore_batch_set_tiling(restore_batch *b, const restore_batch_tiling *tiling);
/* The tiling in use (host struct). */
restore_status restore_batch_get_tiling(const restore_batch *b, restore_batch_tiling *tiling);
/* Enqueue one full pass.  GRAPH captures the pass into a hipGraph on the
 * first call (on a private stream) and replays it on `stream`. */
restore_status restore_batch_run(restore_batch *b, int32_t mode, void *stream);
/* Per-target estimates of the last pass into out[n_targets]; synchronises. */
restore_status restore_batch_estimates(restore_batch *b, restore_estimate_out *out, void *stream);
/* Device addresses of one target's per-chain tour sums of the last pass
 * (for tests; the layout of restore_chain_sums); INVALID_ARG for a target
 * outside 0..n_targets-1. */
restore_status restore_batch_chain_sums(const restore_batch *b, int32_t target, restore_chain_sums *out);
/* Time every tiling (block 64/128/256 x order x bucketing) on this batch
 * with HIP events, keep the fastest and write it to `cache_path` (JSON,
 * keyed by GPU architecture and batch shape); a matching cache entry is
 * applied without timing.  cache_path may be NULL. */
restore_status restore_batch_autotune(restore_batch *b, const char *cache_path, restore_batch_tiling *chosen,
                                      double *best_ms, void *stream);
/* Release the batch handle and its graph (device memory stays the
 * caller's).  Library bookkeeping, no passage of the paper. */
restore_status restore_batch_destroy(restore_batch *b);

/* ---- sample collection -------------------------------------------------
 * Like restore_step, and additionally records, for chains [0, n_record) and
 * every one of the n_steps steps, the pair (x_{i-1}, dt_i) of Alg. 2's
 * output: x_out float32 [n_steps][n_record][d], w_out float32
 * [n_steps][n_record] (caller-owned device memory).  The time-weighted
 * pairs are draws of pi in the sense of Sec. 7.4, eq. (approx): the
 * training data of the learned regeneration distribution.  UNSUPPORTED for
 * tile-stratified runs (their chains sample p on one tile each). */
restore_status restore_step_record(restore_ctx *ctx, int32_t n_steps, int64_t n_record, float *x_out,
                                   float *w_out, void *stream);

/* ---- learned regeneration distribution ---------------------------------
 * mu_theta = (1 - beta) GMM(MLP_theta(c)) + beta Uniform(box): an MLP with
 * two GELU hidden layers maps a context vector c to the logits, means and
 * log standard deviations of a diagonal Gaussian mixture, laid out exactly
 * as restore_mu expects ([logits K | means K*d | log_std K*d]).  It is
 * trained between runs on restore samples (restore_step_record) by
 * minimising -sum w log u_theta(x) / sum w, and frozen during a run (mu must
 * be state-independent for k = c_tilde u / p, Sec. 6.2).
 * Parameters theta (float32, row-major, out x in):
 *   [ W1 (H x in) | b1 (H) | W2 (H x H) | b2 (H) | W3 (O x H) | b3 (O) ],
 *   O = K (1 + 2 d).  Two arithmetic paths (the precision field):
 *   RESTORE_MLP_FP32: float32 FMAs in a fixed order, one fused launch per
 *   pass (each layer a matrix-vector product per context row; in_dim and
 *   hidden at most 256, else UNSUPPORTED); RESTORE_MLP_BF16: the layers
 *   as GEMMs on the matrix cores (v_mfma_f32_32x32x16_bf16: bf16 operands,
 *   float32 accumulation); RESTORE_MLP_AUTO: FP32 for G <= 16 context
 *   rows within those widths, else BF16. */
#define RESTORE_MLP_AUTO 0
#define RESTORE_MLP_FP32 1
#define RESTORE_MLP_BF16 2
typedef struct {
    int32_t in_dim;   /* context length (12 for the learned-mu workload) */
    int32_t hidden;   /* H                                               */
    int32_t n_comp;   /* K <= 64                                         */
    int32_t dim;      /* d <= 16                                         */
    int32_t precision;/* RESTORE_MLP_AUTO, _FP32 or _BF16               */
} restore_mlp_shape;

/* Number of float32 parameters, and activations saved per context row. */
restore_status restore_mlp_param_count(const restore_mlp_shape *shape, int64_t *n_params, int64_t *n_act_per_row);
/* out[G][O] = MLP_theta(ctx[G][in]).  act (4 G H floats, from
 * n_act_per_row) receives four consecutive [G][H] blocks z1, h1, z2, h2
 * (pre- and post-GELU values of the two hidden layers) for the backward
 * pass.  Device pointers, caller-owned; enqueue only. */
restore_status restore_mlp_forward(const restore_mlp_shape *shape, const float *theta, const float *ctx, int32_t G,
                                   float *act, float *out, void *stream);
/* grad[n_params] = d(sum_g dout[g] . out[g]) / d theta (overwritten, not
 * accumulated), from the act of the matching forward call; work: 2 G H
 * floats of scratch.  Device pointers, caller-owned; enqueue only. */
restore_status restore_mlp_backward(const restore_mlp_shape *shape, const float *theta, const float *ctx, int32_t G,
                                    const float *act, const float *dout, float *work, float *grad, void *stream);
/* Bytes of device workspace restore_gmm_nll needs (per-block float64
 * partial sums). */
restore_status restore_gmm_nll_workspace_bytes(size_t *bytes);
/* Weighted NLL of samples x[n][d] with weights w[n] under the defensive
 * mixture of one MLP output row gmm[O] (the training loss of the learned
 * mu above; the weights are the holding times of Sec. 7.4, eq. (approx)):
 * *loss_dev (float64, device) = -sum w log u / sum w and dout[O] = its
 * gradient with respect to gmm.  Float32 arithmetic on centred scores,
 * float64 accumulation, fixed-order reduction (bit-reproducible).  Device
 * pointers, caller-owned; INVALID_ARG for K outside 1..64, d outside
 * 1..16, beta outside [0, 1), a null pointer or n < 1; BUFFER_TOO_SMALL for
 * a workspace below restore_gmm_nll_workspace_bytes.  Enqueue only. */
restore_status restore_gmm_nll(int32_t n_comp, int32_t dim, float beta, const float *gmm, const float *x,
                               const float *w, int64_t n, float *dout, double *loss_dev, void *workspace,
                               size_t workspace_bytes, void *stream);
/* restore_gmm_nll for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving or training loops, harnesses that
 * forbid hipMalloc): the same validation, kernels and result bit for bit,
 * with the workspace taken from a library-owned device array instead of an
 * argument.  That array (restore_gmm_nll_workspace_bytes, about 4.5 MB) is
 * the largest workspace restore_gmm_nll can need -- partial sums of at most
 * 256 workgroups of the largest mixture (d = 16) -- so every valid n, K and
 * d fits; K outside 1..64 or d outside 1..16 is INVALID_ARG as for
 * restore_gmm_nll.  Each GPU holds its own copy from the first call on it
 * until the process ends; the call allocates nothing (no hipMalloc, hipFree
 * or allocating library routine) and needs no zeroed memory (the kernels
 * write every partial sum they read).  All calls on one GPU share its copy:
 * calls that overlap on one GPU (on different streams, or from different
 * threads without ordering) race and their results are undefined.  Device
 * pointers, caller-owned; enqueue only. */
restore_status restore_gmm_nll_noalloc(int32_t n_comp, int32_t dim, float beta, const float *gmm, const float *x,
                                       const float *w, int64_t n, float *dout, double *loss_dev, void *stream);
/* One Adam step (t >= 1) on float32 master weights theta[n] with moments
 * m[n], v[n] (device, caller-owned, updated in place) from grad[n]: the
 * optimiser of the learned mu's training.  Enqueue only. */
restore_status restore_adam_step(float *theta, const float *grad, float *m, float *v, int64_t n, int32_t t, float lr,
                                 float beta1, float beta2, float eps, void *stream);

/* Message of the last failed call on this thread ("" if none); the string
 * is owned by the library and valid until the next failing call on this
 * thread. */
const char *restore_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RESTORE_H */
