/*
 * FP64 CPU oracle of the Jump Restore process -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header or table with the HIP path:
 * it has its own Philox, its own uniform/normal/exponential mapping, its own
 * densities and its own step.  It is deliberately plain and slow: one chain
 * at a time, every quantity in double precision, the steps in the order the
 * paper gives them.
 *
 * What it follows (Holl, Singh, Seidel, "Jump Restore Light Transport"):
 *   - Alg. 2 (Jump Restore): per step draw t1 ~ Exp(1) (holding time) and
 *     t2 ~ Exp(k(x)) (time to the next termination attempt); if t1 < t2 the
 *     chain holds for t1 and makes a local move x' ~ zeta(x, .), otherwise
 *     it holds for t2 and is regenerated x' ~ mu.  The pair (dt, x_{i-1}) is
 *     the output.
 *   - Sec. 6.2, eq. (killing-rate-simplified): with pi-invariant local
 *     dynamics and a state-independent mu of density u, k = c_tilde u / p.
 *   - Alg. 1 with the acceptance function of eq. (optimal-acceptance-
 *     function): accept iff U < alpha(x, y), alpha = min(1, p(y)q(y,x) /
 *     (p(x)q(x,y))) when p(x)q(x,y) > 0, else 1.
 *   - The small-step kernels the paper's study derives from diffusions
 *     (Sec. 9): a Gaussian random walk (Brownian motion), the Langevin
 *     proposal (MALA), and Hamiltonian Monte Carlo: a momentum rho ~ N(0, I)
 *     and n leapfrog steps of size e of the dynamics with potential -log p
 *     and unit mass, accepted with exp(-H(y, rho_n) + H(x, rho_0)),
 *     H = -log p + |rho|^2 / 2.
 *   - Sec. 6.3 / 7.4: the tour decomposition, the estimates
 *     p_lambda ~ (c_tilde / j) sum tau_i and lambda(p f) ~ (c_tilde / j)
 *     int f dt, and the time-weighted left-rectangle sums of eq. (approx).
 *   - Sec. 6.2, eq. (killing-rate), for local dynamics that are NOT
 *     pi-invariant: k = (c_tilde u + L* p) / p, with L* the adjoint of the
 *     local process's generator.  The local process here is the unadjusted
 *     random-walk jump process (rate 1, every jump y = x + sigma z taken,
 *     no acceptance test), whose adjoint generator gives
 *     L* p = Q^T p - p with (Q^T p)(x) = int p(y) N(x; y, sigma^2 I) dy;
 *     for mixtures with diagonal covariances on the box the integral is a
 *     product of Gaussian and erf terms.  The state caches log u_eff with
 *     u_eff = u + L* p / c_tilde, so that k = c_tilde u_eff / p keeps the
 *     form of the invariant case.  k must be non-negative everywhere
 *     (c_tilde >= sup (p - Q^T p) / u); a state with u_eff < 0 makes the
 *     step's holding time NaN, so the chain's sums are NaN and the chain
 *     is excluded and counted as non-finite.  A jump off the box lands
 *     where p = 0: k = +inf, killed at once with dt = 0.
 *   - Sec. 5, eq. (mixture-proposal-kernel), and the reference chain of
 *     Sec. 8 (practical setup): with large-step probability l a local
 *     update proposes y ~ mu instead of a small step.  The mixture is taken
 *     as a mixture of two Metropolis-Hastings kernels, K_l = l K_1 +
 *     (1 - l) K_0 (Theorem B of the supplement), so a large step is
 *     accepted with the independence-sampler ratio p(y) u(x) / (p(x) u(y))
 *     and a small step with the small-step kernel's own ratio.  With
 *     c_tilde = 0 this is the paper's MH baseline M^l: no tours; after a
 *     burn-in, every step adds dt f(x_{i-1}) to the chain's sums, and
 *     pi f ~ sum dt f / sum dt.
 *
 * Readings where the paper is silent (all shared with the GPU side as a
 * specification, never as code):
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), key = (seed lo,
 *     seed hi), counter = (step, chain, target, purpose << 16 | block);
 *     uniforms u = (2 (r >> 9) + 1) 2^-24; normals by Box-Muller; Exp(1)
 *     variates as -ln u.  Block 0 of a step gives (u_E1, u_E2, u_acc,
 *     u_cat); blocks 1.. give the d candidate uniforms.
 *   - k = +inf where p(x) = 0 (immediate kill, dt = 0); k = 0 when
 *     c_tilde = 0 (no killing, a plain MH chain).
 *   - tile-stratified restore (the image integrand, tile_px > 0): the
 *     pixel grid is cut into tiles of tile_px x tile_px pixels (ragged at
 *     the right and bottom edges); chain c of C works on tile
 *     floor(c T / C) only: its target is p restricted to the tile's points
 *     (pixel of (x0, x1) inside the tile), its mu is uniform there,
 *     sampled as x0 = fma(w, u0, px0) / W and x1 = fma(h, u1, py0) / H in
 *     float32, the other coordinates as the uniform mu's, and its killing
 *     rate is the unstratified one, k = c_tilde / p, i.e. the tile's own
 *     constant is c_tilde A_t with A_t the tile's share of the box.  Each
 *     tile is its own restore problem; its estimates carry the factor
 *     c_tilde A_t / j_t (j_t its completed tours) and the tiles add up.
 *   - the large-step choice: u_L < l, with u_L the first uniform of its own
 *     Philox block (purpose LARGE, block 0), drawn only for local updates
 *     when l > 0; the large-step candidate is drawn from mu with the same
 *     uniforms as a regeneration (u_cat and the candidate blocks).
 *   - the step budget: B steps with regeneration, then the tour in flight is
 *     finished without regeneration for at most drain_cap further steps;
 *     tours still alive then are censored (excluded and reported).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define OR_MAXD 16
#define OR_MAXK 64

enum { OR_TARGET_GMM = 0, OR_TARGET_PSS = 1 };
enum { OR_MU_UNIFORM = 0, OR_MU_GMM_DIAG = 1 };
enum { OR_LOCAL_RWMH = 0, OR_LOCAL_MALA = 1, OR_LOCAL_HMC = 2, OR_LOCAL_RW_UNADJUSTED = 3 };
enum { OR_PURPOSE_INIT = 0, OR_PURPOSE_STEP = 1, OR_PURPOSE_LARGE = 2 };
enum { OR_FLAG_KILL = 1, OR_FLAG_ACCEPT = 2, OR_FLAG_OUTSIDE = 4, OR_FLAG_LARGE = 8, OR_FLAG_NEGATIVE_RATE = 16 };

/* Target density p on the unit box.
 * GMM: p(x) = sum_k w_k N(x; m_k, S_k) for x in [0,1]^d, 0 outside.
 *      log_w[k] = ln w_k, mean[k*d + i], prec[k*d*d + i*d + j] = (S_k^-1)_ij,
 *      logdet[k] = ln det S_k.
 * PSS: g(x) = tA(x0,x1) tB(x6..x11) [b + sum_l w_l h_l(x_{2l-2}, x_{2l-1})]. */
typedef struct {
    int32_t kind, d, K, pad;
    const double *log_w, *mean, *prec, *logdet;
    /* pss */
    const double *ta_freq, *ta_amp, *ta_phase;   /* [8*2], [8], [8] */
    const double *tb_freq, *tb_amp, *tb_phase;   /* [8*6], [8], [8] */
    const double *lobe_dir, *lobe_kappa, *lobe_w; /* [3*3], [3], [3] */
    double base;
} or_target;

/* Regeneration distribution mu.
 * UNIFORM: u = 1 on [0,1]^d.
 * GMM_DIAG: u(y) = beta 1_box(y) + (1 - beta) sum_k pi_k N(y; m_k, diag(s_k^2))
 *           with pi = softmax(logit), s_k = exp(log_std_k). */
typedef struct {
    int32_t kind, d, K, pad;
    double beta;
    const double *logit, *mean, *log_std;
} or_mu;

typedef struct {
    int32_t kind;
    int32_t n_leapfrog;       /* HMC: leapfrog steps per update            */
    double step;              /* random-walk sigma, MALA or HMC epsilon   */
    double large_step_prob;   /* l of eq. (mixture-proposal-kernel)        */
} or_local;

typedef struct {
    uint64_t seed;
    uint32_t target_id, pad;
    double c_tilde;
    int32_t integrand_p;     /* accumulate f = p as well as f = 1 */
    int32_t image_w, image_h; /* pixel integrand on (x0, x1); 0 = off */
    int32_t rb_dt;           /* return E[dt | x] = 1 / (1 + k(x)) instead of dt */
    int32_t burn_in;         /* c_tilde = 0: steps not accumulated at the start */
    int32_t tile_px;         /* > 0: tile-stratified restore (image integrand) */
    int64_t n_chains_total;  /* C, for the chain -> tile map                    */
} or_config;

/* ----------------------------------------------------------------------- */
/* Philox4x32-10                                                            */
/* ----------------------------------------------------------------------- */

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* odd 23-bit uniform in (0,1): exactly representable in binary32 */
double oracle_u01(uint32_t r)
{
    return (2.0 * (double)(r >> 9) + 1.0) * ldexp(1.0, -24);
}

static void draw_block(const or_config *cfg, uint32_t step, uint32_t chain,
                       uint32_t purpose, uint32_t block, double u[4])
{
    uint32_t ctr[4] = { step, chain, cfg->target_id, (purpose << 16) | block };
    uint32_t key[2] = { (uint32_t)(cfg->seed & 0xffffffffu), (uint32_t)(cfg->seed >> 32) };
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    for (int i = 0; i < 4; ++i) u[i] = oracle_u01(r[i]);
}

/* All uniforms of one step: head = (u_E1, u_E2, u_acc, u_cat); cand = the
 * candidate uniforms (4 per block, blocks 1..ceil(d/4)). */
static void draw_step(const or_config *cfg, int d, uint32_t step, uint32_t chain,
                      uint32_t purpose, double head[4], double cand[OR_MAXD])
{
    draw_block(cfg, step, chain, purpose, 0, head);
    int nb = (d + 3) / 4;
    for (int b = 0; b < nb; ++b) draw_block(cfg, step, chain, purpose, (uint32_t)(b + 1), cand + 4 * b);
}

/* Box-Muller: z_{2m} = sqrt(-2 ln u_{2m}) cos(2 pi u_{2m+1}),
 *             z_{2m+1} = sqrt(-2 ln u_{2m}) sin(2 pi u_{2m+1}). */
static void box_muller(int d, const double cand[OR_MAXD], double z[OR_MAXD])
{
    for (int m = 0; 2 * m < d; ++m) {
        double r = sqrt(-2.0 * log(cand[2 * m]));
        double a = 2.0 * M_PI * cand[2 * m + 1];
        z[2 * m] = r * cos(a);
        if (2 * m + 1 < d) z[2 * m + 1] = r * sin(a);
    }
}

/* ----------------------------------------------------------------------- */
/* densities                                                                */
/* ----------------------------------------------------------------------- */

static int in_box(int d, const double *x)
{
    for (int i = 0; i < d; ++i)
        if (!(x[i] >= 0.0 && x[i] <= 1.0)) return 0;
    return 1;
}

static double log_sum_exp(int n, const double *a)
{
    double m = -INFINITY;
    for (int i = 0; i < n; ++i) if (a[i] > m) m = a[i];
    if (m == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += exp(a[i] - m);
    return m + log(s);
}

/* log N(x; m, S) = -1/2 (d ln 2 pi + ln det S + (x-m)^T S^-1 (x-m)) */
static double gmm_component_log(const or_target *t, int k, const double *x)
{
    int d = t->d;
    const double *m = t->mean + (size_t)k * d;
    const double *P = t->prec + (size_t)k * d * d;
    double q = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            q += (x[i] - m[i]) * P[i * d + j] * (x[j] - m[j]);
    return t->log_w[k] - 0.5 * (d * log(2.0 * M_PI) + t->logdet[k] + q);
}

/* texture t(y) = 1 + (1/8) sum_m a_m sin(2 pi <n_m, y> + phi_m) */
static double texture(int dim, const double *freq, const double *amp, const double *phase, const double *y)
{
    double s = 0.0;
    for (int m = 0; m < 8; ++m) {
        double dot = 0.0;
        for (int i = 0; i < dim; ++i) dot += freq[m * dim + i] * y[i];
        s += amp[m] * sin(2.0 * M_PI * dot + phase[m]);
    }
    return 1.0 + s / 8.0;
}

/* h(u, v) = 4 pi vMF_kappa(omega(u, v); mu) with z = 1 - 2u, phi = 2 pi v,
 * vMF_kappa(w; mu) = kappa / (2 pi (1 - e^{-2 kappa})) exp(kappa (mu.w - 1)) */
static double lobe(const double *dir, double kappa, double u, double v)
{
    double z = 1.0 - 2.0 * u;
    double r = sqrt(fmax(0.0, 1.0 - z * z));
    double w0 = r * cos(2.0 * M_PI * v), w1 = r * sin(2.0 * M_PI * v), w2 = z;
    double dot = dir[0] * w0 + dir[1] * w1 + dir[2] * w2;
    double vmf = kappa / (2.0 * M_PI * (1.0 - exp(-2.0 * kappa))) * exp(kappa * (dot - 1.0));
    return 4.0 * M_PI * vmf;
}

static double pss_g(const or_target *t, const double *x)
{
    double ta = texture(2, t->ta_freq, t->ta_amp, t->ta_phase, x);
    double tb = texture(6, t->tb_freq, t->tb_amp, t->tb_phase, x + 6);
    double light = t->base;
    for (int l = 0; l < 3; ++l)
        light += t->lobe_w[l] * lobe(t->lobe_dir + 3 * l, t->lobe_kappa[l], x[2 * l], x[2 * l + 1]);
    return ta * tb * light;
}

/* log p(x); for MALA also grad log p(x) = sum_k r_k (-S_k^-1 (x - m_k)),
 * r = softmax over components of the component log terms. */
double oracle_log_target(const or_target *t, const double *x, double *grad)
{
    int d = t->d;
    if (!in_box(d, x)) {
        if (grad) for (int i = 0; i < d; ++i) grad[i] = 0.0;
        return -INFINITY;
    }
    if (t->kind == OR_TARGET_PSS) {
        if (grad) for (int i = 0; i < d; ++i) grad[i] = 0.0;
        return log(pss_g(t, x));
    }
    double a[OR_MAXK];
    for (int k = 0; k < t->K; ++k) a[k] = gmm_component_log(t, k, x);
    double lp = log_sum_exp(t->K, a);
    if (grad) {
        for (int i = 0; i < d; ++i) grad[i] = 0.0;
        for (int k = 0; k < t->K; ++k) {
            double r = exp(a[k] - lp);
            const double *m = t->mean + (size_t)k * d;
            const double *P = t->prec + (size_t)k * d * d;
            for (int i = 0; i < d; ++i) {
                double s = 0.0;
                for (int j = 0; j < d; ++j) s += P[i * d + j] * (x[j] - m[j]);
                grad[i] -= r * s;
            }
        }
    }
    return lp;
}

/* log u(y) of the regeneration distribution */
double oracle_log_mu(const or_mu *mu, const double *y)
{
    int d = mu->d;
    if (mu->kind == OR_MU_UNIFORM) return in_box(d, y) ? 0.0 : -INFINITY;
    /* defensive mixture: beta * uniform + (1 - beta) * diagonal GMM */
    double lse_logit;
    {
        double m = -INFINITY, s = 0.0;
        for (int k = 0; k < mu->K; ++k) if (mu->logit[k] > m) m = mu->logit[k];
        for (int k = 0; k < mu->K; ++k) s += exp(mu->logit[k] - m);
        lse_logit = m + log(s);
    }
    double a[OR_MAXK + 1];
    for (int k = 0; k < mu->K; ++k) {
        double q = 0.0, ls = 0.0;
        for (int i = 0; i < d; ++i) {
            double s = exp(mu->log_std[k * d + i]);
            double zz = (y[i] - mu->mean[k * d + i]) / s;
            q += zz * zz;
            ls += mu->log_std[k * d + i];
        }
        a[k] = log(1.0 - mu->beta) + mu->logit[k] - lse_logit
               - 0.5 * d * log(2.0 * M_PI) - ls - 0.5 * q;
    }
    a[mu->K] = in_box(d, y) ? log(mu->beta) : -INFINITY;
    return log_sum_exp(mu->K + 1, a);
}

/* Tile of a chain in tile-stratified runs: pixel ranges [r[0], r[1]) x
 * [r[2], r[3]).  Returns 0 when tiles are off. */
static int chain_tile(const or_config *cfg, uint32_t chain, int r[4])
{
    if (cfg->tile_px <= 0) return 0;
    int P = cfg->tile_px, W = cfg->image_w, H = cfg->image_h;
    int tx_n = (W + P - 1) / P, ty_n = (H + P - 1) / P;
    int64_t T = (int64_t)tx_n * ty_n;
    int64_t t = (int64_t)chain * T / cfg->n_chains_total;
    int tx = (int)(t % tx_n), ty = (int)(t / tx_n);
    r[0] = tx * P; r[1] = r[0] + P < W ? r[0] + P : W;
    r[2] = ty * P; r[3] = r[2] + P < H ? r[2] + P : H;
    return 1;
}

/* pixel of (x0, x1), as the image splats compute it; -1 off the box */
static int pixel_of(const or_config *cfg, const double *x, int *px, int *py)
{
    if (!(x[0] >= 0.0 && x[0] <= 1.0 && x[1] >= 0.0 && x[1] <= 1.0)) return 0;
    *px = (int)floor(x[0] * cfg->image_w);
    *py = (int)floor(x[1] * cfg->image_h);
    if (*px >= cfg->image_w) *px = cfg->image_w - 1;
    if (*py >= cfg->image_h) *py = cfg->image_h - 1;
    return 1;
}

/* log of the chain's target: p, or in tile-stratified runs p restricted to
 * the chain's tile */
static double log_target_c(const or_target *t, const or_config *cfg, uint32_t chain, const double *x, double *g)
{
    double lp = oracle_log_target(t, x, g);
    int r[4], px, py;
    if (cfg && chain_tile(cfg, chain, r)) {
        if (!pixel_of(cfg, x, &px, &py) || px < r[0] || px >= r[1] || py < r[2] || py >= r[3]) {
            if (g) for (int i = 0; i < t->d; ++i) g[i] = 0.0;
            return -INFINITY;
        }
    }
    return lp;
}

/* distance of y to the edge of the chain's support: the faces of the unit
 * box and, in tile-stratified runs, the edges of the chain's tile (parity
 * bookkeeping: a proposal this close to the edge may fall on the other side
 * in float32) */
static double support_margin(const or_config *cfg, uint32_t chain, int d, const double *y)
{
    double m = INFINITY;
    for (int i = 0; i < d; ++i) m = fmin(m, fmin(fabs(y[i]), fabs(1.0 - y[i])));
    int r[4];
    if (chain_tile(cfg, chain, r)) {
        m = fmin(m, fmin(fabs(y[0] - (double)r[0] / cfg->image_w), fabs(y[0] - (double)r[1] / cfg->image_w)));
        m = fmin(m, fmin(fabs(y[1] - (double)r[2] / cfg->image_h), fabs(y[1] - (double)r[3] / cfg->image_h)));
    }
    return m;
}

/* y ~ mu from the step's category uniform and candidate uniforms; *margin
 * gets the distance of u_cat to the nearest category boundary (INFINITY for
 * uniform mu) */
static void sample_mu(const or_mu *mu, double u_cat, const double cand[OR_MAXD], double *y, double *margin)
{
    int d = mu->d;
    *margin = INFINITY;
    if (mu->kind == OR_MU_UNIFORM) {
        for (int i = 0; i < d; ++i) y[i] = cand[i];
        return;
    }
    /* categorical over (uniform, component 1..K) with probabilities
     * (beta, (1 - beta) pi_1, ..., (1 - beta) pi_K) */
    double m = -INFINITY, s = 0.0;
    for (int k = 0; k < mu->K; ++k) if (mu->logit[k] > m) m = mu->logit[k];
    for (int k = 0; k < mu->K; ++k) s += exp(mu->logit[k] - m);
    double cum = mu->beta;
    *margin = fabs(u_cat - cum);
    int pick = -1;
    for (int k = 0; k < mu->K; ++k) {
        double next = cum + (1.0 - mu->beta) * exp(mu->logit[k] - m) / s;
        if (k < mu->K - 1 && fabs(u_cat - next) < *margin) *margin = fabs(u_cat - next);
        if (pick < 0 && u_cat >= cum && u_cat < next) pick = k;
        cum = next;
    }
    if (u_cat < mu->beta) {
        for (int i = 0; i < d; ++i) y[i] = cand[i];
        return;
    }
    if (pick < 0) pick = mu->K - 1;
    double z[OR_MAXD];
    box_muller(d, cand, z);
    for (int i = 0; i < d; ++i)
        y[i] = mu->mean[pick * d + i] + exp(mu->log_std[pick * d + i]) * z[i];
}

/* ----------------------------------------------------------------------- */
/* one transition of Alg. 2                                                 */
/* ----------------------------------------------------------------------- */

/* the chain's mu: in tile-stratified runs the uniform mu on its tile */
static void sample_mu_c(const or_mu *mu, const or_config *cfg, uint32_t chain, double u_cat,
                        const double cand[OR_MAXD], double *y, double *margin)
{
    sample_mu(mu, u_cat, cand, y, margin);
    int r[4];
    if (chain_tile(cfg, chain, r)) {
        y[0] = (double)(fmaf((float)(r[1] - r[0]), (float)cand[0], (float)r[0]) / (float)cfg->image_w);
        y[1] = (double)(fmaf((float)(r[3] - r[2]), (float)cand[1], (float)r[2]) / (float)cfg->image_h);
    }
}

typedef struct {
    double x[OR_MAXD];
    double lp, lu;   /* log p(x); log u(x), or log u_eff(x) for the unadjusted jump process */
    double g[OR_MAXD];
} or_state;

/* log (Q^T p)(x) for the unadjusted random-walk jump process with jump
 * N(0, sigma^2 I): the density at x of y + sigma z with y ~ p on the box,
 * (Q^T p)(x) = int_box p(y) N(x; y, sigma^2 I) dy.  Needs a mixture whose
 * components have diagonal covariances; per component and coordinate the
 * Gaussian product identity
 *   N(y; m, v) N(x; y, s) = N(x; m, v + s) N(y; c, t),
 *   c = (m s + x v) / (v + s),   t = v s / (v + s),
 * leaves the mass of N(c, t) on [0, 1]:
 *   (erf((1 - c) / sqrt(2 t)) + erf(c / sqrt(2 t))) / 2. */
double oracle_log_inflow(const or_target *t, double sigma, const double *x)
{
    int d = t->d;
    double s = sigma * sigma, a[OR_MAXK];
    for (int k = 0; k < t->K; ++k) {
        const double *m = t->mean + (size_t)k * d;
        const double *P = t->prec + (size_t)k * d * d;
        double ak = t->log_w[k];
        for (int i = 0; i < d; ++i) {
            double v = 1.0 / P[i * d + i];
            double c = (m[i] * s + x[i] * v) / (v + s);
            double r = sqrt(2.0 * v * s / (v + s));
            double dx = x[i] - m[i];
            ak += -0.5 * log(2.0 * M_PI * (v + s)) - 0.5 * dx * dx / (v + s)
                  + log(0.5 * (erf((1.0 - c) / r) + erf(c / r)));
        }
        a[k] = ak;
    }
    return log_sum_exp(t->K, a);
}

/* log u_eff(x), u_eff = u + (Q^T p - p) / c_tilde: the killing rate of
 * eq. (killing-rate) is then k = c_tilde u_eff / p.  NAN where u_eff < 0. */
double oracle_log_u_eff(const or_target *t, const or_mu *mu, double sigma, double c_tilde, const double *x,
                        double lp)
{
    double u = exp(oracle_log_mu(mu, x));
    double q = exp(oracle_log_inflow(t, sigma, x));
    double p = lp == -INFINITY ? 0.0 : exp(lp);
    double ue = u + (q - p) / c_tilde;
    return ue >= 0.0 ? log(ue) : NAN;
}

/* the cached second density of a state: log u, or log u_eff for the
 * unadjusted jump process */
static double state_lu(const or_target *t, const or_mu *mu, const or_local *lk, const or_config *cfg,
                       const double *x, double lp)
{
    if (lk && lk->kind == OR_LOCAL_RW_UNADJUSTED)
        return oracle_log_u_eff(t, mu, lk->step, cfg->c_tilde, x, lp);
    return oracle_log_mu(mu, x);
}

/* log q(a -> b) of the local proposal, up to the constant that cancels in
 * the acceptance ratio */
static double log_q(const or_local *lk, int d, const double *a, const double *ga, const double *b)
{
    if (lk->kind == OR_LOCAL_RWMH) return 0.0;   /* symmetric */
    double e = lk->step, s = 0.0;
    for (int i = 0; i < d; ++i) {
        double r = b[i] - a[i] - 0.5 * e * e * ga[i];
        s += r * r;
    }
    return -s / (2.0 * e * e);
}

/* Leapfrog integration of dq/dt = rho, drho/dt = grad log p(q) (unit
 * mass): half a momentum step, then n position steps separated by full
 * momentum steps, then half a momentum step.  On entry g holds
 * grad log p(q); on return q, rho, *lp = log p(q) and g are those of the
 * end point.  Off the support the gradient is taken as 0.  Returns 0 if a
 * visited point has p = 0 (the trajectory is then rejected). */
static int leapfrog_c(const or_target *t, const or_config *cfg, uint32_t chain, int n, double e, double *q,
                      double *rho, double *lp, double *g)
{
    int d = t->d, inside = 1;
    for (int i = 0; i < d; ++i) rho[i] += 0.5 * e * g[i];
    for (int l = 0; l < n; ++l) {
        for (int i = 0; i < d; ++i) q[i] += e * rho[i];
        *lp = log_target_c(t, cfg, chain, q, g);
        if (*lp == -INFINITY) inside = 0;
        double h = (l == n - 1) ? 0.5 * e : e;
        for (int i = 0; i < d; ++i) rho[i] += h * g[i];
    }
    return inside;
}

int oracle_leapfrog(const or_target *t, int n, double e, double *q, double *rho, double *lp, double *g)
{
    return leapfrog_c(t, NULL, 0, n, e, q, rho, lp, g);
}

/* Initial state: x_0 ~ mu (purpose INIT, step 0). */
void oracle_init_state(const or_target *t, const or_mu *mu, const or_local *lk, const or_config *cfg,
                       uint32_t chain, or_state *st)
{
    double head[4], cand[OR_MAXD], margin;
    draw_step(cfg, t->d, 0, chain, OR_PURPOSE_INIT, head, cand);
    sample_mu_c(mu, cfg, chain, head[3], cand, st->x, &margin);
    st->lp = log_target_c(t, cfg, chain, st->x, st->g);
    st->lu = state_lu(t, mu, lk, cfg, st->x, st->lp);
}

/* One Jump Restore transition from st at step `step`.
 * Returns dt; *flags gets KILL / ACCEPT / OUTSIDE bits; margins[0] is
 * ln t2 - ln t1 (kill iff <= 0), margins[1] is ln u_acc - ln(ratio)
 * (accept iff < 0; NAN when no acceptance test was made), margins[2] is the
 * distance of the category uniform to the nearest mu category boundary
 * (INFINITY unless a learned mu was sampled), margins[3] and margins[4] are
 * log p and log u at the local proposal (NAN when none was made), margins[5]
 * and margins[6] log p and log u of the state the step starts from,
 * margins[7] the distance of a small-step proposal to the edge of the
 * support (INFINITY when none was made). */
double oracle_transition(const or_target *t, const or_mu *mu, const or_local *lk,
                         const or_config *cfg, uint32_t step, uint32_t chain,
                         or_state *st, int32_t *flags, double margins[8])
{
    int d = t->d;
    double head[4], cand[OR_MAXD];
    draw_step(cfg, d, step, chain, OR_PURPOSE_STEP, head, cand);

    /* t1 ~ Exp(1): holding time; t2 ~ Exp(k(x)): time to termination */
    double t1 = -log(head[0]);
    double e2 = -log(head[1]);
    double t2, log_k;
    if (cfg->c_tilde == 0.0) { log_k = -INFINITY; t2 = INFINITY; }
    else if (st->lp == -INFINITY) { log_k = INFINITY; t2 = 0.0; }
    else if (isnan(st->lu)) { log_k = NAN; t2 = NAN; }   /* negative killing rate */
    else { log_k = log(cfg->c_tilde) + st->lu - st->lp; t2 = e2 * exp(-log_k); }
    margins[0] = log(e2) - log_k - log(t1);
    margins[1] = NAN;
    margins[2] = INFINITY;
    margins[3] = NAN;
    margins[4] = NAN;
    margins[5] = st->lp;
    margins[6] = st->lu;
    margins[7] = INFINITY;

    int32_t fl = isnan(t2) ? OR_FLAG_NEGATIVE_RATE : 0;
    double dt;
    if (t1 < t2) {
        /* local state transition: one MH update, with the large-step kernel
           (proposal mu) with probability l, else with the small-step kernel */
        dt = t1;
        int large = 0;
        if (lk->large_step_prob > 0.0) {
            double ul[4];
            draw_block(cfg, step, chain, OR_PURPOSE_LARGE, 0, ul);
            large = ul[0] < lk->large_step_prob;
        }
        double z[OR_MAXD], y[OR_MAXD], gy[OR_MAXD];
        int hmc = !large && lk->kind == OR_LOCAL_HMC, inside = 1;
        double kinetic = 0.0;   /* HMC: |rho_0|^2 / 2 - |rho_n|^2 / 2 */
        if (large) {
            fl |= OR_FLAG_LARGE;
            sample_mu_c(mu, cfg, chain, head[3], cand, y, &margins[2]);
        } else if (hmc) {
            box_muller(d, cand, z);
            double rho[OR_MAXD], lq;
            for (int i = 0; i < d; ++i) { y[i] = st->x[i]; rho[i] = z[i]; gy[i] = st->g[i]; }
            inside = leapfrog_c(t, cfg, chain, lk->n_leapfrog, lk->step, y, rho, &lq, gy);
            for (int i = 0; i < d; ++i) kinetic += 0.5 * (z[i] * z[i] - rho[i] * rho[i]);
        } else {
            box_muller(d, cand, z);
            for (int i = 0; i < d; ++i) {
                y[i] = st->x[i] + lk->step * z[i];
                if (lk->kind == OR_LOCAL_MALA) y[i] += 0.5 * lk->step * lk->step * st->g[i];
            }
        }
        if (!in_box(d, y)) fl |= OR_FLAG_OUTSIDE;
        if (!large) margins[7] = support_margin(cfg, chain, d, y);
        double lpy = log_target_c(t, cfg, chain, y, gy);
        double luy = large ? oracle_log_mu(mu, y) : state_lu(t, mu, lk, cfg, y, lpy);
        double alpha, lratio;
        if (st->lp == -INFINITY || (!large && lk->kind == OR_LOCAL_RW_UNADJUSTED)) {
            /* alpha = 1 where p(x) q(x, y) = 0; the unadjusted jump is always taken */
            alpha = 1.0; lratio = INFINITY;
        } else {
            if (large)   /* independence proposal: q(x, y) = u(y) */
                lratio = (lpy + st->lu) - (st->lp + luy);
            else if (hmc)   /* leapfrog is volume-preserving and reversible */
                lratio = inside ? (lpy - st->lp) + kinetic : -INFINITY;
            else
                lratio = lpy + log_q(lk, d, y, gy, st->x) - st->lp - log_q(lk, d, st->x, st->g, y);
            alpha = lratio >= 0.0 ? 1.0 : exp(lratio);
        }
        margins[1] = log(head[2]) - lratio;
        margins[3] = lpy;
        margins[4] = luy;
        if (head[2] < alpha) {
            fl |= OR_FLAG_ACCEPT;
            for (int i = 0; i < d; ++i) { st->x[i] = y[i]; st->g[i] = gy[i]; }
            st->lp = lpy;
            st->lu = luy;
        }
    } else {
        /* termination: regenerate from mu */
        dt = t2;
        fl |= OR_FLAG_KILL;
        sample_mu_c(mu, cfg, chain, head[3], cand, st->x, &margins[2]);
        st->lp = log_target_c(t, cfg, chain, st->x, st->g);
        st->lu = state_lu(t, mu, lk, cfg, st->x, st->lp);
    }
    *flags = fl;
    if (cfg->rb_dt) {
        /* dt = min(t1, t2) is Exp(1 + k) whichever clock fires, so its
           conditional mean given x can replace it in every time integral */
        if (cfg->c_tilde == 0.0) return 1.0;
        if (log_k == INFINITY) return 0.0;
        return 1.0 / (1.0 + exp(log_k));
    }
    return dt;
}

/* Batched single transitions for parity tests: n independent (state, step,
 * chain) triples.  x/g are [n][d] row-major. */
void oracle_transitions(const or_target *t, const or_mu *mu, const or_local *lk,
                        const or_config *cfg, int64_t n, const uint32_t *steps,
                        const uint32_t *chains, double *x, double *lp, double *lu,
                        double *g, int recompute, double *dt, int32_t *flags,
                        double *margins)
{
    int d = t->d;
    for (int64_t c = 0; c < n; ++c) {
        or_state st;
        for (int i = 0; i < d; ++i) st.x[i] = x[c * d + i];
        if (recompute) {
            st.lp = log_target_c(t, cfg, chains[c], st.x, st.g);
            st.lu = state_lu(t, mu, lk, cfg, st.x, st.lp);
        } else {
            st.lp = lp[c]; st.lu = lu[c];
            for (int i = 0; i < d; ++i) st.g[i] = g[c * d + i];
        }
        dt[c] = oracle_transition(t, mu, lk, cfg, steps[c], chains[c], &st, &flags[c], &margins[8 * c]);
        for (int i = 0; i < d; ++i) { x[c * d + i] = st.x[i]; g[c * d + i] = st.g[i]; }
        lp[c] = st.lp; lu[c] = st.lu;
    }
}

void oracle_init_states(const or_target *t, const or_mu *mu, const or_local *lk, const or_config *cfg,
                        int64_t n, const uint32_t *chains, double *x, double *lp,
                        double *lu, double *g)
{
    int d = t->d;
    for (int64_t c = 0; c < n; ++c) {
        or_state st;
        oracle_init_state(t, mu, lk, cfg, chains[c], &st);
        for (int i = 0; i < d; ++i) { x[c * d + i] = st.x[i]; g[c * d + i] = st.g[i]; }
        lp[c] = st.lp; lu[c] = st.lu;
    }
}

/* ----------------------------------------------------------------------- */
/* whole runs                                                               */
/* ----------------------------------------------------------------------- */

/* Per-chain results of a run. */
typedef struct {
    int64_t *n_done;      /* completed tours                         */
    double *t_done;       /* sum of completed tour lifetimes          */
    double *a_done;       /* sum over completed tours of int f = p dt */
    int32_t *censored;    /* 1 if the tour in flight hit the cap      */
    double *t_censored;   /* lifetime so far of a censored tour        */
    int64_t *transitions; /* steps executed                           */
    int64_t *accepts;     /* accepted local moves                     */
    int64_t *kills;       /* terminations                             */
    double *image;        /* [image_h * image_w], summed dt splats, or NULL */
    int64_t *large_steps;   /* large-step proposals (l > 0)            */
    int64_t *large_accepts; /* accepted large steps                    */
    /* Parity bookkeeping (each may be NULL).  min_margin[4 c + j]: over all
     * of the chain's steps (a burn-in included), the smallest |kill margin| / (1 + |log p(x)| +
     * |log u(x)|) (j = 0), |accept margin| / (1 + |log p(x)| + |log u(x)| +
     * |log p(y)| + |log u(y)|) (j = 1) -- margins of a decision scaled by
     * the size of the log densities it compares -- and the smallest
     * category margin (j = 2), and the smallest distance of a small-step
     * proposal to the edge of the support divided by (moves + 1) (j = 3;
     * moves: accepted local moves since the state was last drawn from mu,
     * each of which may round the float32 state once more).
     * image_count: splats per pixel.
     * image_near: the dt of every splat whose state lies within
     * (moves + 1) 2^-21 of a pixel edge (moves: accepted local moves since
     * the state was last drawn from mu), added to the 3 x 3 pixels around
     * its pixel. */
    double *min_margin;
    double *image_count;
    double *image_near;
} or_outputs;

typedef struct {
    const or_target *t; const or_mu *mu; const or_local *lk; const or_config *cfg;
    int64_t c0, c1;
    int32_t n_steps, drain_cap;
    const or_outputs *out;
    double *image;  /* this thread's image */
    double *image_count, *image_near;
} or_job;

static void run_chain(const or_job *job, int64_t c)
{
    const or_target *t = job->t; const or_config *cfg = job->cfg;
    or_state st;
    oracle_init_state(t, job->mu, job->lk, cfg, (uint32_t)c, &st);
    double a_cur = 0.0, t_cur = 0.0, a_done = 0.0, t_done = 0.0;
    int64_t n_done = 0, trans = 0, acc = 0, kills = 0, large = 0, large_acc = 0, moves = 0;
    double mm[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    int alive = 1;
    /* c_tilde = 0: the MH chain has no tours, so nothing is drained; the
       first burn_in steps are not accumulated */
    const int mh = cfg->c_tilde == 0.0;
    int64_t s_end = (int64_t)job->n_steps + (mh ? 0 : job->drain_cap);
    for (int64_t s = 0; s < s_end; ++s) {
        int drain = s >= job->n_steps;
        if (drain && !alive) break;
        int counted = !mh || s >= cfg->burn_in;
        /* the pair (dt, x_{i-1}) is recorded before the state moves */
        double x_prev[OR_MAXD];
        memcpy(x_prev, st.x, sizeof(double) * t->d);
        double lp_prev = st.lp;
        or_state before = st;
        int32_t fl; double mg[8];
        double dt = oracle_transition(t, job->mu, job->lk, cfg, (uint32_t)s, (uint32_t)c, &st, &fl, mg);
        {
            /* every step counts here, the burn-in's too: a decision there
               shapes the rest of the trajectory */
            double sx = 1.0 + fabs(before.lp) + fabs(before.lu);
            if (isfinite(mg[0]) && isfinite(sx) && fabs(mg[0]) / sx < mm[0]) mm[0] = fabs(mg[0]) / sx;
            double sy = sx + fabs(mg[3]) + fabs(mg[4]);
            if (isfinite(mg[1]) && isfinite(sy) && fabs(mg[1]) / sy < mm[1]) mm[1] = fabs(mg[1]) / sy;
            if (mg[2] < mm[2]) mm[2] = mg[2];
            if (mg[7] / (double)(moves + 1) < mm[3]) mm[3] = mg[7] / (double)(moves + 1);
        }
        if (!counted) continue;
        ++trans;
        double f = lp_prev == -INFINITY ? 0.0 : exp(lp_prev);
        if (mh) {
            t_done += dt;
            if (cfg->integrand_p) a_done += dt * f;
        } else {
            t_cur += dt;
            if (cfg->integrand_p) a_cur += dt * f;
        }
        if (job->image) {
            int px = (int)floor(x_prev[0] * cfg->image_w);
            int py = (int)floor(x_prev[1] * cfg->image_h);
            if (x_prev[0] >= 0.0 && x_prev[0] <= 1.0 && x_prev[1] >= 0.0 && x_prev[1] <= 1.0) {
                if (px >= cfg->image_w) px = cfg->image_w - 1;
                if (py >= cfg->image_h) py = cfg->image_h - 1;
                job->image[(size_t)py * cfg->image_w + px] += dt;
                if (job->image_count) job->image_count[(size_t)py * cfg->image_w + px] += 1.0;
                if (job->image_near) {
                    double ex = fabs(x_prev[0] * cfg->image_w - floor(x_prev[0] * cfg->image_w + 0.5)) / cfg->image_w;
                    double ey = fabs(x_prev[1] * cfg->image_h - floor(x_prev[1] * cfg->image_h + 0.5)) / cfg->image_h;
                    if (fmin(ex, ey) < (double)(moves + 1) * ldexp(1.0, -21)) {
                        for (int qy = py - 1; qy <= py + 1; ++qy)
                            for (int qx = px - 1; qx <= px + 1; ++qx)
                                if (qx >= 0 && qy >= 0 && qx < cfg->image_w && qy < cfg->image_h)
                                    job->image_near[(size_t)qy * cfg->image_w + qx] += dt;
                    }
                }
            }
        }
        if (fl & OR_FLAG_ACCEPT) { ++acc; ++moves; }
        if (fl & OR_FLAG_LARGE) { ++large; if (fl & OR_FLAG_ACCEPT) ++large_acc; }
        if (fl & OR_FLAG_KILL) {
            ++kills;
            a_done += a_cur; t_done += t_cur; ++n_done;
            a_cur = 0.0; t_cur = 0.0;
            moves = 0;
            if (drain) { alive = 0; st = before; }  /* retire: no regeneration */
        }
    }
    if (mh) alive = 0;
    const or_outputs *o = job->out;
    o->n_done[c] = n_done; o->t_done[c] = t_done; o->a_done[c] = a_done;
    o->censored[c] = alive ? 1 : 0;
    o->t_censored[c] = alive ? t_cur : 0.0;
    o->transitions[c] = trans; o->accepts[c] = acc; o->kills[c] = kills;
    if (o->large_steps) o->large_steps[c] = large;
    if (o->large_accepts) o->large_accepts[c] = large_acc;
    if (o->min_margin) for (int j = 0; j < 4; ++j) o->min_margin[4 * c + j] = mm[j];
}

static void *run_job(void *arg)
{
    const or_job *job = (const or_job *)arg;
    for (int64_t c = job->c0; c < job->c1; ++c) run_chain(job, c);
    return NULL;
}

/* Run chains [c0, c1) for n_steps steps plus the drain, over n_threads
 * threads.  Per-chain outputs are indexed by (chain - c0). */
int oracle_run(const or_target *t, const or_mu *mu, const or_local *lk,
               const or_config *cfg, int64_t c0, int64_t c1, int32_t n_steps,
               int32_t drain_cap, int32_t n_threads, const or_outputs *out)
{
    if (n_threads < 1) n_threads = 1;
    int64_t n = c1 - c0;
    if (n <= 0) return 0;
    if (n_threads > n) n_threads = (int32_t)n;
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    or_job *jobs = (or_job *)calloc((size_t)n_threads, sizeof(or_job));
    size_t npix = (size_t)cfg->image_w * (size_t)cfg->image_h;
    or_outputs shifted = *out;
    /* shift outputs so run_chain can index by global chain id */
    shifted.n_done -= c0; shifted.t_done -= c0; shifted.a_done -= c0;
    shifted.censored -= c0; shifted.t_censored -= c0; shifted.transitions -= c0;
    shifted.accepts -= c0; shifted.kills -= c0;
    if (shifted.large_steps) shifted.large_steps -= c0;
    if (shifted.large_accepts) shifted.large_accepts -= c0;
    if (shifted.min_margin) shifted.min_margin -= 4 * c0;
    for (int i = 0; i < n_threads; ++i) {
        jobs[i].t = t; jobs[i].mu = mu; jobs[i].lk = lk; jobs[i].cfg = cfg;
        jobs[i].c0 = c0 + n * i / n_threads;
        jobs[i].c1 = c0 + n * (i + 1) / n_threads;
        jobs[i].n_steps = n_steps; jobs[i].drain_cap = drain_cap;
        jobs[i].out = &shifted;
        jobs[i].image = (out->image && npix) ? (double *)calloc(npix, sizeof(double)) : NULL;
        jobs[i].image_count = (out->image_count && npix) ? (double *)calloc(npix, sizeof(double)) : NULL;
        jobs[i].image_near = (out->image_near && npix) ? (double *)calloc(npix, sizeof(double)) : NULL;
        pthread_create(&th[i], NULL, run_job, &jobs[i]);
    }
    for (int i = 0; i < n_threads; ++i) {
        pthread_join(th[i], NULL);
        if (jobs[i].image) {
            for (size_t p = 0; p < npix; ++p) out->image[p] += jobs[i].image[p];
            free(jobs[i].image);
        }
        if (jobs[i].image_count) {
            for (size_t p = 0; p < npix; ++p) out->image_count[p] += jobs[i].image_count[p];
            free(jobs[i].image_count);
        }
        if (jobs[i].image_near) {
            for (size_t p = 0; p < npix; ++p) out->image_near[p] += jobs[i].image_near[p];
            free(jobs[i].image_near);
        }
    }
    free(th); free(jobs);
    return 0;
}
