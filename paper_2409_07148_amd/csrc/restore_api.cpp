// Host runtime of the C ABI declared in include/restore.h: descriptor
// validation, float64 parameter factorisation and float32 packing, the
// structure-of-arrays layout of the caller's state buffer, kernel launches
// and the float64 estimates with their delta-method standard errors.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "trace.h"
#include "../../include/restore.h"
#include "launch.h"
#include "restore_internal.h"

using namespace restore;

namespace {

thread_local std::string g_last_error;

restore_status fail(restore_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

restore_status hip_fail(hipError_t e, const char *what) {
    return fail(RESTORE_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr int RED_BLOCKS = 1024;
constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    size_t x, logp, logu, grad, a_cur, t_cur, last_dt, a_done, t_done, n_done, status;
    size_t list0, list1, counts, counters, params, mu, partials, results;
    size_t bin_pix, bin_val, bin_count, bin_partial, img_tours, tile_results, rand, img_fx, total;
};

// Small populations (fewer than 2^16 chains: a few waves, each step a long
// serial instruction stream) with the uniform mu: the state-independent
// random inputs of every step -- Philox blocks, the clocks' logarithms,
// Box-Muller -- come from a chip-wide pre-pass, `chunk` steps at a time, into
// one half of a buffer of 2 x rand_fields(d) x chunk x C floats (at most
// 32 MiB per half).  Each step launch reads one half while its extra
// workgroups fill the other with the next chunk (which the next step
// launch or the drain then finds ready).  The chains are the same either
// way.  Off for the MH chain, the image integrand, the learned mu,
// LDS-staged parameters and RESTORE_FLAG_INLINE_RNG.
struct RandPlan {
    int chunk = 0;   // steps per pre-pass (0: off)
    int fields = 0;
};

// Binned splats (image integrand): bands of 2^SPLAT_BAND_SHIFT pixels, each
// with a bucket for 1.5 times its even share of one launch's records (at
// most n_chains (SPLAT_LAUNCH_STEPS + 1)); records beyond a full bucket go to
// the image directly.  RESTORE_FLAG_SPLAT_TIGHT shrinks the buckets 64-fold.
// n_bins = 0: splats go straight to the image.
struct SplatPlan {
    int n_bins = 0;
    int n_slices = 0;
    int64_t cap = 0;
    int64_t n_pix = 0;   // pixels of all batch images (binned or fixed-point runs)
    int batches = 0;     // image batches (0: no image)
    bool fixed = false;  // RESTORE_FLAG_IMAGE_FIXED: direct splats into u64 sums
    // tile-stratified runs: tiles of tile_px x tile_px pixels, tiles_x per
    // row, n_tiles in all (0: off)
    int tile_px = 0, tiles_x = 0, n_tiles = 0;
};

int image_batches_of(const restore_config *cfg) { return cfg->image_batches > 1 ? cfg->image_batches : 1; }

SplatPlan splat_plan(const restore_config *cfg, int tgt) {
    SplatPlan sp;
    if (tgt != TGT_PSS || !(cfg->integrands & RESTORE_INTEGRAND_PIXEL)) return sp;
    sp.batches = image_batches_of(cfg);
    if (cfg->tile_px > 0) {
        // tile-stratified: splats go to each workgroup's LDS copy of its tile
        sp.tile_px = cfg->tile_px;
        sp.tiles_x = (cfg->image_w + cfg->tile_px - 1) / cfg->tile_px;
        sp.n_tiles = sp.tiles_x * ((cfg->image_h + cfg->tile_px - 1) / cfg->tile_px);
        return sp;
    }
    const int64_t n_pix = (int64_t)cfg->image_w * cfg->image_h * sp.batches;
    if (cfg->flags & RESTORE_FLAG_IMAGE_FIXED) {
        // fixed-point sums: every splat goes straight to its u64 pixel
        sp.fixed = true;
        sp.n_pix = n_pix;
        return sp;
    }
    // the MH chain's kernel splats directly
    if ((cfg->flags & RESTORE_FLAG_SPLAT_DIRECT) || cfg->c_tilde == 0.0) return sp;
    const int64_t band = 1LL << SPLAT_BAND_SHIFT;
    const int64_t n_bins = (n_pix + band - 1) / band;
    const int64_t records = cfg->n_chains * (int64_t)(SPLAT_LAUNCH_STEPS + 1);
    if (n_bins > SPLAT_MAX_BANDS || records >= (1LL << 31)) return sp;
    int64_t cap = (3 * records + 2 * n_bins - 1) / (2 * n_bins);
    if (cfg->flags & RESTORE_FLAG_SPLAT_TIGHT) cap = std::max<int64_t>(64, cap / 64);
    sp.n_bins = (int)n_bins;
    // about 512 accumulation workgroups per launch
    sp.n_slices = (int)std::max<int64_t>(1, std::min<int64_t>(SPLAT_MAX_SLICES, 512 / n_bins));
    sp.cap = cap;
    sp.n_pix = n_pix;
    return sp;
}

constexpr int64_t RAND_HALF_BYTES = 32LL << 20;

RandPlan rand_plan(const restore_config *cfg, int tgt, int d, int mu) {
    RandPlan rp;
    if (cfg->n_chains >= (1LL << 16) || mu != MU_UNIFORM || tgt == TGT_PSS || cfg->c_tilde == 0.0 ||
        (cfg->flags & (RESTORE_FLAG_INLINE_RNG | RESTORE_FLAG_PARAMS_LDS)))
        return rp;
    const int64_t per_step = cfg->n_chains * (int64_t)rand_fields(d) * (int64_t)sizeof(float);
    const int64_t chunk = std::min<int64_t>(256, RAND_HALF_BYTES / per_step);
    if (chunk < 16) return rp;
    rp.chunk = (int)chunk;
    rp.fields = rand_fields(d);
    return rp;
}

int n_param_floats(int tgt, int loc, int d, int K) {
    if (tgt == TGT_PSS) return PSS_SLAB;
    return comp_stride(tgt, d) * K + (loc == LOC_RWU ? INFLOW_STRIDE * K : 0);
}

Layout make_layout(int64_t C, int d, bool grad, int n_params, int n_mu_floats, const SplatPlan &sp,
                   const RandPlan &rp) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    const size_t c = (size_t)C;
    L.x = take(4 * c * d);
    L.logp = take(4 * c);
    L.logu = take(4 * c);
    L.grad = grad ? take(4 * c * d) : (size_t)-1;
    L.a_cur = take(4 * c);
    L.t_cur = take(4 * c);
    L.last_dt = take(4 * c);
    L.a_done = take(8 * c);
    L.t_done = take(8 * c);
    L.n_done = take(4 * c);
    L.status = take(4 * c);
    L.list0 = take(4 * c);
    L.list1 = take(4 * c);
    L.counts = take(4 * 4);
    L.counters = take(8 * (size_t)CNT_SPREAD * CNT_LINE);
    L.params = take(4 * (size_t)n_params);
    L.mu = n_mu_floats > 0 ? take(4 * (size_t)n_mu_floats) : (size_t)-1;
    L.partials = take(8 * (size_t)RED_BLOCKS * RED_SLOTS);
    L.results = take(8 * RED_SLOTS);
    const size_t nb = (size_t)sp.n_bins;
    L.bin_pix = nb ? take(4 * nb * (size_t)sp.cap) : (size_t)-1;
    L.bin_val = nb ? take(4 * nb * (size_t)sp.cap) : (size_t)-1;
    L.bin_count = nb ? take(4 * (size_t)SPLAT_MAX_BANDS * SPLAT_COUNTER_STRIDE) : (size_t)-1;
    L.bin_partial = nb ? take(4 * (size_t)sp.n_slices * (nb << SPLAT_BAND_SHIFT)) : (size_t)-1;
    L.img_tours = sp.batches ? take(8 * (size_t)sp.batches * std::max(1, sp.n_tiles)) : (size_t)-1;
    L.tile_results = sp.n_tiles ? take(8 * (size_t)sp.n_tiles * TR_SLOTS) : (size_t)-1;
    L.rand = rp.chunk ? take(2 * 4 * (size_t)rp.fields * (size_t)rp.chunk * c) : (size_t)-1;
    L.img_fx = sp.fixed ? take(8 * (size_t)sp.n_pix) : (size_t)-1;
    L.total = o;
    return L;
}

struct Validated {
    int tgt, d, K, loc, mu;
    double step;   // jump sigma of the unadjusted random-walk process (LOC_RWU)
};

bool all_finite(const double *p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

restore_status validate(const restore_target *t, const restore_mu *mu, const restore_local_kernel *lk,
                        const restore_config *cfg, Validated *v) {
    if (!t || !mu || !lk || !cfg) return fail(RESTORE_E_INVALID_ARG, "null descriptor");
    if (t->kind != RESTORE_TARGET_GMM_ISO && t->kind != RESTORE_TARGET_GMM_FULL && t->kind != RESTORE_TARGET_PSS)
        return fail(RESTORE_E_INVALID_ARG, "unknown target kind %d", t->kind);
    if (t->dim < 1 || t->dim > RESTORE_MAX_DIM)
        return fail(RESTORE_E_INVALID_ARG, "dim %d outside 1..%d", t->dim, RESTORE_MAX_DIM);
    const int d = t->dim, K = t->n_comp;
    int64_t need = 0;
    if (t->kind == RESTORE_TARGET_PSS) {
        if (d != 12) return fail(RESTORE_E_INVALID_ARG, "the PSS target has dim 12");
        need = 16 + 8 + 8 + 48 + 8 + 8 + 9 + 3 + 3 + 1;
    } else {
        if (K < 1 || K > RESTORE_MAX_COMP)
            return fail(RESTORE_E_INVALID_ARG, "n_comp %d outside 1..%d", K, RESTORE_MAX_COMP);
        need = t->kind == RESTORE_TARGET_GMM_ISO ? (int64_t)K * (2 + d) : (int64_t)K * (1 + d + d * d);
    }
    if (!t->params) return fail(RESTORE_E_INVALID_ARG, "null target params");
    if (t->params_count != need)
        return fail(RESTORE_E_INVALID_ARG, "target params: %lld doubles given, %lld expected",
                    (long long)t->params_count, (long long)need);
    if (!all_finite(t->params, need)) return fail(RESTORE_E_NONFINITE, "non-finite target parameter");
    if (mu->kind != RESTORE_MU_UNIFORM_BOX && mu->kind != RESTORE_MU_GMM_DIAG)
        return fail(RESTORE_E_INVALID_ARG, "unknown mu kind %d", mu->kind);
    if (mu->kind == RESTORE_MU_GMM_DIAG) {
        if (mu->n_comp < 1 || mu->n_comp > RESTORE_MAX_COMP || !mu->params_dev)
            return fail(RESTORE_E_INVALID_ARG, "GMM_DIAG mu needs 1..%d components and device params",
                        RESTORE_MAX_COMP);
        if (!(mu->beta >= 0.0f && mu->beta <= 1.0f)) return fail(RESTORE_E_INVALID_ARG, "mu beta outside [0,1]");
    }
    if (lk->kind != RESTORE_LOCAL_RWMH && lk->kind != RESTORE_LOCAL_MALA && lk->kind != RESTORE_LOCAL_HMC &&
        lk->kind != RESTORE_LOCAL_RW_UNADJUSTED)
        return fail(RESTORE_E_INVALID_ARG, "unknown local kernel %d", lk->kind);
    if (!std::isfinite(lk->step) || lk->step < 0.0f) return fail(RESTORE_E_INVALID_ARG, "step must be >= 0");
    if (lk->kind != RESTORE_LOCAL_RWMH && !(lk->step > 0.0f))
        return fail(RESTORE_E_INVALID_ARG, "MALA, HMC and the unadjusted jump process need step > 0");
    if (lk->kind == RESTORE_LOCAL_RW_UNADJUSTED) {
        // Q^T p in closed form needs diagonal covariances; the killing rate
        // (c_tilde u + L* p) / p needs c_tilde > 0; only the uniform mu is built
        if (t->kind != RESTORE_TARGET_GMM_ISO || mu->kind != RESTORE_MU_UNIFORM_BOX)
            return fail(RESTORE_E_UNSUPPORTED,
                        "the unadjusted random-walk jump process is built for the isotropic mixture with uniform mu");
        if (!(cfg->c_tilde > 0.0))
            return fail(RESTORE_E_INVALID_ARG, "the unadjusted random-walk jump process needs c_tilde > 0");
    }
    if (lk->kind == RESTORE_LOCAL_HMC ? (lk->n_leapfrog < 1 || lk->n_leapfrog > 64) : lk->n_leapfrog != 0)
        return fail(RESTORE_E_INVALID_ARG, "n_leapfrog must be 1..64 for HMC and 0 otherwise");
    if (!(lk->large_step_prob >= 0.0f && lk->large_step_prob <= 1.0f))
        return fail(RESTORE_E_INVALID_ARG, "large_step_prob outside [0,1]");
    if (cfg->n_chains < 1 || cfg->n_chains > 0x7fffffffLL)
        return fail(RESTORE_E_INVALID_ARG, "n_chains %lld outside 1..2^31-1", (long long)cfg->n_chains);
    if (cfg->first_chain < 0) return fail(RESTORE_E_INVALID_ARG, "first_chain must be >= 0");
    if (cfg->first_chain > 0 && cfg->tile_px != 0)
        return fail(RESTORE_E_UNSUPPORTED, "first_chain > 0 with tile_px: the chain-to-tile map spans the whole population");
    if (!std::isfinite(cfg->c_tilde) || cfg->c_tilde < 0.0) return fail(RESTORE_E_INVALID_ARG, "c_tilde must be >= 0");
    if (lk->large_step_prob != 0.0f && cfg->c_tilde > 0.0)
        return fail(RESTORE_E_UNSUPPORTED,
                    "restore runs the small-step chain M^0: large_step_prob must be 0 unless c_tilde = 0 (MH chain)");
    if (cfg->drain_cap < 0) return fail(RESTORE_E_INVALID_ARG, "drain_cap must be >= 0");
    if (cfg->block_size != 0 && (cfg->block_size < 64 || cfg->block_size > 256 || cfg->block_size % 64))
        return fail(RESTORE_E_INVALID_ARG, "block_size must be a multiple of 64 in 64..256");
    if (cfg->integrands & RESTORE_INTEGRAND_PIXEL) {
        if (cfg->image_w < 1 || cfg->image_h < 1 || (int64_t)cfg->image_w * cfg->image_h > (1LL << 28))
            return fail(RESTORE_E_INVALID_ARG, "image size must be >= 1 and at most 2^28 pixels");
        if (t->kind != RESTORE_TARGET_PSS)
            return fail(RESTORE_E_UNSUPPORTED, "pixel splats are built for the rendering-shaped target");
        if (cfg->image_batches < 0 || cfg->image_batches > 4096)
            return fail(RESTORE_E_INVALID_ARG, "image_batches must be in 0..4096");
        if ((int64_t)cfg->image_w * cfg->image_h * std::max(1, cfg->image_batches) > 0x7fffffffLL)
            return fail(RESTORE_E_INVALID_ARG, "image_batches x image pixels must stay below 2^31");
        if ((int64_t)std::max(1, cfg->image_batches) > cfg->n_chains)
            return fail(RESTORE_E_INVALID_ARG, "more image batches than chains");
    } else if (cfg->image_batches > 1) {
        return fail(RESTORE_E_INVALID_ARG, "image_batches needs the PIXEL integrand");
    }
    if (cfg->flags & RESTORE_FLAG_IMAGE_FIXED) {
        if (!(cfg->integrands & RESTORE_INTEGRAND_PIXEL))
            return fail(RESTORE_E_INVALID_ARG, "RESTORE_FLAG_IMAGE_FIXED needs the PIXEL integrand");
        if (cfg->tile_px != 0)
            return fail(RESTORE_E_UNSUPPORTED, "RESTORE_FLAG_IMAGE_FIXED is built for untiled runs");
    }
    if (cfg->tile_px != 0) {
        if (cfg->tile_px < 1 || cfg->tile_px > 64) return fail(RESTORE_E_INVALID_ARG, "tile_px must be in 0..64");
        if (!(cfg->integrands & RESTORE_INTEGRAND_PIXEL))
            return fail(RESTORE_E_INVALID_ARG, "tile-stratified runs need the PIXEL integrand");
        if (mu->kind != RESTORE_MU_UNIFORM_BOX || cfg->c_tilde == 0.0)
            return fail(RESTORE_E_UNSUPPORTED, "tile-stratified runs are restore runs with the uniform mu");
        const int64_t T = (int64_t)((cfg->image_w + cfg->tile_px - 1) / cfg->tile_px) *
                          ((cfg->image_h + cfg->tile_px - 1) / cfg->tile_px);
        if (cfg->n_chains / T < std::max(1, cfg->image_batches))
            return fail(RESTORE_E_INVALID_ARG, "every tile needs at least max(1, image_batches) chains (%lld tiles)",
                        (long long)T);
    }
    v->tgt = t->kind == RESTORE_TARGET_GMM_ISO ? TGT_ISO : t->kind == RESTORE_TARGET_GMM_FULL ? TGT_FULL : TGT_PSS;
    v->d = d;
    v->K = t->kind == RESTORE_TARGET_PSS ? 0 : K;
    v->loc = lk->kind == RESTORE_LOCAL_MALA ? LOC_MALA
             : lk->kind == RESTORE_LOCAL_HMC ? LOC_HMC
             : lk->kind == RESTORE_LOCAL_RW_UNADJUSTED ? LOC_RWU : LOC_RWMH;
    v->step = lk->step;
    v->mu = mu->kind == RESTORE_MU_GMM_DIAG ? MU_GMM : MU_UNIFORM;
    return RESTORE_OK;
}

// A natural log-weight as the slab's base-2 term (the mixture densities'
// layout in restore_internal.h): scaled by log2 e, -inf floored at -2^100 so
// that the kernels' log-sum-exp never subtracts two infinities.
float log_weight2(double ln_w) {
    const double v = ln_w * M_LOG2E;
    return v > -0x1p100 ? (float)v : -0x1p100f;
}

// Float64 factorisation of the canonical parameters into the float32 slab.
restore_status pack_params(const restore_target *t, const Validated &v, std::vector<float> *out) {
    const int d = v.d, K = v.K;
    const double *p = t->params;
    const double LN2PI = std::log(2.0 * M_PI);
    if (v.tgt == TGT_ISO) {
        const int S = comp_stride(TGT_ISO, d);
        out->assign((size_t)n_param_floats(v.tgt, v.loc, d, K), 0.0f);
        const double *w = p, *m = p + K, *s = p + K + (size_t)K * d;
        const double j2 = v.step * v.step;
        for (int k = 0; k < K; ++k) {
            if (!(w[k] >= 0.0) || !(s[k] > 0.0)) return fail(RESTORE_E_INVALID_ARG, "weights >= 0, sigmas > 0");
            float *o = out->data() + (size_t)k * S;
            o[0] = log_weight2(std::log(w[k]) - 0.5 * d * (LN2PI + 2.0 * std::log(s[k])));
            for (int i = 0; i < d; ++i) o[1 + i] = (float)m[(size_t)k * d + i];
            o[1 + d] = (float)(0.5 * M_LOG2E / (s[k] * s[k]));
            if (v.loc == LOC_RWU) {
                // Q^T p terms (layout in restore_internal.h)
                const double s2 = s[k] * s[k], tot = s2 + j2, alpha = s2 / tot;
                float *q = out->data() + (size_t)K * S + (size_t)k * INFLOW_STRIDE;
                q[0] = (float)(std::log(w[k]) - 0.5 * d * (LN2PI + std::log(tot)));
                q[1] = (float)(1.0 / tot);
                q[2] = (float)alpha;
                q[3] = (float)(1.0 / std::sqrt(2.0 * alpha * j2));
            }
        }
        return RESTORE_OK;
    }
    if (v.tgt == TGT_FULL) {
        const int S = comp_stride(TGT_FULL, d);
        out->assign((size_t)S * K, 0.0f);
        const double *w = p, *m = p + K, *cov = p + K + (size_t)K * d;
        std::vector<double> L((size_t)d * d), W((size_t)d * d);
        for (int k = 0; k < K; ++k) {
            if (!(w[k] >= 0.0)) return fail(RESTORE_E_INVALID_ARG, "mixture weights must be >= 0");
            const double *A = cov + (size_t)k * d * d;
            // Cholesky A = L L^T
            std::fill(L.begin(), L.end(), 0.0);
            double logdiag = 0.0;
            for (int j = 0; j < d; ++j) {
                double s = A[j * d + j];
                for (int q = 0; q < j; ++q) s -= L[j * d + q] * L[j * d + q];
                if (!(s > 0.0)) return fail(RESTORE_E_INVALID_ARG, "covariance %d is not positive definite", k);
                L[j * d + j] = std::sqrt(s);
                logdiag += std::log(L[j * d + j]);
                for (int i = j + 1; i < d; ++i) {
                    double r = A[i * d + j];
                    for (int q = 0; q < j; ++q) r -= L[i * d + q] * L[j * d + q];
                    L[i * d + j] = r / L[j * d + j];
                }
            }
            // W = L^-1 (lower triangular), column by column
            std::fill(W.begin(), W.end(), 0.0);
            for (int c = 0; c < d; ++c) {
                for (int i = c; i < d; ++i) {
                    double r = (i == c) ? 1.0 : 0.0;
                    for (int q = c; q < i; ++q) r -= L[i * d + q] * W[q * d + c];
                    W[i * d + c] = r / L[i * d + i];
                }
            }
            float *o = out->data() + (size_t)k * S;
            o[0] = log_weight2(std::log(w[k]) - 0.5 * d * LN2PI - logdiag);
            for (int i = 0; i < d; ++i) o[1 + i] = (float)m[(size_t)k * d + i];
            const double scale = std::sqrt(0.5 * M_LOG2E);
            int at = 1 + d;
            for (int i = 0; i < d; ++i)
                for (int j = 0; j <= i; ++j) o[at++] = (float)(scale * W[i * d + j]);
        }
        return RESTORE_OK;
    }
    // rendering-shaped integrand: see the slab layout in restore_internal.h
    out->assign(PSS_SLAB, 0.0f);
    float *o = out->data();
    const double *nA = p, *aA = p + 16, *phA = p + 24, *nB = p + 32, *aB = p + 80, *phB = p + 88;
    const double *dir = p + 96, *kap = p + 105, *wl = p + 108, b = p[111];
    double sa = 0.0, sb = 0.0;
    for (int m = 0; m < 8; ++m) { sa += std::fabs(aA[m]); sb += std::fabs(aB[m]); }
    if (!(sa < 8.0 && sb < 8.0)) return fail(RESTORE_E_INVALID_ARG, "texture amplitudes must keep t > 0");
    for (int i = 0; i < 16; ++i) {
        if (nA[i] != std::floor(nA[i])) return fail(RESTORE_E_INVALID_ARG, "texture frequencies must be integers");
        o[i] = (float)nA[i];
    }
    for (int i = 0; i < 48; ++i) {
        if (nB[i] != std::floor(nB[i])) return fail(RESTORE_E_INVALID_ARG, "texture frequencies must be integers");
        o[32 + i] = (float)nB[i];
    }
    auto frac = [](double x) { return x - std::floor(x); };
    for (int m = 0; m < 8; ++m) {
        o[16 + m] = (float)(aA[m] / 8.0);
        o[24 + m] = (float)frac(phA[m] / (2.0 * M_PI));
        o[80 + m] = (float)(aB[m] / 8.0);
        o[88 + m] = (float)frac(phB[m] / (2.0 * M_PI));
    }
    for (int l = 0; l < 3; ++l) {
        const double n2 = dir[3 * l] * dir[3 * l] + dir[3 * l + 1] * dir[3 * l + 1] + dir[3 * l + 2] * dir[3 * l + 2];
        if (std::fabs(n2 - 1.0) > 1e-9) return fail(RESTORE_E_INVALID_ARG, "lobe directions must be unit vectors");
        if (!(kap[l] > 0.0) || !(wl[l] >= 0.0)) return fail(RESTORE_E_INVALID_ARG, "kappa > 0 and w >= 0");
        for (int i = 0; i < 3; ++i) o[96 + 3 * l + i] = (float)dir[3 * l + i];
        o[105 + l] = (float)kap[l];
        // ln(4 pi w kappa / (2 pi (1 - e^{-2 kappa}))) = ln(2 w kappa / (1 - e^{-2 kappa}))
        o[108 + l] = wl[l] > 0.0 ? (float)std::log(2.0 * wl[l] * kap[l] / -std::expm1(-2.0 * kap[l])) : -INFINITY;
    }
    if (!(b >= 0.0)) return fail(RESTORE_E_INVALID_ARG, "base level b must be >= 0");
    o[111] = (float)b;
    return RESTORE_OK;
}

// Learned mu slab (layout in restore_internal.h) from logits, means and log
// standard deviations, in float64.
restore_status pack_mu(const std::vector<float> &raw, int K, int d, float beta, std::vector<float> *out) {
    for (float f : raw)
        if (!std::isfinite(f)) return fail(RESTORE_E_NONFINITE, "non-finite learned mu parameter");
    const float *logit = raw.data(), *mean = logit + K, *lstd = mean + (size_t)K * d;
    double mx = -INFINITY;
    for (int k = 0; k < K; ++k) mx = std::max(mx, (double)logit[k]);
    double den = 0.0;
    for (int k = 0; k < K; ++k) den += std::exp((double)logit[k] - mx);
    const double b = beta;
    const int S = mu_stride(d);
    out->assign((size_t)mu_slab_floats(d, K), 0.0f);
    float *o = out->data();
    o[0] = b > 0.0 ? (float)std::log2(b) : -INFINITY;
    const double scale = std::sqrt(0.5 * M_LOG2E);
    double cum = b;
    for (int k = 0; k < K; ++k) {
        const double pk = std::exp((double)logit[k] - mx) / den;
        double c = (b < 1.0 ? std::log1p(-b) : -INFINITY) + std::log(pk) - 0.5 * d * std::log(2.0 * M_PI);
        float *ck = o + 4 + (size_t)k * S;
        float *ms = o + 4 + (size_t)K * S + K + (size_t)k * 2 * d;
        for (int i = 0; i < d; ++i) {
            const double ls = lstd[(size_t)k * d + i];
            // n from the float32 r: fma(y, r, n) is then (y - m) r up to
            // the one rounding of n
            const float r = (float)(scale * std::exp(-ls));
            c -= ls;
            ck[i] = r;
            ck[d + i] = (float)(-(double)mean[(size_t)k * d + i] * (double)r);
            ms[i] = mean[(size_t)k * d + i];
            ms[d + i] = (float)std::exp(ls);
        }
        ck[2 * d] = log_weight2(c);
        o[4 + (size_t)K * S + k] = (float)cum;
        cum += (1.0 - b) * pk;
    }
    return RESTORE_OK;
}

}  // namespace

// Entry points shared with the batched runtime (batch_api.cpp).
restore_status restore_internal_fail(restore_status code, const char *msg) { return fail(code, "%s", msg); }

restore_status restore_internal_pack_mu(const std::vector<float> &raw, int K, int d, float beta,
                                        std::vector<float> *out) {
    return pack_mu(raw, K, d, beta, out);
}

restore_status restore_internal_pack_full(const restore_target *t, std::vector<float> *out) {
    Validated v{};
    v.tgt = TGT_FULL;
    v.d = t->dim;
    v.K = t->n_comp;
    v.loc = LOC_RWMH;
    v.mu = MU_UNIFORM;
    return pack_params(t, v, out);
}

struct restore_ctx {
    Validated v{};
    restore_config cfg{};
    KernelSet ks{};
    Layout lay{};
    char *base = nullptr;
    int n_params = 0;
    int block = 256;
    bool lds = false;
    bool drained = false;
    bool mh = false;            // c_tilde = 0: the MH chain M^l
    int32_t steps_taken = 0;
    float step = 0.0f;
    float large_prob = 0.0f;
    int32_t n_leapfrog = 0;
    float *image = nullptr;
    restore_mu mu{};
    SplatPlan splat{};
    RandPlan rand{};
    // pre-pass buffer: half pre_half holds the inputs of steps
    // [pre_s0, pre_s0 + pre_n) (pre_n = 0: nothing yet)
    int pre_half = 0;
    int64_t pre_s0 = 0;
    int32_t pre_n = 0;
    StepArgs args{};
};

namespace {

template <typename T>
T *at(restore_ctx *c, size_t off) {
    return off == (size_t)-1 ? nullptr : reinterpret_cast<T *>(c->base + off);
}

void fill_args(restore_ctx *c) {
    StepArgs &a = c->args;
    a.x = at<float>(c, c->lay.x);
    a.logp = at<float>(c, c->lay.logp);
    a.logu = at<float>(c, c->lay.logu);
    a.grad = at<float>(c, c->lay.grad);
    a.a_cur = at<float>(c, c->lay.a_cur);
    a.t_cur = at<float>(c, c->lay.t_cur);
    a.last_dt = at<float>(c, c->lay.last_dt);
    a.a_done = at<double>(c, c->lay.a_done);
    a.t_done = at<double>(c, c->lay.t_done);
    a.n_done = at<uint32_t>(c, c->lay.n_done);
    a.status = at<uint32_t>(c, c->lay.status);
    a.counters = at<unsigned long long>(c, c->lay.counters);
    a.params = at<float>(c, c->lay.params);
    a.mu_params = c->v.mu == MU_GMM ? at<float>(c, c->lay.mu) : nullptr;
    a.image = c->image;
    a.list = nullptr;
    a.list_count = nullptr;
    a.n_chains = c->cfg.n_chains;
    a.n_comp = c->v.K;
    a.mu_comp = c->mu.n_comp;
    a.mu_beta = c->mu.beta;
    a.no_kill = c->cfg.c_tilde == 0.0 ? 1 : 0;
    a.log_c = c->cfg.c_tilde > 0.0 ? (float)std::log(c->cfg.c_tilde) : 0.0f;
    a.step = c->step;
    a.large_prob = c->large_prob;
    a.n_leapfrog = c->n_leapfrog;
    a.key0 = (uint32_t)(c->cfg.seed & 0xffffffffu);
    a.key1 = (uint32_t)(c->cfg.seed >> 32);
    a.target_id = (uint32_t)c->cfg.target_id;
    a.chain0 = (uint32_t)c->cfg.first_chain;
    a.s0 = 0;
    a.n_steps = 0;
    a.integrand_p = (c->cfg.integrands & RESTORE_INTEGRAND_P) ? 1 : 0;
    a.rb_dt = (c->cfg.flags & RESTORE_FLAG_RB_DT) ? 1 : 0;
    a.image_w = c->cfg.image_w;
    a.image_h = c->cfg.image_h;
    a.image_batches = image_batches_of(&c->cfg);
    a.image_pixels = c->cfg.image_w * c->cfg.image_h;
    a.tile_px = c->splat.tile_px;
    a.tiles_x = c->splat.tiles_x;
    a.n_tiles = c->splat.n_tiles;
    a.rec_x = nullptr;
    a.rec_w = nullptr;
    a.rec_chains = 0;
    a.bin_pix = at<uint32_t>(c, c->lay.bin_pix);
    a.bin_val = at<float>(c, c->lay.bin_val);
    a.bin_count = at<uint32_t>(c, c->lay.bin_count);
    a.bin_cap = (int32_t)c->splat.cap;
    a.n_bins = c->splat.n_bins;
    a.image_fx = c->splat.fixed ? at<unsigned long long>(c, c->lay.img_fx) : nullptr;
}

// Dynamic LDS bytes of a step or drain launch (mu_lds_offset in
// restore_internal.h): staged target parameters, then the learned mu's
// component blocks and cumulative weights.
size_t kernel_lds_bytes(const restore_ctx *c, bool params_lds) {
    size_t floats = (size_t)mu_lds_offset(params_lds, c->n_params);
    if (c->v.mu == MU_GMM) floats += (size_t)c->mu.n_comp * (size_t)(mu_stride(c->v.d) + 1);
    return floats * sizeof(float);
}

// Half h of the pre-pass buffer.
float *rand_half(restore_ctx *c, int h) {
    return at<float>(c, c->lay.rand) + (size_t)h * c->rand.fields * (size_t)c->rand.chunk * c->cfg.n_chains;
}

// Make the current half of the pre-pass buffer hold steps [s, s + n)
// (n <= chunk): kept from the previous step launch if it drew them, else
// drawn by a pre-pass launch.
restore_status ensure_pre(restore_ctx *c, int64_t s, int32_t n, hipStream_t stream) {
    if (n <= 0 || (c->pre_n > 0 && c->pre_s0 == s && c->pre_n >= n)) return RESTORE_OK;
    StepArgs a = c->args;
    a.s0 = (uint32_t)s;
    a.n_steps = n;
    float *buf = rand_half(c, c->pre_half);
    int chunk = c->rand.chunk;
    void *pargs[] = {&a, &buf, &chunk};
    hipError_t e = hipLaunchKernel(c->ks.rand_prepass, dim3((unsigned)((c->cfg.n_chains + 255) / 256), (unsigned)n),
                                   dim3(256), pargs, 0, stream);
    if (e != hipSuccess) return hip_fail(e, "random pre-pass launch");
    c->pre_s0 = s;
    c->pre_n = n;
    return RESTORE_OK;
}

// Fixed-point image runs: the caller's float image from the u64 sums.
hipError_t publish_fixed_image(restore_ctx *c, hipStream_t s) {
    if (!c->splat.fixed) return hipSuccess;
    return launch_image_from_fixed(c->args.image_fx, c->image, c->splat.n_pix, s);
}

dim3 grid_for(int64_t n, int block) { return dim3((unsigned)((n + block - 1) / block)); }

__global__ void zero_u32_kernel(uint32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void zero_f32_kernel(float *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ void reset_sums_kernel(float *a_cur, float *t_cur, double *a_done, double *t_done, uint32_t *n_done,
                                  int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        a_cur[i] = 0.0f;
        t_cur[i] = 0.0f;
        a_done[i] = 0.0;
        t_done[i] = 0.0;
        n_done[i] = 0u;
    }
}

}  // namespace

extern "C" {

const char *restore_last_error(void) { return g_last_error.c_str(); }

restore_status restore_state_bytes(const restore_target *target, const restore_mu *mu,
                                   const restore_local_kernel *local, const restore_config *cfg,
                                   size_t *bytes_out) {
    if (!bytes_out) return fail(RESTORE_E_INVALID_ARG, "null bytes_out");
    Validated v;
    restore_status st = validate(target, mu, local, cfg, &v);
    if (st != RESTORE_OK) return st;
    *bytes_out = make_layout(cfg->n_chains, v.d, uses_grad(v.loc), n_param_floats(v.tgt, v.loc, v.d, v.K),
                             v.mu == MU_GMM ? mu_slab_floats(v.d, mu->n_comp) : 0, splat_plan(cfg, v.tgt),
                             rand_plan(cfg, v.tgt, v.d, v.mu)).total;
    return RESTORE_OK;
}

restore_status restore_init(restore_ctx **out, const restore_target *target, const restore_mu *mu,
                            const restore_local_kernel *local, const restore_config *cfg, void *state_dev,
                            size_t state_bytes, float *image_dev, void *stream) {
    restore::TraceRange trace_range("restore_init");
    if (!out) return fail(RESTORE_E_INVALID_ARG, "null out");
    *out = nullptr;
    Validated v;
    restore_status st = validate(target, mu, local, cfg, &v);
    if (st != RESTORE_OK) return st;
    if (!state_dev) return fail(RESTORE_E_INVALID_ARG, "null state buffer");
    if (reinterpret_cast<uintptr_t>(state_dev) % ALIGN)
        return fail(RESTORE_E_INVALID_ARG, "state buffer must be 256-byte aligned");
    if ((cfg->integrands & RESTORE_INTEGRAND_PIXEL) && !image_dev)
        return fail(RESTORE_E_INVALID_ARG, "pixel integrand needs an image buffer");
    const int n_params = n_param_floats(v.tgt, v.loc, v.d, v.K);
    const int n_mu = v.mu == MU_GMM ? mu_slab_floats(v.d, mu->n_comp) : 0;
    const SplatPlan sp = splat_plan(cfg, v.tgt);
    const RandPlan rp = rand_plan(cfg, v.tgt, v.d, v.mu);
    const Layout lay = make_layout(cfg->n_chains, v.d, uses_grad(v.loc), n_params, n_mu, sp, rp);
    if (state_bytes < lay.total)
        return fail(RESTORE_E_BUFFER_TOO_SMALL, "state buffer holds %zu bytes, %zu needed", state_bytes, lay.total);
    KernelSet ks = find_kernels(v.tgt, v.d, v.loc, v.mu);
    if (!ks.step) return fail(RESTORE_E_UNSUPPORTED, "no kernels built for target %d, dim %d, local %d, mu %d",
                              v.tgt, v.d, v.loc, v.mu);
    std::vector<float> slab;
    st = pack_params(target, v, &slab);
    if (st != RESTORE_OK) return st;

    restore_ctx *c = new (std::nothrow) restore_ctx();
    if (!c) return fail(RESTORE_E_INVALID_ARG, "out of host memory");
    c->v = v;
    c->cfg = *cfg;
    c->ks = ks;
    c->lay = lay;
    c->base = static_cast<char *>(state_dev);
    c->n_params = n_params;
    // default: 256 threads; populations too small to give every CU a
    // workgroup of 256 (fewer than 2^16 chains) run one wave per workgroup,
    // which spreads their few waves over more CUs (their runs are latency-bound)
    c->block = cfg->block_size ? cfg->block_size : (cfg->n_chains < (1LL << 16) ? 64 : 256);
    c->lds = (cfg->flags & RESTORE_FLAG_PARAMS_LDS) != 0;
    c->step = local->step;
    c->mh = cfg->c_tilde == 0.0;
    c->large_prob = local->large_step_prob;
    c->n_leapfrog = local->n_leapfrog;
    c->image = (cfg->integrands & RESTORE_INTEGRAND_PIXEL) ? image_dev : nullptr;
    c->mu = *mu;
    c->splat = sp;
    c->rand = ks.step_pre ? rp : RandPlan{};
    fill_args(c);

    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(const_cast<float *>(c->args.params), slab.data(), slab.size() * sizeof(float),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) { delete c; return hip_fail(e, "parameter upload"); }
    std::vector<float> mu_slab;
    if (v.mu == MU_GMM) {
        // the learned mu is frozen for the run: read the caller's parameters
        // once and factorise them in float64
        const int K = mu->n_comp, d = v.d;
        std::vector<float> raw((size_t)K * (1 + 2 * d));
        e = hipMemcpyAsync(raw.data(), mu->params_dev, raw.size() * sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { delete c; return hip_fail(e, "mu parameter read"); }
        st = pack_mu(raw, K, d, mu->beta, &mu_slab);
        if (st != RESTORE_OK) { delete c; return st; }
        e = hipMemcpyAsync(at<float>(c, c->lay.mu), mu_slab.data(), mu_slab.size() * sizeof(float),
                           hipMemcpyHostToDevice, s);
        if (e != hipSuccess) { delete c; return hip_fail(e, "mu upload"); }
    }
    // the upload reads a host vector that goes away: finish it before returning
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) { delete c; return hip_fail(e, "parameter upload"); }
    hipLaunchKernelGGL(zero_u64_kernel, dim3(CNT_SPREAD * CNT_LINE / 256), dim3(256), 0, s, c->args.counters,
                       CNT_SPREAD * CNT_LINE);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, at<uint32_t>(c, c->lay.counts), 4);
    if (sp.n_bins)
        hipLaunchKernelGGL(zero_u32_kernel, dim3(SPLAT_MAX_BANDS * SPLAT_COUNTER_STRIDE / 256), dim3(256), 0, s,
                           c->args.bin_count, SPLAT_MAX_BANDS * SPLAT_COUNTER_STRIDE);
    if (sp.fixed)
        hipLaunchKernelGGL(zero_u64_kernel, grid_for(sp.n_pix, 256), dim3(256), 0, s, c->args.image_fx,
                           (int)sp.n_pix);
    StepArgs a = c->args;
    void *kargs[] = {&a};
    e = hipLaunchKernel(ks.init, grid_for(cfg->n_chains, 256), dim3(256), kargs, 0, s);
    if (e != hipSuccess) { delete c; return hip_fail(e, "init launch"); }
    *out = c;
    return RESTORE_OK;
}

static restore_status step_impl(restore_ctx *c, int32_t n_steps, int64_t n_record, float *x_out, float *w_out,
                                void *stream) {
    if (!c) return fail(RESTORE_E_INVALID_ARG, "null ctx");
    if (c->drained) return fail(RESTORE_E_BAD_STATE, "restore_step after restore_drain");
    if (n_steps < 0) return fail(RESTORE_E_INVALID_ARG, "n_steps must be >= 0");
    if ((int64_t)c->steps_taken + n_steps > 0x7fffffffLL - c->cfg.drain_cap)
        return fail(RESTORE_E_INVALID_ARG, "step counter would overflow");
    if (n_steps == 0) return RESTORE_OK;
    StepArgs a = c->args;
    a.s0 = (uint32_t)c->steps_taken;
    a.n_steps = n_steps;
    a.rec_x = x_out;
    a.rec_w = w_out;
    a.rec_chains = n_record;
    int np = c->n_params;
    void *kargs[] = {&a, &np};
    const size_t shm = kernel_lds_bytes(c, c->lds);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (c->mh) {
        // the MH chain: parameters through the scalar cache, direct splats
        hipError_t e = hipLaunchKernel(c->ks.step_mh, grid_for(c->cfg.n_chains, c->block), dim3(c->block), kargs,
                                       kernel_lds_bytes(c, false), s);
        if (e != hipSuccess) return hip_fail(e, "MH step launch");
    } else if (c->splat.n_tiles) {
        // tile-stratified: an LDS copy of the workgroup's tile takes the splats
        const size_t tile_shm = (size_t)c->splat.tile_px * c->splat.tile_px * sizeof(float);
        hipError_t e = hipLaunchKernel(c->ks.step_tiled, grid_for(c->cfg.n_chains, c->block), dim3(c->block), kargs,
                                       tile_shm, s);
        if (e != hipSuccess) return hip_fail(e, "tiled step launch");
    } else if (c->rand.chunk && !x_out) {
        // small population: per chunk, the steps reading their random inputs
        // from one half of the pre-pass buffer while extra workgroups of the
        // same launch fill the other half with the next chunk
        int chunk = c->rand.chunk;
        const int64_t step_blocks = (c->cfg.n_chains + c->block - 1) / c->block;
        const int64_t gen_blocks = step_blocks * ((chunk + PRE_GEN_STEPS - 1) / PRE_GEN_STEPS);
        for (int32_t done = 0; done < n_steps; done += chunk) {
            const int64_t s_first = c->steps_taken + done;
            a.s0 = (uint32_t)s_first;
            a.n_steps = std::min<int32_t>(chunk, n_steps - done);
            restore_status st = ensure_pre(c, s_first, a.n_steps, s);
            if (st != RESTORE_OK) return st;
            const float *cur = rand_half(c, c->pre_half);
            PreGen g{rand_half(c, 1 - c->pre_half), (uint32_t)(s_first + a.n_steps), chunk, (int32_t)step_blocks};
            void *sargs[] = {&a, &cur, &chunk, &g};
            hipError_t e = hipLaunchKernel(c->ks.step_pre, dim3((unsigned)(step_blocks + gen_blocks)),
                                           dim3(c->block), sargs, 0, s);
            if (e != hipSuccess) return hip_fail(e, "step launch");
            c->pre_half = 1 - c->pre_half;
            c->pre_s0 = s_first + a.n_steps;
            c->pre_n = chunk;
        }
    } else if (!c->splat.n_bins) {
        const void *fn = c->lds ? c->ks.step_lds : c->ks.step;
        hipError_t e = hipLaunchKernel(fn, grid_for(c->cfg.n_chains, c->block), dim3(c->block), kargs, shm, s);
        if (e != hipSuccess) return hip_fail(e, "step launch");
    } else {
        // binned splats: launches of at most SPLAT_LAUNCH_STEPS steps, each
        // followed by the accumulation of its bucketed records into the image
        const void *fn = c->lds ? c->ks.step_binned_lds : c->ks.step_binned;
        SplatArgs sa{};
        sa.pix = a.bin_pix;
        sa.val = a.bin_val;
        sa.count = a.bin_count;
        sa.partial = at<float>(c, c->lay.bin_partial);
        sa.image = c->image;
        sa.cap = (int32_t)c->splat.cap;
        sa.n_bins = c->splat.n_bins;
        sa.n_slices = c->splat.n_slices;
        sa.n_pix = c->splat.n_pix;
        for (int32_t done = 0; done < n_steps; done += SPLAT_LAUNCH_STEPS) {
            a.s0 = (uint32_t)(c->steps_taken + done);
            a.n_steps = std::min<int32_t>(SPLAT_LAUNCH_STEPS, n_steps - done);
            a.rec_x = x_out ? x_out + (int64_t)done * n_record * c->v.d : nullptr;
            a.rec_w = w_out ? w_out + (int64_t)done * n_record : nullptr;
            hipError_t e = hipLaunchKernel(fn, grid_for(c->cfg.n_chains, c->block), dim3(c->block), kargs, shm, s);
            if (e != hipSuccess) return hip_fail(e, "step launch");
            e = launch_splat_accumulate(sa, s);
            if (e != hipSuccess) return hip_fail(e, "splat accumulation launch");
        }
    }
    c->steps_taken += n_steps;
    hipError_t e = publish_fixed_image(c, s);
    if (e != hipSuccess) return hip_fail(e, "fixed-point image launch");
    return RESTORE_OK;
}

restore_status restore_step(restore_ctx *c, int32_t n_steps, void *stream) {
    restore::TraceRange trace_range("restore_step");
    return step_impl(c, n_steps, 0, nullptr, nullptr, stream);
}

restore_status restore_step_record(restore_ctx *c, int32_t n_steps, int64_t n_record, float *x_out, float *w_out,
                                   void *stream) {
    restore::TraceRange trace_range("restore_step_record");
    if (!c) return fail(RESTORE_E_INVALID_ARG, "null ctx");
    if (n_record < 1 || n_record > c->cfg.n_chains || !x_out || !w_out)
        return fail(RESTORE_E_INVALID_ARG, "n_record must be in 1..n_chains with non-null buffers");
    if (c->splat.n_tiles) return fail(RESTORE_E_UNSUPPORTED, "no sample recording in tile-stratified runs");
    return step_impl(c, n_steps, n_record, x_out, w_out, stream);
}

restore_status restore_drain(restore_ctx *c, void *stream) {
    restore::TraceRange trace_range("restore_drain");
    if (!c) return fail(RESTORE_E_INVALID_ARG, "null ctx");
    if (c->drained) return fail(RESTORE_E_BAD_STATE, "restore_drain called twice");
    if (c->mh) {
        // no tours in flight
        c->drained = true;
        return RESTORE_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (c->rand.chunk) {
        // small population: one launch over the whole cap, its first steps'
        // random inputs from the pre-pass buffer (usually drawn already by
        // the last step launch)
        const int32_t n_pre = std::min<int32_t>(c->rand.chunk, c->cfg.drain_cap);
        restore_status st = ensure_pre(c, c->steps_taken, n_pre, s);
        if (st != RESTORE_OK) return st;
        StepArgs a = c->args;
        a.s0 = (uint32_t)c->steps_taken;
        a.n_steps = c->cfg.drain_cap;
        const float *cur = rand_half(c, c->pre_half);
        int chunk = c->rand.chunk, np = n_pre;
        void *kargs[] = {&a, &cur, &chunk, &np};
        hipError_t e = hipLaunchKernel(c->ks.drain_pre, grid_for(c->cfg.n_chains, c->block), dim3(c->block), kargs,
                                       0, s);
        if (e != hipSuccess) return hip_fail(e, "drain launch");
        c->drained = true;
        return RESTORE_OK;
    }
    uint32_t *counts = at<uint32_t>(c, c->lay.counts);
    uint32_t *lists[2] = {at<uint32_t>(c, c->lay.list0), at<uint32_t>(c, c->lay.list1)};
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, counts, 4);
    const bool tiled = c->splat.n_tiles > 0;
    const void *fn = tiled ? c->ks.drain_tiled : c->lds ? c->ks.drain_lds : c->ks.drain;
    const size_t shm = tiled ? 0 : kernel_lds_bytes(c, c->lds);
    // chunks of 1, 2, 4, ... steps: survivors are compacted between chunks
    // while many chains retire, and the long tail takes few launches.  A
    // population below 2^16 chains has too few waves to fill the chip, so
    // the lanes a long chunk leaves idle cost nothing: one launch runs the
    // whole cap (each wave ends when its last lane retires) and saves the
    // launches and compactions.  Each chain takes the same steps either way.
    int32_t remaining = c->cfg.drain_cap;
    int64_t chunk = c->cfg.n_chains < (1LL << 16) ? std::max<int64_t>(1, c->cfg.drain_cap) : 1;
    uint32_t s0 = (uint32_t)c->steps_taken;
    for (int j = 0;; ++j) {
        const int32_t L = remaining < chunk ? remaining : (int32_t)chunk;
        const int last = (remaining - L) == 0 ? 1 : 0;
        StepArgs a = c->args;
        a.list = j == 0 ? nullptr : lists[(j - 1) % 2];
        a.list_count = j == 0 ? nullptr : counts + (j % 3);
        a.s0 = s0;
        a.n_steps = L;
        int np = c->n_params;
        uint32_t *list_out = lists[j % 2];
        uint32_t *count_out = counts + ((j + 1) % 3);
        uint32_t *count_zero = counts + ((j + 2) % 3);
        void *kargs[] = {&a, &np, &list_out, &count_out, &count_zero, (void *)&last};
        hipError_t e = hipLaunchKernel(fn, grid_for(c->cfg.n_chains, c->block), dim3(c->block), kargs, shm, s);
        if (e != hipSuccess) return hip_fail(e, "drain launch");
        s0 += (uint32_t)L;
        remaining -= L;
        if (last) break;
        chunk *= 2;
    }
    hipError_t e = publish_fixed_image(c, s);
    if (e != hipSuccess) return hip_fail(e, "fixed-point image launch");
    c->drained = true;
    return RESTORE_OK;
}

// Run counters summed over their spread copies (synchronises the stream).
static restore_status read_counters(restore_ctx *c, hipStream_t s, unsigned long long cnt[CNT_SLOTS]) {
    std::vector<unsigned long long> lines((size_t)CNT_SPREAD * CNT_LINE);
    hipError_t e = hipMemcpyAsync(lines.data(), c->args.counters, lines.size() * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "counter readback");
    for (int j = 0; j < CNT_SLOTS; ++j) cnt[j] = 0;
    for (int l = 0; l < CNT_SPREAD; ++l)
        for (int j = 0; j < CNT_SLOTS; ++j) cnt[j] += lines[(size_t)l * CNT_LINE + j];
    return RESTORE_OK;
}

// Stratified estimates of a tile-stratified run: tile t is a restore problem
// with constant c_tilde A_t (A_t its share of the box), so p_lambda =
// sum_t c_tilde A_t T_t / N_t and lambda(p f) = sum_t c_tilde A_t A_t' / N_t
// (Sec. 6.3 per tile); pi f is their ratio.  Standard errors: per tile the
// delta-method variances and covariance of the two tour ratios over the
// tile's chains, tiles independent, and the delta method for pi f.
static restore_status estimate_tiles(restore_ctx *c, restore_estimate_out *out, hipStream_t s) {
    const SplatPlan &sp = c->splat;
    TileReduceArgs r;
    r.a_done = c->args.a_done;
    r.t_done = c->args.t_done;
    r.n_done = c->args.n_done;
    r.status = c->args.status;
    r.t_cur = c->args.t_cur;
    r.n_chains = c->cfg.n_chains;
    r.n_tiles = sp.n_tiles;
    r.results = at<double>(c, c->lay.tile_results);
    hipError_t e = launch_tile_reduce(r, s);
    if (e != hipSuccess) return hip_fail(e, "tile reduce launch");
    std::vector<double> res((size_t)sp.n_tiles * TR_SLOTS);
    e = hipMemcpyAsync(res.data(), r.results, res.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "tile estimate readback");
    unsigned long long cnt[CNT_SLOTS];
    restore_status st = read_counters(c, s, cnt);
    if (st != RESTORE_OK) return st;
    const double ct = c->cfg.c_tilde, W = c->cfg.image_w, H = c->cfg.image_h;
    double P = 0, L = 0, vP = 0, vL = 0, cPL = 0, N = 0, T = 0, cens = 0, cens_t = 0, nonfin = 0;
    bool ok = true;
    for (int t = 0; t < sp.n_tiles; ++t) {
        const double *o = res.data() + (size_t)t * TR_SLOTS;
        const int tx = t % sp.tiles_x, ty = t / sp.tiles_x;
        const double w = std::min<double>(sp.tile_px, W - tx * sp.tile_px);
        const double h = std::min<double>(sp.tile_px, H - ty * sp.tile_px);
        const double st_ = ct * w * h / (W * H);
        const double n_ok = o[TR_CHAINS] - o[TR_NONFINITE];
        N += o[TR_N];
        T += o[TR_T];
        cens += o[TR_CENS];
        cens_t += o[TR_CENS_T];
        nonfin += o[TR_NONFINITE];
        if (!(o[TR_N] > 0) || n_ok < 2) {
            ok = false;
            continue;
        }
        P += st_ * o[TR_T] / o[TR_N];
        L += st_ * o[TR_A] / o[TR_N];
        const double den = (n_ok - 1) * n_ok * (o[TR_N] / n_ok) * (o[TR_N] / n_ok);
        vP += st_ * st_ * o[TR_SS_TT] / den;
        vL += st_ * st_ * o[TR_SS_AA] / den;
        cPL += st_ * st_ * o[TR_SS_TA] / den;
    }
    std::memset(out, 0, sizeof(*out));
    out->p_lambda = ok ? P : NAN;
    out->p_lambda_se = ok ? std::sqrt(vP) : NAN;
    out->lam_pf = ok ? L : NAN;
    out->lam_pf_se = ok ? std::sqrt(vL) : NAN;
    const double pi = L / P;
    out->pi_f = ok ? pi : NAN;
    out->pi_f_se = ok ? std::sqrt(std::max(0.0, (vL - 2 * pi * cPL + pi * pi * vP) / (P * P))) : NAN;
    out->tours_done = (int64_t)N;
    out->tours_censored = (int64_t)cens;
    out->transitions = (int64_t)cnt[CNT_TRANSITIONS];
    out->accepts = (int64_t)cnt[CNT_ACCEPTS];
    out->kills = (int64_t)cnt[CNT_KILLS];
    out->nonfinite = (int64_t)nonfin;
    out->censored_time_frac = T + cens_t > 0 ? cens_t / (T + cens_t) : 0.0;
    out->accept_rate = cnt[CNT_TRANSITIONS] ? (double)cnt[CNT_ACCEPTS] / (double)cnt[CNT_TRANSITIONS] : 0.0;
    out->kill_rate = cnt[CNT_TRANSITIONS] ? (double)cnt[CNT_KILLS] / (double)cnt[CNT_TRANSITIONS] : 0.0;
    out->image_scale = NAN;   // per tile: c_tilde A_t / j_t (restore_image_estimate applies it)
    return RESTORE_OK;
}

restore_status restore_estimate(restore_ctx *c, restore_estimate_out *out, void *stream) {
    restore::TraceRange trace_range("restore_estimate");
    if (!c || !out) return fail(RESTORE_E_INVALID_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (c->splat.n_tiles) return estimate_tiles(c, out, s);
    ReduceArgs r;
    r.a_done = c->args.a_done;
    r.t_done = c->args.t_done;
    r.n_done = c->args.n_done;
    r.status = c->args.status;
    r.t_cur = c->args.t_cur;
    r.n_chains = c->cfg.n_chains;
    r.partials = at<double>(c, c->lay.partials);
    r.results = at<double>(c, c->lay.results);
    const int64_t want = (c->cfg.n_chains + 255) / 256;
    r.n_blocks = (int32_t)(want < RED_BLOCKS ? want : RED_BLOCKS);
    hipError_t e = launch_reduce(r, s);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
    double res[RED_SLOTS];
    std::vector<unsigned long long> lines((size_t)CNT_SPREAD * CNT_LINE);
    e = hipMemcpyAsync(res, r.results, sizeof(res), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(lines.data(), c->args.counters, lines.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "estimate readback");
    unsigned long long cnt[CNT_SLOTS] = {};
    for (int l = 0; l < CNT_SPREAD; ++l)
        for (int j = 0; j < CNT_SLOTS; ++j) cnt[j] += lines[(size_t)l * CNT_LINE + j];

    const double N = res[RED_N], T = res[RED_T], A = res[RED_A];
    const double n_ok = (double)c->cfg.n_chains - res[RED_NONFINITE];
    const double ct = c->cfg.c_tilde;
    auto se = [&](double ss, double den_sum) -> double {
        if (n_ok < 2 || den_sum <= 0) return NAN;
        const double mean = den_sum / n_ok;
        return std::sqrt(ss / ((n_ok - 1) * n_ok)) / mean;
    };
    std::memset(out, 0, sizeof(*out));
    out->p_lambda = N > 0 ? ct * T / N : NAN;
    out->p_lambda_se = ct * se(res[RED_SS_T_N], N);
    out->lam_pf = N > 0 ? ct * A / N : NAN;
    out->lam_pf_se = ct * se(res[RED_SS_A_N], N);
    out->pi_f = T > 0 ? A / T : NAN;
    out->pi_f_se = se(res[RED_SS_A_T], T);
    out->tours_done = (int64_t)N;
    out->tours_censored = (int64_t)res[RED_CENS];
    out->transitions = (int64_t)cnt[CNT_TRANSITIONS];
    out->accepts = (int64_t)cnt[CNT_ACCEPTS];
    out->kills = (int64_t)cnt[CNT_KILLS];
    out->nonfinite = (int64_t)res[RED_NONFINITE];
    const double tot_t = T + res[RED_CENS_T];
    out->censored_time_frac = tot_t > 0 ? res[RED_CENS_T] / tot_t : 0.0;
    out->accept_rate = cnt[CNT_TRANSITIONS] ? (double)cnt[CNT_ACCEPTS] / (double)cnt[CNT_TRANSITIONS] : 0.0;
    out->kill_rate = cnt[CNT_TRANSITIONS] ? (double)cnt[CNT_KILLS] / (double)cnt[CNT_TRANSITIONS] : 0.0;
    out->image_scale = N > 0 ? ct / N : 0.0;
    out->large_steps = (int64_t)cnt[CNT_LARGE];
    out->large_accepts = (int64_t)cnt[CNT_LARGE_ACCEPTS];
    return RESTORE_OK;
}

restore_status restore_reset_sums(restore_ctx *c, void *stream) {
    restore::TraceRange trace_range("restore_reset_sums");
    if (!c) return fail(RESTORE_E_INVALID_ARG, "null ctx");
    if (!c->mh)
        return fail(RESTORE_E_BAD_STATE, "sums are reset only for the MH chain (c_tilde = 0): a restore tour in "
                                         "flight would lose its start");
    if (c->drained) return fail(RESTORE_E_BAD_STATE, "restore_reset_sums after restore_drain");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const StepArgs &a = c->args;
    hipLaunchKernelGGL(reset_sums_kernel, grid_for(c->cfg.n_chains, 256), dim3(256), 0, s, a.a_cur, a.t_cur,
                       a.a_done, a.t_done, a.n_done, (int64_t)c->cfg.n_chains);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(CNT_SPREAD * CNT_LINE / 256), dim3(256), 0, s, c->args.counters,
                       CNT_SPREAD * CNT_LINE);
    if (c->image) {
        const int64_t n = (int64_t)c->cfg.image_w * c->cfg.image_h * image_batches_of(&c->cfg);
        hipLaunchKernelGGL(zero_f32_kernel, grid_for(n, 256), dim3(256), 0, s, c->image, n);
        if (c->splat.fixed)
            hipLaunchKernelGGL(zero_u64_kernel, grid_for(n, 256), dim3(256), 0, s, c->args.image_fx, (int)n);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "reset launch");
    return RESTORE_OK;
}

restore_status restore_image_estimate(restore_ctx *c, float *mean_dev, float *se_dev, void *stream) {
    restore::TraceRange trace_range("restore_image_estimate");
    if (!c || !mean_dev || !se_dev) return fail(RESTORE_E_INVALID_ARG, "null argument");
    if (!c->image) return fail(RESTORE_E_BAD_STATE, "the run has no PIXEL integrand");
    ImageEstimateArgs a{};
    a.image = c->image;
    a.image_fx = c->args.image_fx;
    a.n_done = c->args.n_done;
    a.t_done = c->args.t_done;
    a.a_done = c->args.a_done;
    a.n_chains = c->cfg.n_chains;
    a.batches = image_batches_of(&c->cfg);
    a.n_pix = (int64_t)c->cfg.image_w * c->cfg.image_h;
    a.c_tilde = c->cfg.c_tilde;
    a.tours = at<double>(c, c->lay.img_tours);
    a.tile_px = c->splat.tile_px;
    a.tiles_x = c->splat.tiles_x;
    a.n_tiles = c->splat.n_tiles;
    a.image_w = c->cfg.image_w;
    a.image_h = c->cfg.image_h;
    a.mean = mean_dev;
    a.se = se_dev;
    hipError_t e = launch_image_estimate(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "image estimate launch");
    return RESTORE_OK;
}

restore_status restore_get_state_view(const restore_ctx *c, restore_state_view *v) {
    if (!c || !v) return fail(RESTORE_E_INVALID_ARG, "null argument");
    const StepArgs &a = c->args;
    v->x = a.x; v->logp = a.logp; v->logu = a.logu; v->grad = a.grad;
    v->a_cur = a.a_cur; v->t_cur = a.t_cur; v->last_dt = a.last_dt;
    v->a_done = a.a_done; v->t_done = a.t_done; v->n_done = a.n_done; v->status = a.status;
    v->n_chains = c->cfg.n_chains;
    v->dim = c->v.d;
    v->steps_taken = c->steps_taken;
    return RESTORE_OK;
}

restore_status restore_refresh_cache(restore_ctx *c, void *stream) {
    restore::TraceRange trace_range("restore_refresh_cache");
    if (!c) return fail(RESTORE_E_INVALID_ARG, "null ctx");
    StepArgs a = c->args;
    void *kargs[] = {&a};
    hipError_t e = hipLaunchKernel(c->ks.refresh, grid_for(c->cfg.n_chains, 256), dim3(256), kargs, 0,
                                   static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "refresh launch");
    return RESTORE_OK;
}

restore_status restore_destroy(restore_ctx *c) {
    delete c;
    return RESTORE_OK;
}

}  // extern "C"
