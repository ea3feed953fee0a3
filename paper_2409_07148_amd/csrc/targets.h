// Target densities p and regeneration densities u evaluated per lane.
//
// The Gaussian mixtures are evaluated in log space, in base 2 (log2 e is
// folded into the packed parameters on the host), with a blocked online
// log-sum-exp: a block of components' terms, one maximum over them and the
// running maximum, one exponential per term and one per block.  Neither far
// tails nor sharp peaks leave the float32 range.  Parameters are read from
// a packed slab whose addresses are wave-uniform: from global memory they
// become scalar loads (SGPR operands of the FMAs); with LDS staging they
// are broadcast reads.
#pragma once

#include <type_traits>

#include "../../include/restore.h"
#include "device_common.h"

namespace restore {

// Parameters read through the constant address space: wave-uniform loads
// from it always become scalar (SMEM) loads feeding SGPR operands, even
// when the kernel also writes global memory (image splats) that the
// compiler cannot prove disjoint from the slab.
typedef const __attribute__((address_space(4))) float *const_fptr;
// An LDS copy of read-only parameters (per-lane indexed reads are ds_reads).
typedef const __attribute__((address_space(3))) float *lds_fptr;

// Components per log-sum-exp block: four for values alone, two when the
// gradient needs each component's vector until the block's weights are
// known (fewer live registers), and fewer while the block's parameters
// (STRIDE floats per component, scalar operands of the FMAs) would take
// more than LSE_SGPR_BUDGET scalar registers at once: past that the
// compiler reloads and spills them, which costs more than the shared
// maximum saves.
// BMAX caps the block for kernels whose own state already crowds the
// scalar registers.
constexpr int LSE_SGPR_BUDGET = 96;
template <int STRIDE, bool GRAD, int BMAX = 4>
struct LseBlock {
    static constexpr int cap(int b) { return (b > 1 && b * STRIDE > LSE_SGPR_BUDGET) ? cap(b / 2) : b; }
    static constexpr int value = cap((GRAD ? 2 : 4) < BMAX ? (GRAD ? 2 : 4) : BMAX);
};

// Isotropic Gaussian mixture, slab terms in base 2 (h_k = log2 e / (2 s_k^2)):
//   a_k = c_k - h_k |y - m_k|^2 = log2(w_k N(y; m_k, s_k^2 I)),
//   grad log p = -2 ln 2 sum_k r_k h_k (y - m_k),  r = softmax of the a_k in base 2.
template <int D>
struct GmmIso {
    static constexpr int STRIDE = comp_stride(TGT_ISO, D);

    template <int B, bool GRAD, class PT>
    __device__ __forceinline__ static void push(PT P, int k0, const float y[D], float &M, float &S, float G[D],
                                                bool want) {
        float a[B], dx[B][D];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const auto pk = P + (k0 + b) * STRIDE;
            float q = 0.0f;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                dx[b][i] = y[i] - pk[1 + i];
                q = fmaf(dx[b][i], dx[b][i], q);
            }
            a[b] = pk[0] - pk[1 + D] * q;
        }
        float sc, w[B];
        lse2_block<B>(M, S, a, sc, w);
        if (GRAD && want) {
#pragma unroll
            for (int i = 0; i < D; ++i) G[i] *= sc;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const float wh = w[b] * P[(k0 + b) * STRIDE + 1 + D];
#pragma unroll
                for (int i = 0; i < D; ++i) G[i] = fmaf(wh, dx[b][i], G[i]);
            }
        }
    }

    template <bool GRAD, int BMAX = 4, class PT>
    __device__ __forceinline__ static float eval(PT P, int K, const float y[D], float g[D], bool want) {
        constexpr int B = LseBlock<STRIDE, GRAD, BMAX>::value;
        float M = -INFINITY, S = 0.0f;
        float G[D];
#pragma unroll
        for (int i = 0; i < D; ++i) G[i] = 0.0f;
        int k = 0;
        for (; k + B <= K; k += B) push<B, GRAD>(P, k, y, M, S, G, want);
        for (; k < K; ++k) push<1, GRAD>(P, k, y, M, S, G, want);
        if (GRAD && want) {
            const float f = (-2.0f * LN2) / S;
#pragma unroll
            for (int i = 0; i < D; ++i) g[i] = G[i] * f;
        }
        return lse2_ln(M, S);
    }
};

// log (Q^T p)(y) of the isotropic mixture for the unadjusted random-walk
// jump process with jump N(0, sigma^2 I): the density at y of x + sigma z
// with x ~ p on the box, (Q^T p)(y) = int_box p(x) N(y; x, sigma^2 I) dx.
// Per component and coordinate the Gaussian product identity leaves
// N(y_i; m_i, s^2 + sigma^2) times the box mass of a Gaussian centred at
// c_i = m_i + alpha (y_i - m_i) with 1 / sqrt(2 var) = beta:
//   (erf(beta (1 - c_i)) + erf(beta c_i)) / 2.
// The parameters (INFLOW_STRIDE per component) follow the K components.
template <int D>
struct GmmIsoInflow {
    template <class PT>
    __device__ __forceinline__ static float log_inflow(PT P, int K, const float y[D]) {
        const auto A = P + K * GmmIso<D>::STRIDE;
        float M = -INFINITY, S = 0.0f;
        // unrolled by four for wide scalar loads, as in GmmIso::eval
#pragma unroll 4
        for (int k = 0; k < K; ++k) {
            const auto pk = P + k * GmmIso<D>::STRIDE;
            const auto qk = A + k * INFLOW_STRIDE;
            const float ivar = qk[1], alpha = qk[2], beta = qk[3];
            float q = 0.0f, mass = 1.0f;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const float dx = y[i] - pk[1 + i];
                q = fmaf(dx, dx, q);
                const float c = fmaf(alpha, dx, pk[1 + i]);
                mass *= 0.5f * (erff(beta * (1.0f - c)) + erff(beta * c));
            }
            const float ak = fmaf(-0.5f * ivar, q, qk[0]) + logf(mass);
            float sc, w;
            lse_push(M, S, ak, sc, w);
        }
        return M + logf(S);
    }
};

// Full-covariance Gaussian mixture with scaled whitening factors
// W_k = sqrt(log2 e / 2) L_k^-1 (S_k = L_k L_k^T, W_k lower triangular),
// terms in base 2:
//   v_k = W_k (y - m_k),  a_k = c_k - |v_k|^2 = log2(w_k N(y; m_k, S_k)),
//   grad log p = -2 ln 2 sum_k r_k W_k^T v_k  (= -sum_k r_k S_k^-1 (y - m_k)).
template <int D>
struct GmmFull {
    static constexpr int STRIDE = comp_stride(TGT_FULL, D);

    template <int B, bool GRAD, class PT>
    __device__ __forceinline__ static void push(PT P, int k0, const float y[D], float &M, float &S, float G[D],
                                                bool want) {
        float a[B], v[B][D];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const auto pk = P + (k0 + b) * STRIDE;
            const auto W = pk + 1 + D;
            float dx[D];
#pragma unroll
            for (int i = 0; i < D; ++i) dx[i] = y[i] - pk[1 + i];
            // -a_k accumulated from -c_k: the sign folds into the maximum
            // and the differences of lse2_block
            float t = -pk[0];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                float acc = W[i * (i + 1) / 2] * dx[0];
#pragma unroll
                for (int j = 1; j <= i; ++j) acc = fmaf(W[i * (i + 1) / 2 + j], dx[j], acc);
                v[b][i] = acc;
                t = fmaf(acc, acc, t);
            }
            a[b] = -t;
        }
        float sc, w[B];
        lse2_block<B>(M, S, a, sc, w);
        if (GRAD && want) {
#pragma unroll
            for (int j = 0; j < D; ++j) G[j] *= sc;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const auto W = P + (k0 + b) * STRIDE + 1 + D;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    float u = 0.0f;
#pragma unroll
                    for (int i = j; i < D; ++i) u = fmaf(W[i * (i + 1) / 2 + j], v[b][i], u);
                    G[j] = fmaf(w[b], u, G[j]);
                }
            }
        }
    }

    template <bool GRAD, int BMAX = 4, class PT>
    __device__ __forceinline__ static float eval(PT P, int K, const float y[D], float g[D], bool want) {
        constexpr int B = LseBlock<STRIDE, GRAD, BMAX>::value;
        float M = -INFINITY, S = 0.0f;
        float G[D];
#pragma unroll
        for (int i = 0; i < D; ++i) G[i] = 0.0f;
        int k = 0;
        for (; k + B <= K; k += B) push<B, GRAD>(P, k, y, M, S, G, want);
        for (; k < K; ++k) push<1, GRAD>(P, k, y, M, S, G, want);
        if (GRAD && want) {
            const float f = (-2.0f * LN2) / S;
#pragma unroll
            for (int i = 0; i < D; ++i) g[i] = G[i] * f;
        }
        return lse2_ln(M, S);
    }
};

// Rendering-shaped integrand on [0,1]^12 (slab layout in restore_internal.h):
//   g(x) = tA(x0,x1) tB(x6..x11) [b + sum_l w_l h_l(x_{2l}, x_{2l+1})],
//   t(y) = 1 + (1/8) sum_m a_m sin(2 pi (<n_m, y> + phi_m / 2 pi)),
//   w_l h_l(u, v) = C_l exp(-kappa_l |omega(u,v) - dir_l|^2 / 2)  (= exp(kappa (dir.omega - 1))
//   for unit vectors, without the cancellation of dir.omega - 1 near the lobe),
//   omega = (2 sqrt(u (1 - u)) cos 2 pi v, 2 sqrt(u (1 - u)) sin 2 pi v, 1 - 2u).
// Texture phases are reduced modulo one revolution term by term (the
// frequencies are integers), so the hardware sine sees arguments in [0, 1).
template <int D>
struct Pss {
    // one sinusoid per iteration (not unrolled): only that row's scalars are
    // live, which keeps the slab from overflowing the SGPR file
    template <int DIM, class PT>
    __device__ __forceinline__ static float texture(PT freq, PT amp, PT phase, const float *y) {
        float t = 1.0f;
#pragma unroll 1
        for (int m = 0; m < 8; ++m) {
            float s = phase[m];
#pragma unroll
            for (int i = 0; i < DIM; ++i) s = __builtin_amdgcn_fractf(s + __builtin_amdgcn_fractf(freq[m * DIM + i] * y[i]));
            t = fmaf(amp[m], __builtin_amdgcn_sinf(s), t);
        }
        return t;
    }

    template <bool GRAD, int BMAX = 4, class PT>
    __device__ __forceinline__ static float eval(PT P, int K, const float y[D], float g[D], bool want) {
        static_assert(D == 12, "the rendering-shaped integrand lives on [0,1]^12");
        (void)K; (void)g; (void)want;
        const float ta = texture<2>(P + 0, P + 16, P + 24, y);
        const float tb = texture<6>(P + 32, P + 80, P + 88, y + 6);
        float light = P[111];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const float u = y[2 * l], v = y[2 * l + 1];
            const float z = 1.0f - 2.0f * u;
            const float r = 2.0f * sqrtf(fmaxf(u * (1.0f - u), 0.0f));
            const auto dir = P + 96 + 3 * l;
            // the lobe exponent amplifies direction errors by ~kappa |omega - dir|,
            // so the azimuth uses the correctly rounded sin/cos of pi (2v)
            float sv, cv;
            sincospif(2.0f * v, &sv, &cv);
            const float d0 = r * cv - dir[0];
            const float d1 = r * sv - dir[1];
            const float d2 = z - dir[2];
            const float q = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
            light += expf(fmaf(-0.5f * P[105 + l], q, P[108 + l]));
        }
        // one logarithm of the product (ta, tb in (0, 2], light >= b: no
        // overflow; the product's two roundings add 2^-23 relative)
        return logf(ta * tb * light);
    }
};

// Learned regeneration distribution: defensive mixture
//   u(y) = beta 1_box(y) + (1 - beta) sum_k pi_k N(y; m_k, diag(s_k^2))
// (slab layout in restore_internal.h).  log u by the blocked base-2
// log-sum-exp with scalar-loaded parameters; sampling picks the share by
// the cumulative weights and gathers the chosen component per lane.
template <int D>
struct MuGmm {
    static constexpr int STRIDE = mu_stride(D);

    // log u(y).  P: the slab (scalar loads); R: its component blocks, either
    // P + 4 or an LDS copy.  The score fma(y_i, r_ki, n_ki) has two
    // per-component operands and a VALU instruction reads at most one
    // scalar register, so from P alone one of them costs a VALU move; from
    // the LDS copy r_ki arrives in a vector register by a ds_read.
    template <class PT, class RT>
    __device__ __forceinline__ static float log_u(PT P, RT R, int K, const float y[D]) {
        // the defensive share as the first term of the sum: log2 beta on the
        // box (S = 1), nothing outside it (S = 0)
        const bool in = in_unit_box<D>(y);
        float M = in ? P[0] : -INFINITY, S = 1.0f;
        if (M == -INFINITY) S = 0.0f;
        constexpr int B = LseBlock<STRIDE, false>::value;
        int k = 0;
        for (; k + B <= K; k += B) push<B>(P, R, k, y, M, S);
        for (; k < K; ++k) push<1>(P, R, k, y, M, S);
        return lse2_ln(M, S);
    }

    // B components' terms a_k = c_k - |(y - m_k) r_k|^2 with the scaled
    // score fma(y_i, r_ki, -m_ki r_ki), accumulated from -c_k as in GmmFull
    template <int B, class PT, class RT>
    __device__ __forceinline__ static void push(PT P, RT R, int k0, const float y[D], float &M, float &S) {
        float a[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const auto pk = P + 4 + (k0 + b) * STRIDE;
            const auto rk = R + (k0 + b) * STRIDE;
            // from the LDS copy in 16-byte reads (component blocks are a
            // multiple of 4 floats from a 16-byte aligned start)
            float r[D];
            if constexpr (std::is_same<typename std::remove_cv<RT>::type, lds_fptr>::value && D % 4 == 0) {
                typedef float v4f __attribute__((ext_vector_type(4)));
                typedef const __attribute__((address_space(3))) v4f *lds_v4ptr;
                const auto r4 = (lds_v4ptr)rk;
#pragma unroll
                for (int i = 0; i < D / 4; ++i) {
                    const v4f v = r4[i];
                    r[4 * i] = v.x; r[4 * i + 1] = v.y; r[4 * i + 2] = v.z; r[4 * i + 3] = v.w;
                }
            } else {
#pragma unroll
                for (int i = 0; i < D; ++i) r[i] = rk[i];
            }
            float t = -pk[2 * D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const float z = fmaf(y[i], r[i], pk[D + i]);
                t = fmaf(z, z, t);
            }
            a[b] = -t;
        }
        float sc, w[B];
        lse2_block<B>(M, S, a, sc, w);
    }

    // y ~ mu from the category uniform, the candidate uniforms (uniform
    // share) and their Box-Muller normals (Gaussian components)
    // (R as in log_u: with the LDS copy, which also holds the cumulative
    // weights, the component is found by a binary search with per-lane LDS
    // reads instead of K - 1 compares; both give the largest j with
    // cum[j] <= u_cat, the cumulative weights being non-decreasing)
    template <class PT, int NC, class RT = PT>
    __device__ __forceinline__ static void sample(PT P, const float *G, int K, float u_cat, const float cand[NC],
                                                  float y[D], RT R = RT()) {
        const auto cum = P + 4 + K * STRIDE;
        if (u_cat < cum[0]) {
#pragma unroll
            for (int i = 0; i < D; ++i) y[i] = cand[i];
            return;
        }
        int pick = 0;
        if constexpr (std::is_same<typename std::remove_cv<RT>::type, lds_fptr>::value) {
            static_assert(RESTORE_MAX_COMP <= 64, "six halvings cover the components");
            const auto lcum = R + K * STRIDE;
#pragma unroll
            for (int h = 32; h > 0; h >>= 1) {
                const int j = pick + h;
                if (j < K && lcum[j] <= u_cat) pick = j;
            }
        } else {
            (void)R;
            // eight weights per scalar-load wait
#pragma unroll 8
            for (int j = 1; j < K; ++j) pick += (cum[j] <= u_cat) ? 1 : 0;
        }
        float z[D];
        box_muller<D, NC, true>(cand, z);
        const float *ms = G + 4 + K * STRIDE + K + pick * 2 * D;
#pragma unroll
        for (int i = 0; i < D; ++i) y[i] = fmaf(ms[D + i], z[i], ms[i]);
    }
};

template <int D, int TGT>
struct TargetOf;
template <int D>
struct TargetOf<D, TGT_ISO> { using type = GmmIso<D>; };
template <int D>
struct TargetOf<D, TGT_FULL> { using type = GmmFull<D>; };
template <int D>
struct TargetOf<D, TGT_PSS> { using type = Pss<D>; };

// log p(y) with p = 0 outside the unit box; with GRAD, lanes that `want` it
// also get grad log p(y) (the gradient work is skipped by waves where no
// lane wants it).
template <int D, int TGT, bool GRAD, int BMAX = 4, class PT>
__device__ __forceinline__ float log_target(PT P, int K, const float y[D], float g[D], bool want = true) {
    const float lp = TargetOf<D, TGT>::type::template eval<GRAD, BMAX>(P, K, y, g, want);
    const bool in = in_unit_box<D>(y);
    if (GRAD && want) {
#pragma unroll
        for (int i = 0; i < D; ++i) g[i] = in ? g[i] : 0.0f;
    }
    return in ? lp : -INFINITY;
}

}  // namespace restore
