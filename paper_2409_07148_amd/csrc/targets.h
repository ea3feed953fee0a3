// Target densities p and regeneration densities u evaluated per lane.
//
// All mixtures are evaluated in log space with a running maximum (online
// log-sum-exp) so that neither the far tails nor the sharp peaks of the
// components leave the float32 range.  Parameters are read from a packed
// slab whose addresses are wave-uniform: from global memory they become
// scalar loads (SGPR operands of the FMAs); with LDS staging they are
// broadcast reads.
#pragma once

#include "device_common.h"

namespace restore {

// Isotropic Gaussian mixture: a_k = c_k - (1/(2 s_k^2)) |y - m_k|^2,
// grad log p = sum_k r_k (-(y - m_k) / s_k^2), r = softmax(a).
template <int D>
struct GmmIso {
    static constexpr int STRIDE = comp_stride(TGT_ISO, D);

    template <bool GRAD>
    __device__ __forceinline__ static float eval(const float *__restrict__ P, int K, const float y[D],
                                                 float g[D], bool want) {
        float M = -INFINITY, S = 0.0f;
        float G[D];
#pragma unroll
        for (int i = 0; i < D; ++i) G[i] = 0.0f;
        for (int k = 0; k < K; ++k) {
            const float *pk = P + k * STRIDE;
            const float ivar = pk[1 + D];
            float dx[D], q = 0.0f;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                dx[i] = y[i] - pk[1 + i];
                q = fmaf(dx[i], dx[i], q);
            }
            const float ak = fmaf(-0.5f * ivar, q, pk[0]);
            const float Mn = fmaxf(M, ak);
            const float sc = exp_rel(M - Mn);
            const float w = exp_rel(ak - Mn);
            S = fmaf(S, sc, w);
            if (GRAD && want) {
                const float wi = -w * ivar;
#pragma unroll
                for (int i = 0; i < D; ++i) G[i] = fmaf(G[i], sc, wi * dx[i]);
            }
            M = Mn;
        }
        const float lp = M + logf(S);
        if (GRAD && want) {
            const float inv = 1.0f / S;
#pragma unroll
            for (int i = 0; i < D; ++i) g[i] = G[i] * inv;
        }
        return lp;
    }
};

// Full-covariance Gaussian mixture with whitening factors W_k = L_k^-1
// (S_k = L_k L_k^T, W_k lower triangular):
//   v_k = W_k (y - m_k),  a_k = c_k - |v_k|^2 / 2,
//   grad log p = sum_k r_k (-W_k^T v_k)  (= -S_k^-1 (y - m_k)).
template <int D>
struct GmmFull {
    static constexpr int STRIDE = comp_stride(TGT_FULL, D);

    template <bool GRAD>
    __device__ __forceinline__ static float eval(const float *__restrict__ P, int K, const float y[D],
                                                 float g[D], bool want) {
        float M = -INFINITY, S = 0.0f;
        float G[D];
#pragma unroll
        for (int i = 0; i < D; ++i) G[i] = 0.0f;
        for (int k = 0; k < K; ++k) {
            const float *pk = P + k * STRIDE;
            const float *W = pk + 1 + D;
            float dx[D], v[D];
#pragma unroll
            for (int i = 0; i < D; ++i) dx[i] = y[i] - pk[1 + i];
            float q = 0.0f;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                float acc = W[i * (i + 1) / 2] * dx[0];
#pragma unroll
                for (int j = 1; j <= i; ++j) acc = fmaf(W[i * (i + 1) / 2 + j], dx[j], acc);
                v[i] = acc;
                q = fmaf(acc, acc, q);
            }
            const float ak = fmaf(-0.5f, q, pk[0]);
            const float Mn = fmaxf(M, ak);
            const float sc = exp_rel(M - Mn);
            const float w = exp_rel(ak - Mn);
            S = fmaf(S, sc, w);
            if (GRAD && want) {
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    float u = 0.0f;
#pragma unroll
                    for (int i = j; i < D; ++i) u = fmaf(W[i * (i + 1) / 2 + j], v[i], u);
                    G[j] = fmaf(G[j], sc, -w * u);
                }
            }
            M = Mn;
        }
        const float lp = M + logf(S);
        if (GRAD && want) {
            const float inv = 1.0f / S;
#pragma unroll
            for (int i = 0; i < D; ++i) g[i] = G[i] * inv;
        }
        return lp;
    }
};

template <int D, int TGT>
struct TargetOf;
template <int D>
struct TargetOf<D, TGT_ISO> { using type = GmmIso<D>; };
template <int D>
struct TargetOf<D, TGT_FULL> { using type = GmmFull<D>; };

// log p(y) with p = 0 outside the unit box; with GRAD, lanes that `want` it
// also get grad log p(y) (the gradient work is skipped by waves where no
// lane wants it).
template <int D, int TGT, bool GRAD>
__device__ __forceinline__ float log_target(const float *__restrict__ P, int K, const float y[D], float g[D],
                                            bool want = true) {
    const float lp = TargetOf<D, TGT>::type::template eval<GRAD>(P, K, y, g, want);
    const bool in = in_unit_box<D>(y);
    if (GRAD && want) {
#pragma unroll
        for (int i = 0; i < D; ++i) g[i] = in ? g[i] : 0.0f;
    }
    return in ? lp : -INFINITY;
}

}  // namespace restore
