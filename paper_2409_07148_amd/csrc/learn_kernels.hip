// gfx950 kernels of the learned regeneration distribution: an MLP maps a
// context vector to the parameters of a diagonal Gaussian mixture, which
// (mixed with a defensive uniform share) is the regeneration distribution
// mu of the next restore runs.  Training minimises the time-weighted
// negative log-likelihood of restore samples: the pairs (x_{i-1}, dt_i) of a
// run are time-weighted draws of pi (Sec. 7.4, eq. (approx)), and mu has to
// stay a fixed, state-independent density during a run (Sec. 6.2).
//
//  * gemm_bf16_kernel: C = op(A) op(B) on the matrix cores
//    (v_mfma_f32_32x32x16_bf16: bf16 operands, float32 accumulation), one
//    wave per 32 x 32 output tile -- the MLP layers, forward and backward.
//  * gmm_nll_kernel: the weighted NLL and its per-component statistics: the
//    mixture densities in float32 (4 samples x 64 components per wave and
//    pass, log-sum-exp over 16-lane rows), the responsibility-weighted
//    moments on the FP64 matrix cores (v_mfma_f64_16x16x4f64); fixed-order
//    block and grid reductions, so the result is bit-reproducible.
//  * adam_kernel: Adam on float32 master weights.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "learn.h"

namespace restore {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// element (r, c) of op(X) for a row-major X with leading dimension ld
__device__ __forceinline__ float load_op(const float *X, int64_t ld, bool trans, int r, int c, int rows, int cols) {
    if (r >= rows || c >= cols) return 0.0f;
    return trans ? X[(int64_t)c * ld + r] : X[(int64_t)r * ld + c];
}

// C[M x N] (+)= op(A)[M x K] op(B)[K x N].  Lane layout of the 32x32x16
// instruction: lane l holds A[l % 32][8 (l / 32) + j] and
// B[8 (l / 32) + j][l % 32], j < 8, and receives
// C[8 (i / 4) + 4 (l / 32) + i % 4][l % 32], i < 16.
__global__ __launch_bounds__(64) void gemm_bf16_kernel(int M, int N, int K, const float *A, int64_t lda, int transA,
                                                        const float *B, int64_t ldb, int transB, float *C,
                                                        int64_t ldc, int accumulate) {
    const int l = threadIdx.x;
    const int row0 = blockIdx.x * 32, col0 = blockIdx.y * 32;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int kk = k0 + 8 * (l / 32) + j;
            a[j] = (__bf16)load_op(A, lda, transA != 0, row0 + l % 32, kk, M, K);
            b[j] = (__bf16)load_op(B, ldb, transB != 0, kk, col0 + l % 32, K, N);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r = row0 + 8 * (i / 4) + 4 * (l / 32) + (i % 4);
        const int c = col0 + l % 32;
        if (r < M && c < N) {
            float *p = C + (int64_t)r * ldc + c;
            *p = accumulate ? *p + acc[i] : acc[i];
        }
    }
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// z[g][j] += bias[j]; h = gelu(z) (h may be null: bias only)
__global__ void bias_gelu_kernel(float *z, float *h, const float *bias, int G, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= G * n) return;
    const float v = z[i] + bias[i % n];
    z[i] = v;
    if (h) h[i] = gelu(v);
}

// dz = dh * gelu'(z)
__global__ void gelu_back_kernel(const float *dh, const float *z, float *dz, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dz[i] = dh[i] * gelu_grad(z[i]);
}

// db[j] = sum_g d[g][j]
__global__ void colsum_kernel(const float *d, float *db, int G, int n) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float s = 0.0f;
    for (int g = 0; g < G; ++g) s += d[(int64_t)g * n + j];
    db[j] = s;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Lane exchange within a row of 16 lanes (DPP): quad_perm [1,0,3,2] and
// [2,3,0,1], row_half_mirror, row_mirror.  Applied in that order with an
// associative operation they leave every lane of the row with the
// operation over the whole row.
template <int CTRL>
__device__ __forceinline__ float dpp_row(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_max(float v) {
    v = fmaxf(v, dpp_row<0xB1>(v));
    v = fmaxf(v, dpp_row<0x4E>(v));
    v = fmaxf(v, dpp_row<0x141>(v));
    return fmaxf(v, dpp_row<0x140>(v));
}
__device__ __forceinline__ float row16_sum(float v) {
    v += dpp_row<0xB1>(v);
    v += dpp_row<0x4E>(v);
    v += dpp_row<0x141>(v);
    return v + dpp_row<0x140>(v);
}

// Weighted NLL statistics of one block's share of the samples, on the
// FP64 matrix cores.
//
// A wave handles 4 samples x 64 components per pass, in the lane layout of
// v_mfma_f64_16x16x4f64 (lane l provides A[l % 16][l / 16] and
// B[l / 16][l % 16], and receives D[4 r + l / 16][l % 16], r < 4): lane l
// takes sample l / 16 of the pass and components l % 16 + 16 t, t < 4.  For
// each it evaluates a_k = c_k - |(x - m_k) / s_k|^2 / 2 in float32 (c_k =
// ln(1 - beta) + ln pi_k - d/2 ln 2 pi - sum ln s_k); log u(x) = LSE(a,
// ln beta 1_box) is reduced over the 16 lanes of the sample's row (DPP) and
// the 4 tiles; the responsibility r_k = e^{a_k - M} / sum e^{a - M}.  Then
//   A[k][s] = w_s r_sk (float64),   B[s][f] = x_sf (f < d), x_s,f-d^2 (f < 2d)
// (exact in float64), and D += A B accumulates the uncentred moments
//   P1_ki = sum w r x_i,  P2_ki = sum w r x_i^2
// in float64, where the centring (x - m)^2 = x^2 - 2 m x + m^2 that the
// gradient needs costs nothing (float32 would lose the m^2 / s^2 ~ 2500
// cancelled digits).  S0_k = sum w r, LW = sum w log u and W = sum w go
// through the vector unit.  The NLL_WAVES waves add their statistics into
// LDS in wave order and the block writes one partial row set:
// partials[block][row][64], rows: 0 S0, 1 + i P1_i, 1 + d + i P2_i,
// 1 + 2d [LW, W].  Samples: the block's contiguous range in passes of 4,
// two passes per iteration, wave v taking pass pairs v, v + NLL_WAVES, ...
// Exponentials and logarithms go through the base-2 hardware instructions
// (e^y = 2^{y log2 e}; the rounding of y log2 e adds |y| 2^-24 relative).
__host__ __device__ constexpr int nll_feature_tiles(int D) { return (2 * D + 15) / 16; }

// x[0..D) of one sample row (16-byte loads where the rows are 16-byte aligned)
template <int D, bool VEC>
__device__ __forceinline__ void load_row(const float *p, float (&x)[D]) {
    if constexpr (VEC && D % 4 == 0) {
#pragma unroll
        for (int i = 0; i < D; i += 4) {
            const float4 v = *reinterpret_cast<const float4 *>(p + i);
            x[i] = v.x;
            x[i + 1] = v.y;
            x[i + 2] = v.z;
            x[i + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < D; ++i) x[i] = p[i];
    }
}

template <int D, bool VEC>
__global__ __launch_bounds__(64 * NLL_WAVES) void gmm_nll_kernel(NllArgs a) {
    typedef double double4_t __attribute__((ext_vector_type(4)));
    constexpr int NF = nll_feature_tiles(D);
    constexpr int ROWS = nll_rows(D);
    __shared__ double red[ROWS * 64];
    __shared__ float lse_part[64];
    const int l = threadIdx.x % 64, wv = threadIdx.x / 64;
    const int K = a.n_comp;

    // the mixture weights ln pi = logits - LSE(logits) (one wave-wide pass)
    {
        const float logit = l < K ? a.gmm[l] : -INFINITY;
        const float lmax = wave_max(logit);
        const float lse = lmax + logf(wave_sum(l < K ? expf(logit - lmax) : 0.0f));
        if (wv == 0) lse_part[l] = lse;
    }
    __syncthreads();
    const float logit_lse = lse_part[0];
    const float lbeta = a.beta > 0.0f ? logf(a.beta) : -INFINITY;
    const float l1mb = a.beta < 1.0f ? log1pf(-a.beta) : -INFINITY;

    // this lane's four components
    float m[4][D], is[4][D], c[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = l % 16 + 16 * t;
        const bool act = k < K;
        c[t] = act ? l1mb + a.gmm[k] - logit_lse - 0.5f * D * 1.8378770664093453f : -INFINITY;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            m[t][i] = 0.0f;
            is[t][i] = 0.0f;
            if (act) {
                const float ls = a.gmm[K + K * D + k * D + i];
                m[t][i] = a.gmm[K + k * D + i];
                is[t][i] = expf(-ls);
                c[t] -= ls;
            }
        }
    }

    double4_t acc[4][NF];
    double s0[4], lw = 0.0, wsum = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        s0[t] = 0.0;
#pragma unroll
        for (int u = 0; u < NF; ++u) acc[t][u] = double4_t{0.0, 0.0, 0.0, 0.0};
    }
    constexpr float LOG2E = 1.4426950408889634f, LN2 = 0.6931471805599453f;
    const bool defensive = l % 16 == 0 && a.beta > 0.0f;  // the uniform share, once per sample row
    const int64_t lo = (int64_t)blockIdx.x * a.per_block;
    const int64_t hi = lo + a.per_block < a.n ? lo + a.per_block : a.n;
    const int sl = l / 16;  // this lane's sample within a pass
    // NP passes per iteration, so that the lane exchanges of one pass overlap
    // the arithmetic of the other; a sample past the range is replaced by
    // the range's last one with weight 0 (loads stay unconditional)
    constexpr int NP = D <= 10 ? 2 : 1;
    // feature 16 u + l % 16 of this lane: coordinate fx[u], squared or not,
    // or zero past 2d
    int fx[NF];
    bool fsq[NF];
    double fone[NF];
#pragma unroll
    for (int u = 0; u < NF; ++u) {
        const int f = 16 * u + l % 16;
        fx[u] = f < D ? f : (f < 2 * D ? f - D : 0);
        fsq[u] = f >= D && f < 2 * D;
        fone[u] = f < 2 * D ? 1.0 : 0.0;
    }
    for (int64_t p = lo + 4 * NP * (int64_t)wv; p < hi; p += 4 * NP * NLL_WAVES) {
        float x[NP][D], w[NP], at[NP][4], mx[NP], xf[NP][NF];
        bool in[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int64_t n = p + 4 * j + sl;
            const bool valid = n < hi;
            const int64_t nl = valid ? n : hi - 1;
            load_row<D, VEC>(a.x + nl * D, x[j]);
            // this lane's B column: feature 16 u + l % 16 is x or x^2 of
            // coordinate fx[u] (a second load of the same row, in cache)
#pragma unroll
            for (int u = 0; u < NF; ++u) xf[j][u] = a.x[nl * D + fx[u]];
            const float wl = a.w[nl];
            w[j] = valid ? wl : 0.0f;
            float xlo = x[j][0], xhi = x[j][0];
#pragma unroll
            for (int i = 1; i < D; ++i) {
                xlo = fminf(xlo, x[j][i]);
                xhi = fmaxf(xhi, x[j][i]);
            }
            in[j] = xlo >= 0.0f && xhi <= 1.0f;
            mx[j] = in[j] ? lbeta : -INFINITY;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                float q = 0.0f;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const float z = (x[j][i] - m[t][i]) * is[t][i];
                    q = fmaf(z, z, q);
                }
                at[j][t] = fmaf(-0.5f, q, c[t]);   // -inf for components past K
                mx[j] = fmaxf(mx[j], at[j][t]);
            }
        }
        float M[NP], S[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            M[j] = row16_max(mx[j]);
            M[j] = M[j] > -INFINITY ? M[j] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            float se = 0.0f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                at[j][t] = __builtin_amdgcn_exp2f((at[j][t] - M[j]) * LOG2E);   // e^{a - M}
                se += at[j][t];
            }
            if (defensive && in[j]) se += __builtin_amdgcn_exp2f((lbeta - M[j]) * LOG2E);
            S[j] = row16_sum(se);
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const float inv_s = S[j] > 0.0f ? __builtin_amdgcn_rcpf(S[j]) : 0.0f;
            const double wd = (double)w[j];
            if (l % 16 == 0) {
                lw += wd * (double)(M[j] + __builtin_amdgcn_logf(S[j]) * LN2);
                wsum += wd;
            }
            double bf[NF];
#pragma unroll
            for (int u = 0; u < NF; ++u) {
                const double xv = (double)xf[j][u];
                bf[u] = fsq[u] ? xv * xv : xv * fone[u];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double wr = wd * (double)(at[j][t] * inv_s);
                s0[t] += wr;
#pragma unroll
                for (int u = 0; u < NF; ++u) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(wr, bf[u], acc[t][u], 0, 0, 0);
            }
        }
    }

    // S0 and [LW, W] over the 4 sample rows of the wave
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        s0[t] += __shfl_xor(s0[t], 16);
        s0[t] += __shfl_xor(s0[t], 32);
    }
    lw += __shfl_xor(lw, 16);
    lw += __shfl_xor(lw, 32);
    wsum += __shfl_xor(wsum, 16);
    wsum += __shfl_xor(wsum, 32);

    // add the waves' statistics into LDS in wave order
    for (int v = 0; v < NLL_WAVES; ++v) {
        if (wv == v) {
            const bool first = v == 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (l < 16) {
                    double *r0 = &red[16 * t + l];
                    *r0 = first ? s0[t] : *r0 + s0[t];
                }
#pragma unroll
                for (int u = 0; u < NF; ++u) {
                    const int f = 16 * u + l % 16;
                    if (f < 2 * D) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            double *q = &red[(1 + f) * 64 + 16 * t + 4 * r + l / 16];
                            *q = first ? acc[t][u][r] : *q + acc[t][u][r];
                        }
                    }
                }
            }
            if (l == 0) {
                double *q = &red[(1 + 2 * D) * 64];
                q[0] = first ? lw : q[0] + lw;
                q[1] = first ? wsum : q[1] + wsum;
            }
            if (first && l >= 2) red[(1 + 2 * D) * 64 + l] = 0.0;
        }
        __syncthreads();
    }
    double *out = a.partials + (int64_t)blockIdx.x * ROWS * 64;
    for (int j = threadIdx.x; j < ROWS * 64; j += 64 * NLL_WAVES) out[j] = red[j];
}

// totals[j] = sum over blocks b (fixed order) of partials[b][j].
__global__ __launch_bounds__(256) void gmm_nll_sum_kernel(const double *partials, int entries, int n_blocks,
                                                           double *totals) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= entries) return;
    double v = 0.0;
    for (int b = 0; b < n_blocks; ++b) v += partials[(int64_t)b * entries + j];
    totals[j] = v;
}

// Gradient of L = -sum w log u / sum w with respect to the mixture outputs,
// from the uncentred moments (float64): with S1 = sum w r (x - m) / s and
// S2 = sum w r ((x - m) / s)^2,
//   S1_ki = (P1_ki - m_ki S0_k) / s_ki
//   S2_ki = (P2_ki - 2 m_ki P1_ki + m_ki^2 S0_k) / s_ki^2
//   dL/dlogit_k = -(S0_k - pi_k sum_j S0_j) / W
//   dL/dm_ki    = -S1_ki / (W s_ki)
//   dL/dlog s_ki = -(S2_ki - S0_k) / W
template <int D>
__global__ __launch_bounds__(64) void gmm_nll_grad_kernel(NllArgs a, const double *totals) {
    const int k = threadIdx.x;
    const int K = a.n_comp;
    const double *S = totals;
    const double s0 = S[k], lw = S[(1 + 2 * D) * 64], W = S[(1 + 2 * D) * 64 + 1];
    const bool act = k < K;
    const float logit = act ? a.gmm[k] : -INFINITY;
    const float lmax = wave_max(logit);
    const float pk = act ? expf(logit - lmax) : 0.0f;
    const float pi = pk / wave_sum(pk);
    double s0tot = 0.0;
    for (int j = 0; j < K; ++j) s0tot += S[j];
    if (act) {
        a.dout[k] = (float)(-(s0 - (double)pi * s0tot) / W);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double mk = (double)a.gmm[K + k * D + i];
            const double inv_s = (double)expf(-a.gmm[K + K * D + k * D + i]);
            const double p1 = S[(1 + i) * 64 + k], p2 = S[(1 + D + i) * 64 + k];
            const double s1 = (p1 - mk * s0) * inv_s;
            const double s2 = (p2 - 2.0 * mk * p1 + mk * mk * s0) * inv_s * inv_s;
            a.dout[K + k * D + i] = (float)(-s1 * inv_s / W);
            a.dout[K + K * D + k * D + i] = (float)(-(s2 - s0) / W);
        }
    }
    if (k == 0) a.loss[0] = -lw / W;
}

__global__ void adam_kernel(float *theta, const float *grad, float *m, float *v, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_gemm_bf16(int M, int N, int K, const float *A, int64_t lda, bool transA, const float *B, int64_t ldb,
                            bool transB, float *C, int64_t ldc, bool accumulate, hipStream_t s) {
    const dim3 grid((M + 31) / 32, (N + 31) / 32);
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(64), 0, s, M, N, K, A, lda, (int)transA, B, ldb, (int)transB, C,
                       ldc, (int)accumulate);
    return hipGetLastError();
}

hipError_t launch_bias_gelu(float *z, float *h, const float *bias, int G, int n, hipStream_t s) {
    hipLaunchKernelGGL(bias_gelu_kernel, dim3((G * n + 255) / 256), dim3(256), 0, s, z, h, bias, G, n);
    return hipGetLastError();
}

hipError_t launch_gelu_back(const float *dh, const float *z, float *dz, int count, hipStream_t s) {
    hipLaunchKernelGGL(gelu_back_kernel, dim3((count + 255) / 256), dim3(256), 0, s, dh, z, dz, count);
    return hipGetLastError();
}

hipError_t launch_colsum(const float *d, float *db, int G, int n, hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, db, G, n);
    return hipGetLastError();
}

template <int D>
static void launch_nll_d(const NllArgs &a, hipStream_t s) {
    const int entries = nll_rows(D) * 64;
    // rows of D % 4 == 0 floats are 16-byte aligned when x is
    if (D % 4 == 0 && reinterpret_cast<uintptr_t>(a.x) % 16 == 0)
        hipLaunchKernelGGL((gmm_nll_kernel<D, true>), dim3(a.n_blocks), dim3(64 * NLL_WAVES), 0, s, a);
    else
        hipLaunchKernelGGL((gmm_nll_kernel<D, false>), dim3(a.n_blocks), dim3(64 * NLL_WAVES), 0, s, a);
    hipLaunchKernelGGL(gmm_nll_sum_kernel, dim3((entries + 255) / 256), dim3(256), 0, s, (const double *)a.partials,
                       entries, a.n_blocks, a.totals);
    hipLaunchKernelGGL(gmm_nll_grad_kernel<D>, dim3(1), dim3(64), 0, s, a, (const double *)a.totals);
}

hipError_t launch_gmm_nll(const NllArgs &a, hipStream_t s) {
    switch (a.dim) {
        case 1: launch_nll_d<1>(a, s); break;
        case 2: launch_nll_d<2>(a, s); break;
        case 3: launch_nll_d<3>(a, s); break;
        case 4: launch_nll_d<4>(a, s); break;
        case 5: launch_nll_d<5>(a, s); break;
        case 6: launch_nll_d<6>(a, s); break;
        case 7: launch_nll_d<7>(a, s); break;
        case 8: launch_nll_d<8>(a, s); break;
        case 9: launch_nll_d<9>(a, s); break;
        case 10: launch_nll_d<10>(a, s); break;
        case 11: launch_nll_d<11>(a, s); break;
        case 12: launch_nll_d<12>(a, s); break;
        case 13: launch_nll_d<13>(a, s); break;
        case 14: launch_nll_d<14>(a, s); break;
        case 15: launch_nll_d<15>(a, s); break;
        case 16: launch_nll_d<16>(a, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adam(float *theta, const float *grad, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, int t, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, grad, m, v, n, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace restore
