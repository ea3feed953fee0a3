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
//  * gmm_nll_kernel: per-component statistics of the weighted NLL in float32
//    with centred scores z = (x - m)/s (one lane per component, samples
//    broadcast to the wave), accumulated in float64; fixed-order block and
//    grid reductions, so the result is bit-reproducible.
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

// Weighted NLL statistics.  Lane k of every wave is mixture component k;
// the NLL_WAVES waves of a block take interleaved samples.  For each
// sample x_i: a_k = ln(1-beta) + ln pi_k - d/2 ln 2 pi - sum ln s_k -
// |z|^2/2 with z = (x_i - m_k)/s_k, log u(x_i) = LSE(a, ln beta 1_box),
// r_k = exp(a_k - log u), and the weighted sums
//   S0 = sum w r, S1 = sum w r z, S2 = sum w r z^2, LW = sum w log u,
//   W = sum w,
// accumulated in float64 per lane, combined over the block's waves in a
// fixed order through LDS and written as one partial per block:
// partials[block][j][k], j < nll_stats(D).
constexpr int NLL_WAVES = 4;
__host__ __device__ constexpr int nll_stats(int D) { return 3 + 2 * D; }

template <int D>
__global__ __launch_bounds__(64 * NLL_WAVES) void gmm_nll_kernel(NllArgs a) {
    constexpr int R = nll_stats(D);
    __shared__ double red[NLL_WAVES - 1][64];
    const int k = threadIdx.x % 64, wv = threadIdx.x / 64;
    const int K = a.n_comp;
    const bool act = k < K;
    const float logit = act ? a.gmm[k] : -INFINITY;
    const float lmax = wave_max(logit);
    const float lse = lmax + logf(wave_sum(act ? expf(logit - lmax) : 0.0f));
    float m[D], inv_s[D];
    float c = act ? (a.beta < 1.0f ? log1pf(-a.beta) : -INFINITY) + logit - lse - 0.5f * D * 1.8378770664093453f
                  : -INFINITY;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        m[i] = 0.0f;
        inv_s[i] = 0.0f;
        if (act) {
            const float ls = a.gmm[K + K * D + k * D + i];
            m[i] = a.gmm[K + k * D + i];
            inv_s[i] = expf(-ls);
            c -= ls;
        }
    }
    const float lbeta = a.beta > 0.0f ? logf(a.beta) : -INFINITY;
    double acc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * NLL_WAVES;
    for (int64_t n = (int64_t)blockIdx.x * NLL_WAVES + wv; n < a.n; n += stride) {
        const float w = a.w[n];
        const float *x = a.x + n * D;
        float z[D], q = 0.0f;
        bool in = true;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float xi = x[i];
            in = in && xi >= 0.0f && xi <= 1.0f;
            z[i] = (xi - m[i]) * inv_s[i];
            q = fmaf(z[i], z[i], q);
        }
        const float ak = act ? fmaf(-0.5f, q, c) : -INFINITY;
        const float au = in ? lbeta : -INFINITY;
        const float M = fmaxf(wave_max(ak), au);
        const float S = wave_sum(act ? expf(ak - M) : 0.0f) + (au > -INFINITY ? expf(au - M) : 0.0f);
        const float logu = M + logf(S);
        const double wr = (double)w * (double)(act ? expf(ak - logu) : 0.0f);
        acc[0] += wr;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            acc[1 + i] += wr * z[i];
            acc[1 + D + i] += wr * z[i] * z[i];
        }
        acc[1 + 2 * D] += (double)w * (double)logu;
        acc[2 + 2 * D] += (double)w;
    }
    double *out = a.partials + (int64_t)blockIdx.x * R * 64;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (wv > 0) red[wv - 1][k] = acc[j];
        __syncthreads();
        if (wv == 0) {
            double v = acc[j];
#pragma unroll
            for (int u = 0; u < NLL_WAVES - 1; ++u) v += red[u][k];
            out[j * 64 + k] = v;
        }
        __syncthreads();
    }
}

// totals[j][k] = sum over blocks b (fixed order) of partials[b][j][k]: one
// block per statistic j; wave v takes blocks b = v, v + NW, ... and the
// waves' sums are added in wave order.
constexpr int NLL_SUM_WAVES = 16;
__global__ __launch_bounds__(64 * NLL_SUM_WAVES) void gmm_nll_sum_kernel(const double *partials, int R,
                                                                          int n_blocks, double *totals) {
    __shared__ double red[NLL_SUM_WAVES][64];
    const int k = threadIdx.x % 64, wv = threadIdx.x / 64, j = blockIdx.x;
    double v = 0.0;
    for (int b = wv; b < n_blocks; b += NLL_SUM_WAVES) v += partials[((int64_t)b * R + j) * 64 + k];
    red[wv][k] = v;
    __syncthreads();
    if (wv == 0) {
        double t = 0.0;
        for (int u = 0; u < NLL_SUM_WAVES; ++u) t += red[u][k];
        totals[j * 64 + k] = t;
    }
}

// Gradient of L = -sum w log u / sum w with respect to the mixture outputs:
//   dL/dlogit_k = -(S0_k - pi_k sum_j S0_j) / W
//   dL/dm_ki    = -S1_ki / (W s_ki)
//   dL/dlog s_ki = -(S2_ki - S0_k) / W
template <int D>
__global__ __launch_bounds__(64) void gmm_nll_grad_kernel(NllArgs a, const double *totals) {
    const int k = threadIdx.x;
    const int K = a.n_comp;
    const double *S = totals;
    const double s0 = S[k], lw = S[(1 + 2 * D) * 64], W = S[(2 + 2 * D) * 64];
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
            const float inv_s = expf(-a.gmm[K + K * D + k * D + i]);
            a.dout[K + k * D + i] = (float)(-S[(1 + i) * 64 + k] * inv_s / W);
            a.dout[K + K * D + k * D + i] = (float)(-(S[(1 + D + i) * 64 + k] - s0) / W);
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
    hipLaunchKernelGGL(gmm_nll_kernel<D>, dim3(a.n_blocks), dim3(64 * NLL_WAVES), 0, s, a);
    hipLaunchKernelGGL(gmm_nll_sum_kernel, dim3(nll_stats(D)), dim3(64 * NLL_SUM_WAVES), 0, s,
                       (const double *)a.partials, nll_stats(D), a.n_blocks, a.totals);
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
