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
//  * mlp_forward_f32_kernel / mlp_backward_f32_kernel: the same MLP in
//    float32 for a few context rows, where each layer is a matrix-vector
//    product: one launch per pass, plain FMAs in a fixed order.
//  * adam_kernel: Adam on float32 master weights.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>
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

// ---- float32 MLP for a few context rows ---------------------------------

// z[j] = b[j] + sum_i W[j][i] src[i] (row-major W, n_out x n_in), summed in
// order of i; h[j] = gelu(z[j]).  src, z and h in LDS.
__device__ __forceinline__ void dense_f32(const float *W, const float *b, const float *src, int n_in, int n_out,
                                          float *z, float *h) {
    for (int j = threadIdx.x; j < n_out; j += blockDim.x) {
        const float *w = W + (int64_t)j * n_in;
        float acc = 0.0f;
        for (int i = 0; i < n_in; ++i) acc = fmaf(w[i], src[i], acc);
        acc += b[j];
        z[j] = acc;
        h[j] = gelu(acc);
    }
}

// Workgroup (x, g): the hidden layers of context row g, then outputs
// [256 x, 256 x + 256) of that row; workgroup (0, g) also stores the row's
// activations z1, h1, z2, h2 (four [G][H] blocks).
__global__ __launch_bounds__(256) void mlp_forward_f32_kernel(MlpDims m, const float *theta, const float *ctx,
                                                              int G, float *act, float *out) {
    __shared__ float c[MLP_F32_MAX_WIDTH], z1[MLP_F32_MAX_WIDTH], h1[MLP_F32_MAX_WIDTH];
    __shared__ float z2[MLP_F32_MAX_WIDTH], h2[MLP_F32_MAX_WIDTH];
    const int g = blockIdx.y, t = threadIdx.x;
    for (int i = t; i < m.in; i += blockDim.x) c[i] = ctx[(int64_t)g * m.in + i];
    __syncthreads();
    dense_f32(theta + m.W1, theta + m.b1, c, m.in, m.H, z1, h1);
    __syncthreads();
    dense_f32(theta + m.W2, theta + m.b2, h1, m.H, m.H, z2, h2);
    __syncthreads();
    if (blockIdx.x == 0) {
        const int64_t GH = (int64_t)G * m.H, row = (int64_t)g * m.H;
        for (int j = t; j < m.H; j += blockDim.x) {
            act[row + j] = z1[j];
            act[GH + row + j] = h1[j];
            act[2 * GH + row + j] = z2[j];
            act[3 * GH + row + j] = h2[j];
        }
    }
    const int o = blockIdx.x * blockDim.x + t;
    if (o < m.O) {
        const float *w = theta + m.W3 + (int64_t)o * m.H;
        float acc = 0.0f;
        for (int i = 0; i < m.H; ++i) acc = fmaf(w[i], h2[i], acc);
        out[(int64_t)g * m.O + o] = acc + theta[m.b3 + o];
    }
}

// sum over rows r = p, p + groups, ... < n_rows of v[r] W[r][col] (row-major
// W with n_cols columns): eight running sums (eight loads in flight), added
// pairwise at the end -- a fixed order.
__device__ __forceinline__ float strided_dot(const float *v, const float *W, int n_rows, int n_cols, int col, int p,
                                             int groups) {
    const float *w = W + col;
    float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    int r = p;
    for (; r + 7 * groups < n_rows; r += 8 * groups) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int ru = r + u * groups;
            acc[u] = fmaf(v[ru], w[(int64_t)ru * n_cols], acc[u]);
        }
    }
    for (; r < n_rows; r += groups) acc[0] = fmaf(v[r], w[(int64_t)r * n_cols], acc[0]);
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// grad = d(sum_g dout[g] . out[g]) / d theta.  Workgroups 1.. take dW3 and
// db3 (sums over the rows g, in order); workgroup 0 takes the chain through
// the hidden layers row by row (dh2 = dout W3 and dh1 = dz2 W2 each split
// over 256 / H thread groups and combined in group order; dz2 and dz1 into
// work),
// then dW2, db2, dW1, db1 (sums over g in order).
__global__ __launch_bounds__(256) void mlp_backward_f32_kernel(MlpDims m, const float *theta, const float *ctx,
                                                               int G, const float *act, const float *dout,
                                                               float *work, float *grad) {
    const int t = threadIdx.x;
    const int64_t GH = (int64_t)G * m.H;
    const float *z1 = act, *h1 = act + GH, *z2 = act + 2 * GH, *h2 = act + 3 * GH;
    if (blockIdx.x > 0) {
        const int64_t n3 = (int64_t)m.O * m.H;
        for (int64_t e = (int64_t)(blockIdx.x - 1) * blockDim.x + t; e < n3 + m.O;
             e += (int64_t)(gridDim.x - 1) * blockDim.x) {
            float acc = 0.0f;
            if (e < n3) {
                const int64_t o = e / m.H, h = e - o * m.H;
                for (int g = 0; g < G; ++g) acc = fmaf(dout[(int64_t)g * m.O + o], h2[(int64_t)g * m.H + h], acc);
                grad[m.W3 + e] = acc;
            } else {
                const int64_t o = e - n3;
                for (int g = 0; g < G; ++g) acc += dout[(int64_t)g * m.O + o];
                grad[m.b3 + o] = acc;
            }
        }
        return;
    }
    __shared__ float part[256], dz2s[MLP_F32_MAX_WIDTH];
    float *dz2w = work, *dz1w = work + GH;
    const int groups = max(1, (int)blockDim.x / m.H);
    for (int g = 0; g < G; ++g) {
        const float *dg = dout + (int64_t)g * m.O;
        if (t < groups * m.H) part[t] = strided_dot(dg, theta + m.W3, m.O, m.H, t % m.H, t / m.H, groups);
        __syncthreads();
        for (int h = t; h < m.H; h += blockDim.x) {
            float dh = 0.0f;
            for (int p = 0; p < groups; ++p) dh += part[p * m.H + h];
            const float dz = dh * gelu_grad(z2[(int64_t)g * m.H + h]);
            dz2s[h] = dz;
            dz2w[(int64_t)g * m.H + h] = dz;
        }
        __syncthreads();
        if (t < groups * m.H) part[t] = strided_dot(dz2s, theta + m.W2, m.H, m.H, t % m.H, t / m.H, groups);
        __syncthreads();
        for (int i = t; i < m.H; i += blockDim.x) {
            float dh = 0.0f;
            for (int p = 0; p < groups; ++p) dh += part[p * m.H + i];
            dz1w[(int64_t)g * m.H + i] = dh * gelu_grad(z1[(int64_t)g * m.H + i]);
        }
        __syncthreads();
    }
    for (int64_t e = t; e < (int64_t)m.H * m.H; e += blockDim.x) {
        const int64_t j = e / m.H, i = e - j * m.H;
        float acc = 0.0f;
        for (int g = 0; g < G; ++g) acc = fmaf(dz2w[(int64_t)g * m.H + j], h1[(int64_t)g * m.H + i], acc);
        grad[m.W2 + e] = acc;
    }
    for (int64_t e = t; e < (int64_t)m.H * m.in; e += blockDim.x) {
        const int64_t j = e / m.in, i = e - j * m.in;
        float acc = 0.0f;
        for (int g = 0; g < G; ++g) acc = fmaf(dz1w[(int64_t)g * m.H + j], ctx[(int64_t)g * m.in + i], acc);
        grad[m.W1 + e] = acc;
    }
    for (int j = t; j < m.H; j += blockDim.x) {
        float a2 = 0.0f, a1 = 0.0f;
        for (int g = 0; g < G; ++g) {
            a2 += dz2w[(int64_t)g * m.H + j];
            a1 += dz1w[(int64_t)g * m.H + j];
        }
        grad[m.b2 + j] = a2;
        grad[m.b1 + j] = a1;
    }
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

__device__ __forceinline__ double wave_sum(double v) {
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
    // the completion counter of the sum launch that follows on the stream
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.done = 0u;

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

    // this lane's four components: the score of coordinate i is
    // z_i = (x_i - m_i) / s_i = fma(x_i, is_i, nm_i) with is_i = 1 / s_i and
    // nm_i = -m_i is_i (one instruction per coordinate)
    float nm[4][D], is[4][D], c[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = l % 16 + 16 * t;
        const bool act = k < K;
        c[t] = act ? l1mb + a.gmm[k] - logit_lse - 0.5f * D * 1.8378770664093453f : -INFINITY;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            nm[t][i] = 0.0f;
            is[t][i] = 0.0f;
            if (act) {
                const float ls = a.gmm[K + K * D + k * D + i];
                is[t][i] = expf(-ls);
                nm[t][i] = -a.gmm[K + k * D + i] * is[t][i];
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
    // scores in base 2 from here on: a_k log2 e = c_k log2 e - (log2 e / 2) q,
    // so that the exponentials take the hardware 2^x directly
    constexpr float LOG2E = 1.4426950408889634f, LN2 = 0.6931471805599453f, HALF_LOG2E = 0.7213475204444817f;
    const float lbeta2 = lbeta * LOG2E;
#pragma unroll
    for (int t = 0; t < 4; ++t) c[t] *= LOG2E;
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
    // the rows of the next iteration are loaded while this one computes
    // (two waves per SIMD hide little latency on their own); above d = 12
    // the second set of registers would spill, and the rows are loaded at
    // the top of their own iteration
    constexpr int64_t STRIDE = 4 * NP * NLL_WAVES;
    constexpr bool PREFETCH = D <= 12;
    float xn[NP][D], xfn[NP][NF], wn[NP];
    auto fetch = [&](int64_t p) {
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int64_t n = p + 4 * j + sl;
            const int64_t nl = n < hi ? n : hi - 1;
            load_row<D, VEC>(a.x + nl * D, xn[j]);
            // this lane's B column: feature 16 u + l % 16 is x or x^2 of
            // coordinate fx[u] (a second load of the same row, in cache)
#pragma unroll
            for (int u = 0; u < NF; ++u) xfn[j][u] = a.x[nl * D + fx[u]];
            wn[j] = a.w[nl];
        }
    };
    const int64_t p0 = lo + 4 * NP * (int64_t)wv;
    if (PREFETCH && p0 < hi) fetch(p0);
    for (int64_t p = p0; p < hi; p += STRIDE) {
        float x[NP][D], w[NP], at[NP][4], mx[NP], xf[NP][NF];
        bool in[NP];
        if (!PREFETCH) fetch(p);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
#pragma unroll
            for (int i = 0; i < D; ++i) x[j][i] = xn[j][i];
#pragma unroll
            for (int u = 0; u < NF; ++u) xf[j][u] = xfn[j][u];
            w[j] = p + 4 * j + sl < hi ? wn[j] : 0.0f;
        }
        if (PREFETCH && p + STRIDE < hi) fetch(p + STRIDE);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            // the sample lies in the box when none of its coordinates lies
            // outside: the 16 lanes of its row hold every coordinate in
            // xf[j][0] (coordinate l % 16, or l % 16 - d), one ballot
            const float xc = xf[j][0];
            const unsigned long long out = __ballot(!(xc >= 0.0f && xc <= 1.0f));
            in[j] = ((out >> (l & 48)) & 0xFFFFull) == 0ull;
            mx[j] = in[j] ? lbeta2 : -INFINITY;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                float q = 0.0f;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const float z = fmaf(x[j][i], is[t][i], nm[t][i]);
                    q = fmaf(z, z, q);
                }
                at[j][t] = fmaf(-HALF_LOG2E, q, c[t]);   // -inf for components past K
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
                at[j][t] = __builtin_amdgcn_exp2f(at[j][t] - M[j]);   // e^{a - M ln 2}
                se += at[j][t];
            }
            if (defensive && in[j]) se += __builtin_amdgcn_exp2f(lbeta2 - M[j]);
            S[j] = row16_sum(se);
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const float inv_s = S[j] > 0.0f ? __builtin_amdgcn_rcpf(S[j]) : 0.0f;
            const float w_inv_s = w[j] * inv_s;   // w r = e^{a - M} w / S
            const double wd = (double)w[j];
            if (l % 16 == 0) {
                lw += wd * (double)((M[j] + __builtin_amdgcn_logf(S[j])) * LN2);
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
                const double wr = (double)(at[j][t] * w_inv_s);
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
// Gradient of L = -sum w log u / sum w with respect to the mixture outputs,
// from the uncentred moments (float64): with S1 = sum w r (x - m) / s and
// S2 = sum w r ((x - m) / s)^2,
//   S1_ki = (P1_ki - m_ki S0_k) / s_ki
//   S2_ki = (P2_ki - 2 m_ki P1_ki + m_ki^2 S0_k) / s_ki^2
//   dL/dlogit_k = -(S0_k - pi_k sum_j S0_j) / W
//   dL/dm_ki    = -S1_ki / (W s_ki)
//   dL/dlog s_ki = -(S2_ki - S0_k) / W
// (one wave: lane k takes component k)
template <int D>
__device__ __forceinline__ void nll_grad_wave(const NllArgs &a, const double *totals) {
    const int k = threadIdx.x;
    const int K = a.n_comp;
    const double *S = totals;
    const double s0 = S[k], lw = S[(1 + 2 * D) * 64], W = S[(1 + 2 * D) * 64 + 1];
    const bool act = k < K;
    const float logit = act ? a.gmm[k] : -INFINITY;
    const float lmax = wave_max(logit);
    const float pk = act ? expf(logit - lmax) : 0.0f;
    const float pi = pk / wave_sum(pk);
    // sum_j S0_j by a butterfly over the wave (a fixed order)
    const double s0tot = wave_sum(act ? s0 : 0.0);
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

// totals[j] = sum over blocks b of partials[b][j]: a workgroup takes 16
// entries; its thread (part q, entry e) sums blocks q, q + 16, ... in order,
// and the 16 parts are then added in order of q (a fixed order, so the
// totals are bit-reproducible).  The workgroup that finishes last (a
// device-scope counter, zeroed by the NLL launch) then turns the totals
// into the loss and the gradient.
template <int D>
__global__ __launch_bounds__(256) void gmm_nll_sum_kernel(NllArgs a) {
    constexpr int entries = nll_rows(D) * 64;
    __shared__ double part[256];
    __shared__ bool last;
    const int e = threadIdx.x % 16, q = threadIdx.x / 16;
    const int j = blockIdx.x * 16 + e;
    const double *partials = a.partials;
    double v = 0.0;
    if (j < entries)
        for (int b = q; b < a.n_blocks; b += 16) v += partials[(int64_t)b * entries + j];
    part[threadIdx.x] = v;
    __syncthreads();
    if (q == 0 && j < entries) {
        double t = part[e];
        for (int r = 1; r < 16; ++r) t += part[16 * r + e];
        a.totals[j] = t;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(a.done, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (threadIdx.x < 64) nll_grad_wave<D>(a, a.totals);
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

hipError_t launch_mlp_forward_f32(const MlpDims &m, const float *theta, const float *ctx, int G, float *act,
                                  float *out, hipStream_t s) {
    hipLaunchKernelGGL(mlp_forward_f32_kernel, dim3((m.O + 255) / 256, G), dim3(256), 0, s, m, theta, ctx, G, act,
                       out);
    return hipGetLastError();
}

hipError_t launch_mlp_backward_f32(const MlpDims &m, const float *theta, const float *ctx, int G, const float *act,
                                   const float *dout, float *work, float *grad, hipStream_t s) {
    const int64_t n3 = (int64_t)m.O * m.H + m.O;
    const int64_t blocks = 1 + std::min<int64_t>((n3 + 255) / 256, 4096);
    hipLaunchKernelGGL(mlp_backward_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, m, theta, ctx, G, act, dout,
                       work, grad);
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
    hipLaunchKernelGGL(gmm_nll_sum_kernel<D>, dim3((entries + 15) / 16), dim3(256), 0, s, a);
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
