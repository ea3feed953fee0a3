// Launch interface of the learned-mu training kernels (learn_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace restore {

constexpr int LEARN_MAX_DIM = 16;
// The NLL statistics: at most NLL_MAX_BLOCKS workgroups of NLL_WAVES waves,
// each writing nll_rows(d) x 64 float64 partial sums; the workspace holds
// them, the totals and a completion counter (one more line of 64), for any
// n, K and d (about 4.5 MB).
constexpr int NLL_MAX_BLOCKS = 256;
constexpr int NLL_WAVES = 8;
__host__ __device__ constexpr int nll_rows(int D) { return 2 + 2 * D; }
constexpr size_t NLL_WORKSPACE_DOUBLES = (size_t)(NLL_MAX_BLOCKS + 1) * 64 * (2 + 2 * LEARN_MAX_DIM) + 64;

struct NllArgs {
    int32_t n_comp, dim;
    float beta;
    const float *gmm;      // [logits K | means K*d | log_std K*d]
    const float *x;        // [n][d]
    const float *w;        // [n]
    int64_t n;
    int32_t n_blocks;      // <= NLL_MAX_BLOCKS
    int64_t per_block;     // samples per workgroup (a multiple of 4 NLL_WAVES)
    double *partials;      // [n_blocks][nll_rows(dim)][64]
    double *totals;        // [nll_rows(dim)][64]
    unsigned int *done;    // workgroups of the sum launch that have finished
    float *dout;           // [K (1 + 2d)]
    double *loss;          // [1]
};

hipError_t launch_gemm_bf16(int M, int N, int K, const float *A, int64_t lda, bool transA, const float *B, int64_t ldb,
                            bool transB, float *C, int64_t ldc, bool accumulate, hipStream_t s);
hipError_t launch_bias_gelu(float *z, float *h, const float *bias, int G, int n, hipStream_t s);
hipError_t launch_gelu_back(const float *dh, const float *z, float *dz, int count, hipStream_t s);
hipError_t launch_colsum(const float *d, float *db, int G, int n, hipStream_t s);
hipError_t launch_gmm_nll(const NllArgs &a, hipStream_t s);

// Float32 MLP for a few context rows (matrix-vector products: plain VALU
// FMAs in a fixed order, each layer fused with its bias and GELU).
constexpr int MLP_F32_MAX_WIDTH = 256;   // in_dim and hidden
struct MlpDims {
    int in, H, O;
    int64_t W1, b1, W2, b2, W3, b3;      // offsets into theta
};
hipError_t launch_mlp_forward_f32(const MlpDims &m, const float *theta, const float *ctx, int G, float *act,
                                  float *out, hipStream_t s);
hipError_t launch_mlp_backward_f32(const MlpDims &m, const float *theta, const float *ctx, int G, const float *act,
                                   const float *dout, float *work, float *grad, hipStream_t s);
hipError_t launch_adam(float *theta, const float *grad, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, int t, hipStream_t s);

}  // namespace restore
