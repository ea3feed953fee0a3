// Float64 reduction of the per-chain tour sums into the sums and residual
// sums of squares behind the tour-ratio estimates (Sec. 6.3, Sec. 7.4) and
// their delta-method standard errors over chains.
//
// Two passes over the chains with a fixed grid and fixed-order trees, so
// the result is bit-reproducible: pass 1 gives sum N, sum T, sum A (and the
// censoring / non-finite counts), the ratios R = T/N, A/N, A/T follow, and
// pass 2 gives sum (T - R N)^2, sum (A - R N)^2, sum (A - R T)^2.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace restore {

constexpr int RED_THREADS = 256;

__device__ __forceinline__ void block_sum(double *sh, double v[], int nv, double *out) {
    const int t = threadIdx.x;
    for (int s = 0; s < nv; ++s) sh[s * RED_THREADS + t] = v[s];
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int s = 0; s < nv; ++s) sh[s * RED_THREADS + t] += sh[s * RED_THREADS + t + w];
        __syncthreads();
    }
    if (t == 0)
        for (int s = 0; s < nv; ++s) out[s] = sh[s * RED_THREADS];
}

__device__ __forceinline__ bool chain_ok(const ReduceArgs &r, int64_t c) {
    return isfinite(r.t_done[c]) && isfinite(r.a_done[c]);
}

__global__ __launch_bounds__(RED_THREADS) void reduce_pass1(ReduceArgs r) {
    __shared__ double sh[6 * RED_THREADS];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t c = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; c < r.n_chains;
         c += (int64_t)gridDim.x * RED_THREADS) {
        if (!chain_ok(r, c)) {
            v[5] += 1.0;
            continue;
        }
        v[0] += (double)r.n_done[c];
        v[1] += r.t_done[c];
        v[2] += r.a_done[c];
        if (r.status[c] & ST_CENSORED) {
            v[3] += 1.0;
            v[4] += (double)r.t_cur[c];
        }
    }
    block_sum(sh, v, 6, r.partials + (size_t)blockIdx.x * RED_SLOTS);
}

__global__ __launch_bounds__(RED_THREADS) void reduce_final(ReduceArgs r, int first, int count) {
    __shared__ double sh[6 * RED_THREADS];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < r.n_blocks; b += RED_THREADS)
        for (int s = 0; s < count; ++s) v[s] += r.partials[(size_t)b * RED_SLOTS + first + s];
    block_sum(sh, v, count, r.results + first);
}

__global__ __launch_bounds__(RED_THREADS) void reduce_pass2(ReduceArgs r) {
    __shared__ double sh[3 * RED_THREADS];
    const double N = r.results[RED_N], T = r.results[RED_T], A = r.results[RED_A];
    const double R_tn = N > 0 ? T / N : 0.0, R_an = N > 0 ? A / N : 0.0, R_at = T > 0 ? A / T : 0.0;
    double v[3] = {0, 0, 0};
    for (int64_t c = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; c < r.n_chains;
         c += (int64_t)gridDim.x * RED_THREADS) {
        if (!chain_ok(r, c)) continue;
        const double n = (double)r.n_done[c], t = r.t_done[c], a = r.a_done[c];
        const double e1 = t - R_tn * n, e2 = a - R_an * n, e3 = a - R_at * t;
        v[0] += e1 * e1;
        v[1] += e2 * e2;
        v[2] += e3 * e3;
    }
    block_sum(sh, v, 3, r.partials + (size_t)blockIdx.x * RED_SLOTS + RED_SS_T_N);
}

hipError_t launch_reduce(const ReduceArgs &r, hipStream_t stream) {
    const dim3 grid(r.n_blocks), block(RED_THREADS);
    hipLaunchKernelGGL(reduce_pass1, grid, block, 0, stream, r);
    hipLaunchKernelGGL(reduce_final, dim3(1), block, 0, stream, r, (int)RED_N, 6);
    hipLaunchKernelGGL(reduce_pass2, grid, block, 0, stream, r);
    hipLaunchKernelGGL(reduce_final, dim3(1), block, 0, stream, r, (int)RED_SS_T_N, 3);
    return hipGetLastError();
}

// Tile-stratified runs: one workgroup per tile, the same two passes over
// the tile's chains (fixed strides and trees: bit-reproducible), giving the
// tile's sums and the residual sums of squares and products of its two
// tour ratios T/N and A/N.
__global__ __launch_bounds__(RED_THREADS) void tile_reduce_kernel(TileReduceArgs r) {
    __shared__ double sh[6 * RED_THREADS];
    __shared__ double res[9];
    const int64_t T = r.n_tiles, t = blockIdx.x;
    const int64_t lo = (t * r.n_chains + T - 1) / T, hi = ((t + 1) * r.n_chains + T - 1) / T;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t c = lo + threadIdx.x; c < hi; c += RED_THREADS) {
        if (!(isfinite(r.t_done[c]) && isfinite(r.a_done[c]))) {
            v[5] += 1.0;
            continue;
        }
        v[0] += (double)r.n_done[c];
        v[1] += r.t_done[c];
        v[2] += r.a_done[c];
        if (r.status[c] & ST_CENSORED) {
            v[3] += 1.0;
            v[4] += (double)r.t_cur[c];
        }
    }
    block_sum(sh, v, 6, res);
    __syncthreads();
    const double N = res[0], RT = N > 0 ? res[1] / N : 0.0, RA = N > 0 ? res[2] / N : 0.0;
    double w[3] = {0, 0, 0};
    for (int64_t c = lo + threadIdx.x; c < hi; c += RED_THREADS) {
        if (!(isfinite(r.t_done[c]) && isfinite(r.a_done[c]))) continue;
        const double n = (double)r.n_done[c];
        const double eT = r.t_done[c] - RT * n, eA = r.a_done[c] - RA * n;
        w[0] += eT * eT;
        w[1] += eA * eA;
        w[2] += eT * eA;
    }
    block_sum(sh, w, 3, res + 6);
    if (threadIdx.x == 0) {
        double *o = r.results + t * TR_SLOTS;
        for (int s = 0; s < TR_SLOTS; ++s) o[s] = 0.0;
        o[TR_N] = res[0];
        o[TR_T] = res[1];
        o[TR_A] = res[2];
        o[TR_CENS] = res[3];
        o[TR_CENS_T] = res[4];
        o[TR_NONFINITE] = res[5];
        o[TR_SS_TT] = res[6];
        o[TR_SS_AA] = res[7];
        o[TR_SS_TA] = res[8];
        o[TR_CHAINS] = (double)(hi - lo);
    }
}

hipError_t launch_tile_reduce(const TileReduceArgs &r, hipStream_t stream) {
    hipLaunchKernelGGL(tile_reduce_kernel, dim3(r.n_tiles), dim3(RED_THREADS), 0, stream, r);
    return hipGetLastError();
}

}  // namespace restore
