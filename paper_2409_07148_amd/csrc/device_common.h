// Device helpers of the gfx950 restore kernels: the counter-based random
// stream, the uniform / normal / exponential mappings and small math.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "restore_internal.h"

namespace restore {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with a Weyl-sequence key schedule.  The key and all
// counter words except the chain id are wave-uniform, so the first rounds
// run largely on the scalar unit.  From the fourth round on every word
// differs between lanes, and each of the round's two three-way xors is one
// gfx950 three-input bit operation (truth table 0x96 = a ^ b ^ c) instead
// of two xors; the first three rounds keep plain xors, whose wave-uniform
// parts the compiler moves to the scalar unit.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

struct Philox {
    static constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    static constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;

    __device__ __forceinline__ static void block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            const uint64_t p0 = (uint64_t)M0 * c0;
            const uint64_t p1 = (uint64_t)M1 * c2;
            const uint32_t h1 = (uint32_t)(p1 >> 32), h0 = (uint32_t)(p0 >> 32);
            const uint32_t n0 = r < 3 ? h1 ^ c1 ^ k0 : xor3(h1, c1, k0);
            const uint32_t n2 = r < 3 ? h0 ^ c3 ^ k1 : xor3(h0, c3, k1);
            c1 = (uint32_t)p1;
            c3 = (uint32_t)p0;
            c0 = n0;
            c2 = n2;
            k0 += W0;
            k1 += W1;
        }
        out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
    }
};

// Odd 23-bit uniform in (0,1): (2 (r >> 9) + 1) 2^-24 == ((r >> 8) | 1) 2^-24,
// exact in float32.  Built from the exponent bits: f = 1 + (r >> 9) 2^-23
// lies in [1, 2), and f - (1 - 2^-24) is exact (Sterbenz) and equals
// (r >> 9) 2^-23 + 2^-24.  The bits of f, (r >> 9) | 0x3F800000, are one
// funnel shift of the 64-bit pair (0x7F, r).
__device__ __forceinline__ float u01(uint32_t r) {
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, r, 9)) - 0x1.fffffep-1f;
}

// ln u of a uniform from u01 (u >= 2^-24, so no denormal-range handling):
// the hardware base-2 logarithm times ln 2, a few ulps of ln u.
__device__ __forceinline__ float ln_u01(float u) {
    return __builtin_amdgcn_logf(u) * 0.6931471805599453f;
}

// Uniforms of one step: head = (u_E1, u_E2, u_acc, u_cat) from block 0;
// cand[0 .. 4*NB) from blocks 1..NB.
template <int NB>
__device__ __forceinline__ void draw_step(uint32_t step, uint32_t chain, uint32_t target,
                                          uint32_t purpose, uint32_t k0, uint32_t k1,
                                          float head[4], float cand[4 * NB]) {
    uint32_t r[4];
    Philox::block(step, chain, target, purpose << 16, k0, k1, r);
#pragma unroll
    for (int i = 0; i < 4; ++i) head[i] = u01(r[i]);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        Philox::block(step, chain, target, (purpose << 16) | (uint32_t)(b + 1), k0, k1, r);
#pragma unroll
        for (int i = 0; i < 4; ++i) cand[4 * b + i] = u01(r[i]);
    }
}

// Box-Muller on consecutive candidate pairs: z_{2m} = rho cos(2 pi u_{2m+1}),
// z_{2m+1} = rho sin(2 pi u_{2m+1}), rho = sqrt(-2 ln u_{2m}).  The hardware
// sine/cosine take their argument in revolutions.  -2 ln u >= 1.1e-7 for
// the odd 23-bit uniforms, so HW_SQRT may take the hardware square root
// without the library's denormal and rounding fix-ups (about 1 ulp): the
// learned mu's sampler does; the local proposals keep sqrtf, with which the
// uniform-mu step kernel schedules 1% faster.
template <int D, int NC, bool HW_SQRT = false>
__device__ __forceinline__ void box_muller(const float cand[NC], float z[D]) {
#pragma unroll
    for (int m = 0; 2 * m < D; ++m) {
        const float r2 = -2.0f * ln_u01(cand[2 * m]);
        const float rho = HW_SQRT ? __builtin_amdgcn_sqrtf(r2) : sqrtf(r2);
        const float ang = cand[2 * m + 1];
        z[2 * m] = rho * __builtin_amdgcn_cosf(ang);
        if (2 * m + 1 < D) z[2 * m + 1] = rho * __builtin_amdgcn_sinf(ang);
    }
}

// e^x through the hardware base-2 exponential (relative error about
// |x| 2^-24 from the rounding of x log2 e, plus the instruction's own);
// used for the killing rate, the integrand p = e^{log p} and the natural-
// log sums of lse_push.
__device__ __forceinline__ float exp_rel(float x) {
    return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
}

// One term of an online log-sum-exp in natural logs (the inflow density of
// the unadjusted jump process; the mixture densities use lse2_block below),
// (M, S) <- (max(M, a), S e^{M - max} + e^{a - max}), with a single
// exponential: of the two factors one is exactly 1 and the other is
// e^{-|a - M|}.  sc and w return the factors applied to the old sum and to
// the new term (for running gradient sums).  Same values, bit for bit, as
// evaluating both factors.
__device__ __forceinline__ void lse_push(float &M, float &S, float a, float &sc, float &w) {
    const float d = a - M;
    const float e = exp_rel(-fabsf(d));
    const bool up = d > 0.0f;
    sc = up ? e : 1.0f;
    w = up ? 1.0f : e;
    S = up ? fmaf(S, e, 1.0f) : S + e;
    M = up ? a : M;
}

// Mixture log-densities in base 2.  The host folds log2 e into the packed
// component parameters, so a component's term a_k = log2(w_k N_k(y)) comes
// straight out of its quadratic form and its weight is exp2 of a difference
// of terms: no scaling per component.  log2 of a sum is converted back to a
// natural logarithm once, at the end.
constexpr float LOG2E = 1.4426950408889634f;
constexpr float LN2 = 0.6931471805599453f;

// B terms of a blocked online log-sum-exp in base 2:
//   m = max(M, a_0, .., a_{B-1}),  S <- S 2^{M - m} + sum_b 2^{a_b - m},  M <- m.
// sc = 2^{M - m} and w_b = 2^{a_b - m} are returned for running gradient
// sums.  One max per term and one exponential per term plus one per block
// (the per-term update of lse_push costs a compare, two selects and a
// choice of sums instead).  S >= 1 once a term has been pushed (the largest
// term contributes 2^0).  M = -inf (empty sum) gives sc = 0; every a_b must
// be > -inf, which the packed parameters guarantee by flooring each
// component's log-weight at -2^100 instead of -inf.  A block of one term
// takes lse_push's form in base 2 (one exponential instead of two).
template <int B>
__device__ __forceinline__ void lse2_block(float &M, float &S, const float (&a)[B], float &sc, float (&w)[B]) {
    if constexpr (B == 1) {
        const float d = a[0] - M;
        const float e = __builtin_amdgcn_exp2f(-fabsf(d));
        const bool up = d > 0.0f;
        sc = up ? e : 1.0f;
        w[0] = up ? 1.0f : e;
        S = up ? fmaf(S, e, 1.0f) : S + e;
        M = up ? a[0] : M;
        return;
    }
    float m = M;
#pragma unroll
    for (int b = 0; b < B; ++b) m = fmaxf(m, a[b]);
    sc = __builtin_amdgcn_exp2f(M - m);
#pragma unroll
    for (int b = 0; b < B; ++b) w[b] = __builtin_amdgcn_exp2f(a[b] - m);
    float t;
    if constexpr (B == 4) {
        t = (w[0] + w[1]) + (w[2] + w[3]);
    } else {
        t = w[0];
#pragma unroll
        for (int b = 1; b < B; ++b) t += w[b];
    }
    S = fmaf(S, sc, t);
    M = m;
}

// ln of the base-2 log-sum-exp (M, S): (M + log2 S) ln 2, with S >= 1 (no
// denormal range for the hardware logarithm).
__device__ __forceinline__ float lse2_ln(float M, float S) {
    return fmaf(M, LN2, __builtin_amdgcn_logf(S) * LN2);
}

// y in [0,1]^d.  A float in [+0, 1] has bits 0 .. 0x3F800000 as an unsigned
// integer, while negative values and NaNs lie above that, so the test is one
// unsigned maximum over the coordinates (three-input maxima) and one compare
// instead of two float compares per coordinate.  -0 counts as outside; no
// state holds it: uniforms are >= 2^-24, and a move adds a nonzero Gaussian
// step (the Box-Muller cosine and sine of an odd multiple of 2^-24
// revolutions are never zero), whose exact cancellation gives +0.
template <int D>
__device__ __forceinline__ bool in_unit_box(const float y[D]) {
    uint32_t m = __float_as_uint(y[0]);
#pragma unroll
    for (int i = 1; i < D; ++i) m = max(m, __float_as_uint(y[i]));
    return m <= 0x3F800000u;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

}  // namespace restore
