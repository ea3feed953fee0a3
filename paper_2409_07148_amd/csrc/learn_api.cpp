// Host runtime of the learned-mu C ABI (include/restore.h, "learned
// regeneration distribution"): parameter layout of the MLP, the forward and
// backward passes as sequences of matrix-core GEMMs and elementwise kernels,
// the weighted NLL of restore samples, and Adam.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "trace.h"
#include "../../include/restore.h"
#include "learn.h"

using namespace restore;

restore_status restore_internal_fail(restore_status code, const char *msg);

namespace {

restore_status fail(restore_status code, const std::string &m) { return restore_internal_fail(code, m.c_str()); }
restore_status hip_fail(hipError_t e, const char *what) {
    return fail(RESTORE_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}


struct Offsets {
    int64_t W1, b1, W2, b2, W3, b3, total;
    int in, H, O;
};

restore_status shape_ok(const restore_mlp_shape *s) {
    if (!s) return fail(RESTORE_E_INVALID_ARG, "null shape");
    if (s->in_dim < 1 || s->in_dim > 4096 || s->hidden < 1 || s->hidden > 4096)
        return fail(RESTORE_E_INVALID_ARG, "in_dim and hidden must be in 1..4096");
    if (s->n_comp < 1 || s->n_comp > 64) return fail(RESTORE_E_INVALID_ARG, "n_comp must be in 1..64");
    if (s->dim < 1 || s->dim > LEARN_MAX_DIM) return fail(RESTORE_E_INVALID_ARG, "dim must be in 1..16");
    if (s->precision < RESTORE_MLP_AUTO || s->precision > RESTORE_MLP_BF16)
        return fail(RESTORE_E_INVALID_ARG, "precision must be RESTORE_MLP_AUTO, _FP32 or _BF16");
    if (s->precision == RESTORE_MLP_FP32 && (s->in_dim > MLP_F32_MAX_WIDTH || s->hidden > MLP_F32_MAX_WIDTH))
        return fail(RESTORE_E_UNSUPPORTED, "the float32 MLP takes in_dim and hidden up to " + std::to_string(MLP_F32_MAX_WIDTH));
    return RESTORE_OK;
}

// The float32 path for explicit FP32, and for AUTO with few context rows
// (matrix-vector products, where bf16 GEMM tiles would be mostly padding).
bool use_f32(const restore_mlp_shape *s, int G) {
    if (s->precision == RESTORE_MLP_FP32) return true;
    return s->precision == RESTORE_MLP_AUTO && G <= 16 && s->in_dim <= MLP_F32_MAX_WIDTH &&
           s->hidden <= MLP_F32_MAX_WIDTH;
}

Offsets offsets(const restore_mlp_shape *s) {
    Offsets o{};
    o.in = s->in_dim;
    o.H = s->hidden;
    o.O = s->n_comp * (1 + 2 * s->dim);
    o.W1 = 0;
    o.b1 = o.W1 + (int64_t)o.H * o.in;
    o.W2 = o.b1 + o.H;
    o.b2 = o.W2 + (int64_t)o.H * o.H;
    o.W3 = o.b2 + o.H;
    o.b3 = o.W3 + (int64_t)o.O * o.H;
    o.total = o.b3 + o.O;
    return o;
}

MlpDims dims(const Offsets &o) {
    MlpDims m{};
    m.in = (int)o.in;
    m.H = (int)o.H;
    m.O = (int)o.O;
    m.W1 = o.W1;
    m.b1 = o.b1;
    m.W2 = o.W2;
    m.b2 = o.b2;
    m.W3 = o.W3;
    m.b3 = o.b3;
    return m;
}

}  // namespace

extern "C" {

restore_status restore_mlp_param_count(const restore_mlp_shape *shape, int64_t *n_params, int64_t *n_act_per_row) {
    restore_status st = shape_ok(shape);
    if (st != RESTORE_OK) return st;
    const Offsets o = offsets(shape);
    if (n_params) *n_params = o.total;
    if (n_act_per_row) *n_act_per_row = 4LL * o.H;
    return RESTORE_OK;
}

restore_status restore_mlp_forward(const restore_mlp_shape *shape, const float *theta, const float *ctx, int32_t G,
                                   float *act, float *out, void *stream) {
    restore::TraceRange trace_range("restore_mlp_forward");
    restore_status st = shape_ok(shape);
    if (st != RESTORE_OK) return st;
    if (!theta || !ctx || !act || !out || G < 1) return fail(RESTORE_E_INVALID_ARG, "null buffer or G < 1");
    const Offsets o = offsets(shape);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (use_f32(shape, G)) {
        hipError_t e = launch_mlp_forward_f32(dims(o), theta, ctx, G, act, out, s);
        if (e != hipSuccess) return hip_fail(e, "mlp forward");
        return RESTORE_OK;
    }
    float *z1 = act, *h1 = act + (int64_t)G * o.H, *z2 = act + 2LL * G * o.H, *h2 = act + 3LL * G * o.H;
    // z1 = ctx W1^T + b1, h1 = gelu(z1); z2 = h1 W2^T + b2, h2 = gelu(z2); out = h2 W3^T + b3
    hipError_t e = launch_gemm_bf16(G, o.H, o.in, ctx, o.in, false, theta + o.W1, o.in, true, z1, o.H, false, s);
    if (e == hipSuccess) e = launch_bias_gelu(z1, h1, theta + o.b1, G, o.H, s);
    if (e == hipSuccess) e = launch_gemm_bf16(G, o.H, o.H, h1, o.H, false, theta + o.W2, o.H, true, z2, o.H, false, s);
    if (e == hipSuccess) e = launch_bias_gelu(z2, h2, theta + o.b2, G, o.H, s);
    if (e == hipSuccess) e = launch_gemm_bf16(G, o.O, o.H, h2, o.H, false, theta + o.W3, o.H, true, out, o.O, false, s);
    if (e == hipSuccess) e = launch_bias_gelu(out, nullptr, theta + o.b3, G, o.O, s);
    if (e != hipSuccess) return hip_fail(e, "mlp forward");
    return RESTORE_OK;
}

restore_status restore_mlp_backward(const restore_mlp_shape *shape, const float *theta, const float *ctx, int32_t G,
                                    const float *act, const float *dout, float *work, float *grad, void *stream) {
    restore::TraceRange trace_range("restore_mlp_backward");
    restore_status st = shape_ok(shape);
    if (st != RESTORE_OK) return st;
    if (!theta || !ctx || !act || !dout || !work || !grad || G < 1) return fail(RESTORE_E_INVALID_ARG, "null buffer");
    const Offsets o = offsets(shape);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (use_f32(shape, G)) {
        hipError_t e = launch_mlp_backward_f32(dims(o), theta, ctx, G, act, dout, work, grad, s);
        if (e != hipSuccess) return hip_fail(e, "mlp backward");
        return RESTORE_OK;
    }
    const float *z1 = act, *h1 = act + (int64_t)G * o.H, *z2 = act + 2LL * G * o.H, *h2 = act + 3LL * G * o.H;
    float *dh = work, *dz = work + (int64_t)G * o.H;
    // out layer: dW3 = dout^T h2, db3 = colsum(dout), dh2 = dout W3
    hipError_t e = launch_gemm_bf16(o.O, o.H, G, dout, o.O, true, h2, o.H, false, grad + o.W3, o.H, false, s);
    if (e == hipSuccess) e = launch_colsum(dout, grad + o.b3, G, o.O, s);
    if (e == hipSuccess) e = launch_gemm_bf16(G, o.H, o.O, dout, o.O, false, theta + o.W3, o.H, false, dh, o.H, false, s);
    // second layer
    if (e == hipSuccess) e = launch_gelu_back(dh, z2, dz, G * o.H, s);
    if (e == hipSuccess) e = launch_gemm_bf16(o.H, o.H, G, dz, o.H, true, h1, o.H, false, grad + o.W2, o.H, false, s);
    if (e == hipSuccess) e = launch_colsum(dz, grad + o.b2, G, o.H, s);
    if (e == hipSuccess) e = launch_gemm_bf16(G, o.H, o.H, dz, o.H, false, theta + o.W2, o.H, false, dh, o.H, false, s);
    // first layer
    if (e == hipSuccess) e = launch_gelu_back(dh, z1, dz, G * o.H, s);
    if (e == hipSuccess) e = launch_gemm_bf16(o.H, o.in, G, dz, o.H, true, ctx, o.in, false, grad + o.W1, o.in, false, s);
    if (e == hipSuccess) e = launch_colsum(dz, grad + o.b1, G, o.H, s);
    if (e != hipSuccess) return hip_fail(e, "mlp backward");
    return RESTORE_OK;
}

restore_status restore_gmm_nll_workspace_bytes(size_t *bytes) {
    if (!bytes) return fail(RESTORE_E_INVALID_ARG, "null bytes");
    *bytes = NLL_WORKSPACE_DOUBLES * sizeof(double);
    return RESTORE_OK;
}

restore_status restore_gmm_nll(int32_t n_comp, int32_t dim, float beta, const float *gmm, const float *x,
                               const float *w, int64_t n, float *dout, double *loss_dev, void *workspace,
                               size_t workspace_bytes, void *stream) {
    restore::TraceRange trace_range("restore_gmm_nll");
    if (n_comp < 1 || n_comp > 64 || dim < 1 || dim > LEARN_MAX_DIM) return fail(RESTORE_E_INVALID_ARG, "bad mixture shape");
    if (!(beta >= 0.0f && beta < 1.0f)) return fail(RESTORE_E_INVALID_ARG, "beta must be in [0, 1)");
    if (!gmm || !x || !w || !dout || !loss_dev || !workspace || n < 1) return fail(RESTORE_E_INVALID_ARG, "null buffer");
    size_t need = 0;
    restore_gmm_nll_workspace_bytes(&need);
    if (workspace_bytes < need) return fail(RESTORE_E_BUFFER_TOO_SMALL, "NLL workspace too small");
    NllArgs a{};
    a.n_comp = n_comp;
    a.dim = dim;
    a.beta = beta;
    a.gmm = gmm;
    a.x = x;
    a.w = w;
    a.n = n;
    // contiguous sample ranges of at least 2048 samples (64 passes of 4 per
    // wave) per workgroup, at most NLL_MAX_BLOCKS workgroups
    const int64_t want = (n + 2047) / 2048;
    a.n_blocks = (int32_t)(want < NLL_MAX_BLOCKS ? want : NLL_MAX_BLOCKS);
    const int64_t quantum = 4 * NLL_WAVES;
    a.per_block = ((n + a.n_blocks - 1) / a.n_blocks + quantum - 1) / quantum * quantum;
    a.partials = static_cast<double *>(workspace);
    a.totals = a.partials + (size_t)NLL_MAX_BLOCKS * 64 * nll_rows(dim);
    a.done = reinterpret_cast<unsigned int *>(a.partials + NLL_WORKSPACE_DOUBLES - 64);
    a.dout = dout;
    a.loss = loss_dev;
    hipError_t e = launch_gmm_nll(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "gmm nll");
    return RESTORE_OK;
}

// Scratch of restore_gmm_nll_noalloc: the NLL workspace (partial sums of at
// most NLL_MAX_BLOCKS workgroups and the totals, for d up to 16), one copy
// per GPU, held until the process ends.  Host code never passes the
// symbol itself to a kernel: its device address is looked up once per
// device with hipGetSymbolAddress and kept in scratch_dev.
static __device__ __align__(256) double scratch[NLL_WORKSPACE_DOUBLES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[SCRATCH_MAX_DEVICES] = {};

restore_status scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(RESTORE_E_UNSUPPORTED, "device id beyond 63");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(RESTORE_E_HIP, "hipGetSymbolAddress(scratch) returned no address");
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return RESTORE_OK;
}
}  // namespace

restore_status restore_gmm_nll_noalloc(int32_t n_comp, int32_t dim, float beta, const float *gmm, const float *x,
                                       const float *w, int64_t n, float *dout, double *loss_dev, void *stream) {
    restore::TraceRange trace_range("restore_gmm_nll_noalloc");
    void *ws = nullptr;
    restore_status st = scratch_address(&ws);
    if (st != RESTORE_OK) return st;
    // the same validation, grid and kernels as restore_gmm_nll; the scratch
    // is the largest workspace that call can ask for, so every valid n, K
    // and d fits, and the kernels write every partial they later read
    return restore_gmm_nll(n_comp, dim, beta, gmm, x, w, n, dout, loss_dev, ws, sizeof(scratch), stream);
}

restore_status restore_adam_step(float *theta, const float *grad, float *m, float *v, int64_t n, int32_t t, float lr,
                                 float beta1, float beta2, float eps, void *stream) {
    restore::TraceRange trace_range("restore_adam_step");
    if (!theta || !grad || !m || !v || n < 1 || t < 1) return fail(RESTORE_E_INVALID_ARG, "bad Adam arguments");
    hipError_t e = launch_adam(theta, grad, m, v, n, lr, beta1, beta2, eps, t, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "adam");
    return RESTORE_OK;
}

}  // extern "C"
