// Host runtime of the batched C ABI (include/restore.h, "batched targets"):
// descriptor validation, parameter packing for every target, the work
// queue (tiles of chains ordered longest-processing-time first), hipGraph
// capture of one batch pass, the per-target comparison mode, and the
// autotuner that picks the tiling and caches its choice in a JSON file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "trace.h"
#include "../../include/restore.h"
#include "batch.h"
#include "restore_internal.h"

using namespace restore;

// defined in restore_api.cpp
restore_status restore_internal_fail(restore_status code, const char *msg);
restore_status restore_internal_pack_full(const restore_target *t, std::vector<float> *out);
restore_status restore_internal_pack_mu(const std::vector<float> &raw, int K, int d, float beta,
                                        std::vector<float> *out);

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

restore_status fail(restore_status code, const std::string &msg) { return restore_internal_fail(code, msg.c_str()); }
restore_status hip_fail(hipError_t e, const char *what) {
    return fail(RESTORE_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct BLayout {
    size_t targets, items, params, heads, counters, results, n_done, t_done, a_done, status, t_cur, total;
    size_t max_items, n_param_floats;
    int64_t total_chains;
};

bool learned(const restore_mu *mus, int i) { return mus && mus[i].kind == RESTORE_MU_GMM_DIAG; }

BLayout make_layout(int n, const restore_target *t, const restore_config *c, const restore_mu *mus) {
    BLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    L.max_items = 0;
    L.n_param_floats = 0;
    L.total_chains = 0;
    for (int i = 0; i < n; ++i) {
        L.max_items += (size_t)((c[i].n_chains + 63) / 64);
        L.n_param_floats += (size_t)comp_stride(TGT_FULL, t[i].dim) * t[i].n_comp;
        if (learned(mus, i)) L.n_param_floats += (size_t)mu_slab_floats(t[i].dim, mus[i].n_comp);
        L.total_chains += c[i].n_chains;
    }
    const size_t C = (size_t)L.total_chains;
    L.targets = take(sizeof(BatchTarget) * n);
    L.items = take(sizeof(WorkItem) * L.max_items);
    L.params = take(4 * L.n_param_floats);
    L.heads = take(4 * BATCH_HEADS);
    L.counters = take(8 * BC_SLOTS * (size_t)n);
    L.results = take(8 * BS_SLOTS * (size_t)n);
    L.n_done = take(4 * C);
    L.t_done = take(8 * C);
    L.a_done = take(8 * C);
    L.status = take(4 * C);
    L.t_cur = take(4 * C);
    L.total = o;
    return L;
}

restore_status validate(int n, const restore_target *t, const restore_local_kernel *lk, const restore_config *c,
                        const restore_mu *mus) {
    if (n < 1 || n > (1 << 16)) return fail(RESTORE_E_INVALID_ARG, "n_targets outside 1..65536");
    if (!t || !lk || !c) return fail(RESTORE_E_INVALID_ARG, "null descriptor array");
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        const std::string at = "target " + std::to_string(i) + ": ";
        if (mus) {
            if (mus[i].kind != RESTORE_MU_UNIFORM_BOX && mus[i].kind != RESTORE_MU_GMM_DIAG)
                return fail(RESTORE_E_INVALID_ARG, at + "unknown mu kind");
            if (mus[i].kind == RESTORE_MU_GMM_DIAG) {
                if (mus[i].n_comp < 1 || mus[i].n_comp > RESTORE_MAX_COMP || !mus[i].params_dev)
                    return fail(RESTORE_E_INVALID_ARG, at + "GMM_DIAG mu needs 1..64 components and device params");
                if (!(mus[i].beta >= 0.0f && mus[i].beta <= 1.0f))
                    return fail(RESTORE_E_INVALID_ARG, at + "mu beta outside [0,1]");
            }
        }
        if (t[i].kind != RESTORE_TARGET_GMM_FULL)
            return fail(RESTORE_E_UNSUPPORTED, at + "the batched path takes full-covariance mixtures");
        if (t[i].dim < 1 || t[i].dim > RESTORE_MAX_DIM) return fail(RESTORE_E_INVALID_ARG, at + "dim outside 1..16");
        if (t[i].n_comp < 1 || t[i].n_comp > RESTORE_MAX_COMP) return fail(RESTORE_E_INVALID_ARG, at + "n_comp outside 1..64");
        const int d = t[i].dim, K = t[i].n_comp;
        if (!t[i].params || t[i].params_count != (int64_t)K * (1 + d + d * d))
            return fail(RESTORE_E_INVALID_ARG, at + "params missing or of the wrong length");
        for (int64_t j = 0; j < t[i].params_count; ++j)
            if (!std::isfinite(t[i].params[j])) return fail(RESTORE_E_NONFINITE, at + "non-finite parameter");
        if (lk[i].kind != RESTORE_LOCAL_RWMH)
            return fail(RESTORE_E_UNSUPPORTED, at + "the batched path runs random-walk MH local moves");
        if (!std::isfinite(lk[i].step) || lk[i].step < 0.0f) return fail(RESTORE_E_INVALID_ARG, at + "step must be >= 0");
        if (lk[i].large_step_prob != 0.0f)
            return fail(RESTORE_E_UNSUPPORTED, at + "large_step_prob must be 0 (restore runs the small-step chain M^0)");
        if (c[i].n_chains < 1 || c[i].n_chains > 0x7fffffffLL) return fail(RESTORE_E_INVALID_ARG, at + "n_chains outside 1..2^31-1");
        if (!std::isfinite(c[i].c_tilde) || c[i].c_tilde < 0.0) return fail(RESTORE_E_INVALID_ARG, at + "c_tilde must be >= 0");
        if (c[i].c_tilde == 0.0)
            return fail(RESTORE_E_UNSUPPORTED, at + "c_tilde = 0 (the MH chain) runs on the single-target path");
        if (c[i].drain_cap < 0) return fail(RESTORE_E_INVALID_ARG, at + "drain_cap must be >= 0");
        if (c[i].first_chain < 0) return fail(RESTORE_E_INVALID_ARG, at + "first_chain must be >= 0");
        if (c[i].integrands & RESTORE_INTEGRAND_PIXEL) return fail(RESTORE_E_UNSUPPORTED, at + "no pixel integrand in batches");
        total += c[i].n_chains;
    }
    if (total > 0x7fffffffLL) return fail(RESTORE_E_INVALID_ARG, "more than 2^31-1 chains in the batch");
    return RESTORE_OK;
}

struct Bucket {
    int dlo, dhi, mu;
    BatchKernels k;
    size_t item_begin, item_count;
    int grid;
};

}  // namespace

struct restore_batch {
    int n = 0;
    int32_t n_steps = 0;
    std::vector<BatchTarget> targets;
    std::vector<double> c_tilde;
    BLayout lay{};
    char *base = nullptr;
    restore_batch_tiling tiling{};
    std::vector<Bucket> buckets;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    int n_cu = 0;
};

namespace {

template <typename T>
T *at(restore_batch *b, size_t off) { return reinterpret_cast<T *>(b->base + off); }

BatchArgs args_for(restore_batch *b, const Bucket *bk, int head_index) {
    BatchArgs a{};
    a.targets = at<BatchTarget>(b, b->lay.targets);
    a.items = at<WorkItem>(b, b->lay.items) + (bk ? bk->item_begin : 0);
    a.n_items = bk ? (int32_t)bk->item_count : 0;
    a.n_targets = b->n;
    a.queue_head = at<int32_t>(b, b->lay.heads) + head_index;
    a.params = at<float>(b, b->lay.params);
    a.n_done = at<uint32_t>(b, b->lay.n_done);
    a.t_done = at<double>(b, b->lay.t_done);
    a.a_done = at<double>(b, b->lay.a_done);
    a.status = at<uint32_t>(b, b->lay.status);
    a.t_cur = at<float>(b, b->lay.t_cur);
    a.counters = at<unsigned long long>(b, b->lay.counters);
    a.results = at<double>(b, b->lay.results);
    return a;
}

void drop_graph(restore_batch *b) {
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
}

// Build the work items of every bucket for the current tiling and upload
// them (the upload is synchronous: the host vector goes away).
restore_status build_items(restore_batch *b, hipStream_t s) {
    const int block = b->tiling.block_size;
    std::vector<std::pair<int, int>> ranges;
    if (b->tiling.buckets == RESTORE_BATCH_BUCKETS_DIM4) ranges = {{1, 4}, {5, 8}, {9, 12}, {13, 16}};
    else ranges = {{1, 16}};
    std::vector<WorkItem> all;
    b->buckets.clear();
    for (int mu : {(int)MU_UNIFORM, (int)MU_GMM})
    for (auto r : ranges) {
        Bucket bk{};
        bk.dlo = r.first;
        bk.dhi = r.second;
        bk.mu = mu;
        bk.k = find_batch_kernels(r.first, r.second, mu);
        if (!bk.k.persistent) return fail(RESTORE_E_UNSUPPORTED, "batch kernels for this dimension range are not built");
        std::vector<std::pair<double, WorkItem>> items;
        for (int i = 0; i < b->n; ++i) {
            const BatchTarget &t = b->targets[i];
            if (t.d < r.first || t.d > r.second || t.mu_kind != mu) continue;
            // cost of a tile ~ chains x (components x (d^2 + 3d) + mu components x 3d) per step
            const double per_chain = (double)t.K * (t.d * t.d + 3 * t.d + 7) +
                                     (mu == MU_GMM ? (double)t.mu_comp * (3 * t.d + 9) : 0.0);
            for (int f = 0; f < t.n_chains; f += block) {
                WorkItem w{};
                w.target = i;
                w.first = f;
                w.count = std::min(block, t.n_chains - f);
                items.push_back({per_chain * w.count, w});
            }
        }
        if (b->tiling.order == RESTORE_BATCH_ORDER_LPT)
            std::stable_sort(items.begin(), items.end(),
                             [](const std::pair<double, WorkItem> &x, const std::pair<double, WorkItem> &y) {
                                 return x.first > y.first;
                             });
        bk.item_begin = all.size();
        bk.item_count = items.size();
        for (auto &it : items) all.push_back(it.second);
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bk.k.persistent, block, 0);
        if (e != hipSuccess) return hip_fail(e, "occupancy query");
        bk.grid = std::max(1, per_cu) * b->n_cu;
        if (bk.item_count) b->buckets.push_back(bk);
    }
    if (all.size() > b->lay.max_items) return fail(RESTORE_E_INVALID_ARG, "work item overflow");
    hipError_t e = hipMemcpyAsync(at<WorkItem>(b, b->lay.items), all.data(), all.size() * sizeof(WorkItem),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "work item upload");
    drop_graph(b);
    return RESTORE_OK;
}

hipError_t enqueue_persistent(restore_batch *b, hipStream_t s) {
    BatchArgs z = args_for(b, nullptr, 0);
    hipError_t e = launch_batch_zero(z, s);
    if (e != hipSuccess) return e;
    for (size_t i = 0; i < b->buckets.size(); ++i) {
        const Bucket &bk = b->buckets[i];
        BatchArgs a = args_for(b, &bk, (int)i + 1);
        void *kargs[] = {&a};
        e = hipLaunchKernel(bk.k.persistent, dim3(bk.grid), dim3(b->tiling.block_size), kargs, 0, s);
        if (e != hipSuccess) return e;
    }
    return launch_batch_reduce(z, s);
}

// zero kernel also clears the queue heads of every bucket
__global__ void heads_zero_kernel(int32_t *h) {
    if (threadIdx.x < BATCH_HEADS) h[threadIdx.x] = 0;
}

}  // namespace

extern "C" {

restore_status restore_batch_state_bytes(int32_t n_targets, const restore_target *targets,
                                         const restore_local_kernel *locals, const restore_config *cfgs,
                                         const restore_mu *mus, size_t *bytes_out) {
    if (!bytes_out) return fail(RESTORE_E_INVALID_ARG, "null bytes_out");
    restore_status st = validate(n_targets, targets, locals, cfgs, mus);
    if (st != RESTORE_OK) return st;
    *bytes_out = make_layout(n_targets, targets, cfgs, mus).total;
    return RESTORE_OK;
}

restore_status restore_batch_init(restore_batch **out, int32_t n_targets, const restore_target *targets,
                                  const restore_local_kernel *locals, const restore_config *cfgs,
                                  const restore_mu *mus, int32_t n_steps, void *state_dev, size_t state_bytes,
                                  void *stream) {
    restore::TraceRange trace_range("restore_batch_init");
    if (!out) return fail(RESTORE_E_INVALID_ARG, "null out");
    *out = nullptr;
    restore_status st = validate(n_targets, targets, locals, cfgs, mus);
    if (st != RESTORE_OK) return st;
    if (n_steps < 0) return fail(RESTORE_E_INVALID_ARG, "n_steps must be >= 0");
    if (!state_dev || reinterpret_cast<uintptr_t>(state_dev) % ALIGN)
        return fail(RESTORE_E_INVALID_ARG, "state buffer must be non-null and 256-byte aligned");
    const BLayout lay = make_layout(n_targets, targets, cfgs, mus);
    if (state_bytes < lay.total) return fail(RESTORE_E_BUFFER_TOO_SMALL, "batch state buffer too small");
    for (int i = 0; i < n_targets; ++i)
        if ((int64_t)n_steps + cfgs[i].drain_cap > 0x7fffffffLL) return fail(RESTORE_E_INVALID_ARG, "step counter overflow");

    restore_batch *b = new (std::nothrow) restore_batch();
    if (!b) return fail(RESTORE_E_INVALID_ARG, "out of host memory");
    b->n = n_targets;
    b->n_steps = n_steps;
    b->lay = lay;
    b->base = static_cast<char *>(state_dev);
    std::vector<float> slab, one;
    int64_t offset = 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < n_targets; ++i) {
        st = restore_internal_pack_full(&targets[i], &one);
        if (st != RESTORE_OK) { delete b; return st; }
        BatchTarget t{};
        t.d = targets[i].dim;
        t.K = targets[i].n_comp;
        t.no_kill = cfgs[i].c_tilde == 0.0 ? 1 : 0;
        t.log_c = cfgs[i].c_tilde > 0.0 ? (float)std::log(cfgs[i].c_tilde) : 0.0f;
        t.step = locals[i].step;
        t.target_id = (uint32_t)cfgs[i].target_id;
        t.key0 = (uint32_t)(cfgs[i].seed & 0xffffffffu);
        t.key1 = (uint32_t)(cfgs[i].seed >> 32);
        t.chain0 = (uint32_t)cfgs[i].first_chain;
        t.chain_offset = offset;
        t.n_chains = (int32_t)cfgs[i].n_chains;
        t.param_offset = (int32_t)slab.size();
        t.n_steps = n_steps;
        t.drain_cap = cfgs[i].drain_cap;
        t.integrand_p = (cfgs[i].integrands & RESTORE_INTEGRAND_P) ? 1 : 0;
        slab.insert(slab.end(), one.begin(), one.end());
        t.mu_kind = MU_UNIFORM;
        if (learned(mus, i)) {
            // the learned-mu form: the caller's device row, read once and
            // factorised in float64 as for a single-target run
            const int K = mus[i].n_comp, d = t.d;
            std::vector<float> raw((size_t)K * (1 + 2 * d));
            hipError_t e = hipMemcpyAsync(raw.data(), mus[i].params_dev, raw.size() * sizeof(float),
                                          hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) { delete b; return hip_fail(e, "mu parameter read"); }
            st = restore_internal_pack_mu(raw, K, d, mus[i].beta, &one);
            if (st != RESTORE_OK) { delete b; return st; }
            t.mu_kind = MU_GMM;
            t.mu_comp = K;
            t.mu_beta = mus[i].beta;
            t.mu_offset = (int32_t)slab.size();
            slab.insert(slab.end(), one.begin(), one.end());
        }
        b->targets.push_back(t);
        b->c_tilde.push_back(cfgs[i].c_tilde);
        offset += cfgs[i].n_chains;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) { delete b; return hip_fail(e, "device query"); }
    b->n_cu = prop.multiProcessorCount;
    e = hipMemcpyAsync(at<BatchTarget>(b, lay.targets), b->targets.data(), sizeof(BatchTarget) * n_targets,
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(at<float>(b, lay.params), slab.data(), slab.size() * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { delete b; return hip_fail(e, "batch upload"); }
    hipLaunchKernelGGL(heads_zero_kernel, dim3(1), dim3(64), 0, s, at<int32_t>(b, lay.heads));
    e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { delete b; return hip_fail(e, "capture stream"); }
    b->tiling.block_size = 256;
    b->tiling.order = RESTORE_BATCH_ORDER_LPT;
    b->tiling.buckets = RESTORE_BATCH_BUCKETS_ONE;
    st = build_items(b, s);
    if (st != RESTORE_OK) { (void)hipStreamDestroy(b->cap_stream); delete b; return st; }
    *out = b;
    return RESTORE_OK;
}

restore_status restore_batch_set_tiling(restore_batch *b, const restore_batch_tiling *tiling) {
    if (!b || !tiling) return fail(RESTORE_E_INVALID_ARG, "null argument");
    if (tiling->block_size != 64 && tiling->block_size != 128 && tiling->block_size != 256)
        return fail(RESTORE_E_INVALID_ARG, "block_size must be 64, 128 or 256");
    if (tiling->order != RESTORE_BATCH_ORDER_LPT && tiling->order != RESTORE_BATCH_ORDER_TARGET)
        return fail(RESTORE_E_INVALID_ARG, "unknown order");
    if (tiling->buckets != RESTORE_BATCH_BUCKETS_ONE && tiling->buckets != RESTORE_BATCH_BUCKETS_DIM4)
        return fail(RESTORE_E_INVALID_ARG, "unknown bucketing");
    b->tiling = *tiling;
    b->tiling.reserved = 0;
    return build_items(b, nullptr);
}

restore_status restore_batch_get_tiling(const restore_batch *b, restore_batch_tiling *tiling) {
    if (!b || !tiling) return fail(RESTORE_E_INVALID_ARG, "null argument");
    *tiling = b->tiling;
    return RESTORE_OK;
}

restore_status restore_batch_run(restore_batch *b, int32_t mode, void *stream) {
    restore::TraceRange trace_range("restore_batch_run");
    if (!b) return fail(RESTORE_E_INVALID_ARG, "null batch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (mode == RESTORE_BATCH_MODE_GRAPH) {
        if (!b->exec) {
            // capture zero + persistent kernel(s) + per-target reduction once
            hipGraph_t g = nullptr;
            e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "begin capture");
            hipError_t e2 = enqueue_persistent(b, b->cap_stream);
            e = hipStreamEndCapture(b->cap_stream, &g);
            if (e2 != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_fail(e2, "captured launch"); }
            if (e != hipSuccess) return hip_fail(e, "end capture");
            e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) { b->exec = nullptr; return hip_fail(e, "graph instantiate"); }
        }
        e = hipGraphLaunch(b->exec, s);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
        return RESTORE_OK;
    }
    if (mode == RESTORE_BATCH_MODE_PERSISTENT) {
        e = enqueue_persistent(b, s);
        if (e != hipSuccess) return hip_fail(e, "persistent launch");
        return RESTORE_OK;
    }
    if (mode == RESTORE_BATCH_MODE_SEPARATE) {
        BatchArgs z = args_for(b, nullptr, 0);
        e = launch_batch_zero(z, s);
        if (e != hipSuccess) return hip_fail(e, "zero launch");
        for (int i = 0; i < b->n; ++i) {
            const BatchTarget &t = b->targets[i];
            const Bucket *bk = nullptr;
            for (const Bucket &x : b->buckets)
                if (t.d >= x.dlo && t.d <= x.dhi && t.mu_kind == x.mu) bk = &x;
            if (!bk) return fail(RESTORE_E_UNSUPPORTED, "no bucket for a target");
            BatchArgs a = args_for(b, bk, 0);
            int32_t ti = i;
            void *kargs[] = {&a, &ti};
            const int block = b->tiling.block_size;
            e = hipLaunchKernel(bk->k.per_target, dim3((t.n_chains + block - 1) / block), dim3(block), kargs, 0, s);
            if (e != hipSuccess) return hip_fail(e, "per-target launch");
        }
        e = launch_batch_reduce(z, s);
        if (e != hipSuccess) return hip_fail(e, "reduce launch");
        return RESTORE_OK;
    }
    return fail(RESTORE_E_INVALID_ARG, "unknown batch mode");
}

restore_status restore_batch_estimates(restore_batch *b, restore_estimate_out *out, void *stream) {
    restore::TraceRange trace_range("restore_batch_estimates");
    if (!b || !out) return fail(RESTORE_E_INVALID_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<double> res((size_t)b->n * BS_SLOTS);
    std::vector<unsigned long long> cnt((size_t)b->n * BC_SLOTS);
    hipError_t e = hipMemcpyAsync(res.data(), at<double>(b, b->lay.results), res.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cnt.data(), at<unsigned long long>(b, b->lay.counters), cnt.size() * 8,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batch readback");
    for (int i = 0; i < b->n; ++i) {
        const double *r = res.data() + (size_t)i * BS_SLOTS;
        const unsigned long long *c = cnt.data() + (size_t)i * BC_SLOTS;
        const double N = r[BS_N], T = r[BS_T], A = r[BS_A];
        const double n_ok = (double)b->targets[i].n_chains - r[BS_NONFINITE];
        const double ct = b->c_tilde[i];
        auto se = [&](double ss, double den) -> double {
            if (n_ok < 2 || den <= 0) return NAN;
            return std::sqrt(ss / ((n_ok - 1) * n_ok)) / (den / n_ok);
        };
        restore_estimate_out &o = out[i];
        std::memset(&o, 0, sizeof(o));
        o.p_lambda = N > 0 ? ct * T / N : NAN;
        o.p_lambda_se = ct * se(r[BS_SS_T_N], N);
        o.lam_pf = N > 0 ? ct * A / N : NAN;
        o.lam_pf_se = ct * se(r[BS_SS_A_N], N);
        o.pi_f = T > 0 ? A / T : NAN;
        o.pi_f_se = se(r[BS_SS_A_T], T);
        o.tours_done = (int64_t)N;
        o.tours_censored = (int64_t)r[BS_CENS];
        o.transitions = (int64_t)c[BC_TRANSITIONS];
        o.accepts = (int64_t)c[BC_ACCEPTS];
        o.kills = (int64_t)c[BC_KILLS];
        o.nonfinite = (int64_t)r[BS_NONFINITE];
        const double tot = T + r[BS_CENS_T];
        o.censored_time_frac = tot > 0 ? r[BS_CENS_T] / tot : 0.0;
        o.accept_rate = c[BC_TRANSITIONS] ? (double)c[BC_ACCEPTS] / (double)c[BC_TRANSITIONS] : 0.0;
        o.kill_rate = c[BC_TRANSITIONS] ? (double)c[BC_KILLS] / (double)c[BC_TRANSITIONS] : 0.0;
        o.image_scale = N > 0 ? ct / N : 0.0;
    }
    return RESTORE_OK;
}

restore_status restore_batch_chain_sums(const restore_batch *b, int32_t target, restore_chain_sums *out) {
    if (!b || !out) return fail(RESTORE_E_INVALID_ARG, "null argument");
    if (target < 0 || target >= b->n) return fail(RESTORE_E_INVALID_ARG, "target index out of range");
    restore_batch *m = const_cast<restore_batch *>(b);
    const int64_t o = b->targets[target].chain_offset;
    out->n_done = at<uint32_t>(m, b->lay.n_done) + o;
    out->t_done = at<double>(m, b->lay.t_done) + o;
    out->a_done = at<double>(m, b->lay.a_done) + o;
    out->status = at<uint32_t>(m, b->lay.status) + o;
    out->t_cur = at<float>(m, b->lay.t_cur) + o;
    out->n_chains = b->targets[target].n_chains;
    return RESTORE_OK;
}

static uint64_t batch_key(const restore_batch *b) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h ^= v; h *= 1099511628211ull; };
    mix((uint64_t)b->n);
    mix((uint64_t)b->n_steps);
    for (const BatchTarget &t : b->targets) {
        mix((uint64_t)t.d);
        mix((uint64_t)t.K);
        mix((uint64_t)t.n_chains);
        mix((uint64_t)t.drain_cap);
        mix((uint64_t)t.mu_kind);
        mix((uint64_t)t.mu_comp);
    }
    return h;
}

restore_status restore_batch_autotune(restore_batch *b, const char *cache_path, restore_batch_tiling *chosen,
                                      double *best_ms, void *stream) {
    restore::TraceRange trace_range("restore_batch_autotune");
    if (!b) return fail(RESTORE_E_INVALID_ARG, "null batch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    char arch[64];
    std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
    for (char *p = arch; *p; ++p)
        if (*p == ':' || *p == '"') { *p = 0; break; }
    const unsigned long long key = (unsigned long long)batch_key(b);
    // cached choice?
    if (cache_path && *cache_path) {
        FILE *f = std::fopen(cache_path, "r");
        if (f) {
            char carch[64] = {0};
            unsigned long long ckey = 0;
            restore_batch_tiling t{};
            double ms = 0;
            const int got = std::fscanf(f, " { \"arch\" : \"%63[^\"]\" , \"key\" : %llu , \"block_size\" : %d , "
                                           "\"order\" : %d , \"buckets\" : %d , \"ms\" : %lf",
                                        carch, &ckey, &t.block_size, &t.order, &t.buckets, &ms);
            std::fclose(f);
            if (got == 6 && ckey == key && std::strcmp(carch, arch) == 0) {
                restore_status st = restore_batch_set_tiling(b, &t);
                if (st != RESTORE_OK) return st;
                if (chosen) *chosen = b->tiling;
                if (best_ms) *best_ms = ms;
                return RESTORE_OK;
            }
        }
    }
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(e, "event"); }
    restore_batch_tiling best{};
    double best_t = 1e30;
    restore_status st = RESTORE_OK;
    const int blocks[3] = {64, 128, 256};
    for (int bk = 0; bk < 2 && st == RESTORE_OK; ++bk)
        for (int order = 0; order < 2 && st == RESTORE_OK; ++order)
            for (int bs = 0; bs < 3 && st == RESTORE_OK; ++bs) {
                restore_batch_tiling t{blocks[bs], order, bk, 0};
                if ((st = restore_batch_set_tiling(b, &t)) != RESTORE_OK) break;
                if ((st = restore_batch_run(b, RESTORE_BATCH_MODE_GRAPH, stream)) != RESTORE_OK) break;  // capture + warm
                double tmin = 1e30;
                for (int rep = 0; rep < 2 && st == RESTORE_OK; ++rep) {
                    e = hipEventRecord(e0, s);
                    if (e == hipSuccess && (st = restore_batch_run(b, RESTORE_BATCH_MODE_GRAPH, stream)) != RESTORE_OK) break;
                    if (e == hipSuccess) e = hipEventRecord(e1, s);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e != hipSuccess) { st = hip_fail(e, "autotune timing"); break; }
                    tmin = std::min(tmin, (double)ms);
                }
                if (st == RESTORE_OK && tmin < best_t) { best_t = tmin; best = b->tiling; }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RESTORE_OK) return st;
    st = restore_batch_set_tiling(b, &best);
    if (st != RESTORE_OK) return st;
    if (cache_path && *cache_path) {
        FILE *f = std::fopen(cache_path, "w");
        if (f) {
            std::fprintf(f, "{\"arch\": \"%s\", \"key\": %llu, \"block_size\": %d, \"order\": %d, \"buckets\": %d, \"ms\": %.4f}\n",
                         arch, key, best.block_size, best.order, best.buckets, best_t);
            std::fclose(f);
        }
    }
    if (chosen) *chosen = best;
    if (best_ms) *best_ms = best_t;
    return RESTORE_OK;
}

restore_status restore_batch_destroy(restore_batch *b) {
    if (!b) return RESTORE_OK;
    drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return RESTORE_OK;
}

}  // extern "C"
