"""Thin ctypes binding of the C ABI in include/restore.h.

The functions here carry the C names and only marshal arguments: every step
of the chains runs in the gfx950 kernels of ``librestore.so``.  PyTorch
provides device memory (the caller-owned state buffer and image) and the
stream.  There is no CPU fallback: if the library is missing, importing
this module fails.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librestore.so")

OK, E_INVALID_ARG, E_UNSUPPORTED, E_HIP, E_NONFINITE, E_BAD_STATE, E_BUFFER_TOO_SMALL = 0, -1, -2, -3, -4, -5, -6
TARGET_GMM_ISO, TARGET_GMM_FULL, TARGET_PSS = 0, 1, 2
MU_UNIFORM_BOX, MU_GMM_DIAG = 0, 1
LOCAL_RWMH, LOCAL_MALA, LOCAL_HMC, LOCAL_RW_UNADJUSTED = 0, 1, 2, 3
INTEGRAND_ONE, INTEGRAND_P, INTEGRAND_PIXEL = 1, 2, 4
FLAG_PARAMS_LDS, FLAG_SPLAT_DIRECT, FLAG_SPLAT_TIGHT, FLAG_RB_DT, FLAG_INLINE_RNG, FLAG_IMAGE_FIXED = 1, 2, 4, 8, 16, 32
MLP_AUTO, MLP_FP32, MLP_BF16 = 0, 1, 2
ST_ALIVE, ST_CENSORED, ST_LAST_KILL, ST_LAST_ACCEPT, ST_GRAD_VALID, ST_LAST_LARGE = 1, 2, 4, 8, 16, 32


class RestoreError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"restore status {status}: {msg}")
        self.status = status


class restore_target(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("n_comp", C.c_int32), ("reserved", C.c_int32),
                ("params", C.POINTER(C.c_double)), ("params_count", C.c_int64)]


class restore_mu(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_comp", C.c_int32), ("beta", C.c_float), ("reserved", C.c_int32),
                ("params_dev", C.c_void_p)]


class restore_local_kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("step", C.c_float), ("large_step_prob", C.c_float),
                ("n_leapfrog", C.c_int32)]


class restore_config(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_chains", C.c_int64), ("target_id", C.c_int32),
                ("integrands", C.c_int32), ("c_tilde", C.c_double), ("drain_cap", C.c_int32),
                ("image_w", C.c_int32), ("image_h", C.c_int32), ("flags", C.c_int32),
                ("block_size", C.c_int32), ("image_batches", C.c_int32), ("tile_px", C.c_int32),
                ("first_chain", C.c_int32)]


class restore_estimate_out(C.Structure):
    _fields_ = [("p_lambda", C.c_double), ("p_lambda_se", C.c_double), ("lam_pf", C.c_double),
                ("lam_pf_se", C.c_double), ("pi_f", C.c_double), ("pi_f_se", C.c_double),
                ("tours_done", C.c_int64), ("tours_censored", C.c_int64), ("transitions", C.c_int64),
                ("accepts", C.c_int64), ("kills", C.c_int64), ("nonfinite", C.c_int64),
                ("censored_time_frac", C.c_double), ("accept_rate", C.c_double),
                ("kill_rate", C.c_double), ("image_scale", C.c_double), ("large_steps", C.c_int64),
                ("large_accepts", C.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class restore_state_view(C.Structure):
    _fields_ = [("x", C.c_void_p), ("logp", C.c_void_p), ("logu", C.c_void_p), ("grad", C.c_void_p),
                ("a_cur", C.c_void_p), ("t_cur", C.c_void_p), ("last_dt", C.c_void_p),
                ("a_done", C.c_void_p), ("t_done", C.c_void_p), ("n_done", C.c_void_p),
                ("status", C.c_void_p), ("n_chains", C.c_int64), ("dim", C.c_int32),
                ("steps_taken", C.c_int32)]


BATCH_ORDER_LPT, BATCH_ORDER_TARGET = 0, 1
BATCH_BUCKETS_ONE, BATCH_BUCKETS_DIM4 = 0, 1
BATCH_MODE_GRAPH, BATCH_MODE_PERSISTENT, BATCH_MODE_SEPARATE = 0, 1, 2


class restore_batch_tiling(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("order", C.c_int32), ("buckets", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self) -> dict:
        return {"block_size": self.block_size, "order": ["lpt", "target"][self.order],
                "buckets": ["one", "dim4"][self.buckets]}


class restore_mlp_shape(C.Structure):
    _fields_ = [("in_dim", C.c_int32), ("hidden", C.c_int32), ("n_comp", C.c_int32), ("dim", C.c_int32),
                ("precision", C.c_int32)]


class restore_chain_sums(C.Structure):
    _fields_ = [("n_done", C.c_void_p), ("t_done", C.c_void_p), ("a_done", C.c_void_p), ("status", C.c_void_p),
                ("t_cur", C.c_void_p), ("n_chains", C.c_int64)]


EXPORTS = ["restore_state_bytes", "restore_init", "restore_step", "restore_drain", "restore_estimate",
           "restore_get_state_view", "restore_refresh_cache", "restore_destroy",
           "restore_batch_state_bytes", "restore_batch_init", "restore_batch_set_tiling",
           "restore_batch_get_tiling", "restore_batch_run", "restore_batch_estimates", "restore_batch_chain_sums",
           "restore_batch_autotune", "restore_batch_destroy", "restore_step_record", "restore_mlp_param_count",
           "restore_mlp_forward", "restore_mlp_backward", "restore_gmm_nll_workspace_bytes", "restore_gmm_nll",
           "restore_gmm_nll_noalloc", "restore_adam_step", "restore_image_estimate", "restore_reset_sums", "restore_last_error"]


def _load(path: str = LIB_PATH) -> C.CDLL:
    """The C ABI library at `path` (the in-tree build by default) with its
    prototypes declared."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() "
                          "(there is no fallback implementation)")
    lib = C.CDLL(path)
    P = C.POINTER
    lib.restore_state_bytes.argtypes = [P(restore_target), P(restore_mu), P(restore_local_kernel),
                                        P(restore_config), P(C.c_size_t)]
    lib.restore_init.argtypes = [P(C.c_void_p), P(restore_target), P(restore_mu), P(restore_local_kernel),
                                 P(restore_config), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]
    lib.restore_step.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
    lib.restore_drain.argtypes = [C.c_void_p, C.c_void_p]
    lib.restore_reset_sums.argtypes = [C.c_void_p, C.c_void_p]
    lib.restore_estimate.argtypes = [C.c_void_p, P(restore_estimate_out), C.c_void_p]
    lib.restore_image_estimate.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.restore_get_state_view.argtypes = [C.c_void_p, P(restore_state_view)]
    lib.restore_refresh_cache.argtypes = [C.c_void_p, C.c_void_p]
    lib.restore_destroy.argtypes = [C.c_void_p]
    lib.restore_batch_state_bytes.argtypes = [C.c_int32, P(restore_target), P(restore_local_kernel),
                                              P(restore_config), P(restore_mu), P(C.c_size_t)]
    lib.restore_batch_init.argtypes = [P(C.c_void_p), C.c_int32, P(restore_target), P(restore_local_kernel),
                                       P(restore_config), P(restore_mu), C.c_int32, C.c_void_p, C.c_size_t,
                                       C.c_void_p]
    lib.restore_batch_set_tiling.argtypes = [C.c_void_p, P(restore_batch_tiling)]
    lib.restore_batch_get_tiling.argtypes = [C.c_void_p, P(restore_batch_tiling)]
    lib.restore_batch_run.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
    lib.restore_batch_estimates.argtypes = [C.c_void_p, P(restore_estimate_out), C.c_void_p]
    lib.restore_batch_chain_sums.argtypes = [C.c_void_p, C.c_int32, P(restore_chain_sums)]
    lib.restore_batch_autotune.argtypes = [C.c_void_p, C.c_char_p, P(restore_batch_tiling), P(C.c_double),
                                           C.c_void_p]
    lib.restore_batch_destroy.argtypes = [C.c_void_p]
    lib.restore_step_record.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.restore_mlp_param_count.argtypes = [P(restore_mlp_shape), P(C.c_int64), P(C.c_int64)]
    lib.restore_mlp_forward.argtypes = [P(restore_mlp_shape), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                        C.c_void_p, C.c_void_p]
    lib.restore_mlp_backward.argtypes = [P(restore_mlp_shape), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.restore_gmm_nll_workspace_bytes.argtypes = [P(C.c_size_t)]
    lib.restore_gmm_nll.argtypes = [C.c_int32, C.c_int32, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    lib.restore_gmm_nll_noalloc.argtypes = [C.c_int32, C.c_int32, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.restore_adam_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                      C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p]
    lib.restore_last_error.restype = C.c_char_p
    for name in EXPORTS[:-1]:
        getattr(lib, name).restype = C.c_int32
    return lib


_lib = _load()


def _check(status: int) -> None:
    if status != OK:
        raise RestoreError(status, _lib.restore_last_error().decode())


def _record_on(stream, *tensors) -> None:
    """Tell torch's caching allocator that kernels on `stream` (a torch
    stream other than the current one) use these buffers, so their memory
    is not reused before that stream's work is done."""
    if isinstance(stream, torch.cuda.Stream) and stream != torch.cuda.current_stream():
        for t in tensors:
            if t is not None:
                t.record_stream(stream)


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


# ---------------------------------------------------------------------------
# the C functions, one to one
# ---------------------------------------------------------------------------

def restore_state_bytes(target, mu, local, cfg) -> int:
    out = C.c_size_t(0)
    _check(_lib.restore_state_bytes(C.byref(target), C.byref(mu), C.byref(local), C.byref(cfg), C.byref(out)))
    return out.value


def restore_init(target, mu, local, cfg, state_ptr: int, state_bytes: int, image_ptr: int = 0,
                 stream=None) -> C.c_void_p:
    ctx = C.c_void_p()
    _check(_lib.restore_init(C.byref(ctx), C.byref(target), C.byref(mu), C.byref(local), C.byref(cfg),
                             C.c_void_p(state_ptr), state_bytes, C.c_void_p(image_ptr or None),
                             C.c_void_p(_stream(stream))))
    return ctx


def restore_step(ctx, n_steps: int, stream=None) -> None:
    _check(_lib.restore_step(ctx, int(n_steps), C.c_void_p(_stream(stream))))


def restore_drain(ctx, stream=None) -> None:
    _check(_lib.restore_drain(ctx, C.c_void_p(_stream(stream))))


def restore_reset_sums(ctx, stream=None) -> None:
    _check(_lib.restore_reset_sums(ctx, C.c_void_p(_stream(stream))))


def restore_estimate(ctx, stream=None) -> restore_estimate_out:
    out = restore_estimate_out()
    _check(_lib.restore_estimate(ctx, C.byref(out), C.c_void_p(_stream(stream))))
    return out


def restore_image_estimate(ctx, mean_ptr: int, se_ptr: int, stream=None) -> None:
    _check(_lib.restore_image_estimate(ctx, C.c_void_p(mean_ptr), C.c_void_p(se_ptr), C.c_void_p(_stream(stream))))


def restore_get_state_view(ctx) -> restore_state_view:
    v = restore_state_view()
    _check(_lib.restore_get_state_view(ctx, C.byref(v)))
    return v


def restore_refresh_cache(ctx, stream=None) -> None:
    _check(_lib.restore_refresh_cache(ctx, C.c_void_p(_stream(stream))))


def restore_destroy(ctx) -> None:
    _check(_lib.restore_destroy(ctx))


def restore_last_error() -> str:
    return _lib.restore_last_error().decode()


def _arr(cls, items):
    a = (cls * len(items))()
    for i, it in enumerate(items):
        a[i] = it
    return a


def restore_batch_state_bytes(targets, locals_, cfgs, mus=None) -> int:
    out = C.c_size_t(0)
    n = len(targets)
    _check(_lib.restore_batch_state_bytes(n, _arr(restore_target, targets), _arr(restore_local_kernel, locals_),
                                          _arr(restore_config, cfgs), _arr(restore_mu, mus) if mus else None,
                                          C.byref(out)))
    return out.value


def restore_batch_init(targets, locals_, cfgs, n_steps: int, state_ptr: int, state_bytes: int,
                       stream=None, mus=None) -> C.c_void_p:
    b = C.c_void_p()
    n = len(targets)
    _check(_lib.restore_batch_init(C.byref(b), n, _arr(restore_target, targets), _arr(restore_local_kernel, locals_),
                                   _arr(restore_config, cfgs), _arr(restore_mu, mus) if mus else None, int(n_steps),
                                   C.c_void_p(state_ptr), state_bytes, C.c_void_p(_stream(stream))))
    return b


def restore_batch_set_tiling(b, tiling: restore_batch_tiling) -> None:
    _check(_lib.restore_batch_set_tiling(b, C.byref(tiling)))


def restore_batch_get_tiling(b) -> restore_batch_tiling:
    t = restore_batch_tiling()
    _check(_lib.restore_batch_get_tiling(b, C.byref(t)))
    return t


def restore_batch_run(b, mode: int = BATCH_MODE_GRAPH, stream=None) -> None:
    _check(_lib.restore_batch_run(b, int(mode), C.c_void_p(_stream(stream))))


def restore_batch_estimates(b, n_targets: int, stream=None) -> list:
    out = (restore_estimate_out * n_targets)()
    _check(_lib.restore_batch_estimates(b, out, C.c_void_p(_stream(stream))))
    return [o.as_dict() for o in out]


def restore_batch_chain_sums(b, target: int) -> restore_chain_sums:
    v = restore_chain_sums()
    _check(_lib.restore_batch_chain_sums(b, int(target), C.byref(v)))
    return v


def restore_batch_autotune(b, cache_path=None, stream=None):
    t = restore_batch_tiling()
    ms = C.c_double(0.0)
    _check(_lib.restore_batch_autotune(b, cache_path.encode() if cache_path else None, C.byref(t), C.byref(ms),
                                       C.c_void_p(_stream(stream))))
    return t, ms.value


def restore_batch_destroy(b) -> None:
    _check(_lib.restore_batch_destroy(b))


def restore_step_record(ctx, n_steps: int, n_record: int, x_out_ptr: int, w_out_ptr: int, stream=None) -> None:
    _check(_lib.restore_step_record(ctx, int(n_steps), int(n_record), C.c_void_p(x_out_ptr), C.c_void_p(w_out_ptr),
                                    C.c_void_p(_stream(stream))))


def restore_mlp_param_count(shape: restore_mlp_shape):
    n, a = C.c_int64(0), C.c_int64(0)
    _check(_lib.restore_mlp_param_count(C.byref(shape), C.byref(n), C.byref(a)))
    return n.value, a.value


def restore_mlp_forward(shape, theta_ptr: int, ctx_ptr: int, G: int, act_ptr: int, out_ptr: int,
                        stream=None) -> None:
    _check(_lib.restore_mlp_forward(C.byref(shape), C.c_void_p(theta_ptr), C.c_void_p(ctx_ptr), int(G),
                                    C.c_void_p(act_ptr), C.c_void_p(out_ptr), C.c_void_p(_stream(stream))))


def restore_mlp_backward(shape, theta_ptr: int, ctx_ptr: int, G: int, act_ptr: int, dout_ptr: int, work_ptr: int,
                         grad_ptr: int, stream=None) -> None:
    _check(_lib.restore_mlp_backward(C.byref(shape), C.c_void_p(theta_ptr), C.c_void_p(ctx_ptr), int(G),
                                     C.c_void_p(act_ptr), C.c_void_p(dout_ptr), C.c_void_p(work_ptr),
                                     C.c_void_p(grad_ptr), C.c_void_p(_stream(stream))))


def restore_gmm_nll_workspace_bytes() -> int:
    n = C.c_size_t(0)
    _check(_lib.restore_gmm_nll_workspace_bytes(C.byref(n)))
    return n.value


def restore_gmm_nll(n_comp: int, dim: int, beta: float, gmm_ptr: int, x_ptr: int, w_ptr: int, n: int,
                    dout_ptr: int, loss_ptr: int, workspace_ptr: int, workspace_bytes: int, stream=None) -> None:
    _check(_lib.restore_gmm_nll(int(n_comp), int(dim), float(beta), C.c_void_p(gmm_ptr), C.c_void_p(x_ptr),
                                C.c_void_p(w_ptr), int(n), C.c_void_p(dout_ptr), C.c_void_p(loss_ptr),
                                C.c_void_p(workspace_ptr), int(workspace_bytes), C.c_void_p(_stream(stream))))


def restore_gmm_nll_noalloc(n_comp: int, dim: int, beta: float, gmm_ptr: int, x_ptr: int, w_ptr: int, n: int,
                            dout_ptr: int, loss_ptr: int, stream=None) -> None:
    _check(_lib.restore_gmm_nll_noalloc(int(n_comp), int(dim), float(beta), C.c_void_p(gmm_ptr), C.c_void_p(x_ptr),
                                        C.c_void_p(w_ptr), int(n), C.c_void_p(dout_ptr), C.c_void_p(loss_ptr),
                                        C.c_void_p(_stream(stream))))


def restore_adam_step(theta_ptr: int, grad_ptr: int, m_ptr: int, v_ptr: int, n: int, t: int, lr: float,
                      beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    _check(_lib.restore_adam_step(C.c_void_p(theta_ptr), C.c_void_p(grad_ptr), C.c_void_p(m_ptr), C.c_void_p(v_ptr),
                                  int(n), int(t), float(lr), float(beta1), float(beta2), float(eps),
                                  C.c_void_p(_stream(stream))))


# ---------------------------------------------------------------------------
# descriptors from canonical parameters
# ---------------------------------------------------------------------------

def target_params(kind: str, d: int, K: int, params: dict) -> np.ndarray:
    """Flatten canonical float64 parameters into the layout restore_target
    documents for each target kind."""
    if kind == "gmm_iso":
        parts = [params["weights"], params["means"], params["sigmas"]]
    elif kind == "gmm_full":
        parts = [params["weights"], params["means"], params["covs"]]
    elif kind == "pss":
        parts = [params[k] for k in ("tex_a_freq", "tex_a_amp", "tex_a_phase", "tex_b_freq", "tex_b_amp",
                                     "tex_b_phase", "lobe_dirs", "lobe_kappa", "lobe_weights", "base")]
    else:
        raise ValueError(kind)
    return np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts]))


_KIND = {"gmm_iso": TARGET_GMM_ISO, "gmm_full": TARGET_GMM_FULL, "pss": TARGET_PSS}


@dataclass
class Problem:
    """Descriptors of one run, built from canonical parameters.  Holds the
    host parameter array for as long as the descriptors point at it."""
    target: restore_target
    mu: restore_mu
    local: restore_local_kernel
    cfg: restore_config
    _params: np.ndarray
    _mu_params: Optional[torch.Tensor] = None


def make_problem(kind: str, d: int, K: int, params: dict, *, local: str, step: float, n_chains: int,
                 c_tilde: float, seed: int, drain_cap: int, target_id: int = 0, integrand_p: bool = True,
                 image: Optional[tuple] = None, lds: bool = False, block_size: int = 0,
                 mu: Optional[dict] = None, flags: int = 0, image_batches: int = 0,
                 large_step_prob: float = 0.0, n_leapfrog: int = 0, tile_px: int = 0,
                 first_chain: int = 0) -> Problem:
    flat = target_params(kind, d, K, params)
    t = restore_target(_KIND[kind], d, K if kind != "pss" else 0, 0,
                       flat.ctypes.data_as(C.POINTER(C.c_double)), flat.size)
    mu_t = None
    if mu is None:
        m = restore_mu(MU_UNIFORM_BOX, 0, 0.0, 0, None)
    elif "params_dev" in mu:
        # a device row [logits K | means K*d | log_std K*d] (a learned mu)
        mu_t = mu["params_dev"].reshape(-1)
        if mu_t.dtype != torch.float32 or not mu_t.is_cuda or not mu_t.is_contiguous():
            raise ValueError("params_dev must be a contiguous float32 device tensor")
        m = restore_mu(MU_GMM_DIAG, int(mu["n_comp"]), float(mu["beta"]), 0, mu_t.data_ptr())
    else:
        mu_t = torch.cat([torch.as_tensor(np.asarray(mu[k], dtype=np.float32).ravel())
                          for k in ("logits", "means", "log_std")]).cuda()
        m = restore_mu(MU_GMM_DIAG, int(np.asarray(mu["logits"]).size), float(mu["beta"]), 0, mu_t.data_ptr())
    kind = {"rwmh": LOCAL_RWMH, "mala": LOCAL_MALA, "hmc": LOCAL_HMC, "rw_unadjusted": LOCAL_RW_UNADJUSTED}[local]
    lk = restore_local_kernel(kind, float(step), float(large_step_prob), int(n_leapfrog))
    integrands = INTEGRAND_ONE | (INTEGRAND_P if integrand_p else 0) | (INTEGRAND_PIXEL if image else 0)
    w, h = (image or (0, 0))
    cfg = restore_config(int(seed), int(n_chains), int(target_id), integrands, float(c_tilde), int(drain_cap),
                         int(w), int(h), (FLAG_PARAMS_LDS if lds else 0) | int(flags), int(block_size),
                         int(image_batches), int(tile_px), int(first_chain))
    return Problem(t, m, lk, cfg, flat, mu_t)


def problem_from_workload(wl, **overrides) -> Problem:
    """Descriptors for an object with the attributes of a synthetic workload
    (target, d, K, params, local, step, n_chains, c_tilde, seed, drain_cap,
    image)."""
    kw = dict(local=wl.local, step=wl.step, n_chains=wl.n_chains, c_tilde=wl.c_tilde, seed=wl.seed,
              drain_cap=wl.drain_cap, image=getattr(wl, "image", None),
              image_batches=getattr(wl, "image_batches", 0) if getattr(wl, "image", None) else 0,
              n_leapfrog=getattr(wl, "n_leapfrog", 0), tile_px=getattr(wl, "tile_px", 0))
    kw.update(overrides)
    if not kw["image"]:
        # no pixel integrand: no image batches or tiles either
        kw["image_batches"], kw["tile_px"] = 0, 0
    return make_problem(wl.target, wl.d, wl.K, wl.params, **kw)


class Run:
    """A chain population on the current GPU: owns the torch state buffer
    (and image) and the library context."""

    def __init__(self, prob: Problem, stream=None):
        self.prob = prob
        self.stream = stream
        nbytes = restore_state_bytes(prob.target, prob.mu, prob.local, prob.cfg)
        self.state = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.state.data_ptr()
        self._state_ptr = (base + 255) // 256 * 256
        self.nbytes = nbytes
        self.image = None
        if prob.cfg.integrands & INTEGRAND_PIXEL:
            nb = max(1, prob.cfg.image_batches)
            shape = (nb, prob.cfg.image_h, prob.cfg.image_w) if nb > 1 else (prob.cfg.image_h, prob.cfg.image_w)
            self.image = torch.zeros(shape, dtype=torch.float32, device="cuda")
        _record_on(stream, self.state, self.image)
        self.ctx = restore_init(prob.target, prob.mu, prob.local, prob.cfg, self._state_ptr, nbytes,
                                self.image.data_ptr() if self.image is not None else 0, stream)
        self.n_chains = prob.cfg.n_chains
        self.d = prob.target.dim

    def step(self, n: int):
        restore_step(self.ctx, n, self.stream)

    def step_record(self, n: int, n_record: int):
        """Advance n steps; return the recorded (x_{i-1}, dt_i) of chains
        [0, n_record) as tensors x [n][n_record][d], w [n][n_record]."""
        x = torch.empty((n, n_record, self.d), dtype=torch.float32, device="cuda")
        w = torch.empty((n, n_record), dtype=torch.float32, device="cuda")
        restore_step_record(self.ctx, n, n_record, x.data_ptr(), w.data_ptr(), self.stream)
        return x, w

    def drain(self):
        restore_drain(self.ctx, self.stream)

    def reset_sums(self):
        """End of the MH chain's burn-in (c_tilde = 0): zero the sums."""
        restore_reset_sums(self.ctx, self.stream)

    def estimate(self) -> dict:
        return restore_estimate(self.ctx, self.stream).as_dict()

    def refresh_cache(self):
        restore_refresh_cache(self.ctx, self.stream)

    def image_estimate(self):
        """(per-pixel estimate, batch-means standard error) as [h][w] tensors."""
        h, w = self.prob.cfg.image_h, self.prob.cfg.image_w
        mean = torch.empty((h, w), dtype=torch.float32, device="cuda")
        se = torch.empty((h, w), dtype=torch.float32, device="cuda")
        restore_image_estimate(self.ctx, mean.data_ptr(), se.data_ptr(), self.stream)
        return mean, se

    # --- views of the state arrays (no copies) -----------------------------
    def _view(self, ptr: int, shape, dtype) -> torch.Tensor:
        base = self.state.data_ptr()
        off = ptr - base
        nbytes = int(np.prod(shape)) * torch.empty((), dtype=dtype).element_size()
        return self.state[off:off + nbytes].view(dtype).view(*shape)

    def arrays(self) -> dict:
        v = restore_get_state_view(self.ctx)
        C_, d = self.n_chains, self.d
        out = {
            "x": self._view(v.x, (d, C_), torch.float32),
            "logp": self._view(v.logp, (C_,), torch.float32),
            "logu": self._view(v.logu, (C_,), torch.float32),
            "a_cur": self._view(v.a_cur, (C_,), torch.float32),
            "t_cur": self._view(v.t_cur, (C_,), torch.float32),
            "last_dt": self._view(v.last_dt, (C_,), torch.float32),
            "a_done": self._view(v.a_done, (C_,), torch.float64),
            "t_done": self._view(v.t_done, (C_,), torch.float64),
            "n_done": self._view(v.n_done, (C_,), torch.int32),
            "status": self._view(v.status, (C_,), torch.int32),
        }
        if v.grad:
            out["grad"] = self._view(v.grad, (d, C_), torch.float32)
        return out

    def state_region(self) -> torch.Tensor:
        """The aligned bytes the library owns inside ``state`` (for
        checkpoints: copy them out, and back into a context that has taken the
        same number of steps)."""
        off = self._state_ptr - self.state.data_ptr()
        return self.state[off:off + self.nbytes]

    @property
    def steps_taken(self) -> int:
        return restore_get_state_view(self.ctx).steps_taken

    def close(self):
        if self.ctx:
            restore_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many targets advanced together on the current GPU: owns the torch
    state buffer and the library's batch handle."""

    def __init__(self, workloads, n_steps: int, stream=None, mus=None, first_chains=None):
        """mus: None (uniform mu everywhere) or one entry per workload, None
        or a regeneration distribution as make_problem takes it.
        first_chains: None (0 everywhere) or the global id of each target's
        chain 0."""
        self.stream = stream
        mus = list(mus) if mus is not None else [None] * len(workloads)
        firsts = list(first_chains) if first_chains is not None else [0] * len(workloads)
        self.probs = [problem_from_workload(w, target_id=i, integrand_p=True, mu=m, first_chain=f)
                      for i, (w, m, f) in enumerate(zip(workloads, mus, firsts))]
        targets = [p.target for p in self.probs]
        locs = [p.local for p in self.probs]
        cfgs = [p.cfg for p in self.probs]
        mu_desc = [p.mu for p in self.probs] if any(m is not None for m in mus) else None
        self.n = len(self.probs)
        nbytes = restore_batch_state_bytes(targets, locs, cfgs, mu_desc)
        self.state = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = (self.state.data_ptr() + 255) // 256 * 256
        _record_on(stream, self.state)
        self.handle = restore_batch_init(targets, locs, cfgs, n_steps, ptr, nbytes, stream, mu_desc)

    def run(self, mode: int = BATCH_MODE_GRAPH):
        restore_batch_run(self.handle, mode, self.stream)

    def estimates(self) -> list:
        return restore_batch_estimates(self.handle, self.n, self.stream)

    def set_tiling(self, block_size=256, order=BATCH_ORDER_LPT, buckets=BATCH_BUCKETS_ONE):
        restore_batch_set_tiling(self.handle, restore_batch_tiling(block_size, order, buckets, 0))

    def tiling(self) -> restore_batch_tiling:
        return restore_batch_get_tiling(self.handle)

    def autotune(self, cache_path=None):
        return restore_batch_autotune(self.handle, cache_path, self.stream)

    def chain_sums(self, target: int) -> dict:
        v = restore_batch_chain_sums(self.handle, target)
        n = int(v.n_chains)
        base = self.state.data_ptr()

        def view(ptr, dtype):
            size = torch.empty((), dtype=dtype).element_size()
            off = ptr - base
            return self.state[off:off + n * size].view(dtype)
        return {"n_done": view(v.n_done, torch.int32), "t_done": view(v.t_done, torch.float64),
                "a_done": view(v.a_done, torch.float64), "status": view(v.status, torch.int32),
                "t_cur": view(v.t_cur, torch.float32)}

    def close(self):
        if self.handle:
            restore_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
