"""Python front of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module.  It loads ``oracle/liboracle.so`` (plain C,
double precision, built by ``oracle/build.py`` with gcc), marshals a
:class:`workloads.Workload` into the oracle's structs and exposes

* :func:`init_states`     -- x_0 ~ mu for a set of chains (Alg. 2 input);
* :func:`transitions`     -- single Jump Restore transitions (Alg. 2 body);
* :func:`run`             -- whole runs: B steps, drain, per-chain tour sums;
* :func:`estimate`        -- the tour-ratio estimates of Sec. 6.3 / 7.4 with
                             delta-method standard errors over chains;
* :func:`asymptotic_variance` -- the time-average variance constant of pi f
                             (the quantity Theorem B of the supplement orders).

With ``c_tilde = 0`` and a large-step probability ``l > 0`` the same runs are
the paper's reference chain M^l (Sec. 5, eq. (mixture-proposal-kernel);
Sec. 8): a Metropolis-Hastings chain with the mixture proposal, whose
ergodic average after a burn-in estimates pi f.

It shares nothing with the HIP path except the seeded inputs drawn by
``workloads``.  The Gaussian-mixture precision matrices and log-determinants
are taken from numpy's ``inv`` / ``slogdet`` (library primitives); the HIP
side computes its own Cholesky factors.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

TARGET_GMM, TARGET_PSS = 0, 1
MU_UNIFORM, MU_GMM_DIAG = 0, 1
LOCAL_RWMH, LOCAL_MALA, LOCAL_HMC, LOCAL_RW_UNADJUSTED = 0, 1, 2, 3
FLAG_KILL, FLAG_ACCEPT, FLAG_OUTSIDE, FLAG_LARGE, FLAG_NEGATIVE_RATE = 1, 2, 4, 8, 16

_dp = C.POINTER(C.c_double)


class OrTarget(C.Structure):
    _fields_ = [("kind", C.c_int32), ("d", C.c_int32), ("K", C.c_int32), ("pad", C.c_int32),
                ("log_w", _dp), ("mean", _dp), ("prec", _dp), ("logdet", _dp),
                ("ta_freq", _dp), ("ta_amp", _dp), ("ta_phase", _dp),
                ("tb_freq", _dp), ("tb_amp", _dp), ("tb_phase", _dp),
                ("lobe_dir", _dp), ("lobe_kappa", _dp), ("lobe_w", _dp),
                ("base", C.c_double)]


class OrMu(C.Structure):
    _fields_ = [("kind", C.c_int32), ("d", C.c_int32), ("K", C.c_int32), ("pad", C.c_int32),
                ("beta", C.c_double), ("logit", _dp), ("mean", _dp), ("log_std", _dp)]


class OrLocal(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_leapfrog", C.c_int32), ("step", C.c_double),
                ("large_step_prob", C.c_double)]


class OrConfig(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("target_id", C.c_uint32), ("pad", C.c_uint32),
                ("c_tilde", C.c_double), ("integrand_p", C.c_int32),
                ("image_w", C.c_int32), ("image_h", C.c_int32), ("rb_dt", C.c_int32),
                ("burn_in", C.c_int32), ("tile_px", C.c_int32), ("n_chains_total", C.c_int64)]


class OrOutputs(C.Structure):
    _fields_ = [("n_done", C.POINTER(C.c_int64)), ("t_done", _dp), ("a_done", _dp),
                ("censored", C.POINTER(C.c_int32)), ("t_censored", _dp),
                ("transitions", C.POINTER(C.c_int64)), ("accepts", C.POINTER(C.c_int64)),
                ("kills", C.POINTER(C.c_int64)), ("image", _dp),
                ("large_steps", C.POINTER(C.c_int64)), ("large_accepts", C.POINTER(C.c_int64)),
                ("min_margin", _dp), ("image_count", _dp), ("image_near", _dp)]


_lib = None


def load():
    """Load the oracle library, building it first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = C.CDLL(_LIB_PATH)
    lib.oracle_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
    lib.oracle_u01.argtypes = [C.c_uint32]
    lib.oracle_u01.restype = C.c_double
    lib.oracle_log_target.argtypes = [C.POINTER(OrTarget), _dp, _dp]
    lib.oracle_log_target.restype = C.c_double
    lib.oracle_log_mu.argtypes = [C.POINTER(OrMu), _dp]
    lib.oracle_log_mu.restype = C.c_double
    lib.oracle_transitions.argtypes = [C.POINTER(OrTarget), C.POINTER(OrMu), C.POINTER(OrLocal),
                                       C.POINTER(OrConfig), C.c_int64, C.POINTER(C.c_uint32),
                                       C.POINTER(C.c_uint32), _dp, _dp, _dp, _dp, C.c_int,
                                       _dp, C.POINTER(C.c_int32), _dp]
    lib.oracle_init_states.argtypes = [C.POINTER(OrTarget), C.POINTER(OrMu), C.POINTER(OrLocal),
                                       C.POINTER(OrConfig), C.c_int64, C.POINTER(C.c_uint32), _dp, _dp, _dp, _dp]
    lib.oracle_log_inflow.argtypes = [C.POINTER(OrTarget), C.c_double, _dp]
    lib.oracle_log_inflow.restype = C.c_double
    lib.oracle_log_u_eff.argtypes = [C.POINTER(OrTarget), C.POINTER(OrMu), C.c_double, C.c_double, _dp, C.c_double]
    lib.oracle_log_u_eff.restype = C.c_double
    lib.oracle_run.argtypes = [C.POINTER(OrTarget), C.POINTER(OrMu), C.POINTER(OrLocal),
                               C.POINTER(OrConfig), C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                               C.c_int32, C.POINTER(OrOutputs)]
    lib.oracle_run.restype = C.c_int
    lib.oracle_leapfrog.argtypes = [C.POINTER(OrTarget), C.c_int, C.c_double, _dp, _dp, _dp, _dp]
    lib.oracle_leapfrog.restype = C.c_int
    _lib = lib
    return lib


class use_library:
    """Context manager that points this module at another build of the
    oracle (the mutation tests load deliberately broken copies)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib, _LIB_PATH
        self._saved = (_lib, _LIB_PATH)
        _lib, _LIB_PATH = None, self.path
        return load()

    def __exit__(self, *exc):
        global _lib, _LIB_PATH
        _lib, _LIB_PATH = self._saved
        return False


def _ptr(a: Optional[np.ndarray], ctype=C.c_double):
    if a is None:
        return C.POINTER(ctype)()
    return a.ctypes.data_as(C.POINTER(ctype))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Problem:
    """A workload marshalled for the oracle.  Keeps the numpy arrays alive
    for as long as the ctypes structs point at them."""

    def __init__(self, wl, mu: Optional[dict] = None, target_id: int = 0,
                 c_tilde: Optional[float] = None, seed: Optional[int] = None,
                 integrand_p: bool = True, image: Optional[tuple] = None,
                 step: Optional[float] = None, local: Optional[str] = None, rb_dt: bool = False,
                 large_step_prob: float = 0.0, burn_in: int = 0, n_leapfrog: Optional[int] = None,
                 tile_px: Optional[int] = None, n_chains_total: Optional[int] = None):
        self.wl = wl
        self.d = wl.d
        self._keep = []
        t = OrTarget()
        t.d, t.K = wl.d, wl.K
        p = wl.params
        if wl.target in ("gmm_iso", "gmm_full"):
            t.kind = TARGET_GMM
            w = _f64(p["weights"])
            means = _f64(p["means"]).reshape(wl.K, wl.d)
            if wl.target == "gmm_iso":
                covs = np.stack([np.eye(wl.d) * s * s for s in _f64(p["sigmas"])])
            else:
                covs = _f64(p["covs"]).reshape(wl.K, wl.d, wl.d)
            prec = _f64(np.linalg.inv(covs))
            logdet = _f64(np.linalg.slogdet(covs)[1])
            log_w = _f64(np.log(w))
            self._keep += [log_w, means, prec, logdet]
            t.log_w, t.mean, t.prec, t.logdet = _ptr(log_w), _ptr(means), _ptr(prec), _ptr(logdet)
        elif wl.target == "pss":
            t.kind = TARGET_PSS
            arrs = {k: _f64(p[k]) for k in ("tex_a_freq", "tex_a_amp", "tex_a_phase",
                                            "tex_b_freq", "tex_b_amp", "tex_b_phase",
                                            "lobe_dirs", "lobe_kappa", "lobe_weights")}
            self._keep += list(arrs.values())
            t.ta_freq, t.ta_amp, t.ta_phase = (_ptr(arrs["tex_a_freq"]), _ptr(arrs["tex_a_amp"]),
                                               _ptr(arrs["tex_a_phase"]))
            t.tb_freq, t.tb_amp, t.tb_phase = (_ptr(arrs["tex_b_freq"]), _ptr(arrs["tex_b_amp"]),
                                               _ptr(arrs["tex_b_phase"]))
            t.lobe_dir, t.lobe_kappa, t.lobe_w = (_ptr(arrs["lobe_dirs"]), _ptr(arrs["lobe_kappa"]),
                                                  _ptr(arrs["lobe_weights"]))
            t.base = float(p["base"][0])
        else:
            raise ValueError(wl.target)
        self.target = t

        m = OrMu()
        m.d = wl.d
        if mu is None:
            m.kind = MU_UNIFORM
        else:
            m.kind = MU_GMM_DIAG
            logit = _f64(mu["logits"])
            mmean = _f64(mu["means"]).reshape(-1, wl.d)
            lstd = _f64(mu["log_std"]).reshape(-1, wl.d)
            self._keep += [logit, mmean, lstd]
            m.K = logit.shape[0]
            m.beta = float(mu["beta"])
            m.logit, m.mean, m.log_std = _ptr(logit), _ptr(mmean), _ptr(lstd)
        self.mu = m

        lk = OrLocal()
        local = local or wl.local
        lk.kind = {"rwmh": LOCAL_RWMH, "mala": LOCAL_MALA, "hmc": LOCAL_HMC,
                   "rw_unadjusted": LOCAL_RW_UNADJUSTED}[local]
        lk.n_leapfrog = int(getattr(wl, "n_leapfrog", 0) if n_leapfrog is None else n_leapfrog)
        lk.step = float(wl.step if step is None else step)
        # l is a float32 at the library boundary; the oracle compares the
        # (float32-exact) uniform with the same value
        lk.large_step_prob = float(np.float32(large_step_prob))
        self.local = lk

        cfg = OrConfig()
        cfg.seed = int(wl.seed if seed is None else seed)
        cfg.target_id = int(target_id)
        cfg.c_tilde = float(wl.c_tilde if c_tilde is None else c_tilde)
        cfg.integrand_p = 1 if integrand_p else 0
        cfg.rb_dt = 1 if rb_dt else 0
        cfg.burn_in = int(burn_in)
        tile_px = int(getattr(wl, "tile_px", 0) if tile_px is None else tile_px)
        cfg.tile_px = tile_px
        cfg.n_chains_total = int(wl.n_chains if n_chains_total is None else n_chains_total)
        if tile_px and (mu is not None or not (image if image is not None else wl.image)):
            raise ValueError("tile-stratified runs need the image integrand and the uniform mu")
        if lk.kind == LOCAL_RW_UNADJUSTED:
            # the closed form of Q^T p needs diagonal covariances; the killing
            # rate of the non-invariant process needs c_tilde > 0 and M^0
            if wl.target != "gmm_iso" or not cfg.c_tilde > 0 or lk.large_step_prob != 0.0:
                raise ValueError("the unadjusted jump process needs the isotropic mixture, c_tilde > 0 and l = 0")
        img = image if image is not None else wl.image
        if img:
            cfg.image_w, cfg.image_h = int(img[0]), int(img[1])
        self.cfg = cfg

    @property
    def c_tilde(self) -> float:
        return self.cfg.c_tilde


# ---------------------------------------------------------------------------
# primitives exposed for pins
# ---------------------------------------------------------------------------

def philox(counter, key) -> np.ndarray:
    lib = load()
    c = (C.c_uint32 * 4)(*[int(v) & 0xffffffff for v in counter])
    k = (C.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    out = (C.c_uint32 * 4)()
    lib.oracle_philox4x32_10(c, k, out)
    return np.array(list(out), dtype=np.uint32)


def u01(r: int) -> float:
    return load().oracle_u01(int(r) & 0xffffffff)


def log_target(prob: Problem, x: np.ndarray, grad: bool = False):
    """log p at each row of x (and grad log p if requested)."""
    lib = load()
    x = _f64(x).reshape(-1, prob.d)
    lp = np.empty(x.shape[0])
    g = np.zeros_like(x)
    for i in range(x.shape[0]):
        xi = np.ascontiguousarray(x[i])
        gi = np.zeros(prob.d)
        lp[i] = lib.oracle_log_target(C.byref(prob.target), _ptr(xi), _ptr(gi) if grad else _dp())
        g[i] = gi
    return (lp, g) if grad else lp


def leapfrog(prob: Problem, q, rho, n: int, e: float):
    """n leapfrog steps of size e from (q, rho): returns (q, rho, log p(q),
    grad log p(q), inside) at the end point."""
    lib = load()
    q = _f64(q).copy()
    rho = _f64(rho).copy()
    lp0, g = log_target(prob, q, grad=True)
    g = np.ascontiguousarray(g[0])
    lp = C.c_double(float(lp0[0]))
    inside = lib.oracle_leapfrog(C.byref(prob.target), int(n), float(e), _ptr(q), _ptr(rho), C.byref(lp), _ptr(g))
    return q, rho, lp.value, g, bool(inside)


def log_inflow(prob: Problem, x: np.ndarray, sigma: Optional[float] = None) -> np.ndarray:
    """log (Q^T p)(x) = log int_box p(y) N(x; y, sigma^2 I) dy at each row
    of x (sigma defaults to the problem's step)."""
    lib = load()
    x = _f64(x).reshape(-1, prob.d)
    s = float(prob.local.step if sigma is None else sigma)
    return np.array([lib.oracle_log_inflow(C.byref(prob.target), s, _ptr(np.ascontiguousarray(r))) for r in x])


def log_u_eff(prob: Problem, x: np.ndarray) -> np.ndarray:
    """log u_eff(x), u_eff = u + (Q^T p - p) / c_tilde, the density the
    killing rate k = c_tilde u_eff / p of the unadjusted jump process uses
    (NaN where u_eff < 0)."""
    lib = load()
    x = _f64(x).reshape(-1, prob.d)
    lp = log_target(prob, x)
    return np.array([lib.oracle_log_u_eff(C.byref(prob.target), C.byref(prob.mu), float(prob.local.step),
                                          float(prob.c_tilde), _ptr(np.ascontiguousarray(r)), float(v))
                     for r, v in zip(x, lp)])


def log_mu(prob: Problem, y: np.ndarray) -> np.ndarray:
    lib = load()
    y = _f64(y).reshape(-1, prob.d)
    return np.array([lib.oracle_log_mu(C.byref(prob.mu), _ptr(np.ascontiguousarray(r))) for r in y])


# ---------------------------------------------------------------------------
# transitions
# ---------------------------------------------------------------------------

@dataclass
class States:
    x: np.ndarray      # [n, d]
    lp: np.ndarray     # [n]
    lu: np.ndarray     # [n]
    g: np.ndarray      # [n, d]

    def copy(self) -> "States":
        return States(self.x.copy(), self.lp.copy(), self.lu.copy(), self.g.copy())


def init_states(prob: Problem, chains) -> States:
    lib = load()
    chains = np.ascontiguousarray(np.asarray(chains, dtype=np.uint32))
    n, d = chains.shape[0], prob.d
    st = States(np.zeros((n, d)), np.zeros(n), np.zeros(n), np.zeros((n, d)))
    lib.oracle_init_states(C.byref(prob.target), C.byref(prob.mu), C.byref(prob.local), C.byref(prob.cfg), n,
                           _ptr(chains, C.c_uint32), _ptr(st.x), _ptr(st.lp), _ptr(st.lu), _ptr(st.g))
    return st


def transitions(prob: Problem, states: States, steps, chains, recompute: bool = True):
    """One Alg. 2 transition for each (state, step, chain).  With
    ``recompute`` the oracle recomputes log p, log u and grad log p of the
    input states in FP64 (the usual case: the input x is shared, the cached
    values are each side's own).  Returns (new States, dt, flags, margins);
    margins[:, 0] is ln t2 - ln t1, margins[:, 1] ln u_acc - ln(ratio) (NaN
    without an acceptance test), margins[:, 2] the distance of the category
    uniform to the nearest mu category boundary, margins[:, 3:5] log p and
    log u at the local proposal (NaN without one), margins[:, 5:7] log p and
    log u of the input state, margins[:, 7] the distance of a small-step
    proposal to the edge of the support (inf without one)."""
    lib = load()
    st = states.copy()
    st.x = _f64(st.x); st.lp = _f64(st.lp); st.lu = _f64(st.lu); st.g = _f64(st.g)
    n = st.x.shape[0]
    steps = np.ascontiguousarray(np.broadcast_to(np.asarray(steps, dtype=np.uint32), (n,)))
    chains = np.ascontiguousarray(np.asarray(chains, dtype=np.uint32))
    dt = np.zeros(n)
    flags = np.zeros(n, dtype=np.int32)
    margins = np.zeros((n, 8))
    lib.oracle_transitions(C.byref(prob.target), C.byref(prob.mu), C.byref(prob.local),
                           C.byref(prob.cfg), n, _ptr(steps, C.c_uint32), _ptr(chains, C.c_uint32),
                           _ptr(st.x), _ptr(st.lp), _ptr(st.lu), _ptr(st.g), 1 if recompute else 0,
                           _ptr(dt), _ptr(flags, C.c_int32), _ptr(margins))
    return st, dt, flags, margins


# ---------------------------------------------------------------------------
# runs and estimates
# ---------------------------------------------------------------------------

@dataclass
class RunResult:
    n_done: np.ndarray
    t_done: np.ndarray
    a_done: np.ndarray
    censored: np.ndarray
    t_censored: np.ndarray
    transitions: np.ndarray
    accepts: np.ndarray
    kills: np.ndarray
    image: Optional[np.ndarray]
    c_tilde: float
    large_steps: Optional[np.ndarray] = None
    large_accepts: Optional[np.ndarray] = None
    # parity bookkeeping: per chain the smallest scaled kill and accept
    # margins, the smallest category margin and the smallest distance of a
    # proposal to the support's edge per local move since the last
    # regeneration, over all its steps [n, 4]; splats per pixel and the dt of splats near a pixel edge
    min_margin: Optional[np.ndarray] = None
    image_count: Optional[np.ndarray] = None
    image_near: Optional[np.ndarray] = None


def run(prob: Problem, c0: int, c1: int, n_steps: Optional[int] = None,
        drain_cap: Optional[int] = None, threads: Optional[int] = None) -> RunResult:
    """Chains [c0, c1): x_0 ~ mu, ``n_steps`` steps with regeneration, then
    the tours in flight are finished for at most ``drain_cap`` steps.  With
    c_tilde = 0 (the MH chain) there are no tours: steps from the problem's
    ``burn_in`` on add to the chain sums, and nothing is drained."""
    lib = load()
    n = c1 - c0
    n_steps = prob.wl.n_steps if n_steps is None else n_steps
    drain_cap = prob.wl.drain_cap if drain_cap is None else drain_cap
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    r = RunResult(np.zeros(n, np.int64), np.zeros(n), np.zeros(n), np.zeros(n, np.int32),
                  np.zeros(n), np.zeros(n, np.int64), np.zeros(n, np.int64), np.zeros(n, np.int64),
                  None, prob.c_tilde, np.zeros(n, np.int64), np.zeros(n, np.int64))
    out = OrOutputs()
    out.n_done, out.t_done, out.a_done = _ptr(r.n_done, C.c_int64), _ptr(r.t_done), _ptr(r.a_done)
    out.censored, out.t_censored = _ptr(r.censored, C.c_int32), _ptr(r.t_censored)
    out.transitions, out.accepts = _ptr(r.transitions, C.c_int64), _ptr(r.accepts, C.c_int64)
    out.kills = _ptr(r.kills, C.c_int64)
    out.large_steps, out.large_accepts = _ptr(r.large_steps, C.c_int64), _ptr(r.large_accepts, C.c_int64)
    r.min_margin = np.full((n, 4), np.inf)
    out.min_margin = _ptr(r.min_margin)
    if prob.cfg.image_w > 0:
        r.image = np.zeros((prob.cfg.image_h, prob.cfg.image_w))
        r.image_count = np.zeros_like(r.image)
        r.image_near = np.zeros_like(r.image)
        out.image, out.image_count, out.image_near = _ptr(r.image), _ptr(r.image_count), _ptr(r.image_near)
    else:
        out.image = out.image_count = out.image_near = _dp()
    rc = lib.oracle_run(C.byref(prob.target), C.byref(prob.mu), C.byref(prob.local),
                        C.byref(prob.cfg), int(c0), int(c1), int(n_steps), int(drain_cap),
                        int(threads), C.byref(out))
    if rc != 0:
        raise RuntimeError("oracle_run failed")
    return r


def _ratio(num: np.ndarray, den: np.ndarray):
    """Pooled ratio R = sum num / sum den over chains and its delta-method
    standard error sqrt(sum (num_c - R den_c)^2 / ((C - 1) C mean(den)^2))."""
    num = np.asarray(num, dtype=np.float64)
    den = np.asarray(den, dtype=np.float64)
    C_ = num.shape[0]
    R = num.sum() / den.sum()
    if C_ < 2:
        return R, float("nan")
    resid = num - R * den
    se = np.sqrt((resid * resid).sum() / ((C_ - 1) * C_)) / den.mean()
    return float(R), float(se)


def estimate(r: RunResult) -> dict:
    """Sec. 6.3: p_lambda ~ (c_tilde / j) sum tau_i; lambda(p f) ~ (c_tilde / j)
    int f dt; Sec. 7.4 eq. (approx): pi f ~ sum dt f / sum dt.  j counts the
    completed tours of all chains; censored tours are excluded, and so are
    chains whose sums are not finite (a negative killing rate of the
    unadjusted jump process makes them NaN), which are counted."""
    c = r.c_tilde
    ok = np.isfinite(r.t_done) & np.isfinite(r.a_done)
    nonfinite = int((~ok).sum())
    if nonfinite:
        r = RunResult(r.n_done[ok], r.t_done[ok], r.a_done[ok], r.censored[ok], r.t_censored[ok],
                      r.transitions[ok], r.accepts[ok], r.kills[ok], r.image, r.c_tilde,
                      None if r.large_steps is None else r.large_steps[ok],
                      None if r.large_accepts is None else r.large_accepts[ok])
    if r.n_done.sum() > 0:
        pl, pl_se = _ratio(r.t_done, r.n_done)
        lpf, lpf_se = _ratio(r.a_done, r.n_done)
    else:
        # no completed tour (the MH chain, c_tilde = 0): only pi f exists
        pl = pl_se = lpf = lpf_se = float("nan")
    pif, pif_se = _ratio(r.a_done, r.t_done)
    tot_t = r.t_done.sum() + r.t_censored.sum()
    return {
        "p_lambda": c * pl, "p_lambda_se": c * pl_se,
        "lam_pf": c * lpf, "lam_pf_se": c * lpf_se,
        "pi_f": pif, "pi_f_se": pif_se,
        "tours_done": int(r.n_done.sum()), "tours_censored": int(r.censored.sum()),
        "censored_time_frac": float(r.t_censored.sum() / tot_t) if tot_t > 0 else 0.0,
        "transitions": int(r.transitions.sum()),
        "accept_rate": float(r.accepts.sum() / max(1, r.transitions.sum())),
        "kill_rate": float(r.kills.sum() / max(1, r.transitions.sum())),
        "large_steps": int(r.large_steps.sum()) if r.large_steps is not None else 0,
        "large_accepts": int(r.large_accepts.sum()) if r.large_accepts is not None else 0,
        "nonfinite": nonfinite,
    }


def asymptotic_variance(r: RunResult) -> float:
    """Time-average variance constant of f = p: sigma^2 with
    Var(int_0^t f dt / t) ~ sigma^2 / t, estimated per unit of process time
    as sum_c (A_c - R T_c)^2 / sum_c T_c with R = sum A / sum T.

    For the restore process A_c - R T_c is a sum over the chain's completed
    tours of i.i.d. centred tour terms (the tours are the regeneration
    cycles), so by Wald's identities its second moment is E[tours] times
    the per-tour one and the ratio is the regenerative estimate
    E[(A - pi f tau)^2] / E[tau].  For the MH chain every chain is one long
    stationary run after its burn-in and the ratio is the usual estimate
    of the variance constant from independent replicates."""
    A = np.asarray(r.a_done, dtype=np.float64)
    T = np.asarray(r.t_done, dtype=np.float64)
    R = A.sum() / T.sum()
    res = A - R * T
    return float((res * res).sum() / T.sum())


def image_estimate(r: RunResult) -> np.ndarray:
    """lambda(p h_j) per pixel j: (c_tilde / j) times the summed dt splats."""
    return r.c_tilde * r.image / r.n_done.sum()


def image_batch_estimate(images: np.ndarray, tours: np.ndarray, c_tilde: float):
    """Per-pixel estimate and standard error from batch images.

    images[b] holds the dt splatted by the chains of batch b, tours[b] the
    tours those chains completed.  The estimate of lambda(p h_j) is the
    ratio c_tilde sum_b S_bj / sum_b N_b (Sec. 6.3 with f the pixel
    indicator), and its standard error the delta-method one with the
    batches as the independent units: the same ratio-estimator variance
    as for chains (see _ratio), here over B batches."""
    S = np.asarray(images, dtype=np.float64).reshape(len(tours), -1)
    N = np.asarray(tours, dtype=np.float64)
    B = len(N)
    R = S.sum(axis=0) / N.sum()
    resid = S - R[None, :] * N[:, None]
    var = (resid ** 2).sum(axis=0) / ((B - 1) * B) / (N.mean() ** 2) if B > 1 else np.full(R.shape, np.nan)
    shape = np.asarray(images).shape[1:]
    return (c_tilde * R).reshape(shape), (c_tilde * np.sqrt(var)).reshape(shape)


def batch_ranges(n_chains: int, batches: int):
    """Chain ranges of the image batches: chain c belongs to batch
    floor(c batches / n_chains)."""
    return [(-(-b * n_chains // batches), -(-(b + 1) * n_chains // batches)) for b in range(batches)]


# ---------------------------------------------------------------------------
# tile-stratified runs
# ---------------------------------------------------------------------------

def tiles(prob: Problem):
    """Pixel ranges (px0, px1, py0, py1) of the tiles, in tile order (row by
    row), and each tile's share A_t of the unit square."""
    P, W, H = prob.cfg.tile_px, prob.cfg.image_w, prob.cfg.image_h
    out = []
    for ty in range(-(-H // P)):
        for tx in range(-(-W // P)):
            px0, py0 = tx * P, ty * P
            out.append((px0, min(W, px0 + P), py0, min(H, py0 + P)))
    area = np.array([(a1 - a0) * (b1 - b0) / (W * H) for a0, a1, b0, b1 in out])
    return out, area


def tile_of_chain(prob: Problem, chains) -> np.ndarray:
    """Chain c of C works on tile floor(c T / C)."""
    T = len(tiles(prob)[0])
    return (np.asarray(chains, dtype=np.int64) * T) // int(prob.cfg.n_chains_total)


def estimate_tiles(prob: Problem, r: RunResult, c0: int = 0) -> dict:
    """Stratified estimates of a tile-stratified run over chains [c0, ...):
    each tile t is a restore problem with constant c_tilde A_t, so
    p_lambda = sum_t c_tilde A_t T_t / N_t and lambda(p f) = sum_t c_tilde
    A_t A_t' / N_t (Sec. 6.3 per tile, tiles added); pi f is their ratio.
    Standard errors: per tile the delta-method variance and covariance of
    the two tour ratios over the tile's chains, tiles independent, and the
    delta method for the ratio pi f."""
    _, area = tiles(prob)
    c = r.c_tilde
    tid = tile_of_chain(prob, np.arange(c0, c0 + len(r.n_done)))
    P = L = vP = vL = cPL = 0.0
    per_tile = []
    for t in np.unique(tid):
        m = tid == t
        N, Tt, At = r.n_done[m].astype(np.float64), r.t_done[m], r.a_done[m]
        n = m.sum()
        RT, RA = Tt.sum() / N.sum(), At.sum() / N.sum()
        eT, eA = Tt - RT * N, At - RA * N
        den = (n - 1) * n * N.mean() ** 2
        s_t = c * area[t]
        P += s_t * RT
        L += s_t * RA
        vP += s_t ** 2 * (eT @ eT) / den
        vL += s_t ** 2 * (eA @ eA) / den
        cPL += s_t ** 2 * (eT @ eA) / den
        per_tile.append({"tile": int(t), "p_lambda": s_t * RT, "p_lambda_se": s_t * math.sqrt((eT @ eT) / den),
                         "tours": int(N.sum()), "chains": int(n)})
    pi = L / P
    v_pi = (vL - 2 * pi * cPL + pi * pi * vP) / (P * P)
    return {"p_lambda": P, "p_lambda_se": math.sqrt(vP), "lam_pf": L, "lam_pf_se": math.sqrt(vL),
            "pi_f": pi, "pi_f_se": math.sqrt(max(v_pi, 0.0)), "tiles": per_tile,
            "tours_done": int(r.n_done.sum()), "tours_censored": int(r.censored.sum())}


def image_estimate_tiles(prob: Problem, r: RunResult, c0: int = 0) -> np.ndarray:
    """lambda(p h_j) per pixel j of a tile-stratified run: c_tilde A_t S_j /
    N_t for the tile t that holds pixel j."""
    rng, area = tiles(prob)
    tid = tile_of_chain(prob, np.arange(c0, c0 + len(r.n_done)))
    out = np.zeros_like(r.image)
    for t, (a0, a1, b0, b1) in enumerate(rng):
        m = tid == t
        if m.any():
            out[b0:b1, a0:a1] = r.c_tilde * area[t] * r.image[b0:b1, a0:a1] / r.n_done[m].sum()
    return out
