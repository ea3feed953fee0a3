"""Learned regeneration distribution: the refit loop around the library.

mu_theta = (1 - beta) GMM(MLP_theta(c)) + beta Uniform([0,1]^d).  The MLP
maps a fixed, seeded context vector c in R^12 to the K logits, K d means and
K d log standard deviations of a diagonal Gaussian mixture (the layout the
step kernels read as restore_mu parameters).  mu has to be one fixed,
state-independent density for the whole of a run, since the kill rate
k = c~ u / p needs u pointwise (Sec. 6.2); it is refitted between runs.

Refit r: run the chains with mu_r (uniform for r = 0), record the
pairs (x_{i-1}, dt_i) of the last few steps of every chain
(restore_step_record; the time-weighted pairs are draws of pi, Sec. 7.4,
eq. (approx)), then take full-batch Adam steps on the time-weighted negative
log-likelihood -sum dt log u_theta(x) / sum dt.  Every step (MLP forward/backward on the
matrix cores, NLL and its gradient, Adam) runs in the library's kernels;
this module only allocates the buffers and sequences the calls.

With G > 1 context rows, one MLP gives one mixture per row: the batched
targets' regeneration distributions from one shared network (one seeded
context vector per target), trained on the sum of the targets' losses, so
that the layers run as G-row GEMMs on the matrix cores.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import restore as R


@dataclass
class MlpGmm:
    """Parameters, optimiser state and work buffers of one MLP -> GMM map
    on the current GPU, for G context rows (one mixture per row)."""
    d: int
    K: int = 64
    in_dim: int = 12
    hidden: int = 64
    beta: float = 0.1
    seed: int = 3004
    init_std: float = 0.15
    G: int = 1
    t: int = 0
    rollbacks: int = 0
    history: list = field(default_factory=list)

    def __post_init__(self):
        self.shape = R.restore_mlp_shape(self.in_dim, self.hidden, self.K, self.d)
        self.n_params, n_act = R.restore_mlp_param_count(self.shape)
        self.O = self.K * (1 + 2 * self.d)
        rng = np.random.default_rng(self.seed)
        theta = np.zeros(self.n_params, dtype=np.float32)
        H, i, O = self.hidden, self.in_dim, self.O
        off = 0
        for rows, cols in ((H, i), (H, H), (O, H)):
            # fan-in scaled weights; the output layer starts small so that
            # the initial mixture is set by its bias
            scale = 1.0 / math.sqrt(cols) if rows != O else 0.01 / math.sqrt(cols)
            theta[off:off + rows * cols] = rng.standard_normal(rows * cols) * scale
            off += rows * cols + rows
        b3 = theta[-O:]
        b3[:self.K] = 0.0
        b3[self.K:self.K + self.K * self.d] = rng.uniform(0.1, 0.9, self.K * self.d)
        b3[self.K + self.K * self.d:] = math.log(self.init_std)
        dev = "cuda"
        self.theta = torch.from_numpy(theta).to(dev)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.zeros_like(self.theta)
        self.ctx = torch.from_numpy(rng.standard_normal((self.G, self.in_dim)).astype(np.float32)).to(dev)
        self.act = torch.empty((self.G, n_act), dtype=torch.float32, device=dev)
        self.out = torch.empty((self.G, O), dtype=torch.float32, device=dev)
        self.dout = torch.empty((self.G, O), dtype=torch.float32, device=dev)
        self.work = torch.empty((2 * self.G, self.hidden), dtype=torch.float32, device=dev)
        self.loss = torch.zeros(self.G, dtype=torch.float64, device=dev)
        ws = R.restore_gmm_nll_workspace_bytes()
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=dev)
        self.forward()

    # --- one pass of each library call --------------------------------------
    def forward(self) -> torch.Tensor:
        R.restore_mlp_forward(self.shape, self.theta.data_ptr(), self.ctx.data_ptr(), self.G, self.act.data_ptr(),
                              self.out.data_ptr())
        return self.out

    def nll_and_grad(self, x: torch.Tensor, w: torch.Tensor, g: int = 0) -> None:
        """loss[g] and dL/d(out[g]) on (x [n][d], w [n]) for the current out."""
        n = w.numel()
        R.restore_gmm_nll(self.K, self.d, self.beta, self.out[g].data_ptr(), x.data_ptr(), w.data_ptr(), n,
                          self.dout[g].data_ptr(), self.loss[g:].data_ptr(), self.workspace.data_ptr(),
                          self.workspace.numel())

    def backward(self) -> None:
        """grad = d(sum_g dout[g] . out[g]) / d theta."""
        R.restore_mlp_backward(self.shape, self.theta.data_ptr(), self.ctx.data_ptr(), self.G, self.act.data_ptr(),
                               self.dout.data_ptr(), self.work.data_ptr(), self.grad.data_ptr())

    def adam(self, lr: float) -> None:
        self.t += 1
        R.restore_adam_step(self.theta.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                            self.n_params, self.t, lr)

    def fit(self, x, w, epochs: int, lr: float, log_every: int = 0, rise_tol: float = 0.5) -> list:
        """Full-batch Adam on the weighted NLL of (x, w) -- with G rows,
        x and w are lists of G sample sets and the objective is the sum of
        the rows' losses; returns the (summed) loss after each logged epoch
        (losses are read back only when logged)."""
        xs = list(x) if self.G > 1 else [x]
        ws = list(w) if self.G > 1 else [w]
        assert len(xs) == self.G and len(ws) == self.G
        xs = [xi.reshape(-1, self.d).contiguous() for xi in xs]
        ws = [wi.reshape(-1).contiguous() for wi in ws]

        def losses_of_rows():
            for g in range(self.G):
                self.nll_and_grad(xs[g], ws[g], g)

        # Adam can leave the stable region (heavy-tailed time weights make
        # single samples dominate the gradient): at every check the loss on
        # this fixed data set must be finite and must not have risen by more
        # than `rise_tol` nats per context row over the lowest loss of the good
        # checks so far (the loss is the sum of the rows' losses); otherwise
        # the parameters and the optimiser state roll back to the last good
        # check and the learning rate is halved for the rest of the fit
        log_every = log_every or max(1, epochs // 4)
        self.forward()
        losses_of_rows()
        best = float(self.loss.sum().item())
        good = self._snapshot()
        losses = []

        def acceptable(loss: float) -> bool:
            return (math.isfinite(loss) and loss <= best + rise_tol * self.G
                    and bool(torch.isfinite(self.theta).all()))

        for e in range(epochs):
            self.forward()
            losses_of_rows()
            if e % log_every == 0 or e == epochs - 1:
                # the loss of the current parameters, before this epoch's step
                loss = float(self.loss.sum().item())
                if acceptable(loss):
                    losses.append((e, loss))
                    best = min(best, loss)
                    good = self._snapshot()
                else:
                    self._restore(good)
                    lr *= 0.5
                    self.rollbacks += 1
                    losses.append((e, float("nan")))
                    self.forward()
                    losses_of_rows()
            self.backward()
            self.adam(lr)
        self.forward()
        losses_of_rows()
        if not acceptable(float(self.loss.sum().item())):
            self._restore(good)
            self.rollbacks += 1
            self.forward()
            losses_of_rows()
        losses.append((epochs, float(self.loss.sum().item())))
        self.history.append(losses)
        return losses

    def _snapshot(self):
        return (self.theta.clone(), self.m.clone(), self.v.clone(), self.t)

    def _restore(self, snap) -> None:
        theta, m, v, t = snap
        self.theta.copy_(theta)
        self.m.copy_(m)
        self.v.copy_(v)
        self.t = t

    def mu(self, g: int = 0) -> dict:
        """restore_mu descriptor fields of row g for the current parameters
        (the device row is copied by restore_init, so later training does
        not touch a run that has started)."""
        self.forward()
        return {"params_dev": self.out[g], "n_comp": self.K, "beta": self.beta}


def provable_c_tilde(c_tilde_uniform: float, beta: float) -> float:
    """c~ for a learned mu with defensive share beta, from the c~ of the
    uniform rule c~_U = max(1, 8 P / B) (P an upper bound of p on the box):
    u >= beta on the box, so c~ = c~_U / beta keeps the mean lifetime
    p / (c~ u) of every tour at most B / 8 steps for any learned mixture,
    and tours in flight at the end of the budget finish within the drain
    with overwhelming probability."""
    return max(1.0, c_tilde_uniform / beta)


def record_samples(wl, mu: Optional[dict], c_tilde: float, seed: int, record_steps: int,
                   n_record: Optional[int] = None):
    """Run the workload once with regeneration distribution mu and return
    the pairs (x_{i-1}, dt_i) of the last record_steps steps of chains
    [0, n_record) (default: every chain)."""
    n_record = wl.n_chains if n_record is None else n_record
    prob = R.problem_from_workload(wl, mu=mu, seed=seed, c_tilde=c_tilde, integrand_p=False, image=None)
    run = R.Run(prob)
    if wl.n_steps > record_steps:
        run.step(wl.n_steps - record_steps)
    x, w = run.step_record(min(record_steps, wl.n_steps), n_record)
    run.close()
    return x.reshape(-1, wl.d), w.reshape(-1)


def effective_fraction(w: torch.Tensor) -> float:
    """(sum w)^2 / (n sum w^2): the effective sample fraction of weights."""
    w = w.double()
    return float(w.sum() ** 2 / (w.numel() * (w * w).sum()))


def refit(wl, model: MlpGmm, c_tilde_eval: float, refits: int = 5, record_steps: int = 4, epochs: int = 300,
          lr: float = 2e-2, seed: int = 3004, c_tilde_explore: float = 1.0, log=print) -> list:
    """`refits` refits of model on restore samples of the workload.

    Refit 0 samples with uniform mu at the exploratory c~_explore: tours
    that reach a region of high p live long there and the local moves
    climb to the modes, so the recorded pairs cover the modes (weighted by
    how often they are found rather than by their mass).  Later refits
    sample with the current learned mu at the c~ of the evaluation runs;
    their time-weighted pairs are then draws of pi (Sec. 7.4), which
    corrects the mixture weights and shapes.  mu only has to be a fixed
    density during a run, so the training data can come from any of these
    runs without biasing later estimates.  Returns per-refit diagnostics."""
    out = []
    mu = None
    for r in range(refits):
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        ct = c_tilde_explore if mu is None else c_tilde_eval
        x, w = record_samples(wl, mu, ct, seed + 7919 * r, record_steps)
        losses = model.fit(x, w, epochs, lr, log_every=max(1, epochs // 4))
        t1.record()
        torch.cuda.synchronize()
        sec = t0.elapsed_time(t1) / 1e3
        ess = effective_fraction(w)
        log(f"[refit {r}] {w.numel()} samples (c~ {ct:.3g}, effective fraction {ess:.3g}), "
            f"nll {losses[0][1]:.4f} -> {losses[-1][1]:.4f}, {sec:.2f} s")
        out.append({"refit": r, "samples": int(w.numel()), "c_tilde": ct, "effective_fraction": ess,
                    "nll_first": losses[0][1], "nll_last": losses[-1][1], "seconds": sec})
        mu = model.mu()
        del x, w
    return out


def refit_shared(wls, model: MlpGmm, refits: int = 3, record_steps: int = 4, epochs: int = 300,
                 lr: float = 2e-2, seed: int = 3004, c_tilde_explore: float = 1.0, explore_chains: int = 0,
                 log=print) -> list:
    """refit() for G targets of one dimension sharing one model (row g is
    target g's mixture): every refit records each target with its current
    mixture (uniform mu at c~_explore in refit 0, with explore_chains
    chains if given; afterwards at its provable c~) and fits the shared
    parameters on the sum of the targets' losses.  Returns per-refit
    diagnostics."""
    assert model.G == len(wls) and all(w.d == model.d for w in wls)
    out = []
    for r in range(refits):
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        xs, ws = [], []
        for g, wl in enumerate(wls):
            mu = None if r == 0 else model.mu(g)
            ct = c_tilde_explore if r == 0 else provable_c_tilde(wl.c_tilde, model.beta)
            src = wl.with_(n_chains=explore_chains) if (r == 0 and explore_chains) else wl
            x, w = record_samples(src, mu, ct, seed + 7919 * r + 104729 * g, record_steps)
            xs.append(x)
            ws.append(w)
        losses = model.fit(xs, ws, epochs, lr, log_every=max(1, epochs // 4))
        t1.record()
        torch.cuda.synchronize()
        sec = t0.elapsed_time(t1) / 1e3
        log(f"[shared refit {r}] {model.G} targets x {ws[0].numel()} samples, summed nll "
            f"{losses[0][1]:.4f} -> {losses[-1][1]:.4f}, {sec:.2f} s")
        out.append({"refit": r, "targets": model.G, "samples_per_target": int(ws[0].numel()),
                    "nll_first": losses[0][1], "nll_last": losses[-1][1], "seconds": sec})
        del xs, ws
    return out
