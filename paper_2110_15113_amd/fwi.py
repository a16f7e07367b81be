"""Multi-source frequency-domain FWI update loop.

The paper presents the solver as the engine of frequency-domain full-waveform
inversion: every model update needs the incident wavefields of all sources
and the adjoint wavefields, i.e. two block solves with the same factors
(sec. 1 and sec. 4).  This module iterates m <- m + alpha p with
    p = -H g,   g = dJ/dm from the differentiable forward map,
H the limited-memory BFGS inverse-Hessian estimate (two-loop recursion,
Nocedal 1980), the step accepted by backtracking on the sufficient-decrease
(Armijo) test, and the model kept inside [m_min, m_max] by projection
(entries held at a bound by their gradient are left out of the direction).

The optimiser is written for torch tensors and a callable
``misfit_and_gradient(m) -> (J, g)``, so the GPU map (``gpu_objective``)
and any other backend run the same loop.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Tuple

import torch

Objective = Callable[[torch.Tensor], Tuple[float, torch.Tensor]]


def two_loop(g: torch.Tensor, S: List[torch.Tensor], Y: List[torch.Tensor]) -> torch.Tensor:
    """H g for the L-BFGS inverse Hessian built from the pairs (s_i, y_i),
    oldest first, with the initial scaling gamma = s^T y / y^T y of the
    newest pair (identity when there is none)."""
    q = g.clone()
    rho = [1.0 / float(torch.sum(y * s)) for s, y in zip(S, Y)]
    a = [0.0] * len(S)
    for i in range(len(S) - 1, -1, -1):
        a[i] = rho[i] * float(torch.sum(S[i] * q))
        q -= a[i] * Y[i]
    if S:
        q *= float(torch.sum(S[-1] * Y[-1])) / float(torch.sum(Y[-1] * Y[-1]))
    for i in range(len(S)):
        b = rho[i] * float(torch.sum(Y[i] * q))
        q += (a[i] - b) * S[i]
    return q


@dataclass
class FwiResult:
    m: torch.Tensor
    history: List[dict] = field(default_factory=list)


def lbfgs(objective: Objective, m0: torch.Tensor, iters: int, *, m_min=None, m_max=None,
          mask: Optional[torch.Tensor] = None, memory: int = 5, first_step: float = 0.02,
          c1: float = 1e-4, max_backtracks: int = 8,
          callback: Optional[Callable[[int, torch.Tensor, dict], None]] = None) -> FwiResult:
    """Minimise J(m) from m0 for ``iters`` accepted updates.

    mask: 1 where the model may change (e.g. outside the absorbing layers),
    0 elsewhere; applied to every gradient.  first_step: without curvature
    pairs (first iteration, restarts) the trial step moves the model by at
    most this fraction of max |m0| (of 1 when m0 = 0).  Each history entry records J before the update, the accepted
    step, the objective evaluations used and the wall time."""
    m = m0.clone()
    lo = None if m_min is None else torch.as_tensor(m_min, dtype=m.dtype, device=m.device)
    hi = None if m_max is None else torch.as_tensor(m_max, dtype=m.dtype, device=m.device)

    def project(x):
        if lo is not None:
            x = torch.maximum(x, lo)
        if hi is not None:
            x = torch.minimum(x, hi)
        return x

    def evaluate(x):
        J, g = objective(x)
        if mask is not None:
            g = g * mask
        return float(J), g

    J, g = evaluate(m)
    S: List[torch.Tensor] = []
    Y: List[torch.Tensor] = []
    res = FwiResult(m)
    evals = 1
    for it in range(iters):
        t0 = time.perf_counter()
        # entries at a bound whose gradient points outward stay where they are
        held = torch.zeros_like(m, dtype=torch.bool)
        if lo is not None:
            held |= (m <= lo) & (g > 0)
        if hi is not None:
            held |= (m >= hi) & (g < 0)
        gf = torch.where(held, torch.zeros_like(g), g)
        p = -two_loop(gf, S, Y)
        p = torch.where(held, torch.zeros_like(p), p)
        if float(torch.sum(p * gf)) >= 0.0:          # not a descent direction: restart
            S.clear()
            Y.clear()
            p = -gf
        alpha = 1.0
        if not S:
            scale = float(m0.abs().max()) or 1.0
            alpha = first_step * scale / max(float(p.abs().max()), 1e-300)
        accepted = False
        for _ in range(max_backtracks + 1):
            m_try = project(m + alpha * p)
            step = m_try - m
            J_try, g_try = evaluate(m_try)
            evals += 1
            if J_try <= J + c1 * float(torch.sum(g * step)):
                accepted = True
                break
            alpha *= 0.5
        rec = {"iter": it, "J": J, "alpha": alpha, "evals": evals, "accepted": accepted}
        if not accepted:
            rec["time_s"] = time.perf_counter() - t0
            res.history.append(rec)
            break
        y = g_try - g
        if float(torch.sum(y * step)) > 1e-12 * float(torch.sum(step * step)) ** 0.5 * \
                float(torch.sum(y * y)) ** 0.5:
            S.append(step)
            Y.append(y)
            if len(S) > memory:
                S.pop(0)
                Y.pop(0)
        m, J, g = m_try, J_try, g_try
        rec["J_new"] = J
        rec["time_s"] = time.perf_counter() - t0
        res.history.append(rec)
        res.m = m
        if callback is not None:
            callback(it, m, rec)
    res.m = m
    return res


def gpu_objective(fs, d_obs: torch.Tensor) -> Objective:
    """J(m) = 1/2 sum |P A(m)^{-1} b_s - d_obs|^2 and its gradient through the
    HIP forward map and adjoint (``fs``: an autograd.ForwardSetup)."""
    from .autograd import receiver_data

    def f(m: torch.Tensor):
        x = m.detach().clone().requires_grad_(True)
        d = receiver_data(x, fs)
        J = 0.5 * (d - d_obs).abs().pow(2).sum()
        J.backward()
        return J.item(), x.grad.detach()

    return f


class MultiFrequencyObjective:
    """J(m) = sum over frequencies of 1/2 sum |P A_f(m)^{-1} b_s - d_obs_f|^2 and
    its gradient, with every frequency in flight on the GPU at once (sec. 1:
    frequency-domain FWI inverts a few frequencies; each has its own operator
    and factors).  One context and HIP stream per frequency
    (``frequencies.FrequencyBatch``, assembled on the start model, which fixes
    the PML and Q); each evaluation runs, per frequency and in its own host
    thread, set_m, factorisation (optionally BLR), the forward block solve,
    sampling, the adjoint (conjugate) solve of the spread residuals and the
    gradient -- the steps of ``autograd.HelmholtzData`` called directly."""

    def __init__(self, fb, sources, receivers, d_obs, parts, overlap: int = 2,
                 tol: float = 1e-8, restart: int = 30, maxit: int = 2000,
                 weights: str = "follow", blr_eps: Optional[float] = None,
                 concurrent: bool = True):
        if len(d_obs) != len(fb.items):
            raise ValueError("one observed-data block per frequency")
        self.fb, self.sources, self.receivers = fb, sources, receivers
        self.d_obs = d_obs
        self.parts, self.overlap, self.tol = parts, overlap, tol
        self.restart, self.maxit = restart, maxit
        self.weights, self.blr_eps, self.concurrent = weights, blr_eps, concurrent
        self.stats = {"iters": []}

    def __call__(self, m: torch.Tensor):
        n = len(self.fb.items)
        Js = [0.0] * n
        gs = [None] * n
        iters = [None] * n
        m = m.detach().contiguous()

        def one(i, it):
            S = it.solver
            S.set_m(m, weights=self.weights)
            S.factor(self.parts, self.overlap, self.fb.prec)
            if self.blr_eps is not None:
                S.compress(self.blr_eps)
            b = S.point_sources(self.sources)
            r = S.solve(b, self.tol, restart=self.restart, maxit=self.maxit)
            if not r.converged.all():
                raise RuntimeError("forward solve did not converge")
            res = S.sample(r.x, self.receivers) - self.d_obs[i]
            Js[i] = 0.5 * float(res.abs().pow(2).sum())
            ra = S.solve(S.spread(res.contiguous(), self.receivers), self.tol,
                         restart=self.restart, maxit=self.maxit, conj=True)
            if not ra.converged.all():
                raise RuntimeError("adjoint solve did not converge")
            gs[i] = S.gradient(r.x, ra.x, weights=self.weights == "follow")
            iters[i] = (int(r.total_iters), int(ra.total_iters))

        self.fb._run(one, self.concurrent)
        self.stats["iters"].append(iters)
        g = gs[0].clone()
        for x in gs[1:]:
            g += x
        # the per-frequency tensors were made on the frequencies' streams: finish
        # the sum before they return to the allocator
        torch.cuda.synchronize(g.device)
        return sum(Js), g
