"""Differentiable forward map m -> receiver data for frequency-domain FWI.

The paper presents the solver as the forward engine of frequency-domain FWI,
where incident and adjoint wavefields are needed (sec. 1, sec. 4), and notes
that the Helmholtz matrix is complex symmetric (sec. 2).  For
d_s = P A(m)^{-1} b_s and a real loss L(d) whose gradient torch passes as
g = dL/dRe(d) + i dL/dIm(d):

    mu_s = A^{-H} P^T g_s      (A^H = conj(A): a conjugate solve, same factors)
    dL/dm_i = -Re sum_s mu_s^H (dA/dm_i) u_s

By default the stencil weights, PML and Q stay frozen at the last
``assemble`` (so only the mass term depends on m).  With weights="follow" the
lambda-adaptive weights are picked again from the local G at every m (sec.
2.3) and the gradient adds their derivative through the table slope (the
exact gradient of that discretisation); the PML and Q stay fixed.  Every step
runs in the HIP library; this module wires the calls into torch's autograd.

Memory policy: the forward wavefields are kept for the backward pass when
their size fits ``save_budget_bytes``; otherwise the backward recomputes them
with one more forward solve.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import oras


@dataclass
class ForwardSetup:
    solver: oras.Solver
    sources: Sequence[Sequence[int]]
    receivers: Sequence[Sequence[int]]
    parts: Sequence[int]
    overlap: int = 2
    prec: int = oras.C128
    tol: float = 1e-8
    restart: int = 30
    maxit: int = 2000
    save_budget_bytes: float = 32e9
    stats: Optional[dict] = None
    weights: str = "frozen"       # or "follow": weights picked from G(m)
    blr_eps: Optional[float] = None   # block low-rank plane inverses after each factorisation


def _prepare(fs: ForwardSetup, m: torch.Tensor):
    """Operator and factors for squared slowness m (skipped when current)."""
    S = fs.solver
    # the last m is kept referenced, so its memory cannot be reused by another
    # tensor while (address, version) identifies the factors
    key = (m.data_ptr(), m._version)
    if getattr(S, "_m_key", None) != key:
        S.set_m(m.detach().contiguous(), weights=fs.weights)
        S.factor(fs.parts, fs.overlap, fs.prec)
        if fs.blr_eps is not None:
            S.compress(fs.blr_eps)
        S._m_key = key
        S._m_ref = m


def _forward_fields(fs: ForwardSetup, m: torch.Tensor):
    _prepare(fs, m)
    S = fs.solver
    b = S.point_sources(fs.sources)
    r = S.solve(b, fs.tol, restart=fs.restart, maxit=fs.maxit)
    if not r.converged.all():
        raise RuntimeError("forward solve did not converge")
    if fs.stats is not None:
        fs.stats.setdefault("forward_iters", []).append(r.iters.tolist())
    return r.x


class HelmholtzData(torch.autograd.Function):
    """d = P A(m)^{-1} b for all sources; m (nz, ny, nx) float64 on the GPU."""

    @staticmethod
    def forward(ctx, m: torch.Tensor, fs: ForwardSetup):
        u = _forward_fields(fs, m)
        d = fs.solver.sample(u, fs.receivers)
        nbytes = u.numel() * u.element_size()
        ctx.fs = fs
        ctx.saved_u = u if nbytes <= fs.save_budget_bytes else None
        ctx.save_for_backward(m)
        return d

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (m,) = ctx.saved_tensors
        fs = ctx.fs
        S = fs.solver
        u = ctx.saved_u
        if u is None:
            u = _forward_fields(fs, m)          # recompute when not kept
        else:
            _prepare(fs, m)                     # factors of this m
        bt = S.spread(g.contiguous().to(torch.complex128), fs.receivers)
        r = S.solve(bt, fs.tol, restart=fs.restart, maxit=fs.maxit, conj=True)
        if not r.converged.all():
            raise RuntimeError("adjoint solve did not converge")
        if fs.stats is not None:
            fs.stats.setdefault("adjoint_iters", []).append(r.iters.tolist())
        grad = S.gradient(u, r.x, weights=fs.weights == "follow")
        return grad, None


def receiver_data(m: torch.Tensor, fs: ForwardSetup) -> torch.Tensor:
    return HelmholtzData.apply(m, fs)
