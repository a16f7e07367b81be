"""Right-preconditioned flexible GMRES, pseudo-block over columns (oracle).
TEST INFRASTRUCTURE.

Paper sec. 2.1: right preconditioning, solve A M^{-1} y = f, u = M^{-1} y, so
the monitored residual does not depend on M.  Sec. 2.2: the flexible variant
(FGMRES) stores the preconditioned vectors z_j = M^{-1} v_j; multiple
right-hand sides are processed by a pseudo-block method (each column keeps its
own Krylov space; the operations are merely grouped); classical Gram-Schmidt
(CGS) orthogonalisation (sec. 3.2, local solvers and multiple RHS).

Stopping test (reading of the paper's relative backward error, printed with
squared norms): per column ||b - A x|| <= tol ||b||, unsquared, with the true
residual recomputed at the end of every cycle.  Givens rotations use a real
cosine: for a = H_jj, b = H_{j+1,j}, r = sqrt(|a|^2 + |b|^2), c = |a| / r,
s = (a / |a|) conj(b) / r (c = 0, s = 1 when a = 0).
"""
from __future__ import annotations

import numpy as np


def fgmres(Aop, Mop, b: np.ndarray, tol: float, restart: int, maxit: int, x0=None):
    """Single column.  Aop, Mop act on flat complex vectors.  Returns
    (x, iterations, converged, residual history)."""
    b = b.astype(np.complex128)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, True, [0.0]
    hist = []
    it = 0
    r = b - Aop(x)
    while True:
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta <= tol * bnorm:
            return x, it, True, hist
        if it >= maxit:
            return x, it, False, hist
        m = restart
        V = np.zeros((m + 1, b.size), dtype=np.complex128)
        Z = np.zeros((m, b.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        jend = 0
        for j in range(m):
            Z[j] = Mop(V[j])
            w = Aop(Z[j])
            h = V[:j + 1].conj() @ w            # CGS: one projection pass
            w = w - V[:j + 1].T @ h
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            rr = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if abs(a) == 0.0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / rr
                sn[j] = (a / abs(a)) * np.conj(bb) / rr
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            jend = j + 1
            if abs(g[j + 1]) <= tol * bnorm or hn == 0.0 or it >= maxit:
                break
            V[j + 1] = w / hn
        y = np.zeros(jend, dtype=np.complex128)
        for i in range(jend - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:jend] @ y[i + 1:jend]) / H[i, i]
        x = x + Z[:jend].T @ y
        r = b - Aop(x)


def fgmres_block(Aop, Mop, B: np.ndarray, tol, restart, maxit):
    """Pseudo-block: each column solved with its own Krylov space.
    B shaped (s, n).  Returns (X, iters, converged)."""
    X = np.zeros_like(B, dtype=np.complex128)
    its, conv = [], []
    for c in range(B.shape[0]):
        x, it, ok, _ = fgmres(Aop, Mop, B[c], tol, restart, maxit)
        X[c] = x
        its.append(it)
        conv.append(ok)
    return X, its, conv
