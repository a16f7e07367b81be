"""Pivots of the plane Schur complements without row exchanges (oracle side).
TEST INFRASTRUCTURE.

Paper sec. 2.2: every local matrix B_j is factorised once at set-up.  With
its nodes numbered plane by plane (z slowest) B_j is block tridiagonal and
block elimination over the planes gives the Schur complements

    S_0 = D_0,   S_k = D_k - L_k S_{k-1}^{-1} U_{k-1},

(the same recursion as ``direct.BlockTridiagLU``).  The device inverts each
S_k by elimination without row exchanges, and its pivots are then the
diagonal of U in S_k = L U with unit lower L.  This module computes those
pivots in FP64 from their definition (Gaussian elimination without
exchanges: d_i is entry (i, i) after the rank-one updates of the earlier
steps), and from them the statistic the library reports per plane,

    r_k = min_i |d_i| / max |S_k|.

Pins (tests/test_oracle_pivots.py): the pivots are the ratios of successive
leading principal minors, d_i = det S[:i+1, :i+1] / det S[:i, :i]; the
closed-form recursion of a tridiagonal Toeplitz matrix; the product of the
pivots is det S_k; a singular B_j (the Neumann-only Laplacian of an interior
box at omega = 0) is detected.
"""
from __future__ import annotations

from typing import List

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def unpivoted_pivots(S: np.ndarray) -> np.ndarray:
    """Diagonal of U in S = L U (unit lower L, no row exchanges)."""
    A = np.array(S, dtype=np.complex128, copy=True)
    n = A.shape[0]
    d = np.empty(n, dtype=np.complex128)
    for i in range(n):
        d[i] = A[i, i]
        if i + 1 < n:
            if d[i] == 0:
                d[i + 1:] = np.nan
                break
            A[i + 1:, i + 1:] -= np.outer(A[i + 1:, i] / d[i], A[i, i + 1:])
    return d


def plane_schur(B: sp.spmatrix, plane: int, nplanes: int) -> List[np.ndarray]:
    """The plane Schur complements S_0 .. S_{K-1} of B (planes of ``plane``
    nodes, z slowest)."""
    B = B.tocsr()
    p = plane
    out = []
    prevW = None
    for k in range(nplanes):
        rs = slice(k * p, (k + 1) * p)
        D = B[rs, rs].toarray()
        if k > 0:
            D = D - B[rs, (k - 1) * p:k * p].toarray() @ prevW
        out.append(D)
        if k + 1 < nplanes:
            prevW = sla.lu_solve(sla.lu_factor(D), B[rs, (k + 1) * p:(k + 2) * p].toarray())
    return out


def plane_pivot_ratios(B: sp.spmatrix, plane: int, nplanes: int) -> np.ndarray:
    """r_k = min |d_i(S_k)| / max |S_k| for every plane k."""
    r = []
    for S in plane_schur(B, plane, nplanes):
        d = unpivoted_pivots(S)
        r.append(float(np.min(np.abs(d)) / np.max(np.abs(S))))
    return np.array(r)


def check_nonsingular(B: sp.spmatrix, plane: int, nplanes: int, rtol: float = 1e-12):
    """Raise numpy.linalg.LinAlgError when some plane's pivot ratio is below
    rtol (B singular to working precision); return the ratios otherwise."""
    r = plane_pivot_ratios(B, plane, nplanes)
    k = int(np.argmin(r))
    if not np.isfinite(r[k]) or r[k] < rtol:
        raise np.linalg.LinAlgError(f"singular local matrix: plane {k} pivot ratio {r[k]:.3e}")
    return r
