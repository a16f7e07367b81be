"""The plain definition u = A^{-1} b (oracle side).  TEST INFRASTRUCTURE.

The method's result is the exact solution of the discrete system A u = f
(paper eq. 1.1); ORAS-GMRES only reaches it to a tolerance.  This module
computes it with its own direct solver: A is block tridiagonal over z-planes
(the 27-point stencil couples plane k only to k-1 and k+1), so

    S_0 = D_0,   S_k = D_k - L_k S_{k-1}^{-1} U_{k-1}
    y_0 = S_0^{-1} b_0,   y_k = S_k^{-1} (b_k - L_k y_{k-1})
    x_{K-1} = y_{K-1},    x_k = y_k - S_k^{-1} U_k x_{k+1}

with every S_k factorised by LAPACK getrf (partial pivoting inside the plane).
Cross-checked in tests against dense numpy.linalg.solve (brute force) and
SciPy's SuperLU on small grids.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


class BlockTridiagLU:
    def __init__(self, A: sp.csr_matrix, plane: int, nplanes: int):
        self.p = plane
        self.K = nplanes
        A = A.tocsr()
        p = plane
        self.lu = []
        self.W = []      # S_k^{-1} U_k
        self.L = []
        prevW = None
        for k in range(nplanes):
            rs = slice(k * p, (k + 1) * p)
            D = A[rs, rs].toarray()
            if k > 0:
                Lk = A[rs, (k - 1) * p:k * p].toarray()
                D = D - Lk @ prevW
                self.L.append(Lk)
            else:
                self.L.append(None)
            lu = sla.lu_factor(D, check_finite=True)
            self.lu.append(lu)
            if k + 1 < nplanes:
                Uk = A[rs, (k + 1) * p:(k + 2) * p].toarray()
                prevW = sla.lu_solve(lu, Uk)
                self.W.append(prevW)

    def solve(self, b: np.ndarray) -> np.ndarray:
        """b shaped (n,) or (n, s)."""
        p, K = self.p, self.K
        b2 = b.reshape(K, p, -1)
        y = np.empty_like(b2, dtype=np.complex128)
        for k in range(K):
            r = b2[k] if k == 0 else b2[k] - self.L[k] @ y[k - 1]
            y[k] = sla.lu_solve(self.lu[k], r)
        x = np.empty_like(y)
        x[K - 1] = y[K - 1]
        for k in range(K - 2, -1, -1):
            x[k] = y[k] - self.W[k] @ x[k + 1]
        return x.reshape(b.shape)


def solve(A: sp.csr_matrix, shape, b: np.ndarray) -> np.ndarray:
    """u = A^{-1} b for b shaped (nsrc, nz, ny, nx) or (nz, ny, nx)."""
    nz, ny, nx = shape
    lu = BlockTridiagLU(A, nx * ny, nz)
    if b.ndim == 3:
        return lu.solve(b.reshape(-1)).reshape(shape)
    B = b.reshape(b.shape[0], -1).T
    return lu.solve(B).T.reshape(b.shape)
