"""Block low-rank (BLR) compressed local solves for ORAS (oracle side).
TEST INFRASTRUCTURE.

Sec. 3 (the local factorisations and Table 4): the subdomain factors may be
stored in the block low-rank format, where off-diagonal blocks are replaced
by low-rank products whose error is controlled by a threshold eps_BLR (1e-3
in the paper's runs); the paper reports a faster solve in spite of a few
more iterations.

Reading used here.  The local solver is the plane recursion over the z-planes
of the subdomain box, whose factors are the explicit plane inverses
    S_1 = D_1,  S_k = D_k - L_k S_{k-1}^{-1} U_{k-1},
    forward  y_k = S_k^{-1} (r_k - L_k y_{k-1}),
    backward x_k = y_k - S_k^{-1} U_k x_{k+1}.
Each S_k^{-1} is stored in BLR form:
  * patches: the plane (sx x sy nodes) is cut along x into ceil(sx / pmax)
    parts by floor split (part t holds x in [floor(t sx / n), floor((t+1) sx / n))),
    likewise along y; patch index py * npx + px; inside a patch the nodes keep
    plane order (x fastest);
  * diagonal patch blocks stay dense;
  * every off-diagonal block M (b_I x b_J) is replaced by U V from a cross
    approximation with complete pivoting (Gaussian elimination with complete
    pivoting stopped early): with R = M, repeat
        (a, b) = the first position (row-major) of the largest |R_ab|;
        stop if |R_ab| <= eps * max|S_k^{-1}|;
        u = R[:, b], v = R[a, :] / R_ab, R -= u v, append u to U and v to V;
    so every entry of M - U V is at most eps * max|S_k^{-1}| in modulus;
  * a block whose rank would exceed floor(b_I b_J / (b_I + b_J)) (where the
    product costs as much as the block) before the test passes stays dense.
eps = 0 keeps every block exact (dense, or a cross approximation whose
residual is exactly zero).
"""
from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np

from . import operator as op
from . import oras


def patch_cuts(n: int, pmax: int) -> List[int]:
    parts = -(-n // pmax)
    return [(t * n) // parts for t in range(parts + 1)]


def patches(sx: int, sy: int, pmax: int) -> List[np.ndarray]:
    """Plane node indices (y * sx + x) of every patch, patch order py-major."""
    cx, cy = patch_cuts(sx, pmax), patch_cuts(sy, pmax)
    out = []
    for py in range(len(cy) - 1):
        for px in range(len(cx) - 1):
            ys = np.arange(cy[py], cy[py + 1])
            xs = np.arange(cx[px], cx[px + 1])
            out.append((ys[:, None] * sx + xs[None, :]).reshape(-1))
    return out


def cross_approx(M: np.ndarray, tol: float, rank_cap: int) -> Optional[Tuple[np.ndarray, np.ndarray]]:
    """U (b_I x r), V (r x b_J) with max|M - U V| <= tol, or None if that
    needs more than rank_cap terms (complete-pivoting cross approximation)."""
    R = np.array(M, dtype=np.complex128)
    us, vs = [], []
    while True:
        a, b = np.unravel_index(int(np.argmax(np.abs(R))), R.shape)
        piv = R[a, b]
        if abs(piv) <= tol:
            break
        if len(us) == rank_cap:
            return None
        u = R[:, b].copy()
        v = R[a, :] / piv
        R -= np.outer(u, v)
        us.append(u)
        vs.append(v)
    bi, bj = M.shape
    U = np.array(us).T if us else np.zeros((bi, 0), dtype=np.complex128)
    V = np.array(vs) if vs else np.zeros((0, bj), dtype=np.complex128)
    return U, V


class BlrPlane:
    """One plane inverse in BLR form."""

    def __init__(self, Sinv: np.ndarray, groups: List[np.ndarray], eps: float):
        self.groups = groups
        self.P = Sinv.shape[0]
        self.smax = float(np.abs(Sinv).max())
        tol = eps * self.smax
        npch = len(groups)
        self.blocks = {}
        self.rank = np.full((npch, npch), -1, dtype=np.int64)   # -1: dense
        for I, gi in enumerate(groups):
            for J, gj in enumerate(groups):
                M = Sinv[np.ix_(gi, gj)]
                if I == J:
                    self.blocks[I, J] = ("dense", M)
                    continue
                cap = (len(gi) * len(gj)) // (len(gi) + len(gj))
                uv = cross_approx(M, tol, cap)
                if uv is None:
                    self.blocks[I, J] = ("dense", M)
                else:
                    self.blocks[I, J] = ("lr", uv)
                    self.rank[I, J] = uv[0].shape[1]

    def matrix(self) -> np.ndarray:
        """The approximated S^{-1} as a dense matrix (for tests)."""
        out = np.zeros((self.P, self.P), dtype=np.complex128)
        for (I, J), (kind, val) in self.blocks.items():
            blk = val if kind == "dense" else val[0] @ val[1]
            out[np.ix_(self.groups[I], self.groups[J])] = blk
        return out

    def apply(self, x: np.ndarray) -> np.ndarray:
        """S~^{-1} x for x (P, s)."""
        y = np.zeros((self.P, x.shape[1]), dtype=np.complex128)
        for (I, J), (kind, val) in self.blocks.items():
            xj = x[self.groups[J]]
            y[self.groups[I]] += val @ xj if kind == "dense" else val[0] @ (val[1] @ xj)
        return y

    def stored_entries(self) -> int:
        tot = 0
        for kind, val in self.blocks.values():
            tot += val.size if kind == "dense" else val[0].size + val[1].size
        return tot


class PlaneSolver:
    """Plane recursion for one subdomain matrix with BLR plane inverses
    (eps=None: exact inverses)."""

    def __init__(self, B, sx: int, sy: int, sz: int, eps: Optional[float], pmax: int = 8):
        B = B.tocsr()
        p = sx * sy
        self.p, self.sz = p, sz
        self.L, self.U, self.inv = [], [], []
        groups = patches(sx, sy, pmax)
        Sinv_prev = None
        for k in range(sz):
            rs = slice(k * p, (k + 1) * p)
            D = B[rs, rs].toarray()
            Lk = B[rs, (k - 1) * p:k * p].toarray() if k > 0 else None
            if k > 0:
                D = D - Lk @ Sinv_prev @ self.U[k - 1]
            Sinv = np.linalg.inv(D)
            self.L.append(Lk)
            self.U.append(B[rs, (k + 1) * p:(k + 2) * p].toarray() if k + 1 < sz else None)
            self.inv.append(Sinv if eps is None else BlrPlane(Sinv, groups, eps))
            Sinv_prev = Sinv        # the recursion itself uses the exact inverse

    def _ap(self, k, x):
        S = self.inv[k]
        return S @ x if isinstance(S, np.ndarray) else S.apply(x)

    def solve(self, b: np.ndarray) -> np.ndarray:
        """b (n, s) in box order (x fastest, then y, then z)."""
        p, K = self.p, self.sz
        b2 = b.reshape(K, p, -1)
        y = np.empty_like(b2, dtype=np.complex128)
        for k in range(K):
            r = b2[k] if k == 0 else b2[k] - self.L[k] @ y[k - 1]
            y[k] = self._ap(k, r)
        x = np.empty_like(y)
        x[K - 1] = y[K - 1]
        for k in range(K - 2, -1, -1):
            x[k] = y[k] - self._ap(k, self.U[k] @ x[k + 1])
        return x.reshape(b.shape)


class OrasBLR:
    """ORAS whose local solves use the BLR plane recursion."""

    def __init__(self, F: op.Fields, parts, overlap, eps: Optional[float], pmax: int = 8,
                 interface: str = "robin"):
        self.F = F
        self.subs = oras.partition((F.nx, F.ny, F.nz), parts, overlap)
        self.solvers = []
        for s in self.subs:
            B = op.csr_from_coeffs(oras.local_coeffs(F, s, interface))
            sx, sy, sz = (s.hi[a] - s.lo[a] for a in range(3))
            self.solvers.append(PlaneSolver(B, sx, sy, sz, eps, pmax))

    def apply(self, v: np.ndarray) -> np.ndarray:
        single = v.ndim == 3
        V = v[None] if single else v
        out = np.zeros_like(V, dtype=np.complex128)
        for s, sol in zip(self.subs, self.solvers):
            box = (slice(s.lo[2], s.hi[2]), slice(s.lo[1], s.hi[1]), slice(s.lo[0], s.hi[0]))
            bshape = tuple(s.hi[a] - s.lo[a] for a in (2, 1, 0))
            r = V[(slice(None),) + box].reshape(V.shape[0], -1).T
            y = sol.solve(np.ascontiguousarray(r)).T.reshape((V.shape[0],) + bshape)
            own = tuple(slice(s.olo[a] - s.lo[a], s.ohi[a] - s.lo[a]) for a in (2, 1, 0))
            dst = (slice(None),) + tuple(slice(s.olo[a], s.ohi[a]) for a in (2, 1, 0))
            out[dst] = y[(slice(None),) + own]
        return out[0] if single else out
