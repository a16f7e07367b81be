"""One-level ORAS preconditioner (oracle side).  TEST INFRASTRUCTURE.

Paper sec. 2.1: M^{-1} = sum_j R_j^T D_j B_j^{-1} R_j with Boolean
restrictions R_j to overlapping subdomains, a diagonal partition of unity D_j
(sum_j R_j^T D_j R_j = I) and local matrices B_j carrying Robin (impedance)
conditions on the interior part of their boundary.  Sec. 2.2: for finite
differences the regular grid is cut into cuboids that are extended by a few
grid layers ("overlap").

Reading used here:
  * owned cuboids by floor split: along axis a with P_a parts, part t owns
    nodes [floor(t n_a / P_a), floor((t+1) n_a / P_a));
  * the subdomain box extends the owned cuboid by ``overlap`` layers on every
    side that is not a global boundary (clipped to the grid);
  * D_j is Boolean: 1 on the owned nodes (restricted additive Schwarz), so
    every node takes its value from its owner's local solve;
  * B_j from operator.row_coeffs(..., restrict=True) (cut fluxes + Robin);
    or, with interface='pml' (PML transmission conditions, sec. 2.2 note on
    the size of overlap), B_j = R_j A(s_j) R_j^T: the operator assembled with
    the subdomain's stretching profile (global PML plus an interface PML over
    the overlap layers, operator.interface_pml_profile), restricted to the
    box (couplings to nodes outside the box dropped: Dirichlet truncation);
  * local solves by SciPy SuperLU, a library routine unrelated to the GPU's
    plane-block factorisation.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse.linalg as spla

from . import operator as op


@dataclass
class Sub:
    lo: tuple       # box (x, y, z) inclusive lower corner
    hi: tuple       # box exclusive upper corner
    olo: tuple      # owned cuboid
    ohi: tuple


def partition(n, parts, overlap) -> List[Sub]:
    """n = (nx, ny, nz), parts = (Px, Py, Pz)."""
    cuts = [[(t * n[a]) // parts[a] for t in range(parts[a] + 1)] for a in range(3)]
    subs = []
    for tz in range(parts[2]):
        for ty in range(parts[1]):
            for tx in range(parts[0]):
                t = (tx, ty, tz)
                olo = tuple(cuts[a][t[a]] for a in range(3))
                ohi = tuple(cuts[a][t[a] + 1] for a in range(3))
                lo = tuple(max(0, olo[a] - overlap) for a in range(3))
                hi = tuple(min(n[a], ohi[a] + overlap) for a in range(3))
                subs.append(Sub(lo, hi, olo, ohi))
    return subs


def local_coeffs(F: op.Fields, s: Sub, interface: str = "robin", R0: float = 0.3,
                 power: int = 2) -> np.ndarray:
    """The 27 coefficients of the rows of B_j for subdomain ``s``."""
    if interface == "robin":
        return op.row_coeffs(F, s.lo, s.hi, restrict=True)
    if interface != "pml":
        raise ValueError(interface)
    n = (F.nx, F.ny, F.nz)
    prof = tuple(op.interface_pml_profile(F.prof[a], n[a], s.lo[a], s.hi[a], s.olo[a],
                                          s.ohi[a], F.h, F.omega, F.c_ref, R0, power)
                 for a in range(3))
    C = op.row_coeffs(dataclasses.replace(F, prof=prof), s.lo, s.hi, restrict=False)
    # Dirichlet truncation at the box: drop couplings to nodes outside it
    bz, by, bx = C.shape[1:]
    kk, jj, ii = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    for ei, (ex, ey, ez) in enumerate(op.OFFSETS):
        out = ((ii + ex < 0) | (ii + ex >= bx) | (jj + ey < 0) | (jj + ey >= by)
               | (kk + ez < 0) | (kk + ez >= bz))
        C[ei][out] = 0.0
    return C


class ORAS:
    def __init__(self, F: op.Fields, parts, overlap, interface: str = "robin",
                 R0: float = 0.3, power: int = 2):
        self.F = F
        self.interface, self.R0, self.power = interface, R0, power
        self.subs = partition((F.nx, F.ny, F.nz), parts, overlap)
        self.lus = []
        for s in self.subs:
            B = op.csr_from_coeffs(local_coeffs(F, s, interface, R0, power))
            self.lus.append(spla.splu(B.tocsc()))

    def local_matrix(self, j):
        s = self.subs[j]
        return op.csr_from_coeffs(local_coeffs(self.F, s, self.interface, self.R0, self.power))

    def apply(self, v: np.ndarray) -> np.ndarray:
        """M^{-1} v for v shaped (nz, ny, nx) or (s, nz, ny, nx)."""
        single = v.ndim == 3
        V = v[None] if single else v
        out = np.zeros_like(V, dtype=np.complex128)
        for s, lu in zip(self.subs, self.lus):
            box = (slice(s.lo[2], s.hi[2]), slice(s.lo[1], s.hi[1]), slice(s.lo[0], s.hi[0]))
            bshape = tuple(s.hi[a] - s.lo[a] for a in (2, 1, 0))
            r = V[(slice(None),) + box].reshape(V.shape[0], -1).T
            y = lu.solve(np.ascontiguousarray(r)).T.reshape((V.shape[0],) + bshape)
            own = tuple(slice(s.olo[a] - s.lo[a], s.ohi[a] - s.lo[a]) for a in (2, 1, 0))
            dst = (slice(None),) + tuple(slice(s.olo[a], s.ohi[a]) for a in (2, 1, 0))
            out[dst] = y[(slice(None),) + own]
        return out[0] if single else out
