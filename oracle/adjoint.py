"""Receiver sampling, adjoint solve and misfit gradient (oracle side).
TEST INFRASTRUCTURE.

The paper motivates the solver as the forward engine of frequency-domain FWI
(sec. 1 and sec. 4: incident and adjoint wavefields are kept in memory, and
the Helmholtz operator is complex symmetric, so A^H = conj(A)).  For the
least-squares misfit J = 1/2 sum_{s,r} |P u_s - d_obs|^2 with A(m) u_s = b_s:

    rho_s = P u_s - d_obs                    (torch's grad of J w.r.t. d)
    A^H mu_s = P^T rho_s   <=>   A conj(mu_s) = conj(P^T rho_s)
    dJ/dm_i = -Re sum_s mu_s^H (dA/dm_i) u_s

The stencil weights are frozen at assemble time (they depend on the start
model through G, a reading that excludes the table derivative), and the PML
is independent of m (c_ref frozen), so only the mass term depends on m:
m~_i = m_i q_i with q_i = (1 + i/(2Q_i))^2 and

    mu^H (dA/dm_i) u = omega^2 q_i [ wm0_i S_i conj(mu_i) u_i
        + sum_{j ~ i} 1/2 mhat_ij ( conj(mu_i) u_j + conj(mu_j) u_i ) ],
    mhat_ij = 1/2 (wm_t,i + wm_t,j) * 1/2 (S_i + S_j).

Parity: pinned in tests by central finite differences of J (direct solves at
machine precision), the adjoint identity <P A^{-1} b, g> = <b, A^{-H} P^T g>,
and the lumped-mass special case (wm0 = 1) reducing to
-omega^2 Re(q conj(mu) u S).
"""
from __future__ import annotations

import numpy as np

from . import operator as op


def sample(U: np.ndarray, receivers) -> np.ndarray:
    """d[s, r] = U[s, k_r, j_r, i_r]."""
    idx = np.array(receivers)
    return U[:, idx[:, 2], idx[:, 1], idx[:, 0]]


def spread(G: np.ndarray, receivers, shape) -> np.ndarray:
    """P^T g: (s, nrec) -> (s, nz, ny, nx), summing duplicates."""
    out = np.zeros((G.shape[0],) + tuple(shape), dtype=np.complex128)
    for r, (i, j, k) in enumerate(receivers):
        out[:, k, j, i] += G[:, r]
    return out


def gradient(F: op.Fields, U: np.ndarray, MU: np.ndarray) -> np.ndarray:
    """-Re sum_s mu_s^H (dA/dm) u_s for every node; U, MU (s, nz, ny, nx)."""
    nz, ny, nx = F.shape
    S = F.S()
    w = F.w
    acc = w[..., 3] * S * np.sum(np.conj(MU) * U, axis=0)
    Up = np.zeros((U.shape[0], nz + 2, ny + 2, nx + 2), dtype=np.complex128)
    Mp = np.zeros_like(Up)
    Up[:, 1:-1, 1:-1, 1:-1] = U
    Mp[:, 1:-1, 1:-1, 1:-1] = MU
    wp = np.zeros((nz + 2, ny + 2, nx + 2, 7))
    wp[1:-1, 1:-1, 1:-1] = w
    Sp = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.complex128)
    Sp[1:-1, 1:-1, 1:-1] = S
    inner = (slice(1, nz + 1), slice(1, ny + 1), slice(1, nx + 1))
    for (ex, ey, ez) in op.OFFSETS:
        if (ex, ey, ez) == (0, 0, 0):
            continue
        t = 3 + abs(ex) + abs(ey) + abs(ez)
        js = (slice(1 + ez, nz + 1 + ez), slice(1 + ey, ny + 1 + ey), slice(1 + ex, nx + 1 + ex))
        # ghost neighbours carry u = mu = 0, so their terms vanish
        mhat = 0.5 * (w[..., t] + wp[js][..., t]) * 0.5 * (S + Sp[js])
        term = np.sum(np.conj(MU) * Up[(slice(None),) + js] + np.conj(Mp[(slice(None),) + js]) * U, axis=0)
        acc = acc + 0.5 * mhat * term
    return -np.real(F.omega ** 2 * F.qfac * acc)


def misfit_and_gradient(F: op.Fields, sources, receivers, d_obs, solve):
    """J and dJ/dm with ``solve(b)`` returning A^{-1} b for a stack of RHS."""
    b = op.point_sources(F, sources)
    U = solve(b)
    d = sample(U, receivers)
    rho = d - d_obs
    J = 0.5 * float(np.sum(np.abs(rho) ** 2))
    rhs = np.conj(spread(rho, receivers, F.shape))
    MU = np.conj(solve(rhs))
    return J, gradient(F, U, MU), U, MU
