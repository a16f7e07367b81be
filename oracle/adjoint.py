"""Receiver sampling, adjoint solve and misfit gradient (oracle side).
TEST INFRASTRUCTURE.

The paper motivates the solver as the forward engine of frequency-domain FWI
(sec. 1 and sec. 4: incident and adjoint wavefields are kept in memory, and
the Helmholtz operator is complex symmetric, so A^H = conj(A)).  For the
least-squares misfit J = 1/2 sum_{s,r} |P u_s - d_obs|^2 with A(m) u_s = b_s:

    rho_s = P u_s - d_obs                    (torch's grad of J w.r.t. d)
    A^H mu_s = P^T rho_s   <=>   A conj(mu_s) = conj(P^T rho_s)
    dJ/dm_i = -Re sum_s mu_s^H (dA/dm_i) u_s

gradient(): the stencil weights are frozen at assemble time (they depend on
the start model through G, a reading that excludes the table derivative), and
the PML is independent of m (c_ref frozen), so only the mass term depends on m:
m~_i = m_i q_i with q_i = (1 + i/(2Q_i))^2 and

    mu^H (dA/dm_i) u = omega^2 q_i [ wm0_i S_i conj(mu_i) u_i
        + sum_{j ~ i} 1/2 mhat_ij ( conj(mu_i) u_j + conj(mu_j) u_i ) ],
    mhat_ij = 1/2 (wm_t,i + wm_t,j) * 1/2 (S_i + S_j).

gradient_exact(): the weights follow m through G = 2 pi / (omega h sqrt(m))
and the piecewise-linear table (sec. 2.3), adding
-Re sum_k H_k,i dw_k/dG dG/dm_i, with H_k,i = sum_s d(mu_s^H A u_s)/dw_k,i
from weight_sensitivity().

Parity: pinned in tests by central finite differences of J (direct solves at
machine precision; frozen and following weights), the adjoint identity
<P A^{-1} b, g> = <b, A^{-H} P^T g>, the lumped-mass special case (wm0 = 1)
reducing to -omega^2 Re(q conj(mu) u S), exact central differences of
mu^H A(w) u in single weights (A is linear in each weight), and the table
slope against differences of the lookup.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import operator as op
from . import stencil_table as st


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


def weight_sensitivity(F: op.Fields, U: np.ndarray, MU: np.ndarray) -> np.ndarray:
    """H[..., k] = sum_s d(mu_s^H A u_s) / d w_k at every node, for the seven
    stencil weights w1 w2 w3 wm0 wmf wme wmc (the reading of the operator in
    oracle.operator: a staggered point's family weight is the mean of its
    support nodes' weights, a ghost support node taking the weights of the
    grid node it clamps to; the mass coupling uses the mean of the two
    nodes' shell weights).  U, MU: (s, nz, ny, nx)."""
    nz, ny, nx = F.shape
    n = (nx, ny, nz)
    ns = U.shape[0]
    h2 = F.h * F.h
    H = np.zeros((nz, ny, nx, 7), dtype=np.complex128)
    # zero-padded fields: ghost nodes carry u = mu = 0
    Up = np.zeros((ns, nz + 2, ny + 2, nx + 2), dtype=np.complex128)
    Mp = np.zeros_like(Up)
    Up[:, 1:-1, 1:-1, 1:-1] = U
    Mp[:, 1:-1, 1:-1, 1:-1] = MU
    sx, sy, sz = F.prof
    prof = (sx, sy, sz)
    # stiffness: staggered point with base node b (b_a in [-1, n_a - 1] on the
    # family axes, [0, n_a - 1] otherwise) and support nodes b + rho
    for axes, widx, ffac in op.FAMILIES:
        dim = len(axes)
        dscale = 1.0 / 2 ** (dim - 1)
        base = [np.arange(-1, n[a]) if a in axes else np.arange(n[a]) for a in range(3)]
        tcen = [2 * base[a] + 2 if a in axes else 2 * base[a] + 1 for a in range(3)]
        sc = [prof[a][tcen[a]] for a in range(3)]
        scz, scy, scx = sc[2][:, None, None], sc[1][None, :, None], sc[0][None, None, :]
        Scen = scz * scy * scx
        svals = {0: scx, 1: scy, 2: scz}
        rhos = list(itertools.product((0, 1), repeat=dim))

        def padded_slice(rho):
            off = [0, 0, 0]
            for q, a in enumerate(axes):
                off[a] = rho[q]
            # padded index of node b + off is b + off + 1
            return tuple(slice(base[a][0] + off[a] + 1, base[a][-1] + off[a] + 2) for a in (2, 1, 0))

        T = np.zeros(Scen.shape, dtype=np.complex128)
        for q, a in enumerate(axes):
            Dm = 0.0
            Du = 0.0
            for rho in rhos:
                d = (2 * rho[q] - 1) * dscale
                sl = (slice(None),) + padded_slice(rho)
                Dm = Dm + d * Mp[sl]
                Du = Du + d * Up[sl]
            T = T - ffac * Scen / (svals[a] ** 2) / h2 * np.sum(np.conj(Dm) * Du, axis=0)
        # distribute dT/dwbar = T over the support (mean weight), clamping ghosts
        for rho in rhos:
            idx = []
            for a in range(3):
                qa = axes.index(a) if a in axes else None
                o = rho[qa] if qa is not None else 0
                idx.append(np.clip(base[a] + o, 0, n[a] - 1))
            iz, iy, ix = np.ix_(idx[2], idx[1], idx[0])
            np.add.at(H[..., widx], (iz, iy, ix), T / len(rhos))
    # consistent mass
    S = F.S()
    om2 = F.omega ** 2
    H[..., 3] += om2 * F.mt * S * np.sum(np.conj(MU) * U, axis=0)
    mtp = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.complex128)
    Sp = np.zeros_like(mtp)
    mtp[1:-1, 1:-1, 1:-1] = F.mt
    Sp[1:-1, 1:-1, 1:-1] = S
    for (ex, ey, ez) in op.OFFSETS:
        if (ex, ey, ez) == (0, 0, 0):
            continue
        t = 3 + abs(ex) + abs(ey) + abs(ez)
        js = (slice(1 + ez, nz + 1 + ez), slice(1 + ey, ny + 1 + ey), slice(1 + ex, nx + 1 + ex))
        # d/dwm_t,i of the couplings (i, j) and (j, i); ghost j carries u = mu = 0
        coup = 0.5 * 0.5 * (F.mt + mtp[js]) * 0.5 * (S + Sp[js])
        term = np.sum(np.conj(MU) * Up[(slice(None),) + js] + np.conj(Mp[(slice(None),) + js]) * U, axis=0)
        H[..., t] += om2 * coup * term
    return H


def fields_from_m(m, Q, omega, h, npml, c_ref, **kw) -> op.Fields:
    """Operator fields with both the stencil weights and the mass following
    the squared slowness m (velocity 1/sqrt(m)); the PML's c_ref is fixed."""
    return op.make_fields(1.0 / np.sqrt(np.asarray(m, dtype=np.float64)), Q, omega, h, npml,
                          c_ref=c_ref, **kw)


def gradient_exact(F: op.Fields, U: np.ndarray, MU: np.ndarray, m: np.ndarray,
                   tab: np.ndarray | None = None) -> np.ndarray:
    """-Re sum_s mu_s^H (dA/dm) u_s with the stencil weights following m
    through G = 2 pi c / (omega h), c = 1 / sqrt(m) (sec. 2.3: the weights are
    picked per node from its local G): the frozen-weight gradient plus
    -Re sum_k H_k dw_k/dG dG/dm, dG/dm = -G / (2 m), dw/dG the table slope."""
    m = np.asarray(m, dtype=np.float64)
    G = 2.0 * np.pi / (F.omega * F.h * np.sqrt(m))
    dw = st.lookup_slope(G, tab) * (-G / (2.0 * m))[..., None]
    H = weight_sensitivity(F, U, MU)
    return gradient(F, U, MU) - np.real(np.sum(H * dw, axis=-1))


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
