"""Pins of the oracle's adjoint gradient (the FWI use of the forward engine,
paper sec. 1 and sec. 4)."""
import numpy as np

from oracle import adjoint, direct, operator as op, stencil_table as st
from paper_2110_15113_amd import workloads as wl


def _setup(q=None, seed=21):
    w = wl.small_random((9, 8, 10), npml=2, q=q, nsrc=2, seed=seed)
    rec = [(3, 3, 3), (5, 4, 3), (6, 5, 6), (3, 5, 7)]
    m0 = 1.0 / w.vel ** 2
    return w, rec, m0


def _J(w, rec, m, d_obs):
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml, weights_from=w.vel, m=m,
                       c_ref=float(w.vel.max()))
    A = op.assemble(F)
    J, g, U, MU = adjoint.misfit_and_gradient(F, w.sources, rec, d_obs,
                                              lambda b: direct.solve(A, F.shape, b))
    return J, g


def test_gradient_matches_finite_differences():
    for q in (None, 40.0):
        w, rec, m0 = _setup(q)
        rng = np.random.default_rng(1)
        d_obs = rng.normal(size=(2, len(rec))) * 1e-5 + 1j * rng.normal(size=(2, len(rec))) * 1e-5
        J0, g = _J(w, rec, m0, d_obs)
        for t in range(4):
            dm = rng.normal(size=m0.shape) * m0
            dm /= np.abs(dm).max()
            eps = 1e-4 * np.abs(m0).max()
            Jp, _ = _J(w, rec, m0 + eps * dm, d_obs)
            Jm, _ = _J(w, rec, m0 - eps * dm, d_obs)
            fd = (Jp - Jm) / (2 * eps)
            an = float(np.sum(g * dm))
            assert abs(fd - an) <= 1e-6 * abs(fd), (q, t, fd, an)


def test_adjoint_identity():
    """<P A^{-1} b, g> = <b, A^{-H} P^T g> with A^{-H} v = conj(A^{-1} conj(v))."""
    w, rec, m0 = _setup(60.0)
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml)
    A = op.assemble(F)
    rng = np.random.default_rng(3)
    b = rng.normal(size=(1,) + F.shape) + 1j * rng.normal(size=(1,) + F.shape)
    g = rng.normal(size=(1, len(rec))) + 1j * rng.normal(size=(1, len(rec)))
    lhs = np.vdot(g, adjoint.sample(direct.solve(A, F.shape, b), rec))
    mu = np.conj(direct.solve(A, F.shape, np.conj(adjoint.spread(g, rec, F.shape))))
    rhs = np.vdot(mu, b)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_lumped_mass_reduces_to_pointwise_product():
    """With wm0 = 1 (no off-diagonal mass) the gradient is
    -omega^2 Re(q S sum_s conj(mu) u) per cell."""
    w, rec, m0 = _setup(30.0)
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml)
    F.w[..., 3] = 1.0
    F.w[..., 4:] = 0.0
    rng = np.random.default_rng(5)
    U = rng.normal(size=(2,) + F.shape) + 1j * rng.normal(size=(2,) + F.shape)
    MU = rng.normal(size=(2,) + F.shape) + 1j * rng.normal(size=(2,) + F.shape)
    g = adjoint.gradient(F, U, MU)
    ref = -np.real(F.omega ** 2 * F.qfac * F.S() * np.sum(np.conj(MU) * U, axis=0))
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


def test_sample_spread_are_transposes():
    rec = [(1, 2, 3), (4, 0, 2), (1, 2, 3)]
    rng = np.random.default_rng(0)
    U = rng.normal(size=(2, 5, 6, 7)) + 1j * rng.normal(size=(2, 5, 6, 7))
    G = rng.normal(size=(2, 3)) + 1j * rng.normal(size=(2, 3))
    assert abs(np.vdot(G, adjoint.sample(U, rec)) - np.vdot(adjoint.spread(G, rec, (5, 6, 7)), U)) < 1e-12


def _mu_A_u(F, U, MU):
    A = op.assemble(F)
    return sum(np.vdot(MU[s].ravel(), A @ U[s].ravel()) for s in range(U.shape[0]))


def test_weight_sensitivity_matches_assembly_derivative():
    """A is linear in every stencil weight of every node, so a central
    difference of mu^H A(w) u in one weight is exact up to rounding; nodes on
    the grid boundary check the ghost-clamp distribution."""
    import dataclasses
    w = wl.small_random((7, 6, 8), npml=2, q=30.0, seed=5)
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml)
    rng = np.random.default_rng(4)
    U = rng.normal(size=(2,) + F.shape) + 1j * rng.normal(size=(2,) + F.shape)
    MU = rng.normal(size=(2,) + F.shape) + 1j * rng.normal(size=(2,) + F.shape)
    H = adjoint.weight_sensitivity(F, U, MU)
    nodes = [(0, 0, 0), (3, 2, 4), (6, 5, 7), (0, 3, 5), (5, 0, 2)]
    for (i, j, k) in nodes:
        for kk in range(7):
            eps = 1e-3
            wp = F.w.copy()
            wm = F.w.copy()
            wp[k, j, i, kk] += eps
            wm[k, j, i, kk] -= eps
            fd = (_mu_A_u(dataclasses.replace(F, w=wp), U, MU)
                  - _mu_A_u(dataclasses.replace(F, w=wm), U, MU)) / (2 * eps)
            assert abs(fd - H[k, j, i, kk]) <= 1e-9 * max(abs(fd), 1e-30) + 1e-12 * np.abs(H).max(), \
                ((i, j, k), kk, fd, H[k, j, i, kk])


def test_table_slope_matches_lookup_differences():
    G = np.array([3.1, 5.1, 9.37, 17.1, 31.8, 47.9])   # inside segments (knots every 0.25)
    s = st.lookup_slope(G)
    for d in (1e-7,):
        fd = (st.lookup(G + d) - st.lookup(G - d)) / (2 * d)
        assert np.abs(fd - s).max() <= 1e-6 * np.abs(s).max()
    assert np.all(st.lookup_slope(np.array([2.0, 50.0])) == 0.0)   # clamped outside the table


def _J_follow(w, rec, m, d_obs, cref):
    F = adjoint.fields_from_m(m, w.Q, w.omega, w.h, w.npml, cref)
    A = op.assemble(F)
    J, g_frozen, U, MU = adjoint.misfit_and_gradient(F, w.sources, rec, d_obs,
                                                     lambda b: direct.solve(A, F.shape, b))
    return J, adjoint.gradient_exact(F, U, MU, m), g_frozen


def test_exact_gradient_matches_finite_differences():
    """Weights following m (the lambda-adaptive stencil picks them from the
    local G, sec. 2.3): the exact gradient against central differences of
    the misfit, which the frozen-weight gradient misses.  The weights are
    piecewise linear in G, so the directions move only nodes whose G lies
    inside a table segment away from its knots: J is smooth along them."""
    for q in (None, 40.0):
        w, rec, m0 = _setup(q)
        cref = float(w.vel.max())
        rng = np.random.default_rng(11)
        d_obs = rng.normal(size=(2, len(rec))) * 1e-5 + 1j * rng.normal(size=(2, len(rec))) * 1e-5
        J0, g, g_frozen = _J_follow(w, rec, m0, d_obs, cref)
        G = 2 * np.pi / (w.omega * w.h * np.sqrt(m0))
        frac = np.modf((G - st.G_MIN) / st.G_STEP)[0]
        smooth = (frac > 0.1) & (frac < 0.9)
        assert smooth.mean() > 0.5
        frozen_err = 0.0
        for t in range(4):
            dm = rng.normal(size=m0.shape) * m0 * smooth
            dm /= np.abs(dm).max()
            eps = 1e-4 * np.abs(m0).max()
            Jp = _J_follow(w, rec, m0 + eps * dm, d_obs, cref)[0]
            Jm = _J_follow(w, rec, m0 - eps * dm, d_obs, cref)[0]
            fd = (Jp - Jm) / (2 * eps)
            an = float(np.sum(g * dm))
            assert abs(fd - an) <= 1e-6 * abs(fd), (q, t, fd, an)
            frozen_err = max(frozen_err, abs(fd - float(np.sum(g_frozen * dm))) / abs(fd))
        assert frozen_err > 1e-3, frozen_err
