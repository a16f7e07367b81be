"""The FWI update loop (paper sec. 1 and sec. 4: inversion needs the incident
and adjoint wavefields of all sources at every model update): its L-BFGS
recursion against the explicit BFGS inverse-Hessian update, convergence on
quadratics with and without active bounds, and monotone misfit decrease on a
small inversion driven by the oracle's direct solves and exact gradient."""
import numpy as np
import torch

from oracle import adjoint, direct, operator as op
from paper_2110_15113_amd import fwi, workloads as wl


def test_two_loop_equals_explicit_bfgs_update():
    rng = np.random.default_rng(0)
    n = 12
    Q = rng.normal(size=(n, n))
    A = Q @ Q.T + n * np.eye(n)
    S = [rng.normal(size=n) for _ in range(5)]
    Y = [A @ s for s in S]
    g = rng.normal(size=n)
    gamma = (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1])
    H = gamma * np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / (y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    got = fwi.two_loop(torch.tensor(g), [torch.tensor(s) for s in S],
                       [torch.tensor(y) for y in Y]).numpy()
    assert np.abs(got - H @ g).max() <= 1e-12 * np.abs(H @ g).max()
    # no pairs: the identity
    assert torch.equal(fwi.two_loop(torch.tensor(g), [], []), torch.tensor(g))


def _quadratic(n=30, seed=1):
    rng = np.random.default_rng(seed)
    Q = rng.normal(size=(n, n))
    A = torch.tensor(Q @ Q.T / n + np.diag(np.linspace(0.5, 5.0, n)))
    b = torch.tensor(rng.normal(size=n))

    def f(x):
        return float(0.5 * x @ (A @ x) - b @ x), A @ x - b
    return A, b, f


def test_converges_on_a_convex_quadratic():
    A, b, f = _quadratic()
    x_star = torch.linalg.solve(A, b)
    res = fwi.lbfgs(f, torch.zeros_like(b) + 1.0, 60, memory=8, first_step=0.5)
    Js = [h["J"] for h in res.history]
    assert all(Js[i + 1] <= Js[i] for i in range(len(Js) - 1))
    assert float((res.m - x_star).abs().max()) < 1e-6


def test_bounds_are_respected_and_the_projected_minimum_is_reached():
    A, b, f = _quadratic(n=10, seed=3)
    lo, hi = -0.1, 0.1
    res = fwi.lbfgs(f, torch.zeros_like(b), 200, m_min=lo, m_max=hi, memory=5, first_step=1.0)
    m = res.m
    assert float(m.min()) >= lo and float(m.max()) <= hi
    # projected-gradient stationarity: no feasible descent left (to the tolerance
    # a first-order method reaches)
    g = A @ m - b
    pg = m - torch.clamp(m - g, lo, hi)
    assert float(pg.abs().max()) < 1e-4
    Js = [h["J"] for h in res.history]
    assert all(Js[i + 1] <= Js[i] for i in range(len(Js) - 1))


def test_mask_freezes_the_masked_entries():
    A, b, f = _quadratic(n=8, seed=5)
    mask = torch.tensor([1.0, 0, 1, 1, 0, 1, 1, 1], dtype=torch.float64)
    x0 = torch.full_like(b, 0.3)
    res = fwi.lbfgs(f, x0, 10, mask=mask)
    assert torch.equal(res.m[mask == 0], x0[mask == 0])


def test_small_inversion_with_oracle_solves_decreases_the_misfit():
    w = wl.small_random((10, 9, 10), npml=2, q=None, nsrc=3, seed=51)
    rec = [(3, 3, 3), (6, 3, 3), (3, 6, 3), (6, 6, 3), (4, 4, 7), (6, 5, 7)]
    m_true = 1.0 / w.vel ** 2
    m0 = np.full_like(m_true, float(np.mean(m_true)))
    cref = float(w.vel.max())

    def solve_fields(m):
        F = adjoint.fields_from_m(m, w.Q, w.omega, w.h, w.npml, cref)
        A = op.assemble(F)
        return F, (lambda b: direct.solve(A, F.shape, b))

    F, solve = solve_fields(m_true)
    d_obs = adjoint.sample(solve(op.point_sources(F, w.sources)), rec)

    def objective(mt):
        m = mt.numpy()
        F, solve = solve_fields(m)
        J, _, U, MU = adjoint.misfit_and_gradient(F, w.sources, rec, d_obs, solve)
        return J, torch.tensor(adjoint.gradient_exact(F, U, MU, m))

    res = fwi.lbfgs(objective, torch.tensor(m0), 4, m_min=1 / 3500.0 ** 2, m_max=1 / 1400.0 ** 2)
    Js = [h["J"] for h in res.history] + [res.history[-1]["J_new"]]
    assert all(h["accepted"] for h in res.history)
    assert all(Js[i + 1] < Js[i] for i in range(len(Js) - 1))
    assert Js[-1] < 0.5 * Js[0]
