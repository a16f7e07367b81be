"""The differentiable forward map against the oracle's adjoint gradient and
finite differences."""
import numpy as np
import pytest
import torch

from oracle import adjoint, direct, operator as op, stencil_table as st
from paper_2110_15113_amd import workloads as wl

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _setup(w, rec, parts, tol, prec=2, budget=32e9):
    from paper_2110_15113_amd import oras
    from paper_2110_15113_amd.autograd import ForwardSetup
    S = oras.Solver(0)
    vel = torch.as_tensor(w.vel, device=S.device)
    Q = None if w.Q is None else torch.as_tensor(w.Q, device=S.device)
    S.assemble(vel, w.h, w.npml, w.omega, Q, prec=prec)   # freezes weights at this model
    return ForwardSetup(S, w.sources, rec, parts, w.overlap, prec, tol, save_budget_bytes=budget)


def _oracle_J_grad(w, rec, m, d_obs):
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml, weights_from=w.vel, m=m)
    A = op.assemble(F)
    J, g, _, _ = adjoint.misfit_and_gradient(F, w.sources, rec, d_obs,
                                             lambda b: direct.solve(A, F.shape, b))
    return J, g


def test_gradient_matches_oracle_and_recompute_policy():
    need_gpu()
    from paper_2110_15113_amd.autograd import receiver_data
    w = wl.small_random((12, 11, 10), npml=2, q=60.0, nsrc=3, seed=31, parts=(2, 2, 2))
    rec = [(3, 3, 3), (6, 4, 3), (8, 7, 5), (4, 8, 6), (6, 5, 7)]
    say("autograd vs oracle")
    rng = np.random.default_rng(2)
    m_np = (1.0 / w.vel ** 2) * (1 + 0.05 * rng.standard_normal(w.vel.shape))
    d_obs = (rng.normal(size=(3, len(rec))) + 1j * rng.normal(size=(3, len(rec)))) * 1e-5
    J_ref, g_ref = _oracle_J_grad(w, rec, m_np, d_obs)
    for budget in (32e9, 0.0):
        fs = _setup(w, rec, (2, 2, 2), 1e-11, budget=budget)
        m = torch.tensor(m_np, device=fs.solver.device, requires_grad=True)
        d = receiver_data(m, fs)
        J = 0.5 * (d - torch.as_tensor(d_obs, device=d.device)).abs().pow(2).sum()
        J.backward()
        assert abs(J.item() - J_ref) <= 1e-8 * J_ref
        g = m.grad.cpu().numpy()
        assert np.abs(g - g_ref).max() <= 1e-6 * np.abs(g_ref).max(), budget


def test_gradcheck_tiny_grid():
    need_gpu()
    from paper_2110_15113_amd.autograd import receiver_data
    w = wl.small_random((7, 6, 6), npml=1, q=50.0, nsrc=2, seed=33)
    rec = [(2, 2, 2), (4, 3, 3), (3, 4, 2)]
    fs = _setup(w, rec, (1, 1, 1), 1e-13)
    m0 = torch.as_tensor(1.0 / w.vel ** 2, device=fs.solver.device)
    with torch.no_grad():
        d0 = receiver_data(m0.clone(), fs)
    scale = d0.abs().max()

    def f(p):
        return receiver_data(m0 * p, fs) / scale

    p = torch.ones_like(m0, requires_grad=True)
    assert torch.autograd.gradcheck(f, (p,), eps=1e-6, atol=1e-6, rtol=1e-4, fast_mode=False)


def test_finite_differences_random_directions():
    need_gpu()
    from paper_2110_15113_amd.autograd import receiver_data
    w = wl.small_random((16, 15, 14), npml=3, q=None, nsrc=4, seed=35, parts=(2, 2, 2))
    rec = [(5, 5, 5), (8, 6, 5), (10, 9, 7), (6, 10, 9)]
    fs = _setup(w, rec, (2, 2, 2), 1e-12)
    dev = fs.solver.device
    rng = np.random.default_rng(4)
    m0 = torch.as_tensor(1.0 / w.vel ** 2, device=dev)
    d_obs = torch.as_tensor((rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))) * 1e-5,
                            device=dev)

    def J(m):
        return 0.5 * (receiver_data(m, fs) - d_obs).abs().pow(2).sum()

    m = m0.clone().requires_grad_(True)
    J(m).backward()
    g = m.grad.clone()
    for t in range(4):
        dm = torch.as_tensor(rng.standard_normal(w.vel.shape), device=dev)
        dm = dm / dm.abs().max() * m0
        eps = 1e-4
        with torch.no_grad():
            fd = (J(m0 + eps * dm) - J(m0 - eps * dm)) / (2 * eps)
        an = (g * dm).sum()
        assert abs(fd - an) <= 1e-5 * abs(fd), (t, float(fd), float(an))


def test_exact_weights_gradient_matches_oracle_and_differences():
    """weights='follow': the forward picks the stencil weights from G(m) at
    every model (sec. 2.3) and the backward adds their table-slope term; the
    gradient matches the oracle's exact gradient and central differences."""
    need_gpu()
    from paper_2110_15113_amd.autograd import receiver_data
    w = wl.small_random((14, 12, 11), npml=2, q=50.0, nsrc=3, seed=37, parts=(2, 2, 1))
    rec = [(4, 4, 3), (7, 5, 4), (9, 8, 6), (5, 9, 7)]
    say("autograd exact weights")
    rng = np.random.default_rng(8)
    m_np = (1.0 / w.vel ** 2) * (1 + 0.05 * rng.standard_normal(w.vel.shape))
    d_obs = (rng.normal(size=(3, len(rec))) + 1j * rng.normal(size=(3, len(rec)))) * 1e-5
    F = adjoint.fields_from_m(m_np, w.Q, w.omega, w.h, w.npml, float(w.vel.max()))
    A = op.assemble(F)
    J_ref, _, U, MU = adjoint.misfit_and_gradient(F, w.sources, rec, d_obs,
                                                  lambda b: direct.solve(A, F.shape, b))
    g_ref = adjoint.gradient_exact(F, U, MU, m_np)
    fs = _setup(w, rec, (2, 2, 1), 1e-12)
    fs.weights = "follow"
    dev = fs.solver.device
    d_obs_t = torch.as_tensor(d_obs, device=dev)

    def J(m):
        return 0.5 * (receiver_data(m, fs) - d_obs_t).abs().pow(2).sum()

    m = torch.tensor(m_np, device=dev, requires_grad=True)
    Jv = J(m)
    Jv.backward()
    assert abs(Jv.item() - J_ref) <= 1e-8 * J_ref
    g = m.grad.cpu().numpy()
    assert np.abs(g - g_ref).max() <= 1e-6 * np.abs(g_ref).max()
    m0 = torch.as_tensor(m_np, device=dev)
    # the weights are piecewise linear in G: directions move only nodes whose
    # G lies inside a table segment, away from its knots, so J is smooth along
    # them and central differences are second-order accurate
    G = 2 * np.pi / (w.omega * w.h * np.sqrt(m_np))
    frac = np.modf((G - st.G_MIN) / st.G_STEP)[0]
    smooth = torch.as_tensor(((frac > 0.1) & (frac < 0.9)).astype(np.float64), device=dev)
    for t in range(3):
        dm = torch.as_tensor(rng.standard_normal(w.vel.shape), device=dev)
        dm = dm / dm.abs().max() * m0 * smooth
        eps = 1e-4
        with torch.no_grad():
            fd = (J(m0 + eps * dm) - J(m0 - eps * dm)) / (2 * eps)
        an = (m.grad * dm).sum()
        assert abs(fd - an) <= 1e-5 * abs(fd), (t, float(fd), float(an))


def test_blr_preconditioner_leaves_the_gradient_unchanged():
    """BLR plane inverses change only the preconditioner: with solves to
    1e-12 the data and the exact gradient agree with the dense factors'."""
    need_gpu()
    from paper_2110_15113_amd.autograd import receiver_data
    w = wl.small_random((18, 17, 16), npml=2, q=60.0, nsrc=3, seed=39, parts=(2, 2, 2))
    rec = [(5, 5, 4), (9, 6, 5), (12, 11, 8), (7, 12, 10)]
    say("autograd with BLR plane inverses")
    rng = np.random.default_rng(12)
    m_np = (1.0 / w.vel ** 2) * (1 + 0.05 * rng.standard_normal(w.vel.shape))
    d_obs = (rng.normal(size=(3, len(rec))) + 1j * rng.normal(size=(3, len(rec)))) * 1e-5
    out = []
    for blr in (None, 1e-3):
        fs = _setup(w, rec, (2, 2, 2), 1e-12)
        fs.weights = "follow"
        fs.blr_eps = blr
        m = torch.tensor(m_np, device=fs.solver.device, requires_grad=True)
        d = receiver_data(m, fs)
        J = 0.5 * (d - torch.as_tensor(d_obs, device=d.device)).abs().pow(2).sum()
        J.backward()
        out.append((J.item(), m.grad.cpu().numpy()))
    assert abs(out[1][0] - out[0][0]) <= 1e-9 * out[0][0]
    assert np.abs(out[1][1] - out[0][1]).max() <= 1e-7 * np.abs(out[0][1]).max()
