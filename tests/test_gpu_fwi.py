"""The FWI update loop on the GPU map against the same loop driven by the
oracle's direct solves and exact gradient (same optimiser, same data)."""
import numpy as np
import pytest
import torch

from oracle import adjoint, direct, operator as op
from paper_2110_15113_amd import workloads as wl

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def test_fwi_loop_matches_oracle_driven_loop():
    need_gpu()
    from paper_2110_15113_amd import fwi, oras
    from paper_2110_15113_amd.autograd import ForwardSetup
    w = wl.small_random((12, 11, 12), npml=2, q=80.0, nsrc=3, seed=52, parts=(2, 2, 2))
    rec = [(3, 3, 3), (7, 3, 3), (3, 7, 3), (7, 7, 3), (5, 4, 8), (8, 6, 8)]
    say("fwi loop gpu vs oracle")
    m_true = 1.0 / w.vel ** 2
    m0 = np.full_like(m_true, float(np.mean(m_true)))
    cref = float(w.vel.max())
    bounds = dict(m_min=1 / 3500.0 ** 2, m_max=1 / 1400.0 ** 2)

    def oracle_solver(m):
        F = adjoint.fields_from_m(m, w.Q, w.omega, w.h, w.npml, cref)
        A = op.assemble(F)
        return F, (lambda b: direct.solve(A, F.shape, b))

    F, solve = oracle_solver(m_true)
    d_obs = adjoint.sample(solve(op.point_sources(F, w.sources)), rec)

    def oracle_objective(mt):
        m = mt.numpy()
        F, solve = oracle_solver(m)
        J, _, U, MU = adjoint.misfit_and_gradient(F, w.sources, rec, d_obs, solve)
        return J, torch.tensor(adjoint.gradient_exact(F, U, MU, m))

    ref = fwi.lbfgs(oracle_objective, torch.tensor(m0), 3, **bounds)

    S = oras.Solver(0)
    dev = S.device
    vel = torch.as_tensor(w.vel, device=dev)      # c_ref and Q from the true model's assembly
    S.assemble(vel, w.h, w.npml, w.omega, torch.as_tensor(w.Q, device=dev), prec=oras.C128)
    fs = ForwardSetup(S, w.sources, rec, w.parts, w.overlap, oras.C128, 1e-12, weights="follow")
    obj = fwi.gpu_objective(fs, torch.as_tensor(d_obs, device=dev))
    got = fwi.lbfgs(obj, torch.as_tensor(m0, device=dev), 3, **bounds)
    assert len(got.history) == len(ref.history) == 3
    for a, b in zip(got.history, ref.history):
        assert a["accepted"] and b["accepted"]
        assert abs(a["J"] - b["J"]) <= 1e-7 * b["J"], (a, b)
        assert a["evals"] == b["evals"]
    assert got.history[-1]["J_new"] < 0.5 * got.history[0]["J"]
    err = np.abs(got.m.cpu().numpy() - ref.m.numpy()).max() / np.abs(ref.m.numpy()).max()
    assert err < 1e-6, err


def test_multi_frequency_objective_matches_oracle_and_sequential():
    """Two frequencies in flight: misfit and exact gradient equal the sums of
    the oracle's single-frequency values, the concurrent evaluation equals the
    sequential one bitwise, and two L-BFGS updates lower the misfit."""
    need_gpu()
    from paper_2110_15113_amd import fwi, oras
    from paper_2110_15113_amd.frequencies import FrequencyBatch
    w = wl.small_random((14, 13, 12), npml=2, q=60.0, nsrc=3, seed=53, parts=(2, 2, 1))
    rec = [(3, 3, 3), (8, 4, 3), (4, 8, 4), (9, 9, 3), (6, 6, 8)]
    freqs = [4.0, 5.5]
    omegas = [2 * np.pi * f for f in freqs]
    say("multi-frequency objective")
    m_true = 1.0 / w.vel ** 2
    m0 = np.full_like(m_true, float(np.mean(m_true)))
    vel0 = 1.0 / np.sqrt(m0)
    cref = float(vel0.max())                          # the start model's assembly fixes c_ref
    d_obs, J_ref, g_ref = [], 0.0, 0.0
    for om in omegas:
        Ft = adjoint.fields_from_m(m_true, w.Q, om, w.h, w.npml, cref)
        dt = adjoint.sample(direct.solve(op.assemble(Ft), Ft.shape,
                                         op.point_sources(Ft, w.sources)), rec)
        d_obs.append(dt)
        F0 = adjoint.fields_from_m(m0, w.Q, om, w.h, w.npml, cref)
        A0 = op.assemble(F0)
        J, _, U, MU = adjoint.misfit_and_gradient(F0, w.sources, rec, dt,
                                                  lambda b: direct.solve(A0, F0.shape, b))
        J_ref += J
        g_ref = g_ref + adjoint.gradient_exact(F0, U, MU, m0)
    dev = torch.device("cuda", 0)
    fb = FrequencyBatch(torch.as_tensor(vel0, device=dev), w.h, w.npml, omegas,
                        Q=torch.as_tensor(w.Q, device=dev), prec=oras.C128)
    dobs_t = [torch.as_tensor(d, device=dev) for d in d_obs]
    obj = fwi.MultiFrequencyObjective(fb, w.sources, rec, dobs_t, w.parts, w.overlap, tol=1e-12)
    m0_t = torch.as_tensor(m0, device=dev)
    J, g = obj(m0_t)
    assert abs(J - J_ref) <= 1e-8 * J_ref
    assert np.abs(g.cpu().numpy() - g_ref).max() <= 1e-6 * np.abs(g_ref).max()
    obj.concurrent = False
    J2, g2 = obj(m0_t)
    assert J2 == J and torch.equal(g2, g)
    obj.concurrent = True
    res = fwi.lbfgs(obj, m0_t, 2, m_min=1 / 3500.0 ** 2, m_max=1 / 1400.0 ** 2)
    assert all(h["accepted"] for h in res.history)
    assert res.history[-1]["J_new"] < res.history[0]["J"]
    fb.close()
