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
