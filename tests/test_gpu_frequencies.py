"""Several frequencies in flight on one GPU (one context and stream per
frequency, solves driven from concurrent host threads): each frequency's
result equals its solve run alone, and the oracle's direct solution."""
import numpy as np
import pytest
import torch

from oracle import direct, operator as op
from paper_2110_15113_amd import workloads as wl

from gpu_util import need_gpu, rel, say

pytestmark = pytest.mark.gpu


def test_concurrent_frequencies_match_sequential_and_oracle():
    need_gpu()
    from paper_2110_15113_amd import oras
    from paper_2110_15113_amd.frequencies import FrequencyBatch
    w = wl.small_random((20, 18, 16), npml=3, q=70.0, nsrc=3, seed=61, parts=(2, 2, 2))
    freqs = [4.0, 5.0, 6.5]
    omegas = [2 * np.pi * f for f in freqs]
    say("frequency batch")
    dev = torch.device("cuda", 0)
    vel = torch.as_tensor(w.vel, device=dev)
    Q = torch.as_tensor(w.Q, device=dev)
    fb = FrequencyBatch(vel, w.h, w.npml, omegas, Q=Q, prec=oras.C128)
    fb.factor(w.parts, w.overlap)
    bs = fb.point_sources(w.sources)
    seq = fb.solve(bs, 1e-10, restart=20, concurrent=False)
    xs = [r.x.clone() for r in seq]
    con = fb.solve(bs, 1e-10, restart=20, concurrent=True)
    for i, om in enumerate(omegas):
        assert bool(con[i].converged.all())
        assert torch.equal(con[i].x, xs[i]), i            # the same kernels, the same result
        assert np.array_equal(con[i].iters, seq[i].iters)
        F = op.make_fields(w.vel, w.Q, om, w.h, w.npml)
        b = op.point_sources(F, w.sources)
        u = direct.solve(op.assemble(F), F.shape, b)
        assert rel(con[i].x.cpu().numpy(), u) < 1e-7, (i, rel(con[i].x.cpu().numpy(), u))
    fb.close()
