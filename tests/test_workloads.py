"""The seeded synthetic workloads are deterministic and shaped as stated."""
import numpy as np

from paper_2110_15113_amd import workloads as wl


def test_config1_exact():
    c = wl.config1()
    assert c.vel.shape == (32, 32, 32)
    assert c.vel[0].min() == 1500.0 and c.vel[-1].max() == 3000.0
    assert c.sources == [(16, 16, 16)] and c.Q is None


def test_generators_deterministic_and_in_range():
    for k in (2, 3, 4, 5):
        a = wl.CONFIGS[k]()
        b = wl.CONFIGS[k]()
        assert a.digest() == b.digest()
        assert a.vel.shape == (a.nz, a.ny, a.nx)
        assert np.isfinite(a.vel).all() and a.vel.min() >= 1500.0 - 1e-9
        for (i, j, kk) in a.sources:
            assert a.npml <= i < a.nx - a.npml and a.npml <= j < a.ny - a.npml
            assert a.npml <= kk < a.nz - a.npml
    c3 = wl.config3()
    assert set(np.unique(c3.vel)) <= {1500.0 + 700 * l for l in range(6)}
    assert len(c3.sources) == 64
    c4 = wl.config4()
    assert len(c4.receivers) == 400 and len(c4.sources) == 32
    assert abs(c4.vel / 2500.0 - 1).max() <= 0.2
