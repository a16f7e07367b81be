"""Pins of the oracle's wavefield error measure Err (eq. eqerror): l1 norms of
the real and imaginary misfits, each relative to the reference's, under a
linear gain with distance from the source and a mute near it."""
import numpy as np

from oracle import metrics


def _field(seed=3, shape=(9, 10, 11)):
    rng = np.random.default_rng(seed)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


SRC, H = (5, 4, 4), 10.0        # (x, y, z) node of the source, grid step


def test_closed_forms():
    u = _field()
    assert metrics.err(u, u, SRC, H) == 0.0
    # both terms equal one when the field is missing entirely
    assert abs(metrics.err(u, np.zeros_like(u), SRC, H) - 2.0) < 1e-14
    # a real scaling (1 + t) misfits both parts by |t|
    for t in (0.5, -0.25, 2.0):
        assert abs(metrics.err(u, (1 + t) * u, SRC, H) - 2 * abs(t)) < 1e-13
    # a change of the imaginary part alone leaves the real term at zero
    for t in (0.3, -1.5):
        assert abs(metrics.err(u, u + 1j * t * u.imag, SRC, H) - abs(t)) < 1e-13
        assert abs(metrics.err(u, u + t * u.real, SRC, H) - abs(t)) < 1e-13


def test_mute_and_linear_gain():
    u = _field(4)
    x0, y0, z0 = SRC
    # a change within 4 grid steps of the source is muted
    v = u.copy()
    v[z0, y0, x0] += 10.0
    v[z0, y0, x0 + 3] += 10.0
    v[z0 + 2, y0 + 2, x0 + 2] += 10.0          # r = sqrt(12) h < 4 h
    assert metrics.err(u, v, SRC, H) == 0.0
    v[z0, y0, x0 + 4] += 1e-3                  # r = 4 h: counted
    assert metrics.err(u, v, SRC, H) > 0.0
    # equal changes at 4 h and 5 h: Err grows with the distance, linearly
    a, b = u.copy(), u.copy()
    a[z0, y0, x0 + 4] += 0.1
    b[z0, y0, x0 + 5] += 0.1
    e4, e5 = metrics.err(u, a, SRC, H), metrics.err(u, b, SRC, H)
    assert abs(e5 / e4 - 5.0 / 4.0) < 1e-12
    # the gain is the distance in metres, also off the axes (3-4-0 triangle)
    c = u.copy()
    c[z0, y0 + 4, x0 + 3] += 0.1                # r = 5 h
    assert abs(metrics.err(u, c, SRC, H) / e5 - 1.0) < 1e-12
    # a region mask drops what lies outside it
    reg = np.ones(u.shape)
    reg[z0, y0, x0 + 5] = 0.0
    assert metrics.err(u, b, SRC, H, region=reg) == 0.0
