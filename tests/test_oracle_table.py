"""Pins of the oracle's lambda-adaptive weight table (paper sec. 2.3, FDFD
discretisation and dispersion analysis)."""
import numpy as np

from oracle import stencil_table as st


def test_constraints_hold():
    tab = st.table()
    assert tab.shape == (st.G_COUNT, 7)
    assert np.allclose(tab[:, 0] + tab[:, 1] + tab[:, 2], 1.0, atol=1e-15, rtol=0)
    mass = tab[:, 3] + 6 * tab[:, 4] + 12 * tab[:, 5] + 8 * tab[:, 6]
    assert np.allclose(mass, 1.0, atol=1e-14, rtol=0)


def test_fit_is_stationary():
    """The stored weights satisfy the ridge normal equations, checked with
    finite differences of the objective written out independently."""
    dirs = st.directions()

    def objective(p, G):
        k = 2 * np.pi / G
        xi = k * dirs
        c = np.cos(xi)
        S1 = c.sum(1)
        S2 = c[:, 0] * c[:, 1] + c[:, 0] * c[:, 2] + c[:, 1] * c[:, 2]
        S3 = c.prod(1)
        wmf, wme, wmc = p
        lam = 0.5 * 2 * (3 - S1) + (1 / 3) * (3 - S2) + (1 / 6) * (3 + S1 - S2 - 3 * S3) / 2
        mu = (1 - 6 * wmf - 12 * wme - 8 * wmc) + 2 * wmf * S1 + 4 * wme * S2 + 8 * wmc * S3
        r = (lam - k * k * mu) / (2 * k * k)
        return np.sum(r * r) + 1e-8 * np.sum(np.asarray(p) ** 2)

    for G in (3.0, 5.5, 9.25, 20.0, 48.0):
        w = st.fit_one(G)
        p = w[4:7]
        for q in range(3):
            e = np.zeros(3)
            e[q] = 1e-6
            g = (objective(p + e, G) - objective(p - e, G)) / 2e-6
            curv = (objective(p + e, G) - 2 * objective(p, G) + objective(p - e, G)) / 1e-12
            assert abs(g) <= 1e-6 * max(curv, 1e-30) + 1e-14, (G, q, g, curv)


def test_dispersion_beats_7pt_everywhere():
    """True (non-linearised) phase velocity on 2000 random directions."""
    rng = np.random.default_rng(7)
    d = rng.normal(size=(2000, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    seven = np.array([1, 0, 0, 1, 0, 0, 0], dtype=float)
    for G, w in zip(st.g_grid(), st.table()):
        e_fit = np.abs(st.phase_velocity(w, G, d) - 1).max()
        e_7 = np.abs(st.phase_velocity(seven, G, d) - 1).max()
        assert e_fit < 0.05 * e_7, (G, e_fit, e_7)
        assert e_fit < 3e-4
        if G >= 9.0:
            assert e_fit < 2e-6, (G, e_fit)


def test_lookup_interpolates_and_clamps():
    tab = st.table()
    assert np.allclose(st.lookup(np.array([3.0]))[0], tab[0])
    assert np.allclose(st.lookup(np.array([1.0]))[0], tab[0])
    assert np.allclose(st.lookup(np.array([100.0]))[0], tab[-1])
    mid = st.lookup(np.array([3.125]))[0]
    assert np.allclose(mid, 0.5 * (tab[0] + tab[1]))
