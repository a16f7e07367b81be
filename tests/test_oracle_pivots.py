"""Pins of the oracle's plane pivots (elimination without row exchanges)."""
import numpy as np
import pytest

from oracle import operator as op, oras as ooras, pivots
from paper_2110_15113_amd import workloads as wl


def test_pivots_are_ratios_of_leading_minors():
    rng = np.random.default_rng(3)
    S = rng.normal(size=(6, 6)) + 1j * rng.normal(size=(6, 6)) + 4 * np.eye(6)
    d = pivots.unpivoted_pivots(S)
    minors = [1.0] + [np.linalg.det(S[:i, :i]) for i in range(1, 7)]
    ref = np.array([minors[i + 1] / minors[i] for i in range(6)])
    assert np.allclose(d, ref, rtol=1e-12, atol=0)
    assert abs(np.prod(d) - np.linalg.det(S)) <= 1e-12 * abs(np.linalg.det(S))


def test_tridiagonal_toeplitz_closed_form():
    a, b = 2.5 + 0.3j, -1.0 + 0.2j
    n = 9
    S = a * np.eye(n) + b * (np.eye(n, k=1) + np.eye(n, k=-1))
    d = pivots.unpivoted_pivots(S)
    ref = [a]
    for _ in range(n - 1):
        ref.append(a - b * b / ref[-1])
    assert np.allclose(d, ref, rtol=1e-14, atol=0)


def test_single_plane_ratio_and_decoupled_planes():
    rng = np.random.default_rng(5)
    p, K = 7, 3
    D = [rng.normal(size=(p, p)) + 5 * np.eye(p) for _ in range(K)]
    import scipy.sparse as sp
    B = sp.block_diag(D).tocsr()
    r = pivots.plane_pivot_ratios(B, p, K)
    for k in range(K):
        dk = pivots.unpivoted_pivots(D[k])
        assert np.isclose(r[k], np.abs(dk).min() / np.abs(D[k]).max(), rtol=1e-14)


def test_schur_recursion_matches_dense_elimination():
    """Eliminating the planes of B one after another leaves S_k as the
    trailing block: its pivots are the matching pivots of B itself."""
    w = wl.small_random((5, 4, 4), npml=1, q=40.0, seed=8)
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml)
    B = op.assemble(F)
    p, K = 20, 4
    d_all = pivots.unpivoted_pivots(B.toarray())
    for k, S in enumerate(pivots.plane_schur(B, p, K)):
        assert np.allclose(pivots.unpivoted_pivots(S), d_all[k * p:(k + 1) * p], rtol=1e-9)


def test_singular_neumann_box_is_detected():
    """omega = 0 and no PML: the local matrix of an interior box keeps only
    stiffness fluxes inside the box (Neumann cuts on every face), so constants
    are in its null space and the last pivot vanishes."""
    n = (12, 12, 12)
    vel = np.full(n[::-1], 2000.0)
    with np.errstate(divide="ignore"):
        F = op.make_fields(vel, None, 0.0, 25.0, 0)
    subs = ooras.partition(n, (3, 3, 3), 1)
    inner = [s for s in subs if all(s.lo[a] > 0 and s.hi[a] < n[a] for a in range(3))]
    assert inner
    s = inner[0]
    B = op.csr_from_coeffs(ooras.local_coeffs(F, s))
    sx, sy, sz = (s.hi[a] - s.lo[a] for a in range(3))
    with pytest.raises(np.linalg.LinAlgError):
        pivots.check_nonsingular(B, sx * sy, sz)
    # the same box at 5 Hz with Q is comfortably regular
    Fq = op.make_fields(vel, np.full(n[::-1], 80.0), 2 * np.pi * 5.0, 25.0, 0)
    Bq = op.csr_from_coeffs(ooras.local_coeffs(Fq, s))
    r = pivots.check_nonsingular(Bq, sx * sy, sz)
    assert r.min() > 1e-4
