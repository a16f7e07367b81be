"""Pins of the oracle's PML transmission conditions in ORAS (paper sec. 2.2,
note on the size of overlap: for FD, the subdomain matrices carry a PML in
the overlap region instead of an impedance condition).

B_j = R_j A(s_j) R_j^T with the subdomain profile s_j = global PML plus an
interface PML over the overlap layers (oracle.operator.interface_pml_profile).
"""
import numpy as np
import pytest

from oracle import direct, krylov, operator as op, oras
from paper_2110_15113_amd import workloads as wl


def _fields(w):
    return op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml)


def test_single_subdomain_is_the_operator():
    w = wl.small_random((12, 11, 10), npml=2, q=60.0, seed=4)
    F = _fields(w)
    M = oras.ORAS(F, (1, 1, 1), 2, interface="pml")
    assert abs(M.local_matrix(0) - op.assemble(F)).max() == 0.0


@pytest.mark.parametrize("parts,ov", [((2, 2, 1), 2), ((3, 1, 2), 3)])
def test_local_matrices_complex_symmetric(parts, ov):
    w = wl.small_random((16, 13, 12), npml=2, q=50.0, seed=6)
    F = _fields(w)
    M = oras.ORAS(F, parts, ov, interface="pml")
    for j in range(len(M.subs)):
        B = M.local_matrix(j)
        assert abs(B - B.T).max() <= 1e-12 * abs(B).max()


def test_rows_away_from_the_overlap_are_rows_of_A():
    """Owned nodes whose stencil touches no overlap layer keep A's row (only
    couplings leaving the box are dropped, and those nodes have none)."""
    w = wl.small_random((18, 16, 14), npml=2, q=70.0, seed=9)
    F = _fields(w)
    M = oras.ORAS(F, (2, 2, 2), 2, interface="pml")
    CA = op.row_coeffs(F)
    n = (F.nx, F.ny, F.nz)
    checked = 0
    for s in M.subs:
        C = oras.local_coeffs(F, s, "pml")
        # owned nodes at least one layer inside the owned range on interior sides
        rng = []
        for a in range(3):
            lo_ = s.olo[a] + (1 if s.lo[a] > 0 else 0)
            hi_ = s.ohi[a] - (1 if s.hi[a] < n[a] else 0)
            rng.append(range(lo_, hi_))
        for z in rng[2]:
            for y in rng[1]:
                for x in rng[0]:
                    got = C[:, z - s.lo[2], y - s.lo[1], x - s.lo[0]]
                    assert np.array_equal(got, CA[:, z, y, x]), (s, x, y, z)
                    checked += 1
    assert checked > 100


def test_interface_profile_shape_and_designed_absorption():
    """Zero added absorption on the owned range, increasing through the
    overlap, and sigma integrated across the layer equal to the designed
    round trip: exp(-2 int sigma / c_ref dx) = R0 for the continuous layer
    (the discrete half-grid quadrature converges to it as the layer refines)."""
    h, omega, c_ref, R0 = 20.0, 2 * np.pi * 6.0, 3000.0, 0.3
    for delta in (2, 3, 8, 32):
        n = 2 * delta + 16
        base = np.ones(2 * n + 1, dtype=np.complex128)
        lo, olo = 4, 4 + delta
        ohi, hi = n - 4 - delta, n - 4
        s = op.interface_pml_profile(base, n, lo, hi, olo, ohi, h, omega, c_ref, R0)
        sig = (s.imag * omega)
        xi = (np.arange(2 * n + 1) - 1.0) / 2.0
        assert np.all(sig[(xi >= olo) & (xi <= ohi - 1)] == 0.0)
        left = sig[(xi >= lo) & (xi <= olo)]
        assert np.all(np.diff(left) < 0)                       # decreasing into the owned range
        right = sig[(xi >= ohi - 1) & (xi <= hi - 1)]
        assert np.all(np.diff(right) > 0)
        # midpoint rule on the half grid over [lo, olo] (the layer of thickness delta h)
        seg = sig[(xi >= lo) & (xi <= olo)]
        integral = 0.5 * h * (0.5 * seg[0] + seg[1:-1].sum() + 0.5 * seg[-1])
        expected = 0.5 * c_ref * np.log(1.0 / R0)
        rel = abs(integral - expected) / expected
        assert rel < 0.6 / delta ** 2, (delta, rel)


def test_global_boundary_sides_get_no_interface_layer():
    n, h, omega = 20, 25.0, 2 * np.pi * 5.0
    base = np.ones(2 * n + 1, dtype=np.complex128)
    s = op.interface_pml_profile(base, n, 0, 12, 0, 10, h, omega, 2500.0)
    xi = (np.arange(2 * n + 1) - 1.0) / 2.0
    assert np.all(s[xi <= 9] == 1.0)          # low side is the grid boundary
    assert np.all(s.imag[(xi > 9) & (xi <= 11)] > 0)


def test_fgmres_with_pml_interfaces_reaches_the_direct_solution():
    w = wl.config1()
    F = _fields(w)
    A = op.assemble(F)
    b = op.point_sources(F, w.sources)[0]
    x_ref = direct.solve(A, F.shape, b[None])[0]
    for ov in (2, 3):
        M = oras.ORAS(F, w.parts, ov, interface="pml")
        x, it, ok, _ = krylov.fgmres(lambda v: A @ v,
                                     lambda v: M.apply(v.reshape(F.shape)).reshape(-1),
                                     b.reshape(-1), 1e-10, 30, 300)
        assert ok
        err = np.linalg.norm(x - x_ref.reshape(-1)) / np.linalg.norm(x_ref)
        assert err < 1e-7, (ov, err)
        assert it < 60, (ov, it)
