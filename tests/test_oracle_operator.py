"""Pins of the oracle's discrete operator (paper eq. 1, sec. 2.3) and of the
subdomain matrices with Robin faces (sec. 2.1)."""
import json
import os

import numpy as np
import pytest

from oracle import operator as op, stencil_table as st
from paper_2110_15113_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _homog(n=9, c=2000.0, h=25.0, f=5.0, npml=0, Q=None):
    vel = np.full((n, n, n), c)
    Qa = None if Q is None else np.full_like(vel, Q)
    return op.make_fields(vel, Qa, 2 * np.pi * f, h, npml)


def test_symmetric_heterogeneous_pml_q():
    w = wl.small_random((11, 10, 9), npml=3, q=60)
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml)
    A = op.assemble(F)
    assert abs(A - A.T).max() == 0.0
    assert A.nnz <= 27 * F.n


def test_family_shells_match_golden():
    """Unstretched homogeneous coefficients of each stiffness family (x h^2),
    derived by hand from the staggered-point definitions."""
    with open(os.path.join(GOLDEN, "family_shells.json")) as fh:
        gold = json.load(fh)["families"]
    F = _homog()
    for fam, ref in enumerate(gold):
        F.w[...] = 0.0
        F.w[..., fam] = 1.0
        C = op.row_coeffs(F) * F.h ** 2
        c = C[:, 4, 4, 4].reshape(3, 3, 3)
        got = {"centre": c[1, 1, 1], "face": c[1, 1, 2], "edge": c[1, 2, 2], "corner": c[2, 2, 2]}
        for key in ref:
            assert abs(got[key] - ref[key]) < 1e-13, (fam, key, got[key], ref[key])
        # every face / edge / corner of the shell is equal (cubic symmetry)
        for ex, ey, ez in op.OFFSETS:
            shell = abs(ex) + abs(ey) + abs(ez)
            name = ["centre", "face", "edge", "corner"][shell]
            assert abs(c[1 + ez, 1 + ey, 1 + ex] - ref[name]) < 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plane_wave_symbol(seed):
    """Away from the boundary, A e^{i xi.x} = (-Lambda/h^2 + omega^2 m mu) e^{i xi.x}
    for a homogeneous model: ties the assembly to the dispersion formulas."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(1500, 5000)
    F = _homog(n=9, c=c, f=rng.uniform(3, 9))
    xi = rng.uniform(-np.pi, np.pi, size=3)
    n = 9
    kk, jj, ii = np.meshgrid(*[np.arange(n)] * 3, indexing="ij")
    u = np.exp(1j * (xi[0] * ii + xi[1] * jj + xi[2] * kk))
    y = op.apply_coeffs(op.row_coeffs(F), u)
    lam, mu = st.lam_mu(F.w[0, 0, 0], xi)
    pred = (-lam / F.h ** 2 + F.omega ** 2 / c ** 2 * mu) * u
    err = np.abs(y - pred)[1:-1, 1:-1, 1:-1].max() / np.abs(pred).max()
    assert err < 1e-12


def test_row_sums_of_stiffness_vanish():
    """Constant fields are in the kernel of every stiffness family (interior,
    no PML), heterogeneous weights included."""
    w = wl.small_random((10, 10, 10), npml=0)
    F = op.make_fields(w.vel, None, w.omega, w.h, 0)
    F.mt[...] = 0.0
    C = op.row_coeffs(F)
    s = C.sum(0)[1:-1, 1:-1, 1:-1]
    assert np.abs(s).max() < 1e-12 * np.abs(C).max()


def test_pml_plane_wave_in_stretched_coordinate():
    """Homogeneous medium, PML along x only: u = exp(i k X(x)) with X' = s_x
    solves the stretched equation d/dx (1/s_x du/dx) + k^2 s_x u = 0, so the
    discrete residual is a small fraction of each term inside the PML."""
    n, npml = 40, 12
    c, h, f = 2000.0, 10.0, 5.0
    vel = np.full((3, 3, n), c)
    F = op.make_fields(vel, None, 2 * np.pi * f, h, npml)
    F.prof = (F.prof[0], np.ones_like(F.prof[1]), np.ones_like(F.prof[2]))
    sx = F.prof[0]
    # X at node i = h * sum_{i' <= i} s_x(i' - 1/2)  (midpoint rule, the
    # points where the stencil evaluates the PML metric)
    X = h * np.concatenate([[0.0], np.cumsum(sx[2:2 * n:2])])
    # numerical wavenumber along x (exact dispersion of the stencil on axis)
    k = 2 * np.pi * f / c
    u1 = np.exp(1j * k * X)
    u = np.broadcast_to(u1[None, None, :], (3, 3, n)).astype(np.complex128)
    C = op.row_coeffs(F)
    y = op.apply_coeffs(C, u)[1, 1, 2:-2]
    scale = (np.abs(C[op.eidx(0, 0, 0)]) * np.abs(u)).max()
    ratio = np.abs(y).max() / scale
    assert ratio < 1e-2, ratio


def test_robin_face_absorbs_outgoing_wave():
    """At an interior face of a subdomain, an outgoing plane wave (e^{+ikx}
    towards the face) nearly satisfies the subdomain equation; the incoming
    wave and the plain Neumann cut do not."""
    c, h, f = 2000.0, 20.0, 5.0
    n = 24
    vel = np.full((n, n, n), c)
    F = op.make_fields(vel, None, 2 * np.pi * f, h, 0)
    lo, hi = (0, 0, 0), (12, n, n)          # interior face at x = 11
    C = op.row_coeffs(F, lo, hi, restrict=True)
    k = 2 * np.pi * f / c
    ii = np.arange(12)
    face = (slice(4, -4), slice(4, -4), 11)
    res = {}
    for name, sgn in (("out", 1.0), ("in", -1.0)):
        u = np.broadcast_to(np.exp(sgn * 1j * k * h * ii)[None, None, :], (n, n, 12)).astype(complex)
        res[name] = np.abs(op.apply_coeffs(C, u)[face]).max()
    Cn = C.copy()
    Cn[op.eidx(0, 0, 0)][:, :, 11] -= 1j * k / h          # remove the Robin term
    u = np.broadcast_to(np.exp(1j * k * h * ii)[None, None, :], (n, n, 12)).astype(complex)
    res["neumann"] = np.abs(op.apply_coeffs(Cn, u)[face]).max()
    assert res["out"] < 0.15 * res["neumann"], res
    assert res["in"] > 1.5 * res["neumann"], res


def test_subdomain_matrix_equals_A_when_box_is_grid():
    w = wl.small_random((8, 9, 10), npml=2, q=40)
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml)
    B = op.row_coeffs(F, (0, 0, 0), (8, 9, 10), restrict=True)
    assert np.array_equal(B, op.row_coeffs(F))


def test_subdomain_matrix_symmetric_and_cut():
    w = wl.small_random((12, 12, 12), npml=2, q=40)
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml)
    lo, hi = (3, 0, 5), (10, 12, 12)
    Bc = op.row_coeffs(F, lo, hi, restrict=True)
    B = op.csr_from_coeffs(Bc)
    assert abs(B - B.T).max() == 0.0
    Ac = op.row_coeffs(F)
    # deep inside the box (two layers away from interior faces) B equals A
    inner = Bc[:, 2:, :, 2:-2]
    ref = Ac[:, lo[2] + 2:hi[2], lo[1]:hi[1], lo[0] + 2:hi[0] - 2]
    assert np.abs(inner - ref).max() < 1e-12 * np.abs(ref).max()


def test_pml_profile_properties():
    s = op.pml_profile(30, 6, 25.0, 2 * np.pi * 5, 3000.0)
    xi = (np.arange(61) - 1) / 2
    inside = (xi >= 6) & (xi <= 23)
    assert np.all(s[inside] == 1.0)
    assert np.all(s.imag[~inside] > 0)
    assert np.all(np.diff(s.imag[xi <= 6]) <= 0) and np.all(np.diff(s.imag[xi >= 23]) >= 0)
    # sigma_max = 3 c ln(1/R0) / (2 L) at d = L
    L = 6 * 25.0
    smax = 3 * 3000.0 * np.log(1e3) / (2 * L)
    assert abs(s[1].imag - smax / (2 * np.pi * 5)) < 1e-12 * smax


def test_point_source_rhs():
    w = wl.small_random((10, 10, 10), npml=2, nsrc=3)
    F = op.make_fields(w.vel, None, w.omega, w.h, w.npml)
    b = op.point_sources(F, w.sources)
    assert b.shape == (3, 10, 10, 10)
    for s, (i, j, k) in enumerate(w.sources):
        assert b[s, k, j, i] == 1.0
        assert np.count_nonzero(b[s]) == 1
