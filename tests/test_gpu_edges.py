"""Edge cases of the GPU path at the limits the library accepts: the widest
right-hand-side block (256 columns), the longest restart (200), the largest
subdomain plane (8192 nodes), the thinnest boxes (2 nodes), zero overlap and
the smallest grid (3 nodes per axis)."""
import numpy as np
import pytest
import torch

from oracle import blr as oblr, direct, operator as op, oras as ooras
from paper_2110_15113_amd import workloads as wl

from gpu_util import (BLR32_BOX, EPS32, FP32_BOX, FP64_BOX, box_err, need_gpu, oracle_fields, rand_field,
                      rel, say, setup, to_dev)

pytestmark = pytest.mark.gpu


def test_widest_block_of_right_hand_sides():
    """256 columns (the maximum): ORAS apply in both precisions and with BLR
    plane inverses against the oracle, and an FP64 block solve against the
    direct solution."""
    need_gpu()
    w = wl.small_random((14, 13, 12), npml=2, q=70.0, seed=31, parts=(2, 2, 1), overlap=2)
    say("256 right-hand sides")
    F = oracle_fields(w)
    x = rand_field((w.nz, w.ny, w.nx), 256, 17)
    ref = ooras.ORAS(F, w.parts, w.overlap).apply(x)
    S = setup(w, prec=2, parts=w.parts)
    got = S.apply_M(to_dev(x, S)).cpu().numpy()
    assert rel(got, ref) < 1e-9 and box_err(got, ref, w.parts, w.overlap) < FP64_BOX
    S32 = setup(w, prec=1, parts=w.parts)
    e32 = box_err(S32.apply_M(to_dev(x, S32)).cpu().numpy(), ref, w.parts, w.overlap)
    say(f"  per-box error complex64 {e32:.2e} = {e32 / EPS32:.0f} eps32")
    assert e32 < FP32_BOX, e32
    S32.compress(1e-3, 4)
    ref_blr = oblr.OrasBLR(F, w.parts, w.overlap, 1e-3, 4).apply(x)
    eb = box_err(S32.apply_M(to_dev(x, S32)).cpu().numpy(), ref_blr, w.parts, w.overlap)
    say(f"  per-box error complex64 BLR {eb:.2e}")
    assert eb < BLR32_BOX * 1e-3, eb
    A = op.assemble(F)
    b = x[:, ::-1].copy()                   # any 256 right-hand sides
    u = direct.solve(A, F.shape, b)
    r = S.solve(to_dev(b, S), 1e-10, restart=30)
    assert r.converged.all()
    assert rel(r.x.cpu().numpy(), u) < 1e-7


def test_longest_restart():
    """restart = 200 (the maximum): one cycle reaches the tolerance; a
    restart of 4 needs several cycles; both match the direct solution."""
    need_gpu()
    w = wl.small_random((16, 15, 14), npml=3, q=60.0, nsrc=3, seed=32, parts=(2, 2, 2))
    say("restart 200")
    F = oracle_fields(w)
    b = op.point_sources(F, w.sources)
    u = direct.solve(op.assemble(F), F.shape, b)
    S = setup(w, prec=2, parts=w.parts)
    r200 = S.solve(to_dev(b, S), 1e-10, restart=200, maxit=200)
    assert r200.converged.all() and r200.cycles == 1
    r4 = S.solve(to_dev(b, S), 1e-10, restart=4, maxit=400)
    assert r4.converged.all() and r4.cycles > 1
    assert rel(r200.x.cpu().numpy(), u) < 1e-7
    assert rel(r4.x.cpu().numpy(), u) < 1e-7


@pytest.mark.parametrize("prec", [2, 1])
def test_largest_subdomain_plane(prec):
    """One subdomain whose planes hold 128 x 64 = 8192 nodes (the largest
    accepted): ORAS with a single subdomain is A^{-1} (sec. 2.1), so
    A M^{-1} b = b checks the whole factorisation and substitution; one
    FGMRES step solves.  One more column per plane is refused."""
    need_gpu()
    from paper_2110_15113_amd import oras
    w = wl.small_random((128, 64, 6), npml=2, q=80.0, nsrc=2, seed=33, parts=(1, 1, 1), overlap=0)
    say(f"plane of 8192 nodes, prec {prec}")
    S = setup(w, prec=prec, parts=(1, 1, 1), overlap=0)
    b = S.point_sources(w.sources)
    y = S.apply_M(b)
    r = b - S.apply_A(y, prec=oras.C128)
    res = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))
    say(f"  |b - A M^-1 b| / |b| = {res:.2e}")
    # measured 4.9e-14 (FP64) and 1.5e-5 = 250 eps32 (FP32: the rounding of
    # the plane inverses, amplified by the conditioning of A); the bars keep a
    # factor of about 20 and 7
    assert res < (1e-12 if prec == 2 else 1e-4), res
    sol = S.solve(b, 1e-6 if prec == 1 else 1e-10)
    assert sol.converged.all() and sol.total_iters <= (6 if prec == 1 else 1), sol.total_iters
    S.close()
    w2 = wl.small_random((129, 64, 6), npml=2, seed=33, parts=(1, 1, 1), overlap=0)
    S2 = setup(w2, prec=prec)
    with pytest.raises(oras.OrasError, match="8192"):
        S2.factor((1, 1, 1), 0, prec)


@pytest.mark.parametrize("parts,ov", [((6, 1, 2), 0), ((2, 2, 2), 0), ((6, 5, 4), 1)])
def test_thin_boxes_and_zero_overlap(parts, ov):
    """Boxes two nodes wide and overlap 0 (block Jacobi with Robin faces):
    ORAS apply against the oracle in both precisions."""
    need_gpu()
    w = wl.small_random((12, 10, 8), npml=2, q=90.0, seed=34, parts=parts, overlap=ov)
    say(f"thin boxes {parts} overlap {ov}")
    F = oracle_fields(w)
    x = rand_field((w.nz, w.ny, w.nx), 5, 19)
    ref = ooras.ORAS(F, parts, ov).apply(x)
    S = setup(w, prec=2, parts=parts, overlap=ov)
    got = S.apply_M(to_dev(x, S)).cpu().numpy()
    assert rel(got, ref) < 1e-9 and box_err(got, ref, parts, ov) < FP64_BOX
    S32 = setup(w, prec=1, parts=parts, overlap=ov)
    e32 = box_err(S32.apply_M(to_dev(x, S32)).cpu().numpy(), ref, parts, ov)
    say(f"  per-box error complex64 {e32:.2e} = {e32 / EPS32:.0f} eps32")
    assert e32 < FP32_BOX, e32


@pytest.mark.parametrize("prec", [2, 1])
def test_smallest_grid(prec):
    """The smallest accepted grid (3 nodes per axis, one PML layer, so one
    physical node) as one subdomain, and with npml = 0 split 1 x 1 x 1: the
    solve against the oracle's direct solution."""
    need_gpu()
    from paper_2110_15113_amd import oras
    for npml in (1, 0):
        vel = np.full((3, 3, 3), 2000.0)
        vel[1, 1, 2] = 2500.0
        Q = np.full_like(vel, 80.0)
        F = op.make_fields(vel, Q, 2 * np.pi * 5.0, 25.0, npml)
        b = op.point_sources(F, [(1, 1, 1)])
        u = direct.solve(op.assemble(F), F.shape, b)
        S = oras.Solver(0)
        dev = S.device
        S.assemble(torch.as_tensor(vel, device=dev), 25.0, npml, 2 * np.pi * 5.0,
                   torch.as_tensor(Q, device=dev), prec=prec)
        S.factor((1, 1, 1), 0, prec)
        r = S.solve(to_dev(b, S), 1e-6 if prec == 1 else 1e-12)
        assert r.converged.all()
        assert rel(r.x.cpu().numpy(), u) < (1e-5 if prec == 1 else 1e-11), (npml, prec)
        S.close()


def test_rejected_models_leave_the_context_unchanged():
    """Model arrays are checked entry by entry on the device before the
    context changes: a NaN, infinite, zero or negative velocity, Q or squared
    slowness anywhere is refused (ORAS_E_ARG, with the count of offending
    entries), and the operator and factors of the last valid call stay in
    use bit for bit."""
    need_gpu()
    from paper_2110_15113_amd import oras
    w = wl.small_random((14, 12, 11), npml=2, q=60.0, seed=41, parts=(2, 2, 1), overlap=2)
    say("rejected models")
    S = setup(w, prec=2, parts=w.parts)
    dev = S.device
    x = to_dev(rand_field((w.nz, w.ny, w.nx), 3, 2), S)
    y0 = S.apply_A(x)
    z0 = S.apply_M(x)
    vel = torch.as_tensor(w.vel, device=dev)
    Q = torch.as_tensor(w.Q, device=dev)
    m = 1.0 / vel ** 2

    def spoil(t, vals):
        t = t.clone()
        flat = t.view(-1)
        for k, v in enumerate(vals):
            flat[(97 * k + 13) % flat.numel()] = v
        return t

    bad_values = [[float("nan")], [0.0], [-1500.0], [float("inf")], [float("nan"), -1.0, 0.0]]
    for vals in bad_values:
        with pytest.raises(oras.OrasError, match=f"velocity: {len(vals)} entries") as e:
            S.assemble(spoil(vel, vals), w.h, w.npml, w.omega, Q, prec=2)
        assert e.value.code == 1
        with pytest.raises(oras.OrasError, match=f"Q: {len(vals)} entries") as e:
            S.assemble(vel, w.h, w.npml, w.omega, spoil(Q, vals), prec=2)
        assert e.value.code == 1
        with pytest.raises(oras.OrasError, match=f"m: {len(vals)} entries") as e:
            S.set_m(spoil(m, vals))
        assert e.value.code == 1
        assert torch.equal(S.apply_A(x), y0)
        assert torch.equal(S.apply_M(x), z0)
    S.close()


def test_non_finite_pivot_is_reported_and_leaves_no_factors():
    """A velocity so small at one node that its squared slowness overflows
    (finite and positive, so accepted) makes the plane Schur complement of the
    subdomain holding it non-finite: the factorisation returns ORAS_E_NUMERIC,
    keeps no factors (a solve is then out of order), and a valid model
    factors again afterwards."""
    need_gpu()
    from paper_2110_15113_amd import oras
    w = wl.small_random((12, 12, 10), npml=2, q=None, seed=42, parts=(2, 2, 1), overlap=2)
    say("non-finite pivot")
    S = oras.Solver(0)
    dev = S.device
    vel = w.vel.copy()
    vel[5, 6, 7] = 1e-200                  # m = 1e400 overflows to inf
    S.assemble(torch.as_tensor(vel, device=dev), w.h, w.npml, w.omega, None, prec=2,
               c_ref=float(w.vel.max()))
    for prec in (2, 1):
        if prec == 1:
            S.assemble(torch.as_tensor(vel, device=dev), w.h, w.npml, w.omega, None, prec=1,
                       c_ref=float(w.vel.max()))
        with pytest.raises(oras.OrasError, match="pivot") as e:
            S.factor(w.parts, w.overlap, prec)
        assert e.value.code == 5
        b = S.point_sources([(4, 4, 4)])
        with pytest.raises(oras.OrasError) as e:
            S.solve(b, 1e-8)
        assert e.value.code == 2
    S.assemble(torch.as_tensor(w.vel, device=dev), w.h, w.npml, w.omega, None, prec=2)
    S.factor(w.parts, w.overlap, 2)
    r = S.solve(S.point_sources([(4, 4, 4)]), 1e-8)
    assert r.converged.all()
    S.close()


def test_pivot_ratio_flags_a_nearly_singular_box():
    """With omega near zero and no PML the local matrices of interior boxes
    approach the Neumann-only Laplacian, which is singular: the factorisation
    still succeeds (no pivot is zero) but its pivot statistic drops by many
    orders against the same boxes at 5 Hz with attenuation."""
    need_gpu()
    from paper_2110_15113_amd import oras
    n = (12, 12, 12)
    vel = np.full(n[::-1], 2000.0)
    ratios = {}
    for omega, Q in ((1e-8, None), (2 * np.pi * 5.0, np.full(n[::-1], 80.0))):
        S = oras.Solver(0)
        dev = S.device
        S.assemble(torch.as_tensor(vel, device=dev), 25.0, 0, omega,
                   None if Q is None else torch.as_tensor(Q, device=dev), prec=2)
        S.factor((3, 3, 3), 1, 2)
        ratios[omega] = S.factor_stats()[0]
        S.close()
    say(f"pivot ratio near omega 0: {ratios[1e-8]:.2e}; at 5 Hz: {ratios[2 * np.pi * 5.0]:.2e}")
    assert ratios[1e-8] < 1e-7
    assert ratios[2 * np.pi * 5.0] > 1e-4
