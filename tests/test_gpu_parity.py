"""Parity of the HIP path with the oracle, element by element on seeded
inputs (assembly, stencil, ORAS apply, sources, sampling, gradient)."""
import numpy as np
import pytest
import torch

from oracle import adjoint, operator as op, oras as ooras
from paper_2110_15113_amd import workloads as wl

from gpu_util import (EPS32, FP32_BOX, FP64_BOX, box_err, need_gpu, oracle_fields, rand_field,
                      rel, say, setup, to_dev)

pytestmark = pytest.mark.gpu

CASES = [
    dict(n=(13, 11, 12), npml=3, q=60.0, seed=1),
    dict(n=(20, 17, 9), npml=2, q=None, seed=2),
]


@pytest.mark.parametrize("case", CASES)
def test_assemble_coefficients(case):
    need_gpu()
    w = wl.small_random(case["n"], npml=case["npml"], q=case["q"], seed=case["seed"])
    say(f"assemble {w.name}")
    S = setup(w)
    got = S.coefficients().cpu().numpy()
    ref = op.row_coeffs(oracle_fields(w))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 1e-11, err


@pytest.mark.parametrize("nrhs", [1, 3, 9])
def test_apply_A_c128_and_c64(nrhs):
    need_gpu()
    w = wl.small_random((19, 13, 11), npml=3, q=80.0, seed=4)
    say(f"apply_A nrhs={nrhs}")
    S = setup(w, prec=1)          # complex64 stencil (plus the FP64 copy)
    x = rand_field((w.nz, w.ny, w.nx), nrhs, 7)
    C = op.row_coeffs(oracle_fields(w))
    ref = op.apply_coeffs(C, x)
    y128 = S.apply_A(to_dev(x, S), prec=2).cpu().numpy()
    assert rel(y128, ref) < 1e-12
    y64 = S.apply_A(to_dev(x, S), prec=1).cpu().numpy()
    assert rel(y64, ref) < 2e-6


ORAS_CASES = [
    dict(n=(16, 16, 16), parts=(2, 2, 2), ov=2, npml=3, q=100.0, nrhs=2),
    dict(n=(19, 17, 15), parts=(2, 3, 2), ov=1, npml=2, q=50.0, nrhs=3),
    dict(n=(26, 14, 12), parts=(3, 1, 2), ov=3, npml=2, q=None, nrhs=9),
    dict(n=(12, 12, 12), parts=(1, 1, 1), ov=2, npml=2, q=70.0, nrhs=1),
    # column blocks of the FP32 plane GEMM: a pair with masked columns, a pair
    # plus a single block, two pairs
    dict(n=(18, 16, 14), parts=(2, 2, 1), ov=2, npml=2, q=60.0, nrhs=20),
    dict(n=(15, 19, 13), parts=(1, 2, 2), ov=1, npml=2, q=None, nrhs=37),
    dict(n=(14, 14, 14), parts=(2, 2, 2), ov=2, npml=2, q=80.0, nrhs=64),
    # 24 subdomains: the factorisation runs 8 and 16 of them on two streams
    dict(n=(26, 23, 21), parts=(4, 3, 2), ov=2, npml=2, q=60.0, nrhs=5),
]


@pytest.mark.parametrize("case", ORAS_CASES)
def test_apply_M_matches_oracle(case):
    need_gpu()
    w = wl.small_random(case["n"], npml=case["npml"], q=case["q"], seed=5,
                        parts=case["parts"], overlap=case["ov"])
    say(f"apply_M {case}")
    F = oracle_fields(w)
    M = ooras.ORAS(F, case["parts"], case["ov"])
    x = rand_field((w.nz, w.ny, w.nx), case["nrhs"], 11)
    ref = M.apply(x)
    S = setup(w, prec=2, parts=case["parts"], overlap=case["ov"])
    got = S.apply_M(to_dev(x, S)).cpu().numpy()
    S64 = setup(w, prec=1, parts=case["parts"], overlap=case["ov"])
    got64 = S64.apply_M(to_dev(x, S64)).cpu().numpy()
    e128 = box_err(got, ref, case["parts"], case["ov"])
    e64 = box_err(got64, ref, case["parts"], case["ov"])
    say(f"  per-box error: complex128 {e128:.2e}, complex64 {e64:.2e} = {e64 / EPS32:.0f} eps32")
    assert rel(got, ref) < 1e-9 and e128 < FP64_BOX, (rel(got, ref), e128)
    assert e64 < FP32_BOX, e64


PML_CASES = [
    dict(n=(16, 16, 16), parts=(2, 2, 2), ov=2, npml=3, q=100.0, nrhs=2),
    dict(n=(19, 17, 15), parts=(2, 3, 2), ov=3, npml=2, q=50.0, nrhs=9),
    dict(n=(22, 14, 18), parts=(3, 1, 2), ov=1, npml=2, q=None, nrhs=20),
]


@pytest.mark.parametrize("case", PML_CASES)
def test_apply_M_pml_interfaces_matches_oracle(case):
    """PML transmission conditions: B_j = R_j A(s_j) R_j^T with the interface
    layer over the overlap (paper sec. 2.2, note on the size of overlap)."""
    need_gpu()
    w = wl.small_random(case["n"], npml=case["npml"], q=case["q"], seed=7,
                        parts=case["parts"], overlap=case["ov"])
    say(f"apply_M pml {case}")
    F = oracle_fields(w)
    M = ooras.ORAS(F, case["parts"], case["ov"], interface="pml")
    x = rand_field((w.nz, w.ny, w.nx), case["nrhs"], 17)
    ref = M.apply(x)
    S = setup(w, prec=2, parts=case["parts"], overlap=case["ov"], interface="pml")
    got = S.apply_M(to_dev(x, S)).cpu().numpy()
    S64 = setup(w, prec=1, parts=case["parts"], overlap=case["ov"], interface="pml")
    got64 = S64.apply_M(to_dev(x, S64)).cpu().numpy()
    e128 = box_err(got, ref, case["parts"], case["ov"])
    e64 = box_err(got64, ref, case["parts"], case["ov"])
    say(f"  per-box error: complex128 {e128:.2e}, complex64 {e64:.2e} = {e64 / EPS32:.0f} eps32")
    assert rel(got, ref) < 1e-9 and e128 < FP64_BOX, (rel(got, ref), e128)
    assert e64 < FP32_BOX, e64


def test_subdomain_boxes_match_oracle_partition():
    need_gpu()
    w = wl.small_random((19, 17, 15), npml=2, seed=3)
    S = setup(w, parts=(2, 3, 2), overlap=2)
    boxes = S.subdomains()
    ref = ooras.partition((19, 17, 15), (2, 3, 2), 2)
    assert len(boxes) == len(ref)
    for b, r in zip(boxes, ref):
        assert tuple(b[0:3]) == r.lo and tuple(b[3:6]) == r.hi
        assert tuple(b[6:9]) == r.olo and tuple(b[9:12]) == r.ohi


def test_sources_sample_spread_gradient():
    need_gpu()
    w = wl.small_random((14, 12, 10), npml=2, q=40.0, nsrc=3, seed=8)
    say("sources/sample/spread/gradient")
    S = setup(w)
    F = oracle_fields(w)
    amps = [1.0, 2.0 - 1.0j, 0.5j]
    b = S.point_sources(w.sources, amps).cpu().numpy()
    assert np.array_equal(b, op.point_sources(F, w.sources, amps))
    rec = [(3, 3, 3), (5, 4, 3), (6, 5, 6), (3, 3, 3)]
    U = rand_field((w.nz, w.ny, w.nx), 3, 1)
    MU = rand_field((w.nz, w.ny, w.nx), 3, 2)
    d = S.sample(to_dev(U, S), rec).cpu().numpy()
    assert np.array_equal(d, adjoint.sample(U, rec))
    G = rand_field((len(rec),), 3, 3).reshape(3, len(rec))
    sp = S.spread(to_dev(G, S), rec).cpu().numpy()
    assert np.abs(sp - adjoint.spread(G, rec, F.shape)).max() < 1e-15
    g = S.gradient(to_dev(U, S), to_dev(MU, S)).cpu().numpy()
    ref = adjoint.gradient(F, U, MU)
    assert np.abs(g - ref).max() < 1e-11 * np.abs(ref).max()


GRAD_CASES = [
    dict(n=(13, 11, 12), npml=3, q=60.0, nrhs=2, seed=41),
    dict(n=(20, 17, 9), npml=2, q=None, nrhs=3, seed=42),
]


@pytest.mark.parametrize("case", GRAD_CASES)
def test_exact_gradient_matches_oracle(case):
    """Weights following m (sec. 2.3): gradient with the table-slope term, at
    the assembled model and after set_m(..., weights='follow') to a perturbed
    model; the coefficients after the update match the oracle's fields."""
    need_gpu()
    w = wl.small_random(case["n"], npml=case["npml"], q=case["q"], seed=case["seed"])
    say(f"exact gradient {case}")
    S = setup(w)
    shape = (w.nz, w.ny, w.nx)
    U = rand_field(shape, case["nrhs"], 5)
    MU = rand_field(shape, case["nrhs"], 6)
    cref = float(w.vel.max())
    m0 = 1.0 / w.vel ** 2
    rng = np.random.default_rng(case["seed"])
    m1 = m0 * (1 + 0.08 * rng.standard_normal(m0.shape))
    for m, update in ((m0, False), (m1, True)):
        if update:
            S.set_m(to_dev(m, S), weights="follow")
        F = adjoint.fields_from_m(m, w.Q, w.omega, w.h, w.npml, cref)
        C = S.coefficients().cpu().numpy()
        ref_c = op.row_coeffs(F)
        assert np.abs(C - ref_c).max() <= 1e-11 * np.abs(ref_c).max()
        ref = adjoint.gradient_exact(F, U, MU, m)
        frozen = adjoint.gradient(F, U, MU)
        g = S.gradient(to_dev(U, S), to_dev(MU, S), weights=True).cpu().numpy()
        assert np.abs(g - ref).max() <= 1e-11 * np.abs(ref).max(), update
        # the weight term is a sizeable part of the result
        assert np.abs(ref - frozen).max() > 1e-3 * np.abs(ref).max()
        g0 = S.gradient(to_dev(U, S), to_dev(MU, S)).cpu().numpy()
        assert np.abs(g0 - frozen).max() <= 1e-11 * np.abs(frozen).max()


def test_exact_gradient_needs_weights_that_follow_m():
    need_gpu()
    from paper_2110_15113_amd import oras
    w = wl.small_random((9, 8, 7), npml=1, seed=43)
    S = setup(w)
    U = to_dev(rand_field((w.nz, w.ny, w.nx), 1, 1), S)
    S.set_m(to_dev(1.01 / w.vel ** 2, S))             # frozen weights
    with pytest.raises(oras.OrasError):
        S.gradient(U, U, weights=True)
    S.set_m(to_dev(1.01 / w.vel ** 2, S), weights="follow")
    S.gradient(U, U, weights=True)


def test_free_surface_assembly_and_solve():
    """Free-surface top (no PML on the low z side, Dirichlet ghost layer):
    coefficients against the oracle's, and an FP64 ORAS-FGMRES solve against
    the oracle's direct solution."""
    need_gpu()
    from oracle import direct
    from paper_2110_15113_amd import oras
    w = wl.small_random((15, 14, 13), npml=3, q=70.0, nsrc=2, seed=23, parts=(2, 2, 2))
    say("free surface")
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml, free_surface=True)
    S = oras.Solver(0)
    dev = S.device
    S.assemble(torch.as_tensor(w.vel, device=dev), w.h, w.npml, w.omega,
               torch.as_tensor(w.Q, device=dev), prec=oras.C128, free_surface=True)
    got = S.coefficients().cpu().numpy()
    ref = op.row_coeffs(F)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
    # the flag changes the top rows only
    ref_pml = op.row_coeffs(oracle_fields(w))
    diff = np.abs(ref - ref_pml).max(axis=(0, 2, 3))      # per z-plane (27, nz, ny, nx)
    assert diff[0] > 0 and not diff[w.npml + 1:].any()
    S.factor(w.parts, w.overlap, oras.C128)
    b = op.point_sources(F, w.sources)
    u = direct.solve(op.assemble(F), F.shape, b)
    r = S.solve(to_dev(b, S), 1e-10)
    assert r.converged.all()
    assert rel(r.x.cpu().numpy(), u) < 1e-7


@pytest.mark.parametrize("R0,power,c_ref", [(1e-2, 3, 3500.0), (1e-4, 1, 0.0)])
def test_pml_parameters(R0, power, c_ref):
    """PML law parameters of the assembly (reflection R0, profile power, and a
    reference velocity; c_ref <= 0 takes the model maximum) against the
    oracle's coefficients."""
    need_gpu()
    from paper_2110_15113_amd import oras
    w = wl.small_random((13, 12, 11), npml=3, q=50.0, seed=24)
    say(f"pml R0={R0} power={power} c_ref={c_ref}")
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml, R0=R0, power=power,
                       c_ref=None if c_ref <= 0 else c_ref)
    S = oras.Solver(0)
    dev = S.device
    S.assemble(torch.as_tensor(w.vel, device=dev), w.h, w.npml, w.omega,
               torch.as_tensor(w.Q, device=dev), prec=oras.C128, R0=R0, power=power, c_ref=c_ref)
    got = S.coefficients().cpu().numpy()
    ref = op.row_coeffs(F)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
    assert np.abs(ref - op.row_coeffs(oracle_fields(w))).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("prec", [1, 2])
def test_gemm_accounting(prec):
    """The per-launch accounting behind the plane-GEMM roofline: one launch
    per plane step (2 max_sz - 1 per apply) and, per active subdomain plane,
    8 p^2 nrhs flops and p^2 + (2 or 3) p nrhs complex entries, where the
    backward sweep runs from the second-to-last plane down to the lowest
    owned one; recomputed here from the oracle's partition."""
    need_gpu()
    w = wl.small_random((17, 15, 14), npml=2, q=60.0, seed=25, parts=(2, 2, 2), overlap=2)
    say(f"gemm accounting prec={prec}")
    S = setup(w, prec=prec, parts=w.parts)
    nrhs = 5
    x = rand_field((w.nz, w.ny, w.nx), nrhs, 13)
    S.profile(True)
    S.apply_M(to_dev(x, S))
    secs, launches, flops, nbytes = S.kernel_stats()
    subs = ooras.partition((w.nx, w.ny, w.nz), w.parts, w.overlap)
    sz = [s.hi[2] - s.lo[2] for s in subs]
    assert launches == 2 * max(sz) - 1
    f = b = 0.0
    cs = 8 if prec == 1 else 16
    for s in subs:
        p = (s.hi[0] - s.lo[0]) * (s.hi[1] - s.lo[1])
        nz_ = s.hi[2] - s.lo[2]
        for k in range(nz_):
            f += 8.0 * p * p * nrhs
            b += cs * (p * p + 2 * p * nrhs)
            if k <= nz_ - 2 and k >= s.olo[2] - s.lo[2]:
                f += 8.0 * p * p * nrhs
                b += cs * (p * p + 3 * p * nrhs)
    assert flops == f and nbytes == b, (flops, f, nbytes, b)
    assert secs > 0
    # the right-hand-side kernels (restriction fused): per active plane,
    # p nrhs (16 forward + cs if coupled + t written) + 9 p cs if coupled,
    # t as six bf16 pieces (12 bytes) in FP32, one value in FP64
    rsecs, rbytes = S.rhs_stats()
    tw = 12 if prec == 1 else 16
    rb = 0.0
    for s in subs:
        p = (s.hi[0] - s.lo[0]) * (s.hi[1] - s.lo[1])
        nz_ = s.hi[2] - s.lo[2]
        for k in range(nz_):
            rb += p * nrhs * (16 + (cs if k > 0 else 0) + tw) + (9 * p * cs if k > 0 else 0)
            if k <= nz_ - 2 and k >= s.olo[2] - s.lo[2]:
                rb += p * nrhs * (cs + tw) + 9 * p * cs
    assert rbytes == rb and rsecs > 0, (rbytes, rb, rsecs)


PIVOT_CASES = [
    dict(n=(16, 16, 16), parts=(2, 2, 2), ov=2, npml=3, q=100.0, iface="robin"),
    dict(n=(19, 17, 15), parts=(2, 3, 2), ov=3, npml=2, q=50.0, iface="pml"),
]


@pytest.mark.parametrize("case", PIVOT_CASES)
def test_factor_pivot_ratios_match_oracle(case):
    """The factorisation's pivot statistic min |pivot| / max |S_k| of every
    subdomain plane (sec. 2.2, factorisation at set-up; the plane inverses
    are formed without row exchanges) against the oracle's pivots of the
    same Schur complements by elimination without exchanges."""
    need_gpu()
    from oracle import pivots
    w = wl.small_random(case["n"], npml=case["npml"], q=case["q"], seed=21,
                        parts=case["parts"], overlap=case["ov"])
    say(f"pivot ratios {case}")
    F = oracle_fields(w)
    ref = []
    for s in ooras.partition(case["n"], case["parts"], case["ov"]):
        B = op.csr_from_coeffs(ooras.local_coeffs(F, s, case["iface"]))
        sx, sy, sz = (s.hi[a] - s.lo[a] for a in range(3))
        ref.append(pivots.plane_pivot_ratios(B, sx * sy, sz))
    for prec, tol in ((2, 1e-9), (1, 2e-3)):
        S = setup(w, prec=prec, parts=case["parts"], overlap=case["ov"], interface=case["iface"])
        rmin, where, got = S.factor_stats()
        worst = 0.0
        for j, r in enumerate(ref):
            g = got[j, :len(r)]
            assert np.all(np.isnan(got[j, len(r):]))
            worst = max(worst, float(np.max(np.abs(g - r) / r)))
        allref = np.concatenate(ref)
        say(f"  prec {prec}: min ratio {rmin:.3e} at {where} (oracle {allref.min():.3e}); "
            f"largest relative gap {worst:.1e}")
        assert worst <= tol, worst
        assert abs(rmin - allref.min()) <= tol * allref.min()
        S.close()
