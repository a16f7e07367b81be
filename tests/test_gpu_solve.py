"""End-to-end ORAS-FGMRES solves on the GPU against the oracle."""
import numpy as np
import pytest
import torch

from oracle import direct, krylov, operator as op, oras as ooras
from paper_2110_15113_amd import workloads as wl

from gpu_util import need_gpu, oracle_fields, rand_field, rel, say, setup, to_dev

pytestmark = pytest.mark.gpu


def _direct(w, b):
    F = oracle_fields(w)
    A = op.assemble(F)
    return direct.solve(A, F.shape, b), A


def test_config1_fp64_matches_direct_and_oracle_fgmres():
    need_gpu()
    c = wl.config1()
    say("config1 fp64")
    F = oracle_fields(c)
    b = op.point_sources(F, c.sources)
    u, A = _direct(c, b)
    S = setup(c, prec=2, parts=c.parts)
    r = S.solve(to_dev(b, S), c.tol, restart=c.restart)
    x = r.x.cpu().numpy()
    assert r.converged.all()
    assert np.linalg.norm(A @ x[0].ravel() - b[0].ravel()) <= c.tol * np.linalg.norm(b[0]) * 1.0001
    assert rel(x, u) < 1e-6, rel(x, u)
    M = ooras.ORAS(F, c.parts, c.overlap)
    _, it, ok, _ = krylov.fgmres(lambda v: A @ v, lambda v: M.apply(v.reshape(F.shape)).reshape(-1),
                                 b[0].ravel(), c.tol, c.restart, c.maxit)
    assert ok and abs(int(r.iters[0]) - it) <= 1, (r.iters, it)


@pytest.mark.parametrize("ov", [2, 3])
def test_config1_pml_interfaces_match_direct_and_oracle_fgmres(ov):
    need_gpu()
    c = wl.config1()
    say(f"config1 fp64, PML interfaces, overlap {ov}")
    F = oracle_fields(c)
    b = op.point_sources(F, c.sources)
    u, A = _direct(c, b)
    S = setup(c, prec=2, parts=c.parts, overlap=ov, interface="pml")
    r = S.solve(to_dev(b, S), c.tol, restart=c.restart)
    x = r.x.cpu().numpy()
    assert r.converged.all()
    assert rel(x, u) < 1e-6, rel(x, u)
    M = ooras.ORAS(F, c.parts, ov, interface="pml")
    _, it, ok, _ = krylov.fgmres(lambda v: A @ v, lambda v: M.apply(v.reshape(F.shape)).reshape(-1),
                                 b[0].ravel(), c.tol, c.restart, c.maxit)
    assert ok and abs(int(r.iters[0]) - it) <= 1, (r.iters, it)


@pytest.mark.parametrize("mixed", [False, True])
def test_multi_rhs_small_model(mixed):
    need_gpu()
    w = wl.small_random((24, 22, 20), npml=4, q=90.0, nsrc=5, seed=12, parts=(2, 2, 2))
    say(f"small multi-rhs mixed={mixed}")
    b = op.point_sources(oracle_fields(w), w.sources)
    u, A = _direct(w, b)
    prec = 1 if mixed else 2
    S = setup(w, prec=prec, parts=w.parts)
    tol = 1e-6 if mixed else 1e-8
    r = S.solve(to_dev(b, S), tol, restart=20)
    x = r.x.cpu().numpy()
    assert r.converged.all()
    for c in range(b.shape[0]):
        res = np.linalg.norm(A @ x[c].ravel() - b[c].ravel()) / np.linalg.norm(b[c])
        assert res <= tol * 1.0001, (c, res)
    assert rel(x, u) < (1e-4 if mixed else 1e-6), rel(x, u)


def test_pseudo_block_equals_single_columns():
    need_gpu()
    w = wl.small_random((18, 16, 14), npml=3, q=60.0, nsrc=3, seed=13, parts=(2, 2, 1))
    say("pseudo-block vs single")
    b = op.point_sources(oracle_fields(w), w.sources)
    S = setup(w, prec=2, parts=w.parts)
    xb = S.solve(to_dev(b, S), 1e-9).x.cpu().numpy()
    for c in range(3):
        xs = S.solve(to_dev(b[c:c + 1], S), 1e-9).x.cpu().numpy()
        assert np.abs(xs[0] - xb[c]).max() <= 1e-13 * np.abs(xb[c]).max()


def test_zero_column_warm_start_and_conjugate():
    need_gpu()
    w = wl.small_random((16, 15, 14), npml=3, q=70.0, nsrc=2, seed=14, parts=(2, 1, 2))
    say("zero column / x0 / conj")
    F = oracle_fields(w)
    b = op.point_sources(F, w.sources)
    b = np.concatenate([b, np.zeros_like(b[:1])])
    u, A = _direct(w, b)
    S = setup(w, prec=2, parts=w.parts)
    r = S.solve(to_dev(b, S), 1e-10)
    x = r.x.cpu().numpy()
    assert r.converged.all() and not np.any(x[2]) and r.iters[2] == 0
    assert rel(x[:2], u[:2]) < 1e-7
    # warm start from the solution: converges without iterating
    r2 = S.solve(to_dev(b, S), 1e-9, x0=r.x)
    assert r2.total_iters == 0 and r2.converged.all()
    # adjoint: A conj(x) = conj(b)
    g = rand_field((w.nz, w.ny, w.nx), 1, 5)
    rc = S.solve(to_dev(g, S), 1e-10, conj=True).x.cpu().numpy()
    ref = np.conj(direct.solve(A, F.shape, np.conj(g)))
    assert rel(rc, ref) < 1e-7


def test_not_converged_warning_and_maxit():
    need_gpu()
    w = wl.small_random((16, 16, 16), npml=3, seed=15, parts=(2, 2, 2))
    b = op.point_sources(oracle_fields(w), w.sources)
    S = setup(w, prec=2, parts=w.parts)
    r = S.solve(to_dev(b, S), 1e-12, restart=2, maxit=3)
    assert r.status == 100 and not r.converged.any() and r.total_iters == 3


def test_krylov_and_basis_precisions():
    """opts.krylov_in_prec / z_prec on complex64 factors: every combination
    meets the FP64 residual bar; a basis stored in complex128 holds the
    complex64 local solutions exactly, so the pairs that differ only in the
    storage of Z give bitwise equal results; the paper's single-precision
    setting (factors in single, Krylov in double: A z_j in complex128)
    reaches an FP64 tolerance."""
    need_gpu()
    from paper_2110_15113_amd import oras
    w = wl.small_random((24, 22, 20), npml=4, q=90.0, nsrc=4, seed=21, parts=(2, 2, 2))
    say("krylov / basis precisions on c64 factors")
    b = op.point_sources(oracle_fields(w), w.sources)
    u, A = _direct(w, b)
    S = setup(w, prec=1, parts=w.parts)
    bd = to_dev(b, S)
    tol = 1e-6
    out = {}
    for kp, zp in ((0, 0), (1, 1), (1, 2), (2, 2), (2, 1)):
        r = S.solve(bd, tol, restart=20, krylov_in_prec=kp, z_prec=zp)
        assert r.converged.all(), (kp, zp)
        x = r.x.cpu().numpy()
        for c in range(b.shape[0]):
            res = np.linalg.norm(A @ x[c].ravel() - b[c].ravel()) / np.linalg.norm(b[c])
            assert res <= tol * 1.0001, (kp, zp, c, res)
        assert rel(x, u) < 1e-4, (kp, zp, rel(x, u))
        out[kp, zp] = (x, r.iters.copy())
    for a, c in (((0, 0), (1, 1)), ((1, 1), (1, 2)), ((2, 2), (2, 1))):
        assert np.array_equal(out[a][0], out[c][0]), (a, c)
        assert np.array_equal(out[a][1], out[c][1]), (a, c)
    r = S.solve(bd, 1e-10, restart=20, maxit=400, krylov_in_prec=2, z_prec=2)
    assert r.converged.all()
    x = r.x.cpu().numpy()
    for c in range(b.shape[0]):
        res = np.linalg.norm(A @ x[c].ravel() - b[c].ravel()) / np.linalg.norm(b[c])
        assert res <= 1e-10 * 1.0001, (c, res)
    assert rel(x, u) < 1e-7, rel(x, u)
    # complex64 work needs a complex64 context
    S2 = setup(w, prec=2, parts=w.parts)
    bd2 = to_dev(b, S2)
    for kp, zp in ((1, 0), (0, 1)):
        with pytest.raises(oras.OrasError):
            S2.solve(bd2, tol, krylov_in_prec=kp, z_prec=zp)
    r0 = S2.solve(bd2, tol, restart=20)
    r1 = S2.solve(bd2, tol, restart=20, krylov_in_prec=2, z_prec=2)
    assert torch.equal(r0.x, r1.x)
