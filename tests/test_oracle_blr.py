"""Pins of the oracle's block low-rank local solves (sec. 3: BLR factors with
threshold eps_BLR; Table 4)."""
import numpy as np
import pytest

from oracle import blr, direct, krylov, operator as op, oras
from paper_2110_15113_amd import workloads as wl


def _crand(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def test_cross_approx_recovers_exact_low_rank():
    rng = np.random.default_rng(0)
    for r in (1, 2, 5):
        M = _crand(rng, 20, r) @ _crand(rng, r, 17)
        U, V = blr.cross_approx(M, 1e-12 * np.abs(M).max(), 8)
        assert U.shape[1] == r and V.shape[0] == r
        assert np.abs(U @ V - M).max() <= 1e-12 * np.abs(M).max()


def test_cross_approx_rank_one_closed_form():
    """One step: u = M[:, b], v = M[a, :] / M[a, b] at the largest entry."""
    rng = np.random.default_rng(1)
    x, y = _crand(rng, 6), _crand(rng, 5)
    M = np.outer(x, y)
    a, b = np.unravel_index(np.argmax(np.abs(M)), M.shape)
    U, V = blr.cross_approx(M, 1e-12 * np.abs(M).max(), 3)
    assert U.shape[1] == 1
    assert np.array_equal(U[:, 0], M[:, b]) and np.array_equal(V[0], M[a, :] / M[a, b])


def test_cross_approx_diagonal_order_and_stopping():
    """On a diagonal matrix complete pivoting takes the entries in decreasing
    modulus and stops at the first one below the threshold."""
    d = np.array([0.3, -5.0, 2e-4, 1.0j, 0.05, 7e-3])
    M = np.diag(d)
    U, V = blr.cross_approx(M, 1e-2, 6)
    assert U.shape[1] == 4                      # 5, 1, 0.3, 0.05 exceed 1e-2
    picked = [int(np.argmax(np.abs(U[:, t]))) for t in range(4)]
    assert picked == [1, 3, 0, 4]
    assert blr.cross_approx(M, 1e-2, 3) is None  # would need rank 4
    assert np.abs(M - U @ V).max() == pytest.approx(7e-3)


def test_patches_partition_the_plane():
    for sx, sy, pm in [(24, 24, 8), (22, 19, 8), (7, 30, 8), (5, 5, 8), (28, 28, 7)]:
        g = blr.patches(sx, sy, pm)
        allidx = np.sort(np.concatenate(g))
        assert np.array_equal(allidx, np.arange(sx * sy))
        assert max(len(x) for x in g) <= pm * pm
        for x in g:   # rectangles, plane order inside
            xs, ys = x % sx, x // sx
            assert len(x) == (xs.max() - xs.min() + 1) * (ys.max() - ys.min() + 1)
            assert np.all(np.diff(x) > 0)


def _sub_matrix(n=(14, 13, 12), parts=(2, 2, 1), ov=2, seed=3, j=1, q=60.0):
    w = wl.small_random(n, npml=2, q=q, seed=seed)
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml)
    s = oras.partition((F.nx, F.ny, F.nz), parts, ov)[j]
    B = op.csr_from_coeffs(oras.local_coeffs(F, s))
    return F, s, B, tuple(s.hi[a] - s.lo[a] for a in range(3))


def test_exact_plane_recursion_is_the_local_solve():
    F, s, B, (sx, sy, sz) = _sub_matrix()
    rng = np.random.default_rng(4)
    b = _crand(rng, B.shape[0], 3)
    ref = direct.BlockTridiagLU(B, sx * sy, sz).solve(b)
    for eps in (None, 0.0):
        x = blr.PlaneSolver(B, sx, sy, sz, eps, pmax=4).solve(b)
        assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max(), eps


def test_blr_planes_meet_the_entry_bound_and_compress():
    F, s, B, (sx, sy, sz) = _sub_matrix(n=(26, 26, 10), parts=(1, 1, 1), ov=0, q=None, j=0)
    eps = 1e-3
    sol_exact = blr.PlaneSolver(B, sx, sy, sz, None, pmax=8)
    sol = blr.PlaneSolver(B, sx, sy, sz, eps, pmax=8)
    for k in (0, sz // 2, sz - 1):
        S, Sb = sol_exact.inv[k], sol.inv[k]
        err = np.abs(Sb.matrix() - S).max()
        assert err <= eps * np.abs(S).max() * (1 + 1e-12)
        assert Sb.stored_entries() < 0.6 * S.size
        assert np.all(Sb.rank[~np.eye(len(Sb.groups), dtype=bool)] >= 0)   # nothing left dense


def test_blr_oras_fgmres_reaches_the_direct_solution():
    w = wl.config1()
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml)
    A = op.assemble(F)
    b = op.point_sources(F, w.sources)[0]
    x_ref = direct.solve(A, F.shape, b[None])[0]
    its = {}
    for eps in (None, 1e-3):
        M = blr.OrasBLR(F, w.parts, w.overlap, eps)
        x, it, ok, _ = krylov.fgmres(lambda v: A @ v,
                                     lambda v: M.apply(v.reshape(F.shape)).reshape(-1),
                                     b.reshape(-1), 1e-10, 30, 300)
        assert ok
        assert np.linalg.norm(x - x_ref.reshape(-1)) <= 1e-7 * np.linalg.norm(x_ref)
        its[eps] = it
    Md = oras.ORAS(F, w.parts, w.overlap)
    v = np.random.default_rng(5).normal(size=F.shape) + 0j
    assert np.abs(blr.OrasBLR(F, w.parts, w.overlap, None).apply(v) - Md.apply(v)).max() \
        <= 1e-10 * np.abs(Md.apply(v)).max()
    assert its[1e-3] <= its[None] + 5, its
