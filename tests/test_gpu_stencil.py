"""Parity of the matrix-free 27-point apply with the oracle's assembled rows,
element by element (paper sec. 2.3, FDFD stencil).

The apply forms each row's coefficients from node fields and the 1D PML
profiles inside the kernel, with a reduced form on tiles the PML does not
reach.  The grids below are sized so that both kinds of tile run in one apply (8 x 8
x 16 tiles: with npml = 3 the nodes 4 .. n - 5 use only unit profile values,
so the first grid has PML-free tiles at planes 16 .. 31), with ragged tiles
on every axis, and one grid has no PML at all.  The chunk widths differ by
kind (32 right-hand sides on PML tiles, 16 elsewhere in single precision), so
the right-hand-side counts cover full and partial chunks of both.  The bar is per
entry, relative to sum_e |c_e| |x_e| of that row (the size of the terms the
entry sums), so a wrong coupling in one row or one tile fails on its own.
"""
import numpy as np
import pytest

from oracle import operator as op
from paper_2110_15113_amd import workloads as wl

from gpu_util import EPS32, need_gpu, oracle_fields, rand_field, say, setup, to_dev

pytestmark = pytest.mark.gpu

FP64_ROW = 1e-12
# x, the node fields and the coefficient arithmetic in single precision: a
# few roundings per term and 27 terms per row
FP32_ROW = 32 * EPS32

CASES = [
    dict(n=(40, 36, 38), npml=3, q=80.0, nrhs=1, seed=31),    # PML and interior tiles
    dict(n=(37, 20, 19), npml=2, q=None, nrhs=13, seed=32),   # ragged tiles, 2 chunks
    dict(n=(21, 18, 11), npml=0, q=50.0, nrhs=40, seed=33),   # no PML: interior tiles only
    dict(n=(33, 17, 21), npml=2, q=70.0, nrhs=50, seed=37),   # chunks of 32, 16 and 8 RHS
    dict(n=(18, 17, 9), npml=2, q=None, nrhs=256, seed=38),   # the widest block
]


def _row_err(got, ref, scale):
    return float((np.abs(got - ref) / scale).max())


@pytest.mark.parametrize("case", CASES)
def test_matrix_free_apply_matches_oracle_rows(case):
    need_gpu()
    w = wl.small_random(case["n"], npml=case["npml"], q=case["q"], seed=case["seed"])
    say(f"matrix-free apply {w.name} nrhs={case['nrhs']}")
    S = setup(w, prec=1)          # single-precision stencil (plus the FP64 one)
    x = rand_field((w.nz, w.ny, w.nx), case["nrhs"], case["seed"] + 100)
    C = op.row_coeffs(oracle_fields(w))
    ref = op.apply_coeffs(C, x)
    scale = op.apply_coeffs(np.abs(C), np.abs(x)).real
    assert scale.min() > 0
    y128 = S.apply_A(to_dev(x, S), prec=2).cpu().numpy()
    e128 = _row_err(y128, ref, scale)
    y64 = S.apply_A(to_dev(x, S), prec=1).cpu().numpy()
    e64 = _row_err(y64, ref, scale)
    say(f"  row error: FP64 {e128:.2e}, FP32 {e64:.2e}")
    assert e128 < FP64_ROW
    assert e64 < FP32_ROW


def test_matrix_free_apply_after_set_m():
    """A new squared slowness rebuilds the node fields the apply reads."""
    need_gpu()
    import torch
    w = wl.small_random((34, 19, 18), npml=2, q=60.0, seed=34)
    S = setup(w, prec=1)
    rng = np.random.default_rng(35)
    m = (1.0 / w.vel ** 2) * (1.0 + 0.2 * rng.random(w.vel.shape))
    S.set_m(torch.as_tensor(m, device=S.device))
    x = rand_field((w.nz, w.ny, w.nx), 3, 36)
    F = op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml, m=m)   # weights kept from vel
    C = op.row_coeffs(F)
    ref = op.apply_coeffs(C, x)
    scale = op.apply_coeffs(np.abs(C), np.abs(x)).real
    y128 = S.apply_A(to_dev(x, S), prec=2).cpu().numpy()
    y64 = S.apply_A(to_dev(x, S), prec=1).cpu().numpy()
    assert _row_err(y128, ref, scale) < FP64_ROW
    assert _row_err(y64, ref, scale) < FP32_ROW
