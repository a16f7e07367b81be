"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/oras.h declares, validates arguments before touching
a device, and its own weight table matches the oracle's fit."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from oracle import stencil_table as st

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2110_15113_amd import oras
    return oras


def test_library_exports_every_declared_symbol():
    oras = _lib()
    L = oras.lib()
    hdr = open(os.path.join(ROOT, "include", "oras.h")).read()
    names = set(re.findall(r"\b(oras_[a-z_A-Z]+)\s*\(", hdr))
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert names <= set(oras.SIGNATURES), names - set(oras.SIGNATURES)


def test_weight_table_matches_oracle_fit():
    """Parity of the library's host fitter with the oracle's (independent
    implementations of the same least-squares problem)."""
    oras = _lib()
    G, tab = oras.weight_table()
    assert np.allclose(G, st.g_grid(), rtol=0, atol=1e-12)
    ref = st.table()
    assert np.abs(tab - ref).max() < 1e-9
    assert np.abs(tab[:, 0] + tab[:, 1] + tab[:, 2] - 1).max() < 1e-15


def test_host_only_context_validates_before_device():
    oras = _lib()
    L = oras.lib()
    ctx = ct.c_void_p()
    assert L.oras_create(ct.byref(ctx), -1, None) == 0
    try:
        g = oras.Grid(16, 16, 16, 25.0, 4, 0)
        p = oras.Pml(1e-3, 2, 0.0)
        fake = ct.c_void_p(0x1000)
        # argument errors are reported before any device call
        assert L.oras_assemble(ctx, None, fake, None, 1.0, ct.byref(p), 2) == 1
        bad = oras.Grid(2, 16, 16, 25.0, 4, 0)
        assert L.oras_assemble(ctx, ct.byref(bad), fake, None, 1.0, ct.byref(p), 2) == 1
        thick = oras.Grid(16, 16, 16, 25.0, 8, 0)
        assert L.oras_assemble(ctx, ct.byref(thick), fake, None, 1.0, ct.byref(p), 2) == 1
        assert L.oras_assemble(ctx, ct.byref(g), fake, None, -1.0, ct.byref(p), 2) == 1
        assert L.oras_assemble(ctx, ct.byref(g), fake, None, 1.0, ct.byref(p), 7) == 1
        badp = oras.Pml(2.0, 2, 0.0)
        assert L.oras_assemble(ctx, ct.byref(g), fake, None, 1.0, ct.byref(badp), 2) == 1
        huge = oras.Grid(4096, 4096, 4096, 25.0, 4, 0)
        assert L.oras_assemble(ctx, ct.byref(huge), fake, None, 1.0, ct.byref(p), 2) == 3
        # valid arguments but no device in this context
        assert L.oras_assemble(ctx, ct.byref(g), fake, None, 1.0, ct.byref(p), 2) == 4
        assert b"no device" in L.oras_last_error(ctx)
        # state errors
        parts = (ct.c_int * 3)(2, 2, 2)
        assert L.oras_factor_subdomains(ctx, parts, 2, 2) == 2
        assert L.oras_factor_subdomains(ctx, parts, 9, 2) == 1
        assert L.oras_factor_subdomains(ctx, parts, 2, 5) == 1
        # interface descriptors are checked before the state
        pml = oras.Interface(oras.IFACE_PML, 2, 0.3)
        assert L.oras_factor_subdomains_ex(ctx, parts, 2, 2, ct.byref(pml)) == 2
        for bad_if, ov in ((oras.Interface(7, 2, 0.3), 2), (oras.Interface(oras.IFACE_PML, 2, 1.5), 2),
                           (oras.Interface(oras.IFACE_PML, 0, 0.3), 2),
                           (oras.Interface(oras.IFACE_PML, 2, 0.3), 0)):
            assert L.oras_factor_subdomains_ex(ctx, parts, ov, 2, ct.byref(bad_if)) == 1
        assert L.oras_factor_subdomains_ex(ctx, parts, 2, 2, None) == 2
        opts = oras.SolveOpts(30, 100, 0, 0)
        assert L.oras_solve(ctx, fake, fake, 1, 1e-6, ct.byref(opts), None) == 2
        assert L.oras_solve(ctx, fake, fake, 1, 0.0, ct.byref(opts), None) == 1
        assert L.oras_solve(ctx, fake, fake, 0, 1e-6, ct.byref(opts), None) == 1
        assert L.oras_solve(ctx, fake, fake, 257, 1e-6, ct.byref(opts), None) == 1
        bado = oras.SolveOpts(0, 100, 0, 0)
        assert L.oras_solve(ctx, fake, fake, 1, 1e-6, ct.byref(bado), None) == 1
        flg = oras.SolveOpts(30, 100, 64, 0)
        assert L.oras_solve(ctx, fake, fake, 1, 1e-6, ct.byref(flg), None) == 1
        # precisions of A z_j and of Z: values first, then the missing state
        for kp, zp in ((3, 0), (0, 3), (-1, 0), (0, 5)):
            o = oras.SolveOpts(30, 100, 0, kp, zp)
            assert L.oras_solve(ctx, fake, fake, 1, 1e-6, ct.byref(o), None) == 1
        for kp, zp in ((1, 0), (2, 2), (1, 2), (2, 1)):
            o = oras.SolveOpts(30, 100, 0, kp, zp)
            assert L.oras_solve(ctx, fake, fake, 1, 1e-6, ct.byref(o), None) == 2
        assert L.oras_apply_M(ctx, fake, fake, 1) == 2
        assert L.oras_apply_A(ctx, fake, fake, 1, 2) == 2
        assert L.oras_set_m(ctx, fake) == 2
        assert L.oras_gradient(ctx, fake, fake, 1, fake) == 2
        idx = (ct.c_int * 3)(1, 2, 3)
        assert L.oras_point_sources(ctx, idx, None, 1, fake) == 2
        # BLR compression: arguments first, then the missing factors
        assert L.oras_compress_factors(ctx, -1e-3, 8, None) == 1
        assert L.oras_compress_factors(ctx, 1.0, 8, None) == 1
        assert L.oras_compress_factors(ctx, float("nan"), 8, None) == 1
        assert L.oras_compress_factors(ctx, 1e-3, 1, None) == 1
        assert L.oras_compress_factors(ctx, 1e-3, 9, None) == 1
        assert L.oras_compress_factors(ctx, 1e-3, 8, None) == 2
        assert L.oras_blr_ranks(ctx, 0, 0, None, 0, None) == 2
        assert L.oras_factor_stats(ctx, None, None, None, None, 0, None) == 2
    finally:
        L.oras_destroy(ctx)
    assert L.oras_create(None, 0, None) == 1
    L.oras_destroy(None)


def test_weight_table_capacity_check():
    L = _lib().lib()
    cnt = ct.c_int()
    assert L.oras_weight_table(None, 0, None, None, ct.byref(cnt)) == 0
    buf = (ct.c_double * 7)()
    assert L.oras_weight_table(buf, 1, None, None, None) == 1
