"""The allocation-free variant of the 27-point apply (for callers that cannot
allocate device memory) against oras_apply_A, through the C ABI: two calls in
a row, the second with fewer right-hand sides, in both precisions, and a size
beyond the fixed scratch refused."""
import numpy as np
import pytest
import torch

from paper_2110_15113_amd import workloads as wl

from gpu_util import need_gpu, rand_field, say, setup, to_dev

pytestmark = pytest.mark.gpu


def test_apply_A_noalloc_matches_apply_A():
    need_gpu()
    from paper_2110_15113_amd import oras
    w = wl.small_random((21, 17, 13), npml=3, q=70.0, seed=51)
    say("apply_A_noalloc")
    S = setup(w, prec=oras.C64)              # complex64 stencil plus the FP64 one
    for prec in (oras.C128, oras.C64):
        for nrhs, seed in ((7, 1), (3, 2)):  # the second call is smaller
            x = to_dev(rand_field((w.nz, w.ny, w.nx), nrhs, seed), S)
            ref = S.apply_A(x, prec=prec)
            y = torch.full_like(x, float("nan"))
            got = S.apply_A_noalloc(x, y, prec=prec)
            assert got.data_ptr() == y.data_ptr()
            assert torch.equal(got, ref), (prec, nrhs)
    S.close()
    # staging above the fixed scratch is refused before any device work
    cap = int(oras.lib().oras_noalloc_scratch_bytes())
    w2 = wl.small_random((40, 40, 40), npml=3, q=70.0, seed=52)
    S = setup(w2, prec=oras.C64)
    nrhs = 32
    assert w2.nx * w2.ny * w2.nz * nrhs * (16 + 16 + 8) > cap
    x = torch.zeros((nrhs,) + S.shape, dtype=torch.complex128, device=S.device)
    y = torch.zeros_like(x)
    with pytest.raises(oras.OrasError, match="staging") as e:
        S.apply_A_noalloc(x, y, prec=oras.C64)
    assert e.value.code == 1
    assert int(torch.count_nonzero(y)) == 0
    S.close()
