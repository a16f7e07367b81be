"""Shared helpers of the GPU parity tests (inputs and comparison only)."""
import numpy as np
import pytest
import torch

from oracle import operator as op


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def solver():
    from paper_2110_15113_amd import oras
    return oras


def setup(w, prec=2, parts=None, overlap=None, fprec=None, interface="robin"):
    """Assemble (and optionally factor) workload ``w`` on the GPU."""
    oras = solver()
    S = oras.Solver(0)
    dev = S.device
    vel = torch.as_tensor(w.vel, device=dev)
    Q = None if w.Q is None else torch.as_tensor(w.Q, device=dev)
    S.assemble(vel, w.h, w.npml, w.omega, Q, prec=prec)
    if parts is not None:
        S.factor(parts, w.overlap if overlap is None else overlap, prec if fprec is None else fprec,
                 interface=interface)
    return S


def oracle_fields(w):
    return op.make_fields(w.vel, w.Q, w.omega, w.h, w.npml)


def rand_field(shape, nrhs, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(nrhs,) + tuple(shape)) + 1j * rng.normal(size=(nrhs,) + tuple(shape))


def to_dev(a, S):
    return torch.as_tensor(np.ascontiguousarray(a), device=S.device)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def say(msg):
    print(msg, flush=True)


# Element-wise bars of the ORAS apply.  A subdomain writes only its owned box
# (Boolean partition of unity, sec. 2.1), so the apply is compared box by box:
# the largest error in an owned box, relative to the largest reference entry
# of the same box and column.  A defect confined to one subdomain (a wrong
# plane, row or sign) then fails even where a global L2 ratio would not see it.
EPS32 = 2.0 ** -24   # unit roundoff of IEEE single precision
EPS64 = 2.0 ** -53   # unit roundoff of IEEE double precision
FP32_BOX = 256 * EPS32   # complex FP32 factors and products (1.5e-5)
FP64_BOX = 1e-12         # complex FP64 factors and products
# complex FP32 BLR inverses against the oracle's BLR recursion (pivots chosen
# in FP64 there): a block whose rank or pivot order differs holds a different,
# equally valid approximation whose entries differ by up to eps_BLR times the
# plane's largest entry, so the bar is a fraction of eps_BLR, not of eps32
BLR32_BOX = 0.1          # times eps_BLR


def box_err(got, ref, parts, overlap):
    """max over owned boxes b and columns c of
    max_{i in b} |got_c,i - ref_c,i| / max_{i in b} |ref_c,i|.
    got, ref: (nrhs, nz, ny, nx)."""
    from oracle import oras as ooras
    nz, ny, nx = ref.shape[1:]
    worst = 0.0
    for s in ooras.partition((nx, ny, nz), parts, overlap):
        sl = (slice(None),) + tuple(slice(s.olo[a], s.ohi[a]) for a in (2, 1, 0))
        d = np.abs(got[sl] - ref[sl]).reshape(ref.shape[0], -1).max(axis=1)
        m = np.abs(ref[sl]).reshape(ref.shape[0], -1).max(axis=1)
        worst = max(worst, float((d / np.maximum(m, 1e-300)).max()))
    return worst
