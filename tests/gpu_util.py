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
