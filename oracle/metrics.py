"""Wavefield error measure Err (oracle side).  TEST INFRASTRUCTURE.

Paper eq. (eqerror): Err = |W Re(u_ref - u)| / |W Re(u_ref)| +
|W Im(u_ref - u)| / |W Im(u_ref)| with l1 norms, W a diagonal linear gain with
distance from the source, and the points nearest the source muted.
Reading: W_ii = r_i (distance in metres), mute r < ``mute`` grid steps.
"""
from __future__ import annotations

import numpy as np


def err(u_ref: np.ndarray, u: np.ndarray, src, h: float, mute: float = 4.0,
        region=None) -> float:
    nz, ny, nx = u.shape
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = h * np.sqrt((ii - src[0]) ** 2 + (jj - src[1]) ** 2 + (kk - src[2]) ** 2)
    W = np.where(r < mute * h, 0.0, r)
    if region is not None:
        W = W * region
    d = u_ref - u
    return float(np.sum(np.abs(W * d.real)) / np.sum(np.abs(W * u_ref.real))
                 + np.sum(np.abs(W * d.imag)) / np.sum(np.abs(W * u_ref.imag)))
