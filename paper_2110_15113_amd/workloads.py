"""Seeded synthetic inputs for the ORAS-FGMRES Helmholtz path.

This module only draws numbers: velocity and attenuation models, source and
receiver grid positions, and the solver settings of each named workload.  It
holds none of the method's arithmetic (no stencil, no PML, no solver), so both
the HIP path and the CPU oracle may consume what it produces.

The paper's benchmark models (SEG/EAGE overthrust, GO_3D_OBS, the CBS
reference fields) are not available; each workload below is a synthetic stand
in of the same kind (smooth heterogeneous crust, flat layers with relief,
attenuation through a quality factor Q, point sources on a surface grid),
sized for one GPU.  Paper, section 3.1 (benchmarks and experimental design).

Conventions shared by every generator:
  * arrays are shaped (nz, ny, nx), C order, x fastest, k = depth index;
  * the PML occupies ``npml`` nodes on all six faces; the "physical region"
    is the rest;
  * ``numpy.random.Generator(PCG64(seed))`` with ``seed`` = workload number;
  * a "smooth random field" is white N(0,1) noise filtered in the Fourier
    domain by exp(-sigma^2 |kappa|^2 / 2) with sigma = ell / sqrt(2) (its
    covariance is exp(-r^2 / (2 ell^2))), then min-max normalised and mapped
    linearly onto the requested velocity range.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    npml: int
    freq: float
    vel: np.ndarray                      # (nz, ny, nx) float64, m/s
    Q: Optional[np.ndarray]              # (nz, ny, nx) float64 or None
    sources: List[Tuple[int, int, int]]  # (i, j, k) grid indices
    parts: Tuple[int, int, int]          # subdomains along (x, y, z)
    overlap: int
    krylov_prec: str                     # "c128" or "mixed"
    tol: float
    restart: int
    maxit: int = 400
    receivers: Optional[List[Tuple[int, int, int]]] = None
    vel_start: Optional[np.ndarray] = None
    notes: dict = field(default_factory=dict)

    @property
    def omega(self) -> float:
        return 2.0 * np.pi * self.freq

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def digest(self) -> str:
        """SHA-256 over the model arrays and source list (determinism check)."""
        hs = hashlib.sha256()
        hs.update(np.ascontiguousarray(self.vel).tobytes())
        if self.Q is not None:
            hs.update(np.ascontiguousarray(self.Q).tobytes())
        hs.update(np.asarray(self.sources, dtype=np.int64).tobytes())
        return hs.hexdigest()


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def smooth_field(shape, h: float, ell: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian-correlated random field, min-max normalised to [0, 1]."""
    white = rng.standard_normal(shape)
    sigma = ell / np.sqrt(2.0)
    spec = np.fft.fftn(white)
    kk = [2.0 * np.pi * np.fft.fftfreq(s, d=h) for s in shape]
    grids = np.meshgrid(*kk, indexing="ij")
    k2 = sum(g * g for g in grids)
    f = np.real(np.fft.ifftn(spec * np.exp(-0.5 * sigma * sigma * k2)))
    f -= f.min()
    mx = f.max()
    return f / mx if mx > 0 else f


def surface_grid(npml: int, nphys_x: int, nphys_y: int, a: int, b: int, depth: int):
    """a x b regular grid of (i, j, k) positions over the physical region."""
    out = []
    for jb in range(b):
        for ia in range(a):
            i = npml + int(np.floor((ia + 0.5) * nphys_x / a))
            j = npml + int(np.floor((jb + 0.5) * nphys_y / b))
            out.append((i, j, npml + depth))
    return out


def config1() -> Workload:
    """32^3, h=25 m, 6-node PML, velocity linear in depth 1500->3000 m/s, 5 Hz,
    one source at the grid centre, 2x2x2 subdomains, complex128, tol 1e-8."""
    nx = ny = nz = 32
    k = np.arange(nz, dtype=np.float64)
    c = 1500.0 + 1500.0 * k / (nz - 1)
    vel = np.broadcast_to(c[:, None, None], (nz, ny, nx)).copy()
    return Workload("c1-gradient-32", nx, ny, nz, 25.0, 6, 5.0, vel, None,
                    [(16, 16, 16)], (2, 2, 2), 2, "c128", 1e-8, 30)


def config2() -> Workload:
    """128^3, h=20 m, 8-node PML, smooth field (ell=300 m) in 1500-4500 m/s plus
    a 5000 m/s layer at 60% depth, Q=150, 7 Hz, 16 surface sources (4x4),
    4x4x4 subdomains, complex128, tol 1e-6."""
    nx = ny = nz = 128
    npml = 8
    rng = _rng(2)
    f = smooth_field((nz, ny, nx), 20.0, 300.0, rng)
    vel = 1500.0 + 3000.0 * f
    k0 = int(np.floor(0.6 * nz))
    vel[k0:k0 + 8] = 5000.0
    Q = np.full_like(vel, 150.0)
    np_ = nx - 2 * npml
    src = surface_grid(npml, np_, np_, 4, 4, 2)
    return Workload("c2-random-128", nx, ny, nz, 20.0, npml, 7.0, vel, Q, src,
                    (4, 4, 4), 2, "c128", 1e-6, 30,
                    notes={"layer": [k0, k0 + 8]})


def config3() -> Workload:
    """192x192x96, h=25 m, 8-node PML, 6 flat layers (1500+700 l m/s,
    Q=100+20 l) with smooth relief of +/-50 m on each interface, 6 Hz, 64
    surface sources (8x8), 8x8x4 subdomains of 24^3, mixed precision, tol 1e-6,
    restart 20."""
    nx, ny, nz = 192, 192, 96
    h = 25.0
    npml = 8
    rng = _rng(3)
    nlay = 6
    z = np.arange(nz, dtype=np.float64) * h
    zphys0 = npml * h
    zphys1 = (nz - 1 - npml) * h
    nominal = zphys0 + (zphys1 - zphys0) * np.arange(1, nlay) / nlay
    layer = np.zeros((nz, ny, nx), dtype=np.int64)
    for iface in range(nlay - 1):
        relief = smooth_field((ny, nx), h, 500.0, rng)
        relief = (relief * 2.0 - 1.0) * 50.0
        depth = nominal[iface] + relief                 # (ny, nx)
        layer += (z[:, None, None] >= depth[None, :, :]).astype(np.int64)
    vel = 1500.0 + 700.0 * layer.astype(np.float64)
    Q = 100.0 + 20.0 * layer.astype(np.float64)
    src = surface_grid(npml, nx - 2 * npml, ny - 2 * npml, 8, 8, 2)
    return Workload("c3-layered-192x192x96", nx, ny, nz, h, npml, 6.0, vel, Q, src,
                    (8, 8, 4), 2, "mixed", 1e-6, 20)


def config4() -> Workload:
    """96^3, h=25 m, 8-node PML, 2500 m/s background plus 10 Gaussian anomalies
    (+/-10 %, e-folding radius 150 m), 5 Hz, 32 sources (4x8) and 400
    receivers (20x20) at depth index 4 below the PML, 4x4x4 subdomains,
    complex128, tol 1e-8.  ``vel`` is the true model, ``vel_start`` the start."""
    nx = ny = nz = 96
    h = 25.0
    npml = 8
    rng = _rng(4)
    R = 150.0
    lo = npml * h + R
    hi = (nx - 1 - npml) * h - R
    centres = rng.uniform(lo, hi, size=(10, 3))
    signs = rng.choice([-1.0, 1.0], size=10)
    zz, yy, xx = np.meshgrid(*(np.arange(s) * h for s in (nz, ny, nx)), indexing="ij")
    pert = np.zeros((nz, ny, nx))
    for q in range(10):
        cx, cy, cz = centres[q]
        r2 = (xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2
        pert += 0.10 * signs[q] * np.exp(-r2 / (R * R))
    vel = 2500.0 * (1.0 + pert)
    nphys = nx - 2 * npml
    src = surface_grid(npml, nphys, nphys, 4, 8, 2)
    rec = surface_grid(npml, nphys, nphys, 20, 20, 4)
    return Workload("c4-anomalies-96", nx, ny, nz, h, npml, 5.0, vel, None, src,
                    (4, 4, 4), 2, "c128", 1e-8, 30, receivers=rec,
                    vel_start=np.full_like(vel, 2500.0))


def config5(n: int = 160) -> Workload:
    """160^3 (4.1 M unknowns), h=20 m, 10-node PML, smooth field (ell=300 m) in
    1500-5500 m/s, Q=100, 8 Hz, 32 sources (4x8), 8x8x8 subdomains of 20^3,
    mixed precision, restart 20, tol 1e-6.  n < 160 draws a smaller replica
    with the same recipe (same h, PML, frequency, velocity range, correlation
    length, Q and source grid) and n / 20 subdomains per axis, so the owned
    cuboids stay 20^3 (n must be a multiple of 20)."""
    if n % 20 or n < 40:
        raise ValueError("n must be a multiple of 20, at least 40")
    nx = ny = nz = n
    npml = 10
    rng = _rng(5)
    f = smooth_field((nz, ny, nx), 20.0, 300.0, rng)
    vel = 1500.0 + 4000.0 * f
    Q = np.full_like(vel, 100.0)
    nphys = nx - 2 * npml
    src = surface_grid(npml, nphys, nphys, 4, 8, 2)
    name = "c5-random-160" if n == 160 else f"c5-replica-{n}"
    return Workload(name, nx, ny, nz, 20.0, npml, 8.0, vel, Q, src,
                    (n // 20,) * 3, 2, "mixed", 1e-6, 20)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def small_random(n=(16, 16, 16), h=25.0, npml=4, freq=5.0, seed=11, q=None,
                 vmin=1500.0, vmax=3000.0, parts=(2, 2, 2), overlap=2,
                 nsrc=1) -> Workload:
    """Small seeded heterogeneous model for parity tests (sizes the oracle
    finishes in seconds).  ``n`` = (nx, ny, nz)."""
    nx, ny, nz = n
    rng = _rng(seed)
    f = smooth_field((nz, ny, nx), h, 3.0 * h, rng)
    vel = vmin + (vmax - vmin) * f
    Q = None if q is None else np.full_like(vel, float(q))
    srcs = []
    for s in range(nsrc):
        i = npml + int(rng.integers(0, max(1, nx - 2 * npml)))
        j = npml + int(rng.integers(0, max(1, ny - 2 * npml)))
        k = npml + int(rng.integers(0, max(1, nz - 2 * npml)))
        srcs.append((i, j, k))
    return Workload(f"small-{nx}x{ny}x{nz}-s{seed}", nx, ny, nz, h, npml, freq, vel, Q,
                    srcs, parts, overlap, "c128", 1e-10, 30)
