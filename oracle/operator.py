"""Discrete Helmholtz operator A and subdomain matrices B_j (oracle side).
TEST INFRASTRUCTURE.

Paper eq. (1): (Delta + k^2) u = f with k = omega / c, c complex in viscous
media; Robin or PML on the outer boundary (sec. 2, Method).  Discretised by
the compact 27-point lambda-adaptive stencil on a regular grid (sec. 2.3,
FDFD) with PML layers on every face of the grid (sec. 3.1, experimental
setup).  The paper prints neither the stencil coefficients nor the PML, Robin
or attenuation formulas; this module implements the following reading.

Conventions
  * time dependence e^{-i omega t}; outgoing waves behave like e^{+ikr};
  * A = sum_f ( -D_f^T diag(wbar_f K) D_f ) + omega^2 M, the paper's sign;
  * attenuation: 1 / c~ = (1 / c)(1 + i / (2Q)), m~ = 1 / c~^2;
  * PML: s_a(xi) = 1 + i sigma(xi) / omega, sigma = sigma_max (d / L)^2,
    d = h max(0, npml - xi, xi - (n - 1 - npml)), L = npml h,
    sigma_max = 3 c_ref ln(1 / R0) / (2 L), R0 = 1e-3, c_ref = max velocity;
    S = s_x s_y s_z and K_a = S / s_a^2 (stretched-coordinate form
    multiplied through by S, which keeps A complex symmetric);
  * nodes outside the grid are Dirichlet zeros ("ghosts"); a ghost takes the
    stencil weights of the nearest grid node;
  * the family weight at a staggered point is the mean of its support nodes'
    weights; the mass coupling of nodes i, j is
    1/2 (wm_t,i + wm_t,j) * 1/2 (m~_i + m~_j) * 1/2 (S_i + S_j),
    t = shell (face, edge, corner) of j - i; the diagonal is wm0_i m~_i S_i;
  * B_j keeps only the staggered points whose support nodes all lie in the
    box or outside the grid (fluxes across interior interfaces are cut), the
    mass couplings inside the box, and adds the Robin term
    i k_i S_i / (s_a,i h) to the diagonal once per interior face of the box
    that node i lies on (outgoing impedance d_n u = i k u), with
    k_i = omega sqrt(m~_i).

The 27 coefficients of row i are stored as C[e, ...] with e = (ez+1)*9 +
(ey+1)*3 + (ex+1) for the neighbour offset (ex, ey, ez).

Parity: pinned in tests by A = A^T, the plane-wave symbol on a periodic grid
(ties the assembly to the dispersion formulas), the homogeneous stiffness
shell coefficients, the Green's function, reciprocity, and brute-force dense
solves.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import stencil_table

FAMILIES = (  # (axes, weight index, family factor)
    ((0,), 0, 1.0), ((1,), 0, 1.0), ((2,), 0, 1.0),
    ((0, 1), 1, 0.5), ((0, 2), 1, 0.5), ((1, 2), 1, 0.5),
    ((0, 1, 2), 2, 1.0),
)


def eidx(ex: int, ey: int, ez: int) -> int:
    return (ez + 1) * 9 + (ey + 1) * 3 + (ex + 1)


OFFSETS = [(ex, ey, ez) for ez in (-1, 0, 1) for ey in (-1, 0, 1) for ex in (-1, 0, 1)]


def pml_profile(n: int, npml: int, h: float, omega: float, c_ref: float,
                R0: float = 1e-3, power: int = 2, low: bool = True, high: bool = True):
    """s(xi) on the half grid xi = -0.5, 0, 0.5, ..., n - 0.5 (index 2 xi + 1)."""
    xi = (np.arange(2 * n + 1, dtype=np.float64) - 1.0) / 2.0
    if npml <= 0:
        return np.ones_like(xi, dtype=np.complex128)
    L = npml * h
    dl = np.maximum(0.0, npml - xi) if low else np.zeros_like(xi)
    dh = np.maximum(0.0, xi - (n - 1 - npml)) if high else np.zeros_like(xi)
    d = h * np.maximum(dl, dh)
    smax = (power + 1) * c_ref * np.log(1.0 / R0) / (2.0 * L)
    sigma = smax * (d / L) ** power
    return 1.0 + 1j * sigma / omega


def interface_pml_profile(prof, n: int, lo: int, hi: int, olo: int, ohi: int, h: float,
                          omega: float, c_ref: float, R0: float = 0.3, power: int = 2):
    """One axis of a subdomain's stretching profile with PML transmission
    conditions: the global half-grid profile ``prof`` plus an interface PML in
    the overlap layers beyond the owned range [olo, ohi) on each side that is
    not a global boundary (sec. 2.2, note on the size of overlap).  Reading
    (the paper gives no interface profile): the outer PML's law on a layer of
    thickness L = (olo - lo) h (resp. (hi - ohi) h), d = h (olo - xi) (resp.
    h (xi - (ohi - 1))), sigma = sigma_max (d / L)^power with sigma_max =
    (power + 1) c_ref ln(1 / R0) / (2 L), added to the global absorption."""
    xi = (np.arange(2 * n + 1, dtype=np.float64) - 1.0) / 2.0
    sig = np.zeros_like(xi)
    for interior, L, d in ((lo > 0, (olo - lo) * h, h * np.maximum(0.0, olo - xi)),
                           (hi < n, (hi - ohi) * h, h * np.maximum(0.0, xi - (ohi - 1)))):
        if interior and L > 0:
            smax = (power + 1) * c_ref * np.log(1.0 / R0) / (2.0 * L)
            sig = sig + smax * (d / L) ** power
    return np.asarray(prof) + 1j * sig / omega


@dataclass
class Fields:
    nx: int
    ny: int
    nz: int
    h: float
    omega: float
    w: np.ndarray        # (nz, ny, nx, 7) stencil weights
    mt: np.ndarray       # (nz, ny, nx) complex squared slowness m~
    prof: tuple          # (s_x, s_y, s_z) half-grid PML profiles
    qfac: np.ndarray     # (nz, ny, nx) complex d m~ / d m  ((1 + i/2Q)^2)
    c_ref: float = 0.0   # reference velocity of the PML profiles

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    def S(self) -> np.ndarray:
        sx, sy, sz = self.prof
        return (sz[1:2 * self.nz:2][:, None, None] * sy[1:2 * self.ny:2][None, :, None]
                * sx[1:2 * self.nx:2][None, None, :])


def make_fields(vel, Q, omega, h, npml, R0=1e-3, power=2, c_ref=None,
                free_surface=False, tab=None, weights_from=None, m=None) -> Fields:
    """Node fields of the operator.  ``weights_from`` (a velocity model) freezes
    the stencil weights at another model; ``m`` overrides the real squared
    slowness (the attenuation factor from Q is still applied)."""
    vel = np.asarray(vel, dtype=np.float64)
    nz, ny, nx = vel.shape
    wv = vel if weights_from is None else np.asarray(weights_from, dtype=np.float64)
    G = 2.0 * np.pi * wv / (omega * h)
    w = stencil_table.lookup(G, tab)
    qf = np.ones_like(vel, dtype=np.complex128) if Q is None else (1.0 + 0.5j / np.asarray(Q, dtype=np.float64)) ** 2
    mreal = 1.0 / vel ** 2 if m is None else np.asarray(m, dtype=np.float64)
    mt = mreal * qf
    cr = float(np.max(wv)) if c_ref is None else float(c_ref)
    prof = (pml_profile(nx, npml, h, omega, cr, R0, power),
            pml_profile(ny, npml, h, omega, cr, R0, power),
            pml_profile(nz, npml, h, omega, cr, R0, power, low=not free_surface))
    return Fields(nx, ny, nz, h, omega, w, mt, prof, qf, cr)


def _window(F: Fields, lo, hi):
    """Per-axis global coordinates of the box extended by one layer."""
    n = (F.nx, F.ny, F.nz)
    g = [np.arange(lo[a] - 1, hi[a] + 1) for a in range(3)]
    ingrid = [(g[a] >= 0) & (g[a] < n[a]) for a in range(3)]
    inbox = [(g[a] >= lo[a]) & (g[a] < hi[a]) for a in range(3)]
    clamp = [np.clip(g[a], 0, n[a] - 1) for a in range(3)]
    return g, ingrid, inbox, clamp


def _to3(arrs):
    """Per-axis (x, y, z) 1D arrays -> broadcastable (z, y, x) arrays."""
    ax, ay, az = arrs
    return az[:, None, None], ay[None, :, None], ax[None, None, :]


def row_coeffs(F: Fields, lo=(0, 0, 0), hi=None, restrict: bool = False) -> np.ndarray:
    """27 coefficients of every row in the box [lo, hi) (x, y, z order).

    restrict=False gives the rows of the global operator A; restrict=True gives
    the subdomain matrix B_j of the box (cut fluxes, Robin faces)."""
    n = (F.nx, F.ny, F.nz)
    hi = n if hi is None else tuple(hi)
    lo = tuple(lo)
    b = [hi[a] - lo[a] for a in range(3)]
    g, ingrid, inbox, clamp = _window(F, lo, hi)
    gz, gy, gx = _to3(g)
    igz, igy, igx = _to3(ingrid)
    ibz, iby, ibx = _to3(inbox)
    in_grid = igz & igy & igx
    in_box = ibz & iby & ibx
    ok = in_box | ~in_grid
    cz, cy, cx = _to3(clamp)
    wn = F.w[cz, cy, cx]                       # (Wz, Wy, Wx, 7)
    mt = F.mt[cz, cy, cx]
    sx, sy, sz = F.prof
    Sn = sz[2 * cz + 1] * sy[2 * cy + 1] * sx[2 * cx + 1]
    Wshape = (b[2] + 2, b[1] + 2, b[0] + 2)
    C = np.zeros((27,) + Wshape, dtype=np.complex128)
    row_ok = in_box & in_grid
    h2 = F.h * F.h
    prof = (sx, sy, sz)

    for axes, widx, ffac in FAMILIES:
        dim = len(axes)
        # base window index ranges, per axis (x, y, z)
        rng = [slice(0, b[a] + 1) if a in axes else slice(1, b[a] + 1) for a in range(3)]
        base_sl = (rng[2], rng[1], rng[0])
        bshape = tuple(s.stop - s.start for s in base_sl)
        # centre half-grid indices per axis
        tcen = []
        for a in range(3):
            ga = g[a][rng[a]]
            tcen.append(2 * ga + 2 if a in axes else 2 * ga + 1)
        sc = [prof[a][tcen[a]] for a in range(3)]
        scz, scy, scx = _to3(sc)
        Scen = scz * scy * scx
        svals3 = {0: scx, 1: scy, 2: scz}
        supports = list(itertools.product((0, 1), repeat=dim))

        def shifted(arr, rho):
            off = [0, 0, 0]
            for q, a in enumerate(axes):
                off[a] = rho[q]
            sl = tuple(slice(base_sl[2 - a].start + off[a], base_sl[2 - a].stop + off[a])
                       for a in (2, 1, 0))
            return arr[sl]

        valid = np.ones(bshape, dtype=bool)
        wbar = np.zeros(bshape)
        for rho in supports:
            if restrict:
                valid &= shifted(ok, rho)
            wbar += shifted(wn[..., widx], rho)
        wbar /= len(supports)
        Wa = {}
        for a in axes:
            Wa[a] = np.where(valid, ffac * wbar * Scen / (svals3[a] ** 2) / h2, 0.0)
        dscale = 1.0 / (2 ** (dim - 1))
        for r1 in supports:
            rowmask = shifted(row_ok, r1)
            for r2 in supports:
                colmask = shifted(in_grid, r2)
                val = np.zeros(bshape, dtype=np.complex128)
                for q, a in enumerate(axes):
                    d1 = (2 * r1[q] - 1) * dscale
                    d2 = (2 * r2[q] - 1) * dscale
                    val -= Wa[a] * d1 * d2
                e = [0, 0, 0]
                for q, a in enumerate(axes):
                    e[a] = r2[q] - r1[q]
                ei = eidx(*e)
                off = [0, 0, 0]
                for q, a in enumerate(axes):
                    off[a] = r1[q]
                sl = tuple(slice(base_sl[2 - a].start + off[a], base_sl[2 - a].stop + off[a])
                           for a in (2, 1, 0))
                C[ei][sl] += np.where(rowmask & colmask, val, 0.0)

    # mass term
    om2 = F.omega ** 2
    inner = (slice(1, b[2] + 1), slice(1, b[1] + 1), slice(1, b[0] + 1))
    C[eidx(0, 0, 0)][inner] += om2 * wn[inner][..., 3] * mt[inner] * Sn[inner]
    for (ex, ey, ez) in OFFSETS:
        if (ex, ey, ez) == (0, 0, 0):
            continue
        shell = abs(ex) + abs(ey) + abs(ez)          # 1 face, 2 edge, 3 corner
        widx = 3 + shell
        js = (slice(1 + ez, b[2] + 1 + ez), slice(1 + ey, b[1] + 1 + ey),
              slice(1 + ex, b[0] + 1 + ex))
        colmask = in_box[js] if restrict else in_grid[js]
        colmask = colmask & in_grid[js]
        mu = (0.5 * (wn[inner][..., widx] + wn[js][..., widx]) * 0.5 * (mt[inner] + mt[js])
              * 0.5 * (Sn[inner] + Sn[js]))
        C[eidx(ex, ey, ez)][inner] += np.where(colmask & row_ok[inner], om2 * mu, 0.0)

    # Robin faces of the subdomain
    if restrict:
        kk = F.omega * np.sqrt(mt[inner])
        Sin = Sn[inner]
        for a in range(3):
            pa = prof[a]
            ga = g[a][1:b[a] + 1]
            for side, face, interior in ((0, lo[a], lo[a] > 0), (1, hi[a] - 1, hi[a] < n[a])):
                if not interior:
                    continue
                m1 = (ga == face)
                sa = pa[2 * ga + 1]
                if a == 0:
                    mask = m1[None, None, :]; sav = sa[None, None, :]
                elif a == 1:
                    mask = m1[None, :, None]; sav = sa[None, :, None]
                else:
                    mask = m1[:, None, None]; sav = sa[:, None, None]
                C[eidx(0, 0, 0)][inner] += np.where(mask, 1j * kk * Sin / (sav * F.h), 0.0)
    return np.ascontiguousarray(C[(slice(None),) + inner])


def csr_from_coeffs(C: np.ndarray) -> sp.csr_matrix:
    """Sparse matrix of the box rows; columns outside the box are dropped."""
    _, bz, by, bx = C.shape
    nloc = bx * by * bz
    kk, jj, ii = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    rows, cols, vals = [], [], []
    for ei, (ex, ey, ez) in enumerate(OFFSETS):
        ci, cj, ck = ii + ex, jj + ey, kk + ez
        m = (ci >= 0) & (ci < bx) & (cj >= 0) & (cj < by) & (ck >= 0) & (ck < bz)
        v = C[ei]
        m = m & (v != 0)
        rows.append(((kk * by + jj) * bx + ii)[m])
        cols.append(((ck * by + cj) * bx + ci)[m])
        vals.append(v[m])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nloc, nloc))
    A.sum_duplicates()
    return A


def assemble(F: Fields) -> sp.csr_matrix:
    """The global operator A as CSR (lexicographic, x fastest)."""
    return csr_from_coeffs(row_coeffs(F))


def apply_coeffs(C: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = A x for x shaped (..., nz, ny, nx) with zero values outside."""
    bz, by, bx = C.shape[1:]
    lead = x.shape[:-3]
    xp = np.zeros(lead + (bz + 2, by + 2, bx + 2), dtype=np.complex128)
    xp[..., 1:-1, 1:-1, 1:-1] = x
    y = np.zeros(lead + (bz, by, bx), dtype=np.complex128)
    for ei, (ex, ey, ez) in enumerate(OFFSETS):
        y += C[ei] * xp[..., 1 + ez:bz + 1 + ez, 1 + ey:by + 1 + ey, 1 + ex:bx + 1 + ex]
    return y


def point_sources(F: Fields, sources, amps=None) -> np.ndarray:
    """Right-hand sides b = S f for unit (or given) point sources, shape
    (nsrc, nz, ny, nx).  Sources must lie outside the PML (S = 1 there)."""
    S = F.S()
    b = np.zeros((len(sources),) + F.shape, dtype=np.complex128)
    for s, (i, j, k) in enumerate(sources):
        a = 1.0 if amps is None else amps[s]
        b[s, k, j, i] = a * S[k, j, i]
    return b
