"""Lambda-adaptive 27-point weight table (oracle side).  TEST INFRASTRUCTURE.

Paper, sec. 2.3 "Finite-difference frequency-domain (FDFD) discretization":
the stiffness and consistent-mass parts of the compact 27-point stencil are
mixed over three rotated coordinate systems with weights obtained by a
least-squares fit of the numerical phase velocity; the fit is made separately
for each number of grid points per wavelength G = lambda / h, so the weights
become functions of G, and each row of A takes the weights of its local G.
The paper does not print the weights, so this module fixes the reading:

Families (stiffness), each a symmetric flux form -D^T diag(w K) D:
  F1 two-point differences at face midpoints          (7-point Laplacian)
  F2 2x2-averaged differences at in-plane cell centres (rotated in-plane)
  F3 2x2x2-averaged differences at cube centres        (rotated 3D)
Their plane-wave symbols (times -1/h^2), with c_a = cos(xi_a):
  L1 = 2 (3 - S1),  L2 = 3 - S2,  L3 = (3 + S1 - S2 - 3 S3) / 2
  S1 = sum c_a,  S2 = sum_{a<b} c_a c_b,  S3 = c_x c_y c_z.
Mass: mu = wm0 + 2 wmf S1 + 4 wme S2 + 8 wmc S3 (centre, 6 faces, 12 edges,
8 corners), with wm0 + 6 wmf + 12 wme + 8 wmc = 1 and w1 + w2 + w3 = 1.

Reading of the fit (see the design notes): to first order the dispersion
residual  Lambda - k^2 mu  lies in span{1, S1, S2, S3} and its constant part
is pinned by the two consistency constraints, so the 5 free weights map onto
a 3-dimensional space; a 5-weight fit is therefore not unique.  We fix the
stiffness weights at the fourth-order isotropic choice (w1, w2, w3) =
(1/2, 1/3, 1/6) (every family has Laplacian part |xi|^2 - sum xi^4/12 - c_f
sum_{a<b} xi_a^2 xi_b^2 with c = 0, 1/4, 1/2; isotropy needs w2/4 + w3/2 =
1/6) and fit the three mass weights per G by linear least squares on the
linearised phase-velocity error

    r_d = (Lambda(xi_d) - k^2 mu(xi_d)) / (2 k^2),   k = 2 pi / G,
    xi_d = k n_d,  n_d on a 16 x 8 (theta, phi) grid over
    theta in [0, pi/2], phi in [0, pi/4] (end points included),

plus a ridge term 1e-8 * |(wmf, wme, wmc)|^2 toward lumped mass.  The
minimiser is unique; this module solves it with LAPACK least squares on the
stacked system.  G grid: 3, 3.25, ..., 48; lookup is linear in G, clamped.

Parity: pinned in tests by (i) the constraints, (ii) stationarity of the
normal equations, (iii) the true (non-linearised) phase-velocity error being
below the 7-point stencil's at every G, (iv) the assembled operator's plane
wave symbol matching Lambda and mu (operator tests).
"""
from __future__ import annotations

import numpy as np

G_MIN = 3.0
G_STEP = 0.25
G_COUNT = 181           # 3.0 ... 48.0
STIFF = (0.5, 1.0 / 3.0, 1.0 / 6.0)
RIDGE = 1e-8


def directions() -> np.ndarray:
    """The 128 unit directions of the fit, shape (128, 3)."""
    th = np.array([i * (np.pi / 2) / 15 for i in range(16)])
    ph = np.array([j * (np.pi / 4) / 7 for j in range(8)])
    out = []
    for t in th:
        for p in ph:
            out.append((np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)))
    return np.array(out)


def symbols(xi: np.ndarray):
    """Family stiffness symbols (L1, L2, L3) and mass-shell symbols
    (centre, faces, edges, corners) at wave vectors xi (..., 3), grid units."""
    c = np.cos(xi)
    S1 = c[..., 0] + c[..., 1] + c[..., 2]
    S2 = c[..., 0] * c[..., 1] + c[..., 0] * c[..., 2] + c[..., 1] * c[..., 2]
    S3 = c[..., 0] * c[..., 1] * c[..., 2]
    L = (2.0 * (3.0 - S1), 3.0 - S2, (3.0 + S1 - S2 - 3.0 * S3) / 2.0)
    M = (np.ones_like(S1), 2.0 * S1, 4.0 * S2, 8.0 * S3)
    return L, M


def lam_mu(w7, xi):
    """Stiffness symbol Lambda and mass symbol mu of a 7-weight stencil."""
    w1, w2, w3, wm0, wmf, wme, wmc = w7
    L, M = symbols(xi)
    return (w1 * L[0] + w2 * L[1] + w3 * L[2],
            wm0 * M[0] + wmf * M[1] + wme * M[2] + wmc * M[3])


def phase_velocity(w7, G, dirs) -> np.ndarray:
    """Normalised numerical phase velocity v_ph / c along ``dirs`` at G."""
    k = 2.0 * np.pi / G
    lam, mu = lam_mu(w7, k * dirs)
    return np.sqrt(lam / mu) / k


def fit_one(G: float) -> np.ndarray:
    """Weights (w1, w2, w3, wm0, wmf, wme, wmc) for one G."""
    k = 2.0 * np.pi / G
    dirs = directions()
    L, M = symbols(k * dirs)
    w1, w2, w3 = STIFF
    lam = w1 * L[0] + w2 * L[1] + w3 * L[2]
    # mu = M0 + wmf (Mf - 6 M0) + wme (Me - 12 M0) + wmc (Mc - 8 M0)
    base = (lam - k * k * M[0]) / (2.0 * k * k)
    cols = [-(M[1] - 6.0 * M[0]) / 2.0, -(M[2] - 12.0 * M[0]) / 2.0,
            -(M[3] - 8.0 * M[0]) / 2.0]
    J = np.stack(cols, axis=1)
    Jaug = np.vstack([J, np.sqrt(RIDGE) * np.eye(3)])
    raug = np.concatenate([-base, np.zeros(3)])
    p, *_ = np.linalg.lstsq(Jaug, raug, rcond=None)
    wmf, wme, wmc = p
    return np.array([w1, w2, w3, 1.0 - 6.0 * wmf - 12.0 * wme - 8.0 * wmc, wmf, wme, wmc])


def g_grid() -> np.ndarray:
    return G_MIN + G_STEP * np.arange(G_COUNT)


def fit_table() -> np.ndarray:
    """(G_COUNT, 7) table of weights on the G grid."""
    return np.stack([fit_one(G) for G in g_grid()])


_TABLE = None


def table() -> np.ndarray:
    global _TABLE
    if _TABLE is None:
        _TABLE = fit_table()
    return _TABLE


def lookup_slope(G: np.ndarray, tab: np.ndarray | None = None) -> np.ndarray:
    """d lookup / dG: the slope of the table segment the interpolation uses,
    zero where the lookup clamps (G outside the table range); (..., 7)."""
    tab = table() if tab is None else tab
    t = (np.asarray(G, dtype=np.float64) - G_MIN) / G_STEP
    inside = (t > 0.0) & (t < G_COUNT - 1.0)
    tc = np.clip(t, 0.0, G_COUNT - 1.0)
    i0 = np.minimum(np.floor(tc).astype(np.int64), G_COUNT - 2)
    slope = (tab[i0 + 1] - tab[i0]) / G_STEP
    return np.where(inside[..., None], slope, 0.0)


def lookup(G: np.ndarray, tab: np.ndarray | None = None) -> np.ndarray:
    """Linear interpolation in G (clamped to the table range); returns
    (..., 7)."""
    tab = table() if tab is None else tab
    t = (np.asarray(G, dtype=np.float64) - G_MIN) / G_STEP
    t = np.clip(t, 0.0, G_COUNT - 1.0)
    i0 = np.minimum(np.floor(t).astype(np.int64), G_COUNT - 2)
    f = (t - i0)[..., None]
    return (1.0 - f) * tab[i0] + f * tab[i0 + 1]
