"""Thin ctypes binding of liboras.so (argument marshalling only).

Every step of the solver runs in the HIP library; this module only checks
tensor placement, dtype and contiguity, passes device pointers and the
current HIP stream, and raises on error codes.  The library is loaded from
this package folder; when it is missing the import fails loudly (there is no
CPU fallback).
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# ORAS_LIB selects another build of the library (the AddressSanitizer build of
# build.py --asan); by default the one in this package folder
LIB_PATH = os.environ.get("ORAS_LIB") or os.path.join(HERE, "liboras.so")

C64 = 1
C128 = 2
CONJ = 1
X0 = 2

STATUS = {0: "ORAS_OK", 1: "ORAS_E_ARG", 2: "ORAS_E_STATE", 3: "ORAS_E_OOM", 4: "ORAS_E_HIP",
          5: "ORAS_E_NUMERIC", 100: "ORAS_W_NOT_CONVERGED"}


class OrasError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Grid(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int), ("h", ct.c_double),
                ("npml", ct.c_int), ("free_surface", ct.c_int)]


class Pml(ct.Structure):
    _fields_ = [("R0", ct.c_double), ("power", ct.c_int), ("c_ref", ct.c_double)]


class Interface(ct.Structure):
    _fields_ = [("kind", ct.c_int), ("power", ct.c_int), ("R0", ct.c_double)]


IFACE_ROBIN, IFACE_PML = 0, 1
WEIGHTS_FOLLOW_M = 1   # set_m flag
GRAD_WEIGHTS = 1       # gradient flag


class SolveOpts(ct.Structure):
    _fields_ = [("restart", ct.c_int), ("maxit", ct.c_int), ("flags", ct.c_int),
                ("krylov_in_prec", ct.c_int), ("z_prec", ct.c_int)]


class SolveInfo(ct.Structure):
    _fields_ = [("iters", ct.POINTER(ct.c_int)), ("rel_res", ct.POINTER(ct.c_double)),
                ("converged", ct.POINTER(ct.c_int)), ("t_solve", ct.c_double),
                ("t_stencil", ct.c_double), ("t_oras", ct.c_double), ("t_ortho", ct.c_double),
                ("cycles", ct.c_int), ("total_iters", ct.c_int)]


_LIB = None

class BlrInfo(ct.Structure):
    _fields_ = [("eps", ct.c_double), ("pmax", ct.c_int), ("max_rank", ct.c_int),
                ("blocks", ct.c_longlong), ("lowrank", ct.c_longlong), ("mean_rank", ct.c_double),
                ("stored_entries", ct.c_double), ("dense_entries", ct.c_double),
                ("t_compress", ct.c_double)]


SIGNATURES = {
    "oras_create": (ct.c_int, [ct.POINTER(ct.c_void_p), ct.c_int, ct.c_void_p]),
    "oras_destroy": (None, [ct.c_void_p]),
    "oras_last_error": (ct.c_char_p, [ct.c_void_p]),
    "oras_weight_table": (ct.c_int, [ct.c_void_p, ct.c_int, ct.POINTER(ct.c_double),
                                     ct.POINTER(ct.c_double), ct.POINTER(ct.c_int)]),
    "oras_assemble": (ct.c_int, [ct.c_void_p, ct.POINTER(Grid), ct.c_void_p, ct.c_void_p,
                                 ct.c_double, ct.POINTER(Pml), ct.c_int]),
    "oras_set_m": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "oras_factor_subdomains": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int), ct.c_int, ct.c_int]),
    "oras_factor_subdomains_ex": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int), ct.c_int, ct.c_int,
                                             ct.c_void_p]),
    "oras_set_m_ex": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int]),
    "oras_gradient_ex": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_int,
                                    ct.c_void_p]),
    "oras_solve": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_double,
                              ct.POINTER(SolveOpts), ct.POINTER(SolveInfo)]),
    "oras_point_sources": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int,
                                      ct.c_void_p]),
    "oras_sample": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int,
                               ct.c_void_p]),
    "oras_spread": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int,
                               ct.c_void_p]),
    "oras_gradient": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p]),
    "oras_apply_A": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_int]),
    "oras_apply_M": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int]),
    "oras_timings": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]),
    "oras_profile": (ct.c_int, [ct.c_void_p, ct.c_int]),
    "oras_kernel_stats": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_double),
                                     ct.POINTER(ct.c_longlong), ct.POINTER(ct.c_double),
                                     ct.POINTER(ct.c_double)]),
    "oras_rhs_stats": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_double),
                                  ct.POINTER(ct.c_double)]),
    "oras_coefficients": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "oras_subdomain": (ct.c_int, [ct.c_void_p, ct.c_int, ct.POINTER(ct.c_int),
                                  ct.POINTER(ct.c_int)]),
    "oras_compress_factors": (ct.c_int, [ct.c_void_p, ct.c_double, ct.c_int,
                                         ct.POINTER(BlrInfo)]),
    "oras_blr_ranks": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_int, ct.c_void_p, ct.c_int,
                                  ct.POINTER(ct.c_int)]),
    "oras_factor_stats": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int),
                                     ct.POINTER(ct.c_int), ct.c_void_p, ct.c_int,
                                     ct.POINTER(ct.c_int)]),
    "oras_apply_A_noalloc": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_int]),
    "oras_noalloc_scratch_bytes": (ct.c_size_t, []),
}


def lib():
    """Load liboras.so from the package folder (raises if it is not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2110_15113_amd.build`")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def weight_table():
    """The library's own fitted weight table: (G grid, (count, 7) weights)."""
    L = lib()
    cnt = ct.c_int()
    g0 = ct.c_double()
    dg = ct.c_double()
    L.oras_weight_table(None, 0, ct.byref(g0), ct.byref(dg), ct.byref(cnt))
    out = np.zeros((cnt.value, 7))
    rc = L.oras_weight_table(out.ctypes.data_as(ct.c_void_p), cnt.value, None, None, None)
    if rc != 0:
        raise OrasError(rc, "weight table")
    return g0.value + dg.value * np.arange(cnt.value), out


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, device, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must live on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


@dataclass
class SolveResult:
    x: torch.Tensor
    iters: np.ndarray
    rel_res: np.ndarray
    converged: np.ndarray
    t_solve: float
    t_stencil: float
    t_oras: float
    t_ortho: float
    cycles: int
    total_iters: int
    status: int


class Solver:
    """One library context: a grid, its operator, its subdomain factors.

    Every library call runs on the HIP stream that was current when the
    Solver was created; tensors passed in must be ready in that stream's
    order (made on it, or the stream made to wait for theirs), and the calls
    that return host results synchronise with it."""

    def __init__(self, device: int = 0, host_only: bool = False):
        L = lib()
        self._ctx = ct.c_void_p()
        if host_only:
            self.device = None
            stream = None
            dev = -1
        else:
            self.device = torch.device("cuda", device)
            stream = ct.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            dev = device
        rc = L.oras_create(ct.byref(self._ctx), dev, stream)
        if rc != 0:
            raise OrasError(rc, f"oras_create(device={dev}) failed")
        self.shape = None

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().oras_destroy(self._ctx)
            self._ctx = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, allow_warn: bool = False):
        if rc == 0 or (allow_warn and rc == 100):
            return rc
        raise OrasError(rc, lib().oras_last_error(self._ctx).decode())

    # -- set-up ------------------------------------------------------------
    def assemble(self, vel: torch.Tensor, h: float, npml: int, omega: float,
                 Q: Optional[torch.Tensor] = None, prec: int = C128, R0: float = 1e-3,
                 power: int = 2, c_ref: float = 0.0, free_surface: bool = False):
        nz, ny, nx = vel.shape
        _need(vel, torch.float64, self.device or vel.device, name="vel")
        if Q is not None:
            _need(Q, torch.float64, vel.device, vel.shape, name="Q")
        g = Grid(nx, ny, nz, float(h), int(npml), int(bool(free_surface)))
        p = Pml(float(R0), int(power), float(c_ref))
        self._check(lib().oras_assemble(self._ctx, ct.byref(g), _ptr(vel), _ptr(Q), float(omega),
                                        ct.byref(p), int(prec)))
        self.shape = (nz, ny, nx)
        self.prec = prec

    def set_m(self, m: torch.Tensor, weights: str = "frozen"):
        """New squared slowness.  weights: "frozen" (kept from assemble) or
        "follow" (picked again from the local G at m)."""
        _need(m, torch.float64, self.device, self.shape, name="m")
        if weights not in ("frozen", "follow"):
            raise ValueError("weights must be 'frozen' or 'follow'")
        flags = WEIGHTS_FOLLOW_M if weights == "follow" else 0
        self._check(lib().oras_set_m_ex(self._ctx, _ptr(m), flags))

    def factor(self, parts: Sequence[int], overlap: int = 2, prec: int = C128,
               interface: str = "robin", R0: float = 0.3, power: int = 2):
        """interface: "robin" (impedance faces) or "pml" (PML transmission
        conditions over the overlap layers; R0, power: the layer's law)."""
        arr = (ct.c_int * 3)(*[int(p) for p in parts])
        if interface not in ("robin", "pml"):
            raise ValueError("interface must be 'robin' or 'pml'")
        ifc = Interface(IFACE_PML if interface == "pml" else IFACE_ROBIN, int(power), float(R0))
        self._check(lib().oras_factor_subdomains_ex(self._ctx, arr, int(overlap), int(prec),
                                                    ct.addressof(ifc)))

    def factor_stats(self):
        """(smallest min|pivot| / max|S_k| over all subdomain planes, (sub,
        plane) where it occurs, the ratio per subdomain plane (nsub, planes))."""
        r, j, k, mp = ct.c_double(), ct.c_int(), ct.c_int(), ct.c_int()
        self._check(lib().oras_factor_stats(self._ctx, ct.byref(r), ct.byref(j), ct.byref(k),
                                            None, 0, ct.byref(mp)))
        nsub = len(self.subdomains())
        out = np.zeros(nsub * mp.value)
        self._check(lib().oras_factor_stats(self._ctx, None, None, None,
                                            out.ctypes.data_as(ct.c_void_p), out.size, None))
        return r.value, (j.value, k.value), out.reshape(nsub, mp.value)

    def timings(self):
        ta, tf = ct.c_double(), ct.c_double()
        self._check(lib().oras_timings(self._ctx, ct.byref(ta), ct.byref(tf)))
        return ta.value, tf.value

    def profile(self, enable: bool = True):
        """Time every plane GEMM of the ORAS apply with HIP events (resets)."""
        self._check(lib().oras_profile(self._ctx, int(bool(enable))))

    def kernel_stats(self):
        """(seconds, launches, algorithmic flops, algorithmic bytes) of the
        plane GEMM since the last profile() call."""
        s, f, b = ct.c_double(), ct.c_double(), ct.c_double()
        n = ct.c_longlong()
        self._check(lib().oras_kernel_stats(self._ctx, ct.byref(s), ct.byref(n), ct.byref(f),
                                            ct.byref(b)))
        return s.value, n.value, f.value, b.value

    def rhs_stats(self):
        """(seconds, algorithmic bytes) of the plane right-hand-side kernels
        (restriction fused) since the last profile() call."""
        s, b = ct.c_double(), ct.c_double()
        self._check(lib().oras_rhs_stats(self._ctx, ct.byref(s), ct.byref(b)))
        return s.value, b.value

    # -- solve -------------------------------------------------------------
    def solve(self, b: torch.Tensor, tol: float, restart: int = 30, maxit: int = 1000,
              conj: bool = False, x0: Optional[torch.Tensor] = None,
              out: Optional[torch.Tensor] = None, krylov_in_prec: int = 0,
              z_prec: int = 0) -> SolveResult:
        """krylov_in_prec / z_prec: precision of A z_j in the Arnoldi step and
        of the stored basis Z (0: the context's stencil / factor precision)."""
        nrhs = b.shape[0]
        _need(b, torch.complex128, self.device, (nrhs,) + self.shape, name="b")
        flags = CONJ if conj else 0
        if out is None:
            out = torch.empty_like(b)
        _need(out, torch.complex128, self.device, b.shape, name="out")
        if x0 is not None:
            _need(x0, torch.complex128, self.device, b.shape, name="x0")
            out.copy_(x0)
            flags |= X0
        it = (ct.c_int * nrhs)()
        rr = (ct.c_double * nrhs)()
        cv = (ct.c_int * nrhs)()
        info = SolveInfo(it, rr, cv, 0.0, 0.0, 0.0, 0.0, 0, 0)
        opts = SolveOpts(int(restart), int(maxit), flags, int(krylov_in_prec), int(z_prec))
        rc = self._check(lib().oras_solve(self._ctx, _ptr(b), _ptr(out), nrhs, float(tol),
                                          ct.byref(opts), ct.byref(info)), allow_warn=True)
        return SolveResult(out, np.array(it[:]), np.array(rr[:]), np.array(cv[:], dtype=bool),
                           info.t_solve, info.t_stencil, info.t_oras, info.t_ortho, info.cycles,
                           info.total_iters, rc)

    def point_sources(self, idx: Sequence[Sequence[int]], amp=None) -> torch.Tensor:
        nrhs = len(idx)
        ia = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(nrhs, 3))
        aa = None
        if amp is not None:
            a = np.asarray(amp, dtype=np.complex128).reshape(nrhs)
            aa = np.ascontiguousarray(np.stack([a.real, a.imag], 1))
        b = torch.empty((nrhs,) + self.shape, dtype=torch.complex128, device=self.device)
        self._check(lib().oras_point_sources(self._ctx, ia.ctypes.data_as(ct.c_void_p),
                                             None if aa is None else aa.ctypes.data_as(ct.c_void_p),
                                             nrhs, _ptr(b)))
        return b

    def _rec(self, rec) -> torch.Tensor:
        if isinstance(rec, torch.Tensor):
            _need(rec, torch.int32, self.device, name="receivers")
            return rec
        return torch.as_tensor(np.asarray(rec, dtype=np.int32).reshape(-1, 3), device=self.device)

    def sample(self, u: torch.Tensor, rec) -> torch.Tensor:
        r = self._rec(rec)
        nrhs = u.shape[0]
        _need(u, torch.complex128, self.device, (nrhs,) + self.shape, name="u")
        d = torch.empty((nrhs, r.shape[0]), dtype=torch.complex128, device=self.device)
        self._check(lib().oras_sample(self._ctx, _ptr(u), nrhs, _ptr(r), r.shape[0], _ptr(d)))
        return d

    def spread(self, d: torch.Tensor, rec) -> torch.Tensor:
        r = self._rec(rec)
        nrhs = d.shape[0]
        _need(d, torch.complex128, self.device, (nrhs, r.shape[0]), name="d")
        b = torch.empty((nrhs,) + self.shape, dtype=torch.complex128, device=self.device)
        self._check(lib().oras_spread(self._ctx, _ptr(d), nrhs, _ptr(r), r.shape[0], _ptr(b)))
        return b

    def gradient(self, u: torch.Tensor, mu: torch.Tensor, weights: bool = False) -> torch.Tensor:
        """-Re sum_c mu_c^H (dA/dm) u_c; weights=True adds the stencil weights'
        dependence on m (requires weights that follow m)."""
        nrhs = u.shape[0]
        _need(u, torch.complex128, self.device, (nrhs,) + self.shape, name="u")
        _need(mu, torch.complex128, self.device, u.shape, name="mu")
        g = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._check(lib().oras_gradient_ex(self._ctx, _ptr(u), _ptr(mu), nrhs,
                                           GRAD_WEIGHTS if weights else 0, _ptr(g)))
        return g

    # -- test hooks ----------------------------------------------------------
    def apply_A(self, x: torch.Tensor, prec: int = C128) -> torch.Tensor:
        _need(x, torch.complex128, self.device, (x.shape[0],) + self.shape, name="x")
        y = torch.empty_like(x)
        self._check(lib().oras_apply_A(self._ctx, _ptr(x), _ptr(y), x.shape[0], int(prec)))
        return y

    def apply_A_noalloc(self, x: torch.Tensor, y: torch.Tensor, prec: int = C128) -> torch.Tensor:
        """y = A x into the caller's y with no device allocation (the staging
        lives in the library's fixed per-device scratch array)."""
        _need(x, torch.complex128, self.device, (x.shape[0],) + self.shape, name="x")
        _need(y, torch.complex128, self.device, x.shape, name="y")
        self._check(lib().oras_apply_A_noalloc(self._ctx, _ptr(x), _ptr(y), x.shape[0], int(prec)))
        return y

    def apply_M(self, x: torch.Tensor) -> torch.Tensor:
        _need(x, torch.complex128, self.device, (x.shape[0],) + self.shape, name="x")
        y = torch.empty_like(x)
        self._check(lib().oras_apply_M(self._ctx, _ptr(x), _ptr(y), x.shape[0]))
        return y

    def coefficients(self) -> torch.Tensor:
        out = torch.empty((27,) + self.shape, dtype=torch.complex128, device=self.device)
        self._check(lib().oras_coefficients(self._ctx, _ptr(out)))
        return out

    def compress(self, eps: float = 1e-3, pmax: int = 8) -> dict:
        """Block low-rank plane inverses (threshold eps, patches of at most
        pmax x pmax nodes) for every later apply and solve."""
        info = BlrInfo()
        self._check(lib().oras_compress_factors(self._ctx, float(eps), int(pmax), ct.byref(info)))
        return {f: getattr(info, f) for f, _ in BlrInfo._fields_}

    def blr_ranks(self, sub: int, plane: int) -> np.ndarray:
        """Rank table (npatch, npatch) of one plane inverse; -1 = dense."""
        n = ct.c_int()
        self._check(lib().oras_blr_ranks(self._ctx, sub, plane, None, 0, ct.byref(n)))
        out = np.zeros((n.value, n.value), dtype=np.int32)
        self._check(lib().oras_blr_ranks(self._ctx, sub, plane, out.ctypes.data_as(ct.c_void_p),
                                         out.size, None))
        return out

    def subdomains(self):
        n = ct.c_int()
        self._check(lib().oras_subdomain(self._ctx, 0, ct.byref(n), None))
        out = []
        for j in range(n.value):
            b = (ct.c_int * 12)()
            self._check(lib().oras_subdomain(self._ctx, j, None, b))
            out.append(tuple(b[:]))
        return out
