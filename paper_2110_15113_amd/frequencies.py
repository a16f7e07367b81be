"""Several frequencies in flight on one GPU.

Frequency-domain inversion solves the Helmholtz system at several
frequencies, each with its own operator and local factors (sec. 1; sec. 4
on multi-frequency inversion).  The frequencies are independent, so their
solves can overlap on one device: each frequency gets its own library
context (own factors, own workspace, own HIP stream at default priority) and
one host thread drives its solve.  Each solve synchronises only with its own
stream once per Arnoldi step, so while one frequency's host loop waits, the
kernels of the others keep the device busy.  The library call releases the
Python interpreter lock (ctypes), so the threads run concurrently.

Memory: every frequency holds its own factors and Krylov basis; the caller
chooses how many fit in HBM.
"""
from __future__ import annotations

import threading
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import oras


@dataclass
class FrequencyState:
    omega: float
    solver: oras.Solver
    stream: torch.cuda.Stream


class FrequencyBatch:
    """One context per angular frequency over the same model and partition."""

    def __init__(self, vel: torch.Tensor, h: float, npml: int, omegas: Sequence[float],
                 Q: Optional[torch.Tensor] = None, prec: int = oras.C128, device: int = 0):
        self.prec = prec
        self.items: List[FrequencyState] = []
        dev = torch.device("cuda", device)
        self.device = dev
        caller = torch.cuda.current_stream(dev)
        for om in omegas:
            st = torch.cuda.Stream(device=dev)           # default priority
            st.wait_stream(caller)                        # vel and Q come from the caller's stream
            with torch.cuda.stream(st):
                S = oras.Solver(device)
                S.assemble(vel, h, npml, float(om), Q, prec=prec)
            self.items.append(FrequencyState(float(om), S, st))
        torch.cuda.synchronize(dev)

    def _run(self, fn, concurrent: bool):
        """fn(i, state) for every frequency, on its stream; in one thread each
        when concurrent.  Each frequency's stream first waits for the work
        queued so far on the caller's stream (its inputs may still be in
        flight there), and is synchronised before this returns.  Re-raises
        the first failure."""
        errors: List[BaseException] = []
        caller = torch.cuda.current_stream(self.device)
        for it in self.items:
            it.stream.wait_stream(caller)

        def body(i, it):
            try:
                with torch.cuda.stream(it.stream):
                    fn(i, it)
                it.stream.synchronize()
            except BaseException as e:   # propagated below
                errors.append(e)

        if concurrent and len(self.items) > 1:
            th = [threading.Thread(target=body, args=(i, it)) for i, it in enumerate(self.items)]
            for t in th:
                t.start()
            for t in th:
                t.join()
        else:
            for i, it in enumerate(self.items):
                body(i, it)
        if errors:
            raise errors[0]

    def factor(self, parts, overlap: int = 2, concurrent: bool = True, **kw):
        self._run(lambda i, it: it.solver.factor(parts, overlap, self.prec, **kw), concurrent)

    def point_sources(self, idx, amp=None) -> List[torch.Tensor]:
        out = [None] * len(self.items)

        def f(i, it):
            out[i] = it.solver.point_sources(idx, amp)
        self._run(f, False)
        return out

    def solve(self, bs: Sequence[torch.Tensor], tol: float, restart: int = 30,
              maxit: int = 1000, concurrent: bool = True, **kw) -> List[oras.SolveResult]:
        """Solve A(omega_f) x_f = b_f for every frequency f."""
        if len(bs) != len(self.items):
            raise ValueError("one right-hand-side block per frequency")
        out: List[Optional[oras.SolveResult]] = [None] * len(self.items)

        def f(i, it):
            out[i] = it.solver.solve(bs[i], tol, restart=restart, maxit=maxit, **kw)
        self._run(f, concurrent)
        return out

    def close(self):
        for it in self.items:
            it.solver.close()
        self.items = []
