"""Sequence driver: solves the problems of a correlated sequence one cycle after another, each
warm-started from the previous cycle's Ritz vectors and bounds, or from a random block.

This is the protocol of the paper's experiments (Section 3.2: solve P^(l+1) once from random
vectors, t_rnd, and once from the eigenvectors of P^(l), t_app, and compare t_rnd / t_app), with
the warm start taken from the solver's own previous solution as in a self-consistent cycle.
All work runs in the C-ABI library; this module only moves device pointers around.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np

from . import chfsi, synth


@dataclasses.dataclass
class CycleResult:
    cycle: int
    warm: bool
    status: int
    wall_ms: float
    lam: np.ndarray
    resid: np.ndarray
    stats: dict


class Sequence:
    """Device-resident pencils of one synthetic sequence plus the per-cycle solutions."""

    def __init__(self, spec: synth.SequenceSpec, handle: Optional[chfsi.Handle] = None, device: int = 0,
                 keep_host: bool = False):
        import torch
        self.torch = torch
        self.spec = spec
        self.h = handle or chfsi.Handle(device)
        from . import autotune
        self.tuned_entries = autotune.load(self.h)
        self.dev = f"cuda:{device}"
        self.m = spec.nev + spec.nex
        self.A: List = []
        self.host: List[synth.Pencil] = []
        self.S = None
        for pen in synth.sequence(spec):
            self.A.append(chfsi.to_device(pen.A, self.dev))
            if pen.S is not None and self.S is None:
                self.S = chfsi.to_device(pen.S, self.dev)
            if keep_host:
                self.host.append(pen)
        self.X: List = [None] * spec.cycles          # device solutions (m, n) column-major
        self.lam: List = [None] * spec.cycles

    def new_block(self):
        return self.torch.zeros((self.m, self.spec.n), dtype=self.torch.complex128, device=self.dev)

    def params(self, **kw) -> chfsi.Params:
        base = dict(nev=self.spec.nev, nex=self.spec.nex, deg=self.spec.deg, tol=1e-10, seed=self.spec.seed)
        base.update(kw)
        return chfsi.default_params(**base)

    def solve(self, cycle: int, warm: bool, store: bool = False, X=None, **kw) -> CycleResult:
        """Solve one cycle.  warm: start from the stored solution of cycle-1 (its Ritz vectors and
        the bounds mu1 = lambda_1, a = largest Ritz value)."""
        torch = self.torch
        Xw = self.new_block() if X is None else X
        prm_kw = dict(kw)
        if warm:
            if cycle == 0 or self.X[cycle - 1] is None:
                raise ValueError("warm start needs the stored solution of the previous cycle")
            Xw.copy_(self.X[cycle - 1])
            lam_prev = self.lam[cycle - 1]
            prm_kw.update(have_bounds=1, mu1=float(lam_prev[0]), a=float(lam_prev[-1]))
        prm = self.params(**prm_kw)
        torch.cuda.synchronize(self.dev)
        t0 = time.perf_counter()
        res = self.h.solve(self.A[cycle], self.S, Xw, warm, prm, raise_on_error=False)
        wall = (time.perf_counter() - t0) * 1e3
        if store and res.status == 0:
            self.X[cycle] = Xw.clone()
            self.lam[cycle] = res.lam.copy()
        return CycleResult(cycle, warm, res.status, wall, res.lam, res.resid, res.stats)

    def run_reference(self, **kw) -> List[CycleResult]:
        """Cycle 0 from a random block, then every cycle warm-started from the previous one; the
        solutions are stored as the warm starts of later runs."""
        out = [self.solve(0, warm=False, store=True, **kw)]
        for c in range(1, self.spec.cycles):
            out.append(self.solve(c, warm=True, store=True, **kw))
        return out
