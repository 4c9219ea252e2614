"""Autotuner for the level-scheduled Newton kernel's launch shape.

The search times the real batched Newton launch (pf_newton on the caller's
batch) with HIP events and keeps the fastest setting of:
  * threads per workgroup (256, 512),
  * LDS-tail budget (how many top levels run in LDS),
  * case interleave of the workspace (1, 2, 4, 8),
  * for a single case, the workgroups its launch is spread over (one, or a
    cooperative launch of 16 ... 256 sharing the levels below the LDS tail),
  * lanes per node for each level class (levels grouped by width), by
    coordinate descent over {1, 2, 4, ..., 64}.
Every setting computes the same factorisation; the lanes per node only change
the order in which partial sums are combined, so settings agree to rounding
and each one is bitwise reproducible.  The tuner never changes the symbolic
structure.
"""
from __future__ import annotations

import itertools
import time

import numpy as np
import torch

from . import binding as B

WIDTH_CLASSES = [(1024, 1 << 30), (256, 1023), (64, 255), (16, 63), (4, 15), (2, 3), (1, 1)]
LANES = [1, 2, 4, 8, 16, 32, 64]


def level_classes(sym):
    """Level index lists per width class (empty classes dropped)."""
    ex = sym.export()
    widths = np.diff(ex["level_ptr"])
    out = []
    for lo, hi in WIDTH_CLASSES:
        idx = np.flatnonzero((widths >= lo) & (widths <= hi))
        if len(idx):
            out.append(((lo, hi), idx))
    return out


class _Timer:
    def __init__(self, sym, yval, bus_type, Psp, Qsp, Vm0, Va0, tol, max_iter, reps):
        self.sym, self.yval, self.type = sym, yval, bus_type
        self.Psp, self.Qsp = Psp, Qsp
        self.Vm0, self.Va0 = Vm0, Va0
        self.tol, self.max_iter, self.reps = tol, max_iter, reps
        self.Bn = Psp.shape[0]
        self.Vm = Vm0.clone()
        self.Va = Va0.clone()
        self.ws = None
        self.runs = 0

    def __call__(self):
        sym = self.sym
        info = sym.info
        C = B.pf_newton_interleave(sym.h, self.Bn)
        rows = -(-self.Bn // C) * C
        if self.ws is None or self.ws.shape[0] < rows or self.ws.shape[1] != info.ws_doubles:
            self.ws = torch.empty(rows, info.ws_doubles, dtype=torch.float64,
                                  device=self.Vm.device)
        it = torch.empty(self.Bn, dtype=torch.int32, device=self.Vm.device)
        st = torch.empty(self.Bn, dtype=torch.int32, device=self.Vm.device)
        best = float("inf")
        for r in range(self.reps + 1):
            self.Vm.copy_(self.Vm0)
            self.Va.copy_(self.Va0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            B.pf_newton(sym.h, self.Bn, self.yval, 0 if self.yval.dim() == 1 else
                        self.yval.shape[-1], self.type, 0 if self.type.dim() == 1 else
                        self.type.shape[-1], self.Psp, self.Qsp, self.Psp.shape[-1], self.Vm,
                        self.Va, self.Vm.shape[-1], self.tol, self.max_iter, 0, self.ws,
                        info.ws_doubles, it, None, st)
            e1.record()
            torch.cuda.synchronize()
            if r > 0:  # first run warms caches and the launch path
                best = min(best, e0.elapsed_time(e1))
        self.runs += self.reps + 1
        return best


def tune(sym, yval, bus_type, Psp, Qsp, Vm0, Va0, tol=1e-8, max_iter=20, reps=2,
         threads=(256, 512), budgets=(32768, 65536, 114688, 161792),
         interleaves=(1, 2, 4, 8), spreads=(0, 16, 32, 64, 128, 256), passes=2,
         verbose=False):
    """Tunes `sym` (an uploaded api.Symbolic) for this batch in place.

    Psp, Qsp: [B, n]; Vm0, Va0: [B, n] start states.  Returns a dict with the
    chosen settings, the best time in ms and the number of timed launches.
    """
    t0 = time.time()
    timer = _Timer(sym, yval, bus_type, Psp, Qsp, Vm0, Va0, tol, max_iter, reps)
    Bn = Psp.shape[0]
    if Bn == 1:
        interleaves = (1,)
    else:
        spreads = (0,)  # a batch always runs one workgroup per case
    base_map = sym.get_mapping().copy()
    best = (float("inf"), None)
    for T, bud, C in itertools.product(threads, budgets, interleaves):
        sym.set_launch(T, bud, C)
        for G in spreads:
            sym.set_spread(G)
            ms = timer()
            if verbose:
                print(f"[tune] T={T} budget={bud} C={C} spread={G}: {ms:.3f} ms", flush=True)
            if ms < best[0]:
                best = (ms, (T, bud, C, G))
    T, bud, C, G = best[1]
    sym.set_launch(T, bud, C)
    sym.set_spread(G)
    mapping = base_map.copy()
    best_ms = best[0]
    classes = level_classes(sym)
    for _ in range(passes):
        improved = False
        for (lo, hi), idx in classes:
            cur = int(mapping[idx[0]])
            for g in LANES:
                if g == cur or g > T:
                    continue
                trial = mapping.copy()
                trial[idx] = g
                sym.set_mapping(trial)
                ms = timer()
                if verbose:
                    print(f"[tune] width {lo}-{hi}: lanes {g}: {ms:.3f} ms", flush=True)
                if ms < best_ms * 0.995:
                    best_ms, mapping, cur, improved = ms, trial, g, True
            sym.set_mapping(mapping)
        if not improved:
            break
    sym.set_mapping(mapping)
    return dict(threads=T, tail_budget=bud, interleave=C, spread=G, mapping=mapping.tolist(),
                ms=best_ms, launches=timer.runs, seconds=time.time() - t0)


def apply(sym, settings):
    """Re-applies settings returned by :func:`tune` to a symbolic of the same grid."""
    sym.set_launch(settings["threads"], settings["tail_budget"], settings["interleave"])
    sym.set_spread(settings.get("spread", 0))
    sym.set_mapping(np.asarray(settings["mapping"], np.int32))
