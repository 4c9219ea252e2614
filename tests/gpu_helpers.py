"""Shared helpers for the GPU tests: stage seeded grids on the device and run
the oracle on the same inputs."""
from __future__ import annotations

import functools
import sys

import numpy as np

import gridgen


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def grid(n, seed):
    return gridgen.make_grid(n, seed)


@functools.lru_cache(maxsize=None)
def shunt_grid(n, seed, shunt_seed):
    """The generated grid with seeded bus shunts (capacitors, reactors)."""
    return gridgen.with_shunts(gridgen.make_grid(n, seed), shunt_seed)


def dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


class Staged:
    """One grid on the device: symbolic, Y values, per-bus inputs."""

    def __init__(self, g, ordering=0):
        import torch

        from paper_1811_02512_amd import api

        self.g = g
        self.sym = api.Symbolic(g.n, g.f, g.t, 0, ordering).upload()
        self.info = self.sym.info
        self.r = dev(g.r)
        self.x = dev(g.x)
        self.b = dev(g.b)
        # bus shunts (g, b) per bus, or None when the grid has none
        self.ysh = dev(g.ysh) if g.has_shunts else None
        self.yval = self.sym.build_ybus(self.r, self.x, self.b, self.ysh)
        self.type = dev(g.bus_type.astype(np.int8))
        self.Psp = dev(g.Psp)
        self.Qsp = dev(g.Qsp)
        Vm0, Va0 = g.flat_start()
        self.Vm0 = dev(Vm0)
        self.Va0 = dev(Va0)
        torch.cuda.synchronize()

    def newton(self, Bn=1, Psp=None, Qsp=None, tol=1e-8, max_iter=20, keep=False):
        Vm = self.Vm0.repeat(Bn, 1).contiguous()
        Va = self.Va0.repeat(Bn, 1).contiguous()
        P = self.Psp if Psp is None else Psp
        Q = self.Qsp if Qsp is None else Qsp
        iters, norm, status, ws = self.sym.newton(self.yval[0], self.type, P, Q, Vm, Va, tol,
                                                  max_iter, keep)
        return Vm, Va, iters, norm, status, ws
