"""CPU oracle for weighted-least-squares state estimation (test
infrastructure only: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module).

The paper lists state estimation among the applications studied on the
same graph machinery (Sec. IV) but gives no formulation; this follows the
textbook WLS estimator (our reading): measurements z = h(x) + e with
weights w = 1/sigma^2, state x = (theta of every bus but the reference,
|V| of every bus), Gauss-Newton steps G dx = H^T W (z - h(x)) with the gain
matrix G = H^T W H, until max|dx| < tol.

Measurement kinds: 1 |V_i|, 2 P_i, 3 Q_i (bus injections), 4 P_ft, 5 Q_ft
(flow at the from end of branch e).  h uses the oracle's injections and
branch flows; H is written from complex differentiation of S = V conj(I)
and checked against finite differences in the tests.  Plain scipy sparse
algebra in fp64.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import oracle as O

VM, PINJ, QINJ, PFLOW, QFLOW = 1, 2, 3, 4, 5


def measure(grid, Y, Vm, Va, kinds, locs):
    """h(x) for the measurement set (kinds, locs)."""
    P, Q = O.injections(Y, Vm, Va)
    Pft, Qft, _, _ = O.branch_flows(grid, Vm, Va)
    h = np.empty(len(kinds))
    for t, src in ((VM, Vm), (PINJ, P), (QINJ, Q), (PFLOW, Pft), (QFLOW, Qft)):
        sel = kinds == t
        h[sel] = src[locs[sel]]
    return h


def _columns(n, slack):
    """Column of theta_b (-1 at the reference) and of |V|_b."""
    ct = -np.ones(n, np.int64)
    others = [b for b in range(n) if b != slack]
    ct[others] = np.arange(n - 1)
    cv = n - 1 + np.arange(n)
    return ct, cv


def jacobian(grid, Y, Vm, Va, kinds, locs, slack=0):
    """Sparse H = dh/dx, x = (theta of non-reference buses, |V| of all)."""
    n = grid.n
    ct, cv = _columns(n, slack)
    V = Vm * np.exp(1j * Va)
    Yc = sp.csr_matrix((Y.G + 1j * Y.B, Y.col, Y.rowptr), shape=(n, n))
    I = Yc @ V
    dV = sp.diags(V)
    # dS/dtheta = j diag(V) conj(diag(I) - Y diag(V)),
    # dS/d|V|  = diag(V) conj(Y diag(V/|V|)) + conj(diag(I)) diag(V/|V|)
    dS_dth = 1j * dV @ (sp.diags(I) - Yc @ dV).conj()
    dS_dvm = dV @ (Yc @ sp.diags(V / Vm)).conj() + sp.diags(I.conj()) @ sp.diags(V / Vm)
    dS_dth = dS_dth.tocsr()
    dS_dvm = dS_dvm.tocsr()
    rows, cols, vals = [], [], []

    def put(r, c, v):
        if c >= 0:
            rows.append(r)
            cols.append(c)
            vals.append(v)

    f, t = grid.f, grid.t
    for r, (kind, loc) in enumerate(zip(kinds, locs)):
        if kind == VM:
            put(r, cv[loc], 1.0)
        elif kind in (PINJ, QINJ):
            part = np.real if kind == PINJ else np.imag
            for M, cmap in ((dS_dth, ct), (dS_dvm, cv)):
                row = M.getrow(loc)
                for k, v in zip(row.indices, row.data):
                    put(r, cmap[k], part(v))
        else:
            e = loc
            a, b = f[e], t[e]
            y = 1.0 / (grid.r[e] + 1j * grid.x[e])
            yff, yft = y + 0.5j * grid.b[e], -y
            c = yft * V[b]
            # S_f = |V_f|^2 conj(yff) + V_f conj(yft V_t)
            d_thf = 1j * V[a] * np.conj(c)
            d_tht = -1j * V[a] * np.conj(c)
            d_vf = 2 * Vm[a] * np.conj(yff) + (V[a] / Vm[a]) * np.conj(c)
            d_vt = V[a] * np.conj(c) / Vm[b]
            part = np.real if kind == PFLOW else np.imag
            put(r, ct[a], part(d_thf))
            put(r, ct[b], part(d_tht))
            put(r, cv[a], part(d_vf))
            put(r, cv[b], part(d_vt))
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(kinds), 2 * n - 1))


@dataclass
class SEResult:
    Vm: np.ndarray
    Va: np.ndarray
    iters: int
    norm: float  # max |dx| of the last step
    status: int  # 0 converged, 6 not converged, 7 non-finite


def estimate(grid, kinds, locs, z, w, Vm0, Va0, tol=1e-8, max_iter=20, slack=0, Y=None):
    """Gauss-Newton WLS from (Vm0, Va0): G dx = H^T W (z - h), x += dx,
    stop when the applied step has max|dx| < tol."""
    Y = O.grid_ybus(grid) if Y is None else Y
    kinds = np.asarray(kinds)
    locs = np.asarray(locs)
    n = grid.n
    ct, cv = _columns(n, slack)
    Vm = np.array(Vm0, np.float64)
    Va = np.array(Va0, np.float64)
    W = sp.diags(np.asarray(w, np.float64))
    it, nrm = 0, np.inf
    while it < max_iter:
        r = z - measure(grid, Y, Vm, Va, kinds, locs)
        H = jacobian(grid, Y, Vm, Va, kinds, locs, slack)
        G = (H.T @ W @ H).tocsc()
        dx = spla.spsolve(G, H.T @ (W @ r))
        if not np.all(np.isfinite(dx)):
            return SEResult(Vm, Va, it, np.nan, 7)
        Va[ct >= 0] += dx[ct[ct >= 0]]
        Vm += dx[cv]
        it += 1
        nrm = float(np.abs(dx).max())
        if nrm < tol:
            return SEResult(Vm, Va, it, nrm, 0)
    return SEResult(Vm, Va, it, nrm, 6)


def full_measurement_set(grid):
    """|V| and P, Q at every bus, P_ft and Q_ft at every branch."""
    n, m = grid.n, grid.m
    kinds = np.concatenate([np.full(n, VM), np.full(n, PINJ), np.full(n, QINJ),
                            np.full(m, PFLOW), np.full(m, QFLOW)]).astype(np.int8)
    locs = np.concatenate([np.arange(n), np.arange(n), np.arange(n), np.arange(m),
                           np.arange(m)]).astype(np.int32)
    return kinds, locs
