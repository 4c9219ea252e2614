"""N-1 contingency screening (Sec. III: industrial EMS run the fast decoupled
method first and Newton-Raphson only where it does not converge, over
thousands of contingencies).

Every outage is solved on the base grid's symbolic analysis: the outaged
branch stays in the pattern with its admittance opened (series r = 0,
x = 1e300, charging 0, which puts exact zeros in Y and B'' and 1e-300 in B'),
so one analysis, one set of index arrays and the shared-pattern batched
kernels serve the whole batch; no per-outage re-analysis.  The steps are the
library's kernels: admittances (pf_build_ybus), fast decoupled matrices and
factors per outage (pf_fdpf_matrices, pf_fdpf_factor), the batched fast
decoupled iteration (pf_fdpf), batched NR for the cases it leaves
unconverged (pf_newton, from flat start), and branch flows of every case
(pf_branch_flows).  The module only prepares per-case arrays and picks the
fallback cases.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import binding as B

OPEN_X = 1e300


@dataclass
class Screening:
    Vm: torch.Tensor        # [C, n]
    Va: torch.Tensor        # [C, n]
    status: torch.Tensor    # [C] int32, final status
    method: torch.Tensor    # [C] int8: 1 fast decoupled, 2 Newton-Raphson
    iters: torch.Tensor     # [C] int32, iterations of the method that finished
    flows: tuple            # (Pft, Qft, Ptf, Qtf), each [C, m]
    fallback: int           # cases sent to Newton-Raphson


def outage_branches(r, x, b, outages):
    """Per-case branch arrays [C, m] with branch outages[c] opened."""
    C = len(outages)
    idx = torch.as_tensor(outages, dtype=torch.long, device=r.device)
    rows = torch.arange(C, device=r.device)
    rr = r.expand(C, -1).clone()
    xx = x.expand(C, -1).clone()
    bb = b.expand(C, -1).clone()
    rr[rows, idx] = 0.0
    xx[rows, idx] = OPEN_X
    bb[rows, idx] = 0.0
    return rr, xx, bb


def screen(sym, r, x, b, bus_type, Psp, Qsp, Vm0, Va0, outages, tol=1e-8, fdpf_iter=40,
           nr_iter=20, fdpf_first=True, ysh=None):
    """Screens the outages of branches `outages` on the base symbolic `sym`
    (uploaded api.Symbolic).  r, x, b: [m]; bus_type, Psp, Qsp, Vm0, Va0: [n]
    base-case inputs shared by all outages; ysh: bus shunts [n, 2] (g, b) or
    None.  Returns a Screening."""
    info = sym.info
    dev = r.device
    C = len(outages)
    n, m = info.n, info.m
    rr, xx, bb = outage_branches(r, x, b, outages)
    yv = torch.empty(C, 2 * info.nnz_y, dtype=torch.float64, device=dev)
    B.pf_build_ybus(sym.h, C, rr, xx, bb, m, yv, 2 * info.nnz_y, ysh, 0)
    Vm = Vm0.expand(C, n).contiguous()
    Va = Va0.expand(C, n).contiguous()
    status = torch.full((C,), -1, dtype=torch.int32, device=dev)
    iters = torch.zeros(C, dtype=torch.int32, device=dev)
    method = torch.zeros(C, dtype=torch.int8, device=dev)
    todo = torch.arange(C, device=dev)
    if fdpf_first:
        mat = torch.empty(C, info.fd_mat_doubles, dtype=torch.float64, device=dev)
        fst = torch.empty(C, dtype=torch.int32, device=dev)
        B.pf_fdpf_matrices(sym.h, C, rr, xx, bb, m, bus_type, 0, mat, info.fd_mat_doubles,
                           ysh, 0)
        B.pf_fdpf_factor(sym.h, C, mat, info.fd_mat_doubles, fst)
        ws = torch.empty(C, info.fd_ws_doubles, dtype=torch.float64, device=dev)
        B.pf_fdpf(sym.h, C, yv, 2 * info.nnz_y, bus_type, 0, Psp, Qsp, 0, Vm, Va, n, mat,
                  info.fd_mat_doubles, tol, fdpf_iter, ws, info.fd_ws_doubles, iters, None,
                  status)
        status = torch.where(fst == 0, status, fst)
        method.fill_(1)
        todo = torch.nonzero(status != 0).flatten()
    fallback = int(todo.numel())
    if fallback:
        yk = yv[todo].contiguous()
        Vk = Vm0.expand(fallback, n).contiguous()
        Ak = Va0.expand(fallback, n).contiguous()
        it = torch.empty(fallback, dtype=torch.int32, device=dev)
        st = torch.empty(fallback, dtype=torch.int32, device=dev)
        ws = sym.workspace(fallback, dev)
        B.pf_newton(sym.h, fallback, yk, 2 * info.nnz_y, bus_type, 0, Psp, Qsp, 0, Vk, Ak, n, tol,
                    nr_iter, 0, ws, info.ws_doubles, it, None, st)
        Vm[todo] = Vk
        Va[todo] = Ak
        iters[todo] = it
        status[todo] = st
        method[todo] = 2
    flows = tuple(torch.empty(C, m, dtype=torch.float64, device=dev) for _ in range(4))
    B.pf_branch_flows(sym.h, C, rr, xx, bb, m, Vm, Va, n, *flows, m)
    return Screening(Vm, Va, status, method, iters, flows, fallback)
