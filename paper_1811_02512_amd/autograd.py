"""Differentiable power flow: (P_sp, Q_sp, branch x) -> (|V|, theta).

The forward runs the batched Newton-Raphson kernel and keeps the block LDU
factors of the Jacobian at the returned state.  The backward reuses them in
one fused adjoint call (pf_adjoint):
  g      = dL/d(theta, |V|) gathered into position order
  J^T l  = g by transposed level-scheduled solves
  dL/dP_sp, dL/dQ_sp, dL/dx from l
By the implicit-function theorem on F(x, p) = 0, dL/dp = -l^T dF/dp.  A case
that did not converge (or met a zero pivot, or went non-finite) has no
factors at a solution: its gradients come back NaN, and the forward's
per-case status is available to the caller.  All arithmetic runs in the HIP
kernels; this module only marshals tensors.
"""
from __future__ import annotations

import torch

from . import binding as B


class PowerFlowFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Psp, Qsp, x, sym, r, b, bus_type, Vm0, Va0, tol, max_iter, ysh):
        Bn, n = Psp.shape
        y = sym.build_ybus(r, x, b, ysh)
        Vm = Vm0.expand(Bn, n).contiguous().clone()
        Va = Va0.expand(Bn, n).contiguous().clone()
        yv = y[0] if y.shape[0] == 1 else y
        iters, norm, status, ws = sym.newton(yv, bus_type, Psp, Qsp, Vm, Va, tol, max_iter,
                                             keep_factors=True)
        ctx.sym = sym
        ctx.x_shared = x.dim() == 1
        ctx.save_for_backward(Vm, Va, ws, r, x, bus_type, status)
        ctx.mark_non_differentiable(status, iters)
        return Vm, Va, status, iters

    @staticmethod
    def backward(ctx, gVm, gVa, _gs, _gi):
        Vm, Va, ws, r, x, bus_type, status = ctx.saved_tensors
        sym = ctx.sym
        info = sym.info
        Bn, n = Vm.shape
        dev = Vm.device
        gVm = None if gVm is None else gVm.contiguous()
        gVa = None if gVa is None else gVa.contiguous()
        tstride = 0 if bus_type.dim() == 1 else n
        lam = torch.empty(Bn, 2 * info.nn, dtype=torch.float64, device=dev)
        gP = torch.empty(Bn, n, dtype=torch.float64, device=dev)
        gQ = torch.empty(Bn, n, dtype=torch.float64, device=dev)
        m = x.shape[-1]
        gx = torch.empty(m if ctx.x_shared else Bn * m, dtype=torch.float64, device=dev)
        bstride = 0 if r.dim() == 1 else m
        B.pf_adjoint(sym.h, Bn, ws, info.ws_doubles, gVm, gVa, n, bus_type, tstride, Vm, Va, n,
                     r, x, bstride, status, lam, 2 * info.nn, gP, gQ, n, gx,
                     1 if ctx.x_shared else 0)
        if not ctx.x_shared:
            gx = gx.view(Bn, m)
        return gP, gQ, gx, None, None, None, None, None, None, None, None, None


def power_flow(sym, Psp, Qsp, x, r, b, bus_type, Vm0, Va0, tol=1e-8, max_iter=20, ysh=None,
               with_status=False):
    """Batched differentiable power flow.

    sym: uploaded api.Symbolic; Psp, Qsp: [B, n]; x: [m] (shared, gradient
    summed over cases) or [B, m]; r, b like x (r held fixed); bus_type:
    int8 [n]; Vm0, Va0: [n] start state; ysh: bus shunts (g, b) [n, 2] or
    None.  Returns (Vm, Va), each [B, n], and with with_status also the
    per-case status and iteration counts (int32 [B]); cases whose status is
    not PF_OK get NaN gradients.
    """
    Vm, Va, status, iters = PowerFlowFunction.apply(Psp, Qsp, x, sym, r, b, bus_type, Vm0, Va0,
                                                    tol, max_iter, ysh)
    if with_status:
        return Vm, Va, status, iters
    return Vm, Va
