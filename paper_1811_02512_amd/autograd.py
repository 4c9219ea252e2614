"""Differentiable power flow: (P_sp, Q_sp, branch x) -> (|V|, theta).

The forward runs the batched Newton-Raphson kernel and keeps the block LDU
factors of the Jacobian at the returned state.  The backward reuses them:
  g      = dL/d(theta, |V|) gathered into position order   (pf_adjoint_rhs)
  J^T l  = g by transposed level-scheduled solves            (pf_solve, transpose=1)
  dL/dP_sp, dL/dQ_sp, dL/dx from l                          (pf_adjoint_params)
By the implicit-function theorem on F(x, p) = 0, dL/dp = -l^T dF/dp.  All
arithmetic runs in the HIP kernels; this module only marshals tensors.
"""
from __future__ import annotations

import torch

from . import binding as B


class PowerFlowFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Psp, Qsp, x, sym, r, b, bus_type, Vm0, Va0, tol, max_iter):
        Bn, n = Psp.shape
        info = sym.info
        y = sym.build_ybus(r, x, b)
        Vm = Vm0.expand(Bn, n).contiguous().clone()
        Va = Va0.expand(Bn, n).contiguous().clone()
        yv = y[0] if x.dim() == 1 else y
        iters, norm, status, ws = sym.newton(yv, bus_type, Psp, Qsp, Vm, Va, tol, max_iter,
                                             keep_factors=True)
        ctx.sym = sym
        ctx.x_shared = x.dim() == 1
        ctx.save_for_backward(Vm, Va, ws, r, x, bus_type)
        ctx.info = (iters, norm, status)
        ctx.mark_non_differentiable()
        return Vm, Va

    @staticmethod
    def backward(ctx, gVm, gVa):
        Vm, Va, ws, r, x, bus_type = ctx.saved_tensors
        sym = ctx.sym
        info = sym.info
        Bn, n = Vm.shape
        dev = Vm.device
        gVm = torch.zeros_like(Vm) if gVm is None else gVm.contiguous()
        gVa = torch.zeros_like(Va) if gVa is None else gVa.contiguous()
        tstride = 0 if bus_type.dim() == 1 else n
        lam = torch.empty(Bn, 2 * info.nn, dtype=torch.float64, device=dev)
        B.pf_adjoint_rhs(sym.h, Bn, gVm, gVa, n, bus_type, tstride, lam, 2 * info.nn)
        B.pf_solve(sym.h, Bn, ws, info.ws_doubles, lam, 2 * info.nn, 1,
                   B.pf_newton_interleave(sym.h, Bn))
        gP = torch.empty(Bn, n, dtype=torch.float64, device=dev)
        gQ = torch.empty(Bn, n, dtype=torch.float64, device=dev)
        m = x.shape[-1]
        gx = torch.empty(m if ctx.x_shared else Bn * m, dtype=torch.float64, device=dev)
        bstride = 0 if r.dim() == 1 else m
        B.pf_adjoint_params(sym.h, Bn, lam, 2 * info.nn, bus_type, tstride, Vm, Va, n, r, x,
                            bstride, gP, gQ, n, gx, 1 if ctx.x_shared else 0)
        if not ctx.x_shared:
            gx = gx.view(Bn, m)
        return gP, gQ, gx, None, None, None, None, None, None, None, None


def power_flow(sym, Psp, Qsp, x, r, b, bus_type, Vm0, Va0, tol=1e-8, max_iter=20):
    """Batched differentiable power flow.

    sym: uploaded api.Symbolic; Psp, Qsp: [B, n]; x: [m] (shared, gradient
    summed over cases) or [B, m]; r, b like x (r held fixed); bus_type:
    int8 [n]; Vm0, Va0: [n] start state.  Returns (Vm, Va), each [B, n].
    """
    return PowerFlowFunction.apply(Psp, Qsp, x, sym, r, b, bus_type, Vm0, Va0, tol, max_iter)
