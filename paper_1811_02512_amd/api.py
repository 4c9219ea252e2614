"""Convenience layer over the C ABI: owns handles and torch device buffers.

Nothing here computes power-flow quantities; every numeric step runs in the
HIP kernels behind :mod:`paper_1811_02512_amd.binding`.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def _dev(device):
    return torch.device(device if device is not None else "cuda")


class Symbolic:
    """Host analysis of one grid topology plus its device copy."""

    def __init__(self, n, f, t, slack=0, ordering=B.PF_ORDER_MINDEG):
        self.h = B.pf_analyze(n, f, t, slack, ordering)
        self.n = int(n)
        self.f = np.ascontiguousarray(f, np.int32)
        self.t = np.ascontiguousarray(t, np.int32)
        self.buf = None
        self.device = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and B is not None and getattr(B, "lib", None) is not None:
            try:
                B.pf_symbolic_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.h = None

    @property
    def info(self):
        return B.pf_symbolic_info(self.h)

    def export(self):
        return B.pf_symbolic_export(self.h)

    def ybus_pattern(self):
        return B.pf_symbolic_ybus_pattern(self.h)

    def get_mapping(self):
        return B.pf_symbolic_get_mapping(self.h)

    def set_mapping(self, lanes):
        B.pf_symbolic_set_mapping(self.h, lanes)
        if self.buf is not None:
            B.pf_symbolic_upload(self.h, self.buf)

    def set_launch(self, threads=0, tail_lds_budget=65536, interleave=4):
        B.pf_symbolic_set_launch(self.h, threads, tail_lds_budget, interleave)
        if self.buf is not None:
            self.upload(self.device)

    def set_spread(self, workgroups):
        """Workgroups of a one-case Newton launch (0: one workgroup)."""
        B.pf_symbolic_set_spread(self.h, workgroups)

    def upload(self, device=None):
        dev = _dev(device)
        nbytes = self.info.dev_bytes
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != dev:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        B.pf_symbolic_upload(self.h, self.buf)
        self.device = dev
        return self

    # -- helpers allocating outputs ------------------------------------------------
    def build_ybus(self, r, x, b, ysh=None):
        """r, x, b: [m] or [B, m] fp64 device tensors; ysh: bus shunts (g, b)
        as [n, 2] or [B, n, 2], or None -> yval [B, 2*nnz_y]."""
        info = self.info
        Bn = max(r.shape[0] if r.dim() == 2 else 1,
                 ysh.shape[0] if ysh is not None and ysh.dim() == 3 else 1)
        bstride = r.shape[-1] if r.dim() == 2 else 0
        y = torch.empty(Bn, 2 * info.nnz_y, dtype=torch.float64, device=r.device)
        B.pf_build_ybus(self.h, Bn, r, x, b, bstride, y, 2 * info.nnz_y, ysh, _shunt_stride(ysh))
        return y

    def workspace(self, Bn, device=None):
        """pf_newton workspace for Bn cases: whole interleaved groups of
        info.ws_interleave cases, one row of ws_doubles per case."""
        info = self.info
        C = B.pf_newton_interleave(self.h, Bn)
        rows = -(-Bn // C) * C
        return torch.empty(rows, info.ws_doubles, dtype=torch.float64,
                           device=_dev(device or self.device))

    def newton(self, yval, bus_type, Psp, Qsp, Vm, Va, tol=1e-8, max_iter=20,
               keep_factors=False, ws=None):
        """Batched NR in place on Vm, Va ([B, n]).  Returns (iters, norm, status, ws)."""
        Bn = Vm.shape[0]
        info = self.info
        if ws is None:
            ws = self.workspace(Bn, Vm.device)
        iters = torch.empty(Bn, dtype=torch.int32, device=Vm.device)
        norm = torch.empty(Bn, dtype=torch.float64, device=Vm.device)
        status = torch.empty(Bn, dtype=torch.int32, device=Vm.device)
        B.pf_newton(self.h, Bn, yval, _stride(yval), bus_type, _stride(bus_type), Psp, Qsp,
                    _stride(Psp), Vm, Va, Vm.shape[-1], tol, max_iter,
                    B.PF_NEWTON_KEEP_FACTORS if keep_factors else 0, ws, info.ws_doubles,
                    iters, norm, status)
        return iters, norm, status, ws

    # -- fast decoupled power flow and branch flows ---------------------------
    def fdpf_factors(self, r, x, b, bus_type, ysh=None):
        """B' and B'' built and factored on the device.  r, x, b: [m] (shared)
        or [B, m]; bus_type: [n] or [B, n]; ysh: bus shunts [n, 2] or None.
        Returns (mat, status) with mat [1 or B, fd_mat_doubles]."""
        info = self.info
        Bn = 1 if r.dim() == 1 else r.shape[0]
        mat = torch.empty(Bn, info.fd_mat_doubles, dtype=torch.float64, device=r.device)
        status = torch.empty(Bn, dtype=torch.int32, device=r.device)
        B.pf_fdpf_matrices(self.h, Bn, r, x, b, _stride(r), bus_type, _stride(bus_type), mat,
                           info.fd_mat_doubles, ysh, _shunt_stride(ysh))
        B.pf_fdpf_factor(self.h, Bn, mat, info.fd_mat_doubles, status)
        return mat, status

    def fdpf(self, yval, bus_type, Psp, Qsp, Vm, Va, mat, tol=1e-8, max_iter=40, ws=None):
        """Batched fast decoupled power flow in place on Vm, Va ([B, n]) with
        factors from fdpf_factors (one row shared, or one per case).
        Returns (iters, norm, status, ws)."""
        Bn = Vm.shape[0]
        info = self.info
        if ws is None:
            ws = torch.empty(Bn, info.fd_ws_doubles, dtype=torch.float64, device=Vm.device)
        iters = torch.empty(Bn, dtype=torch.int32, device=Vm.device)
        norm = torch.empty(Bn, dtype=torch.float64, device=Vm.device)
        status = torch.empty(Bn, dtype=torch.int32, device=Vm.device)
        mstride = 0 if mat.shape[0] == 1 else info.fd_mat_doubles
        B.pf_fdpf(self.h, Bn, yval, _stride(yval), bus_type, _stride(bus_type), Psp, Qsp,
                  _stride(Psp), Vm, Va, Vm.shape[-1], mat, mstride, tol, max_iter, ws,
                  info.fd_ws_doubles, iters, norm, status)
        return iters, norm, status, ws

    def branch_flows(self, r, x, b, Vm, Va):
        """(Pft, Qft, Ptf, Qtf), each [B, m], of the states Vm, Va ([B, n])."""
        Bn, m = Vm.shape[0], self.info.m
        out = [torch.empty(Bn, m, dtype=torch.float64, device=Vm.device) for _ in range(4)]
        B.pf_branch_flows(self.h, Bn, r, x, b, _stride(r), Vm, Va, Vm.shape[-1], *out, m)
        return tuple(out)


def _stride(t):
    """0 for a shared [k] array, row length for a [B, k] array."""
    return 0 if t.dim() == 1 else t.shape[-1]


def _shunt_stride(ysh):
    """Doubles between cases of a bus-shunt array: 0 for a shared [n, 2]
    array (or none), 2 n for [B, n, 2]."""
    return 0 if ysh is None or ysh.dim() < 3 else 2 * ysh.shape[-2]


class MultiPlan:
    """Batch of cases with their own symbolic analyses (N-1, mixed grids)."""

    def __init__(self, syms, device=None):
        self.syms = list(syms)
        self.p = B.pf_multi_create([s.h for s in self.syms])
        nbytes, self.offs = B.pf_multi_info(self.p, len(self.syms))
        self.buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=_dev(device))
        B.pf_multi_upload(self.p, self.buf)

    def __del__(self):
        p = getattr(self, "p", None)
        if p is not None and B is not None and getattr(B, "lib", None) is not None:
            try:
                B.pf_multi_destroy(p)
            except Exception:  # interpreter shutdown
                pass
            self.p = None

    def set_spread(self, workgroups):
        """Workgroups of the batch's Newton launch (0: one per case); the
        plan's device table is rebuilt and uploaded again."""
        B.pf_multi_set_spread(self.p, workgroups)
        nbytes, _ = B.pf_multi_info(self.p, len(self.syms))
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.buf.device)
        B.pf_multi_upload(self.p, self.buf)

    def concat(self, arrays, key, dtype, device=None):
        """Concatenate per-case host arrays into one device tensor."""
        tot = int(self.offs[key][-1])
        out = np.zeros(max(tot, 1), dtype)
        for g, a in enumerate(arrays):
            out[self.offs[key][g]:self.offs[key][g + 1]] = a
        return torch.from_numpy(out).to(_dev(device))

    def split(self, t, key):
        t = t.cpu().numpy()
        o = self.offs[key]
        return [t[o[g]:o[g + 1]] for g in range(len(self.syms))]


class StateEstimator:
    """WLS state estimation on the device for a fixed measurement set
    (kinds PF_MEAS_*, locations bus or branch)."""

    def __init__(self, n, from_, to, kind, loc, slack=0, device=None, threads=0,
                 tail_lds_budget=65536):
        import numpy as np

        self.h = B.pf_se_analyze(n, np.asarray(from_), np.asarray(to), slack, kind, loc)
        B.pf_se_set_launch(self.h, threads, tail_lds_budget)
        self.dims = B.pf_se_info(self.h)
        self.device = _dev(device)
        self.buf = torch.empty(self.dims.dev_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.buf.data_ptr()
        self._off = (-base) % 256
        B.pf_se_upload(self.h, self.buf[self._off:], self.dims.dev_bytes)

    def workspace(self, Bn, device=None):
        """Scratch for Bn cases: whole groups of four cases of ws_doubles each."""
        rows = -(-Bn // 4) * 4
        return torch.empty(rows * self.dims.ws_doubles, dtype=torch.float64,
                           device=_dev(device or self.device))

    def estimate(self, r, x, b, z, w, Vm, Va, tol=1e-8, max_iter=20, ws=None, ysh=None):
        """In place on Vm, Va ([B, n]); z, w: [M] shared or [B, M]; r, x, b:
        [m] shared or [B, m]; ysh: bus shunts [n, 2] or [B, n, 2] or None.
        Returns (iters, norm, status, ws)."""
        Bn = Vm.shape[0]
        if ws is None:
            ws = self.workspace(Bn, Vm.device)
        iters = torch.empty(Bn, dtype=torch.int32, device=Vm.device)
        norm = torch.empty(Bn, dtype=torch.float64, device=Vm.device)
        status = torch.empty(Bn, dtype=torch.int32, device=Vm.device)
        B.pf_se_estimate(self.h, Bn, r, x, b, _stride(r), z, _stride(z), w, _stride(w), Vm, Va,
                         Vm.shape[-1], tol, max_iter, ws, ws.numel(), iters, norm, status, ysh,
                         _shunt_stride(ysh))
        return iters, norm, status, ws

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and B is not None and getattr(B, "lib", None) is not None:
            try:
                B.pf_se_destroy(h)
            except Exception:
                pass
            self.h = None
