"""ctypes binding of libpf (include/pf.h): argument marshalling only.

Every function here has the name of the C entry point it calls and takes
torch tensors (device memory) or numpy arrays (host memory) in place of raw
pointers.  All arithmetic happens in the HIP kernels of libpf.so; if the
library is missing this module raises at import time.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PF_LIBPF selects another build of the same sources (the sanitizer check)
LIB_PATH = os.environ.get("PF_LIBPF") or os.path.join(_HERE, "libpf.so")

PF_OK, PF_E_INVALID, PF_E_HIP, PF_E_WORKSPACE, PF_E_DISCONNECTED = 0, 1, 2, 3, 4
PF_E_ZERO_PIVOT, PF_E_NOT_CONVERGED, PF_E_NONFINITE = 5, 6, 7
PF_ORDER_MINDEG, PF_ORDER_NATURAL = 0, 1
PF_BUS_PQ, PF_BUS_PV, PF_BUS_SLACK = 1, 2, 3
PF_NEWTON_KEEP_FACTORS = 1


class PfError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


class pf_info(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("nn", C.c_int32), ("slack", C.c_int32),
                ("nnz_y", C.c_int64), ("nnz_l", C.c_int64), ("n_upd", C.c_int64),
                ("nlevels", C.c_int32), ("max_level_width", C.c_int32),
                ("vals_doubles", C.c_int64), ("ws_doubles", C.c_int64),
                ("dev_bytes", C.c_size_t), ("tail_levels", C.c_int32),
                ("tail_nodes", C.c_int32), ("tail_lds_bytes", C.c_int32),
                ("threads", C.c_int32), ("tail_clique", C.c_int32),
                ("ws_interleave", C.c_int32), ("lu_offset", C.c_int64),
                ("fd_mat_doubles", C.c_int64), ("fd_ws_doubles", C.c_int64),
                ("spread", C.c_int32), ("sub_levels", C.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libpf.so not built ({LIB_PATH}); run __graft_entry__.build()")

# torch bundles its own HIP runtime under the same soname as the system one.
# Loading torch first makes libpf bind to that already-loaded runtime, so
# the process holds one HIP runtime and torch's device memory and streams are
# valid in libpf's calls.
import torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)

_vp, _i, _i64, _d = C.c_void_p, C.c_int, C.c_int64, C.c_double
class pf_se_dims(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("measurements", C.c_int32),
                ("partials", C.c_int64), ("gain_nnz_l", C.c_int64), ("gain_levels", C.c_int32),
                ("contributions", C.c_int64), ("ws_doubles", C.c_int64),
                ("dev_bytes", C.c_size_t)]


_SIGS = {
    "pf_version": ([], C.c_char_p),
    "pf_status_string": ([_i], C.c_char_p),
    "pf_last_error": ([], C.c_char_p),
    "pf_analyze": ([_i, _i, _vp, _vp, _i, _i, C.POINTER(_vp)], _i),
    "pf_symbolic_info": ([_vp, C.POINTER(pf_info)], _i),
    "pf_symbolic_export": ([_vp] + [_vp] * 7, _i),
    "pf_symbolic_set_mapping": ([_vp, _vp], _i),
    "pf_symbolic_get_mapping": ([_vp, _vp], _i),
    "pf_symbolic_set_launch": ([_vp, _i, _i64, _i], _i),
    "pf_symbolic_set_spread": ([_vp, _i], _i),
    "pf_symbolic_set_spread_wait": ([_vp, C.c_uint64], _i),
    "pf_newton_interleave": ([_vp, _i], _i),
    "pf_symbolic_upload": ([_vp, _vp, C.c_size_t, _vp], _i),
    "pf_symbolic_destroy": ([_vp], None),
    "pf_symbolic_ybus_pattern": ([_vp, _vp, _vp], _i),
    "pf_build_ybus": ([_vp, _i, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp], _i),
    "pf_mismatch": ([_vp, _i, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _i64,
                     _vp, _vp, _vp], _i),
    "pf_jacobian": ([_vp, _i, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _i, _vp], _i),
    "pf_factor": ([_vp, _i, _vp, _i64, _i, _vp, _vp, _vp], _i),
    "pf_solve": ([_vp, _i, _vp, _i64, _i, _vp, _i64, _i, _vp], _i),
    "pf_newton": ([_vp, _i, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _d, _i, _i,
                   _vp, _i64, _vp, _vp, _vp, _vp, _vp], _i),
    "pf_adjoint_params": ([_vp, _i, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp,
                           _vp, _i64, _vp, _i, _vp], _i),
    "pf_adjoint_rhs": ([_vp, _i, _vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp], _i),
    "pf_newton_noalloc": ([_vp, _i, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _d,
                           _i, _vp, _vp, _vp, _vp, _vp], _i),
    "pf_adjoint": ([_vp, _i, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _vp,
                    _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _i, _vp], _i),
    "pf_multi_create": ([_i, _vp, C.POINTER(_vp)], _i),
    "pf_multi_info": ([_vp, C.POINTER(C.c_size_t), _vp, _vp, _vp, _vp], _i),
    "pf_multi_upload": ([_vp, _vp, C.c_size_t, _vp], _i),
    "pf_multi_set_spread": ([_vp, _i], _i),
    "pf_build_ybus_multi": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], _i),
    "pf_newton_multi": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _i, _i, _vp, _vp, _vp, _vp,
                         _vp, _vp], _i),
    "pf_multi_destroy": ([_vp], None),
    "pf_fdpf_matrices": ([_vp, _i, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp],
                         _i),
    "pf_fdpf_factor": ([_vp, _i, _vp, _i64, _vp, _vp], _i),
    "pf_fdpf": ([_vp, _i, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _d,
                 _i, _vp, _i64, _vp, _vp, _vp, _vp], _i),
    "pf_branch_flows": ([_vp, _i, _vp, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp,
                         _i64, _vp], _i),
    "pf_se_analyze": ([_i, _i, _vp, _vp, _i, _i, _vp, _vp, C.POINTER(_vp)], _i),
    "pf_se_info": ([_vp, C.POINTER(pf_se_dims)], _i),
    "pf_se_upload": ([_vp, _vp, C.c_size_t, _vp], _i),
    "pf_se_set_launch": ([_vp, _i, _i64], _i),
    "pf_se_estimate": ([_vp, _i, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp,
                        _i64, _d, _i, _vp, _i64, _vp, _vp, _vp, _vp], _i),
    "pf_se_destroy": ([_vp], None),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def last_error() -> str:
    return lib.pf_last_error().decode()


def check(rc: int, fn: str) -> None:
    if rc != PF_OK:
        raise PfError(rc, fn, last_error())


def ptr(t):
    """Device or host address of a torch tensor / numpy array (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def stream_ptr(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _host_i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---- entry points (same names as include/pf.h) ------------------------------
def pf_analyze(n, f, t, slack=0, ordering=PF_ORDER_MINDEG):
    f = _host_i32(f)
    t = _host_i32(t)
    h = C.c_void_p()
    check(lib.pf_analyze(int(n), len(f), ptr(f), ptr(t), int(slack), int(ordering),
                         C.byref(h)), "pf_analyze")
    return h


def pf_symbolic_info(h) -> pf_info:
    info = pf_info()
    check(lib.pf_symbolic_info(h, C.byref(info)), "pf_symbolic_info")
    return info


def pf_symbolic_export(h):
    info = pf_symbolic_info(h)
    nn, nl = info.nn, info.nlevels
    out = dict(perm=np.zeros(nn, np.int32), parent=np.zeros(nn, np.int32),
               level=np.zeros(nn, np.int32), level_ptr=np.zeros(nl + 1, np.int32),
               level_nodes=np.zeros(nn, np.int32), Lp=np.zeros(nn + 1, np.int32),
               Li=np.zeros(max(info.nnz_l, 1), np.int32))
    check(lib.pf_symbolic_export(h, *(ptr(out[k]) for k in
                                      ("perm", "parent", "level", "level_ptr", "level_nodes",
                                       "Lp", "Li"))), "pf_symbolic_export")
    out["Li"] = out["Li"][: info.nnz_l]
    return out


def pf_symbolic_ybus_pattern(h):
    info = pf_symbolic_info(h)
    yptr = np.zeros(info.n + 1, np.int32)
    ycol = np.zeros(max(info.nnz_y, 1), np.int32)
    check(lib.pf_symbolic_ybus_pattern(h, ptr(yptr), ptr(ycol)), "pf_symbolic_ybus_pattern")
    return yptr, ycol[: info.nnz_y]


def pf_symbolic_set_mapping(h, lanes):
    lanes = _host_i32(lanes)
    check(lib.pf_symbolic_set_mapping(h, ptr(lanes)), "pf_symbolic_set_mapping")


def pf_symbolic_set_launch(h, threads=0, tail_lds_budget=65536, interleave=4):
    check(lib.pf_symbolic_set_launch(h, int(threads), int(tail_lds_budget), int(interleave)),
          "pf_symbolic_set_launch")


def pf_symbolic_set_spread(h, workgroups):
    check(lib.pf_symbolic_set_spread(h, int(workgroups)), "pf_symbolic_set_spread")


def pf_symbolic_set_spread_wait(h, ticks):
    check(lib.pf_symbolic_set_spread_wait(h, int(ticks)), "pf_symbolic_set_spread_wait")


def pf_newton_interleave(h, B):
    C = lib.pf_newton_interleave(h, int(B))
    if C < 0:
        raise PfError(PF_E_INVALID, "pf_newton_interleave", last_error())
    return C


def pf_symbolic_get_mapping(h):
    info = pf_symbolic_info(h)
    lanes = np.zeros(max(info.nlevels, 1), np.int32)
    check(lib.pf_symbolic_get_mapping(h, ptr(lanes)), "pf_symbolic_get_mapping")
    return lanes[: info.nlevels]


def pf_symbolic_upload(h, buf, stream=None):
    check(lib.pf_symbolic_upload(h, ptr(buf), buf.numel() * buf.element_size(),
                                 stream_ptr(stream)), "pf_symbolic_upload")


def pf_symbolic_destroy(h):
    lib.pf_symbolic_destroy(h)


def pf_build_ybus(h, B, r, x, b, branch_stride, yval, y_stride, ysh=None, ysh_stride=0,
                  stream=None):
    check(lib.pf_build_ybus(h, B, ptr(r), ptr(x), ptr(b), branch_stride, ptr(ysh), ysh_stride,
                            ptr(yval), y_stride, stream_ptr(stream)), "pf_build_ybus")


def pf_mismatch(h, B, yval, y_stride, bus_type, type_stride, Psp, Qsp, inj_stride, Vm, Va,
                v_stride, rhs, rhs_stride, norm, PQ=None, stream=None):
    check(lib.pf_mismatch(h, B, ptr(yval), y_stride, ptr(bus_type), type_stride, ptr(Psp),
                          ptr(Qsp), inj_stride, ptr(Vm), ptr(Va), v_stride, ptr(rhs),
                          rhs_stride, ptr(norm), ptr(PQ), stream_ptr(stream)), "pf_mismatch")


def pf_jacobian(h, B, yval, y_stride, bus_type, type_stride, Vm, Va, v_stride, vals,
                vals_stride, vals_interleave=1, stream=None):
    check(lib.pf_jacobian(h, B, ptr(yval), y_stride, ptr(bus_type), type_stride, ptr(Vm),
                          ptr(Va), v_stride, ptr(vals), vals_stride, int(vals_interleave),
                          stream_ptr(stream)), "pf_jacobian")


def pf_factor(h, B, vals, vals_stride, status=None, vals_interleave=1, pivot=None,
              stream=None):
    check(lib.pf_factor(h, B, ptr(vals), vals_stride, int(vals_interleave), ptr(status),
                        ptr(pivot), stream_ptr(stream)), "pf_factor")


def pf_solve(h, B, vals, vals_stride, rhs, rhs_stride, transpose=0, vals_interleave=1,
             stream=None):
    check(lib.pf_solve(h, B, ptr(vals), vals_stride, int(vals_interleave), ptr(rhs),
                       rhs_stride, int(transpose), stream_ptr(stream)), "pf_solve")


def pf_newton(h, B, yval, y_stride, bus_type, type_stride, Psp, Qsp, inj_stride, Vm, Va,
              v_stride, tol, max_iter, flags, ws, ws_stride, iters=None, norm=None,
              status=None, pivot=None, stream=None):
    check(lib.pf_newton(h, B, ptr(yval), y_stride, ptr(bus_type), type_stride, ptr(Psp),
                        ptr(Qsp), inj_stride, ptr(Vm), ptr(Va), v_stride, float(tol),
                        int(max_iter), int(flags), ptr(ws), ws_stride, ptr(iters), ptr(norm),
                        ptr(status), ptr(pivot), stream_ptr(stream)), "pf_newton")


def pf_adjoint_params(h, B, lam, lam_stride, bus_type, type_stride, Vm, Va, v_stride, r, x,
                      branch_stride, gP, gQ, g_stride, gx, gx_mode, stream=None):
    check(lib.pf_adjoint_params(h, B, ptr(lam), lam_stride, ptr(bus_type), type_stride,
                                ptr(Vm), ptr(Va), v_stride, ptr(r), ptr(x), branch_stride,
                                ptr(gP), ptr(gQ), g_stride, ptr(gx), int(gx_mode),
                                stream_ptr(stream)), "pf_adjoint_params")


PF_NOALLOC_SCRATCH_BYTES = 64 << 20


def pf_newton_noalloc(h, B, yval, y_stride, bus_type, type_stride, Psp, Qsp, inj_stride, Vm, Va,
                      v_stride, tol, max_iter, iters=None, norm=None, status=None, pivot=None,
                      stream=None):
    check(lib.pf_newton_noalloc(h, B, ptr(yval), y_stride, ptr(bus_type), type_stride,
                                ptr(Psp), ptr(Qsp), inj_stride, ptr(Vm), ptr(Va), v_stride,
                                float(tol), int(max_iter), ptr(iters), ptr(norm), ptr(status),
                                ptr(pivot), stream_ptr(stream)), "pf_newton_noalloc")


def pf_adjoint(h, B, ws, ws_stride, gVm, gVa, gv_stride, bus_type, type_stride, Vm, Va,
               v_stride, r, x, branch_stride, status, lam, lam_stride, gP, gQ, g_stride, gx,
               gx_mode, stream=None):
    check(lib.pf_adjoint(h, B, ptr(ws), ws_stride, ptr(gVm), ptr(gVa), gv_stride, ptr(bus_type),
                         type_stride, ptr(Vm), ptr(Va), v_stride, ptr(r), ptr(x), branch_stride,
                         ptr(status), ptr(lam), lam_stride, ptr(gP), ptr(gQ), g_stride, ptr(gx),
                         int(gx_mode), stream_ptr(stream)), "pf_adjoint")


def pf_adjoint_rhs(h, B, gVm, gVa, v_stride, bus_type, type_stride, rhs, rhs_stride,
                   stream=None):
    check(lib.pf_adjoint_rhs(h, B, ptr(gVm), ptr(gVa), v_stride, ptr(bus_type), type_stride,
                             ptr(rhs), rhs_stride, stream_ptr(stream)), "pf_adjoint_rhs")


def pf_multi_create(handles):
    arr = (C.c_void_p * max(len(handles), 1))(*[h.value for h in handles])
    p = C.c_void_p()
    check(lib.pf_multi_create(len(handles), arr, C.byref(p)), "pf_multi_create")
    return p


def pf_multi_info(p, G):
    nb = C.c_size_t()
    offs = {k: np.zeros(G + 1, np.int64) for k in ("bus", "branch", "y", "ws")}
    check(lib.pf_multi_info(p, C.byref(nb), ptr(offs["bus"]), ptr(offs["branch"]),
                            ptr(offs["y"]), ptr(offs["ws"])), "pf_multi_info")
    return nb.value, offs


def pf_multi_upload(p, buf, stream=None):
    check(lib.pf_multi_upload(p, ptr(buf), buf.numel() * buf.element_size(),
                              stream_ptr(stream)), "pf_multi_upload")


def pf_multi_set_spread(p, workgroups):
    check(lib.pf_multi_set_spread(p, int(workgroups)), "pf_multi_set_spread")


def pf_build_ybus_multi(p, r, x, b, yval, ysh=None, stream=None):
    check(lib.pf_build_ybus_multi(p, ptr(r), ptr(x), ptr(b), ptr(ysh), ptr(yval),
                                  stream_ptr(stream)), "pf_build_ybus_multi")


def pf_newton_multi(p, yval, bus_type, Psp, Qsp, Vm, Va, tol, max_iter, flags, ws, iters=None,
                    norm=None, status=None, pivot=None, stream=None):
    check(lib.pf_newton_multi(p, ptr(yval), ptr(bus_type), ptr(Psp), ptr(Qsp), ptr(Vm),
                              ptr(Va), float(tol), int(max_iter), int(flags), ptr(ws),
                              ptr(iters), ptr(norm), ptr(status), ptr(pivot),
                              stream_ptr(stream)), "pf_newton_multi")


def pf_multi_destroy(p):
    lib.pf_multi_destroy(p)


def pf_fdpf_matrices(h, B, r, x, b, branch_stride, bus_type, type_stride, mat, mat_stride,
                     ysh=None, ysh_stride=0, stream=None):
    check(lib.pf_fdpf_matrices(h, B, ptr(r), ptr(x), ptr(b), branch_stride, ptr(ysh),
                               ysh_stride, ptr(bus_type), type_stride, ptr(mat), mat_stride,
                               stream_ptr(stream)), "pf_fdpf_matrices")


def pf_fdpf_factor(h, B, mat, mat_stride, status=None, stream=None):
    check(lib.pf_fdpf_factor(h, B, ptr(mat), mat_stride, ptr(status), stream_ptr(stream)),
          "pf_fdpf_factor")


def pf_fdpf(h, B, yval, y_stride, bus_type, type_stride, Psp, Qsp, inj_stride, Vm, Va,
            v_stride, mat, mat_stride, tol, max_iter, ws, ws_stride, iters=None, norm=None,
            status=None, stream=None):
    check(lib.pf_fdpf(h, B, ptr(yval), y_stride, ptr(bus_type), type_stride, ptr(Psp), ptr(Qsp),
                      inj_stride, ptr(Vm), ptr(Va), v_stride, ptr(mat), mat_stride, tol,
                      max_iter, ptr(ws), ws_stride, ptr(iters), ptr(norm), ptr(status),
                      stream_ptr(stream)), "pf_fdpf")


def pf_branch_flows(h, B, r, x, b, branch_stride, Vm, Va, v_stride, Pft, Qft, Ptf, Qtf,
                    out_stride, stream=None):
    check(lib.pf_branch_flows(h, B, ptr(r), ptr(x), ptr(b), branch_stride, ptr(Vm), ptr(Va),
                              v_stride, ptr(Pft), ptr(Qft), ptr(Ptf), ptr(Qtf), out_stride,
                              stream_ptr(stream)), "pf_branch_flows")


PF_MEAS_VM, PF_MEAS_P, PF_MEAS_Q, PF_MEAS_PF, PF_MEAS_QF = 1, 2, 3, 4, 5


def pf_se_analyze(n, from_, to, slack, kind, loc):
    """Host arrays in; returns a pf_se handle (release with pf_se_destroy)."""
    import numpy as _np

    f = _np.ascontiguousarray(from_, _np.int32)
    t = _np.ascontiguousarray(to, _np.int32)
    k = _np.ascontiguousarray(kind, _np.int8)
    l = _np.ascontiguousarray(loc, _np.int32)
    h = _vp()
    check(lib.pf_se_analyze(n, len(f), f.ctypes.data, t.ctypes.data, slack, len(k), k.ctypes.data,
                            l.ctypes.data, C.byref(h)), "pf_se_analyze")
    return h


def pf_se_info(h):
    d = pf_se_dims()
    check(lib.pf_se_info(h, C.byref(d)), "pf_se_info")
    return d


def pf_se_set_launch(h, threads, tail_lds_budget):
    check(lib.pf_se_set_launch(h, int(threads), int(tail_lds_budget)), "pf_se_set_launch")


def pf_se_upload(h, buf, nbytes, stream=None):
    check(lib.pf_se_upload(h, ptr(buf), nbytes, stream_ptr(stream)), "pf_se_upload")


def pf_se_estimate(h, B, r, x, b, branch_stride, z, z_stride, w, w_stride, Vm, Va, v_stride,
                   tol, max_iter, ws, ws_size, iters, norm, status, ysh=None, ysh_stride=0,
                   stream=None):
    check(lib.pf_se_estimate(h, B, ptr(r), ptr(x), ptr(b), branch_stride, ptr(ysh), ysh_stride,
                             ptr(z), z_stride,
                             ptr(w), w_stride, ptr(Vm), ptr(Va), v_stride, tol, max_iter,
                             ptr(ws), ws_size, ptr(iters), ptr(norm), ptr(status),
                             stream_ptr(stream)),
          "pf_se_estimate")


def pf_se_destroy(h):
    lib.pf_se_destroy(h)
