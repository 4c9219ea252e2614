"""Python front end of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads ``liboracle.so`` (built from ``pf_oracle.c``
with gcc; see :func:`build`) and shares no code with the GPU library.

Every function mirrors one C routine in ``pf_oracle.c``; the C file's comments
cite the passages of the paper each step follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
# PF_LIBORACLE selects a prebuilt library instead (the sanitizer check)
_LIB_OVERRIDE = os.environ.get("PF_LIBORACLE")
_LIB = _LIB_OVERRIDE or os.path.join(_HERE, "liboracle.so")

PQ, PV, SLACK = 1, 2, 3
STATUS = {0: "ok", 5: "zero_pivot", 6: "not_converged", 7: "nonfinite"}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C99, -O2)."""
    if _LIB_OVERRIDE:
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        f64n = C.POINTER(C.c_double)  # nullable
        L.or_ybus.argtypes = [C.c_int, C.c_int, i32p, i32p, f64p, f64p, f64p, f64n, f64n, i32p,
                              i32p, f64p, f64p]
        L.or_ybus.restype = C.c_int
        L.or_injections.argtypes = [C.c_int, i32p, i32p, f64p, f64p, f64p, f64p, f64p, f64p]
        L.or_injections.restype = None
        L.or_mismatch.argtypes = [C.c_int, i8p, f64p, f64p, f64p, f64p, f64p, f64p]
        L.or_mismatch.restype = C.c_double
        L.or_dense_solve.argtypes = [C.c_int, f64p, f64p]
        L.or_dense_solve.restype = C.c_int
        L.or_dense_jacobian.argtypes = [C.c_int, i32p, i32p, f64p, f64p, i8p, f64p, f64p,
                                        f64p, f64p, f64p]
        L.or_dense_jacobian.restype = C.c_int
        L.or_newton_dense.argtypes = [C.c_int, i32p, i32p, f64p, f64p, i8p, f64p, f64p, f64p,
                                      f64p, C.c_double, C.c_int, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_double)]
        L.or_newton_dense.restype = C.c_int
        L.or_analyze.argtypes = [C.c_int, C.c_int, i32p, i32p, C.c_int, C.c_int]
        L.or_analyze.restype = C.c_void_p
        L.or_sym_free.argtypes = [C.c_void_p]
        L.or_sym_free.restype = None
        L.or_sym_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int32)]
        L.or_sym_sizes.restype = None
        L.or_sym_export.argtypes = [C.c_void_p, i32p, i32p, i32p, i32p, i32p, i32p, i32p]
        L.or_sym_export.restype = None
        L.or_block_jacobian.argtypes = [C.c_void_p, i32p, i32p, f64p, f64p, i8p, f64p, f64p,
                                        f64p, f64p, f64p, f64p, f64p]
        L.or_block_jacobian.restype = None
        L.or_factor.argtypes = [C.c_void_p, f64p, f64p, f64p]
        L.or_factor.restype = C.c_int
        L.or_solve.argtypes = [C.c_void_p, f64p, f64p, f64p, f64p]
        L.or_solve.restype = C.c_int
        L.or_newton_sparse.argtypes = [C.c_void_p, i32p, i32p, f64p, f64p, i8p, f64p, f64p,
                                       f64p, f64p, C.c_double, C.c_int,
                                       C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32)]
        L.or_newton_sparse.restype = C.c_int
        L.or_adjoint_dense.argtypes = [C.c_int, C.c_int, i32p, i32p, f64p, f64p, i32p, i32p,
                                       f64p, f64p, i8p, f64p, f64p, f64p, f64p, f64p, f64p,
                                       f64p]
        L.or_adjoint_dense.restype = C.c_int
        L.or_solve_transpose.argtypes = [C.c_void_p, f64p, f64p, f64p, f64p]
        L.or_solve_transpose.restype = C.c_int
        L.or_adjoint_sparse.argtypes = [C.c_void_p, C.c_int, i32p, i32p, f64p, f64p, i32p, i32p,
                                        f64p, f64p, i8p, f64p, f64p, f64p, f64p, f64p, f64p,
                                        f64p]
        L.or_adjoint_sparse.restype = C.c_int
        L.or_fdpf_matrices.argtypes = [C.c_void_p, C.c_int, i32p, i32p, f64p, f64p, f64p, f64n,
                                       i8p, f64p, f64p, f64p, f64p]
        L.or_fdpf_matrices.restype = None
        L.or_factor1.argtypes = [C.c_void_p, f64p, f64p, f64p]
        L.or_factor1.restype = C.c_int
        L.or_solve1.argtypes = [C.c_void_p, f64p, f64p, f64p, f64p]
        L.or_solve1.restype = None
        L.or_fdpf.argtypes = [C.c_void_p, i32p, i32p, f64p, f64p, i8p, f64p, f64p, f64p, f64p,
                              f64p, f64p, f64p, f64p, f64p, f64p, C.c_double, C.c_int,
                              C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.or_fdpf.restype = C.c_int
        L.or_branch_flows.argtypes = [C.c_int, i32p, i32p, f64p, f64p, f64p, f64p, f64p, f64p,
                                      f64p, f64p, f64p]
        L.or_branch_flows.restype = None
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Ybus:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    G: np.ndarray
    B: np.ndarray

    def dense(self) -> np.ndarray:
        Y = np.zeros((self.n, self.n), complex)
        for i in range(self.n):
            for k in range(self.rowptr[i], self.rowptr[i + 1]):
                Y[i, self.col[k]] = self.G[k] + 1j * self.B[k]
        return Y


def _nullable(a):
    """A C double pointer to a contiguous fp64 array, or NULL for None (the
    array must outlive the call: callers keep it in a local)."""
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def ybus(n, f, t, r, x, b, gsh=None, bsh=None) -> Ybus:
    """Admittance matrix with optional bus shunts gsh + j bsh (float64[n])."""
    m = len(f)
    rowptr = np.zeros(n + 1, np.int32)
    col = np.zeros(n + 4 * m + 1, np.int32)
    G = np.zeros(n + 4 * m + 1)
    B = np.zeros(n + 4 * m + 1)
    gs = None if gsh is None else _f64(gsh)
    bs = None if bsh is None else _f64(bsh)
    nnz = lib().or_ybus(n, m, _i32(f), _i32(t), _f64(r), _f64(x), _f64(b), _nullable(gs),
                        _nullable(bs), rowptr, col, G, B)
    if nnz < 0:
        raise ValueError("invalid branch list")
    return Ybus(n, rowptr, col[:nnz].copy(), G[:nnz].copy(), B[:nnz].copy())


def grid_ybus(grid) -> Ybus:
    return ybus(grid.n, grid.f, grid.t, grid.r, grid.x, grid.b, grid.gsh, grid.bsh)


def injections(Y: Ybus, Vm, Va):
    P = np.zeros(Y.n)
    Q = np.zeros(Y.n)
    lib().or_injections(Y.n, Y.rowptr, Y.col, Y.G, Y.B, _f64(Vm), _f64(Va), P, Q)
    return P, Q


def mismatch(bus_type, P, Q, Psp, Qsp):
    n = len(P)
    FP = np.zeros(n)
    FQ = np.zeros(n)
    nrm = lib().or_mismatch(n, np.ascontiguousarray(bus_type, np.int8), _f64(P), _f64(Q),
                            _f64(Psp), _f64(Qsp), FP, FQ)
    return FP, FQ, nrm


def dense_solve(A, rhs):
    A = np.array(A, np.float64, order="C")
    x = np.array(rhs, np.float64)
    if lib().or_dense_solve(A.shape[0], A, x) != 0:
        raise np.linalg.LinAlgError("singular")
    return x


def dense_jacobian(Y: Ybus, bus_type, Vm, Va):
    P, Q = injections(Y, Vm, Va)
    bt = np.ascontiguousarray(bus_type, np.int8)
    N = int(np.sum(bt != SLACK) + np.sum(bt == PQ))
    J = np.zeros(N * N + 1)
    lib().or_dense_jacobian(Y.n, Y.rowptr, Y.col, Y.G, Y.B, bt, _f64(Vm), _f64(Va), P, Q, J)
    return J[: N * N].reshape(N, N)


@dataclass
class NRResult:
    Vm: np.ndarray
    Va: np.ndarray
    iters: int
    norm: float
    status: int
    bad_node: int = -1


def newton_dense(Y: Ybus, bus_type, Psp, Qsp, Vm0, Va0, tol=1e-8, max_iter=20) -> NRResult:
    Vm = _f64(Vm0).copy()
    Va = _f64(Va0).copy()
    it = C.c_int32()
    nrm = C.c_double()
    st = lib().or_newton_dense(Y.n, Y.rowptr, Y.col, Y.G, Y.B,
                               np.ascontiguousarray(bus_type, np.int8), _f64(Psp), _f64(Qsp),
                               Vm, Va, tol, max_iter, C.byref(it), C.byref(nrm))
    return NRResult(Vm, Va, it.value, nrm.value, st)


class Sym:
    """Oracle symbolic analysis (owns the C object)."""

    def __init__(self, n, f, t, slack=0, ordering=0):
        h = lib().or_analyze(n, len(f), _i32(f), _i32(t), slack, ordering)
        if not h:
            raise ValueError("invalid grid")
        self._h = C.c_void_p(h)
        nn = C.c_int32()
        nnz = C.c_int64()
        nlev = C.c_int32()
        lib().or_sym_sizes(self._h, C.byref(nn), C.byref(nnz), C.byref(nlev))
        self.n, self.nn, self.nnzL, self.nlev = n, nn.value, nnz.value, nlev.value
        self.perm = np.zeros(max(self.nn, 1), np.int32)
        self.parent = np.zeros(max(self.nn, 1), np.int32)
        self.level = np.zeros(max(self.nn, 1), np.int32)
        self.level_ptr = np.zeros(self.nlev + 1, np.int32)
        self.level_nodes = np.zeros(max(self.nn, 1), np.int32)
        self.Lp = np.zeros(self.nn + 1, np.int32)
        self.Li = np.zeros(max(self.nnzL, 1), np.int32)
        lib().or_sym_export(self._h, self.perm, self.parent, self.level, self.level_ptr,
                            self.level_nodes, self.Lp, self.Li)
        for name in ("perm", "parent", "level", "level_nodes"):
            setattr(self, name, getattr(self, name)[: self.nn])
        self.Li = self.Li[: self.nnzL]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.or_sym_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def block_jacobian(self, Y: Ybus, bus_type, Vm, Va):
        P, Q = injections(Y, Vm, Va)
        D = np.zeros(4 * max(self.nn, 1))
        Lb = np.zeros(4 * max(self.nnzL, 1))
        Ub = np.zeros(4 * max(self.nnzL, 1))
        lib().or_block_jacobian(self._h, Y.rowptr, Y.col, Y.G, Y.B,
                                np.ascontiguousarray(bus_type, np.int8), _f64(Vm), _f64(Va),
                                P, Q, D, Lb, Ub)
        return (D[: 4 * self.nn].reshape(-1, 2, 2), Lb[: 4 * self.nnzL].reshape(-1, 2, 2),
                Ub[: 4 * self.nnzL].reshape(-1, 2, 2))

    def factor(self, D, Lb, Ub):
        """In-place right-looking LDU; returns (D, L, U) copies and the bad node."""
        D = np.array(D, np.float64).reshape(-1).copy()
        Lb = np.array(Lb, np.float64).reshape(-1).copy()
        Ub = np.array(Ub, np.float64).reshape(-1).copy()
        if Lb.size == 0:
            Lb = np.zeros(4)
            Ub = np.zeros(4)
        bad = lib().or_factor(self._h, D, Lb, Ub)
        return (D.reshape(-1, 2, 2), Lb[: 4 * self.nnzL].reshape(-1, 2, 2),
                Ub[: 4 * self.nnzL].reshape(-1, 2, 2), bad)

    def solve(self, D, L, U, rhs):
        D = _f64(D).reshape(-1)
        L = _f64(L).reshape(-1)
        U = _f64(U).reshape(-1)
        if L.size == 0:
            L = np.zeros(4)
            U = np.zeros(4)
        x = np.array(rhs, np.float64).reshape(-1).copy()
        if lib().or_solve(self._h, D, L, U, x) != 0:
            raise np.linalg.LinAlgError("singular pivot")
        return x.reshape(-1, 2)

    def solve_transpose(self, D, L, U, rhs):
        D = _f64(D).reshape(-1)
        L = _f64(L).reshape(-1)
        U = _f64(U).reshape(-1)
        if L.size == 0:
            L = np.zeros(4)
            U = np.zeros(4)
        x = np.array(rhs, np.float64).reshape(-1).copy()
        if lib().or_solve_transpose(self._h, D, L, U, x) != 0:
            raise np.linalg.LinAlgError("singular pivot")
        return x.reshape(-1, 2)

    def adjoint(self, grid, Y: Ybus, Vm, Va, gVm, gVa, x=None):
        """Sparse adjoint at a converged state: returns (gP, gQ, gx)."""
        n, m = grid.n, grid.m
        xx = grid.x if x is None else x
        gP = np.zeros(n)
        gQ = np.zeros(n)
        gx = np.zeros(max(m, 1))
        st = lib().or_adjoint_sparse(self._h, m, _i32(grid.f), _i32(grid.t), _f64(grid.r),
                                     _f64(xx), Y.rowptr, Y.col, Y.G, Y.B,
                                     np.ascontiguousarray(grid.bus_type, np.int8), _f64(Vm),
                                     _f64(Va), _f64(gVm), _f64(gVa), gP, gQ, gx)
        if st != 0:
            raise np.linalg.LinAlgError("zero pivot")
        return gP, gQ, gx[:m]

    def newton(self, Y: Ybus, bus_type, Psp, Qsp, Vm0, Va0, tol=1e-8, max_iter=20) -> NRResult:
        Vm = _f64(Vm0).copy()
        Va = _f64(Va0).copy()
        it = C.c_int32()
        nrm = C.c_double()
        bad = C.c_int32()
        st = lib().or_newton_sparse(self._h, Y.rowptr, Y.col, Y.G, Y.B,
                                    np.ascontiguousarray(bus_type, np.int8), _f64(Psp),
                                    _f64(Qsp), Vm, Va, tol, max_iter, C.byref(it),
                                    C.byref(nrm), C.byref(bad))
        return NRResult(Vm, Va, it.value, nrm.value, st, bad.value)

    # -- fast decoupled power flow (scalar elements) --------------------------
    def fdpf_matrices(self, grid, r=None, x=None, b=None):
        """XB matrices in the scalar filled layout: (d1, a1, d2, a2), d per
        position, a per slot (entry (p, Li[q]) = entry (Li[q], p))."""
        nn, nz = self.nn, max(self.nnzL, 1)
        d1, d2 = np.zeros(max(nn, 1)), np.zeros(max(nn, 1))
        a1, a2 = np.zeros(nz), np.zeros(nz)
        bs = _f64(grid.bsh)
        lib().or_fdpf_matrices(self._h, grid.m, _i32(grid.f), _i32(grid.t),
                               _f64(grid.r if r is None else r), _f64(grid.x if x is None else x),
                               _f64(grid.b if b is None else b), _nullable(bs),
                               np.ascontiguousarray(grid.bus_type, np.int8), d1, a1, d2, a2)
        return d1[:nn], a1[: self.nnzL], d2[:nn], a2[: self.nnzL]

    def factor1(self, d, a_lo, a_up=None):
        """Scalar FactorizeGraphA on a full copy: returns (d, L, U, bad)."""
        d = np.array(d, np.float64).copy()
        lo = np.array(a_lo, np.float64).copy()
        up = np.array(a_lo if a_up is None else a_up, np.float64).copy()
        if lo.size == 0:
            lo, up = np.zeros(1), np.zeros(1)
        bad = lib().or_factor1(self._h, d, lo, up)
        return d, lo[: self.nnzL], up[: self.nnzL], bad

    def solve1(self, d, L, U, rhs):
        L = _f64(L) if len(L) else np.zeros(1)
        U = _f64(U) if len(U) else np.zeros(1)
        x = np.array(rhs, np.float64).copy()
        lib().or_solve1(self._h, _f64(d), L, U, x)
        return x

    def fdpf(self, Y: Ybus, grid, Psp, Qsp, Vm0, Va0, tol=1e-8, max_iter=40,
             factors=None) -> NRResult:
        """Fast decoupled iteration (XB) from (Vm0, Va0); factors may be given
        as ((d1, L1, U1), (d2, L2, U2))."""
        if factors is None:
            d1, a1, d2, a2 = self.fdpf_matrices(grid)
            f1 = self.factor1(d1, a1)
            f2 = self.factor1(d2, a2)
            if f1[3] >= 0 or f2[3] >= 0:
                raise np.linalg.LinAlgError("zero pivot in B' or B''")
            factors = (f1[:3], f2[:3])
        (d1, L1, U1), (d2, L2, U2) = factors
        pad = (lambda a: _f64(a) if len(a) else np.zeros(1))
        Vm = _f64(Vm0).copy()
        Va = _f64(Va0).copy()
        it = C.c_int32()
        nrm = C.c_double()
        st = lib().or_fdpf(self._h, Y.rowptr, Y.col, Y.G, Y.B,
                           np.ascontiguousarray(grid.bus_type, np.int8), _f64(Psp), _f64(Qsp),
                           _f64(d1), pad(L1), pad(U1), _f64(d2), pad(L2), pad(U2), Vm, Va, tol,
                           max_iter, C.byref(it), C.byref(nrm))
        return NRResult(Vm, Va, it.value, nrm.value, st)

    def scalar_matrix(self, d, a):
        """Dense symmetric matrix (position order) from scalar filled values."""
        A = np.diag(np.asarray(d, np.float64))
        for p in range(self.nn):
            for q in range(self.Lp[p], self.Lp[p + 1]):
                A[p, self.Li[q]] = A[self.Li[q], p] = a[q]
        return A

    def dense_matrix(self, D, Lb, Ub):
        """Assemble the permuted block matrix from filled-layout blocks."""
        nn = self.nn
        A = np.zeros((2 * nn, 2 * nn))
        for p in range(nn):
            A[2 * p:2 * p + 2, 2 * p:2 * p + 2] = D[p]
            for q in range(self.Lp[p], self.Lp[p + 1]):
                k = self.Li[q]
                A[2 * k:2 * k + 2, 2 * p:2 * p + 2] = Lb[q]
                A[2 * p:2 * p + 2, 2 * k:2 * k + 2] = Ub[q]
        return A


def adjoint_dense(grid, Y: Ybus, Vm, Va, gVm, gVa, x=None):
    """Dense adjoint at a converged state: returns (gP, gQ, gx)."""
    n, m = grid.n, grid.m
    xx = grid.x if x is None else x
    gP = np.zeros(n)
    gQ = np.zeros(n)
    gx = np.zeros(max(m, 1))
    st = lib().or_adjoint_dense(n, m, _i32(grid.f), _i32(grid.t), _f64(grid.r), _f64(xx),
                                Y.rowptr, Y.col, Y.G, Y.B,
                                np.ascontiguousarray(grid.bus_type, np.int8), _f64(Vm),
                                _f64(Va), _f64(gVm), _f64(gVa), gP, gQ, gx)
    if st != 0:
        raise np.linalg.LinAlgError("singular Jacobian")
    return gP, gQ, gx[:m]


def solve_grid(grid, sparse=True, tol=1e-8, max_iter=20, Psp=None, Qsp=None, ordering=0,
               sym=None):
    """Convenience: flat start NR on a gridgen.Grid."""
    Y = grid_ybus(grid)
    Vm0, Va0 = grid.flat_start()
    Psp = grid.Psp if Psp is None else Psp
    Qsp = grid.Qsp if Qsp is None else Qsp
    if sparse:
        s = sym if sym is not None else Sym(grid.n, grid.f, grid.t, 0, ordering)
        return s.newton(Y, grid.bus_type, Psp, Qsp, Vm0, Va0, tol, max_iter)
    return newton_dense(Y, grid.bus_type, Psp, Qsp, Vm0, Va0, tol, max_iter)


def branch_flows(grid, Vm, Va, r=None, x=None, b=None):
    """Complex power at both ends of every branch: (Pft, Qft, Ptf, Qtf)."""
    m = grid.m
    out = [np.zeros(max(m, 1)) for _ in range(4)]
    lib().or_branch_flows(m, _i32(grid.f), _i32(grid.t), _f64(grid.r if r is None else r),
                          _f64(grid.x if x is None else x), _f64(grid.b if b is None else b),
                          _f64(Vm), _f64(Va), *out)
    return tuple(o[:m] for o in out)


def solve_grid_fdpf(grid, tol=1e-8, max_iter=40, Psp=None, Qsp=None, sym=None):
    """Convenience: flat-start fast decoupled power flow on a gridgen.Grid."""
    Y = grid_ybus(grid)
    Vm0, Va0 = grid.flat_start()
    s = sym if sym is not None else Sym(grid.n, grid.f, grid.t)
    return s.fdpf(Y, grid, grid.Psp if Psp is None else Psp, grid.Qsp if Qsp is None else Qsp,
                  Vm0, Va0, tol, max_iter)
