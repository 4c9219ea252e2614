"""Pins for the CPU oracle: each check ties it to something other than itself
(closed forms, conservation laws, finite differences, brute force, LAPACK,
the paper's Table I)."""
import numpy as np
import pytest

import gridgen

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# --------------------------------------------------------------------------
# helpers written independently of the oracle
# --------------------------------------------------------------------------
def two_bus(r=0.02, x=0.08, b=0.04, P=0.9, Q=0.3, E=1.0, pv=False, vs=1.0):
    """Slack bus 0 and bus 1 joined by one branch (pi-model, total charging b)."""
    bt = np.array([gridgen.BUS_SLACK, gridgen.BUS_PV if pv else gridgen.BUS_PQ], np.int8)
    vset = np.array([E, vs if pv else 1.0])
    g = gridgen.Grid(n=2, f=np.array([0], np.int32), t=np.array([1], np.int32),
                     r=np.array([r]), x=np.array([x]), b=np.array([b]), bus_type=bt,
                     vset=vset, Pd=np.array([0.0, P]), Qd=np.array([0.0, Q]),
                     Pg=np.zeros(2), pts=np.zeros((2, 2)))
    return g


def closed_form_pq(r, x, b, P, Q, E=1.0):
    """Load P+jQ at bus 1 behind z = r+jx with charging beta = b/2 at bus 1.

    From V0 conj(V1) = v + z (P - j Q'), Q' = Q - beta v, v = |V1|^2:
      (1 - 2 x beta + |z|^2 beta^2) v^2 + (2rP + 2xQ - E^2 - 2|z|^2 Q beta) v
        + |z|^2 (P^2 + Q^2) = 0, larger root; theta1 = -atan2(xP - rQ', v + rP + xQ').
    """
    beta = b / 2.0
    z2 = r * r + x * x
    a2 = 1 - 2 * x * beta + z2 * beta * beta
    a1 = 2 * r * P + 2 * x * Q - E * E - 2 * z2 * Q * beta
    a0 = z2 * (P * P + Q * Q)
    v = (-a1 + np.sqrt(a1 * a1 - 4 * a2 * a0)) / (2 * a2)
    Qp = Q - beta * v
    th = -np.arctan2(x * P - r * Qp, v + r * P + x * Qp)
    return np.sqrt(v), th


def closed_form_pv(r, x, Pinj, vs, E=1.0):
    """PV bus 1 (|V1| = vs) injecting Pinj into the branch to the slack:
    Re(V1 conj(V1 - V0) / conj(z)) = Pinj gives r cos t - x sin t = c,
    c = (vs^2 r - Pinj |z|^2) / (vs E); small-angle root."""
    R = np.hypot(r, x)
    phi = np.arctan2(x, r)
    c = (vs * vs * r - Pinj * R * R) / (vs * E)
    return np.arccos(c / R) - phi


def branch_currents(grid, Vm, Va):
    V = Vm * np.exp(1j * Va)
    z = grid.r + 1j * grid.x
    return V, (V[grid.f] - V[grid.t]) / z


def kcl_currents(grid, V):
    """Bus current injections summed element by element: each bus's own shunt
    (g_sh + j b_sh) V_i, then every branch's series current and half charging."""
    I = (grid.gsh + 1j * grid.bsh) * V
    z = grid.r + 1j * grid.x
    for e in range(grid.m):
        a, b = grid.f[e], grid.t[e]
        Is = (V[a] - V[b]) / z[e]
        I[a] += Is + 1j * grid.b[e] / 2 * V[a]
        I[b] += -Is + 1j * grid.b[e] / 2 * V[b]
    return I


def shunted(n, seed, shunt_seed=None):
    """A generated grid, with seeded bus shunts when shunt_seed is given."""
    g = gridgen.make_grid(n, seed)
    return g if shunt_seed is None else gridgen.with_shunts(g, shunt_seed)


def random_state(grid, rng, spread=0.3):
    Vm = rng.uniform(0.9, 1.1, grid.n)
    Va = rng.uniform(-spread, spread, grid.n)
    return Vm, Va


def reduced_residual(O, Y, grid, Vm, Va, Psp, Qsp):
    """Residual vector over P(non-slack), Q(PQ) in ascending bus order."""
    P, Q = O.injections(Y, Vm, Va)
    FP, FQ, _ = O.mismatch(grid.bus_type, P, Q, Psp, Qsp)
    ns = grid.bus_type != gridgen.BUS_SLACK
    pq = grid.bus_type == gridgen.BUS_PQ
    return np.concatenate([FP[ns], FQ[pq]])


# --------------------------------------------------------------------------
# admittance matrix and injections
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shunt_seed", [None, 31])
def test_ybus_matches_branchwise_kcl(oracle, shunt_seed):
    g = shunted(60, 11, shunt_seed)
    if shunt_seed is not None:  # a shunt at the slack too
        g.gsh[0], g.bsh[0] = 0.003, -0.02
        assert np.count_nonzero(g.bsh) > 10
    Y = oracle.grid_ybus(g)
    rng = np.random.default_rng(0)
    Vm, Va = random_state(g, rng)
    V = Vm * np.exp(1j * Va)
    np.testing.assert_allclose(Y.dense() @ V, kcl_currents(g, V), rtol=0, atol=1e-11)


def test_ybus_parallel_branches_sum(oracle):
    f = np.array([0, 0, 1], np.int32)
    t = np.array([1, 1, 2], np.int32)
    r = np.array([0.01, 0.03, 0.02])
    x = np.array([0.1, 0.2, 0.05])
    b = np.array([0.02, 0.0, 0.01])
    Y = oracle.ybus(3, f, t, r, x, b).dense()
    y = 1 / (r + 1j * x)
    assert Y[0, 1] == pytest.approx(-(y[0] + y[1]))
    assert Y[1, 1] == pytest.approx(y[0] + y[1] + y[2] + 1j * (0.01 + 0.005))
    assert Y[0, 2] == 0


def test_ybus_rejects_self_loop(oracle):
    with pytest.raises(ValueError):
        oracle.ybus(2, np.array([1], np.int32), np.array([1], np.int32), np.ones(1),
                    np.ones(1), np.zeros(1))


@pytest.mark.parametrize("seed,shunt_seed", [(3, None), (4, None), (3, 41), (6, 42)])
def test_power_balance_tellegen(oracle, seed, shunt_seed):
    """At any voltages: sum P_i = sum r|I|^2 + sum g_sh |V_i|^2 and
    sum Q_i = sum x|I|^2 - sum b/2 (|V_f|^2 + |V_t|^2) - sum b_sh |V_i|^2."""
    g = shunted(80, seed, shunt_seed)
    Y = oracle.grid_ybus(g)
    rng = np.random.default_rng(seed)
    Vm, Va = random_state(g, rng)
    P, Q = oracle.injections(Y, Vm, Va)
    V, I = branch_currents(g, Vm, Va)
    loss_p = np.sum(g.r * np.abs(I) ** 2) + np.sum(g.gsh * Vm ** 2)
    loss_q = (np.sum(g.x * np.abs(I) ** 2) - np.sum(g.b / 2 * (np.abs(V[g.f]) ** 2 +
                                                              np.abs(V[g.t]) ** 2))
              - np.sum(g.bsh * Vm ** 2))
    assert np.sum(P) == pytest.approx(loss_p, rel=1e-11, abs=1e-11)
    assert np.sum(Q) == pytest.approx(loss_q, rel=1e-11, abs=1e-11)
    assert loss_p > 0


def test_lossless_injections_sum_to_zero(oracle):
    g = gridgen.make_grid(50, seed=5)
    Y = oracle.ybus(g.n, g.f, g.t, np.zeros(g.m), g.x, g.b)
    Vm, Va = random_state(g, np.random.default_rng(1))
    P, _ = oracle.injections(Y, Vm, Va)
    assert abs(np.sum(P)) < 1e-11


@pytest.mark.parametrize("shunt_seed", [None, 43])
def test_injection_single_bus_formula(oracle, shunt_seed):
    """S_i = V_i conj(I_i) with I from element-wise KCL."""
    g = shunted(40, 9, shunt_seed)
    Y = oracle.grid_ybus(g)
    Vm, Va = random_state(g, np.random.default_rng(2))
    P, Q = oracle.injections(Y, Vm, Va)
    V = Vm * np.exp(1j * Va)
    S = V * np.conj(kcl_currents(g, V))
    np.testing.assert_allclose(P, S.real, atol=1e-11)
    np.testing.assert_allclose(Q, S.imag, atol=1e-11)


def test_mismatch_norm_excludes_slack_and_pv_q(oracle):
    bt = np.array([3, 2, 1], np.int8)
    P = np.array([5.0, 1.0, 2.0])
    Q = np.array([7.0, 9.0, 3.0])
    FP, FQ, nrm = oracle.mismatch(bt, P, Q, np.zeros(3), np.zeros(3))
    assert FP.tolist() == [0.0, 1.0, 2.0]
    assert FQ.tolist() == [0.0, 0.0, 3.0]
    assert nrm == 3.0
    _, _, nrm = oracle.mismatch(bt, np.array([0, np.nan, 0.0]), Q, np.zeros(3), np.zeros(3))
    assert np.isnan(nrm)


# --------------------------------------------------------------------------
# Newton-Raphson: closed forms and agreement of the two formulations
# --------------------------------------------------------------------------
@pytest.mark.parametrize("sparse", [False, True])
@pytest.mark.parametrize("case", [(0.02, 0.08, 0.04, 0.9, 0.3), (0.01, 0.12, 0.0, 1.5, 0.4),
                                  (0.05, 0.05, 0.1, 0.3, -0.2)])
def test_two_bus_pq_closed_form(oracle, case, sparse):
    r, x, b, P, Q = case
    g = two_bus(r, x, b, P, Q)
    res = oracle.solve_grid(g, sparse=sparse, tol=1e-13, max_iter=30)
    assert res.status == 0
    vm, th = closed_form_pq(r, x, b, P, Q)
    assert res.Vm[1] == pytest.approx(vm, abs=1e-12)
    assert res.Va[1] == pytest.approx(th, abs=1e-12)


@pytest.mark.parametrize("sparse", [False, True])
@pytest.mark.parametrize("bsh", [0.07, -0.03])
def test_two_bus_shunt_closed_form(oracle, sparse, bsh):
    """A shunt susceptance b_sh at the load bus acts as extra charging there:
    the closed form with beta = b/2 + b_sh (a capacitor bank or a reactor)."""
    r, x, b, P, Q = 0.02, 0.08, 0.04, 0.9, 0.3
    g = two_bus(r, x, b, P, Q)
    g.bsh[1] = bsh
    res = oracle.solve_grid(g, sparse=sparse, tol=1e-13, max_iter=30)
    assert res.status == 0
    vm, th = closed_form_pq(r, x, b + 2 * bsh, P, Q)
    assert res.Vm[1] == pytest.approx(vm, abs=1e-12)
    assert res.Va[1] == pytest.approx(th, abs=1e-12)
    # and the shunt really moved the solution
    assert abs(vm - closed_form_pq(r, x, b, P, Q)[0]) > 1e-3


@pytest.mark.parametrize("sparse", [False, True])
def test_two_bus_pv_closed_form(oracle, sparse):
    r, x, vs, Pinj = 0.02, 0.1, 1.03, 0.8
    g = two_bus(r, x, 0.03, 0.0, 0.0, pv=True, vs=vs)
    g.Pg[1] = Pinj
    res = oracle.solve_grid(g, sparse=sparse, tol=1e-13, max_iter=30)
    assert res.status == 0
    assert res.Vm[1] == vs
    assert res.Va[1] == pytest.approx(closed_form_pv(r, x, Pinj, vs), abs=1e-12)


@pytest.mark.parametrize("n,seed,shunt_seed", [(30, 1, None), (200, 1, None), (200, 2, None),
                                               (500, 3, None), (300, 4, 44)])
def test_sparse_paper_path_equals_dense_definition(oracle, n, seed, shunt_seed):
    g = shunted(n, seed, shunt_seed)
    d = oracle.solve_grid(g, sparse=False)
    s = oracle.solve_grid(g, sparse=True)
    nat = oracle.solve_grid(g, sparse=True, ordering=1)
    assert d.status == s.status == nat.status == 0
    assert d.iters == s.iters == nat.iters
    for r in (s, nat):
        np.testing.assert_allclose(r.Vm, d.Vm, atol=1e-12)
        np.testing.assert_allclose(r.Va, d.Va, atol=1e-12)


@pytest.mark.parametrize("shunt_seed", [None, 45])
def test_solution_zeroes_independent_residual(oracle, shunt_seed):
    """The converged state satisfies S = V conj(I) = S_sp computed element-wise."""
    g = shunted(300, 7, shunt_seed)
    res = oracle.solve_grid(g)
    assert res.status == 0
    V = res.Vm * np.exp(1j * res.Va)
    S = V * np.conj(kcl_currents(g, V))
    ns = g.bus_type != gridgen.BUS_SLACK
    pq = g.bus_type == gridgen.BUS_PQ
    assert np.max(np.abs(S.real[ns] - g.Psp[ns])) < 1e-8
    assert np.max(np.abs(S.imag[pq] - g.Qsp[pq])) < 1e-8
    pv = g.bus_type == gridgen.BUS_PV
    np.testing.assert_array_equal(res.Vm[pv], g.vset[pv])


def test_quadratic_convergence(oracle):
    g = gridgen.make_grid(200, 4)
    Y = oracle.grid_ybus(g)
    Vm0, Va0 = g.flat_start()
    norms = []
    for k in range(0, 5):
        r = oracle.newton_dense(Y, g.bus_type, g.Psp, g.Qsp, Vm0, Va0, tol=0.0, max_iter=k)
        norms.append(r.norm)
    # e_{k+1} <= C e_k^2 once in the basin
    for a, b in zip(norms[1:-1], norms[2:]):
        if a < 1e-2 and b > 1e-14:
            assert b < 10 * a * a


def test_not_converged_and_nonfinite_status(oracle):
    g = gridgen.make_grid(50, 2)
    r = oracle.solve_grid(g, max_iter=1)
    assert r.status == 6 and r.iters == 1
    bad = gridgen.make_grid(50, 2)
    bad.Pd[5] = np.nan
    assert oracle.solve_grid(bad).status == 7


# --------------------------------------------------------------------------
# Jacobians against finite differences of the mismatch
# --------------------------------------------------------------------------
def test_dense_jacobian_fd(oracle):
    g = gridgen.make_grid(40, 8)
    Y = oracle.grid_ybus(g)
    rng = np.random.default_rng(3)
    Vm, Va = random_state(g, rng)
    Vm[g.bus_type == gridgen.BUS_PV] = g.vset[g.bus_type == gridgen.BUS_PV]
    J = oracle.dense_jacobian(Y, g.bus_type, Vm, Va)
    ns = np.flatnonzero(g.bus_type != gridgen.BUS_SLACK)
    pq = np.flatnonzero(g.bus_type == gridgen.BUS_PQ)
    h = 1e-7
    cols = []
    for i in ns:
        a, b = Va.copy(), Va.copy()
        a[i] += h
        b[i] -= h
        cols.append((reduced_residual(oracle, Y, g, Vm, a, g.Psp, g.Qsp) -
                     reduced_residual(oracle, Y, g, Vm, b, g.Psp, g.Qsp)) / (2 * h))
    for i in pq:
        a, b = Vm.copy(), Vm.copy()
        a[i] += h
        b[i] -= h
        cols.append((reduced_residual(oracle, Y, g, a, Va, g.Psp, g.Qsp) -
                     reduced_residual(oracle, Y, g, b, Va, g.Psp, g.Qsp)) / (2 * h))
    Jfd = np.array(cols).T
    np.testing.assert_allclose(J, Jfd, rtol=1e-6, atol=1e-6 * np.abs(J).max())


def block_fd(oracle, sym, Y, g, Vm, Va):
    """FD Jacobian over all 2 unknowns per non-slack bus, permuted order, with the
    PV reading applied: |V| rows replaced by the identity, |V| columns dropped."""
    nn = sym.nn
    bus_of_pos = sym.perm
    h = 1e-7

    def F(Vm_, Va_):
        P, Q = oracle.injections(Y, Vm_, Va_)
        out = np.zeros(2 * nn)
        for p in range(nn):
            i = bus_of_pos[p]
            out[2 * p] = P[i]
            out[2 * p + 1] = Q[i] if g.bus_type[i] == gridgen.BUS_PQ else Vm_[i]
        return out

    A = np.zeros((2 * nn, 2 * nn))
    for p in range(nn):
        i = bus_of_pos[p]
        for comp in range(2):
            a_m, a_a, b_m, b_a = Vm.copy(), Va.copy(), Vm.copy(), Va.copy()
            if comp == 0:
                a_a[i] += h
                b_a[i] -= h
            else:
                a_m[i] += h
                b_m[i] -= h
            A[:, 2 * p + comp] = (F(a_m, a_a) - F(b_m, b_a)) / (2 * h)
    for p in range(nn):
        if g.bus_type[bus_of_pos[p]] == gridgen.BUS_PV:
            col = A[:, 2 * p + 1].copy()
            A[:, 2 * p + 1] = 0
            A[2 * p + 1, 2 * p + 1] = col[2 * p + 1]
    return A


@pytest.mark.parametrize("shunt_seed", [None, 46])
def test_block_jacobian_fd_and_pattern(oracle, shunt_seed):
    g = shunted(35, 12, shunt_seed)
    Y = oracle.grid_ybus(g)
    sym = oracle.Sym(g.n, g.f, g.t)
    Vm, Va = random_state(g, np.random.default_rng(5))
    pv = g.bus_type == gridgen.BUS_PV
    Vm[pv] = g.vset[pv]
    D, Lb, Ub = sym.block_jacobian(Y, g.bus_type, Vm, Va)
    A = sym.dense_matrix(D, Lb, Ub)
    Afd = block_fd(oracle, sym, Y, g, Vm, Va)
    np.testing.assert_allclose(A, Afd, rtol=1e-6, atol=1e-6 * np.abs(A).max())


# --------------------------------------------------------------------------
# linear algebra: dense GE vs LAPACK, sparse LDU vs dense
# --------------------------------------------------------------------------
def test_dense_solve_matches_lapack(oracle):
    rng = np.random.default_rng(0)
    for N in (1, 5, 40):
        A = rng.standard_normal((N, N)) + N * np.eye(N)
        b = rng.standard_normal(N)
        np.testing.assert_allclose(oracle.dense_solve(A, b), np.linalg.solve(A, b),
                                   rtol=1e-12, atol=1e-12)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.dense_solve(np.zeros((3, 3)), np.ones(3))


def test_dense_solve_needs_pivoting(oracle):
    A = np.array([[0.0, 1.0], [1.0, 1.0]])
    np.testing.assert_allclose(oracle.dense_solve(A, [2.0, 3.0]), [1.0, 2.0])


@pytest.mark.parametrize("n,seed,ordering", [(30, 1, 0), (120, 2, 0), (120, 2, 1), (400, 5, 0)])
def test_sparse_ldu_reconstructs_and_solves(oracle, n, seed, ordering):
    g = gridgen.make_grid(n, seed)
    Y = oracle.grid_ybus(g)
    sym = oracle.Sym(g.n, g.f, g.t, 0, ordering)
    Vm, Va = g.flat_start()
    D, Lb, Ub = sym.block_jacobian(Y, g.bus_type, Vm, Va)
    A = sym.dense_matrix(D, Lb, Ub)
    Df, L, U, bad = sym.factor(D, Lb, Ub)
    assert bad == -1
    nn = sym.nn
    Lm = np.eye(2 * nn)
    Um = np.eye(2 * nn)
    Dm = np.zeros((2 * nn, 2 * nn))
    for p in range(nn):
        Dm[2 * p:2 * p + 2, 2 * p:2 * p + 2] = Df[p]
        for q in range(sym.Lp[p], sym.Lp[p + 1]):
            k = sym.Li[q]
            Lm[2 * k:2 * k + 2, 2 * p:2 * p + 2] = L[q]
            Um[2 * p:2 * p + 2, 2 * k:2 * k + 2] = U[q]
    assert np.abs(Lm @ Dm @ Um - A).max() <= 1e-13 * np.abs(A).max()
    rhs = np.random.default_rng(seed).standard_normal(2 * nn)
    x = sym.solve(Df, L, U, rhs).reshape(-1)
    np.testing.assert_allclose(x, np.linalg.solve(A, rhs), rtol=1e-9, atol=1e-10)


def test_zero_pivot_reported(oracle):
    # bus 2 hangs off bus 1 with a zero-impedance-free but purely resistive
    # branch and zero injection derivative: construct a singular D directly.
    sym = oracle.Sym(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    D = np.zeros((2, 2, 2))
    D[:] = np.eye(2)
    D[sym.level_nodes[0]] = 0.0
    Lb = np.zeros((max(sym.nnzL, 1), 2, 2))
    _, _, _, bad = sym.factor(D, Lb, Lb)
    assert bad == sym.level_nodes[0]


# --------------------------------------------------------------------------
# symbolic analysis: brute force and definitions
# --------------------------------------------------------------------------
def pattern_sets(sym):
    return [set(sym.Li[sym.Lp[p]:sym.Lp[p + 1]].tolist()) for p in range(sym.nn)]


def permuted_adjacency(g, sym):
    nn = sym.nn
    pos = np.full(g.n, -1)
    pos[sym.perm] = np.arange(nn)
    A = np.zeros((nn, nn), bool)
    for a, b in zip(g.f, g.t):
        pa, pb = pos[a], pos[b]
        if pa >= 0 and pb >= 0:
            A[pa, pb] = A[pb, pa] = True
    return A


def brute_elimination(A):
    """Dense boolean Gaussian elimination: higher-neighbour sets in G+."""
    A = A.copy()
    nn = A.shape[0]
    out = []
    for i in range(nn):
        hi = np.flatnonzero(A[i, i + 1:]) + i + 1
        for a in hi:
            A[a, hi] = True
        out.append(set(hi.tolist()))
    return out


@pytest.mark.parametrize("n,seed,ordering", [(60, 1, 0), (150, 2, 0), (150, 3, 1), (300, 4, 0)])
def test_fill_equals_brute_force_elimination(oracle, n, seed, ordering):
    g = gridgen.make_grid(n, seed)
    sym = oracle.Sym(g.n, g.f, g.t, 0, ordering)
    assert pattern_sets(sym) == brute_elimination(permuted_adjacency(g, sym))


def test_fill_equals_generic_numeric_lu(oracle):
    g = gridgen.make_grid(40, 6)
    sym = oracle.Sym(g.n, g.f, g.t)
    A = permuted_adjacency(g, sym).astype(float)
    rng = np.random.default_rng(1)
    M = np.where(A, rng.uniform(0.1, 1.0, A.shape), 0.0)
    M = M + M.T + np.diag(rng.uniform(5, 10, A.shape[0]) + A.sum(1) * 2)
    nn = M.shape[0]
    for i in range(nn):  # no-pivot LU, right-looking
        M[i + 1:, i] /= M[i, i]
        M[i + 1:, i + 1:] -= np.outer(M[i + 1:, i], M[i, i + 1:])
    pat = [set((np.flatnonzero(np.abs(M[i + 1:, i]) > 1e-300) + i + 1).tolist())
           for i in range(nn)]
    assert pat == pattern_sets(sym)


def liu_etree(A):
    """Liu's elimination tree from the pattern of A alone (path compression)."""
    nn = A.shape[0]
    parent = np.full(nn, -1)
    anc = np.full(nn, -1)
    for i in range(nn):
        for k in np.flatnonzero(A[i, :i]):
            r = k
            while anc[r] != -1 and anc[r] != i:
                nxt = anc[r]
                anc[r] = i
                r = nxt
            if anc[r] == -1:
                anc[r] = i
                parent[r] = i
    return parent


@pytest.mark.parametrize("n,seed", [(80, 1), (250, 9)])
def test_etree_and_levels_by_definition(oracle, n, seed):
    g = gridgen.make_grid(n, seed)
    sym = oracle.Sym(g.n, g.f, g.t)
    np.testing.assert_array_equal(sym.parent, liu_etree(permuted_adjacency(g, sym)))
    # level = 1 + max child level, leaves 1 (height in the tree)
    lev = np.ones(sym.nn, int)
    for i in range(sym.nn):
        if sym.parent[i] >= 0:
            lev[sym.parent[i]] = max(lev[sym.parent[i]], lev[i] + 1)
    np.testing.assert_array_equal(sym.level, lev)
    # level lists: grouped by level, ascending inside each level
    for l in range(sym.nlev):
        nodes = sym.level_nodes[sym.level_ptr[l]:sym.level_ptr[l + 1]]
        assert np.all(np.diff(nodes) > 0)
        assert np.all(sym.level[nodes] == l + 1)
        anc = set()
        for v in nodes:
            p = sym.parent[v]
            while p >= 0:
                anc.add(p)
                p = sym.parent[p]
        assert not anc & set(nodes.tolist())


def test_minimum_degree_property(oracle):
    g = gridgen.make_grid(120, 3)
    sym = oracle.Sym(g.n, g.f, g.t)
    # replay elimination on the bus graph without the slack
    nbr = {v: set() for v in range(1, g.n)}
    for a, b in zip(g.f, g.t):
        if a and b:
            nbr[a].add(b)
            nbr[b].add(a)
    for p in range(sym.nn):
        alive = sorted(nbr)
        degs = {v: len(nbr[v]) for v in alive}
        dmin = min(degs.values())
        expect = min(v for v in alive if degs[v] == dmin)
        v = sym.perm[p]
        assert v == expect
        nb = nbr.pop(v)
        for a in nb:
            nbr[a].discard(v)
            nbr[a] |= nb - {a}


def test_table1_level_partition(oracle):
    """Table I of the paper from an elimination tree consistent with it."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_levels.txt")
    rows = [l.split("\t") for l in open(path) if l.strip() and not l.startswith("#")]
    expect = {int(a): sorted(int(x) for x in b.strip().split(",")) for a, b in rows}
    parent = {1: 3, 2: 3, 4: 5, 3: 7, 5: 7, 6: 7, 7: 8, 8: 9, 9: 10}
    f = np.array(list(parent.keys()), np.int32)
    t = np.array(list(parent.values()), np.int32)
    # bus 0 is an isolated slack; natural order keeps node k = bus k.
    sym = oracle.Sym(11, f, t, 0, 1)
    assert sym.nnzL == len(parent)  # a tree ordered leaves-first has no fill
    got = {}
    for l in range(sym.nlev):
        got[l + 1] = sorted(int(sym.perm[v]) for v in
                            sym.level_nodes[sym.level_ptr[l]:sym.level_ptr[l + 1]])
    assert got == expect


def test_slack_articulation_forest(oracle):
    # slack joins two otherwise separate parts: the tree becomes a forest
    f = np.array([0, 1, 0, 3], np.int32)
    t = np.array([1, 2, 3, 4], np.int32)
    sym = oracle.Sym(5, f, t)
    assert int(np.sum(sym.parent == -1)) == 2


# --------------------------------------------------------------------------
# adjoint
# --------------------------------------------------------------------------
def solve_tight(oracle, g, Psp, Qsp, x):
    Y = oracle.ybus(g.n, g.f, g.t, g.r, x, g.b, g.gsh, g.bsh)
    Vm0, Va0 = g.flat_start()
    r = oracle.newton_dense(Y, g.bus_type, Psp, Qsp, Vm0, Va0, tol=1e-13, max_iter=40)
    assert r.status in (0, 6) and r.norm < 1e-11
    return r


def loss_grad(g, Vm, w):
    gVm = 2 * w * (Vm - 1)
    gVm[g.bus_type != gridgen.BUS_PQ] = 0
    return gVm


@pytest.mark.parametrize("shunt_seed", [None, 47])
def test_adjoint_matches_central_fd(oracle, shunt_seed):
    g = shunted(40, 21, shunt_seed)
    rng = np.random.default_rng(6)
    w = rng.uniform(0, 1, g.n)
    Y = oracle.grid_ybus(g)
    base = solve_tight(oracle, g, g.Psp, g.Qsp, g.x)
    gVm = loss_grad(g, base.Vm, w)
    gVa = np.zeros(g.n)
    gP, gQ, gx = oracle.adjoint_dense(g, Y, base.Vm, base.Va, gVm, gVa)

    def loss(Psp, Qsp, x):
        r = solve_tight(oracle, g, Psp, Qsp, x)
        pq = g.bus_type == gridgen.BUS_PQ
        return np.sum((w * (r.Vm - 1) ** 2)[pq])

    h = 1e-6
    for i in [1, 5, 17, 33]:
        e = np.zeros(g.n)
        e[i] = h
        fdP = (loss(g.Psp + e, g.Qsp, g.x) - loss(g.Psp - e, g.Qsp, g.x)) / (2 * h)
        fdQ = (loss(g.Psp, g.Qsp + e, g.x) - loss(g.Psp, g.Qsp - e, g.x)) / (2 * h)
        assert gP[i] == pytest.approx(fdP, rel=1e-5, abs=1e-9)
        assert gQ[i] == pytest.approx(fdQ, rel=1e-5, abs=1e-9)
    for ei in [0, 7, 30, 45]:
        e = np.zeros(g.m)
        e[ei] = h
        fdx = (loss(g.Psp, g.Qsp, g.x + e) - loss(g.Psp, g.Qsp, g.x - e)) / (2 * h)
        assert gx[ei] == pytest.approx(fdx, rel=1e-5, abs=1e-9)
    assert np.all(gQ[g.bus_type != gridgen.BUS_PQ] == 0)
    assert gP[0] == 0


def test_adjoint_two_bus_closed_form(oracle):
    """d|V1|/dP and dtheta1/dQ of the closed form vs the adjoint with unit seeds."""
    r, x, b, P, Q = 0.02, 0.08, 0.04, 0.9, 0.3
    g = two_bus(r, x, b, P, Q)
    Y = oracle.grid_ybus(g)
    res = oracle.solve_grid(g, sparse=False, tol=1e-13, max_iter=30)
    h = 1e-6
    # load P is -Psp: d/dPsp = -d/dP
    dvm_dP = (closed_form_pq(r, x, b, P + h, Q)[0] - closed_form_pq(r, x, b, P - h, Q)[0]) / (2 * h)
    dth_dQ = (closed_form_pq(r, x, b, P, Q + h)[1] - closed_form_pq(r, x, b, P, Q - h)[1]) / (2 * h)
    dvm_dx = (closed_form_pq(r, x + h, b, P, Q)[0] - closed_form_pq(r, x - h, b, P, Q)[0]) / (2 * h)
    gP, gQ, gx = oracle.adjoint_dense(g, Y, res.Vm, res.Va, np.array([0.0, 1.0]), np.zeros(2))
    assert gP[1] == pytest.approx(-dvm_dP, rel=1e-7)
    assert gx[0] == pytest.approx(dvm_dx, rel=1e-7)
    gP, gQ, gx = oracle.adjoint_dense(g, Y, res.Vm, res.Va, np.zeros(2), np.array([0.0, 1.0]))
    assert gQ[1] == pytest.approx(-dth_dQ, rel=1e-7)


def test_sparse_adjoint_equals_dense_adjoint(oracle):
    for n, seed, shunt_seed in [(60, 2, None), (250, 8, None), (120, 5, 48)]:
        g = shunted(n, seed, shunt_seed)
        Y = oracle.grid_ybus(g)
        res = oracle.solve_grid(g)
        rng = np.random.default_rng(seed)
        gVm = rng.standard_normal(n)
        gVa = rng.standard_normal(n)
        d = oracle.adjoint_dense(g, Y, res.Vm, res.Va, gVm, gVa)
        s = oracle.Sym(g.n, g.f, g.t).adjoint(g, Y, res.Vm, res.Va, gVm, gVa)
        for a, b in zip(d, s):
            np.testing.assert_allclose(b, a, rtol=0, atol=1e-11 * np.abs(a).max())


def test_transpose_solve_matches_lapack(oracle):
    g = gridgen.make_grid(150, 6)
    Y = oracle.grid_ybus(g)
    sym = oracle.Sym(g.n, g.f, g.t)
    Vm, Va = random_state(g, np.random.default_rng(4))
    D, Lb, Ub = sym.block_jacobian(Y, g.bus_type, Vm, Va)
    A = sym.dense_matrix(D, Lb, Ub)
    fD, fL, fU, bad = sym.factor(D, Lb, Ub)
    assert bad == -1
    rhs = np.random.default_rng(1).standard_normal(2 * sym.nn)
    x = sym.solve_transpose(fD, fL, fU, rhs).reshape(-1)
    np.testing.assert_allclose(x, np.linalg.solve(A.T, rhs), rtol=1e-9, atol=1e-10)


# --------------------------------------------------------------------------
# fast decoupled power flow and branch flows
# --------------------------------------------------------------------------
def dense_xb(g):
    """B' and B'' over non-slack buses in bus order, written branch by branch
    from their definitions (independent of the oracle's sparse assembly)."""
    keep = [i for i in range(g.n) if g.bus_type[i] != gridgen.BUS_SLACK]
    idx = {bus: k for k, bus in enumerate(keep)}
    N = len(keep)
    B1 = np.zeros((N, N))
    B2 = np.zeros((N, N))
    for e in range(g.m):
        a, c = int(g.f[e]), int(g.t[e])
        y = 1.0 / complex(g.r[e], g.x[e])
        for u, v in ((a, c), (c, a)):
            if u in idx:
                B1[idx[u], idx[u]] += 1.0 / g.x[e]
                B2[idx[u], idx[u]] += -(y.imag + g.b[e] / 2.0)
                if v in idx:
                    B1[idx[u], idx[v]] -= 1.0 / g.x[e]
                    B2[idx[u], idx[v]] -= -y.imag
    for bus in keep:  # B'' = -Im(Y): a shunt susceptance lowers the diagonal
        B2[idx[bus], idx[bus]] -= g.bsh[bus]
    for bus in keep:
        if g.bus_type[bus] == gridgen.BUS_PV:
            k = idx[bus]
            B2[k, :] = 0.0
            B2[:, k] = 0.0
            B2[k, k] = 1.0
    return keep, B1, B2


def to_bus_order(s, A):
    """Position-order dense matrix -> non-slack bus order."""
    bus_of_pos = s.perm  # perm[p] = bus at position p
    order = np.argsort(bus_of_pos)
    return A[np.ix_(order, order)]


@pytest.mark.parametrize("n,seed,shunt_seed", [(60, 1, None), (200, 2, None), (120, 3, 49)])
def test_fdpf_matrices_match_definition(oracle, n, seed, shunt_seed):
    g = shunted(n, seed, shunt_seed)
    s = oracle.Sym(g.n, g.f, g.t)
    d1, a1, d2, a2 = s.fdpf_matrices(g)
    keep, B1, B2 = dense_xb(g)
    np.testing.assert_allclose(to_bus_order(s, s.scalar_matrix(d1, a1)), B1, rtol=0, atol=1e-10)
    np.testing.assert_allclose(to_bus_order(s, s.scalar_matrix(d2, a2)), B2, rtol=0, atol=1e-10)
    # B'' is -Im(Y) of the admittance matrix (shunts included) off the PV buses
    Yd = oracle.grid_ybus(g).dense()[np.ix_(keep, keep)]
    pq = g.bus_type[keep] == gridgen.BUS_PQ
    np.testing.assert_allclose(B2[np.ix_(pq, pq)], -Yd.imag[np.ix_(pq, pq)], rtol=0, atol=1e-10)
    # lossless, charging-free branches make the two matrices agree away from PV buses
    g0 = gridgen.make_grid(n, seed)
    g0.r[:] = 0.0
    g0.b[:] = 0.0
    e1, b1, e2, b2 = s.fdpf_matrices(g0)
    pq = np.array([g0.bus_type[s.perm[p]] == gridgen.BUS_PQ for p in range(s.nn)])
    np.testing.assert_allclose(e1[pq], e2[pq], rtol=1e-14)


@pytest.mark.parametrize("n,seed,ordering", [(80, 1, 0), (200, 3, 0), (150, 2, 1)])
def test_symmetric_factor_eq2_and_reconstruction(oracle, n, seed, ordering):
    """Eq. 2 (u_ij = l_ji) holds on the factors of a symmetric matrix, and
    L D L^T rebuilds it; solves agree with LAPACK."""
    g = gridgen.make_grid(n, seed)
    s = oracle.Sym(g.n, g.f, g.t, 0, ordering)
    for d, a in (s.fdpf_matrices(g)[:2], s.fdpf_matrices(g)[2:]):
        fd, L, U, bad = s.factor1(d, a)
        assert bad == -1
        np.testing.assert_allclose(L, U, rtol=1e-12, atol=1e-15)
        nn = s.nn
        Lm = np.eye(nn)
        for p in range(nn):
            for q in range(s.Lp[p], s.Lp[p + 1]):
                Lm[s.Li[q], p] = L[q]
        A = s.scalar_matrix(d, a)
        np.testing.assert_allclose(Lm @ np.diag(fd) @ Lm.T, A, rtol=0,
                                   atol=1e-12 * np.abs(A).max())
        rhs = np.random.default_rng(seed).standard_normal(nn)
        np.testing.assert_allclose(s.solve1(fd, L, U, rhs), np.linalg.solve(A, rhs), rtol=0,
                                   atol=1e-10 * np.abs(np.linalg.solve(A, rhs)).max())


def test_symmetric_factor_zero_pivot(oracle):
    g = gridgen.make_grid(60, 1)
    s = oracle.Sym(g.n, g.f, g.t)
    d, a, _, _ = s.fdpf_matrices(g)
    d = d.copy()
    leaf = int(s.level_nodes[0])
    d[leaf] = 0.0
    assert s.factor1(d, a)[3] == leaf


def fdpf_dense(g, Psp, Qsp, tol=1e-8, max_iter=40):
    """The XB iteration with dense matrices and LAPACK solves."""
    O = __import__("oracle.oracle", fromlist=["oracle"])
    keep, B1, B2 = dense_xb(g)
    keep = np.array(keep)
    Y = O.grid_ybus(g)
    Vm, Va = g.flat_start()
    pq = g.bus_type[keep] == gridgen.BUS_PQ
    it, half = 0, 0
    while True:
        P, Q = O.injections(Y, Vm, Va)
        FP, FQ, nrm = O.mismatch(g.bus_type, P, Q, Psp, Qsp)
        if nrm < tol:
            return Vm, Va, it, 0
        if half == 0:
            if it >= max_iter:
                return Vm, Va, it, 6
            Va = Va.copy()
            Va[keep] -= np.linalg.solve(B1, FP[keep] / Vm[keep])
            it += 1
        else:
            Vm = Vm.copy()
            rhs = np.where(pq, FQ[keep] / Vm[keep], 0.0)
            Vm[keep] -= np.where(pq, np.linalg.solve(B2, rhs), 0.0)
        half ^= 1


@pytest.mark.parametrize("n,seed,shunt_seed", [(100, 1, None), (300, 4, None), (200, 6, 50)])
def test_fdpf_sparse_equals_dense_definition(oracle, n, seed, shunt_seed):
    g = shunted(n, seed, shunt_seed)
    Vm, Va, it, st = fdpf_dense(g, g.Psp, g.Qsp)
    r = oracle.solve_grid_fdpf(g)
    assert st == 0 and r.status == 0
    assert r.iters == it
    np.testing.assert_allclose(r.Vm, Vm, rtol=0, atol=1e-11)
    np.testing.assert_allclose(r.Va, Va, rtol=0, atol=1e-11)


@pytest.mark.parametrize("n,seed,shunt_seed", [(200, 1, None), (2000, 2, None), (500, 3, 51)])
def test_fdpf_reaches_the_newton_solution(oracle, n, seed, shunt_seed):
    """Both methods stop at max|F| < 1e-8 on the same equations, so they
    reach the same state up to that tolerance."""
    g = shunted(n, seed, shunt_seed)
    a = oracle.solve_grid_fdpf(g)
    b = oracle.solve_grid(g)
    assert a.status == 0 and b.status == 0
    assert a.iters > b.iters  # decoupled steps are cheaper but more
    np.testing.assert_allclose(a.Vm, b.Vm, rtol=0, atol=1e-8)
    np.testing.assert_allclose(a.Va, b.Va, rtol=0, atol=1e-8)


def test_fdpf_not_converged_and_nonfinite(oracle):
    g = gridgen.make_grid(200, 1)
    assert oracle.solve_grid_fdpf(g, max_iter=2).status == 6
    P = g.Psp.copy()
    P[5] = np.nan
    assert oracle.solve_grid_fdpf(g, Psp=P).status == 7


@pytest.mark.parametrize("n,seed,shunt_seed", [(200, 1, None), (1000, 3, None), (300, 2, 52)])
def test_branch_flows_kcl_and_series_losses(oracle, n, seed, shunt_seed):
    """Flows leaving each bus plus its shunt's consumption |V|^2 (g_sh - j b_sh)
    sum to its injection (Kirchhoff), and each branch's losses equal the
    series-element loss minus the charging."""
    g = shunted(n, seed, shunt_seed)
    r = oracle.solve_grid(g)
    Pft, Qft, Ptf, Qtf = oracle.branch_flows(g, r.Vm, r.Va)
    P, Q = oracle.injections(oracle.grid_ybus(g), r.Vm, r.Va)
    sp = np.zeros(g.n)
    sq = np.zeros(g.n)
    np.add.at(sp, g.f, Pft)
    np.add.at(sp, g.t, Ptf)
    np.add.at(sq, g.f, Qft)
    np.add.at(sq, g.t, Qtf)
    sp += g.gsh * r.Vm ** 2
    sq -= g.bsh * r.Vm ** 2
    np.testing.assert_allclose(sp, P, rtol=0, atol=1e-11)
    np.testing.assert_allclose(sq, Q, rtol=0, atol=1e-11)
    V = r.Vm * np.exp(1j * r.Va)
    i_series = (V[g.f] - V[g.t]) / (g.r + 1j * g.x)
    np.testing.assert_allclose(Pft + Ptf, g.r * np.abs(i_series) ** 2, rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(
        Qft + Qtf, g.x * np.abs(i_series) ** 2 - g.b / 2 * (r.Vm[g.f] ** 2 + r.Vm[g.t] ** 2),
        rtol=1e-9, atol=1e-13)


# --------------------------------------------------------------------------
# WLS state estimation
# --------------------------------------------------------------------------
def _se():
    from oracle import se

    return se


@pytest.mark.parametrize("shunt_seed", [None, 54])
def test_se_jacobian_matches_finite_differences(oracle, shunt_seed):
    se = _se()
    g = shunted(30, 2, shunt_seed)
    Y = oracle.grid_ybus(g)
    rng = np.random.default_rng(1)
    Vm = 1 + 0.05 * rng.standard_normal(g.n)
    Va = 0.1 * rng.standard_normal(g.n)
    kinds, locs = se.full_measurement_set(g)
    H = se.jacobian(g, Y, Vm, Va, kinds, locs).toarray()
    h = 1e-6
    cols = [("a", b) for b in range(1, g.n)] + [("m", b) for b in range(g.n)]
    for c, (which, b) in enumerate(cols):
        Vp, Ap, Vn, An = Vm.copy(), Va.copy(), Vm.copy(), Va.copy()
        if which == "a":
            Ap[b] += h
            An[b] -= h
        else:
            Vp[b] += h
            Vn[b] -= h
        fd = (se.measure(g, Y, Vp, Ap, kinds, locs) - se.measure(g, Y, Vn, An, kinds, locs)) / (2 * h)
        np.testing.assert_allclose(H[:, c], fd, rtol=0, atol=1e-6)


@pytest.mark.parametrize("shunt_seed", [None, 53])
def test_se_recovers_the_power_flow_state(oracle, shunt_seed):
    """Noise-free measurements of a solved power flow: the estimate is that
    state (the estimator and the power flow share no step)."""
    se = _se()
    g = shunted(200, 3, shunt_seed)
    ref = oracle.solve_grid(g)
    kinds, locs = se.full_measurement_set(g)
    z = se.measure(g, oracle.grid_ybus(g), ref.Vm, ref.Va, kinds, locs)
    w = np.where(kinds == se.VM, 1 / 0.004 ** 2, 1 / 0.01 ** 2)
    r = se.estimate(g, kinds, locs, z, w, np.ones(g.n), np.zeros(g.n))
    assert r.status == 0
    np.testing.assert_allclose(r.Vm, ref.Vm, rtol=0, atol=1e-10)
    np.testing.assert_allclose(r.Va, ref.Va, rtol=0, atol=1e-10)


def test_se_step_is_the_least_squares_step(oracle):
    se = _se()
    g = gridgen.make_grid(30, 4)
    Y = oracle.grid_ybus(g)
    kinds, locs = se.full_measurement_set(g)
    rng = np.random.default_rng(2)
    Vm, Va = 1 + 0.02 * rng.standard_normal(g.n), 0.05 * rng.standard_normal(g.n)
    z = se.measure(g, Y, Vm, Va, kinds, locs) + 0.01 * rng.standard_normal(len(kinds))
    w = rng.uniform(100, 10000, len(kinds))
    H = se.jacobian(g, Y, np.ones(g.n), np.zeros(g.n), kinds, locs).toarray()
    res = z - se.measure(g, Y, np.ones(g.n), np.zeros(g.n), kinds, locs)
    dx_ne = np.linalg.solve(H.T @ (w[:, None] * H), H.T @ (w * res))
    dx_ls = np.linalg.lstsq(np.sqrt(w)[:, None] * H, np.sqrt(w) * res, rcond=None)[0]
    np.testing.assert_allclose(dx_ne, dx_ls, rtol=1e-8, atol=1e-10)
    r1 = se.estimate(g, kinds, locs, z, w, np.ones(g.n), np.zeros(g.n), max_iter=1)
    np.testing.assert_allclose(r1.Vm - 1.0, dx_ls[g.n - 1:], rtol=1e-8, atol=1e-10)


def test_se_optimality_with_noise(oracle):
    """At the noisy estimate the weighted residual is orthogonal to H."""
    se = _se()
    g = gridgen.make_grid(200, 5)
    ref = oracle.solve_grid(g)
    Y = oracle.grid_ybus(g)
    kinds, locs = se.full_measurement_set(g)
    sig = np.where(kinds == se.VM, 0.004, 0.01)
    z = se.measure(g, Y, ref.Vm, ref.Va, kinds, locs)
    z = z + sig * np.random.default_rng(7).standard_normal(len(z))
    r = se.estimate(g, kinds, locs, z, 1 / sig ** 2, np.ones(g.n), np.zeros(g.n))
    assert r.status == 0
    H = se.jacobian(g, Y, r.Vm, r.Va, kinds, locs)
    grad = H.T @ ((z - se.measure(g, Y, r.Vm, r.Va, kinds, locs)) / sig ** 2)
    assert np.abs(grad).max() < 1e-6 * np.abs(H.T @ (z / sig ** 2)).max()
