"""Failure reporting (Sec. III-B factorises without pivoting, so a singular
pivot block is reported, never repaired): the position of the first zero
pivot from pf_factor and pf_newton against the oracle's, at a leaf of the
global levels, at a node of the LDS tail below its clique and inside the
clique; and NaN gradients from the adjoint for cases that did not converge."""
import dataclasses

import numpy as np
import pytest

import gridgen
from gpu_helpers import Staged, dev, grid, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OPEN_X = 1e300


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _B():
    from paper_1811_02512_amd import binding

    return binding


def isolate(g, bus):
    """Opens every branch at `bus` (r = 0, x = 1e300, charging 0): the bus
    keeps its place in the pattern, but its Jacobian block is of order 1e-300
    and its determinant underflows to exactly zero."""
    at = (g.f == bus) | (g.t == bus)
    r, x, b = g.r.copy(), g.x.copy(), g.b.copy()
    r[at], x[at], b[at] = 0.0, OPEN_X, 0.0
    return dataclasses.replace(g, r=r, x=x, b=b)


def regions(info, ex):
    """Positions of the global levels' leaves, the tail below the clique and
    the clique, in level order."""
    lp, ln = ex["level_ptr"], ex["level_nodes"]
    nlev = info.nlevels
    t0 = lp[nlev - info.tail_levels]
    kc = info.tail_clique
    return (ln[lp[0]:lp[1]].tolist(), ln[t0:len(ln) - kc].tolist(), ln[len(ln) - kc:].tolist())


def pick(O, g, positions, perm, osym):
    """The first PQ bus among `positions` whose isolation makes the oracle
    fail first at that very position; returns (grid, position)."""
    for p in positions:
        bus = int(perm[p])
        if g.bus_type[bus] != gridgen.BUS_PQ:
            continue
        q = isolate(g, bus)
        ref = osym.newton(O.grid_ybus(q), q.bus_type, q.Psp, q.Qsp, *q.flat_start())
        if ref.status == 5 and ref.bad_node == p:
            return q, p
    raise AssertionError("no isolatable PQ bus in the region")


@pytest.mark.parametrize("where", ["global_leaf", "tail", "clique"])
def test_newton_zero_pivot_position(where):
    from oracle import oracle as O

    g = grid(2000, 3)
    s0 = Staged(g)
    info = s0.info
    ex = s0.sym.export()
    leaves, tail, clique = regions(info, ex)
    assert info.tail_levels > 0 and info.tail_clique >= 3 and len(tail) > 0
    osym = O.Sym(g.n, g.f, g.t)
    region = {"global_leaf": leaves, "tail": tail, "clique": clique}[where]
    q, p = pick(O, g, region, ex["perm"], osym)
    log(f"[failures] {where}: position {p} (bus {ex['perm'][p]})")
    s = Staged(q)
    Bn = 3  # one healthy neighbour case on each side shares the launch
    Vm = s.Vm0.repeat(Bn, 1).contiguous()
    Va = s.Va0.repeat(Bn, 1).contiguous()
    y = torch.stack([Staged(g).yval[0], s.yval[0], Staged(g).yval[0]])
    it = torch.full((Bn,), -2, dtype=torch.int32, device="cuda")
    st = torch.full((Bn,), -2, dtype=torch.int32, device="cuda")
    pv = torch.full((Bn,), -2, dtype=torch.int32, device="cuda")
    B = _B()
    ws = s.sym.workspace(Bn)
    B.pf_newton(s.sym.h, Bn, y, y.shape[1], s.type, 0, s.Psp, s.Qsp, 0, Vm, Va, g.n, 1e-8, 20,
                B.PF_NEWTON_KEEP_FACTORS, ws, info.ws_doubles, it, None, st, pv)
    assert st.cpu().tolist() == [0, B.PF_E_ZERO_PIVOT, 0]
    assert pv.cpu().tolist() == [-1, p, -1]
    assert it[1].item() == 0
    # pf_factor on the same Jacobian reports the same position
    vals = torch.zeros(1, info.vals_doubles, dtype=torch.float64, device="cuda")
    B.pf_jacobian(s.sym.h, 1, s.yval, 0, s.type, 0, s.Vm0, s.Va0, 0, vals, info.vals_doubles)
    fst = torch.full((1,), -2, dtype=torch.int32, device="cuda")
    fpv = torch.full((1,), -2, dtype=torch.int32, device="cuda")
    B.pf_factor(s.sym.h, 1, vals, info.vals_doubles, fst, 1, fpv)
    assert fst.item() == B.PF_E_ZERO_PIVOT and fpv.item() == p


def test_factor_zero_pivot_positions():
    """Identity blocks with singular ones at chosen positions: the reported
    position is the first failure in level order, positions ascending."""
    B = _B()
    s = Staged(grid(200, 1))
    info = s.info
    ex = s.sym.export()
    ln = ex["level_nodes"]
    nn = info.nn
    picks = [[], [int(ln[-1])], [int(ln[40]), int(ln[7])], [int(ln[len(ln) // 2]), int(ln[-2])]]
    Bn = len(picks)
    vals = torch.zeros(Bn, info.vals_doubles, dtype=torch.float64, device="cuda")
    d = vals[:, :4 * nn].view(Bn, nn, 4)
    d[:, :, 0] = 1.0
    d[:, :, 3] = 1.0
    for c, ps in enumerate(picks):
        for p in ps:
            d[c, p] = 0.0
    st = torch.full((Bn,), -2, dtype=torch.int32, device="cuda")
    pv = torch.full((Bn,), -2, dtype=torch.int32, device="cuda")
    B.pf_factor(s.sym.h, Bn, vals, info.vals_doubles, st, 1, pv)
    level_of = np.empty(nn, np.int64)
    level_of[ln] = np.arange(nn)  # level-ordered index of each position
    want = [-1 if not ps else min(ps, key=lambda p: level_of[p]) for ps in picks]
    assert st.cpu().tolist() == [0] + [B.PF_E_ZERO_PIVOT] * 3
    assert pv.cpu().tolist() == want


def test_adjoint_nan_for_failed_cases():
    """A case with a non-finite injection ends PF_E_NONFINITE: its gradients
    are NaN (so is the gradient summed over cases), the others' match the
    oracle, and the status comes back with the solution."""
    from oracle import oracle as O

    from paper_1811_02512_amd import api
    from paper_1811_02512_amd.autograd import power_flow

    g = grid(300, 2)
    sym = api.Symbolic(g.n, g.f, g.t).upload()
    P, Q = gridgen.scenario_injections(g, 3, 2)
    P[1, 17] = np.nan
    w = np.random.default_rng(6).uniform(0, 1, g.n)
    Pt = dev(P).requires_grad_(True)
    Qt = dev(Q).requires_grad_(True)
    xt = dev(g.x).requires_grad_(True)
    Vm0, Va0 = g.flat_start()
    Vm, Va, status, iters = power_flow(sym, Pt, Qt, xt, dev(g.r), dev(g.b),
                                       dev(g.bus_type.astype(np.int8)), dev(Vm0), dev(Va0),
                                       with_status=True)
    assert status.cpu().tolist() == [0, 7, 0]
    pq = dev((g.bus_type == gridgen.BUS_PQ).astype(np.float64))
    ok = torch.tensor([1.0, 0.0, 1.0], dtype=torch.float64, device="cuda")[:, None]
    ((dev(w) * pq * ok * (Vm.nan_to_num() - 1.0) ** 2).sum()).backward()
    gP = Pt.grad.cpu().numpy()
    assert np.isnan(gP[1]).all() and np.isnan(Qt.grad[1].cpu().numpy()).all()
    assert np.isnan(xt.grad.cpu().numpy()).all()
    Vmh = Vm.detach().cpu().numpy()
    Y = O.grid_ybus(g)
    for c in (0, 2):
        gv = 2 * w * (Vmh[c] - 1)
        gv[g.bus_type != gridgen.BUS_PQ] = 0
        rP, _, _ = O.adjoint_dense(g, Y, Vmh[c], Va.detach().cpu().numpy()[c], gv, np.zeros(g.n))
        np.testing.assert_allclose(gP[c], rP, rtol=0, atol=1e-9 * np.abs(rP).max())


def test_adjoint_not_converged_is_nan():
    from paper_1811_02512_amd import api
    from paper_1811_02512_amd.autograd import power_flow

    g = grid(200, 1)
    sym = api.Symbolic(g.n, g.f, g.t).upload()
    Pt = dev(g.Psp[None]).requires_grad_(True)
    Vm0, Va0 = g.flat_start()
    Vm, _, status, iters = power_flow(sym, Pt, dev(g.Qsp[None]), dev(g.x), dev(g.r), dev(g.b),
                                      dev(g.bus_type.astype(np.int8)), dev(Vm0), dev(Va0),
                                      max_iter=1, with_status=True)
    assert status.item() == 6 and iters.item() == 1
    Vm.sum().backward()
    assert torch.isnan(Pt.grad).all()


def _fused_vs_three_step(g, Bn, mode, seed=3):
    B = _B()
    s = Staged(g)
    P, Q = gridgen.scenario_injections(g, Bn, seed)
    Vm, Va, it, _, st, ws = s.newton(Bn, dev(P), dev(Q), keep=True)
    assert (st == 0).all()
    info = s.info
    n, nn, m = g.n, info.nn, g.m
    rng = np.random.default_rng(5)
    gVm, gVa = dev(rng.standard_normal((Bn, n))), dev(rng.standard_normal((Bn, n)))
    C = B.pf_newton_interleave(s.sym.h, Bn)
    f64 = dict(dtype=torch.float64, device="cuda")
    xs = s.x if mode == 1 else s.x.repeat(Bn)
    rs = s.r if mode == 1 else s.r.repeat(Bn)
    bstride = 0 if mode == 1 else m
    gxn = m if mode == 1 else Bn * m
    out = []
    for rep in range(2):  # twice on the same workspace: its scratch sections are rewritten
        lam1 = torch.empty(Bn, 2 * nn, **f64)
        gP1, gQ1, gx1 = (torch.empty(Bn, n, **f64), torch.empty(Bn, n, **f64),
                         torch.empty(gxn, **f64))
        B.pf_adjoint(s.sym.h, Bn, ws, info.ws_doubles, gVm, gVa, n, s.type, 0, Vm, Va, n, rs,
                     xs, bstride, st, lam1, 2 * nn, gP1, gQ1, n, gx1, mode)
        out.append((lam1, gP1, gQ1, gx1))
    lam2 = torch.empty(Bn, 2 * nn, **f64)
    gP2, gQ2, gx2 = torch.empty(Bn, n, **f64), torch.empty(Bn, n, **f64), torch.empty(gxn, **f64)
    B.pf_adjoint_rhs(s.sym.h, Bn, gVm, gVa, n, s.type, 0, lam2, 2 * nn)
    B.pf_solve(s.sym.h, Bn, ws, info.ws_doubles, lam2, 2 * nn, 1, C)
    B.pf_adjoint_params(s.sym.h, Bn, lam2, 2 * nn, s.type, 0, Vm, Va, n, rs, xs, bstride, gP2,
                        gQ2, n, gx2, mode)
    for got in out:
        for a, b in zip(got, (lam2, gP2, gQ2, gx2)):
            assert torch.equal(a, b)
    return s, ws, Vm, Va, st, gVa


@pytest.mark.parametrize("mode", [1, 0])
def test_fused_adjoint_equals_the_three_step_path(mode):
    """pf_adjoint (gather, transposed solves, bus and per-case branch
    gradients in one launch, their sum over cases in a second) gives bitwise
    the results of pf_adjoint_rhs, pf_solve(transpose = 1) and
    pf_adjoint_params, also when called twice on one workspace."""
    B = _B()
    g = grid(2000, 1)
    Bn = 8
    s, ws, Vm, Va, st, gVa = _fused_vs_three_step(g, Bn, mode)
    if mode == 0:
        return
    info = s.info
    n, nn = g.n, info.nn
    f64 = dict(dtype=torch.float64, device="cuda")
    lam1, lam2 = torch.empty(Bn, 2 * nn, **f64), torch.empty(Bn, 2 * nn, **f64)
    gP1, gQ1 = torch.empty(Bn, n, **f64), torch.empty(Bn, n, **f64)
    gP2, gQ2 = torch.empty(Bn, n, **f64), torch.empty(Bn, n, **f64)
    # absent gradients read as zero
    B.pf_adjoint(s.sym.h, Bn, ws, info.ws_doubles, None, gVa, n, s.type, 0, Vm, Va, n, s.r,
                 s.x, 0, None, lam1, 2 * nn, gP1, gQ1, n, None, 1)
    B.pf_adjoint(s.sym.h, Bn, ws, info.ws_doubles, torch.zeros_like(gVa), gVa, n, s.type, 0, Vm,
                 Va, n, s.r, s.x, 0, None, lam2, 2 * nn, gP2, gQ2, n, None, 1)
    assert torch.equal(lam1, lam2) and torch.equal(gP1, gP2)


def test_fused_adjoint_with_more_branches_than_rhs_room():
    """Every branch doubled (m > 2 nn): the workspace's rhs section cannot hold
    a case's branch values, so the summed dL/dx takes its own kernel; the
    results are still those of the three-step path."""
    g = grid(60, 1)
    g2 = dataclasses.replace(g, f=np.concatenate([g.f, g.f]), t=np.concatenate([g.t, g.t]),
                             r=np.concatenate([g.r, g.r]) * 2, x=np.concatenate([g.x, g.x]) * 2,
                             b=np.concatenate([g.b, g.b]) / 2)
    assert g2.m > 2 * (g2.n - 1)
    _fused_vs_three_step(g2, 4, 1)


def test_adjoint_strides_are_checked_before_any_launch():
    """Strides below a row are refused with PF_E_WORKSPACE by pf_adjoint and
    pf_adjoint_params (B > 1), negative ones with PF_E_INVALID; the outputs
    are left as they were."""
    B = _B()
    g = grid(200, 1)
    s = Staged(g)
    Bn = 2
    P, Q = gridgen.scenario_injections(g, Bn, 3)
    Vm, Va, it, _, st, ws = s.newton(Bn, dev(P), dev(Q), keep=True)
    info = s.info
    n, nn, m = g.n, info.nn, g.m
    f64 = dict(dtype=torch.float64, device="cuda")
    gVm = torch.ones(Bn, n, **f64)
    lam = torch.full((Bn, 2 * nn), 7.0, **f64)
    gP, gQ = torch.full((Bn, n), 7.0, **f64), torch.full((Bn, n), 7.0, **f64)
    gx = torch.full((Bn * m,), 7.0, **f64)
    xs, rs = s.x.repeat(Bn), s.r.repeat(Bn)
    cases = [  # (type_stride, branch_stride, expected code)
        (1, m, B.PF_E_WORKSPACE), (0, m - 1, B.PF_E_WORKSPACE), (-1, m, B.PF_E_INVALID)]
    for ts, bs, code in cases:
        with pytest.raises(B.PfError) as ei:
            B.pf_adjoint(s.sym.h, Bn, ws, info.ws_doubles, gVm, None, n, s.type, ts, Vm, Va, n,
                         rs, xs, bs, st, lam, 2 * nn, gP, gQ, n, gx, 0)
        assert ei.value.code == code
        with pytest.raises(B.PfError) as ei:
            B.pf_adjoint_params(s.sym.h, Bn, lam, 2 * nn, s.type, ts, Vm, Va, n, rs, xs, bs, gP,
                                gQ, n, gx, 0)
        assert ei.value.code == code
    with pytest.raises(B.PfError) as ei:
        B.pf_adjoint_params(s.sym.h, Bn, lam, 2 * nn - 2, s.type, 0, Vm, Va, n, rs, xs, m, gP,
                            gQ, n, gx, 0)
    assert ei.value.code == B.PF_E_WORKSPACE
    torch.cuda.synchronize()
    for t in (lam, gP, gQ, gx):
        assert (t == 7.0).all()


def test_shared_or_per_case_strides_are_checked():
    """A per-case stride of an input the cases may share must be 0 or at least
    one row (B > 1): pf_newton, pf_mismatch and pf_branch_flows refuse the
    rest with PF_E_WORKSPACE and leave their outputs alone."""
    B = _B()
    g = grid(200, 1)
    s = Staged(g)
    Bn = 2
    n, m, nn = g.n, g.m, s.info.nn
    f64 = dict(dtype=torch.float64, device="cuda")
    P, Q = gridgen.scenario_injections(g, Bn, 3)
    Pt, Qt = dev(P), dev(Q)
    Vm = torch.full((Bn, n), 7.0, **f64)
    Va = torch.full((Bn, n), 7.0, **f64)
    ws = torch.zeros(Bn * s.info.ws_doubles + 64, **f64)
    it = torch.full((Bn,), -5, dtype=torch.int32, device="cuda")
    st = torch.full((Bn,), -5, dtype=torch.int32, device="cuda")
    nrm = torch.zeros(Bn, **f64)
    for ys, ts, js in ((0, 1, n), (0, 0, n - 1), (1, 0, n)):
        with pytest.raises(B.PfError) as ei:
            B.pf_newton(s.sym.h, Bn, s.yval, ys, s.type, ts, Pt, Qt, js, Vm, Va, n, 1e-8, 20,
                        0, ws, s.info.ws_doubles, it, nrm, st)
        assert ei.value.code == B.PF_E_WORKSPACE
    rhs = torch.full((Bn, 2 * nn), 7.0, **f64)
    with pytest.raises(B.PfError) as ei:
        B.pf_mismatch(s.sym.h, Bn, s.yval, 0, s.type, 0, Pt, Qt, n, Vm, Va, n, rhs, 2 * nn - 2,
                      nrm)
    assert ei.value.code == B.PF_E_WORKSPACE
    out = [torch.full((Bn, m), 7.0, **f64) for _ in range(4)]
    with pytest.raises(B.PfError) as ei:
        B.pf_branch_flows(s.sym.h, Bn, s.r.repeat(Bn), s.x.repeat(Bn), s.b.repeat(Bn), m - 1,
                          Vm, Va, n, *out, m)
    assert ei.value.code == B.PF_E_WORKSPACE
    torch.cuda.synchronize()
    assert (Vm == 7.0).all() and (Va == 7.0).all() and (rhs == 7.0).all()
    assert (it == -5).all() and (st == -5).all()
    for t in out:
        assert (t == 7.0).all()
