"""Bus shunts (Sec. III-A: shunts on the vertices of the grid graph) through
every GPU entry point that takes them, against the oracle on the same
seeded shunted grids: admittance matrix, Newton-Raphson (one workgroup and,
from 2,000 buses, one case spread over 32 workgroups), batches with
per-case shunts, fast decoupled B'' and iteration, per-case-pattern
batches, state estimation, the adjoint and N-1 screening."""
import dataclasses

import numpy as np
import pytest

import gridgen
from gpu_helpers import Staged, dev, log, shunt_grid

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def O():
    from oracle import oracle

    return oracle


def _B():
    from paper_1811_02512_amd import binding

    return binding


def staged(n, seed, shunt_seed):
    g = shunt_grid(n, seed, shunt_seed)
    log(f"[shunt] n={n} seed={seed} shunt_seed={shunt_seed} "
        f"shunted buses={int(np.count_nonzero(g.bsh))}")
    return Staged(g)


@pytest.mark.parametrize("n,seed,shunt_seed", [(200, 1, 61), (2000, 1, 62)])
def test_ybus_with_shunts(O, n, seed, shunt_seed):
    g = shunt_grid(n, seed, shunt_seed)
    g = dataclasses.replace(g, gsh=g.gsh.copy(), bsh=g.bsh.copy())
    g.gsh[0], g.bsh[0] = 0.004, 0.03  # a shunt at the slack as well
    s = Staged(g)
    Y = O.grid_ybus(g)
    yptr, ycol = s.sym.ybus_pattern()
    np.testing.assert_array_equal(yptr, Y.rowptr)
    np.testing.assert_array_equal(ycol, Y.col)
    yv = s.yval[0].cpu().numpy().reshape(-1, 2)
    scale = np.abs(Y.G).max() + np.abs(Y.B).max()
    np.testing.assert_allclose(yv[:, 0], Y.G, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(yv[:, 1], Y.B, rtol=0, atol=1e-12 * scale)
    # the shunt really is in: the diagonal differs from the shunt-free one
    Y0 = O.ybus(g.n, g.f, g.t, g.r, g.x, g.b)
    assert np.abs(Y.B - Y0.B).max() > 1e-3


def test_ybus_per_case_shunts(O):
    """Three cases with their own shunts (stride 2n) and one shared set."""
    g = gridgen.make_grid(150, 3)
    s = Staged(g)
    gs = [gridgen.with_shunts(g, 70 + c) for c in range(3)]
    ysh = dev(np.stack([q.ysh for q in gs]))  # [3, n, 2]
    y = s.sym.build_ybus(s.r, s.x, s.b, ysh).cpu().numpy()
    assert y.shape[0] == 3
    for c in range(3):
        Y = O.grid_ybus(gs[c])
        v = y[c].reshape(-1, 2)
        np.testing.assert_allclose(v[:, 0], Y.G, rtol=0, atol=1e-12 * np.abs(Y.G).max())
        np.testing.assert_allclose(v[:, 1], Y.B, rtol=0, atol=1e-12 * np.abs(Y.B).max())
    shared = s.sym.build_ybus(s.r, s.x, s.b, dev(gs[1].ysh)).cpu().numpy()
    np.testing.assert_array_equal(shared[0], y[1])


@pytest.mark.parametrize("n,seed,shunt_seed", [(200, 2, 63), (2000, 1, 64), (10000, 1, 65)])
def test_newton_with_shunts(O, n, seed, shunt_seed):
    s = staged(n, seed, shunt_seed)
    g = s.g
    ref = O.solve_grid(g)
    assert ref.status == 0
    plain = O.solve_grid(gridgen.make_grid(n, seed))
    assert np.abs(plain.Vm - ref.Vm).max() > 1e-4  # the shunts move the solution
    Vm, Va, iters, norm, status, _ = s.newton()
    torch.cuda.synchronize()
    log(f"[shunt] newton n={n}: gpu iters={iters.item()} oracle {ref.iters}")
    assert status.item() == 0 and iters.item() == ref.iters
    np.testing.assert_allclose(Vm[0].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Va[0].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)
    P, Q = O.injections(O.grid_ybus(g), Vm[0].cpu().numpy(), Va[0].cpu().numpy())
    assert O.mismatch(g.bus_type, P, Q, g.Psp, g.Qsp)[2] < 1e-8
    if n < 2000:
        return
    # the same case spread over 32 workgroups (cooperative launch)
    s.sym.set_spread(32)
    try:
        Vs, As, its, _, sts, _ = s.newton()
        torch.cuda.synchronize()
    finally:
        s.sym.set_spread(0)
    log(f"[shunt] spread newton n={n}: gpu iters={its.item()} status {sts.item()}")
    assert sts.item() == 0 and its.item() == ref.iters
    np.testing.assert_allclose(Vs[0].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(As[0].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)
    assert (Vs - Vm).abs().max().item() < 1e-12 and (As - Va).abs().max().item() < 1e-12


def test_newton_batch_with_per_case_shunts(O):
    """Scenarios whose shunt settings differ (switched capacitor banks): one
    admittance matrix per case, one launch."""
    g = gridgen.make_grid(2000, 2)
    s = Staged(g)
    Bn = 6
    gs = [gridgen.with_shunts(g, 80 + c, frac=0.1 + 0.05 * c) for c in range(Bn)]
    y = s.sym.build_ybus(s.r, s.x, s.b, dev(np.stack([q.ysh for q in gs])))
    Vm = s.Vm0.repeat(Bn, 1).contiguous()
    Va = s.Va0.repeat(Bn, 1).contiguous()
    iters, _, status, _ = s.sym.newton(y, s.type, s.Psp, s.Qsp, Vm, Va)
    osym = O.Sym(g.n, g.f, g.t)
    for c in range(Bn):
        ref = osym.newton(O.grid_ybus(gs[c]), g.bus_type, g.Psp, g.Qsp, *g.flat_start())
        assert status[c].item() == 0 and iters[c].item() == ref.iters
        np.testing.assert_allclose(Vm[c].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va[c].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)


@pytest.mark.parametrize("n,seed,shunt_seed", [(200, 1, 66), (2000, 2, 67)])
def test_fdpf_with_shunts(O, n, seed, shunt_seed):
    B = _B()
    s = staged(n, seed, shunt_seed)
    g = s.g
    info = s.info
    mat = torch.empty(1, info.fd_mat_doubles, dtype=torch.float64, device="cuda")
    B.pf_fdpf_matrices(s.sym.h, 1, s.r, s.x, s.b, 0, s.type, 0, mat, info.fd_mat_doubles,
                       s.ysh, 0)
    osym = O.Sym(g.n, g.f, g.t)
    d1, a1, d2, a2 = osym.fdpf_matrices(g)
    M = info.fd_mat_doubles // 2
    v = mat[0].cpu().numpy()
    nn = info.nn
    np.testing.assert_allclose(v[:nn], d1, rtol=1e-14, atol=0)
    np.testing.assert_allclose(v[M:M + nn], d2, rtol=1e-13, atol=1e-15)
    mat2, st = s.sym.fdpf_factors(s.r, s.x, s.b, s.type, s.ysh)
    assert st.item() == 0
    Vm = s.Vm0.reshape(1, -1).contiguous()
    Va = s.Va0.reshape(1, -1).contiguous()
    it, _, status, _ = s.sym.fdpf(s.yval[0], s.type, s.Psp, s.Qsp, Vm, Va, mat2)
    ref = osym.fdpf(O.grid_ybus(g), g, g.Psp, g.Qsp, *g.flat_start())
    assert status.item() == 0 and ref.status == 0 and it.item() == ref.iters
    np.testing.assert_allclose(Vm[0].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Va[0].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)


def test_multi_pattern_batch_with_shunts(O):
    """N-1 outages of a shunted grid, each with its own analysis, one launch."""
    from paper_1811_02512_amd import api

    B = _B()
    base = shunt_grid(2000, 1, 68)
    outs = gridgen.n1_outages(base, 6, 9)
    grids = [base.without_branch(int(e)) for e in outs]
    syms = [api.Symbolic(q.n, q.f, q.t).upload() for q in grids]
    plan = api.MultiPlan(syms)
    f64 = np.float64
    r = plan.concat([q.r for q in grids], "branch", f64)
    x = plan.concat([q.x for q in grids], "branch", f64)
    b = plan.concat([q.b for q in grids], "branch", f64)
    ysh = plan.concat([q.ysh for q in grids], "bus", np.dtype((f64, 2))).reshape(-1, 2)
    yv = torch.empty(int(plan.offs["y"][-1]) + 2, dtype=torch.float64, device="cuda")
    B.pf_build_ybus_multi(plan.p, r, x, b, yv, ysh)
    ty = plan.concat([q.bus_type for q in grids], "bus", np.int8)
    P = plan.concat([q.Psp for q in grids], "bus", f64)
    Q = plan.concat([q.Qsp for q in grids], "bus", f64)
    Vm = plan.concat([q.flat_start()[0] for q in grids], "bus", f64)
    Va = plan.concat([q.flat_start()[1] for q in grids], "bus", f64)
    ws = torch.empty(int(plan.offs["ws"][-1]) + 32, dtype=torch.float64, device="cuda")
    G = len(grids)
    it = torch.full((G,), -1, dtype=torch.int32, device="cuda")
    st = torch.full((G,), -1, dtype=torch.int32, device="cuda")
    B.pf_newton_multi(plan.p, yv, ty, P, Q, Vm, Va, 1e-8, 20, 0, ws, it, None, st)
    Vms, Vas = plan.split(Vm, "bus"), plan.split(Va, "bus")
    for c, q in enumerate(grids):
        ref = O.solve_grid(q)
        assert st[c].item() == 0 and it[c].item() == ref.iters
        np.testing.assert_allclose(Vms[c], ref.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Vas[c], ref.Va, rtol=0, atol=1e-9)


def test_state_estimation_with_shunts(O):
    from oracle import se

    from paper_1811_02512_amd import api

    g = shunt_grid(200, 3, 69)
    kinds, locs = se.full_measurement_set(g)
    ref = O.solve_grid(g)
    z0 = se.measure(g, O.grid_ybus(g), ref.Vm, ref.Va, kinds, locs)
    sig = np.where(kinds == se.VM, 0.004, 0.01)
    z = z0 + sig * np.random.default_rng(3).standard_normal((2, len(z0)))
    w = 1.0 / sig ** 2
    est = api.StateEstimator(g.n, g.f, g.t, kinds, locs)
    Vm = torch.ones(2, g.n, dtype=torch.float64, device="cuda")
    Va = torch.zeros(2, g.n, dtype=torch.float64, device="cuda")
    it, _, st, _ = est.estimate(dev(g.r), dev(g.x), dev(g.b), dev(z), dev(w), Vm, Va,
                                ysh=dev(g.ysh))
    for c in range(2):
        r = se.estimate(g, kinds, locs, z[c], w, np.ones(g.n), np.zeros(g.n))
        assert r.status == 0 and st[c].item() == 0 and it[c].item() == r.iters
        np.testing.assert_allclose(Vm[c].cpu().numpy(), r.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va[c].cpu().numpy(), r.Va, rtol=0, atol=1e-9)
    # noise-free measurements recover the shunted power-flow state
    Vm1 = torch.ones(1, g.n, dtype=torch.float64, device="cuda")
    Va1 = torch.zeros(1, g.n, dtype=torch.float64, device="cuda")
    _, _, st1, _ = est.estimate(dev(g.r), dev(g.x), dev(g.b), dev(z0), dev(w), Vm1, Va1,
                                ysh=dev(g.ysh))
    assert st1.item() == 0
    np.testing.assert_allclose(Vm1[0].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)


def test_adjoint_with_shunts(O):
    from paper_1811_02512_amd import api
    from paper_1811_02512_amd.autograd import power_flow

    g = shunt_grid(300, 2, 71)
    sym = api.Symbolic(g.n, g.f, g.t).upload()
    P, Q = gridgen.scenario_injections(g, 3, 2)
    w = np.random.default_rng(6).uniform(0, 1, g.n)
    Pt = dev(P).requires_grad_(True)
    Qt = dev(Q).requires_grad_(True)
    xt = dev(g.x).requires_grad_(True)
    Vm0, Va0 = g.flat_start()
    Vm, Va = power_flow(sym, Pt, Qt, xt, dev(g.r), dev(g.b), dev(g.bus_type.astype(np.int8)),
                        dev(Vm0), dev(Va0), ysh=dev(g.ysh))
    pq = dev((g.bus_type == gridgen.BUS_PQ).astype(np.float64))
    ((dev(w) * pq * (Vm - 1.0) ** 2).sum()).backward()
    Vm, Va = Vm.detach().cpu().numpy(), Va.detach().cpu().numpy()
    Y = O.grid_ybus(g)
    gx_ref = np.zeros(g.m)
    for c in range(3):
        gv = 2 * w * (Vm[c] - 1)
        gv[g.bus_type != gridgen.BUS_PQ] = 0
        rP, rQ, rx = O.adjoint_dense(g, Y, Vm[c], Va[c], gv, np.zeros(g.n))
        sc = max(np.abs(rP).max(), np.abs(rQ).max())
        np.testing.assert_allclose(Pt.grad[c].cpu().numpy(), rP, rtol=0, atol=1e-9 * sc)
        np.testing.assert_allclose(Qt.grad[c].cpu().numpy(), rQ, rtol=0, atol=1e-9 * sc)
        gx_ref += rx
    np.testing.assert_allclose(xt.grad.cpu().numpy(), gx_ref, rtol=0,
                               atol=1e-9 * np.abs(gx_ref).max())


def test_screening_with_shunts(O):
    """Fast decoupled first on the base pattern with opened branches, against
    the oracle's fast decoupled solve of each re-analysed shunted outage."""
    from paper_1811_02512_amd import contingency

    s = staged(500, 2, 72)
    g = s.g
    outs = gridgen.n1_outages(g, 5, 4)
    res = contingency.screen(s.sym, s.r, s.x, s.b, s.type, s.Psp, s.Qsp, s.Vm0, s.Va0, outs,
                             ysh=s.ysh)
    assert res.fallback == 0
    for c, e in enumerate(outs):
        q = g.without_branch(int(e))
        ref = O.solve_grid_fdpf(q)
        assert res.status[c].item() == 0 and ref.status == 0
        assert res.iters[c].item() == ref.iters
        Vm, Va = res.Vm[c].cpu().numpy(), res.Va[c].cpu().numpy()
        np.testing.assert_allclose(Vm, ref.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va, ref.Va, rtol=0, atol=1e-9)
        keep = np.arange(g.m) != e
        for got, want in zip((f[c].cpu().numpy()[keep] for f in res.flows),
                             O.branch_flows(q, Vm, Va)):
            np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
