"""GPU parity of every hot-path step against the CPU oracle, through the C ABI.

Tolerances: |V| and angle within 1e-9 (the path's stated bar); Y, injections
and Jacobian entries are single fp64 sums and products, so 1e-12 relative;
factors of the unpivoted LDU within 1e-10 of the largest entry.
"""
import numpy as np
import pytest

import gridgen
from gpu_helpers import Staged, dev, grid, log

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


def staged(n, seed, ordering=0):
    log(f"[stage] n={n} seed={seed} ordering={ordering}")
    return Staged(grid(n, seed), ordering)


def rand_state(g, seed):
    rng = np.random.default_rng(seed)
    Vm = rng.uniform(0.9, 1.1, g.n)
    Va = rng.uniform(-0.3, 0.3, g.n)
    pv = g.bus_type == gridgen.BUS_PV
    Vm[pv] = g.vset[pv]
    Va[0] = 0.0
    Vm[0] = 1.0
    return Vm, Va


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed", [(200, 1), (2000, 1)])
def test_ybus(O, n, seed):
    s = staged(n, seed)
    Y = O.grid_ybus(s.g)
    yptr, ycol = s.sym.ybus_pattern()
    np.testing.assert_array_equal(yptr, Y.rowptr)
    np.testing.assert_array_equal(ycol, Y.col)
    yv = s.yval[0].cpu().numpy().reshape(-1, 2)
    scale = np.abs(Y.G).max() + np.abs(Y.B).max()
    np.testing.assert_allclose(yv[:, 0], Y.G, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(yv[:, 1], Y.B, rtol=0, atol=1e-12 * scale)


def test_ybus_batched_branch_params(O):
    g = grid(120, 3)
    s = Staged(g)
    rng = np.random.default_rng(0)
    xs = g.x[None, :] * rng.uniform(0.8, 1.2, (3, g.m))
    r = dev(np.repeat(g.r[None], 3, 0))
    b = dev(np.repeat(g.b[None], 3, 0))
    y = s.sym.build_ybus(r, dev(xs), b).cpu().numpy()
    for c in range(3):
        Y = O.ybus(g.n, g.f, g.t, g.r, xs[c], g.b)
        np.testing.assert_allclose(y[c].reshape(-1, 2)[:, 1], Y.B, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,seed", [(200, 2), (2000, 1)])
def test_mismatch(O, n, seed):
    B = _B()
    s = staged(n, seed)
    g = s.g
    Y = O.grid_ybus(g)
    Vm, Va = rand_state(g, 7)
    P, Q = O.injections(Y, Vm, Va)
    FP, FQ, nrm = O.mismatch(g.bus_type, P, Q, g.Psp, g.Qsp)
    nn = s.info.nn
    rhs = torch.zeros(1, 2 * nn, dtype=torch.float64, device="cuda")
    norm = torch.zeros(1, dtype=torch.float64, device="cuda")
    PQ = torch.zeros(1, 2 * g.n, dtype=torch.float64, device="cuda")
    B.pf_mismatch(s.sym.h, 1, s.yval, 0, s.type, 0, s.Psp, s.Qsp, 0, dev(Vm), dev(Va), 0, rhs,
                  2 * nn, norm, PQ)
    pq = PQ.cpu().numpy().reshape(-1, 2)
    scale = np.abs(P).max() + 1.0
    np.testing.assert_allclose(pq[:, 0], P, atol=1e-12 * scale * 10)
    np.testing.assert_allclose(pq[:, 1], Q, atol=1e-12 * scale * 10)
    perm = s.sym.export()["perm"]
    r = rhs.cpu().numpy().reshape(-1, 2)
    np.testing.assert_allclose(r[:, 0], FP[perm], atol=1e-11 * scale)
    np.testing.assert_allclose(r[:, 1], FQ[perm], atol=1e-11 * scale)
    assert norm.item() == pytest.approx(nrm, rel=1e-10)


def jac_gpu(s, Vm, Va):
    B = _B()
    vals = torch.zeros(1, s.info.vals_doubles, dtype=torch.float64, device="cuda")
    B.pf_jacobian(s.sym.h, 1, s.yval, 0, s.type, 0, dev(Vm), dev(Va), 0, vals,
                  s.info.vals_doubles)
    v = vals[0].cpu().numpy()
    nn = s.info.nn
    D = v[:4 * nn].reshape(-1, 2, 2)
    LU = v[s.info.lu_offset:].reshape(-1, 2, 2, 2)
    return D, LU[:, 0], LU[:, 1], vals


@pytest.mark.parametrize("n,seed", [(200, 1), (2000, 2)])
def test_jacobian(O, n, seed):
    s = staged(n, seed)
    g = s.g
    Vm, Va = rand_state(g, 3)
    D, Lo, Up, _ = jac_gpu(s, Vm, Va)
    sym = O.Sym(g.n, g.f, g.t)
    oD, oL, oU = sym.block_jacobian(O.grid_ybus(g), g.bus_type, Vm, Va)
    scale = max(np.abs(oD).max(), np.abs(oL).max())
    np.testing.assert_allclose(D, oD, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(Lo, oL, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(Up, oU, rtol=0, atol=1e-12 * scale)


@pytest.mark.parametrize("n,seed,ordering", [(200, 1, 0), (2000, 1, 0), (300, 4, 1),
                                             (12000, 2, 0)])
def test_factor_and_solve(O, n, seed, ordering):
    """Factors and both solves against the oracle; 12,000 buses puts the
    solve vector beyond LDS (the global-memory variant of the solve)."""
    B = _B()
    s = staged(n, seed, ordering)
    g = s.g
    Vm, Va = rand_state(g, 5)
    sym = O.Sym(g.n, g.f, g.t, 0, ordering)
    oD, oL, oU = sym.block_jacobian(O.grid_ybus(g), g.bus_type, Vm, Va)
    fD, fL, fU, bad = sym.factor(oD, oL, oU)
    assert bad == -1
    # factor the oracle's matrix on the GPU
    nn = s.info.nn
    pad = np.zeros(s.info.lu_offset - 4 * nn)
    vals = torch.from_numpy(np.concatenate([oD.reshape(-1), pad, np.stack([oL, oU], 1).reshape(-1)])
                            ).to("cuda").reshape(1, -1).contiguous()
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    B.pf_factor(s.sym.h, 1, vals, s.info.vals_doubles, status)
    assert status.item() == 0
    v = vals[0].cpu().numpy()
    Dinv = v[:4 * nn].reshape(-1, 2, 2)
    LU = v[s.info.lu_offset:].reshape(-1, 2, 2, 2)
    scale = np.abs(fD).max()
    np.testing.assert_allclose(np.linalg.inv(Dinv), fD, rtol=0, atol=1e-10 * scale)
    # lower factor is stored as L D
    W_expect = np.einsum("qij,qjk->qik", fL, fD[np.repeat(np.arange(nn), np.diff(sym.Lp))])
    np.testing.assert_allclose(LU[:, 0], W_expect, rtol=0, atol=1e-10 * scale)
    np.testing.assert_allclose(LU[:, 1], fU, rtol=0, atol=1e-10 * max(1.0, np.abs(fU).max()))
    # solves: A x = b and A^T x = b against the oracle / LAPACK
    A = sym.dense_matrix(oD, oL, oU) if nn <= 700 else None
    rng = np.random.default_rng(9)
    rhs = rng.standard_normal((2, 2 * nn))
    ox = sym.solve(fD, fL, fU, rhs[0]).reshape(-1)
    r = torch.from_numpy(rhs.copy()).to("cuda")
    B.pf_solve(s.sym.h, 1, vals, s.info.vals_doubles, r[0:1], 2 * nn, 0)
    B.pf_solve(s.sym.h, 1, vals, s.info.vals_doubles, r[1:2], 2 * nn, 1)
    got = r.cpu().numpy()
    xs = np.abs(ox).max()
    np.testing.assert_allclose(got[0], ox, rtol=0, atol=1e-9 * xs)
    oxt = sym.solve_transpose(fD, fL, fU, rhs[1]).reshape(-1)
    np.testing.assert_allclose(got[1], oxt, rtol=0, atol=1e-9 * np.abs(oxt).max())
    if A is not None:
        xt = np.linalg.solve(A.T, rhs[1])
        np.testing.assert_allclose(got[1], xt, rtol=0, atol=1e-9 * np.abs(xt).max())
        np.testing.assert_allclose(got[0], np.linalg.solve(A, rhs[0]), rtol=0, atol=1e-9 * xs)


def test_factor_zero_pivot_status():
    B = _B()
    s = staged(200, 1)
    nn = s.info.nn
    vals = torch.zeros(2, s.info.vals_doubles, dtype=torch.float64, device="cuda")
    vals[:, :4 * nn].view(2, nn, 4)[:, :, 0] = 1.0
    vals[:, :4 * nn].view(2, nn, 4)[:, :, 3] = 1.0
    vals[1, 4 * 5:4 * 5 + 4] = 0.0  # singular diagonal block in case 1
    status = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    B.pf_factor(s.sym.h, 2, vals, s.info.vals_doubles, status)
    assert status.cpu().tolist() == [0, B.PF_E_ZERO_PIVOT]


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed", [(200, 1), (200, 2), (2000, 1), (10000, 1)])
def test_newton_matches_oracle(O, n, seed):
    s = staged(n, seed)
    g = s.g
    ref = O.solve_grid(g)
    assert ref.status == 0
    Vm, Va, iters, norm, status, _ = s.newton()
    torch.cuda.synchronize()
    log(f"[newton] n={n} gpu iters={iters.item()} oracle iters={ref.iters} "
        f"norm={norm.item():.3e}")
    assert status.item() == 0
    assert iters.item() == ref.iters
    np.testing.assert_allclose(Vm[0].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Va[0].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)
    # independent residual check with the oracle's own mismatch code
    P, Q = O.injections(O.grid_ybus(g), Vm[0].cpu().numpy(), Va[0].cpu().numpy())
    _, _, nrm = O.mismatch(g.bus_type, P, Q, g.Psp, g.Qsp)
    assert nrm < 1e-8


def test_newton_natural_order(O):
    s = staged(300, 3, ordering=1)
    ref = O.solve_grid(s.g, ordering=1)
    Vm, Va, iters, _, status, _ = s.newton()
    assert status.item() == 0 and iters.item() == ref.iters
    np.testing.assert_allclose(Vm[0].cpu().numpy(), ref.Vm, atol=1e-9)
    np.testing.assert_allclose(Va[0].cpu().numpy(), ref.Va, atol=1e-9)


def test_newton_batched_scenarios_and_determinism(O):
    s = staged(2000, 1)
    g = s.g
    Bn = 8
    Psp, Qsp = gridgen.scenario_injections(g, Bn, seed=2)
    Vm, Va, iters, norm, status, _ = s.newton(Bn, dev(Psp), dev(Qsp))
    Vm2, Va2, iters2, _, _, _ = s.newton(Bn, dev(Psp), dev(Qsp))
    torch.cuda.synchronize()
    assert torch.equal(Vm, Vm2) and torch.equal(Va, Va2) and torch.equal(iters, iters2)
    Y = O.grid_ybus(g)
    sym = O.Sym(g.n, g.f, g.t)
    Vm0, Va0 = g.flat_start()
    for c in range(Bn):
        ref = sym.newton(Y, g.bus_type, Psp[c], Qsp[c], Vm0, Va0)
        assert status[c].item() == 0 and iters[c].item() == ref.iters
        np.testing.assert_allclose(Vm[c].cpu().numpy(), ref.Vm, atol=1e-9)
        np.testing.assert_allclose(Va[c].cpu().numpy(), ref.Va, atol=1e-9)


def test_newton_status_codes(O):
    s = staged(200, 1)
    g = s.g
    _, _, iters, _, status, _ = s.newton(1, max_iter=1)
    assert status.item() == 6 and iters.item() == 1
    P = g.Psp.copy()
    P[7] = np.nan
    _, _, iters, _, status, _ = s.newton(1, Psp=dev(P))
    assert status.item() == 7 and iters.item() == 0
    # already converged start: zero steps
    ref = O.solve_grid(g)
    Vm = dev(ref.Vm).reshape(1, -1).contiguous()
    Va = dev(ref.Va).reshape(1, -1).contiguous()
    it, nrm, st, _ = s.sym.newton(s.yval[0], s.type, s.Psp, s.Qsp, Vm, Va)
    assert st.item() == 0 and it.item() == 0


def test_two_bus_closed_form():
    from test_oracle_pins import closed_form_pq, two_bus

    g = two_bus(0.02, 0.08, 0.04, 0.9, 0.3)
    s = Staged(g)
    Vm, Va, iters, norm, status, _ = s.newton(1, tol=1e-13, max_iter=30)
    vm, th = closed_form_pq(0.02, 0.08, 0.04, 0.9, 0.3)
    assert status.item() == 0
    assert Vm[0, 1].item() == pytest.approx(vm, abs=1e-12)
    assert Va[0, 1].item() == pytest.approx(th, abs=1e-12)


@pytest.mark.parametrize("threads,budget", [(64, 0), (256, 4096), (512, 65536), (512, 161792),
                                            (128, 20000), (64, 161792)])
def test_launch_shapes_and_lds_tail(O, threads, budget):
    """Every workgroup size and LDS-tail size gives the oracle's solution, and
    the standalone factorisation (which writes the tail back) matches too.
    (64, 161792): more than four tail nodes per thread, so the backward sweep
    keeps its vector in global memory."""
    B = _B()
    s = staged(2000, 2)
    g = s.g
    s.sym.set_launch(threads, budget)
    info = s.sym.info
    log(f"[launch] threads={threads} budget={budget} tail_levels={info.tail_levels} "
        f"tail_nodes={info.tail_nodes} lds={info.tail_lds_bytes}")
    ref = O.solve_grid(g)
    Vm, Va, iters, _, status, _ = s.newton(2)
    assert (status.cpu().numpy() == 0).all()
    assert (iters.cpu().numpy() == ref.iters).all()
    np.testing.assert_allclose(Vm[1].cpu().numpy(), ref.Vm, atol=1e-9)
    np.testing.assert_allclose(Va[1].cpu().numpy(), ref.Va, atol=1e-9)
    Vm_, Va_ = rand_state(g, 5)
    _, _, _, vals = jac_gpu(s, Vm_, Va_)
    sym = O.Sym(g.n, g.f, g.t)
    oD, oL, oU = sym.block_jacobian(O.grid_ybus(g), g.bus_type, Vm_, Va_)
    fD, fL, fU, _ = sym.factor(oD, oL, oU)
    B.pf_factor(s.sym.h, 1, vals, info.vals_doubles, None)
    v = vals[0].cpu().numpy()
    nn = info.nn
    np.testing.assert_allclose(v[info.lu_offset:].reshape(-1, 2, 2, 2)[:, 1], fU, rtol=0,
                               atol=1e-10 * max(1.0, np.abs(fU).max()))
    np.testing.assert_allclose(np.linalg.inv(v[:4 * nn].reshape(-1, 2, 2)), fD, rtol=0,
                               atol=1e-10 * np.abs(fD).max())


@pytest.mark.parametrize("C", [1, 2, 8])
def test_interleaved_case_groups_bitwise_equal(C):
    """The workspace grouping (1, 2, 4 or 8 cases per 64-byte-interleaved
    group, groups spread over the XCDs) changes addresses only: results are
    bitwise those of the default grouping, for a batch that is not a
    multiple of the group size."""
    s = staged(2000, 3)
    g = s.g
    Bn = 7
    P, Q = gridgen.scenario_injections(g, Bn, seed=11)
    ref = s.newton(Bn, dev(P), dev(Q))
    s.sym.set_launch(0, 65536, C)
    assert s.sym.info.ws_interleave == C
    got = s.newton(Bn, dev(P), dev(Q))
    s.sym.set_launch(0, 65536, 4)
    for a, b in zip(ref[:5], got[:5]):
        assert torch.equal(a, b)


def test_factor_solve_interleaved_vals():
    B = _B()
    s = staged(300, 5)
    g = s.g
    nn = s.info.nn
    vd = s.info.vals_doubles
    Bn, C = 5, 4
    rows = -(-Bn // C) * C
    rng = np.random.default_rng(3)
    plain = torch.zeros(Bn, vd, dtype=torch.float64, device="cuda")
    inter = torch.zeros(rows, vd, dtype=torch.float64, device="cuda")
    states = [rand_state(g, 20 + c) for c in range(Bn)]
    Vm = dev(np.stack([v for v, _ in states]))
    Va = dev(np.stack([a for _, a in states]))
    B.pf_jacobian(s.sym.h, Bn, s.yval, 0, s.type, 0, Vm, Va, g.n, plain, vd, 1)
    B.pf_jacobian(s.sym.h, Bn, s.yval, 0, s.type, 0, Vm, Va, g.n, inter, vd, C)
    B.pf_factor(s.sym.h, Bn, plain, vd, None, 1)
    B.pf_factor(s.sym.h, Bn, inter, vd, None, C)
    rhs = rng.standard_normal((Bn, 2 * nn))
    r1 = dev(rhs.copy())
    r2 = dev(rhs.copy())
    B.pf_solve(s.sym.h, Bn, plain, vd, r1, 2 * nn, 1, 1)
    B.pf_solve(s.sym.h, Bn, inter, vd, r2, 2 * nn, 1, C)
    assert torch.equal(r1, r2)
    # the interleaved buffer holds the same numbers, just regrouped
    v = inter.view(rows // C, vd // 8, C, 8).permute(0, 2, 1, 3).reshape(rows, vd)[:Bn]
    assert torch.equal(v, plain)
