"""Parity at the benchmark's full sizes and launch shapes: the adjoint of
10,000 buses x 256 scenarios in the tuned launch (every case against the
oracle's sparse adjoint, and central differences on the 10k grid), every
case of 2,000 buses x 1,024 scenarios in the tuned launch, the full launch of
the 64 mixed grids (one workgroup per grid and 256 workgroups), and the 512
re-analysed N-1 outages of the 10k grid
(a seeded quarter of them against the oracle)."""
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gridgen
from gpu_helpers import Staged, dev, grid, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
THREADS = 8


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def tuned(s, P, Q, threads, budget, interleave):
    """The benchmark's launch shape with the per-level mapping from the
    autotuner (mapping search only)."""
    from paper_1811_02512_amd import autotune

    Bn = P.shape[0]
    V0 = s.Vm0.repeat(Bn, 1).contiguous()
    A0 = s.Va0.repeat(Bn, 1).contiguous()
    res = autotune.tune(s.sym, s.yval[0], s.type, P, Q, V0, A0, reps=1, threads=(threads,),
                        budgets=(budget,), interleaves=(interleave,), passes=1)
    log(f"[full] tuned mapping {res['mapping']} ({res['ms']:.3f} ms)")
    return res


def test_adjoint_full_batch_in_the_benchmark_launch():
    from oracle import oracle as O

    from paper_1811_02512_amd import binding as B

    g = grid(10000, 1)
    Bn = 256
    P, Q = gridgen.scenario_injections(g, Bn, 5)
    w = np.random.default_rng(6).uniform(0, 1, g.n)
    s = Staged(g)
    Pt, Qt = dev(P), dev(Q)
    tuned(s, Pt, Qt, 512, 161792, 4)
    info = s.info
    log(f"[full] 10k x 256: tail {info.tail_nodes} nodes, {info.tail_lds_bytes} bytes of LDS")
    assert B.pf_newton_interleave(s.sym.h, Bn) == 4 and info.tail_nodes > 0
    Vm, Va, it, _, st, ws = s.newton(Bn, Pt, Qt, keep=True)
    assert (st == 0).all()
    n, nn = g.n, info.nn
    pq = dev((g.bus_type == gridgen.BUS_PQ).astype(np.float64))
    gVm = (2.0 * dev(w) * pq * (Vm - 1.0)).contiguous()
    f64 = dict(dtype=torch.float64, device="cuda")
    lam = torch.empty(Bn, 2 * nn, **f64)
    gP, gQ, gx = torch.empty(Bn, n, **f64), torch.empty(Bn, n, **f64), torch.empty(g.m, **f64)
    B.pf_adjoint(s.sym.h, Bn, ws, info.ws_doubles, gVm, None, n, s.type, 0, Vm, Va, n, s.r,
                 s.x, 0, st, lam, 2 * nn, gP, gQ, n, gx, 1)
    Vm, Va = Vm.cpu().numpy(), Va.cpu().numpy()
    gP, gQ, gx = gP.cpu().numpy(), gQ.cpu().numpy(), gx.cpu().numpy()
    osym = O.Sym(g.n, g.f, g.t)
    Y = O.grid_ybus(g)

    def one(c):
        gv = 2 * w * (Vm[c] - 1) * (g.bus_type == gridgen.BUS_PQ)
        oP, oQ, ox = osym.adjoint(g, Y, Vm[c], Va[c], gv, np.zeros(n))
        sc = max(np.abs(oP).max(), np.abs(oQ).max())
        return max(np.abs(oP - gP[c]).max(), np.abs(oQ - gQ[c]).max()) / sc, ox

    with ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(one, range(Bn)))
    worst = max(r[0] for r in res)
    ox = np.sum([r[1] for r in res], axis=0)
    log(f"[full] 10k x 256 adjoint: worst relative |dgP|, |dgQ| {worst:.2e}")
    assert worst < 1e-8
    np.testing.assert_allclose(gx, ox, rtol=0, atol=1e-8 * np.abs(ox).max())
    # the solutions themselves, on a seeded subset
    for c in np.random.default_rng(1).choice(Bn, 8, replace=False):
        r = osym.newton(Y, g.bus_type, P[c], Q[c], *g.flat_start())
        assert r.iters == it[c].item()
        np.testing.assert_allclose(Vm[c], r.Vm, rtol=0, atol=1e-9)


def test_adjoint_central_differences_on_the_10k_grid():
    """Central differences (h = 1e-6) of the GPU solve, converged to 1e-12,
    at a few injections and reactances of the 10k grid."""
    from paper_1811_02512_amd.autograd import power_flow
    from paper_1811_02512_amd import api

    g = grid(10000, 1)
    sym = api.Symbolic(g.n, g.f, g.t).upload()
    w = np.random.default_rng(6).uniform(0, 1, g.n)
    Vm0, Va0 = g.flat_start()
    cst = dict(r=dev(g.r), b=dev(g.b), bus_type=dev(g.bus_type.astype(np.int8)),
               Vm0=dev(Vm0), Va0=dev(Va0))
    pq = dev((g.bus_type == gridgen.BUS_PQ).astype(np.float64))
    wt = dev(w)

    def run(P, Q, x, grad=False):
        Pt = dev(P[None]).requires_grad_(grad)
        Qt = dev(Q[None]).requires_grad_(grad)
        xt = dev(x).requires_grad_(grad)
        Vm, _, st, _ = power_flow(sym, Pt, Qt, xt, cst["r"], cst["b"], cst["bus_type"],
                                  cst["Vm0"], cst["Va0"], tol=1e-12, max_iter=40,
                                  with_status=True)
        assert st.item() == 0
        loss = (wt * pq * (Vm - 1.0) ** 2).sum()
        if grad:
            loss.backward()
            return Pt.grad[0].cpu().numpy(), Qt.grad[0].cpu().numpy(), xt.grad.cpu().numpy()
        return loss.item()

    gP, gQ, gx = run(g.Psp, g.Qsp, g.x, grad=True)
    h = 1e-6
    rng = np.random.default_rng(9)
    buses = rng.choice(np.flatnonzero(g.bus_type == gridgen.BUS_PQ), 3, replace=False)
    for i in buses:
        e = np.zeros(g.n)
        e[i] = h
        fd = (run(g.Psp + e, g.Qsp, g.x) - run(g.Psp - e, g.Qsp, g.x)) / (2 * h)
        assert abs(gP[i] - fd) <= 1e-5 * np.abs(gP).max(), (i, gP[i], fd)
        fd = (run(g.Psp, g.Qsp + e, g.x) - run(g.Psp, g.Qsp - e, g.x)) / (2 * h)
        assert abs(gQ[i] - fd) <= 1e-5 * np.abs(gQ).max(), (i, gQ[i], fd)
    for k in rng.choice(g.m, 3, replace=False):
        e = np.zeros(g.m)
        e[k] = h
        fd = (run(g.Psp, g.Qsp, g.x + e) - run(g.Psp, g.Qsp, g.x - e)) / (2 * h)
        assert abs(gx[k] - fd) <= 1e-5 * np.abs(gx).max(), (k, gx[k], fd)


def test_every_case_of_2k_x1024_in_the_tuned_launch():
    from oracle import oracle as O

    g = grid(2000, 1)
    Bn = 1024
    P, Q = gridgen.scenario_injections(g, Bn, 2)
    s = Staged(g)
    Pt, Qt = dev(P), dev(Q)
    tuned(s, Pt, Qt, 256, 65536, 4)
    Vm, Va, it, _, st, _ = s.newton(Bn, Pt, Qt)
    assert (st == 0).all()
    Vm, Va, it = Vm.cpu().numpy(), Va.cpu().numpy(), it.cpu().numpy()
    osym = O.Sym(g.n, g.f, g.t)
    Y = O.grid_ybus(g)

    def one(c):
        r = osym.newton(Y, g.bus_type, P[c], Q[c], *g.flat_start())
        return r.iters == it[c], max(np.abs(r.Vm - Vm[c]).max(), np.abs(r.Va - Va[c]).max())

    with ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(one, range(Bn)))
    assert all(r[0] for r in res)
    worst = max(r[1] for r in res)
    log(f"[full] 2k x 1024: worst |V|/theta difference {worst:.2e}")
    assert worst < 1e-9


def _solve_multi(grids, budget=161792, spread=0):
    from test_gpu_batch import solve_multi

    return solve_multi(grids, tail_budget=budget, spread=spread)


def _check_all(grids, Vms, Vas, it, st, idx):
    from oracle import oracle as O

    def one(c):
        r = O.solve_grid(grids[c])
        return (r.status == 0 and st[c] == 0 and r.iters == it[c],
                max(np.abs(r.Vm - Vms[c]).max(), np.abs(r.Va - Vas[c]).max()))

    with ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(one, idx))
    assert all(r[0] for r in res)
    return max(r[1] for r in res)


@pytest.mark.parametrize("spread", [0, 256])
def test_full_launch_of_the_64_mixed_grids(spread):
    """Every grid of the 64-grid launch against the oracle, with one workgroup
    per grid and with the benchmark's 256 workgroups (the largest grids in
    groups)."""
    spec = json.load(open(os.path.join(ROOT, "tests", "golden", "mixed_batch.json")))
    jobs = [(x["n"], x["seed"], spec["load_scale"]) for x in spec["grids"]]
    grids = gridgen.make_grids(jobs, processes=THREADS)
    log(f"[full] mixed: {len(grids)} grids, {sum(q.n for q in grids)} buses, "
        f"{spread or len(grids)} workgroups")
    Vms, Vas, it, st, _ = _solve_multi(grids, spread=spread)
    worst = _check_all(grids, Vms, Vas, it, st, range(len(grids)))
    log(f"[full] mixed 64: worst |V|/theta difference {worst:.2e}")
    assert worst < 1e-9


def test_n1_10k_x512_full_launch():
    g = grid(10000, 1)
    outs = gridgen.n1_outages(g, 512, 3)
    grids = [g.without_branch(int(e)) for e in outs]
    Vms, Vas, it, st, _ = _solve_multi(grids)
    assert (st == 0).all()
    idx = sorted(np.random.default_rng(23).choice(512, 128, replace=False).tolist())
    worst = _check_all(grids, Vms, Vas, it, st, idx)
    log(f"[full] N-1 10k x 512 (128 checked): worst |V|/theta difference {worst:.2e}")
    assert worst < 1e-9
