"""Edge cases of the hot path on the GPU, against the oracle: empty batches,
graphs whose analysis degenerates (a star: no off-diagonal blocks and a
single level; a path: one node per level; a spanning tree: no fill), a grid
whose every non-slack bus is PV, the largest grid of the mixed-size range,
and the full 10k-bus x 256-scenario batch in the launch configuration the
benchmark times, every case checked; the degenerate grids and the largest
one also as one case spread over several workgroups."""
import dataclasses

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


def _rewired(g, f, t, load=1.0):
    """g's first len(f) branch parameters on the topology (f, t), loads and
    generation scaled by `load`."""
    k = len(f)
    return dataclasses.replace(g, f=np.asarray(f, np.int32), t=np.asarray(t, np.int32),
                               r=g.r[:k].copy(), x=g.x[:k].copy(), b=g.b[:k].copy(),
                               Pd=g.Pd * load, Qd=g.Qd * load, Pg=g.Pg * load)


def _spanning_tree(g):
    parent = list(range(g.n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    keep = []
    for e in range(g.m):
        a, b = find(int(g.f[e])), find(int(g.t[e]))
        if a != b:
            parent[a] = b
            keep.append(e)
    keep = np.array(keep)
    return dataclasses.replace(g, f=g.f[keep], t=g.t[keep], r=g.r[keep], x=g.x[keep],
                               b=g.b[keep])


def _topologies():
    g = grid(300, 5)
    n = g.n
    star = _rewired(g, np.zeros(n - 1), np.arange(1, n))
    path = _rewired(grid(80, 6), np.arange(79), np.arange(1, 80), load=0.05)
    tree = _spanning_tree(grid(500, 7))
    allpv = grid(400, 8)
    ty = np.full(allpv.n, gridgen.BUS_PV, np.int8)
    ty[0] = gridgen.BUS_SLACK
    vset = allpv.vset.copy()
    vset[1:] = np.where(allpv.bus_type[1:] == gridgen.BUS_PV, vset[1:], 1.0)
    allpv = dataclasses.replace(allpv, bus_type=ty, vset=vset)
    return {"star": star, "path": path, "tree": tree, "all_pv": allpv}


@pytest.mark.parametrize("tail", [True, False])
@pytest.mark.parametrize("name", ["star", "path", "tree", "all_pv"])
def test_degenerate_structures(O, name, tail):
    """With the LDS tail (which holds the whole of these small grids) and
    without it (every level through the global sweeps)."""
    g = _topologies()[name]
    s = Staged(g)
    if not tail:
        s.sym.set_launch(256, 0)
    info = s.sym.info
    log(f"[edges] {name}: n={g.n} m={g.m} nnz_l={info.nnz_l} levels={info.nlevels} "
        f"tail_nodes={info.tail_nodes}")
    assert (info.tail_nodes > 0) == tail
    if name == "star":
        assert info.nnz_l == 0 and info.nlevels == 1
    if name == "path":
        assert info.nlevels == g.n - 1
    if name == "tree":  # no fill: one block per branch between non-slack buses
        assert info.nnz_l == int(((g.f != 0) & (g.t != 0)).sum())
    ref = O.solve_grid(g)
    assert ref.status == 0
    Vm, Va, iters, _, status, _ = s.newton(3)
    st = status.cpu().numpy()
    assert (st == 0).all()
    assert (iters.cpu().numpy() == ref.iters).all()
    for c in range(3):
        np.testing.assert_allclose(Vm[c].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va[c].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)


@pytest.mark.parametrize("tail", [True, False])
@pytest.mark.parametrize("name", ["star", "path", "tree", "all_pv"])
def test_degenerate_structures_spread(O, name, tail):
    """The same grids as one case over 8 workgroups (cooperative launch):
    with the tail on the first workgroup, and without a tail (a path then
    meets at a grid barrier after each of its one-node levels)."""
    g = _topologies()[name]
    s = Staged(g)
    if not tail:
        s.sym.set_launch(256, 0)
    ref = O.solve_grid(g)
    s.sym.set_spread(8)
    try:
        Vm, Va, iters, _, status, _ = s.newton()
        torch.cuda.synchronize()
    finally:
        s.sym.set_spread(0)
    log(f"[edges] {name} spread over 8: status {status.item()} iters {iters.item()}")
    assert status.item() == 0 and iters.item() == ref.iters
    np.testing.assert_allclose(Vm[0].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Va[0].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)


def test_empty_batch_is_a_no_op():
    """B = 0 is accepted by every batched entry point and touches nothing."""
    from paper_1811_02512_amd import binding as B

    s = Staged(grid(200, 1))
    h, info = s.sym.h, s.info
    n, m = s.g.n, s.g.m
    sentinel = torch.full((1, 64 + 2 * info.nnz_y), 7.0, dtype=torch.float64, device="cuda")
    ws = torch.full((1, info.ws_doubles), 7.0, dtype=torch.float64, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    Vm = torch.full((1, n), 7.0, dtype=torch.float64, device="cuda")
    B.pf_build_ybus(h, 0, s.r, s.x, s.b, 0, sentinel, 2 * info.nnz_y)
    B.pf_mismatch(h, 0, s.yval, 0, s.type, 0, s.Psp, s.Qsp, 0, Vm, Vm, n, ws, info.ws_doubles,
                  ws)
    B.pf_jacobian(h, 0, s.yval, 0, s.type, 0, Vm, Vm, n, ws, info.ws_doubles, 1)
    B.pf_factor(h, 0, ws, info.ws_doubles, st)
    B.pf_solve(h, 0, ws, info.ws_doubles, ws, info.ws_doubles, 0)
    B.pf_newton(h, 0, s.yval, 0, s.type, 0, s.Psp, s.Qsp, 0, Vm, Vm, n, 1e-8, 20, 0, ws,
                info.ws_doubles, st, ws, st)
    B.pf_fdpf_factor(h, 0, ws, info.ws_doubles, st)
    B.pf_branch_flows(h, 0, s.r, s.x, s.b, 0, Vm, Vm, n, ws, ws, ws, ws, m)
    torch.cuda.synchronize()
    assert (sentinel == 7.0).all() and (ws == 7.0).all() and (Vm == 7.0).all()
    assert st.item() == 99


def test_largest_grid_of_the_mixed_range(O):
    """The largest grid of the mixed-size batch (about 20,000 buses)."""
    import json
    import os

    spec = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mixed_batch.json")))
    gs = max(spec["grids"], key=lambda d: d["n"])
    g = gridgen.make_grid(gs["n"], gs["seed"], load_scale=spec["load_scale"])
    s = Staged(g)
    log(f"[edges] largest mixed grid n={g.n} levels={s.info.nlevels} nnz_l={s.info.nnz_l}")
    ref = O.solve_grid(g)
    assert ref.status == 0
    Vm, Va, iters, _, status, _ = s.newton(2)
    assert (status.cpu().numpy() == 0).all() and (iters.cpu().numpy() == ref.iters).all()
    for c in range(2):
        np.testing.assert_allclose(Vm[c].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va[c].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)
    # one case of it spread over 64 workgroups
    s.sym.set_spread(64)
    try:
        Vs, As, its, _, sts, _ = s.newton()
        torch.cuda.synchronize()
    finally:
        s.sym.set_spread(0)
    assert sts.item() == 0 and its.item() == ref.iters
    np.testing.assert_allclose(Vs[0].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(As[0].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)


def test_full_batch_in_the_benchmark_launch(O):
    """10,000 buses x 256 load scenarios with 512-thread workgroups, the
    158 KB LDS tail and groups of four interleaved cases (the benchmark's
    tuned launch), every case against the oracle's sparse NR."""
    from concurrent.futures import ThreadPoolExecutor

    g = grid(10000, 1)
    Bn = 256
    P, Q = gridgen.scenario_injections(g, Bn, 5)
    s = Staged(g)
    from paper_1811_02512_amd import binding as B

    s.sym.set_launch(512, 161792, 4)
    info = s.sym.info
    C = B.pf_newton_interleave(s.sym.h, Bn)
    log(f"[edges] 10k x {Bn}: tail_nodes={info.tail_nodes} lds={info.tail_lds_bytes} "
        f"interleave={C}")
    assert C == 4
    Vm, Va, iters, _, status, _ = s.newton(Bn, dev(P), dev(Q))
    Vm, Va = Vm.cpu().numpy(), Va.cpu().numpy()
    iters, status = iters.cpu().numpy(), status.cpu().numpy()
    assert (status == 0).all()
    Y = O.grid_ybus(g)
    sym = O.Sym(g.n, g.f, g.t)
    Vm0, Va0 = g.flat_start()

    def check(c):
        ref = sym.newton(Y, g.bus_type, P[c], Q[c], Vm0, Va0)
        return (ref.iters == iters[c], np.abs(ref.Vm - Vm[c]).max(), np.abs(ref.Va - Va[c]).max())

    with ThreadPoolExecutor(8) as ex:
        res = list(ex.map(check, range(Bn)))
    assert all(r[0] for r in res)
    worst = max(max(r[1], r[2]) for r in res)
    log(f"[edges] 10k x {Bn}: worst |V|/theta difference {worst:.2e}")
    assert worst < 1e-9
