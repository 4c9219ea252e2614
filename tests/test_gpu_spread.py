"""One case spread over many workgroups (Sec. III's nodal parallelism across
the whole device for a single Newton-Raphson solve): a cooperative launch
shares the loops over buses and the levels below the LDS tail among its
workgroups, which meet at grid barriers, and runs the tail on the first.
Checked against the oracle and against the one-workgroup launch: solutions,
iteration counts, the kept factors, without a tail, with more workgroups
than the device holds at once, the failure statuses (zero pivot with its
position, non-finite input, iteration limit), repeated calls, and a launch
recorded into a graph (which takes the one-workgroup kernel)."""
import numpy as np
import pytest

from gpu_helpers import Staged, grid, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _B():
    from paper_1811_02512_amd import binding

    return binding


def solve(s, spread, keep=False, Psp=None, Qsp=None, max_iter=20):
    """One case through pf_newton with the given spread; returns
    (Vm, Va, iters, norm, status, pivot, ws)."""
    B = _B()
    s.sym.set_spread(spread)
    g, info = s.g, s.info
    Vm, Va = s.Vm0.clone()[None], s.Va0.clone()[None]
    ws = s.sym.workspace(1)
    out = [torch.full((1,), -9, dtype=torch.int32, device="cuda"),
           torch.full((1,), -9.0, dtype=torch.float64, device="cuda"),
           torch.full((1,), -9, dtype=torch.int32, device="cuda"),
           torch.full((1,), -9, dtype=torch.int32, device="cuda")]
    B.pf_newton(s.sym.h, 1, s.yval, 0, s.type, 0, s.Psp if Psp is None else Psp,
                s.Qsp if Qsp is None else Qsp, 0, Vm, Va, g.n, 1e-8, max_iter,
                B.PF_NEWTON_KEEP_FACTORS if keep else 0, ws, info.ws_doubles, *out)
    torch.cuda.synchronize()
    s.sym.set_spread(0)
    it, nrm, st, pv = (t.item() for t in out)
    return Vm[0], Va[0], it, nrm, st, pv, ws


@pytest.mark.parametrize("n,seed,spread", [(200, 1, 16), (2000, 2, 64), (2000, 2, 256),
                                           (10000, 1, 128)])
def test_spread_matches_oracle_and_one_workgroup(O, n, seed, spread):
    s = Staged(grid(n, seed))
    log(f"[spread] n={n} seed={seed} spread={spread} tail levels={s.info.tail_levels}")
    ref = O.solve_grid(s.g)
    assert ref.status == 0
    Vm, Va, it, nrm, st, pv, _ = solve(s, spread)
    Vm1, Va1, it1, _, st1, _, _ = solve(s, 0)
    log(f"[spread] iters {it} (oracle {ref.iters}), norm {nrm:.3e}")
    assert st == 0 and st1 == 0 and pv == -1
    assert it == ref.iters == it1 and nrm < 1e-8
    np.testing.assert_allclose(Vm.cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Va.cpu().numpy(), ref.Va, rtol=0, atol=1e-9)
    # the same arithmetic per node as one workgroup, to rounding
    assert (Vm - Vm1).abs().max().item() < 1e-12
    assert (Va - Va1).abs().max().item() < 1e-12


@pytest.fixture(scope="module")
def O():
    from oracle import oracle

    return oracle


def test_spread_is_deterministic_and_keeps_the_factors():
    """Two spread calls give the same bits; the factors kept at the solution
    equal the one-workgroup launch's to rounding, and solve the same system."""
    B = _B()
    s = Staged(grid(2000, 3))
    info = s.info
    a = solve(s, 64, keep=True)
    b = solve(s, 64, keep=True)
    one = solve(s, 0, keep=True)
    assert a[4] == b[4] == one[4] == 0
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])

    def factors(r):  # D^-1 of every position, then the slot records (not the padding)
        w = r[6][0]
        return torch.cat([w[:4 * info.nn], w[info.lu_offset:info.vals_doubles]])

    assert torch.equal(factors(a), factors(b))
    fa, fo = factors(a), factors(one)
    scale = fo.abs().max().item()
    assert (fa - fo).abs().max().item() <= 1e-11 * scale
    rhs = torch.linspace(-1.0, 1.0, 2 * info.nn, dtype=torch.float64, device="cuda")[None]
    xa, xo = rhs.clone(), rhs.clone()
    B.pf_solve(s.sym.h, 1, a[6], info.ws_doubles, xa, 2 * info.nn, 0)
    B.pf_solve(s.sym.h, 1, one[6], info.ws_doubles, xo, 2 * info.nn, 0)
    torch.cuda.synchronize()
    assert (xa - xo).abs().max().item() <= 1e-9 * xo.abs().max().item()


def test_spread_without_tail_and_beyond_the_device(O):
    """No LDS tail (every level shared out), and a workgroup count above what
    the device keeps resident (capped)."""
    s = Staged(grid(2000, 4))
    ref = O.solve_grid(s.g)
    s.sym.set_launch(512, 0, 4)
    s.sym.upload()
    assert s.sym.info.tail_levels == 0
    Vm, Va, it, _, st, _, _ = solve(s, 48)
    assert st == 0 and it == ref.iters
    np.testing.assert_allclose(Vm.cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Va.cpu().numpy(), ref.Va, rtol=0, atol=1e-9)
    s.sym.set_launch(512, 161792, 4)
    s.sym.upload()
    Vm, Va, it, _, st, _, _ = solve(s, 1024)
    assert st == 0 and it == ref.iters
    np.testing.assert_allclose(Vm.cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)


def test_spread_failure_statuses():
    """The statuses and pivot position of the one-workgroup launch: a zero
    pivot at a leaf of the shared levels and one in the tail, a NaN
    injection, the iteration limit."""
    import test_gpu_failures as F
    from oracle import oracle as O

    B = _B()
    g = grid(2000, 3)
    s0 = Staged(g)
    ex = s0.sym.export()
    leaves, tail, _ = F.regions(s0.info, ex)
    osym = O.Sym(g.n, g.f, g.t)
    for region in (leaves, tail):
        q, p = F.pick(O, g, region, ex["perm"], osym)
        s = Staged(q)
        r = solve(s, 32)
        log(f"[spread] zero pivot at position {p}: status {r[4]} pivot {r[5]}")
        assert r[4] == B.PF_E_ZERO_PIVOT and r[5] == p and r[2] == 0
    P = s0.Psp.clone()
    P[5] = float("nan")
    r = solve(s0, 32, Psp=P)
    assert r[4] == B.PF_E_NONFINITE and r[2] == 0
    r = solve(s0, 32, max_iter=1)
    r1 = solve(s0, 0, max_iter=1)
    assert r[4] == r1[4] == B.PF_E_NOT_CONVERGED and r[2] == r1[2] == 1
    assert abs(r[3] - r1[3]) <= 1e-9 * r1[3]


def test_spread_under_graph_capture_takes_one_workgroup():
    """A one-case launch recorded into a graph uses the one-workgroup kernel:
    every replay equals that kernel's eager result bit for bit."""
    B = _B()
    s = Staged(grid(2000, 1))
    g, info = s.g, s.info
    Vm1, Va1, it1, _, st1, _, _ = solve(s, 0)
    assert st1 == 0
    Vm, Va = s.Vm0.clone()[None], s.Va0.clone()[None]
    ws = s.sym.workspace(1)
    it = torch.empty(1, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    s.sym.set_spread(64)

    def launch():
        B.pf_newton(s.sym.h, 1, s.yval, 0, s.type, 0, s.Psp, s.Qsp, 0, Vm, Va, g.n, 1e-8, 20, 0,
                    ws, info.ws_doubles, it, None, st)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        launch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        launch()
    s.sym.set_spread(0)
    for rep in range(3):
        Vm.copy_(s.Vm0[None])
        Va.copy_(s.Va0[None])
        it.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert st.item() == 0 and it.item() == it1, rep
        assert torch.equal(Vm[0], Vm1) and torch.equal(Va[0], Va1), rep


def test_spread_gives_up_when_a_barrier_wait_runs_out():
    """With a wait limit of zero ticks the first workgroup that has to wait at
    a grid barrier gives up: no workgroup waits from then on, every one runs
    to its end and the case reports PF_E_HIP.  The next launch with the
    normal limit is whole again."""
    B = _B()
    s = Staged(grid(2000, 1))
    B.pf_symbolic_set_spread_wait(s.sym.h, 0)
    try:
        r = solve(s, 32)
    finally:
        B.pf_symbolic_set_spread_wait(s.sym.h, 100_000_000)
    log(f"[spread] zero wait limit: status {r[4]}")
    assert r[4] == B.PF_E_HIP
    good = solve(s, 32)
    one = solve(s, 0)
    assert good[4] == 0 and one[4] == 0 and good[2] == one[2]
    assert (good[0] - one[0]).abs().max().item() < 1e-12


def test_noalloc_takes_the_spread_launch_too():
    """pf_newton_noalloc with a spread setting: its barrier words sit in the
    library's scratch array; results equal pf_newton's spread launch."""
    B = _B()
    s = Staged(grid(2000, 2))
    g = s.g
    ref = solve(s, 32)
    s.sym.set_spread(32)
    Vm, Va = s.Vm0.clone()[None], s.Va0.clone()[None]
    it = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    st = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    try:
        B.pf_newton_noalloc(s.sym.h, 1, s.yval, 0, s.type, 0, s.Psp, s.Qsp, 0, Vm, Va, g.n,
                            1e-8, 20, it, None, st)
        torch.cuda.synchronize()
    finally:
        s.sym.set_spread(0)
    assert st.item() == 0 and it.item() == ref[2]
    assert torch.equal(Vm[0], ref[0]) and torch.equal(Va[0], ref[1])
