"""pf_newton_noalloc (the workspace in the library's own device scratch array,
for callers that cannot allocate) against pf_newton on the same inputs: two
calls in a row, the second on a smaller grid and batch, each bitwise equal to
pf_newton and within 1e-9 of the oracle with the same iteration counts; a
batch too large for the array is refused before any launch."""
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


def _both(s, Bn, P, Q):
    """(pf_newton outputs, pf_newton_noalloc outputs) for the same batch."""
    from paper_1811_02512_amd import binding as B

    g = s.g
    outs = []
    for noalloc in (False, True):
        Vm = s.Vm0.repeat(Bn, 1).contiguous()
        Va = s.Va0.repeat(Bn, 1).contiguous()
        it = torch.full((Bn,), -2, dtype=torch.int32, device="cuda")
        nrm = torch.full((Bn,), -2.0, dtype=torch.float64, device="cuda")
        st = torch.full((Bn,), -2, dtype=torch.int32, device="cuda")
        pv = torch.full((Bn,), -2, dtype=torch.int32, device="cuda")
        if noalloc:
            B.pf_newton_noalloc(s.sym.h, Bn, s.yval, 0, s.type, 0, P, Q, g.n, Vm, Va, g.n,
                                1e-8, 20, it, nrm, st, pv)
        else:
            ws = s.sym.workspace(Bn)
            B.pf_newton(s.sym.h, Bn, s.yval, 0, s.type, 0, P, Q, g.n, Vm, Va, g.n, 1e-8, 20, 0,
                        ws, s.info.ws_doubles, it, nrm, st, pv)
        torch.cuda.synchronize()
        outs.append((Vm, Va, it, nrm, st, pv))
    return outs


def _check(O, g, P, Q, ref, got):
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    Vm, Va, it, _, st, pv = got
    assert (st == 0).all() and (pv == -1).all()
    osym = O.Sym(g.n, g.f, g.t)
    Y = O.grid_ybus(g)
    for c in range(P.shape[0]):
        r = osym.newton(Y, g.bus_type, P[c], Q[c], *g.flat_start())
        assert r.status == 0 and it[c].item() == r.iters
        np.testing.assert_allclose(Vm[c].cpu().numpy(), r.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va[c].cpu().numpy(), r.Va, rtol=0, atol=1e-9)


def test_noalloc_matches_pf_newton_twice():
    from oracle import oracle as O

    g1 = grid(2000, 1)
    s1 = Staged(g1)
    P1, Q1 = gridgen.scenario_injections(g1, 12, 7)
    log("[noalloc] call 1: 2,000 buses x 12 cases")
    ref, got = _both(s1, 12, dev(P1), dev(Q1))
    _check(O, g1, P1, Q1, ref, got)
    g2 = grid(200, 2)
    s2 = Staged(g2)
    P2, Q2 = gridgen.scenario_injections(g2, 3, 8)
    log("[noalloc] call 2: 200 buses x 3 cases")
    ref, got = _both(s2, 3, dev(P2), dev(Q2))
    _check(O, g2, P2, Q2, ref, got)


def test_noalloc_refuses_a_batch_beyond_the_array():
    from paper_1811_02512_amd import binding as B

    g = grid(2000, 1)
    s = Staged(g)
    Bn = B.PF_NOALLOC_SCRATCH_BYTES // (8 * s.info.ws_doubles) + 8
    Vm = s.Vm0.repeat(Bn, 1).contiguous()
    Va = s.Va0.repeat(Bn, 1).contiguous()
    with pytest.raises(B.PfError) as ei:
        B.pf_newton_noalloc(s.sym.h, Bn, s.yval, 0, s.type, 0, s.Psp, s.Qsp, 0, Vm, Va, g.n,
                            1e-8, 20)
    assert ei.value.code == B.PF_E_WORKSPACE and "scratch" in B.last_error()
    B.pf_newton_noalloc(s.sym.h, 0, s.yval, 0, s.type, 0, s.Psp, s.Qsp, 0, Vm, Va, g.n, 1e-8, 20)
