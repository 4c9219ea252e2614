"""N-1 screening on the base pattern (fast decoupled first, Newton-Raphson
fallback, branch flows) against the oracle on re-analysed outage grids."""
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


def _screen(s, outages, **kw):
    from paper_1811_02512_amd import contingency

    return contingency.screen(s.sym, s.r, s.x, s.b, s.type, s.Psp, s.Qsp, s.Vm0, s.Va0,
                              outages, **kw)


@pytest.mark.parametrize("fdpf_first", [True, False])
def test_screening_matches_reanalysed_outages(fdpf_first):
    from oracle import oracle as O

    g = grid(2000, 1)
    s = Staged(g)
    outages = gridgen.n1_outages(g, 12, seed=5)
    log(f"[n1 screen] fdpf_first={fdpf_first} outages {outages.tolist()}")
    res = _screen(s, outages, fdpf_first=fdpf_first)
    assert res.fallback == (0 if fdpf_first else len(outages))
    st = res.status.cpu().numpy()
    meth = res.method.cpu().numpy()
    its = res.iters.cpu().numpy()
    for c, e in enumerate(outages):
        ge = g.without_branch(int(e))
        ref = O.solve_grid_fdpf(ge) if fdpf_first else O.solve_grid(ge)
        assert ref.status == 0 and st[c] == 0, (c, st[c])
        assert meth[c] == (1 if fdpf_first else 2)
        assert its[c] == ref.iters, (c, its[c], ref.iters)
        np.testing.assert_allclose(res.Vm[c].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(res.Va[c].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)
        # the opened branch carries nothing; the others match the oracle's flows
        Pft, Qft, Ptf, Qtf = (f[c].cpu().numpy() for f in res.flows)
        assert Pft[e] == 0.0 and Qft[e] == 0.0 and Ptf[e] == 0.0 and Qtf[e] == 0.0
        keep = np.arange(g.m) != e
        oP, oQ, oP2, oQ2 = O.branch_flows(ge, res.Vm[c].cpu().numpy(), res.Va[c].cpu().numpy())
        np.testing.assert_allclose(Pft[keep], oP, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(Qft[keep], oQ, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(Ptf[keep], oP2, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(Qtf[keep], oQ2, rtol=1e-12, atol=1e-12)


def test_screening_falls_back_to_newton():
    """Cases the fast decoupled iteration leaves unconverged go to NR."""
    from oracle import oracle as O

    g = grid(500, 2)
    s = Staged(g)
    outages = gridgen.n1_outages(g, 6, seed=1)
    res = _screen(s, outages, fdpf_iter=1)
    assert res.fallback == len(outages)
    for c, e in enumerate(outages):
        ref = O.solve_grid(g.without_branch(int(e)))
        assert res.status[c].item() == 0 and res.method[c].item() == 2
        assert res.iters[c].item() == ref.iters
        np.testing.assert_allclose(res.Vm[c].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
