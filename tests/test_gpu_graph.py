"""The batched Newton launch captured in a HIP graph: every replay (with
eager work and synchronisations between replays) equals the eager result."""
import numpy as np
import pytest

import gridgen
from gpu_helpers import Staged, dev, grid

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_graph_replays_match_eager():
    from paper_1811_02512_amd import binding as B

    s = Staged(grid(2000, 1))
    g = s.g
    Bn = 16
    P, Q = gridgen.scenario_injections(g, Bn, seed=2)
    P, Q = dev(P), dev(Q)
    info = s.info
    Vm_in = s.Vm0.repeat(Bn, 1).contiguous()
    Va_in = s.Va0.repeat(Bn, 1).contiguous()
    Vm, Va = Vm_in.clone(), Va_in.clone()
    ws = s.sym.workspace(Bn)
    it = torch.empty(Bn, dtype=torch.int32, device="cuda")
    nrm = torch.empty(Bn, dtype=torch.float64, device="cuda")
    st = torch.empty(Bn, dtype=torch.int32, device="cuda")

    def launch():
        B.pf_newton(s.sym.h, Bn, s.yval, 0, s.type, 0, P, Q, g.n, Vm, Va, g.n, 1e-8, 20, 0, ws,
                    info.ws_doubles, it, nrm, st)

    launch()
    torch.cuda.synchronize()
    Vm_e, Va_e, it_e = Vm.clone(), Va.clone(), it.clone()
    assert (st == 0).all()

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        Vm.copy_(Vm_in)
        Va.copy_(Va_in)
        launch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        launch()
    for rep in range(4):
        Vm.copy_(Vm_in)
        Va.copy_(Va_in)
        it.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(Vm, Vm_e), rep
        assert torch.equal(Va, Va_e), rep
        assert torch.equal(it, it_e), rep
        junk = torch.randn(4096, device="cuda").cumsum(0)  # eager work between replays
        torch.cuda.synchronize()
        del junk
