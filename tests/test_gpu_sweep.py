"""A sweep of grid sizes between the fixed cases of the other tests (37 to
7,777 buses, seeded), each solved for several load scenarios in three
launch configurations and compared case by case with the oracle's sparse
NR on the same inputs: the default launch (one workgroup per case, groups
of four cases, the last group ragged), a small LDS tail with groups of two,
and one case spread over 16 workgroups."""
import numpy as np
import pytest

import gridgen
from gpu_helpers import Staged, dev, grid, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = [(37, 11), (101, 12), (555, 13), (1234, 14), (3333, 15), (7777, 16)]


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle(g, P, Q):
    from oracle import oracle as O

    Y = O.grid_ybus(g)
    osym = O.Sym(g.n, g.f, g.t)
    Vm0, Va0 = g.flat_start()
    return [osym.newton(Y, g.bus_type, P[c], Q[c], Vm0, Va0) for c in range(len(P))]


def _check(refs, Vm, Va, iters, status, cases):
    st, it = status.cpu().numpy(), iters.cpu().numpy()
    for k, c in enumerate(cases):
        r = refs[c]
        assert r.status == 0 and st[k] == 0 and it[k] == r.iters, (c, st[k], it[k], r.iters)
        np.testing.assert_allclose(Vm[k].cpu().numpy(), r.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va[k].cpu().numpy(), r.Va, rtol=0, atol=1e-9)


@pytest.mark.parametrize("n,seed", SIZES)
def test_sizes_scenarios_and_launches(n, seed):
    g = grid(n, seed)
    Bn = 5
    P, Q = gridgen.scenario_injections(g, Bn, seed + 100)
    refs = _oracle(g, P, Q)
    s = Staged(g)
    log(f"[sweep] n={n} seed={seed} levels={s.info.nlevels} tail={s.info.tail_nodes} "
        f"oracle iters={[r.iters for r in refs]}")
    Pt, Qt = dev(P), dev(Q)
    # default launch: groups of four cases, the second group holds one
    Vm, Va, iters, _, status, _ = s.newton(Bn, Pt, Qt)
    torch.cuda.synchronize()
    _check(refs, Vm, Va, iters, status, range(Bn))
    # a small LDS tail and groups of two cases
    s.sym.set_launch(256, 32768, 2)
    s.sym.upload()
    Vm, Va, iters, _, status, _ = s.newton(Bn, Pt, Qt)
    torch.cuda.synchronize()
    _check(refs, Vm, Va, iters, status, range(Bn))
    # one case over 16 workgroups
    s.sym.set_launch(512, 161792, 4)
    s.sym.upload()
    s.sym.set_spread(16)
    try:
        Vm, Va, iters, _, status, _ = s.newton(1, Pt[2:3].contiguous(), Qt[2:3].contiguous())
        torch.cuda.synchronize()
    finally:
        s.sym.set_spread(0)
    _check(refs, Vm, Va, iters, status, [2])
