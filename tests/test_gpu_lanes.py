"""Every lanes-per-node setting against the CPU oracle.

A node's lanes combine their partial sums with a butterfly whose partners
come from DPP moves (groups up to 16 lanes), a swizzle (32) and a permute
(64).  The autotuner picks per-level lane counts that ordinary grids may never
reach (64 lanes needs a node with more than 32 destinations), so each count is
forced here on every level: Newton with the LDS tail and without it, the fast
decoupled iteration, and both solves on the oracle's factors.  Results must
match the oracle (|V|, angle within 1e-9, equal iteration counts) and repeat
bitwise.
"""
import numpy as np
import pytest

from gpu_helpers import Staged, grid, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LANES = [1, 2, 4, 8, 16, 32, 64]


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def O():
    from oracle import oracle

    return oracle


@pytest.fixture(scope="module")
def staged():
    return Staged(grid(2000, 1))


@pytest.fixture(scope="module")
def refs(O, staged):
    g = staged.g
    nr = O.solve_grid(g)
    fd = O.solve_grid_fdpf(g)
    assert nr.status == 0 and fd.status == 0
    return nr, fd


def _set_lanes(s, lanes):
    m = s.sym.get_mapping()
    s.sym.set_mapping(np.full_like(m, lanes))
    assert (s.sym.get_mapping() == lanes).all()


@pytest.mark.parametrize("budget", [0, 65536])
@pytest.mark.parametrize("lanes", LANES)
def test_newton_every_lane_count(staged, refs, lanes, budget):
    s = staged
    s.sym.set_launch(512, budget, 4)
    _set_lanes(s, lanes)
    log(f"[lanes] newton lanes={lanes} tail budget={budget}")
    ref = refs[0]
    Vm, Va, iters, norm, status, _ = s.newton()
    Vm2, Va2, *_ = s.newton()
    torch.cuda.synchronize()
    assert status.item() == 0 and iters.item() == ref.iters
    np.testing.assert_allclose(Vm[0].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Va[0].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)
    assert torch.equal(Vm, Vm2) and torch.equal(Va, Va2)


@pytest.mark.parametrize("lanes", LANES)
def test_fdpf_every_lane_count(staged, refs, lanes):
    s = staged
    s.sym.set_launch(512, 65536, 4)
    _set_lanes(s, lanes)
    log(f"[lanes] fdpf lanes={lanes}")
    ref = refs[1]
    mat, st = s.sym.fdpf_factors(s.r, s.x, s.b, s.type)
    assert st.item() == 0
    Vm = s.Vm0.repeat(1, 1).contiguous()
    Va = s.Va0.repeat(1, 1).contiguous()
    it, nrm, status, _ = s.sym.fdpf(s.yval[0], s.type, s.Psp, s.Qsp, Vm, Va, mat)
    torch.cuda.synchronize()
    assert status.item() == 0 and it.item() == ref.iters and nrm.item() < 1e-8
    np.testing.assert_allclose(Vm[0].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Va[0].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)


@pytest.mark.parametrize("lanes", LANES)
def test_factor_and_both_solves_every_lane_count(O, staged, lanes):
    from paper_1811_02512_amd import binding as B

    s = staged
    g = s.g
    s.sym.set_launch(512, 65536, 4)
    _set_lanes(s, lanes)
    log(f"[lanes] factor/solve lanes={lanes}")
    rng = np.random.default_rng(21)
    Vm = rng.uniform(0.95, 1.05, g.n)
    Va = rng.uniform(-0.2, 0.2, g.n)
    Vm[0], Va[0] = 1.0, 0.0
    sym = O.Sym(g.n, g.f, g.t)
    oD, oL, oU = sym.block_jacobian(O.grid_ybus(g), g.bus_type, Vm, Va)
    fD, fL, fU, bad = sym.factor(oD, oL, oU)
    assert bad == -1
    info = s.sym.info
    nn = info.nn
    pad = np.zeros(info.lu_offset - 4 * nn)
    vals = torch.from_numpy(np.concatenate([oD.reshape(-1), pad,
                                            np.stack([oL, oU], 1).reshape(-1)])
                            ).to("cuda").reshape(1, -1).contiguous()
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    B.pf_factor(s.sym.h, 1, vals, info.vals_doubles, status)
    assert status.item() == 0
    rhs = rng.standard_normal((2, 2 * nn))
    r = torch.from_numpy(rhs.copy()).to("cuda")
    B.pf_solve(s.sym.h, 1, vals, info.vals_doubles, r[0:1], 2 * nn, 0)
    B.pf_solve(s.sym.h, 1, vals, info.vals_doubles, r[1:2], 2 * nn, 1)
    got = r.cpu().numpy()
    ox = sym.solve(fD, fL, fU, rhs[0]).reshape(-1)
    oxt = sym.solve_transpose(fD, fL, fU, rhs[1]).reshape(-1)
    np.testing.assert_allclose(got[0], ox, rtol=0, atol=1e-9 * np.abs(ox).max())
    np.testing.assert_allclose(got[1], oxt, rtol=0, atol=1e-9 * np.abs(oxt).max())
