"""WLS state estimation on the GPU through the C ABI, against the CPU
oracle on the same seeded measurements."""
import numpy as np
import pytest

import gridgen
from gpu_helpers import dev, grid, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _setup(g, kinds, locs):
    from paper_1811_02512_amd import api

    return api.StateEstimator(g.n, g.f, g.t, kinds, locs)


def _observable(g, kinds, locs):
    """Adds flow pairs on branches that join separate parts of the graph of
    measured active flows until those flows span the grid: a spanning tree
    of flow measurements fixes every angle difference, so the set is
    observable (a connected gain graph alone does not guarantee it)."""
    from oracle import se

    parent = list(range(g.n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for k, l in zip(kinds, locs):
        if k == se.PFLOW:
            parent[find(g.f[l])] = find(g.t[l])
    add_k, add_l = [], []
    for e in range(g.m):
        a, b = find(g.f[e]), find(g.t[e])
        if a != b:
            parent[a] = b
            add_k += [se.PFLOW, se.QFLOW]
            add_l += [e, e]
    log(f"[se] {len(add_k)} flow measurements added for observability")
    return (np.concatenate([kinds, np.array(add_k, kinds.dtype)]),
            np.concatenate([locs, np.array(add_l, locs.dtype)]))


def _noisy(g, kinds, locs, cases, seed):
    from oracle import oracle as O
    from oracle import se

    ref = O.solve_grid(g)
    z0 = se.measure(g, O.grid_ybus(g), ref.Vm, ref.Va, kinds, locs)
    sig = np.where(kinds == se.VM, 0.004, 0.01)
    rng = np.random.default_rng(seed)
    z = z0 + sig * rng.standard_normal((cases, len(z0)))
    return ref, z, 1.0 / sig ** 2


@pytest.mark.parametrize("n,seed", [(200, 1), (2000, 2)])
def test_se_matches_oracle(n, seed):
    from oracle import se

    g = grid(n, seed)
    kinds, locs = se.full_measurement_set(g)
    ref, z, w = _noisy(g, kinds, locs, 3, seed)
    est = _setup(g, kinds, locs)
    log(f"[se] n={n} measurements={len(kinds)} gain levels={est.dims.gain_levels}")
    Vm = torch.ones(3, g.n, dtype=torch.float64, device="cuda")
    Va = torch.zeros(3, g.n, dtype=torch.float64, device="cuda")
    it, nrm, st, _ = est.estimate(dev(g.r), dev(g.x), dev(g.b), dev(z), dev(w), Vm, Va)
    for c in range(3):
        r = se.estimate(g, kinds, locs, z[c], w, np.ones(g.n), np.zeros(g.n))
        assert r.status == 0 and st[c].item() == 0
        assert it[c].item() == r.iters
        np.testing.assert_allclose(Vm[c].cpu().numpy(), r.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va[c].cpu().numpy(), r.Va, rtol=0, atol=1e-9)


def test_se_noise_free_recovers_power_flow_state():
    from oracle import oracle as O
    from oracle import se

    g = grid(2000, 3)
    kinds, locs = se.full_measurement_set(g)
    ref = O.solve_grid(g)
    z = se.measure(g, O.grid_ybus(g), ref.Vm, ref.Va, kinds, locs)
    w = np.where(kinds == se.VM, 1 / 0.004 ** 2, 1 / 0.01 ** 2)
    est = _setup(g, kinds, locs)
    Vm = torch.ones(1, g.n, dtype=torch.float64, device="cuda")
    Va = torch.zeros(1, g.n, dtype=torch.float64, device="cuda")
    _, _, st, _ = est.estimate(dev(g.r), dev(g.x), dev(g.b), dev(z), dev(w), Vm, Va)
    assert st.item() == 0
    np.testing.assert_allclose(Vm[0].cpu().numpy(), ref.Vm, rtol=0, atol=1e-10)
    np.testing.assert_allclose(Va[0].cpu().numpy(), ref.Va, rtol=0, atol=1e-10)


def test_se_partial_measurement_set():
    """A sparser set: every |V|, injections at 70% of buses, flows at 40% of
    branches, in a shuffled order."""
    from oracle import se

    g = grid(500, 4)
    rng = np.random.default_rng(9)
    kinds, locs = se.full_measurement_set(g)
    keep = (kinds == se.VM) | (rng.uniform(size=len(kinds)) < np.where(kinds <= se.QINJ, 0.7, 0.4))
    kinds, locs = _observable(g, kinds[keep], locs[keep])
    order = rng.permutation(len(kinds))
    kinds, locs = kinds[order], locs[order]
    ref, z, w = _noisy(g, kinds, locs, 2, 5)
    est = _setup(g, kinds, locs)
    Vm = torch.ones(2, g.n, dtype=torch.float64, device="cuda")
    Va = torch.zeros(2, g.n, dtype=torch.float64, device="cuda")
    it, _, st, _ = est.estimate(dev(g.r), dev(g.x), dev(g.b), dev(z), dev(w), Vm, Va)
    for c in range(2):
        r = se.estimate(g, kinds, locs, z[c], w, np.ones(g.n), np.zeros(g.n))
        assert r.status == 0 and st[c].item() == 0 and it[c].item() == r.iters
        np.testing.assert_allclose(Vm[c].cpu().numpy(), r.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va[c].cpu().numpy(), r.Va, rtol=0, atol=1e-9)


def test_se_many_cases_per_case_branch_data():
    """70 cases (two 64-case lane groups, a partial group of four) with their
    own branch reactances and noise, each against the oracle on its grid."""
    import dataclasses

    from oracle import oracle as O
    from oracle import se

    g = grid(200, 6)
    kinds, locs = se.full_measurement_set(g)
    Bn = 70
    rng = np.random.default_rng(21)
    xs = g.x[None, :] * rng.uniform(0.9, 1.1, (Bn, g.m))
    sig = np.where(kinds == se.VM, 0.004, 0.01)
    w = 1.0 / sig ** 2
    grids, zs = [], []
    for c in range(Bn):
        gc = dataclasses.replace(g, x=xs[c].copy())
        ref = O.solve_grid(gc)
        assert ref.status == 0
        z0 = se.measure(gc, O.grid_ybus(gc), ref.Vm, ref.Va, kinds, locs)
        grids.append(gc)
        zs.append(z0 + sig * rng.standard_normal(len(z0)))
    z = np.array(zs)
    R = np.repeat(g.r[None, :], Bn, 0)
    Bc = np.repeat(g.b[None, :], Bn, 0)
    est = _setup(g, kinds, locs)
    Vm = torch.ones(Bn, g.n, dtype=torch.float64, device="cuda")
    Va = torch.zeros(Bn, g.n, dtype=torch.float64, device="cuda")
    it, _, st, _ = est.estimate(dev(R), dev(xs), dev(Bc), dev(z), dev(w), Vm, Va)
    it, st = it.cpu().numpy(), st.cpu().numpy()
    Vm, Va = Vm.cpu().numpy(), Va.cpu().numpy()
    for c in range(Bn):
        r = se.estimate(grids[c], kinds, locs, z[c], w, np.ones(g.n), np.zeros(g.n))
        assert r.status == 0 and st[c] == 0 and it[c] == r.iters, (c, st[c], it[c], r.iters)
        np.testing.assert_allclose(Vm[c], r.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va[c], r.Va, rtol=0, atol=1e-9)
