"""Batches whose cases carry their own sparsity (N-1 outages, mixed grid sizes),
solved in one launch, against the oracle case by case."""
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


def solve_multi(grids, tol=1e-8, max_iter=20, tail_budget=None, spread=0):
    from paper_1811_02512_amd import api
    from paper_1811_02512_amd import binding as B

    syms = []
    for g in grids:
        s = api.Symbolic(g.n, g.f, g.t)
        if tail_budget is not None:
            s.set_launch(0, tail_budget)
        syms.append(s.upload())
    plan = api.MultiPlan(syms)
    if spread:
        plan.set_spread(spread)
    f64 = np.float64
    r = plan.concat([g.r for g in grids], "branch", f64)
    x = plan.concat([g.x for g in grids], "branch", f64)
    b = plan.concat([g.b for g in grids], "branch", f64)
    yv = torch.empty(int(plan.offs["y"][-1]) + 2, dtype=torch.float64, device="cuda")
    B.pf_build_ybus_multi(plan.p, r, x, b, yv)
    ty = plan.concat([g.bus_type for g in grids], "bus", np.int8)
    P = plan.concat([g.Psp for g in grids], "bus", f64)
    Q = plan.concat([g.Qsp for g in grids], "bus", f64)
    Vm = plan.concat([g.flat_start()[0] for g in grids], "bus", f64)
    Va = plan.concat([g.flat_start()[1] for g in grids], "bus", f64)
    ws = torch.empty(int(plan.offs["ws"][-1]) + 32, dtype=torch.float64, device="cuda")
    G = len(grids)
    it = torch.full((G,), -1, dtype=torch.int32, device="cuda")
    nrm = torch.empty(G, dtype=torch.float64, device="cuda")
    st = torch.full((G,), -1, dtype=torch.int32, device="cuda")
    pv = torch.full((G,), -9, dtype=torch.int32, device="cuda")
    B.pf_newton_multi(plan.p, yv, ty, P, Q, Vm, Va, tol, max_iter, 0, ws, it, nrm, st, pv)
    torch.cuda.synchronize()
    plan.pivots = pv.cpu().numpy()
    return (plan.split(Vm, "bus"), plan.split(Va, "bus"), it.cpu().numpy(), st.cpu().numpy(),
            plan)


def check_against_oracle(grids, Vms, Vas, it, st):
    from oracle import oracle as O

    for c, g in enumerate(grids):
        ref = O.solve_grid(g)
        assert ref.status == 0
        assert st[c] == 0, (c, st[c])
        assert it[c] == ref.iters, (c, it[c], ref.iters)
        np.testing.assert_allclose(Vms[c], ref.Vm, atol=1e-9)
        np.testing.assert_allclose(Vas[c], ref.Va, atol=1e-9)


def test_n1_outages_reanalysed():
    g = grid(2000, 1)
    outs = gridgen.n1_outages(g, 10, seed=3)
    log(f"[n1] outages {outs.tolist()}")
    grids = [g.without_branch(int(e)) for e in outs]
    Vms, Vas, it, st, _ = solve_multi(grids)
    check_against_oracle(grids, Vms, Vas, it, st)


def test_n1_equals_superset_pattern_with_zero_admittance():
    """An outage solved on its own pattern equals the base pattern with the
    branch's admittance driven to ~0 (x = 1e150) and no charging."""
    g = grid(500, 2)
    e = int(gridgen.n1_outages(g, 1, seed=7)[0])
    gg = g.without_branch(e)
    Vms, Vas, it, st, _ = solve_multi([gg])
    open_ = g.without_branch(e)  # same physics, different pattern source
    assert open_.m == g.m - 1
    x = g.x.copy()
    x[e] = 1e150
    bb = g.b.copy()
    bb[e] = 0.0
    import dataclasses

    s = Staged(dataclasses.replace(g, x=x, b=bb))
    Vm, Va, it2, _, st2, _ = s.newton()
    assert st[0] == 0 and st2.item() == 0
    np.testing.assert_allclose(Vm[0].cpu().numpy(), Vms[0], atol=1e-9)
    np.testing.assert_allclose(Va[0].cpu().numpy(), Vas[0], atol=1e-9)


def test_mixed_grid_sizes_one_launch():
    """The first mixed-batch grids of up to 6,000 buses (sizes and seeds from
    tests/golden/mixed_batch.json) in one launch, each against the oracle."""
    import json
    import os

    spec = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mixed_batch.json")))
    chosen = [gs for gs in spec["grids"] if gs["n"] <= 6000][:7]
    log(f"[mixed] sizes {[gs['n'] for gs in chosen]}")
    grids = [gridgen.make_grid(gs["n"], gs["seed"], load_scale=spec["load_scale"])
             for gs in chosen]
    Vms, Vas, it, st, plan = solve_multi(grids)
    check_against_oracle(grids, Vms, Vas, it, st)


def test_multi_matches_shared_pattern_path():
    """The per-case-pattern kernel and the shared-pattern kernel agree bitwise."""
    g = grid(800, 3)
    Vms, Vas, it, st, _ = solve_multi([g, g])
    s = Staged(g)
    Vm, Va, it2, _, _, _ = s.newton()
    np.testing.assert_array_equal(Vms[0], Vm[0].cpu().numpy())
    np.testing.assert_array_equal(Vms[1], Vm[0].cpu().numpy())
    np.testing.assert_array_equal(Vas[0], Va[0].cpu().numpy())


def test_mixed_launch_with_the_largest_grids():
    """The two largest grids of the mixed range (~18-19k buses, too large for
    the LDS copy of (e, f)) and the two smallest in one launch with the
    largest LDS tail, each against the oracle."""
    import json
    import os

    spec = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mixed_batch.json")))
    by_size = sorted(spec["grids"], key=lambda gs: gs["n"])
    chosen = by_size[-2:] + by_size[:2]
    log(f"[mixed] sizes {[gs['n'] for gs in chosen]}")
    grids = [gridgen.make_grid(gs["n"], gs["seed"], load_scale=spec["load_scale"])
             for gs in chosen]
    Vms, Vas, it, st, plan = solve_multi(grids, tail_budget=161792)
    check_against_oracle(grids, Vms, Vas, it, st)


def test_plan_refuses_members_changed_since_its_upload():
    """Re-uploading a member (its device copy may have moved or changed shape)
    makes the plan stale until the plan itself is uploaded again."""
    from paper_1811_02512_amd import api
    from paper_1811_02512_amd import binding as B

    grids = [grid(300, 1), grid(500, 2)]
    Vms, Vas, it, st, plan = solve_multi(grids)
    assert (st == 0).all()
    syms = plan.syms
    syms[1].set_launch(0, 16384)  # new tail: re-analysed and re-uploaded
    f64 = np.float64
    r = plan.concat([g.r for g in grids], "branch", f64)
    x = plan.concat([g.x for g in grids], "branch", f64)
    b = plan.concat([g.b for g in grids], "branch", f64)
    yv = torch.empty(int(plan.offs["y"][-1]) + 2, dtype=torch.float64, device="cuda")
    with pytest.raises(B.PfError) as ei:
        B.pf_build_ybus_multi(plan.p, r, x, b, yv)
    assert ei.value.code == B.PF_E_INVALID and "upload the plan again" in B.last_error()
    B.pf_multi_upload(plan.p, plan.buf)
    B.pf_build_ybus_multi(plan.p, r, x, b, yv)
    torch.cuda.synchronize()


def test_mixed_grids_with_spread_groups():
    """More workgroups than grids: the 10k and 3k grids share their wide
    levels among groups of workgroups (grid barriers per group) while the
    small ones keep one each; every case matches the oracle and the
    one-workgroup-per-case launch."""
    grids = [grid(10000, 1), grid(200, 4), grid(3000, 2), grid(700, 3)]
    Vms, Vas, it, st, _ = solve_multi(grids, tail_budget=161792, spread=96)
    Vm1, Va1, it1, st1, _ = solve_multi(grids, tail_budget=161792)
    log(f"[multi spread] iterations {it.tolist()} (one workgroup each: {it1.tolist()})")
    assert st.tolist() == st1.tolist() == [0] * len(grids)
    assert it.tolist() == it1.tolist()
    for c in range(len(grids)):
        assert np.abs(Vms[c] - Vm1[c]).max() < 1e-12
        assert np.abs(Vas[c] - Va1[c]).max() < 1e-12
    check_against_oracle(grids, Vms, Vas, it, st)


def test_spread_groups_keep_each_case_status_apart():
    """In a batch with spread groups, a zero pivot in one grid (a bus cut off,
    at a leaf of the shared levels) ends only that case, with its position,
    while the grids around it, spread or not, converge; a plan whose spread
    changed is refused until it is uploaded again."""
    import test_gpu_failures as F
    from oracle import oracle as O
    from paper_1811_02512_amd import binding as B

    g = grid(2000, 3)
    s0 = Staged(g)
    ex = s0.sym.export()
    leaves, _, _ = F.regions(s0.info, ex)
    bad, p = F.pick(O, g, leaves, ex["perm"], O.Sym(g.n, g.f, g.t))
    grids = [grid(10000, 1), bad, grid(700, 3), g]
    Vms, Vas, it, st, plan = solve_multi(grids, tail_budget=161792, spread=96)
    log(f"[multi spread] statuses {st.tolist()} pivots {plan.pivots.tolist()} (position {p})")
    assert st.tolist() == [0, B.PF_E_ZERO_PIVOT, 0, 0]
    assert plan.pivots.tolist() == [-1, p, -1, -1]
    ok = [grids[c] for c in (0, 2, 3)]
    check_against_oracle(ok, [Vms[c] for c in (0, 2, 3)], [Vas[c] for c in (0, 2, 3)],
                         it[[0, 2, 3]], st[[0, 2, 3]])
    B.pf_multi_set_spread(plan.p, 64)
    with pytest.raises(B.PfError) as ei:
        B.pf_newton_multi(plan.p, plan.buf, plan.buf, plan.buf, plan.buf, plan.buf, plan.buf,
                          1e-8, 20, 0, plan.buf)
    assert ei.value.code == B.PF_E_INVALID and "not uploaded" in B.last_error()
