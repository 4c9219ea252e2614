"""CPU tests of libpf: the library loads and exports every symbol of
include/pf.h; its host analysis is bit-exact with the oracle's; argument and
topology errors come back as status codes without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import gridgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_1811_02512_amd import binding

    return binding


def header_symbols():
    src = open(os.path.join(ROOT, "include", "pf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_header_symbol(B):
    syms = header_symbols()
    assert len(syms) >= 20
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    assert B.lib.pf_version().decode().startswith("libpf")
    assert B.lib.pf_status_string(5).decode() == "zero pivot"


@pytest.mark.parametrize("n,seed,ordering", [(30, 2, 0), (200, 1, 0), (200, 1, 1), (2000, 1, 0),
                                             (2000, 3, 1), (10000, 1, 0)])
def test_analysis_bit_exact_with_oracle(B, oracle, n, seed, ordering):
    g = gridgen.make_grid(n, seed)
    h = B.pf_analyze(g.n, g.f, g.t, 0, ordering)
    try:
        ex = B.pf_symbolic_export(h)
        s = oracle.Sym(g.n, g.f, g.t, 0, ordering)
        for k in ("perm", "parent", "level", "level_ptr", "level_nodes", "Lp", "Li"):
            np.testing.assert_array_equal(ex[k], getattr(s, k), err_msg=k)
        info = B.pf_symbolic_info(h)
        assert info.nn == n - 1 and info.nnz_l == s.nnzL and info.nlevels == s.nlev
        assert info.lu_offset == 8 * ((info.nn + 1) // 2)
        assert info.vals_doubles == info.lu_offset + 8 * info.nnz_l
        yptr, ycol = B.pf_symbolic_ybus_pattern(h)
        Y = oracle.grid_ybus(g)
        np.testing.assert_array_equal(yptr, Y.rowptr)
        np.testing.assert_array_equal(ycol, Y.col)
    finally:
        B.pf_symbolic_destroy(h)


def test_analysis_n1_outages_bit_exact(B, oracle):
    g = gridgen.make_grid(500, 5)
    for e in gridgen.n1_outages(g, 6, seed=3):
        gg = g.without_branch(int(e))
        h = B.pf_analyze(gg.n, gg.f, gg.t)
        ex = B.pf_symbolic_export(h)
        s = oracle.Sym(gg.n, gg.f, gg.t)
        for k in ("perm", "parent", "level_ptr", "level_nodes", "Lp", "Li"):
            np.testing.assert_array_equal(ex[k], getattr(s, k))
        B.pf_symbolic_destroy(h)


def test_parallel_branches_and_forest(B, oracle):
    f = np.array([0, 0, 1, 0, 3, 3], np.int32)
    t = np.array([1, 1, 2, 3, 4, 4], np.int32)
    h = B.pf_analyze(5, f, t)
    ex = B.pf_symbolic_export(h)
    s = oracle.Sym(5, f, t)
    np.testing.assert_array_equal(ex["parent"], s.parent)
    assert int(np.sum(ex["parent"] == -1)) == 2
    yptr, ycol = B.pf_symbolic_ybus_pattern(h)
    assert yptr[-1] == 5 + 2 * 4  # diagonal + 4 distinct neighbour pairs
    B.pf_symbolic_destroy(h)


def test_table1_levels_through_libpf(B):
    parent = {1: 3, 2: 3, 4: 5, 3: 7, 5: 7, 6: 7, 7: 8, 8: 9, 9: 10}
    f = np.array(list(parent), np.int32)
    t = np.array(list(parent.values()), np.int32)
    # the analysis requires every bus to reach the slack: hang bus 10 on it
    f = np.append(f, 10).astype(np.int32)
    t = np.append(t, 0).astype(np.int32)
    h = B.pf_analyze(11, f, t, 0, B.PF_ORDER_NATURAL)
    ex = B.pf_symbolic_export(h)
    lp, ln = ex["level_ptr"], ex["level_nodes"]
    got = [sorted(int(ex["perm"][v]) for v in ln[lp[l]:lp[l + 1]]) for l in range(len(lp) - 1)]
    assert got == [[1, 2, 4, 6], [3, 5], [7], [8], [9], [10]]
    B.pf_symbolic_destroy(h)


@pytest.mark.parametrize("n,f,t,slack,code", [
    (1, [], [], 0, 1),
    (3, [0, 1], [1, 1], 0, 1),
    (3, [0, 1], [1, 5], 0, 1),
    (3, [0, -1], [1, 2], 0, 1),
    (3, [0, 1], [1, 2], 3, 1),
    (4, [0, 1], [1, 2], 0, 4),
    (4, [2], [3], 0, 4),
])
def test_analysis_errors(B, n, f, t, slack, code):
    with pytest.raises(B.PfError) as ei:
        B.pf_analyze(n, np.array(f, np.int32), np.array(t, np.int32), slack)
    assert ei.value.code == code
    assert B.last_error()


def test_device_calls_need_upload(B):
    g = gridgen.make_grid(20, 1)
    h = B.pf_analyze(g.n, g.f, g.t)
    buf = np.zeros(8)
    with pytest.raises(B.PfError) as ei:
        B.check(B.lib.pf_factor(h, 1, buf.ctypes.data, 0, 1, None, None, None), "pf_factor")
    assert ei.value.code == B.PF_E_INVALID
    assert "not uploaded" in B.last_error()
    with pytest.raises(B.PfError):
        B.check(B.lib.pf_newton(None, 1, *([None, 0] * 2), None, None, 0, None, None, 0, 1e-8,
                                20, 0, None, 0, None, None, None, None, None), "pf_newton")
    B.pf_symbolic_destroy(h)


def test_mapping_roundtrip_and_validation(B):
    g = gridgen.make_grid(300, 2)
    h = B.pf_analyze(g.n, g.f, g.t)
    m = B.pf_symbolic_get_mapping(h)
    assert set(np.unique(m)) <= {1, 2, 4, 8, 16, 32, 64}
    B.pf_symbolic_set_mapping(h, np.full_like(m, 8))
    assert (B.pf_symbolic_get_mapping(h) == 8).all()
    with pytest.raises(B.PfError):
        B.pf_symbolic_set_mapping(h, np.full_like(m, 3))
    B.pf_symbolic_destroy(h)


def test_multi_plan_offsets(B):
    gs = [gridgen.make_grid(n, s) for n, s in [(40, 1), (90, 2), (25, 3)]]
    hs = [B.pf_analyze(g.n, g.f, g.t) for g in gs]
    p = B.pf_multi_create(hs)
    nbytes, offs = B.pf_multi_info(p, 3)
    assert nbytes > 0
    assert offs["bus"].tolist() == [0, 40, 130, 155]
    assert offs["branch"].tolist() == [0, gs[0].m, gs[0].m + gs[1].m, sum(g.m for g in gs)]
    infos = [B.pf_symbolic_info(h) for h in hs]
    assert np.diff(offs["ws"]).tolist() == [i.ws_doubles for i in infos]
    assert np.diff(offs["y"]).tolist() == [2 * i.nnz_y for i in infos]
    B.pf_multi_destroy(p)
    for h in hs:
        B.pf_symbolic_destroy(h)


def test_single_hip_runtime_whatever_the_import_order():
    """Importing the package before torch must not load a second HIP runtime."""
    import subprocess
    import sys

    code = ("import paper_1811_02512_amd, torch\n"
            "maps = [l.split()[-1] for l in open('/proc/self/maps') "
            "if 'libamdhip64' in l and 'r-xp' in l]\n"
            "print(len(set(maps)))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_state_estimation_analysis_sizes_and_errors():
    """The WLS plan: one partial per (measurement, support bus), the gain
    graph spans every bus, and unobservable or malformed sets are refused."""
    from oracle import se

    from paper_1811_02512_amd import binding as B

    g = gridgen.make_grid(60, 2)
    kinds, locs = se.full_measurement_set(g)
    h = B.pf_se_analyze(g.n, g.f, g.t, 0, kinds, locs)
    d = B.pf_se_info(h)
    deg = np.bincount(np.concatenate([g.f, g.t]), minlength=g.n)
    assert d.measurements == 3 * g.n + 2 * g.m
    assert d.partials == g.n + 2 * (g.n + deg.sum()) + 4 * g.m
    assert d.gain_levels > 0 and d.gain_nnz_l > 0 and d.ws_doubles % 8 == 0
    B.pf_se_destroy(h)
    only_v = np.full(g.n, B.PF_MEAS_VM, np.int8)
    with pytest.raises(B.PfError, match="unobservable"):
        B.pf_se_analyze(g.n, g.f, g.t, 0, only_v, np.arange(g.n))
    with pytest.raises(B.PfError):
        B.pf_se_analyze(g.n, g.f, g.t, 0, np.array([9], np.int8), np.array([0]))
    with pytest.raises(B.PfError):
        B.pf_se_analyze(g.n, g.f, g.t, 0, np.array([B.PF_MEAS_PF], np.int8),
                        np.array([g.m + 3]))


def test_set_launch_checks_every_argument_before_changing_any(B):
    g = gridgen.make_grid(80, 3)
    h = B.pf_analyze(g.n, g.f, g.t)
    before = B.pf_symbolic_info(h)
    for threads, budget, inter in ((100, 65536, 2), (256, -1, 2), (256, 200000, 8),
                                   (256, 65536, 3)):
        with pytest.raises(B.PfError) as ei:
            B.pf_symbolic_set_launch(h, threads, budget, inter)
        assert ei.value.code == B.PF_E_INVALID
        after = B.pf_symbolic_info(h)
        assert (after.ws_interleave, after.threads, after.tail_nodes) == \
            (before.ws_interleave, before.threads, before.tail_nodes)
    B.pf_symbolic_set_launch(h, 256, 65536, 2)
    assert B.pf_symbolic_info(h).ws_interleave == 2
    B.pf_symbolic_destroy(h)


def test_spread_setting_is_checked_and_reported(B):
    """The workgroups of a one-case launch: 0..1024, 0 and 1 both meaning one
    workgroup; the workspace holds the grid-barrier words after the rhs."""
    g = gridgen.make_grid(80, 3)
    h = B.pf_analyze(g.n, g.f, g.t)
    assert B.pf_symbolic_info(h).spread == 0
    for bad in (-1, 1025):
        with pytest.raises(B.PfError) as ei:
            B.pf_symbolic_set_spread(h, bad)
        assert ei.value.code == B.PF_E_INVALID
    B.pf_symbolic_set_spread(h, 32)
    assert B.pf_symbolic_info(h).spread == 32
    B.pf_symbolic_set_spread(h, 1)
    assert B.pf_symbolic_info(h).spread == 0
    i = B.pf_symbolic_info(h)
    rhs_end = i.vals_doubles + 8 * i.n + 2 * i.nn
    sync = (rhs_end + 15) // 16 * 16  # three 128-byte lines on a 128-byte boundary
    assert i.ws_doubles % 32 == 0 and i.ws_doubles >= sync + 48
    B.pf_symbolic_destroy(h)


def test_multi_plan_spread_setting(B):
    """pf_multi_set_spread: 0..65535 workgroups; grids too small to share
    their levels keep one workgroup each (the device table does not grow),
    a 10k grid takes extra workgroups (it grows)."""
    gs = [gridgen.make_grid(n, s) for n, s in [(40, 1), (90, 2)]]
    hs = [B.pf_analyze(g.n, g.f, g.t) for g in gs]
    p = B.pf_multi_create(hs)
    base, _ = B.pf_multi_info(p, 2)
    for bad in (-1, 65536):
        with pytest.raises(B.PfError) as ei:
            B.pf_multi_set_spread(p, bad)
        assert ei.value.code == B.PF_E_INVALID
    B.pf_multi_set_spread(p, 64)
    assert B.pf_multi_info(p, 2)[0] == base
    B.pf_multi_destroy(p)
    big = gridgen.make_grid(10000, 1)
    hb = B.pf_analyze(big.n, big.f, big.t)
    p = B.pf_multi_create(hs + [hb])
    base, _ = B.pf_multi_info(p, 3)
    B.pf_multi_set_spread(p, 64)
    assert B.pf_multi_info(p, 3)[0] > base
    B.pf_multi_set_spread(p, 0)
    assert B.pf_multi_info(p, 3)[0] == base
    B.pf_multi_destroy(p)
    for h in hs + [hb]:
        B.pf_symbolic_destroy(h)


def test_subtree_cut_of_the_spread_batch_groups():
    """The cut below which the groups of a spread batch of grids run whole
    subtrees per workgroup: the highest level at or below the LDS tail with
    at least 768 subtree roots (nodes below it whose parent is at or above
    it), recomputed here from the exported elimination tree."""
    import gridgen
    from paper_1811_02512_amd import api

    for n, seed, budget in [(10000, 1, 161792), (10000, 1, 0), (2000, 2, 65536), (200, 1, 65536)]:
        g = gridgen.make_grid(n, seed)
        sym = api.Symbolic(g.n, g.f, g.t)
        sym.set_launch(512, budget, 1)
        info = sym.info
        ex = sym.export()
        lev = np.asarray(ex["level"]) - 1
        par = np.asarray(ex["parent"])
        top = info.nlevels - info.tail_levels
        want = 0
        for c in range(1, top + 1):
            plev = np.where(par >= 0, lev[np.maximum(par, 0)], info.nlevels)
            roots = int(((lev < c) & (plev >= c)).sum())
            if roots >= 768:
                want = c
        assert info.sub_levels == want, (n, budget, info.sub_levels, want)
    assert want == 0  # 200 buses: too few leaves
