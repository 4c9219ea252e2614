"""Fast decoupled power flow and branch flows on the GPU, through the C ABI,
against the CPU oracle on the same seeded inputs."""
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


def _O():
    from oracle import oracle as O

    return O


def split(s, mat):
    """(d, lo, up) of B' and B'' from one row of the device layout."""
    info = s.info
    M = info.fd_mat_doubles // 2
    nn, nz = info.nn, info.nnz_l
    fd_lu = (nn + 7) // 8 * 8
    v = mat.cpu().numpy()
    out = []
    for k in range(2):
        m = v[k * M:(k + 1) * M]
        assert np.all(m[nn:fd_lu] == 0.0)
        sl = m[fd_lu:fd_lu + 2 * nz].reshape(-1, 2)
        out.append((m[:nn], sl[:, 0], sl[:, 1]))
    return out


@pytest.mark.parametrize("n,seed", [(200, 1), (2000, 2)])
def test_fdpf_matrices_and_factors(n, seed):
    O = _O()
    g = grid(n, seed)
    s = Staged(g)
    log(f"[fdpf] matrices n={n} seed={seed}")
    info = s.info
    mat = torch.empty(1, info.fd_mat_doubles, dtype=torch.float64, device="cuda")
    from paper_1811_02512_amd import binding as B

    B.pf_fdpf_matrices(s.sym.h, 1, s.r, s.x, s.b, 0, s.type, 0, mat, info.fd_mat_doubles)
    osym = O.Sym(g.n, g.f, g.t)
    d1, a1, d2, a2 = osym.fdpf_matrices(g)
    (gd1, gl1, gu1), (gd2, gl2, gu2) = split(s, mat[0])
    for gd, gl, gu, d, a in ((gd1, gl1, gu1, d1, a1), (gd2, gl2, gu2, d2, a2)):
        np.testing.assert_allclose(gd, d, rtol=1e-14, atol=0)
        np.testing.assert_allclose(gl, a, rtol=1e-14, atol=0)
        np.testing.assert_array_equal(gl, gu)
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    B.pf_fdpf_factor(s.sym.h, 1, mat, info.fd_mat_doubles, status)
    assert status.item() == 0
    (fd1, fw1, fu1), (fd2, fw2, fu2) = split(s, mat[0])
    for fd, fw, fu, d, a in ((fd1, fw1, fu1, d1, a1), (fd2, fw2, fu2, d2, a2)):
        od, oL, oU, bad = osym.factor1(d, a)
        assert bad == -1
        np.testing.assert_allclose(1.0 / fd, od, rtol=1e-10)
        np.testing.assert_allclose(fu, oL, rtol=1e-10, atol=1e-13)
        owner = np.repeat(np.arange(info.nn), np.diff(osym.Lp))
        np.testing.assert_allclose(fw, oL * od[owner], rtol=1e-10, atol=1e-12 * np.abs(od).max())


@pytest.mark.parametrize("n,seed", [(200, 1), (2000, 2), (10000, 1)])
def test_fdpf_matches_oracle(n, seed):
    O = _O()
    g = grid(n, seed)
    s = Staged(g)
    log(f"[fdpf] solve n={n} seed={seed}")
    mat, st = s.sym.fdpf_factors(s.r, s.x, s.b, s.type)
    assert st.item() == 0
    Vm = s.Vm0.repeat(1, 1).contiguous()
    Va = s.Va0.repeat(1, 1).contiguous()
    it, nrm, status, _ = s.sym.fdpf(s.yval[0], s.type, s.Psp, s.Qsp, Vm, Va, mat)
    ref = O.solve_grid_fdpf(g)
    assert ref.status == 0 and status.item() == 0
    assert it.item() == ref.iters
    assert nrm.item() < 1e-8
    np.testing.assert_allclose(Vm[0].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Va[0].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)


def test_fdpf_batched_shared_and_per_case_factors():
    """Scenarios share one factorisation; cases with their own reactances
    bring their own.  Each case against the oracle."""
    O = _O()
    g = grid(2000, 3)
    s = Staged(g)
    Bn = 6
    P, Q = gridgen.scenario_injections(g, Bn, seed=4)
    mat, st = s.sym.fdpf_factors(s.r, s.x, s.b, s.type)
    Vm = s.Vm0.repeat(Bn, 1).contiguous()
    Va = s.Va0.repeat(Bn, 1).contiguous()
    it, _, status, _ = s.sym.fdpf(s.yval[0], s.type, dev(P), dev(Q), Vm, Va, mat)
    osym = O.Sym(g.n, g.f, g.t)
    Y = O.grid_ybus(g)
    Vm0, Va0 = g.flat_start()
    for c in range(Bn):
        ref = osym.fdpf(Y, g, P[c], Q[c], Vm0, Va0)
        assert ref.status == 0 and status[c].item() == 0
        assert it[c].item() == ref.iters
        np.testing.assert_allclose(Vm[c].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va[c].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)
    # per-case reactances: case c scales x by 1 + 0.05 c
    scale = 1.0 + 0.05 * np.arange(3)
    xs = np.stack([g.x * k for k in scale])
    rs = np.stack([g.r] * 3)
    bs = np.stack([g.b] * 3)
    xs_d, rs_d, bs_d = dev(xs), dev(rs), dev(bs)
    ymat = torch.empty(3, 2 * s.info.nnz_y, dtype=torch.float64, device="cuda")
    from paper_1811_02512_amd import binding as B

    B.pf_build_ybus(s.sym.h, 3, rs_d, xs_d, bs_d, g.m, ymat, 2 * s.info.nnz_y)
    mats, st = s.sym.fdpf_factors(rs_d, xs_d, bs_d, s.type)
    assert (st.cpu().numpy() == 0).all()
    Vm = s.Vm0.repeat(3, 1).contiguous()
    Va = s.Va0.repeat(3, 1).contiguous()
    it, _, status, _ = s.sym.fdpf(ymat, s.type, s.Psp, s.Qsp, Vm, Va, mats)
    for c in range(3):
        import dataclasses

        gc = dataclasses.replace(g, x=xs[c])
        ref = O.solve_grid_fdpf(gc, sym=osym)
        assert ref.status == 0 and status[c].item() == 0
        assert it[c].item() == ref.iters
        np.testing.assert_allclose(Vm[c].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)


def test_fdpf_status_codes():
    g = grid(200, 1)
    s = Staged(g)
    mat, _ = s.sym.fdpf_factors(s.r, s.x, s.b, s.type)
    P = s.Psp.repeat(2, 1).contiguous()
    P[1, 7] = float("nan")
    Vm = s.Vm0.repeat(2, 1).contiguous()
    Va = s.Va0.repeat(2, 1).contiguous()
    from paper_1811_02512_amd import binding as B

    _, _, st, _ = s.sym.fdpf(s.yval[0], s.type, P, s.Qsp, Vm, Va, mat, max_iter=40)
    assert st.cpu().tolist() == [0, B.PF_E_NONFINITE]
    Vm = s.Vm0.repeat(1, 1).contiguous()
    Va = s.Va0.repeat(1, 1).contiguous()
    it, _, st, _ = s.sym.fdpf(s.yval[0], s.type, s.Psp, s.Qsp, Vm, Va, mat, max_iter=2)
    assert st.item() == B.PF_E_NOT_CONVERGED and it.item() == 2
    # a bus hanging on one branch of infinite reactance has a zero B' pivot
    deg = np.bincount(np.concatenate([g.f, g.t]), minlength=g.n)
    e = next(e for e in range(g.m) if (deg[g.f[e]] == 1 and g.f[e] != 0)
             or (deg[g.t[e]] == 1 and g.t[e] != 0))
    x = g.x.copy()
    x[e] = np.inf
    _, st = s.sym.fdpf_factors(s.r, dev(x), s.b, s.type)
    assert st.item() == B.PF_E_ZERO_PIVOT


@pytest.mark.parametrize("n,seed", [(200, 1), (2000, 2)])
def test_branch_flows_match_oracle(n, seed):
    O = _O()
    g = grid(n, seed)
    s = Staged(g)
    rng = np.random.default_rng(seed)
    Vm = 1.0 + 0.05 * rng.standard_normal((3, g.n))
    Va = 0.1 * rng.standard_normal((3, g.n))
    out = s.sym.branch_flows(s.r, s.x, s.b, dev(Vm), dev(Va))
    for c in range(3):
        ref = O.branch_flows(g, Vm[c], Va[c])
        for got, want in zip(out, ref):
            np.testing.assert_allclose(got[c].cpu().numpy(), want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,seed,budget,efl,vl", [(200, 1, 161792, True, False),
                                                  (10000, 1, 161792, True, True),
                                                  (12000, 3, 65536, False, False)])
def test_fdpf_lds_layouts(n, seed, budget, efl, vl):
    """The kernel's three LDS layouts: both matrix tails resident (no room
    for the (e, f) copy), the copy with the work vector in global memory, and
    the copy with the work vector in LDS; two cases each against the oracle."""
    O = _O()
    g = grid(n, seed)
    s = Staged(g)
    s.sym.set_launch(512, budget)
    info = s.sym.info
    K = info.tail_nodes
    TS = (info.tail_lds_bytes - 48 * K) // 64
    has_ef = 16 * n + 8 * ((n + 63) // 64) + 2048 <= 160 * 1024
    has_vl = has_ef and 16 * (TS + K) + 8 * info.nn <= 16 * n
    log(f"[fdpf] layout n={n} tail K={K} TS={TS} ef={has_ef} vector={has_vl}")
    assert (has_ef, has_vl) == (efl, vl)
    mat, st = s.sym.fdpf_factors(s.r, s.x, s.b, s.type)
    assert st.item() == 0
    Vm = s.Vm0.repeat(2, 1).contiguous()
    Va = s.Va0.repeat(2, 1).contiguous()
    it, nrm, status, _ = s.sym.fdpf(s.yval[0], s.type, s.Psp, s.Qsp, Vm, Va, mat)
    ref = O.solve_grid_fdpf(g)
    assert ref.status == 0
    for c in range(2):
        assert status[c].item() == 0 and it[c].item() == ref.iters
        np.testing.assert_allclose(Vm[c].cpu().numpy(), ref.Vm, rtol=0, atol=1e-9)
        np.testing.assert_allclose(Va[c].cpu().numpy(), ref.Va, rtol=0, atol=1e-9)
