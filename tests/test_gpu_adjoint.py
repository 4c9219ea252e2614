"""Adjoint (torch.autograd.Function) on the GPU against the oracle's dense and
sparse adjoints and against central finite differences of the GPU solve."""
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


def setup(g, Bn, seed):
    from paper_1811_02512_amd import api

    sym = api.Symbolic(g.n, g.f, g.t).upload()
    if Bn == 1:
        P, Q = g.Psp[None], g.Qsp[None]
    else:
        P, Q = gridgen.scenario_injections(g, Bn, seed)
    w = np.random.default_rng(6).uniform(0, 1, g.n)
    return sym, P, Q, w


def run(sym, g, P, Q, x, w, tol=1e-8, max_iter=20):
    from paper_1811_02512_amd.autograd import power_flow

    Pt = dev(P).requires_grad_(True)
    Qt = dev(Q).requires_grad_(True)
    xt = dev(x).requires_grad_(True)
    Vm0, Va0 = g.flat_start()
    r = dev(g.r) if x.ndim == 1 else dev(np.repeat(g.r[None], x.shape[0], 0))
    b = dev(g.b) if x.ndim == 1 else dev(np.repeat(g.b[None], x.shape[0], 0))
    Vm, Va = power_flow(sym, Pt, Qt, xt, r, b, dev(g.bus_type.astype(np.int8)), dev(Vm0),
                        dev(Va0), tol, max_iter)
    wt = dev(w)
    pq = dev((g.bus_type == gridgen.BUS_PQ).astype(np.float64))
    loss = (wt * pq * (Vm - 1.0) ** 2).sum()
    loss.backward()
    return loss.item(), Pt.grad.cpu().numpy(), Qt.grad.cpu().numpy(), xt.grad.cpu().numpy(), \
        Vm.detach().cpu().numpy(), Va.detach().cpu().numpy()


def loss_grad_vm(g, Vm, w):
    gv = 2 * w * (Vm - 1)
    gv[g.bus_type != gridgen.BUS_PQ] = 0
    return gv


@pytest.mark.parametrize("n,seed,Bn", [(200, 1, 1), (300, 2, 3)])
def test_adjoint_matches_oracle_dense(n, seed, Bn):
    from oracle import oracle as O

    g = grid(n, seed)
    sym, P, Q, w = setup(g, Bn, 2)
    _, gP, gQ, gx, Vm, Va = run(sym, g, P, Q, g.x, w)
    Y = O.grid_ybus(g)
    gx_ref = np.zeros(g.m)
    for c in range(Bn):
        rP, rQ, rx = O.adjoint_dense(g, Y, Vm[c], Va[c], loss_grad_vm(g, Vm[c], w), np.zeros(n))
        sc = max(np.abs(rP).max(), np.abs(rQ).max())
        np.testing.assert_allclose(gP[c], rP, rtol=0, atol=1e-9 * sc)
        np.testing.assert_allclose(gQ[c], rQ, rtol=0, atol=1e-9 * sc)
        gx_ref += rx
    np.testing.assert_allclose(gx, gx_ref, rtol=0, atol=1e-9 * np.abs(gx_ref).max())


@pytest.mark.parametrize("n,seed,Bn", [(2000, 1, 4), (10000, 1, 2)])
def test_adjoint_matches_oracle_sparse(n, seed, Bn):
    from oracle import oracle as O

    log(f"[adjoint] n={n} B={Bn}")
    g = grid(n, seed)
    sym, P, Q, w = setup(g, Bn, 5)
    _, gP, gQ, gx, Vm, Va = run(sym, g, P, Q, g.x, w)
    osym = O.Sym(g.n, g.f, g.t)
    Y = O.grid_ybus(g)
    gx_ref = np.zeros(g.m)
    for c in range(Bn):
        ref = osym.newton(Y, g.bus_type, P[c], Q[c], *g.flat_start())
        np.testing.assert_allclose(Vm[c], ref.Vm, atol=1e-9)
        rP, rQ, rx = osym.adjoint(g, Y, Vm[c], Va[c], loss_grad_vm(g, Vm[c], w), np.zeros(n))
        sc = max(np.abs(rP).max(), np.abs(rQ).max())
        np.testing.assert_allclose(gP[c], rP, rtol=0, atol=1e-8 * sc)
        np.testing.assert_allclose(gQ[c], rQ, rtol=0, atol=1e-8 * sc)
        gx_ref += rx
    np.testing.assert_allclose(gx, gx_ref, rtol=0, atol=1e-8 * np.abs(gx_ref).max())


def test_adjoint_per_case_branch_x():
    from oracle import oracle as O

    g = grid(150, 4)
    sym, P, Q, w = setup(g, 2, 3)
    xs = g.x[None] * np.random.default_rng(2).uniform(0.9, 1.1, (2, g.m))
    _, gP, gQ, gx, Vm, Va = run(sym, g, P, Q, xs, w)
    assert gx.shape == (2, g.m)
    for c in range(2):
        Y = O.ybus(g.n, g.f, g.t, g.r, xs[c], g.b)
        _, _, rx = O.adjoint_dense(g, Y, Vm[c], Va[c], loss_grad_vm(g, Vm[c], w), np.zeros(g.n),
                                   x=xs[c])
        np.testing.assert_allclose(gx[c], rx, rtol=0, atol=1e-9 * np.abs(rx).max())


def test_adjoint_central_fd():
    g = grid(60, 7)
    sym, P, Q, w = setup(g, 1, 0)
    tol = 1e-12
    _, gP, gQ, gx, _, _ = run(sym, g, P, Q, g.x, w, tol, 40)
    h = 1e-6

    def L(P_, Q_, x_):
        return run(sym, g, P_, Q_, x_, w, tol, 40)[0]

    # central differences carry O(h^2) truncation and O(eps L / h) rounding
    # error, so each entry is checked to 1e-5 of the gradient's largest entry
    sP = np.abs(gP).max()
    sQ = np.abs(gQ).max()
    sx = np.abs(gx).max()
    for i in (3, 17, 41):
        e = np.zeros_like(P)
        e[0, i] = h
        fd = (L(P + e, Q, g.x) - L(P - e, Q, g.x)) / (2 * h)
        assert abs(gP[0, i] - fd) <= 1e-5 * sP, (i, gP[0, i], fd)
        fd = (L(P, Q + e, g.x) - L(P, Q - e, g.x)) / (2 * h)
        assert abs(gQ[0, i] - fd) <= 1e-5 * sQ, (i, gQ[0, i], fd)
    for k in (0, 25, 70):
        e = np.zeros(g.m)
        e[k] = h
        fd = (L(P, Q, g.x + e) - L(P, Q, g.x - e)) / (2 * h)
        assert abs(gx[k] - fd) <= 1e-5 * sx, (k, gx[k], fd)
