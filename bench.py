"""Benchmark: batched Newton-Raphson AC power flow with adjoint on MI355X.

Headline workload (one "step" = the whole hot path over one batch):
  10,000-bus synthetic grid (seed 1), 256 seeded load scenarios (seed 5):
  admittance assembly -> batched NR to 1e-8 p.u. keeping the factors at the
  solution -> adjoint backward (gather dL/dx, transposed level-scheduled
  solves, injection and branch gradients) for loss = sum_i w_i (|V_i| - 1)^2.
value = cases per second, each case solved to 1e-8 p.u. with its gradient.

Every other configuration is a leg of the same default run, each timed on
the device and each checked against the CPU oracle on a seeded subset of its
cases outside the timed region:
  c1  200-bus grid, one case per launch
  c2  10,000-bus grid, one case per launch, with factor and solve time per
      Newton iteration and their bandwidth
  c3  2,000-bus grid x 1,024 load scenarios, one shared analysis, autotuned
  c4  10,000-bus grid x 512 N-1 outages (each re-analysed) and 64 grids of
      500-20,000 buses, each in one launch
  c5  the headline, also through the torch.autograd.Function
plus the fast decoupled method, the step replayed from a HIP graph, N-1
screening on the base pattern, WLS state estimation, and the CPU oracle on
the host's cores.  --legs selects legs (e.g. --legs c1,c2 for profiling).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = tuple("paper_1811_02512_amd/csrc/" + f for f in (
    "pf_abi.hip", "pf_newton.hip", "pf_fdpf.hip", "pf_se.hip", "pf_device.h", "pf_host.h",
    "pf_kernels.h", "pf_internal.h", "analyze.cpp"))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_newton_10k_x256_hbm_traffic.md")
ALL_LEGS = ("c5", "c1", "c2", "c3", "c4", "fdpf", "graph", "screen", "se")
HOST_THREADS = 16  # the GPU machine's CPU share; also the oracle's thread pool


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_threads():
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(avail, HOST_THREADS))


def newton_bytes_per_iter(info):
    """Algorithmic bytes per NR iteration per case: 16 Y + 128 F + 96 n with
    Y = admittance entries, F = nn + 2 nnz(L) filled 2x2 blocks."""
    F = info.nn + 2 * info.nnz_l
    return 16 * info.nnz_y + 128 * F + 96 * info.n


def filled_blocks(info):
    return info.nn + 2 * info.nnz_l


def kept_factor_bytes(info):
    """The factorisation at the converged state that the launch adds per case
    when it keeps the factors for the adjoint, priced with the iteration's
    own terms less the substitutions and the vectors: 16 Y (admittances read
    for the Jacobian) + 32 F (Jacobian into the filled slots) + 64 F (factor
    read and write)."""
    return 16 * info.nnz_y + 96 * filled_blocks(info)


def adjoint_bytes(info):
    """Fused adjoint kernel per case: the factors read once (32 F), the
    gradient gathered (16 n), lam written (16 nn) and dL/dP, dL/dQ written
    (16 n)."""
    return 32 * filled_blocks(info) + 32 * info.n + 16 * info.nn


def branch_grad_bytes(info):
    """Branch gradients inside the adjoint launch, per case: |V| and theta
    read (16 n), the per-case dL/dx written and read back by the sum over
    cases (16 m); r, x shared."""
    return 16 * info.n + 16 * info.m


def timed(fn, steps, warmup):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def roofline(bytes_per_launch, ms, name, units, per_unit, traffic=None):
    gbs = bytes_per_launch / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "kernel": name,
            "algorithmic_bytes_per_launch": bytes_per_launch, "units_per_launch": units,
            "bytes_per_unit": per_unit, "kernel_ms": ms}


def check_cases(results):
    """Summary of per-case oracle comparisons (iters_equal, dV, dtheta[, dgrad])."""
    out = {"cases": len(results),
           "iterations_equal": bool(all(r[0] for r in results)),
           "max_abs_dV": float(max(r[1] for r in results)),
           "max_abs_dtheta": float(max(r[2] for r in results))}
    if results and len(results[0]) > 3:
        out["max_rel_dgrad"] = float(max(r[3] for r in results))
    ok = out["iterations_equal"] and out["max_abs_dV"] < 1e-9 and out["max_abs_dtheta"] < 1e-9
    if "max_rel_dgrad" in out:
        ok = ok and out["max_rel_dgrad"] < 1e-8
    out["pass"] = bool(ok)
    if not ok:
        raise AssertionError(f"oracle check failed: {out}")
    return out


def pick_cases(B, k, seed):
    rng = np.random.default_rng(seed)
    return sorted(int(c) for c in rng.choice(B, min(k, B), replace=False))


class Workload:
    """One grid with B load scenarios staged on the device, plus the buffers
    of the batched step (symbolic tuned for the batch) and of one case per
    launch (symbolic tuned for a single case)."""

    def __init__(self, n, seed, scen, scen_seed, load_scale=0.1):
        import torch

        import gridgen
        from paper_1811_02512_amd import api

        t0 = time.time()
        self.g = g = gridgen.make_grid(n, seed, load_scale=load_scale)
        self.P, self.Q = gridgen.scenario_injections(g, scen, scen_seed)
        self.w = np.random.default_rng(6).uniform(0, 1, g.n)
        t1 = time.time()
        self.sym = api.Symbolic(g.n, g.f, g.t).upload()   # tuned for the batch
        self.sym1 = api.Symbolic(g.n, g.f, g.t).upload()  # tuned for one case per launch
        t2 = time.time()
        log(f"[bench] grid n={n} m={g.m} generated in {t1 - t0:.1f}s, analysed+uploaded in "
            f"{t2 - t1:.3f}s")
        dev = torch.device("cuda")

        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

        self.t = t
        self.B = scen
        self.info = self.sym.info
        self.r, self.x, self.b = t(g.r), t(g.x), t(g.b)
        self.type = t(g.bus_type.astype(np.int8))
        self.Pt, self.Qt = t(self.P), t(self.Q)
        Vm0, Va0 = g.flat_start()
        self.Vm0, self.Va0 = t(Vm0), t(Va0)
        self.wt = t(self.w)
        self.pq = t((g.bus_type == 1).astype(np.float64))
        self.gcoef = self.wt * self.pq * 2.0  # dLoss/d|V| = gcoef (|V| - 1)
        info = self.info
        Bn = scen
        f64 = dict(dtype=torch.float64, device=dev)
        self.yval = torch.empty(1, 2 * info.nnz_y, **f64)
        self.Vm = torch.empty(Bn, g.n, **f64)
        self.Va = torch.empty_like(self.Vm)
        self.ws = self.sym.workspace(Bn)
        self.it = torch.empty(Bn, dtype=torch.int32, device=dev)
        self.nrm = torch.empty(Bn, **f64)
        self.st = torch.empty(Bn, dtype=torch.int32, device=dev)
        self.lam = torch.empty(Bn, 2 * info.nn, **f64)
        self.gP = torch.empty(Bn, g.n, **f64)
        self.gQ = torch.empty_like(self.gP)
        self.gx = torch.empty(g.m, **f64)
        self.gVm = torch.empty_like(self.Vm)

    def autotune(self, Bn, sym):
        from paper_1811_02512_amd import autotune

        g = self.g
        V0 = self.Vm0.expand(Bn, g.n).contiguous()
        A0 = self.Va0.expand(Bn, g.n).contiguous()
        res = autotune.tune(sym, self.yval[0], self.type, self.Pt[:Bn].contiguous(),
                            self.Qt[:Bn].contiguous(), V0, A0)
        log(f"[bench] autotune n={g.n} B={Bn}: T={res['threads']} tail={res['tail_budget']} "
            f"C={res['interleave']} spread={res['spread']} best {res['ms']:.3f} ms, "
            f"{res['launches']} launches in "
            f"{res['seconds']:.1f}s")
        self.info = self.sym.info
        if sym is self.sym:
            self.ws = self.sym.workspace(self.B)
        return res

    def step(self, ev=None, adjoint=True, Bn=None):
        """One pass of the hot path.  ev: optional dict of (start, end) event
        pairs around the Newton kernel ('newton') and the fused adjoint call
        ('adjoint': the adjoint kernel with the per-case branch gradients and
        their sum over cases), each recorded on the stream its kernels run on
        (the current stream)."""
        import torch

        from paper_1811_02512_amd import binding as B

        g = self.g
        Bn = self.B if Bn is None else Bn
        sym = self.sym if Bn > 1 else self.sym1
        info = sym.info
        B.pf_build_ybus(sym.h, 1, self.r, self.x, self.b, 0, self.yval, 2 * info.nnz_y)
        self.Vm[:Bn].copy_(self.Vm0.expand(Bn, g.n))
        self.Va[:Bn].copy_(self.Va0.expand(Bn, g.n))
        if ev is not None:
            ev["newton"][0].record()
        B.pf_newton(sym.h, Bn, self.yval, 0, self.type, 0, self.Pt, self.Qt, g.n, self.Vm,
                    self.Va, g.n, 1e-8, 20, B.PF_NEWTON_KEEP_FACTORS if adjoint else 0,
                    self.ws, info.ws_doubles, self.it, self.nrm, self.st)
        if ev is not None:
            ev["newton"][1].record()
        if not adjoint:
            return
        # dLoss/d|V| of the caller's loss, written by the caller in torch
        torch.sub(self.Vm[:Bn], 1.0, out=self.gVm[:Bn]).mul_(self.gcoef)
        if ev is not None:
            ev["adjoint"][0].record()
        B.pf_adjoint(sym.h, Bn, self.ws, info.ws_doubles, self.gVm, None, g.n, self.type, 0,
                     self.Vm, self.Va, g.n, self.r, self.x, 0, self.st, self.lam, 2 * info.nn,
                     self.gP, self.gQ, g.n, self.gx, 1)
        if ev is not None:
            ev["adjoint"][1].record()

    def oracle_check(self, cases, adjoint):
        """Per-case comparison of the last step's results with the oracle's
        sparse NR (and sparse adjoint) on the same inputs, in threads."""
        from oracle import oracle as O

        g = self.g
        Y = O.grid_ybus(g)
        osym = O.Sym(g.n, g.f, g.t)
        Vm, Va = self.Vm.cpu().numpy(), self.Va.cpu().numpy()
        it = self.it.cpu().numpy()
        gP, gQ = self.gP.cpu().numpy(), self.gQ.cpu().numpy()
        Vm0, Va0 = g.flat_start()

        def one(c):
            r = osym.newton(Y, g.bus_type, self.P[c], self.Q[c], Vm0, Va0)
            res = [r.status == 0 and r.iters == it[c], float(np.abs(r.Vm - Vm[c]).max()),
                   float(np.abs(r.Va - Va[c]).max())]
            if adjoint:
                gv = 2 * self.w * (Vm[c] - 1) * (g.bus_type == 1)
                oP, oQ, _ = osym.adjoint(g, Y, Vm[c], Va[c], gv, np.zeros(g.n))
                sc = max(np.abs(oP).max(), np.abs(oQ).max())
                res.append(float(max(np.abs(oP - gP[c]).max(), np.abs(oQ - gQ[c]).max()) / sc))
            return res

        with ThreadPoolExecutor(host_threads()) as ex:
            return check_cases(list(ex.map(one, cases)))


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(settings):
    """HBM bytes per launch of the batched Newton kernel from the committed
    PMC summary, or None when the kernel sources or the launch settings have
    changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    for line in open(TRAFFIC_FILE):
        if line.startswith("traffic:"):
            for kv in line.split()[1:]:
                k, v = kv.split("=")
                rec[k] = v
    if rec.get("sources") != kernel_source_hash():
        return None
    if settings is None or rec.get("launch") != launch_tag(settings):
        return None
    return float(rec["bytes_per_launch"])


def launch_tag(s):
    return f"T{s['threads']}-tail{s['tail_budget']}-C{s['interleave']}"


def copy_calibration():
    """One plain 1 GiB device copy (1 GiB read, 1 GiB written): the reference
    for scaling the FETCH_SIZE / WRITE_SIZE counters of a PMC pass."""
    import torch

    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    log("[bench] copy calibration: 1 GiB copied")


def copy_bandwidth():
    """Measured device copy rate (GB/s, bytes read + written) of a 1 GiB
    device-to-device copy, the practical ceiling beside the nominal peak."""
    import torch

    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    ms = timed(lambda: b.copy_(a), 5, 2)
    del a, b
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def host_cpu():
    """Model name and logical core count of the host the oracle runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


# ---------------------------------------------------------------------------
# legs
# ---------------------------------------------------------------------------
def leg_headline(W, args, tuned):
    """C5: Ybus + batched NR keeping the factors + fused adjoint, 10k x 256."""
    import torch

    info = W.info
    names = ("newton", "adjoint")
    evs = [{k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for k in names} for _ in range(args.steps)]
    for _ in range(args.warmup):
        W.step()
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record()
    for k in range(args.steps):
        W.step(evs[k])
    t_end.record()
    torch.cuda.synchronize()
    ms_step = t_start.elapsed_time(t_end) / args.steps
    kms = {k: float(np.mean([e[k][0].elapsed_time(e[k][1]) for e in evs])) for k in names}
    iters = W.it.cpu().numpy()
    status = W.st.cpu().numpy()
    assert (status == 0).all(), f"non-converged cases: {np.unique(status, return_counts=True)}"
    check = W.oracle_check(pick_cases(W.B, 16, 21), adjoint=True)
    log(f"[bench] c5 headline: {ms_step:.3f} ms/step, newton {kms['newton']:.3f} ms, adjoint "
        f"{kms['adjoint']:.3f} ms; oracle check {check}")
    b_it = newton_bytes_per_iter(info)
    units = float(iters.sum())
    kept = kept_factor_bytes(info) * W.B
    rf = roofline(b_it * units + kept, kms["newton"], "k_newton (batched launch)", units, b_it,
                  measured_traffic(tuned))
    rf["launch"] = None if tuned is None else launch_tag(tuned)
    rf["kept_factorisations"] = {"count": W.B, "bytes_each": kept_factor_bytes(info)}
    rf["frac_iterations_only"] = b_it * units / (kms["newton"] * 1e-3) / 1e9 / HBM_PEAK_GBS
    per_case = adjoint_bytes(info) + branch_grad_bytes(info)
    adj = {
        "pf_adjoint": roofline(per_case * W.B, kms["adjoint"],
                               "pf_adjoint: k_adjoint (gather, transposed solves, dL/dP, dL/dQ, "
                               "per-case dL/dx) + k_adj_gx_sum (dL/dx summed over cases)", W.B,
                               per_case),
    }
    return ms_step, iters, rf, adj, check, kms


def leg_autograd(W, steps):
    """The headline step through the product API: autograd.power_flow (its
    own Ybus, workspace and output buffers per call) and loss.backward()."""
    import torch

    from paper_1811_02512_amd.autograd import power_flow

    g = W.g
    P = W.Pt.clone().requires_grad_(True)
    Q = W.Qt.clone().requires_grad_(True)
    x = W.x.clone().requires_grad_(True)
    box = {}

    def step():
        P.grad = Q.grad = x.grad = None
        Vm, Va = power_flow(W.sym, P, Q, x, W.r, W.b, W.type, W.Vm0, W.Va0)
        loss = (W.wt * W.pq * (Vm - 1.0) ** 2).sum()
        loss.backward()
        box["Vm"] = Vm

    ms = timed(step, steps, 1)
    # same answers as the direct-ABI step
    dv = float((box["Vm"].detach() - W.Vm).abs().max().item())
    dg = float((P.grad - W.gP).abs().max().item() / W.gP.abs().max().item())
    dx = float((x.grad - W.gx).abs().max().item() / W.gx.abs().max().item())
    log(f"[bench] c5 through torch.autograd: {ms:.3f} ms/step; vs direct ABI: dV {dv:.1e}, "
        f"dgP {dg:.1e}, dgx {dx:.1e}")
    assert dv < 1e-12 and dg < 1e-12 and dx < 1e-12
    return dict(solves_per_s=W.B / ms * 1e3, ms_per_step=ms,
                max_diff_vs_direct_abi={"Vm": dv, "gP_rel": dg, "gx_rel": dx},
                step="power_flow(...) (Ybus, NR keeping the factors) + loss.backward() "
                     "(pf_adjoint, branch gradients), buffers allocated per call by torch")


def leg_plain(W, steps, label, adjoint=False):
    """One case per launch on W's grid: ms per solve and per iteration, and a
    comparison with the oracle; with adjoint, also one case per launch with
    its gradient (the headline step at B = 1)."""
    ms = timed(lambda: W.step(adjoint=False, Bn=1), steps, 1)
    it = int(W.it[0].item())
    assert int(W.st[0].item()) == 0
    from oracle import oracle as O

    ref = O.solve_grid(W.g, Psp=W.P[0], Qsp=W.Q[0])
    Vm, Va = W.Vm[0].cpu().numpy(), W.Va[0].cpu().numpy()
    check = check_cases([(ref.iters == it, float(np.abs(ref.Vm - Vm).max()),
                          float(np.abs(ref.Va - Va).max()))])
    info1 = W.sym1.info
    spread = int(info1.spread)
    syncs = sync_counts(W.sym1, spread)
    log(f"[bench] {label} one case per launch: {ms * 1e3:.1f} us/solve, {it} iterations, "
        f"{ms * 1e3 / max(it, 1):.1f} us/iteration, spread over {max(spread, 1)} workgroups, "
        f"{syncs}")
    if spread > 1:
        launches = (3, f"k_ybus + k_spread_init + k_newton_spread (the whole NR loop in one "
                       f"cooperative launch of {spread} workgroups); two 16n-byte device copies "
                       f"of the flat start")
    else:
        launches = (2, "k_ybus + k_newton (the whole NR loop in one launch); two 16n-byte "
                       "device copies of the flat start")
    out = dict(solves_per_s=1e3 / ms, ms_per_solve=ms, us_per_iteration=ms * 1e3 / max(it, 1),
               iterations=it, workgroups=max(spread, 1), kernel_launches_per_solve=launches[0],
               launches=launches[1], syncs_per_iteration=syncs, oracle_check=check)
    if adjoint:
        ms_adj = timed(lambda: W.step(adjoint=True, Bn=1), steps, 1)
        assert int(W.st[0].item()) == 0
        check_adj = W.oracle_check([0], adjoint=True)
        log(f"[bench] {label} one case per launch with its gradient: {ms_adj * 1e3:.1f} us "
            f"(oracle check {check_adj})")
        out["with_adjoint"] = dict(grads_per_s=1e3 / ms_adj, ms_per_solve=ms_adj,
                                   step="Ybus + NR keeping the factors + pf_adjoint, one case",
                                   oracle_check=check_adj)
    return out


def sync_counts(sym, spread):
    """Barriers of one NR iteration of a one-case Newton launch, from the
    partition: on one workgroup a workgroup barrier per level step (the
    mismatch, every factorisation and backward level); spread, a grid barrier
    after the mismatch, after each level below the LDS tail in the
    factorisation and after each wide one in the backward sweep, and three
    around the tail (its shared first pass, its factorisation, its backward
    substitution together with the narrow global backward levels).  A
    one-case launch shares its subtree levels too (only the groups of a
    batch of grids run those per workgroup)."""
    info = sym.info
    widths = np.diff(sym.export()["level_ptr"])
    nlev = int(info.nlevels)
    below = nlev - int(info.tail_levels)
    if spread <= 1:
        return {"workgroup_barriers": 1 + 2 * nlev, "grid_barriers": 0}
    threads = int(info.threads) or 512
    back_lo = below
    while back_lo > 0 and widths[back_lo - 1] <= threads:
        back_lo -= 1
    # the tail's three, or without a tail the one after the narrow backward
    # levels on workgroup 0
    tail = 3 if info.tail_nodes > 0 else int(back_lo < below)
    return {"grid_barriers": 1 + below + tail + back_lo,
            "levels_on_workgroup_0": int(info.tail_levels) * 2 + (below - back_lo)}


def leg_c2_breakdown(W, steps):
    """10k single case: the Jacobian at flat start factorised (pf_factor) and
    solved (pf_solve) alone, one case per launch on one workgroup (the
    batch's launch shape), with their bandwidth."""
    import torch

    from paper_1811_02512_amd import binding as B

    sym, info, g = W.sym, W.sym.info, W.g
    f64 = dict(dtype=torch.float64, device="cuda")
    J = torch.zeros(1, info.vals_doubles, **f64)
    B.pf_build_ybus(sym.h, 1, W.r, W.x, W.b, 0, W.yval, 2 * info.nnz_y)
    B.pf_jacobian(sym.h, 1, W.yval, 0, W.type, 0, W.Vm0, W.Va0, 0, J, info.vals_doubles)
    vals = J.clone()
    rhs0 = torch.ones(1, 2 * info.nn, **f64)
    rhs = rhs0.clone()
    st = torch.empty(1, dtype=torch.int32, device="cuda")

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps + 1)]
    for e0, e1 in evs:  # the first pair warms up
        vals.copy_(J)
        e0.record()
        B.pf_factor(sym.h, 1, vals, info.vals_doubles, st)
        e1.record()
    torch.cuda.synchronize()
    fac_ms = float(np.mean([a.elapsed_time(b) for a, b in evs[1:]]))
    assert st.item() == 0
    sol_ms = timed(lambda: B.pf_solve(sym.h, 1, vals, info.vals_doubles, rhs, 2 * info.nn, 0),
                   steps, 1)
    F = filled_blocks(info)
    fb, sb = 64 * F, 32 * F + 32 * info.nn
    log(f"[bench] c2 single case: factor {fac_ms * 1e3:.1f} us, solve {sol_ms * 1e3:.1f} us "
        f"(F = {F} blocks)")
    return dict(factor_us=fac_ms * 1e3, solve_us=sol_ms * 1e3,
                factor_gbs=fb / (fac_ms * 1e-3) / 1e9, solve_gbs=sb / (sol_ms * 1e-3) / 1e9,
                factor_bytes=fb, solve_bytes=sb, levels=int(info.nlevels),
                note="one workgroup per case: each of the levels is a barrier-separated "
                     "chain of dependent loads, so these are latency figures; the bandwidth "
                     "is far below HBM by construction")


def leg_c3(args, tuned_file):
    """C3: 2,000-bus grid x 1,024 load scenarios, shared analysis, tuned."""
    W2 = Workload(2000, 1, 1024, 2)
    W2.step(adjoint=False)
    if tuned_file is None and not args.no_tune:
        W2.autotune(W2.B, W2.sym)
        W2.autotune(1, W2.sym1)
    ms = timed(lambda: W2.step(adjoint=False), max(3, args.steps // 2), 1)
    assert (W2.st.cpu().numpy() == 0).all()
    its = W2.it.cpu().numpy()
    check = W2.oracle_check(pick_cases(W2.B, 16, 22), adjoint=False)
    plain = leg_plain(W2, max(3, args.steps // 2), "c3 2k")
    graph = leg_graph(W2, max(3, args.steps // 2), adjoint=False)
    info = W2.sym.info
    b_it = newton_bytes_per_iter(info)
    log(f"[bench] c3 2k x 1024: {ms:.3f} ms/launch")
    return dict(solves_per_s=W2.B / ms * 1e3, ms_per_step=ms, cases=W2.B, graph_replay=graph,
                mean_iterations=float(its.mean()),
                speedup_vs_plain=(W2.B / ms) / plain["solves_per_s"] * 1e3,
                plain_solves_per_s=plain["solves_per_s"],
                hbm_frac=b_it * float(its.sum()) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                oracle_check=check,
                step="Ybus + batched NR to 1e-8 (k_newton, one launch)")


def bench_multi(grids, label, steps, check_idx, spreads=(0,), launches=((0, 161792),)):
    """One launch over cases with their own analyses; timing, host analysis
    time and an oracle check of the cases in check_idx.  spreads: workgroup
    totals of the launch to try (0: one per case); launches: (threads, LDS
    budget) settings of the symbolics to try; the fastest pair is kept."""
    import torch

    from oracle import oracle as O
    from paper_1811_02512_amd import api
    from paper_1811_02512_amd import binding as B

    t0 = time.time()
    with ThreadPoolExecutor(host_threads()) as ex:
        syms = list(ex.map(lambda g: api.Symbolic(g.n, g.f, g.t), grids))
    t_an = time.time() - t0

    def make_plan(launch):
        for s in syms:
            s.set_launch(*launch)
            s.upload()
        return api.MultiPlan(syms)

    plan = make_plan(launches[0])
    f64 = np.float64
    r = plan.concat([g.r for g in grids], "branch", f64)
    x = plan.concat([g.x for g in grids], "branch", f64)
    b = plan.concat([g.b for g in grids], "branch", f64)
    yv = torch.empty(int(plan.offs["y"][-1]) + 2, dtype=torch.float64, device="cuda")
    ty = plan.concat([g.bus_type for g in grids], "bus", np.int8)
    P = plan.concat([g.Psp for g in grids], "bus", f64)
    Q = plan.concat([g.Qsp for g in grids], "bus", f64)
    V0 = plan.concat([g.flat_start()[0] for g in grids], "bus", f64)
    A0 = plan.concat([g.flat_start()[1] for g in grids], "bus", f64)
    Vm, Va = V0.clone(), A0.clone()
    ws = torch.empty(int(plan.offs["ws"][-1]) + 32, dtype=torch.float64, device="cuda")
    G = len(grids)
    it = torch.empty(G, dtype=torch.int32, device="cuda")
    st = torch.empty(G, dtype=torch.int32, device="cuda")

    def step():
        B.pf_build_ybus_multi(plan.p, r, x, b, yv)
        Vm.copy_(V0)
        Va.copy_(A0)
        B.pf_newton_multi(plan.p, yv, ty, P, Q, Vm, Va, 1e-8, 20, 0, ws, it, None, st)

    tried = {}
    for li, launch in enumerate(launches):
        if li:
            plan = make_plan(launch)
        for sp in spreads:
            plan.set_spread(sp)
            tried[(launch, sp)] = timed(step, steps, 1)
    (best_launch, best), _ = min(tried.items(), key=lambda kv: kv[1])
    if best_launch != launches[-1]:
        plan = make_plan(best_launch)
    plan.set_spread(best)
    ms = timed(step, steps, 1)
    sts = st.cpu().numpy()
    its = it.cpu().numpy()
    ok = int((sts == 0).sum())
    Vms, Vas = plan.split(Vm, "bus"), plan.split(Va, "bus")

    def one(c):
        ref = O.solve_grid(grids[c])
        return (ref.status == 0 and sts[c] == 0 and ref.iters == its[c],
                float(np.abs(ref.Vm - Vms[c]).max()), float(np.abs(ref.Va - Vas[c]).max()))

    with ThreadPoolExecutor(host_threads()) as ex:
        check = check_cases(list(ex.map(one, check_idx)))
    log(f"[bench] {label}: {G} cases, {ms:.2f} ms/launch, converged {ok}/{G}, host analysis "
        f"{t_an:.2f}s; workgroups {max(best, G)}, launch {best_launch} (tried "
        f"{ {f'{k[0]} x {max(k[1], G)}': round(v, 3) for k, v in tried.items()} }); "
        f"oracle check {check}")
    # only converged cases count as solves
    return dict(solves_per_s=ok / ms * 1e3, ms=ms, cases=G, converged=ok,
                workgroups=max(best, G), threads_and_lds_budget=list(best_launch),
                ms_tried={f"threads {k[0][0] or 'auto'}, lds {k[0][1]}, workgroups "
                          f"{max(k[1], G)}": v for k, v in tried.items()},
                host_analysis_s=t_an, host_threads=host_threads(),
                solves_per_s_with_host_analysis=ok / (ms * 1e-3 + t_an),
                buses=int(sum(g.n for g in grids)),
                bus_solves_per_s=sum(g.n for g, s in zip(grids, sts.tolist()) if s == 0) / ms * 1e3,
                oracle_check=check)


def leg_c4(W, args):
    import gridgen

    out = {}
    outs = gridgen.n1_outages(W.g, 512, 3)
    n1 = [W.g.without_branch(int(e)) for e in outs]
    out["n1_10k_x512"] = bench_multi(n1, "c4 N-1 10k x 512", max(3, args.steps // 3),
                                     pick_cases(512, 16, 23))
    spec = json.load(open(os.path.join(ROOT, "tests", "golden", "mixed_batch.json")))
    t0 = time.time()
    jobs = [(gs["n"], gs["seed"], spec["load_scale"]) for gs in spec["grids"]]
    # spawned generator processes hold none of this process's GPU handles; at
    # most 15 of them beside this one
    mixed = gridgen.make_grids(jobs, processes=min(host_threads(), 15))
    log(f"[bench] c4 mixed: 64 grids generated in {time.time() - t0:.1f}s")
    largest = int(np.argmax([g.n for g in mixed]))
    idx = sorted(set(pick_cases(64, 8, 24)) | {largest})
    # 64 grids leave most CUs idle: the launch may give the largest grids
    # groups of workgroups (one per CU at most)
    out["mixed_64_grids"] = bench_multi(mixed, "c4 mixed 64 grids 500-20k buses",
                                        max(3, args.steps // 3), idx, spreads=(0, 128, 256))
    return out


def leg_graph(W, steps, adjoint=True):
    """The whole step (Ybus, batched NR, with adjoint: keeping the factors and
    the adjoint) captured once in a HIP graph and replayed; every replay's
    outputs are checked against the eager step's."""
    import torch

    W.step(adjoint=adjoint)
    torch.cuda.synchronize()
    outs = (W.Vm, W.Va, W.it) + ((W.gP, W.gx) if adjoint else ())
    ref = tuple(t.clone() for t in outs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        W.step(adjoint=adjoint)  # warm the allocator on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        W.step(adjoint=adjoint)
    for _ in range(2):
        graph.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(outs, ref)), \
            "graph replay differs from the eager step"
    ms = timed(graph.replay, steps, 1)
    log(f"[bench] graph replay of the step ({W.g.n} buses x {W.B}): {ms:.3f} ms")
    return dict(solves_per_s=W.B / ms * 1e3, ms_per_step=ms, replays_checked=2)


def leg_fdpf(W, steps):
    """Fast decoupled power flow on the workload's grid and scenarios: one
    step = B' and B'' built and factored once for the batch (shared
    impedances) + the batched decoupled iteration to 1e-8 + branch flows of
    every case.  Also the one-case-per-launch rate.  Both run with the
    batch's tuned launch shape (the one-case Newton tuning may pick a
    workgroup size chosen for its spread launch)."""
    import torch

    from oracle import oracle as O
    from paper_1811_02512_amd import binding as B

    g, sym, info = W.g, W.sym, W.sym.info
    Bn = W.B
    dev = W.Vm.device
    mat = torch.empty(1, info.fd_mat_doubles, dtype=torch.float64, device=dev)
    fst = torch.empty(1, dtype=torch.int32, device=dev)
    ws = torch.empty(Bn, info.fd_ws_doubles, dtype=torch.float64, device=dev)
    it = torch.empty(Bn, dtype=torch.int32, device=dev)
    st = torch.empty(Bn, dtype=torch.int32, device=dev)
    flows = [torch.empty(Bn, g.m, dtype=torch.float64, device=dev) for _ in range(4)]

    def step(b=Bn, with_flows=True):
        B.pf_build_ybus(sym.h, 1, W.r, W.x, W.b, 0, W.yval, 2 * info.nnz_y)
        B.pf_fdpf_matrices(sym.h, 1, W.r, W.x, W.b, 0, W.type, 0, mat, info.fd_mat_doubles)
        B.pf_fdpf_factor(sym.h, 1, mat, info.fd_mat_doubles, fst)
        W.Vm[:b].copy_(W.Vm0.expand(b, g.n))
        W.Va[:b].copy_(W.Va0.expand(b, g.n))
        B.pf_fdpf(sym.h, b, W.yval, 0, W.type, 0, W.Pt, W.Qt, g.n, W.Vm, W.Va, g.n, mat, 0,
                  1e-8, 40, ws, info.fd_ws_doubles, it, None, st)
        if with_flows:
            B.pf_branch_flows(sym.h, b, W.r, W.x, W.b, 0, W.Vm, W.Va, g.n, *flows, g.m)

    ms = timed(step, steps, 1)
    status = st.cpu().numpy()
    ok = int((status == 0).sum())
    iters = it.cpu().numpy()
    Vm, Va = W.Vm.cpu().numpy(), W.Va.cpu().numpy()
    osym = O.Sym(g.n, g.f, g.t)
    Y = O.grid_ybus(g)
    d1, a1, d2, a2 = osym.fdpf_matrices(g)
    f1, f2 = osym.factor1(d1, a1), osym.factor1(d2, a2)
    facs = (f1[:3], f2[:3])

    def one(c):
        r = osym.fdpf(Y, g, W.P[c], W.Q[c], *g.flat_start(), factors=facs)
        return (r.status == 0 and r.iters == iters[c], float(np.abs(r.Vm - Vm[c]).max()),
                float(np.abs(r.Va - Va[c]).max()))

    with ThreadPoolExecutor(host_threads()) as ex:
        check = check_cases(list(ex.map(one, pick_cases(Bn, 16, 25))))
    plain = timed(lambda: step(1, False), max(3, steps // 2), 1)
    log(f"[bench] fdpf {Bn} cases: {ms:.2f} ms/step, converged {ok}/{Bn}, mean iterations "
        f"{iters.mean():.2f}; one case {plain:.2f} ms; oracle check {check}")
    return dict(solves_per_s=ok / ms * 1e3, ms_per_step=ms, converged=ok, cases=Bn,
                mean_iterations=float(iters.mean()), plain_solves_per_s=1e3 / plain,
                plain_ms_per_solve=plain, oracle_check=check,
                step="Ybus + B', B'' built and factored once + batched decoupled iteration "
                     "to 1e-8 + branch flows")


def leg_screen(W, outages, steps=3):
    """N-1 screening on the base pattern (opened branches): fast decoupled
    first with NR fallback, and NR only, both with branch flows."""
    from paper_1811_02512_amd import contingency

    P0, Q0 = W.t(W.g.Psp), W.t(W.g.Qsp)
    out = {}
    for key, first in (("fdpf_first", True), ("nr_only", False)):
        box = {}

        def step():
            box["r"] = contingency.screen(W.sym, W.r, W.x, W.b, W.type, P0, Q0, W.Vm0, W.Va0,
                                          outages, fdpf_first=first)

        ms = timed(step, steps, 1)
        res = box["r"]
        ok = int((res.status == 0).sum().item())
        out[key] = dict(solves_per_s=ok / ms * 1e3, ms=ms, cases=len(outages), converged=ok,
                        solved_by_nr=res.fallback,
                        mean_iterations=float(res.iters.float().mean().item()))
        if first:
            out[key]["fallback_to_nr"] = res.fallback
        log(f"[bench] N-1 screen {key}: {len(outages)} outages, {ms:.2f} ms, converged {ok}, "
            f"solved by NR {res.fallback}")
    return out


def leg_se(W, cases=256, steps=3):
    """WLS state estimation on the workload's grid: the measurements are the
    NR solutions of the first `cases` load scenarios (|V|, P, Q at every bus,
    P, Q at the from end of every branch, all computed on the device) plus
    seeded Gaussian noise (sigma 0.004 for |V|, 0.01 otherwise).  One step =
    Gauss-Newton from a flat start to max|dx| < 1e-8 for every case."""
    import torch

    from paper_1811_02512_amd import api
    from paper_1811_02512_amd import binding as B

    g, sym, info = W.g, W.sym1, W.sym1.info
    n, m, dev = g.n, g.m, W.Vm.device
    W.step(adjoint=False)
    Vm, Va = W.Vm[:cases].clone(), W.Va[:cases].clone()
    PQ = torch.empty(cases, 2 * n, dtype=torch.float64, device=dev)
    rhs = torch.empty(cases, 2 * info.nn, dtype=torch.float64, device=dev)
    nrm = torch.empty(cases, dtype=torch.float64, device=dev)
    B.pf_mismatch(sym.h, cases, W.yval, 0, W.type, 0, W.Pt, W.Qt, n, Vm, Va, n, rhs,
                  2 * info.nn, nrm, PQ)
    fl = [torch.empty(cases, m, dtype=torch.float64, device=dev) for _ in range(4)]
    B.pf_branch_flows(sym.h, cases, W.r, W.x, W.b, 0, Vm, Va, n, *fl, m)
    PQ = PQ.view(cases, n, 2)
    h = torch.cat([Vm, PQ[..., 0], PQ[..., 1], fl[0], fl[1]], dim=1)
    kinds = np.concatenate([np.full(n, B.PF_MEAS_VM), np.full(n, B.PF_MEAS_P),
                            np.full(n, B.PF_MEAS_Q), np.full(m, B.PF_MEAS_PF),
                            np.full(m, B.PF_MEAS_QF)]).astype(np.int8)
    locs = np.concatenate([np.arange(n), np.arange(n), np.arange(n), np.arange(m),
                           np.arange(m)]).astype(np.int32)
    sig = torch.from_numpy(np.where(kinds == B.PF_MEAS_VM, 0.004, 0.01)).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    z = (h + sig * torch.randn(h.shape, generator=gen, dtype=torch.float64, device=dev))
    w = 1.0 / sig ** 2
    t0 = time.time()
    est = api.StateEstimator(n, g.f, g.t, kinds, locs, tail_lds_budget=161792)
    t_an = time.time() - t0
    d = est.dims
    ws = est.workspace(cases, dev)
    eVm = torch.empty_like(Vm)
    eVa = torch.empty_like(Va)
    box = {}

    def step():
        eVm.fill_(1.0)
        eVa.zero_()
        box["r"] = est.estimate(W.r, W.x, W.b, z, w, eVm, eVa, ws=ws)

    ms = timed(step, steps, 1)
    it, _, st, _ = box["r"]
    ok = int((st == 0).sum().item())
    mean_it = float(it.float().mean().item())
    err = float((eVm - Vm).abs().max().item())
    log(f"[bench] WLS SE {cases} cases x {len(kinds)} measurements: {ms:.2f} ms, converged "
        f"{ok}/{cases}, mean steps {mean_it:.2f}, gain levels {d.gain_levels}, "
        f"max |V| error vs the power-flow state {err:.2e}")
    return dict(estimates_per_s=ok / ms * 1e3, ms_per_step=ms, cases=cases, converged=ok,
                measurements=len(kinds), mean_gauss_newton_steps=mean_it,
                gain_nnz_l=int(d.gain_nnz_l), gain_levels=int(d.gain_levels),
                host_analysis_s=t_an, max_vm_error_vs_pf_state=err,
                step="Gauss-Newton WLS from a flat start to max|dx| < 1e-8 (Ybus, h and H, "
                     "gain assembly, level-scheduled factor and solve per step)")


def cpu_baseline(W, wall_s=15.0):
    """The oracle (paper-path sparse NR + sparse adjoint) over the load
    scenarios on a thread pool of the host's cores (ctypes releases the GIL),
    cycling through the scenarios until about `wall_s` seconds of wall time."""
    from oracle import oracle as O

    g = W.g
    Y = O.grid_ybus(g)
    osym = O.Sym(g.n, g.f, g.t)
    Vm0, Va0 = g.flat_start()
    cores = host_threads()

    def one(c):
        c %= W.B
        r = osym.newton(Y, g.bus_type, W.P[c], W.Q[c], Vm0, Va0)
        gVm = 2 * W.w * (r.Vm - 1) * (g.bus_type == 1)
        osym.adjoint(g, Y, r.Vm, r.Va, gVm, np.zeros(g.n))
        return r.status

    one(0)  # warm-up
    singles = []
    for c in range(1, 6):
        t0 = time.time()
        one(c)
        singles.append(time.time() - t0)
    per_case = float(np.median(singles))
    count = max(cores, int(wall_s * cores / max(per_case, 1e-6)))
    log(f"[bench] cpu baseline: {per_case * 1e3:.1f} ms per case on one thread, "
        f"{count} cases on {cores} threads")
    t0 = time.time()
    with ThreadPoolExecutor(cores) as ex:
        sts = list(ex.map(one, range(count)))
    wall = time.time() - t0
    model, nproc = host_cpu()
    return dict(value=count / wall, unit="solves/s", cores=cores, kind="oracle",
                single_thread_ms_per_solve=per_case * 1e3, host_cpu=model, host_nproc=nproc,
                sample=f"{count} solves cycling over the {W.B} load scenarios of the {g.n}-bus "
                       f"grid: forward NR (sparse paper path, tol 1e-8) + sparse adjoint each, "
                       f"{cores} threads, {wall:.1f}s wall, converged "
                       f"{sum(s == 0 for s in sts)}/{count}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--scenarios", type=int, default=256)
    ap.add_argument("--legs", default=",".join(ALL_LEGS),
                    help="comma-separated legs to run: " + ",".join(ALL_LEGS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--settings", help="JSON of launch settings saved by --save-settings "
                    "(applied instead of tuning)")
    ap.add_argument("--save-settings", help="write the tuned launch settings to this JSON file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB copy first (PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(cases are independent, so a multi-GPU run would shard the batch).",
              file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))
    unknown = legs - set(ALL_LEGS)
    if unknown:
        sys.exit(f"bench.py: unknown legs {sorted(unknown)}")

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_begin = time.time()
    if args.copy_calibration:
        copy_calibration()
    W = Workload(args.n, 1, args.scenarios, 5)
    W.step(adjoint=False)  # builds the admittance values the tuner needs
    tuned = tuned1 = None
    if args.settings:
        from paper_1811_02512_amd import autotune

        saved = json.load(open(args.settings))
        tuned, tuned1 = saved["batched"], saved["plain"]
        autotune.apply(W.sym, tuned)
        autotune.apply(W.sym1, tuned1)
        W.info = W.sym.info
        W.ws = W.sym.workspace(W.B)
        log(f"[bench] launch settings from {args.settings}: batched {launch_tag(tuned)}, "
            f"plain {launch_tag(tuned1)}")
    elif not args.no_tune:
        tuned = W.autotune(W.B, W.sym)
        tuned1 = W.autotune(1, W.sym1)
    if args.save_settings and tuned is not None:
        json.dump({"batched": tuned, "plain": tuned1}, open(args.save_settings, "w"))
    info = W.info

    out = {
        "metric": "NR power-flow solves/s to 1e-8 p.u. at 10k buses; batched & adjoint vs plain",
        "value": None, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": f"{info.n}-bus synthetic grid (m={info.m}), {W.B} load scenarios, "
                        "Ybus + batched NR to 1e-8 + adjoint backward per step",
            "buses": info.n, "branches": info.m, "scenarios": W.B,
            "nnz_l": int(info.nnz_l), "levels": int(info.nlevels),
        },
        "legs": sorted(legs),
    }
    if "c5" in legs:
        ms_step, iters, rf, adj, check, kms = leg_headline(W, args, tuned)
        out["value"] = W.B / ms_step * 1e3
        out["ms_per_step"] = ms_step
        out["config"]["mean_iterations"] = float(iters.mean())
        out["adjoint_grads_per_s"] = W.B / ms_step * 1e3
        out["kernel_ms"] = kms
        out["newton_kernel_ms"] = kms["newton"]
        out["oracle_check"] = check
        out["batched_fwd_solves_per_s"] = W.B / timed(lambda: W.step(adjoint=False),
                                                      max(3, args.steps // 2), 1) * 1e3
        out["autograd_10k_x256"] = leg_autograd(W, max(3, args.steps // 2))
        copy_gbs = copy_bandwidth()
        rf["copy_gbs"] = copy_gbs
        rf["frac_of_copy"] = rf["achieved"] / copy_gbs
        out["roofline"] = rf
        out["adjoint_roofline"] = adj
    if "c2" in legs or "c5" in legs:
        plain = leg_plain(W, max(3, args.steps // 2), "c2 10k", adjoint=True)
        out["plain_solves_per_s"] = plain["solves_per_s"]
        out["plain_ms_per_solve"] = plain["ms_per_solve"]
        out["plain_ms_per_iteration"] = plain["us_per_iteration"] * 1e-3
        out["plain_adjoint_grads_per_s"] = plain["with_adjoint"]["grads_per_s"]
        out["c2_plain_10k"] = plain
        if "c2" in legs:
            plain.update(leg_c2_breakdown(W, max(5, args.steps)))
    if "c1" in legs:
        W1 = Workload(200, 1, 4, 5)
        W1.step(adjoint=False)
        if not args.no_tune and args.settings is None:
            W1.autotune(1, W1.sym1)
        out["c1_plain_200"] = leg_plain(W1, max(20, args.steps * 2), "c1 200")
    if "c3" in legs:
        out["c3_2k_x1024"] = leg_c3(args, args.settings)
    if "c4" in legs:
        out.update({"c4_" + k: v for k, v in leg_c4(W, args).items()})
    if "fdpf" in legs:
        out["fdpf_10k_x256"] = leg_fdpf(W, max(3, args.steps // 2))
    if "graph" in legs:
        out["graph_replay"] = leg_graph(W, max(3, args.steps // 2))
    if "screen" in legs:
        import gridgen

        out["n1_screen_10k_x512"] = leg_screen(W, gridgen.n1_outages(W.g, 512, 3))
    if "se" in legs:
        out["wls_se_10k_x256"] = leg_se(W)
    out["autotune"] = None if tuned is None else {
        "batched": {k: tuned[k] for k in ("threads", "tail_budget", "interleave", "ms")},
        "plain": {k: tuned1.get(k, 0) for k in ("threads", "tail_budget", "interleave", "spread",
                                                 "ms")},
        "seconds": tuned["seconds"] + tuned1["seconds"], "from_file": bool(args.settings)}
    out["kernel_sources"] = kernel_source_hash()
    out["paper_context"] = ("Table III: graph-based NR 119.22 ms per solve on a 10790-bus "
                            "system, TigerGraph on 2x6-core x2-thread 2.10 GHz CPUs")
    if not args.no_cpu_baseline and "c5" in legs:
        out["cpu_baseline"] = cpu_baseline(W)
    out["bench_wall_s"] = time.time() - t_begin
    print(json.dumps(out))


if __name__ == "__main__":
    main()
