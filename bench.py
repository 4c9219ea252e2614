"""Benchmark: batched Newton-Raphson AC power flow with adjoint on MI355X.

Default workload (one "step" = the whole hot path over one batch):
  10,000-bus synthetic grid (seed 1), 256 seeded load scenarios (seed 5):
  admittance assembly -> batched NR to 1e-8 p.u. keeping the factors at the
  solution -> adjoint backward (gather dL/dx, transposed level-scheduled
  solves, parameter gradients) for loss = sum_i w_i (|V_i| - 1)^2.
value = cases per second, each case solved to 1e-8 p.u. with its gradient.

Also reported: the plain one-case-per-launch rate on the same grid, the
forward-only batched rate, the roofline of the Newton kernel and the CPU
oracle timed on the host's cores.  --full adds the 2,000-bus x 1,024
scenario batch, the 512 N-1 outages and the 64 mixed-size grids.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = tuple("paper_1811_02512_amd/csrc/" + f for f in (
    "pf_abi.hip", "pf_newton.hip", "pf_fdpf.hip", "pf_se.hip", "pf_device.h", "pf_host.h",
    "pf_kernels.h", "pf_internal.h", "analyze.cpp"))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_newton_10k_x256_hbm_traffic.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes_per_iter(info):
    """Algorithmic bytes per NR iteration per case: 16 Y + 128 F + 96 n with
    Y = admittance entries, F = nn + 2 nnz(L) filled 2x2 blocks."""
    F = info.nn + 2 * info.nnz_l
    return 16 * info.nnz_y + 128 * F + 96 * info.n


class Workload:
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
        info = self.info
        Bn = scen
        self.yval = torch.empty(1, 2 * info.nnz_y, dtype=torch.float64, device=dev)
        self.Vm = torch.empty(Bn, g.n, dtype=torch.float64, device=dev)
        self.Va = torch.empty_like(self.Vm)
        self.ws = self.sym.workspace(Bn)
        self.it = torch.empty(Bn, dtype=torch.int32, device=dev)
        self.nrm = torch.empty(Bn, dtype=torch.float64, device=dev)
        self.st = torch.empty(Bn, dtype=torch.int32, device=dev)
        self.lam = torch.empty(Bn, 2 * info.nn, dtype=torch.float64, device=dev)
        self.gP = torch.empty(Bn, g.n, dtype=torch.float64, device=dev)
        self.gQ = torch.empty_like(self.gP)
        self.gx = torch.empty(g.m, dtype=torch.float64, device=dev)
        self.gVa = torch.zeros_like(self.Vm)

    def autotune(self, Bn, sym):
        from paper_1811_02512_amd import autotune

        g = self.g
        V0 = self.Vm0.expand(Bn, g.n).contiguous()
        A0 = self.Va0.expand(Bn, g.n).contiguous()
        res = autotune.tune(sym, self.yval[0], self.type, self.Pt[:Bn].contiguous(),
                            self.Qt[:Bn].contiguous(), V0, A0)
        log(f"[bench] autotune B={Bn}: T={res['threads']} tail={res['tail_budget']} "
            f"C={res['interleave']} best {res['ms']:.3f} ms, {res['launches']} launches in "
            f"{res['seconds']:.1f}s")
        self.info = self.sym.info
        if sym is self.sym:
            self.ws = self.sym.workspace(self.B)
        return res

    def step(self, ev=None, adjoint=True, Bn=None):
        """One pass of the hot path.  ev: optional (start, end) events around
        the Newton kernel."""
        from paper_1811_02512_amd import binding as B

        g = self.g
        Bn = self.B if Bn is None else Bn
        sym = self.sym if Bn > 1 else self.sym1
        info = sym.info
        B.pf_build_ybus(sym.h, 1, self.r, self.x, self.b, 0, self.yval, 2 * info.nnz_y)
        self.Vm[:Bn].copy_(self.Vm0.expand(Bn, g.n))
        self.Va[:Bn].copy_(self.Va0.expand(Bn, g.n))
        if ev is not None:
            ev[0].record()
        B.pf_newton(sym.h, Bn, self.yval, 0, self.type, 0, self.Pt, self.Qt, g.n, self.Vm,
                    self.Va, g.n, 1e-8, 20, B.PF_NEWTON_KEEP_FACTORS if adjoint else 0,
                    self.ws, info.ws_doubles, self.it, self.nrm, self.st)
        if ev is not None:
            ev[1].record()
        if not adjoint:
            return
        gVm = 2.0 * self.wt * self.pq * (self.Vm[:Bn] - 1.0)  # dLoss/d|V| of the user's loss
        B.pf_adjoint_rhs(sym.h, Bn, gVm, self.gVa, g.n, self.type, 0, self.lam, 2 * info.nn)
        B.pf_solve(sym.h, Bn, self.ws, info.ws_doubles, self.lam, 2 * info.nn, 1,
                   B.pf_newton_interleave(sym.h, Bn))
        B.pf_adjoint_params(sym.h, Bn, self.lam, 2 * info.nn, self.type, 0, self.Vm, self.Va,
                            g.n, self.r, self.x, 0, self.gP, self.gQ, g.n, self.gx, 1)


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


def cpu_baseline(W, wall_s=15.0):
    """The oracle (paper-path sparse NR + sparse adjoint) over the load
    scenarios on a thread pool of the host's cores (ctypes releases the GIL),
    cycling through the scenarios until about `wall_s` seconds of wall time."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O

    g = W.g
    Y = O.grid_ybus(g)
    osym = O.Sym(g.n, g.f, g.t)
    Vm0, Va0 = g.flat_start()
    cores = min(os.cpu_count() or 1, 16)

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


def bench_graph(W, steps):
    """The whole step (Ybus, batched NR keeping the factors, adjoint) captured
    once in a HIP graph and replayed; every replay's outputs are checked
    against the eager step's."""
    import torch

    W.step()
    torch.cuda.synchronize()
    ref = (W.Vm.clone(), W.gP.clone(), W.gx.clone())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        W.step()  # warm the allocator on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        W.step()
    for _ in range(2):
        graph.replay()
        torch.cuda.synchronize()
        same = (torch.equal(W.Vm, ref[0]) and torch.equal(W.gP, ref[1])
                and torch.equal(W.gx, ref[2]))
        assert same, "graph replay differs from the eager step"
    ms = timed(graph.replay, steps, 1)
    log(f"[bench] graph replay of the step: {ms:.3f} ms")
    return dict(solves_per_s=W.B / ms * 1e3, ms_per_step=ms, replays_checked=2)


def bench_fdpf(W, steps):
    """Fast decoupled power flow on the workload's grid and scenarios: one
    step = B' and B'' built and factored once for the batch (shared
    impedances) + the batched decoupled iteration to 1e-8 + branch flows of
    every case.  Also the one-case-per-launch rate."""
    import torch

    from paper_1811_02512_amd import binding as B

    g, sym, info = W.g, W.sym1, W.sym1.info
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
    plain = timed(lambda: step(1, False), max(3, steps // 2), 1)
    log(f"[bench] fdpf {Bn} cases: {ms:.2f} ms/step, converged {ok}/{Bn}, mean iterations "
        f"{iters.mean():.2f}; one case {plain:.2f} ms")
    return dict(solves_per_s=ok / ms * 1e3, ms_per_step=ms, converged=ok, cases=Bn,
                mean_iterations=float(iters.mean()), plain_solves_per_s=1e3 / plain,
                plain_ms_per_solve=plain,
                step="Ybus + B', B'' built and factored once + batched decoupled iteration "
                     "to 1e-8 + branch flows")


def bench_screen(W, outages, steps=3):
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
                        fallback_to_nr=res.fallback,
                        mean_iterations=float(res.iters.float().mean().item()))
        log(f"[bench] N-1 screen {key}: {len(outages)} outages, {ms:.2f} ms, converged {ok}, "
            f"fallback {res.fallback}")
    return out


def bench_se(W, cases=256, steps=3):
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


def bench_multi(grids, label, steps=3):
    """One launch over cases with their own analyses; returns (solves/s, info)."""
    import torch

    from paper_1811_02512_amd import api
    from paper_1811_02512_amd import binding as B
    from concurrent.futures import ThreadPoolExecutor

    t0 = time.time()
    with ThreadPoolExecutor(min(os.cpu_count() or 1, 16)) as ex:
        syms = list(ex.map(lambda g: api.Symbolic(g.n, g.f, g.t), grids))
    t_an = time.time() - t0
    for s in syms:
        s.set_launch(0, 161792)  # the largest LDS tail: the launch waits for its largest grid
        s.upload()
    plan = api.MultiPlan(syms)
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
    G = len(grids)  # per-case patterns: plain (non-interleaved) workspace regions
    it = torch.empty(G, dtype=torch.int32, device="cuda")
    st = torch.empty(G, dtype=torch.int32, device="cuda")

    def step():
        B.pf_build_ybus_multi(plan.p, r, x, b, yv)
        Vm.copy_(V0)
        Va.copy_(A0)
        B.pf_newton_multi(plan.p, yv, ty, P, Q, Vm, Va, 1e-8, 20, 0, ws, it, None, st)

    ms = timed(step, steps, 1)
    ok = int((st == 0).sum().item())
    log(f"[bench] {label}: {G} cases, {ms:.2f} ms/launch, converged {ok}/{G}, host analysis "
        f"{t_an:.2f}s")
    # only converged cases count as solves
    return dict(solves_per_s=ok / ms * 1e3, ms=ms, cases=G, converged=ok,
                host_analysis_s=t_an,
                solves_per_s_with_host_analysis=ok / (ms * 1e-3 + t_an),
                buses=int(sum(g.n for g in grids)),
                bus_solves_per_s=sum(g.n for g, s in zip(grids, st.tolist()) if s == 0) / ms * 1e3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--scenarios", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--full", action="store_true")
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

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
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

    # --- timed steps: whole hot path ---------------------------------------------
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
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
    newton_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    iters = W.it.cpu().numpy()
    status = W.st.cpu().numpy()
    assert (status == 0).all(), f"non-converged cases: {np.unique(status, return_counts=True)}"

    # --- forward-only batched and plain one-case-per-launch rates ------------------
    fwd_ms = timed(lambda: W.step(adjoint=False), max(3, args.steps // 2), 1)
    plain_ms = timed(lambda: W.step(adjoint=False, Bn=1), max(3, args.steps // 2), 1)
    plain_iters = int(W.it[0].item())

    fdpf = bench_fdpf(W, max(3, args.steps // 2))
    graph = bench_graph(W, max(3, args.steps // 2))

    b_it = algorithmic_bytes_per_iter(info)
    units = float(iters.sum())
    alg_bytes = b_it * units  # per launch: bytes per case-iteration x case-iterations
    achieved = alg_bytes / (newton_ms * 1e-3) / 1e9
    traffic = measured_traffic(tuned)
    copy_gbs = copy_bandwidth()
    out = {
        "metric": "NR power-flow solves/s to 1e-8 p.u. at 10k buses; batched & adjoint vs plain",
        "value": W.B / ms_step * 1e3,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{info.n}-bus synthetic grid (m={info.m}), {W.B} load scenarios, "
                        "Ybus + batched NR to 1e-8 + adjoint backward per step",
            "buses": info.n, "branches": info.m, "scenarios": W.B,
            "nnz_l": int(info.nnz_l), "levels": int(info.nlevels),
            "mean_iterations": float(iters.mean()),
        },
        "batched_fwd_solves_per_s": W.B / fwd_ms * 1e3,
        "plain_solves_per_s": 1e3 / plain_ms,
        "plain_ms_per_solve": plain_ms,
        "plain_ms_per_iteration": plain_ms / max(plain_iters, 1),
        "adjoint_grads_per_s": W.B / ms_step * 1e3,
        "newton_kernel_ms": newton_ms,
        "autotune": None if tuned is None else {
            "batched": {k: tuned[k] for k in ("threads", "tail_budget", "interleave", "ms")},
            "plain": {k: tuned1[k] for k in ("threads", "tail_budget", "interleave", "ms")},
            "seconds": tuned["seconds"] + tuned1["seconds"],
            "from_file": bool(args.settings)},
        "kernel_sources": kernel_source_hash(),
        "fdpf_10k_x256": fdpf,
        "graph_replay": graph,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_newton (batched launch)",
            "algorithmic_bytes_per_launch": alg_bytes,
            "bytes_per_case_iteration": b_it,
            "case_iterations_per_launch": units,
            "launch": None if tuned is None else launch_tag(tuned),
            "copy_gbs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
        },
        "paper_context": "Table III: graph-based NR 119.22 ms per solve on a 10790-bus system, "
                         "TigerGraph on 2x6-core x2-thread 2.10 GHz CPUs",
    }
    if args.full:
        import gridgen

        W2 = Workload(2000, 1, 1024, 2)
        W2.step(adjoint=False)
        if not args.no_tune:
            W2.autotune(W2.B, W2.sym)
            W2.autotune(1, W2.sym1)
        ms2 = timed(lambda: W2.step(adjoint=False), 5, 1)
        out["batch_2k_x1024_solves_per_s"] = 1024 / ms2 * 1e3
        out["plain_2k_solves_per_s"] = 1e3 / timed(lambda: W2.step(adjoint=False, Bn=1), 5, 1)
        outs = gridgen.n1_outages(W.g, 512, 3)
        n1 = [W.g.without_branch(int(e)) for e in outs]
        out["n1_10k_x512"] = bench_multi(n1, "N-1 10k x 512")
        out["n1_screen_10k_x512"] = bench_screen(W, outs)
        spec = json.load(open(os.path.join(ROOT, "tests", "golden", "mixed_batch.json")))
        mixed = []
        for i, gs in enumerate(spec["grids"]):
            mixed.append(gridgen.make_grid(gs["n"], gs["seed"], load_scale=spec["load_scale"]))
            if i % 8 == 7:
                log(f"[bench] generated {i + 1}/64 mixed grids")
        out["mixed_64_grids"] = bench_multi(mixed, "mixed 64 grids 500-20k buses")
        out["wls_se_10k_x256"] = bench_se(W)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
