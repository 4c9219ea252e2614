"""Seeded synthetic transmission-grid generator.

This module only draws inputs: bus coordinates, topology, branch impedances,
bus types, voltage set-points and injections.  It holds none of the power-flow
arithmetic (no admittances, no injections from voltages, no Jacobian), so both
the CPU oracle and the GPU library can consume its output without sharing any
of the method's code.

The recipe (the paper's four test systems are not public; these grids stand in
for them, see the case study in Section IV):

* n buses at uniform points in the unit square; bus 0 is the slack bus.
* Topology: a random spanning tree (buses visited in a seeded random order,
  each attached to its Euclidean-nearest bus already placed), then extra
  branches drawn from the 6-nearest-neighbour candidate pairs in a seeded
  shuffled order until m = round(1.3 n).  No parallel branches, no self loops.
* Branches: x ~ lognormal(ln 0.05, 0.5) p.u., r = x * U(0.05, 0.3),
  total line charging b ~ U(0, 0.05) p.u.
* round(0.2 n) PV buses drawn from buses 1..n-1 with |V| set-points
  U(0.98, 1.05); every other non-slack bus is PQ.
* Loads on every bus: P_d ~ U(0, 1) * s, Q_d = P_d * U(0.2, 0.5).  PV
  generation P_g takes U(0, 1) shares of 1.02 * sum(P_d).  The load scale s
  (default 0.1) keeps the slack's balancing injection within what its few
  branches can carry; with s = 1 Newton's method diverges from flat start on
  most grids of this family.
* Scheduled injections: P_sp = P_g - P_d, Q_sp = -Q_d.
* Bus shunts (g_sh + j b_sh per bus) are zero on these grids.  `with_shunts`
  adds seeded ones (capacitor banks and reactors at a fraction of the
  non-slack buses, with a small conductance) for the tests of the shunt term.

Load scenarios multiply each bus load (P_d and Q_d together) by a seeded
lognormal(0, 0.1) factor; generation is unchanged.  N-1 cases remove one
non-bridge branch each, chosen without replacement.
"""
from __future__ import annotations

import dataclasses

import numpy as np

BUS_PQ = 1
BUS_PV = 2
BUS_SLACK = 3

DEFAULT_LOAD_SCALE = 0.1


@dataclasses.dataclass
class Grid:
    """One power-flow case in per-unit.  Bus 0 is the slack bus."""

    n: int
    f: np.ndarray        # int32[m]  from-bus
    t: np.ndarray        # int32[m]  to-bus
    r: np.ndarray        # float64[m] series resistance
    x: np.ndarray        # float64[m] series reactance
    b: np.ndarray        # float64[m] total line charging susceptance
    bus_type: np.ndarray  # int8[n]  BUS_PQ / BUS_PV / BUS_SLACK
    vset: np.ndarray     # float64[n] |V| set-point (PV, slack) or 1.0
    Pd: np.ndarray       # float64[n]
    Qd: np.ndarray       # float64[n]
    Pg: np.ndarray       # float64[n]
    pts: np.ndarray      # float64[n, 2] coordinates (topology provenance only)
    seed: int = 0
    load_scale: float = DEFAULT_LOAD_SCALE
    gsh: np.ndarray = None  # float64[n] bus shunt conductance (None -> zeros)
    bsh: np.ndarray = None  # float64[n] bus shunt susceptance (None -> zeros)

    def __post_init__(self):
        if self.gsh is None:
            self.gsh = np.zeros(self.n)
        if self.bsh is None:
            self.bsh = np.zeros(self.n)

    @property
    def has_shunts(self) -> bool:
        return bool(np.any(self.gsh != 0) or np.any(self.bsh != 0))

    @property
    def ysh(self) -> np.ndarray:
        """Bus shunts as (g, b) pairs, float64[n, 2]."""
        return np.stack([self.gsh, self.bsh], axis=1)

    @property
    def m(self) -> int:
        return int(self.f.shape[0])

    @property
    def Psp(self) -> np.ndarray:
        return self.Pg - self.Pd

    @property
    def Qsp(self) -> np.ndarray:
        return -self.Qd

    def flat_start(self):
        """|V| = set-point at PV and slack buses, 1 elsewhere; all angles 0."""
        return self.vset.copy(), np.zeros(self.n)

    def with_loads(self, Pd, Qd) -> "Grid":
        return dataclasses.replace(self, Pd=np.asarray(Pd, np.float64),
                                   Qd=np.asarray(Qd, np.float64))

    def without_branch(self, e: int) -> "Grid":
        keep = np.ones(self.m, bool)
        keep[e] = False
        return dataclasses.replace(self, f=self.f[keep], t=self.t[keep],
                                   r=self.r[keep], x=self.x[keep], b=self.b[keep])


def _spanning_tree(pts: np.ndarray, order: np.ndarray):
    """Attach each bus (visited in `order`) to its nearest already placed bus."""
    n = pts.shape[0]
    best_d = np.full(n, np.inf)
    best_p = np.full(n, -1, dtype=np.int64)
    placed = np.zeros(n, bool)
    edges = []
    for step, v in enumerate(order):
        if step > 0:
            edges.append((int(best_p[v]), int(v)))
        placed[v] = True
        d = np.sum((pts - pts[v]) ** 2, axis=1)
        upd = (d < best_d) & ~placed
        best_d[upd] = d[upd]
        best_p[upd] = v
    return edges


def _knn_candidates(pts: np.ndarray, k: int):
    from scipy.spatial import cKDTree

    n = pts.shape[0]
    kk = min(k + 1, n)
    _, idx = cKDTree(pts).query(pts, k=kk)
    cand = set()
    for i in range(n):
        for j in idx[i, 1:]:
            j = int(j)
            if j != i:
                cand.add((min(i, j), max(i, j)))
    return sorted(cand)


def make_grid(n: int, seed: int, load_scale: float = DEFAULT_LOAD_SCALE,
              pv_frac: float = 0.2, branch_ratio: float = 1.3, knn: int = 6) -> Grid:
    if n < 2:
        raise ValueError("a grid needs at least 2 buses")
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    order = rng.permutation(n)
    tree = _spanning_tree(pts, order)
    m_target = max(n - 1, int(round(branch_ratio * n)))
    have = {(min(a, b), max(a, b)) for a, b in tree}
    extra = [e for e in _knn_candidates(pts, knn) if e not in have]
    shuffle = rng.permutation(len(extra))
    edges = list(tree)
    for s in shuffle:
        if len(edges) >= m_target:
            break
        edges.append(extra[s])
    m = len(edges)
    f = np.array([e[0] for e in edges], dtype=np.int32)
    t = np.array([e[1] for e in edges], dtype=np.int32)
    x = rng.lognormal(np.log(0.05), 0.5, m)
    r = x * rng.uniform(0.05, 0.3, m)
    b = rng.uniform(0.0, 0.05, m)

    npv = int(round(pv_frac * n))
    npv = min(npv, n - 1)
    pv = 1 + rng.choice(n - 1, npv, replace=False)
    vset_pv = rng.uniform(0.98, 1.05, npv)
    bus_type = np.full(n, BUS_PQ, dtype=np.int8)
    bus_type[0] = BUS_SLACK
    bus_type[pv] = BUS_PV
    vset = np.ones(n)
    vset[pv] = vset_pv

    Pd = rng.uniform(0.0, 1.0, n) * load_scale
    Qd = Pd * rng.uniform(0.2, 0.5, n)
    Pg = np.zeros(n)
    if npv > 0:
        share = rng.uniform(0.0, 1.0, npv)
        Pg[pv] = share / share.sum() * 1.02 * Pd.sum()
    return Grid(n=n, f=f, t=t, r=r, x=x, b=b, bus_type=bus_type, vset=vset,
                Pd=Pd, Qd=Qd, Pg=Pg, pts=pts, seed=seed, load_scale=load_scale)


def with_shunts(grid: Grid, seed: int, frac: float = 0.3) -> Grid:
    """The grid with seeded bus shunts at round(frac * (n - 1)) non-slack buses:
    susceptance b_sh ~ U(-0.05, 0.15) p.u. (reactors below zero, capacitor banks
    above) and conductance g_sh ~ U(0, 0.01) p.u.; other buses keep none."""
    rng = np.random.default_rng(seed)
    k = min(grid.n - 1, int(round(frac * (grid.n - 1))))
    at = 1 + rng.choice(grid.n - 1, k, replace=False)
    gsh = np.zeros(grid.n)
    bsh = np.zeros(grid.n)
    bsh[at] = rng.uniform(-0.05, 0.15, k)
    gsh[at] = rng.uniform(0.0, 0.01, k)
    return dataclasses.replace(grid, gsh=gsh, bsh=bsh)


def load_scenarios(grid: Grid, count: int, seed: int, sigma: float = 0.1):
    """Per (scenario, bus) lognormal(0, sigma) factors on P_d and Q_d.

    Returns (Pd[count, n], Qd[count, n]); generation is left unchanged.
    """
    rng = np.random.default_rng(seed)
    fac = rng.lognormal(0.0, sigma, (count, grid.n))
    return grid.Pd[None, :] * fac, grid.Qd[None, :] * fac


def scenario_injections(grid: Grid, count: int, seed: int, sigma: float = 0.1):
    """(Psp[count, n], Qsp[count, n]) for `load_scenarios`."""
    Pd, Qd = load_scenarios(grid, count, seed, sigma)
    return grid.Pg[None, :] - Pd, -Qd


def bridges(n: int, f: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Boolean mask over branches: True where removing the branch disconnects
    the graph (Tarjan's low-link, iterative; parallel branches are never
    bridges because each is tracked by branch id)."""
    m = len(f)
    adj = [[] for _ in range(n)]
    for e in range(m):
        a, b = int(f[e]), int(t[e])
        adj[a].append((b, e))
        adj[b].append((a, e))
    disc = np.full(n, -1, dtype=np.int64)
    low = np.zeros(n, dtype=np.int64)
    is_bridge = np.zeros(m, bool)
    timer = 0
    for root in range(n):
        if disc[root] >= 0:
            continue
        disc[root] = low[root] = timer
        timer += 1
        stack = [(root, -1, 0)]
        while stack:
            v, pe, it = stack[-1]
            if it < len(adj[v]):
                stack[-1] = (v, pe, it + 1)
                w, e = adj[v][it]
                if e == pe:
                    continue
                if disc[w] < 0:
                    disc[w] = low[w] = timer
                    timer += 1
                    stack.append((w, e, 0))
                else:
                    low[v] = min(low[v], disc[w])
            else:
                stack.pop()
                if stack:
                    u = stack[-1][0]
                    low[u] = min(low[u], low[v])
                    if low[v] > disc[u]:
                        is_bridge[pe] = True
    return is_bridge


def n1_outages(grid: Grid, count: int, seed: int) -> np.ndarray:
    """`count` distinct non-bridge branch indices, seeded, without replacement."""
    cand = np.flatnonzero(~bridges(grid.n, grid.f, grid.t))
    if count > len(cand):
        raise ValueError(f"only {len(cand)} non-bridge branches")
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cand, count, replace=False)).astype(np.int64)


def mixed_sizes(count: int, seed: int, lo: int = 500, hi: int = 20000) -> np.ndarray:
    """Log-uniform grid sizes in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)


def _grid_from_spec(spec):
    n, seed, load_scale = spec
    return make_grid(int(n), int(seed), load_scale=load_scale)


def make_grids(specs, processes=8):
    """make_grid over (n, seed, load_scale) specs in a pool of fresh
    interpreter processes (spawned, so that they inherit no device handles of
    the caller), largest grids first; returns the grids in spec order."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor

    specs = [tuple(s) for s in specs]
    order = sorted(range(len(specs)), key=lambda i: -specs[i][0])
    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(max(1, processes), mp_context=ctx) as ex:
        made = dict(zip(order, ex.map(_grid_from_spec, [specs[i] for i in order])))
    return [made[i] for i in range(len(specs))]
