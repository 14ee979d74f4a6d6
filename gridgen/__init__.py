"""Seeded synthetic power networks and direction blocks.

This module only *draws inputs*: topologies, line data, loads, generator
placement and dispatch set-points, cost coefficients and Gaussian direction
blocks.  It holds none of the reduced-Hessian method's arithmetic (no power
flow, no Jacobian, no solve), so the CPU oracle and the HIP library can both
consume its output without sharing any computation.

Network data follow the paper's power-flow model (Sec. 3.1, eq. (powerflow) and
(powerflowvec)): buses with a reference/PV/PQ partition, branches with series
impedance ``r + j x`` and total line charging ``b`` (split evenly over the two
ends), per-unit on a 100 MVA base.  The paper's PGLIB cases are not available,
so seeded synthetic grids with PGLIB-like ratios stand in for them
(Table 1: branches per bus 1.2-1.7, generator buses 8-46 % of buses).
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field, replace

import numpy as np

PQ, PV, REF = 1, 2, 3


@dataclass
class Grid:
    """A power network in plain arrays (0-based bus ids, one generator per bus)."""

    n_bus: int
    br_from: np.ndarray  # int32 [n_branch]
    br_to: np.ndarray  # int32 [n_branch]
    br_r: np.ndarray  # float64 [n_branch] series resistance (pu)
    br_x: np.ndarray  # float64 [n_branch] series reactance (pu)
    br_b: np.ndarray  # float64 [n_branch] total line charging (pu)
    bus_type: np.ndarray  # int32 [n_bus] 1=PQ 2=PV 3=REF
    Pd: np.ndarray  # float64 [n_bus] active load (pu)
    Qd: np.ndarray  # float64 [n_bus] reactive load (pu)
    gen_bus: np.ndarray  # int32 [n_gen]
    Pg: np.ndarray  # float64 [n_gen] active set-point (ignored for the REF generator)
    Vg: np.ndarray  # float64 [n_gen] voltage-magnitude set-point
    c2: np.ndarray  # float64 [n_gen] quadratic cost coefficient
    c1: np.ndarray  # float64 [n_gen] linear cost coefficient
    c0: np.ndarray  # float64 [n_gen] constant cost term
    name: str = ""
    meta: dict = field(default_factory=dict)
    # initial guess of the voltage magnitudes for Newton (None: flat start)
    v0: np.ndarray | None = None

    @property
    def n_branch(self) -> int:
        return int(self.br_from.shape[0])

    @property
    def n_gen(self) -> int:
        return int(self.gen_bus.shape[0])

    @property
    def ref_bus(self) -> int:
        return int(np.flatnonzero(self.bus_type == REF)[0])

    @property
    def n_pq(self) -> int:
        return int(np.count_nonzero(self.bus_type == PQ))

    @property
    def n_x(self) -> int:
        """Dimension of the state: angles at PV and PQ buses plus PQ magnitudes."""
        return self.n_bus - 1 + self.n_pq

    @property
    def n_p(self) -> int:
        """Dimension of the parameters: PV active powers plus all generator magnitudes."""
        return 2 * self.n_gen - 1

    def copy(self) -> "Grid":
        return replace(
            self,
            **{
                k: getattr(self, k).copy()
                for k in (
                    "br_from", "br_to", "br_r", "br_x", "br_b", "bus_type", "Pd", "Qd",
                    "gen_bus", "Pg", "Vg", "c2", "c1", "c0",
                )
            },
            meta=dict(self.meta),
            v0=None if self.v0 is None else self.v0.copy(),
        )


def _finish(n_bus, f, t, r, x, b, gens, Pd, Qd, Pg, Vg, c2, c1, c0, name, meta) -> Grid:
    bus_type = np.full(n_bus, PQ, dtype=np.int32)
    bus_type[gens[1:]] = PV
    bus_type[gens[0]] = REF
    return Grid(
        n_bus=int(n_bus),
        br_from=np.asarray(f, dtype=np.int32),
        br_to=np.asarray(t, dtype=np.int32),
        br_r=np.asarray(r, dtype=np.float64),
        br_x=np.asarray(x, dtype=np.float64),
        br_b=np.asarray(b, dtype=np.float64),
        bus_type=bus_type,
        Pd=np.asarray(Pd, dtype=np.float64),
        Qd=np.asarray(Qd, dtype=np.float64),
        gen_bus=np.asarray(gens, dtype=np.int32),
        Pg=np.asarray(Pg, dtype=np.float64),
        Vg=np.asarray(Vg, dtype=np.float64),
        c2=np.asarray(c2, dtype=np.float64),
        c1=np.asarray(c1, dtype=np.float64),
        c0=np.asarray(c0, dtype=np.float64),
        name=name,
        meta=meta,
    )


def _costs(rng, n_gen):
    c2 = rng.uniform(0.5, 2.0, n_gen)
    c1 = rng.uniform(1.0, 4.0, n_gen)
    return c2, c1, np.zeros(n_gen)


def ring9(seed: int = 0) -> Grid:
    """9-bus ring plus 3 random chords, 3 generators (first = reference)."""
    rng = np.random.default_rng(seed)
    n = 9
    edges = {(i, (i + 1) % n) if i < (i + 1) % n else ((i + 1) % n, i) for i in range(n)}
    ring = sorted(edges)
    chords = []
    while len(chords) < 3:
        a, c = sorted(int(v) for v in rng.choice(n, 2, replace=False))
        if (a, c) in edges:
            continue
        edges.add((a, c))
        chords.append((a, c))
    pairs = ring + chords
    m = len(pairs)
    f = np.array([p[0] for p in pairs])
    t = np.array([p[1] for p in pairs])
    r = rng.uniform(0.005, 0.05, m)
    x = rng.uniform(0.05, 0.3, m)
    b = rng.uniform(0.0, 0.2, m)
    gens = rng.choice(n, 3, replace=False).astype(np.int32)
    Pd = np.zeros(n)
    Qd = np.zeros(n)
    load_bus = np.setdiff1d(np.arange(n), gens)
    Pd[load_bus] = rng.uniform(0.5, 1.5, load_bus.size)
    Qd[load_bus] = rng.uniform(0.1, 0.5, load_bus.size)
    Pg = np.full(3, Pd.sum() / 3.0)
    Vg = rng.uniform(1.0, 1.05, 3)
    c2, c1, c0 = _costs(rng, 3)
    return _finish(n, f, t, r, x, b, gens, Pd, Qd, Pg, Vg, c2, c1, c0,
                   f"ring9-s{seed}", {"seed": seed, "kind": "ring9"})


def _adjacency(n, f, t):
    deg = np.bincount(np.concatenate([f, t]), minlength=n)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=ptr[1:])
    nbr = np.empty(ptr[-1], dtype=np.int64)
    fill = ptr[:-1].copy()
    for a, c in zip(f, t):
        nbr[fill[a]] = c
        fill[a] += 1
        nbr[fill[c]] = a
        fill[c] += 1
    return ptr, nbr


def _bfs_update(ptr, nbr, src, dist):
    """Lower ``dist`` to hop distances from ``src`` where they improve."""
    dist[src] = 0
    q = deque([src])
    while q:
        u = q.popleft()
        du = dist[u] + 1
        for w in nbr[ptr[u]:ptr[u + 1]]:
            if du < dist[w]:
                dist[w] = du
                q.append(w)


def _voronoi(ptr, nbr, gens, n):
    """Assign each bus to the hop-nearest generator (multi-source BFS, gens in order)."""
    owner = np.full(n, -1, dtype=np.int64)
    q = deque()
    for gi, g in enumerate(gens):
        owner[g] = gi
        q.append(g)
    while q:
        u = q.popleft()
        for w in nbr[ptr[u]:ptr[u + 1]]:
            if owner[w] < 0:
                owner[w] = owner[u]
                q.append(w)
    return owner


def geometric(n_bus: int, n_branch: int, n_gen: int, seed: int, alpha: float,
              kappa: float = 0.0, name: str = "") -> Grid:
    """Planar random geometric grid.

    Buses uniform in the unit square; branches are the Euclidean minimum
    spanning tree of the Delaunay triangulation plus uniformly drawn further
    Delaunay edges up to ``n_branch``.  Generators are placed by farthest-point
    sampling in hop distance (the first one is the reference bus).  Loads sit
    on PQ buses (lognormal, mean 0.3 pu, sigma 0.5, Q = 0.3 P).  Each PV
    generator's set-point is the load of its hop-Voronoi cell times
    ``1 + kappa`` (``kappa`` covers the network losses, so that the slack
    carries little of them); voltage
    set-points follow a smooth field over the plane.  ``alpha`` scales loads,
    active set-points and line charging together (loading factor).
    """
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    pts = rng.random((n_bus, 2))
    tri = Delaunay(pts)
    s = tri.simplices
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [0, 2]]])
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    w = np.linalg.norm(pts[e[:, 0]] - pts[e[:, 1]], axis=1)
    g = coo_matrix((w, (e[:, 0], e[:, 1])), shape=(n_bus, n_bus)).tocsr()
    mst = minimum_spanning_tree(g).tocoo()
    tree = np.stack([np.minimum(mst.row, mst.col), np.maximum(mst.row, mst.col)], 1)
    tree_keys = set(map(tuple, tree.tolist()))
    rest = np.array([p for p in e.tolist() if tuple(p) not in tree_keys], dtype=np.int64)
    extra = n_branch - tree.shape[0]
    if extra < 0 or extra > rest.shape[0]:
        raise ValueError("branch count incompatible with the triangulation")
    pick = rest[rng.choice(rest.shape[0], extra, replace=False)] if extra else rest[:0]
    br = np.concatenate([tree, pick])
    br = br[rng.permutation(br.shape[0])]
    flip = rng.random(br.shape[0]) < 0.5
    f = np.where(flip, br[:, 1], br[:, 0])
    t = np.where(flip, br[:, 0], br[:, 1])
    m = br.shape[0]
    r = rng.uniform(0.005, 0.05, m)
    x = rng.uniform(0.05, 0.3, m)
    b = rng.uniform(0.0, 0.2, m)

    ptr, nbr = _adjacency(n_bus, f, t)
    prio = rng.random(n_bus)
    # reference bus: the best-connected bus near the centre of the square, so
    # that the slack's share of the losses leaves it over several branches
    deg = np.diff(ptr)
    dc = np.linalg.norm(pts - 0.5, axis=1)
    near = np.flatnonzero(dc < 0.1)
    if near.size == 0:
        near = np.argsort(dc)[:3]
    start = int(near[np.lexsort((prio[near], deg[near]))[-1]])
    big = np.iinfo(np.int64).max // 4
    dist = np.full(n_bus, big, dtype=np.int64)
    gens = [start]
    _bfs_update(ptr, nbr, start, dist)
    for _ in range(n_gen - 1):
        dmax = dist.max()
        cand = np.flatnonzero(dist == dmax)
        nxt = int(cand[np.argmax(prio[cand])])
        gens.append(nxt)
        _bfs_update(ptr, nbr, nxt, dist)
    gens = np.asarray(gens, dtype=np.int32)

    is_gen = np.zeros(n_bus, dtype=bool)
    is_gen[gens] = True
    sig = 0.5
    mu = np.log(0.3) - sig * sig / 2.0
    Pd = np.where(is_gen, 0.0, rng.lognormal(mu, sig, n_bus))
    Qd = 0.3 * Pd
    owner = _voronoi(ptr, nbr, gens, n_bus)
    Pg = (1.0 + kappa) * np.bincount(owner, weights=Pd, minlength=n_gen)
    # Voltage set-points in [1.00, 1.05], drawn as a smooth random field over
    # the plane: neighbouring generators get nearly equal set-points, so no
    # large reactive/active flows circulate between them at light load.
    ph = rng.uniform(0.0, 2.0 * np.pi, 4)
    gx, gy = pts[gens, 0], pts[gens, 1]
    field = 0.25 * (2.0 + np.sin(2.0 * np.pi * gx + ph[0]) * np.cos(2.0 * np.pi * gy + ph[1])
                    + np.sin(np.pi * (gx + gy) + ph[2]))
    Vg = 1.0 + 0.05 * np.clip(field, 0.0, 1.0)
    c2, c1, c0 = _costs(rng, n_gen)
    grid = _finish(n_bus, f, t, r, x, alpha * b, gens, alpha * Pd, alpha * Qd, alpha * Pg,
                   Vg, c2, c1, c0, name or f"geo{n_bus}-s{seed}",
                   {"seed": seed, "kind": "geometric", "alpha": alpha, "kappa": kappa})
    # Newton's starting magnitudes: each bus at its cell generator's set-point
    # (a flat 1.0 would start every PQ bus next to a generator with a large
    # reactive mismatch)
    grid.v0 = Vg[owner].astype(np.float64)
    return grid


# Workload shapes.  ``alpha`` is the loading factor (loads, dispatch and line
# charging scaled together) and ``kappa`` the loss factor of the PV dispatch.
# Both were set with tests/golden/calibrate_grids.py: alpha is about 0.8 of
# the smallest loading limit found over the instances used (70k buses: the
# limit is 0.055, so loads are light there), kappa the slack's loss share at
# light load scaled linearly to alpha.
CONFIGS = {
    "c1": dict(n_bus=1_000, n_branch=1_350, n_gen=100, alpha=0.30, kappa=0.0255),
    "c2": dict(n_bus=10_000, n_branch=13_500, n_gen=1_400, alpha=0.22, kappa=0.0113),
    "c3": dict(n_bus=70_000, n_branch=95_000, n_gen=5_000, alpha=0.044, kappa=0.0069),
}
CONFIG_INDEX = {"c0": 0, "c1": 1, "c2": 2, "c3": 3}


def config_grid(name: str, instance: int = 0) -> Grid:
    """Base grid of a workload; ``seed = 1000 * config + instance``."""
    seed = 1000 * CONFIG_INDEX[name] + instance
    if name == "c0":
        return ring9(seed)
    c = CONFIGS[name]
    return geometric(c["n_bus"], c["n_branch"], c["n_gen"], seed, c["alpha"],
                     kappa=c["kappa"], name=f"{name}-i{instance}")


def perturb_loads(grid: Grid, seed: int, frac: float = 0.1) -> Grid:
    """Scale every bus load by an independent factor drawn from U(1-frac, 1+frac)."""
    rng = np.random.default_rng(seed)
    out = grid.copy()
    s = rng.uniform(1.0 - frac, 1.0 + frac, grid.n_bus)
    out.Pd = grid.Pd * s
    out.Qd = grid.Qd * s
    out.meta["perturb_seed"] = seed
    return out


def lossless(grid: Grid) -> Grid:
    """The same network with every series resistance set to zero."""
    out = grid.copy()
    out.br_r[:] = 0.0
    out.name = grid.name + "-lossless"
    return out


def relabel(grid: Grid, perm: np.ndarray) -> Grid:
    """Rename bus ``i`` to ``perm[i]`` (loads and types move with the bus)."""
    perm = np.asarray(perm)
    out = grid.copy()
    out.br_from = perm[grid.br_from].astype(np.int32)
    out.br_to = perm[grid.br_to].astype(np.int32)
    for k in ("bus_type", "Pd", "Qd"):
        v = getattr(grid, k)
        nv = np.empty_like(v)
        nv[perm] = v
        setattr(out, k, nv)
    out.gen_bus = perm[grid.gen_bus].astype(np.int32)
    if grid.v0 is not None:
        out.v0 = np.empty_like(grid.v0)
        out.v0[perm] = grid.v0
    return out


def two_bus(r: float, x: float, P: float, Q: float, v1: float, c2: float, c1: float,
            b: float = 0.0, pv: bool = False, Pg2: float = 0.0, v2: float = 1.0,
            c2b: float = 1.0, c1b: float = 1.0) -> Grid:
    """Reference bus 0 and one further bus (PQ load, or PV generator with a load)."""
    gens = [0, 1] if pv else [0]
    Pd = np.array([0.0, P])
    Qd = np.array([0.0, Q])
    Pg = np.array([0.0, Pg2]) if pv else np.array([0.0])
    Vg = np.array([v1, v2]) if pv else np.array([v1])
    c2v = np.array([c2, c2b]) if pv else np.array([c2])
    c1v = np.array([c1, c1b]) if pv else np.array([c1])
    return _finish(2, [0], [1], [r], [x], [b], np.asarray(gens), Pd, Qd, Pg, Vg, c2v, c1v,
                   np.zeros(len(gens)), "two-bus", {"kind": "two_bus"})


def directions(n_p: int, k: int, seed: int) -> np.ndarray:
    """Gaussian direction block ``W`` of shape ``(n_p, k)``, column-major float64."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n_p, k)))


def load_trajectory(grid: Grid, steps: int = 60, amp: float = 0.03, noise: float = 0.005,
                    seed: int = 0) -> tuple:
    """Loads of a tracking run: one row per minute over ``steps`` minutes.

    Every bus follows a common slow swing
    ``1 + amp (sin(2 pi t / steps + phi) - sin(phi))`` (one random phase; the
    swing starts at the base loads, which the generator set-points balance)
    times its own factor ``1 + noise e_tb`` with ``e_tb ~ N(0, 1)``, applied
    to both P^d and Q^d.  Returns (Pd, Qd) of shape (steps, n_bus)."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * np.pi)
    t = np.arange(steps)[:, None]
    common = 1.0 + amp * (np.sin(2.0 * np.pi * t / steps + phi) - np.sin(phi))
    own = 1.0 + noise * rng.standard_normal((steps, grid.n_bus))
    s = common * own
    return grid.Pd[None, :] * s, grid.Qd[None, :] * s
