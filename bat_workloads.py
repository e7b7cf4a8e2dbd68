"""Seeded synthetic inputs for exact two-terminal reliability.

This module only *builds inputs*: graphs (node count, arc list, source,
sink) and arc-reliability vectors.  It holds none of the method's
arithmetic, so both the CPU oracle side (tests, bench baseline) and the
HIP side (bench, GPU tests) may import it without sharing any compute code.

The paper's own benchmark networks (its Figure 3) are not available, so
seeded random connected graphs and a square grid of the same sizes stand
in for them.  Every generator is deterministic in its seed.

Recipe (all configs): ``numpy.random.default_rng([220909711, config_id])``.
Random connected graph(n, m): a uniformly random labelled spanning tree
grown by attaching node perm[i] to a uniformly chosen earlier node, then
m-(n-1) extra arcs drawn without replacement from the lexicographic list of
remaining node pairs.  Arc order = tree arcs in generation order, then the
extras in draw order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

SEED_BASE = 220909711


@dataclass
class Network:
    """A binary-state network G(V, E, D_b) with a source and a sink.

    Nodes are 0-based (the paper numbers them from 1, with source 1 and
    sink n).  ``arcs[i]`` is the undirected arc a_{i+1}; ``p[i]`` is its
    working probability Pr(a_{i+1}).
    """

    name: str
    n: int
    arcs: List[Tuple[int, int]]
    s: int
    t: int
    p: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def m(self) -> int:
        return len(self.arcs)

    def arc_array(self) -> np.ndarray:
        """Arcs as an int32 array of shape (m, 2), row i = (u_i, v_i)."""
        if not self.arcs:
            return np.zeros((0, 2), dtype=np.int32)
        return np.ascontiguousarray(np.asarray(self.arcs, dtype=np.int32).reshape(-1, 2))

    def with_p(self, p) -> "Network":
        return Network(self.name, self.n, list(self.arcs), self.s, self.t,
                       np.ascontiguousarray(np.asarray(p, dtype=np.float64)))


def rng_for(config_id: int, extra: int | None = None) -> np.random.Generator:
    key = [SEED_BASE, int(config_id)] if extra is None else [SEED_BASE, int(config_id), int(extra)]
    return np.random.default_rng(key)


def random_connected_arcs(n: int, m: int, rng: np.random.Generator) -> List[Tuple[int, int]]:
    """Spanning tree + uniformly drawn extra arcs (simple graph)."""
    if n < 2:
        raise ValueError("need n >= 2")
    if m < n - 1 or m > n * (n - 1) // 2:
        raise ValueError(f"m={m} impossible for a simple connected graph on n={n}")
    perm = rng.permutation(n)
    arcs: List[Tuple[int, int]] = []
    present = set()
    for i in range(1, n):
        a = int(perm[i])
        b = int(perm[int(rng.integers(0, i))])
        e = (min(a, b), max(a, b))
        arcs.append(e)
        present.add(e)
    extra = m - (n - 1)
    if extra > 0:
        pool = [(i, j) for i in range(n) for j in range(i + 1, n) if (i, j) not in present]
        pick = rng.choice(len(pool), size=extra, replace=False)
        arcs.extend(pool[int(k)] for k in pick)
    return arcs


def random_connected(n: int, m: int, seed, s: int = 0, t: int | None = None,
                     p_lo: float = 0.5, p_hi: float = 0.99, name: str | None = None) -> Network:
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    arcs = random_connected_arcs(n, m, rng)
    p = rng.uniform(p_lo, p_hi, size=m)
    return Network(name or f"rand_n{n}_m{m}", n, arcs, s, n - 1 if t is None else t, p)


def random_multigraph(n: int, m: int, seed, p_lo: float = 0.0, p_hi: float = 1.0) -> Network:
    """Arbitrary arcs (possibly disconnected, with self-loops and parallel arcs)."""
    rng = np.random.default_rng(seed)
    arcs = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
    s, t = (int(x) for x in rng.choice(n, size=2, replace=False))
    p = rng.uniform(p_lo, p_hi, size=m)
    return Network(f"multi_n{n}_m{m}", n, arcs, s, t, p)


def grid(rows: int, cols: int, p=None, name: str | None = None) -> Network:
    """rows x cols grid, node id = cols*r + c; horizontal arcs row-major, then
    vertical arcs row-major; source = corner 0, sink = opposite corner."""
    arcs: List[Tuple[int, int]] = []
    for r in range(rows):
        for c in range(cols - 1):
            arcs.append((cols * r + c, cols * r + c + 1))
    for r in range(rows - 1):
        for c in range(cols):
            arcs.append((cols * r + c, cols * r + c + cols))
    n = rows * cols
    pv = np.full(len(arcs), 0.9) if p is None else np.asarray(p, dtype=np.float64)
    return Network(name or f"grid{rows}x{cols}", n, arcs, 0, n - 1, pv)


def bridge(p: float = 0.9) -> Network:
    """4-node / 5-arc bridge: 1-2, 1-3, 2-3, 2-4, 3-4 (1-based), s=1, t=4."""
    return Network("bridge", 4, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)], 0, 3, np.full(5, float(p)))


def series(m: int, p) -> Network:
    """m arcs in a chain 0-1-...-m; s = 0, t = m."""
    return Network(f"series{m}", m + 1, [(i, i + 1) for i in range(m)], 0, m, np.asarray(p, dtype=np.float64))


def parallel(m: int, p) -> Network:
    """m parallel arcs between s = 0 and t = 1."""
    return Network(f"parallel{m}", 2, [(0, 1)] * m, 0, 1, np.asarray(p, dtype=np.float64))


def parallel_paths(j: int, p) -> Network:
    """j disjoint 2-arc paths s=0 -> mid_i -> t=1 (arc order: (s,mid_i), (mid_i,t))."""
    arcs = []
    for i in range(j):
        arcs += [(0, 2 + i), (2 + i, 1)]
    return Network(f"ppaths{j}", 2 + j, arcs, 0, 1, np.asarray(p, dtype=np.float64))


# ---------------------------------------------------------------- configs
# The five headline workloads.  ``config(i)`` returns the network(s) and the
# probability vectors for workload i.

def config0() -> Network:
    """Bridge network, all arc reliabilities 0.9; 32 state vectors."""
    return bridge(0.9)


def config1() -> Network:
    """Random connected graph, 20 nodes, m=30, s=0, t=19, p ~ U[0.80, 0.99]."""
    rng = rng_for(1)
    arcs = random_connected_arcs(20, 30, rng)
    p = rng.uniform(0.80, 0.99, size=30)
    return Network("rand_n20_m30", 20, arcs, 0, 19, p)


def config2() -> Network:
    """5x5 grid, 40 arcs, corner to corner, p ~ U[0.85, 0.99]; 2^40 vectors."""
    rng = rng_for(2)
    g = grid(5, 5, name="grid5x5")
    return g.with_p(rng.uniform(0.85, 0.99, size=g.m))


def config3(n_graphs: int = 256, n_pvec: int = 32) -> Tuple[List[Network], List[np.ndarray]]:
    """Batched: n_graphs random connected graphs, n_g ~ U{8..16},
    m_g ~ U{16..28} (capped at n_g(n_g-1)/2), random s != t, and n_pvec
    probability vectors per graph with p ~ U[0.5, 0.99]."""
    rng = rng_for(3)
    nets: List[Network] = []
    pvs: List[np.ndarray] = []
    for gi in range(n_graphs):
        n = int(rng.integers(8, 17))
        m = int(rng.integers(16, 29))
        m = max(n - 1, min(m, n * (n - 1) // 2))
        arcs = random_connected_arcs(n, m, rng)
        s, t = (int(x) for x in rng.choice(n, size=2, replace=False))
        pv = rng.uniform(0.5, 0.99, size=(n_pvec, m))
        nets.append(Network(f"batch{gi}_n{n}_m{m}", n, arcs, s, t, pv[0].copy()))
        pvs.append(np.ascontiguousarray(pv))
    return nets, pvs


def config4() -> Network:
    """Random connected graph, 18 nodes, m=36, s=0, t=17, p ~ U[0.7, 0.99]."""
    rng = rng_for(4)
    arcs = random_connected_arcs(18, 36, rng)
    p = rng.uniform(0.70, 0.99, size=36)
    return Network("rand_n18_m36", 18, arcs, 0, 17, p)


def figure1(reversed_table1: bool = True) -> Network:
    """The paper's Figure 1 example network (5 nodes, 6 arcs, s=1, t=4).

    The figure itself is not available in text form; the topology below is
    the one consistent with the connected vectors of the paper's Table 4 and
    the layers of its Table 3: two triangles {1,2,3} and {2,4,5} sharing
    node 2.  Arc labelling (1-based): a1=(1,3) a2=(1,2) a3=(2,3) a4=(2,5)
    a5=(2,4) a6=(4,5).  Table 4's per-vector probabilities use Table 1's
    values in reverse order, p = (0.87, 0.85, 0.95, 0.88, 0.89, 0.99);
    ``reversed_table1=False`` gives Table 1's listed order instead.
    """
    arcs = [(0, 2), (0, 1), (1, 2), (1, 4), (1, 3), (3, 4)]
    table1 = [0.99, 0.89, 0.88, 0.95, 0.85, 0.87]
    p = table1[::-1] if reversed_table1 else table1
    return Network("figure1", 5, arcs, 0, 3, np.asarray(p, dtype=np.float64))


# ------------------------------------------------------------ multi-state
# Arcs with several states (the solution space of prod_i sigma_i vectors):
# state k of arc i carries capacity cap[i][k] with probability w[i][k]; the
# question is whether the maximum s-t flow reaches a demand d.  The paper
# has no multi-state benchmark, so these stand in: three capacity levels
# 0, 1, 2 per arc (failed, degraded, full), mostly at full capacity.

@dataclass
class MsNetwork:
    name: str
    n: int
    arcs: List[Tuple[int, int]]
    s: int
    t: int
    sigma: List[int]
    cap: List[List[int]]
    w: List[np.ndarray]
    d: int

    @property
    def m(self) -> int:
        return len(self.arcs)

    @property
    def space(self) -> int:
        N = 1
        for k in self.sigma:
            N *= int(k)
        return N

    def cap_flat(self) -> np.ndarray:
        return np.ascontiguousarray(np.concatenate([np.asarray(c, dtype=np.int32) for c in self.cap])
                                    if self.cap else np.zeros(0, dtype=np.int32))

    def w_flat(self) -> np.ndarray:
        return np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float64) for x in self.w])
                                    if self.w else np.zeros(0, dtype=np.float64))


def three_level_weights(rng: np.random.Generator, m: int) -> List[np.ndarray]:
    """Per arc: failed w ~ U[0.02, 0.10], degraded w ~ U[0.10, 0.30], the
    rest at full capacity."""
    out = []
    for _ in range(m):
        w0 = rng.uniform(0.02, 0.10)
        w1 = rng.uniform(0.10, 0.30)
        out.append(np.array([w0, w1, 1.0 - w0 - w1]))
    return out


def ms_bridge(d: int = 2) -> MsNetwork:
    """The bridge with three capacity levels per arc, w = (0.05, 0.15, 0.80)."""
    b = bridge()
    return MsNetwork(f"ms_bridge_d{d}", b.n, list(b.arcs), b.s, b.t, [3] * 5, [[0, 1, 2]] * 5,
                     [np.array([0.05, 0.15, 0.80])] * 5, d)


def ms_random(n: int, m: int, seed, d: int = 2, s: int = 0, t: int | None = None) -> MsNetwork:
    """Random connected graph (the recipe above) with three capacity levels."""
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    arcs = random_connected_arcs(n, m, rng)
    w = three_level_weights(rng, m)
    return MsNetwork(f"ms_rand_n{n}_m{m}_d{d}", n, arcs, s, n - 1 if t is None else t, [3] * m,
                     [[0, 1, 2]] * m, w, d)


def ms_mixed(n: int, m: int, seed) -> MsNetwork:
    """Arbitrary multigraph (self-loops, parallel arcs), 1 to 4 states per
    arc with random capacities 0..3 and random weights, demand 1 to 3."""
    rng = np.random.default_rng(seed)
    arcs = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
    s, t = (int(x) for x in rng.choice(n, size=2, replace=False))
    sigma = [int(rng.integers(1, 5)) for _ in range(m)]
    cap = [[int(c) for c in rng.integers(0, 4, size=k)] for k in sigma]
    w = [rng.dirichlet(np.ones(k)) for k in sigma]
    return MsNetwork(f"ms_mixed_n{n}_m{m}", n, arcs, s, t, sigma, cap, w, int(rng.integers(1, 4)))


def config_ms() -> MsNetwork:
    """Multi-state workload: random connected graph, 10 nodes, m = 18,
    three capacity levels per arc, demand 2; 3^18 state vectors."""
    return ms_random(10, 18, rng_for(5), d=2)
