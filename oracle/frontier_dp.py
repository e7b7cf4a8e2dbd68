"""Frontier dynamic programme: a second exact method for R and the count.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

This is not the paper's algorithm.  It is an independent exact method of
the kind the paper lists among its competitors (BDD-like, Section 1),
written here only to pin results at sizes where the BAT oracle would take
hours (a 5x5 grid has 2^40 vectors).  It is checked against the BAT oracle
and against exact rational enumeration on small inputs.

Arcs are processed one at a time in an order chosen to keep the frontier
small.  A state is the partition of the current frontier nodes into
connected components (of the working arcs seen so far); each state carries
the total probability of the arc-state prefixes leading to it (a float) and
their number (an exact integer).  Processing arc e = (u, v) splits every
state into "e fails" (weight x (1 - p_e), partition unchanged) and "e works"
(weight x p_e, the blocks of u and v merged).  A node leaves the frontier
after its last arc; s and t never leave.  At the end the connected mass is
the weight of the states where s and t share a block, and likewise the
count.  Summing over all 2^m arc-state vectors this gives exactly Eq. 1.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np


def _node_order(n: int, arcs: Sequence[Tuple[int, int]], s: int) -> List[int]:
    """Greedy order: repeatedly take the node with the most arcs into the
    nodes already taken (ties: fewer arcs to untaken nodes, then id)."""
    adj = [[] for _ in range(n)]
    for (u, v) in arcs:
        if u != v:
            adj[u].append(v)
            adj[v].append(u)
    taken = [False] * n
    order = [s]
    taken[s] = True
    inside = [0] * n
    for w in adj[s]:
        inside[w] += 1
    for _ in range(n - 1):
        best = None
        for v in range(n):
            if taken[v]:
                continue
            key = (-inside[v], len(adj[v]) - inside[v], v)
            if best is None or key < best[0]:
                best = (key, v)
        v = best[1]
        taken[v] = True
        order.append(v)
        for w in adj[v]:
            inside[w] += 1
    return order


def _canon(labels: Sequence[int]) -> Tuple[int, ...]:
    remap: Dict[int, int] = {}
    out = []
    for x in labels:
        if x not in remap:
            remap[x] = len(remap)
        out.append(remap[x])
    return tuple(out)


def reliability(n: int, arcs, p, s: int, t: int, return_width: bool = False):
    """Exact (R, count) of Eq. 1 for undirected arcs by frontier DP."""
    arcs = [(int(u), int(v)) for (u, v) in np.asarray(arcs, dtype=np.int64).reshape(-1, 2)]
    p = [float(x) for x in np.asarray(p, dtype=np.float64).reshape(-1)]
    m = len(arcs)
    assert len(p) == m
    order = _node_order(n, arcs, s)
    pos = {v: i for i, v in enumerate(order)}
    idx = sorted(range(m), key=lambda e: (max(pos[arcs[e][0]], pos[arcs[e][1]]),
                                          min(pos[arcs[e][0]], pos[arcs[e][1]]), e))
    last = {}
    for k, e in enumerate(idx):
        u, v = arcs[e]
        last[u] = k
        last[v] = k
    frontier: List[int] = [s, t]          # s and t are always present
    states: Dict[Tuple[int, ...], Tuple[float, int]] = {(0, 1): (1.0, 1)}
    width = 2
    for k, e in enumerate(idx):
        u, v = arcs[e]
        for w in (u, v):
            if w not in frontier:
                frontier.append(w)
                states = {lab + (max(lab) + 1,): val for lab, val in states.items()}
        width = max(width, len(frontier))
        iu, iv = frontier.index(u), frontier.index(v)
        pe = p[e]
        new: Dict[Tuple[int, ...], Tuple[float, int]] = {}
        for lab, (wgt, cnt) in states.items():
            # arc fails
            w0 = wgt * (1.0 - pe)
            a = new.get(lab)
            new[lab] = (w0, cnt) if a is None else (a[0] + w0, a[1] + cnt)
            # arc works: merge the blocks of u and v
            lu, lv = lab[iu], lab[iv]
            if lu == lv:
                merged = lab
            else:
                merged = _canon([lu if x == lv else x for x in lab])
            w1 = wgt * pe
            a = new.get(merged)
            new[merged] = (w1, cnt) if a is None else (a[0] + w1, a[1] + cnt)
        states = new
        # drop nodes whose last arc this was (never s or t)
        drop = [i for i, w in enumerate(frontier) if w not in (s, t) and last.get(w) == k]
        if drop:
            keep = [i for i in range(len(frontier)) if i not in drop]
            frontier = [frontier[i] for i in keep]
            merged_states: Dict[Tuple[int, ...], Tuple[float, int]] = {}
            for lab, (wgt, cnt) in states.items():
                nl = _canon([lab[i] for i in keep])
                a = merged_states.get(nl)
                merged_states[nl] = (wgt, cnt) if a is None else (a[0] + wgt, a[1] + cnt)
            states = merged_states
    R = 0.0
    count = 0
    vals = []
    for lab, (wgt, cnt) in states.items():
        if lab[0] == lab[1]:
            vals.append(wgt)
            count += cnt
    R = float(np.sum(np.sort(np.asarray(vals))) if vals else 0.0)
    if return_width:
        return R, count, width
    return R, count


def gradient(n: int, arcs, p, s: int, t: int):
    """Birnbaum importances T1_i - T0_i with T1_i = R|p_i<-1 and
    T0_i = R|p_i<-0, each from its own DP run (multilinearity of Eq. 1)."""
    p = np.asarray(p, dtype=np.float64)
    m = p.shape[0]
    T1 = np.zeros(m)
    T0 = np.zeros(m)
    for i in range(m):
        q = p.copy()
        q[i] = 1.0
        T1[i] = reliability(n, arcs, q, s, t)[0]
        q[i] = 0.0
        T0[i] = reliability(n, arcs, q, s, t)[0]
    return T1, T0
