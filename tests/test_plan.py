"""The graph-specialised kernel's relaxation plan, checked on the CPU.

The plan the library hands to hiprtc (bat_jit_source) drops arcs that lie
on no s-t path, joins two arcs in series through a node of degree 2 into
one relaxation whose mask is the AND of theirs, and relaxes arcs at s and
t one way only (out of s, into t).  All three must leave the verdict of
every state vector unchanged.  These tests parse the plan out of the
source text, run its relaxations to a fixed point for every counter value
of small graphs (plain Python, one vector at a time, with the same rules
as the kernel's closure), and compare with a breadth-first search on the
original graph.  No GPU is needed.
"""
import re

import numpy as np
import pytest

import bat_workloads as W


def _B():
    import paper_2209_09711_amd as B
    return B


def _plan(src):
    g = src[src.index("struct JitGraph"):]
    num = lambda k: int(re.search(r"static constexpr int %s = (-?\d+);" % k, g).group(1))
    arr = lambda k: [int(x) for x in re.search(r"unsigned char %s\[\d+\] = \{([^}]*)\}" % k, g).group(1).split(",")]
    nr = num("NR")
    plan = {"N": num("N"), "S": num("S"), "T": num("T"), "NR": nr,
            "DIR": "DIR = true" in g}
    for k in ("RU", "RV", "RB", "RB2"):
        plan[k] = arr(k)[:nr] if nr else []
    return plan


def _plan_verdict(P, c):
    """Fixed point of the plan's relaxations for counter value c."""
    N, S, T = P["N"], P["S"], P["T"]
    r = [False] * N
    r[S] = True
    work = []
    for k in range(P["NR"]):
        u, v, b1, b2 = P["RU"][k], P["RV"][k], P["RB"][k], P["RB2"][k]
        w = bool((c >> b1) & 1) and (b2 == 255 or bool((c >> b2) & 1))
        if P["DIR"] or u == S or v == T:
            way = 1
        elif v == S or u == T:
            way = 2
        else:
            way = 0
        work.append((u, v, w, way))
    changed = True
    while changed:
        changed = False
        for u, v, w, way in work:
            if not w:
                continue
            if u == S:  # out of s only: s's word is all ones
                if not r[v]:
                    r[v] = changed = True
                continue
            if way in (0, 1) and r[u] and not r[v]:
                r[v] = changed = True
            if way in (0, 2) and r[v] and not r[u]:
                r[u] = changed = True
    return r[T]


def _bfs_verdict(n, arcs, s, t, up, directed):
    adj = [[] for _ in range(n)]
    for i, (a, b) in enumerate(arcs):
        if up[i]:
            adj[a].append(b)
            if not directed:
                adj[b].append(a)
    seen = {s}
    stack = [s]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return t in seen


def _cases():
    rng = np.random.default_rng(2209)
    out = [("bridge", W.bridge(), False), ("series7", W.series(7, np.full(7, 0.9)), False),
           ("ppaths3", W.parallel_paths(3, np.full(6, 0.9)), False), ("grid3x3", W.grid(3, 3), False),
           ("grid2x5", W.grid(2, 5), False)]
    for seed in range(4):
        out.append((f"rand{seed}", W.random_connected(8, 11, seed=900 + seed), False))
    out.append(("multi", W.random_multigraph(6, 11, seed=77), False))
    # a small digraph: random arcs with random orientation
    for seed in range(2):
        n, m = 7, 12
        arcs = [tuple(int(x) for x in rng.choice(n, 2, replace=False)) for _ in range(m)]
        out.append((f"di{seed}", W.Network(f"di{seed}", n, arcs, 0, n - 1, np.full(m, 0.9)), True))
    return out


@pytest.mark.parametrize("series", [0, 1])
@pytest.mark.parametrize("name,net,directed", _cases(), ids=[c[0] for c in _cases()])
def test_plan_verdicts_match_search(name, net, directed, series):
    B = _B()
    old = B.bat_get_option("BAT_SERIES")
    try:
        B.bat_set_option("BAT_SERIES", series)
        src = B.bat_jit_source(net.n, net.arcs, net.s, net.t, perm=0, directed=directed)
    finally:
        B.bat_set_option("BAT_SERIES", old)
    P = _plan(src)
    m = len(net.arcs)
    assert m <= 14
    if series == 0 or directed:
        assert all(b == 255 for b in P["RB2"])
    for c in range(1 << m):
        up = [bool((c >> (m - 1 - i)) & 1) for i in range(m)]  # kind 0: arc i on counter bit m-1-i
        assert _plan_verdict(P, c) == _bfs_verdict(net.n, net.arcs, net.s, net.t, up, directed), (name, c)


def test_series_joining_shrinks_the_plan():
    """A path of 7 arcs keeps s, t and every second inner node; the ladder
    loses its two free corners; digraphs and graphs without degree-2 nodes
    keep their plans."""
    B = _B()
    def plan(net, series, directed=False):
        old = B.bat_get_option("BAT_SERIES")
        try:
            B.bat_set_option("BAT_SERIES", series)
            return _plan(B.bat_jit_source(net.n, net.arcs, net.s, net.t, perm=0, directed=directed))
        finally:
            B.bat_set_option("BAT_SERIES", old)
    path = W.series(7, np.full(7, 0.9))
    p0, p1 = plan(path, 0), plan(path, 1)
    assert (p0["N"], p0["NR"]) == (8, 7) and (p1["N"], p1["NR"]) == (5, 4)
    assert sum(b != 255 for b in p1["RB2"]) == 3
    ladder = W.grid(2, 6)
    q0, q1 = plan(ladder, 0), plan(ladder, 1)
    assert (q1["N"], q1["NR"]) == (q0["N"] - 2, q0["NR"] - 2)
    g5 = W.config2()
    assert plan(g5, 1)["N"] == 23 and plan(g5, 1)["NR"] == 38
    d0, d1 = plan(path, 0, True), plan(path, 1, True)
    assert d0 == d1
