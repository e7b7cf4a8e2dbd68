"""Pins for the CPU oracle: what the paper prints and what mathematics fixes.

Each test ties the oracle to something other than itself: the paper's worked
tables, closed forms, exact rational enumeration with a different
connectivity algorithm, the factoring theorem, and invariants.  A plausible
slip in the oracle (a dropped (1 - p) factor, a reversed coordinate order,
a wrong sign in the gradient, directed arcs, a layer that revisits nodes)
fails at least one of them.
"""
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import bat_workloads as W
import oracle
from oracle import frontier_dp, pbat
from exact_ref import brute, factoring, layered_search_work

GOLD = os.path.join(os.path.dirname(__file__), "golden")
EPS = 2.0 ** -53


def _read(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _close_rel(a, b, rel):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300)


# ----------------------------------------------------------- Section 3.1 / 4

def test_table2_backward_order():
    rows = _read("table2_backward_bat_m6.txt")
    want = [tuple(int(v) for v in r[1:]) for r in rows]
    assert [int(r[0]) for r in rows] == list(range(1, 65))
    assert oracle.bat_sequence(6) == want          # Rule 1 from X_1 = 0
    for i, x in enumerate(want, start=1):
        assert oracle.dec_inv(6, i - 1) == x       # Eq. 3
        assert oracle.dec(x) + 1 == i              # Eq. 2


def test_rule1_examples_section_3_1():
    seq = oracle.bat_sequence(3)
    assert seq[seq.index((1, 0, 0)) + 1] == (1, 0, 1)
    assert seq[seq.index((1, 0, 1)) + 1] == (1, 1, 0)
    assert seq[-1] == (1, 1, 1) and len(seq) == 8   # Rule 2 halts at (1,1,1)


def test_dec_examples_section_4_2():
    assert oracle.dec((0, 1, 0, 0, 0, 0)) + 1 == 17
    assert oracle.dec((0, 1, 1, 1, 1, 0)) + 1 == 31
    assert oracle.dec_inv(6, 16) == (0, 1, 0, 0, 0, 0)
    assert oracle.dec_inv(6, 30) == (0, 1, 1, 1, 1, 0)


def test_forward_bat_section_4_2():
    """Forward BAT (updates from x_1): the worked examples of Section 4.2
    (X_3 = (0,1,0,0,0,0), X_31 = (0,1,1,1,1,0) with X_1 = 0), the update
    rule agreeing with the decoding, and the forward order of X being the
    backward order of the reversed coordinate list."""
    assert oracle.dec_inv_fwd(6, 3 - 1) == (0, 1, 0, 0, 0, 0)
    assert oracle.dec_inv_fwd(6, 31 - 1) == (0, 1, 1, 1, 1, 0)
    seq = oracle.bat_sequence(6, forward=True)
    assert len(seq) == 64 and len(set(seq)) == 64
    assert seq == [oracle.dec_inv_fwd(6, c) for c in range(64)]
    back = oracle.bat_sequence(6)
    assert seq == [tuple(reversed(x)) for x in back]
    # the first forward step sets x_1; the last vector is all ones
    assert seq[1] == (1, 0, 0, 0, 0, 0) and seq[-1] == (1,) * 6


def test_forward_ranges_match_reversed_backward_ranges():
    net = W.random_connected(9, 14, seed=404, p_lo=0.2, p_hi=0.95)
    m = net.m
    full_f = oracle.reliability_range(net.n, net.arcs, net.p, net.s, net.t, 0, 1 << m, forward=True)
    full_b = oracle.reliability(net.n, net.arcs, net.p, net.s, net.t)
    assert full_f.count == full_b.count and abs(full_f.sum - full_b.sum) <= 1e-14
    rev = list(reversed(net.arcs))
    prev = np.ascontiguousarray(net.p[::-1])
    for lo, hi in [(0, 1000), (777, 5432), (1 << 13, (1 << 14) - 3)]:
        f = oracle.reliability_range(net.n, net.arcs, net.p, net.s, net.t, lo, hi, forward=True, grad=True)
        b = oracle.reliability_range(net.n, rev, prev, net.s, net.t, lo, hi, grad=True)
        # same terms; only the product order inside each Pr(X) is reversed
        assert f.count == b.count and abs(f.sum - b.sum) <= 1e-15 * f.sum
        assert np.allclose(f.T1, b.T1[::-1], rtol=1e-14, atol=0)
        assert np.allclose(f.T0, b.T0[::-1], rtol=1e-14, atol=0)


def test_equal_divisions_section_4_3_4_4():
    # chi = 4, m = 6: mu = 16; the divisions start at X_1, X_17, X_33, X_49
    starts = [pbat.division_bounds(6, 4, i)[0] + 1 for i in range(1, 5)]
    assert starts == [1, 17, 33, 49]
    # X_{2,16} = X_32 = (0,1,1,1,1,1): last vector of division 2
    lo, hi = pbat.division_bounds(6, 4, 2)
    assert oracle.dec_inv(6, hi - 1) == (0, 1, 1, 1, 1, 1)
    # Eq. 7: the first log2(chi) coordinates are the i-th vector of B^(2)
    assert [pbat.division_prefix(6, 4, i) for i in range(1, 5)] == [(0, 0), (0, 1), (1, 0), (1, 1)]
    for i in range(1, 5):
        lo, hi = pbat.division_bounds(6, 4, i)
        pre = pbat.division_prefix(6, 4, i)
        assert oracle.dec_inv(6, lo)[:2] == pre and oracle.dec_inv(6, hi - 1)[:2] == pre
    # mu = 2^m / chi for chi = 2^0 .. 2^4
    for d in range(5):
        lo, hi = pbat.division_bounds(6, 1 << d, 1)
        assert hi - lo == 64 >> d


# ------------------------------------------------------------- Section 3.2

def test_table3_plsa_layers():
    rows = _read("table3_plsa_layers.txt")
    f = W.figure1()
    conn, nl, lay = oracle.plsa(f.n, f.arcs, f.s, f.t, [1] * f.m)
    assert conn and nl == 3
    for r in rows:
        layer = int(r[0])
        nodes = sorted(int(v) for v in r[1:])
        got = sorted(i + 1 for i in range(f.n) if lay[i] == layer)
        assert got == nodes


def test_plsa_stops_on_empty_layer():
    # s isolated: L_2 is empty at once (STEP P2)
    conn, nl, lay = oracle.plsa(3, [(1, 2)], 0, 2, [1])
    assert not conn and nl == 1


# The layered search's work counters (layers built, arc inspections) are the
# algorithmic work the benchmark's roofline divides by, so they are pinned
# like any other output: values worked out by hand on small cases, and an
# independently written set-based search (tests/exact_ref.py) over whole
# ranges.  An inspection is one look at one arc end of a node being expanded,
# whatever the arc's state: counting only working arcs, or counting the
# expansion of the layer that holds t, fails the hand values below.

@pytest.mark.parametrize("case", [
    # Figure 1, every arc working (Table 3): expand {1}: 2 ends; expand
    # {2, 3}: 4 + 2 ends; t = 4 joins layer 3.
    ("figure1", None, (1, 1, 1, 1, 1, 1), False, (True, 3, 8)),
    # bridge 0-1, 0-2, 1-2, 1-3, 2-3, s = 0, t = 3, all working: 2 + (3 + 3)
    ("bridge", None, (1, 1, 1, 1, 1), False, (True, 3, 8)),
    # only 0-1 works: {0} 2 ends -> {1}; {1} 3 ends -> nothing new
    ("bridge", None, (1, 0, 0, 0, 0), False, (False, 2, 5)),
    # nothing works: {0} 2 ends, layer 2 empty
    ("bridge", None, (0, 0, 0, 0, 0), False, (False, 1, 2)),
    # 0-2 and 2-3 work: {0} 2 ends -> {2}; {2} 3 ends -> {3} = t
    ("bridge", None, (0, 1, 0, 0, 1), False, (True, 3, 5)),
    # directed bridge, all working: out-ends only, 2 + (2 + 1)
    ("bridge", None, (1, 1, 1, 1, 1), True, (True, 3, 5)),
    # a self-loop at s is one end: {0} 2 ends -> {1}; {1} 2 ends -> {2}
    ("custom", (3, [(0, 0), (0, 1), (1, 2)], 0, 2), (1, 1, 1), False, (True, 3, 4)),
    # parallel arcs are separate ends, a failed copy still inspected: {0}
    # 2 ends -> {1}; {1} 3 ends (both copies and 1-2, which is down)
    ("custom", (3, [(0, 1), (0, 1), (1, 2)], 0, 2), (0, 1, 0), False, (False, 2, 5)),
])
def test_plsa_work_hand_values(case):
    kind, g, x, directed, want = case
    if kind == "figure1":
        f = W.figure1()
        n, arcs, s, t = f.n, f.arcs, f.s, f.t
    elif kind == "bridge":
        b = W.bridge()
        n, arcs, s, t = b.n, b.arcs, b.s, b.t
    else:
        n, arcs, s, t = g
    assert oracle.plsa_work(n, arcs, s, t, x, directed=directed) == want
    assert layered_search_work(n, arcs, s, t, x, directed=directed) == want


def _range_work(n, arcs, s, t, m, lo, hi, directed=False):
    lay = insp = 0
    for c in range(lo, hi):
        x = [(c >> (m - 1 - i)) & 1 for i in range(m)]   # arc i at bit m-1-i (Eq. 3)
        _, l, k = layered_search_work(n, arcs, s, t, x, directed=directed)
        lay += l
        insp += k
    return lay, insp


@pytest.mark.parametrize("seed", range(12))
def test_range_work_counters_against_independent_search(seed):
    """Whole-range layer and inspection totals equal the set-based search's."""
    rng = random.Random(seed)
    directed = seed % 3 == 2
    if seed % 2:
        net = W.random_multigraph(rng.randint(3, 7), rng.randint(1, 10), seed=seed, p_lo=0.1, p_hi=0.9)
    else:
        n = rng.randint(4, 8)
        net = W.random_connected(n, rng.randint(n - 1, min(11, n * (n - 1) // 2)), seed=seed)
    m = net.m
    r = oracle.reliability_range(net.n, net.arcs, net.p, net.s, net.t, 0, 1 << m, directed=directed)
    assert (r.layers, r.inspections) == _range_work(net.n, net.arcs, net.s, net.t, m, 0, 1 << m, directed)


def test_range_work_counters_grid_sample():
    """The 5x5 grid's counters (the headline's work per vector) on spread
    slices of Eq. 6 divisions, the way the benchmark samples them."""
    net = W.config2()
    m, chi = net.m, 1 << 17
    for i in pbat.spread_divisions(chi, 4):
        lo, _ = pbat.division_bounds(m, chi, i)
        r = oracle.reliability_range(net.n, net.arcs, net.p, net.s, net.t, lo, lo + 300)
        assert (r.layers, r.inspections) == _range_work(net.n, net.arcs, net.s, net.t, m, lo, lo + 300)
    # the harness adds the divisions' counters in full
    divs = pbat.spread_divisions(1 << 30, 3)
    pr = pbat.run(net.n, net.arcs, net.p, net.s, net.t, 1 << 30, divisions=divs, processes=1)
    want = [0, 0]
    for i in divs:
        lo, hi = pbat.division_bounds(m, 1 << 30, i)
        w = _range_work(net.n, net.arcs, net.s, net.t, m, lo, hi)
        want[0] += w[0]
        want[1] += w[1]
    assert (pr.layers, pr.inspections) == tuple(want)


# ---------------------------------------------------------- Section 5.2 / 5.3

def test_table4_figure1():
    rows = _read("table4_figure1_pbat.txt")
    per = {int(r[0]): (tuple(int(v) for v in r[1:7]), r[7]) for r in rows if r[0].isdigit()}
    divs = [float(v) for v in next(r for r in rows if r[0] == "division_sums")[1:]]
    R_print = next(r for r in rows if r[0] == "R")[1]
    f = W.figure1()
    conn_idx = []
    for c in range(64):
        x = oracle.dec_inv(6, c)
        ok, _, _ = oracle.plsa(f.n, f.arcs, f.s, f.t, x)
        if ok:
            conn_idx.append(c + 1)
    assert conn_idx == sorted(per)                       # the 25 connected vectors
    for i, (x, txt) in per.items():
        assert oracle.dec_inv(6, i - 1) == x
        val = oracle.pr(f.p, x)
        mant, ex = txt.split("E")
        ulp = 10.0 ** (int(ex) - (len(mant.replace(".", "")) - 1))
        assert abs(val - float(txt)) <= 0.5 * ulp + 1e-18, (i, val, txt)
    r = oracle.net_reliability(f)
    assert r.count == 25
    assert abs(r.sum - float(R_print)) <= 0.5e-9             # printed to 9 decimals
    assert _close_rel(r.sum, 4800878611 / 5000000000, 4 * EPS)
    # Table 4 SUM row: chi = 4 division sums (printed to 5 significant digits)
    pr = pbat.run(f.n, f.arcs, f.p, f.s, f.t, 4, processes=1)
    for got, want in zip(pr.division_R, divs):
        tol = 0.5e-4 * 10 ** math.floor(math.log10(want)) if want > 0 else 0.0
        assert abs(got - want) <= tol + 1e-18
    # Table 1's listed order gives the same R (symmetric connected set)
    r2 = oracle.net_reliability(W.figure1(reversed_table1=False))
    assert _close_rel(r2.sum, r.sum, 4 * EPS) and r2.count == 25


def test_table6_row1_bridge_undirected():
    n, m, N, R = _read("table6_bridge.txt")[0]
    b = W.bridge(0.9)
    assert (b.n, b.m, 1 << b.m) == (int(n), int(m), int(N))
    r = oracle.net_reliability(b)
    assert abs(r.sum - float(R)) <= 0.5e-10
    assert r.count == 16
    assert _close_rel(r.sum, 12231 / 12500, 4 * EPS)
    # the directed reading of "directed path" does not reproduce Table 6
    rd = oracle.net_reliability(b, directed=True)
    assert abs(rd.sum - float(R)) > 1e-3
    Rd, cd, *_ = brute(b.n, b.arcs, b.p, b.s, b.t, directed=True)
    assert rd.count == cd == 15 and _close_rel(rd.sum, float(Rd), 8 * EPS)


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("pv", [0.0, 0.1, 0.5, 0.73, 0.9, 0.999, 1.0])
def test_bridge_closed_form(pv):
    r = oracle.net_reliability(W.bridge(pv))
    want = 2 * pv**2 + 2 * pv**3 - 5 * pv**4 + 2 * pv**5
    assert abs(r.sum - want) <= 1e-15
    assert r.count == 16


def test_series_parallel_closed_forms():
    rng = np.random.default_rng(7)
    for m in (1, 2, 5, 9):
        p = rng.uniform(0.05, 0.95, size=m)
        r = oracle.net_reliability(W.series(m, p))
        assert r.count == 1 and _close_rel(r.sum, float(np.prod(p)), (m + 2) * EPS)
        r = oracle.net_reliability(W.parallel(m, p))
        assert r.count == (1 << m) - 1
        assert _close_rel(r.sum, 1.0 - float(np.prod(1 - p)), 1e-14)
    for j in (1, 2, 3, 5):
        p = rng.uniform(0.05, 0.95, size=2 * j)
        r = oracle.net_reliability(W.parallel_paths(j, p))
        assert r.count == 4**j - 3**j
        want = 1.0 - float(np.prod([1 - p[2 * i] * p[2 * i + 1] for i in range(j)]))
        assert _close_rel(r.sum, want, 1e-14)


def test_empty_arc_set():
    r = oracle.reliability(3, np.zeros((0, 2), np.int32), np.zeros(0), 0, 2)
    assert r.count == 0 and r.sum == 0.0 and r.U == 1.0


# ------------------------------------------------------ exact enumeration

def _rand_cases(k, seed):
    rng = random.Random(seed)
    out = []
    for i in range(k):
        n = rng.randint(2, 7)
        m = rng.randint(0, 10)
        arcs = [(rng.randrange(n), rng.randrange(n)) for _ in range(m)]   # loops + parallels allowed
        s, t = rng.sample(range(n), 2)
        p = [rng.choice([0.0, 1.0, 0.5, rng.random(), rng.random(), rng.random()]) for _ in range(m)]
        out.append((n, arcs, p, s, t))
    return out


@pytest.mark.parametrize("case", _rand_cases(40, 11))
def test_exact_rational_bruteforce(case):
    n, arcs, p, s, t = case
    m = len(arcs)
    R, cnt, U, T1, T0 = brute(n, arcs, p, s, t)
    r = oracle.reliability(n, np.asarray(arcs, np.int32).reshape(-1, 2), p, s, t, grad=True)
    tol = (m + 4) * EPS
    assert r.count == cnt
    assert abs(r.sum - float(R)) <= tol * float(R) + 1e-300
    assert abs(r.U - float(U)) <= tol * float(U) + 1e-300
    for i in range(m):
        assert abs(r.T1[i] - float(T1[i])) <= tol * float(T1[i]) + 1e-300
        assert abs(r.T0[i] - float(T0[i])) <= tol * float(T0[i]) + 1e-300


@pytest.mark.parametrize("seed", range(6))
def test_factoring_theorem(seed):
    rng = random.Random(100 + seed)
    n = rng.randint(4, 8)
    m = rng.randint(n - 1, min(14, n * (n - 1) // 2))
    net = W.random_connected(n, m, seed=seed, p_lo=0.05, p_hi=0.95)
    want = factoring(net.n, net.arcs, net.p, net.s, net.t)
    r = oracle.net_reliability(net)
    assert abs(r.sum - float(want)) <= (m + 4) * EPS * float(want)


# ------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", range(4))
def test_half_probability_is_count(seed):
    net = W.random_connected(9, 15 + seed, seed=seed)
    r = oracle.net_reliability(net, p=np.full(net.m, 0.5))
    assert r.sum == r.count * 2.0 ** -net.m        # bit-exact: all partial sums are dyadic


def test_p_one_and_zero():
    net = W.random_connected(8, 13, seed=3)
    assert oracle.net_reliability(net, p=np.ones(net.m)).sum == 1.0
    r0 = oracle.net_reliability(net, p=np.zeros(net.m))
    assert r0.sum == 0.0 and r0.U == 1.0


@pytest.mark.parametrize("seed", range(4))
def test_connected_plus_disconnected_is_one(seed):
    net = W.random_connected(10, 16, seed=20 + seed, p_lo=0.01, p_hi=0.99)
    r = oracle.net_reliability(net)
    assert abs(r.sum + r.U - 1.0) <= 4e-15


@pytest.mark.parametrize("seed", range(3))
def test_relabel_and_permutation_invariance(seed):
    net = W.random_connected(9, 16, seed=40 + seed)
    rng = np.random.default_rng(seed)
    perm_arcs = rng.permutation(net.m)
    perm_nodes = rng.permutation(net.n)
    arcs2 = [(int(perm_nodes[net.arcs[e][0]]), int(perm_nodes[net.arcs[e][1]])) for e in perm_arcs]
    p2 = net.p[perm_arcs]
    r1 = oracle.net_reliability(net, grad=True)
    r2 = oracle.reliability(net.n, arcs2, p2, int(perm_nodes[net.s]), int(perm_nodes[net.t]), grad=True)
    assert r1.count == r2.count
    assert _close_rel(r1.sum, r2.sum, 1e-14)
    assert np.allclose(r1.T1[perm_arcs], r2.T1, rtol=1e-14, atol=0)
    assert np.allclose(r1.T0[perm_arcs], r2.T0, rtol=1e-14, atol=0)


# ---------------------------------------------------------------- gradient

@pytest.mark.parametrize("seed", range(3))
def test_gradient_birnbaum_and_fd(seed):
    net = W.random_connected(8, 12, seed=60 + seed, p_lo=0.2, p_hi=0.95)
    r = oracle.net_reliability(net, grad=True)
    h = 1e-6
    for i in range(net.m):
        q = net.p.copy()
        q[i] = 1.0
        R1 = oracle.net_reliability(net, p=q).sum
        q[i] = 0.0
        R0 = oracle.net_reliability(net, p=q).sum
        assert abs(r.T1[i] - R1) <= 1e-14 and abs(r.T0[i] - R0) <= 1e-14
        q = net.p.copy()
        q[i] += h
        Rp = oracle.net_reliability(net, p=q).sum
        q[i] -= 2 * h
        Rm = oracle.net_reliability(net, p=q).sum
        g_fd = (Rp - Rm) / (2 * h)                 # exact up to rounding: R is multilinear
        assert abs(g_fd - r.grad[i]) <= 1e-9
        assert r.grad[i] >= -1e-15                 # monotone structure function
        # R = p_i T1_i + (1 - p_i) T0_i
        assert abs(net.p[i] * r.T1[i] + (1 - net.p[i]) * r.T0[i] - r.sum) <= 1e-14


def test_gradient_at_boundary_probabilities():
    # p_i in {0, 1}: the prefix/suffix products need no division
    net = W.bridge(0.9)
    p = np.array([1.0, 0.0, 0.7, 1.0, 0.0])
    R, cnt, U, T1, T0 = brute(net.n, net.arcs, p, net.s, net.t)
    r = oracle.net_reliability(net, p=p, grad=True)
    assert np.allclose(r.T1, [float(v) for v in T1], rtol=0, atol=1e-16)
    assert np.allclose(r.T0, [float(v) for v in T0], rtol=0, atol=1e-16)


# ------------------------------------------------------------ harnesses

def test_pbat_matches_single_range():
    net = W.random_connected(10, 18, seed=5)
    full = oracle.net_reliability(net, grad=True)
    for chi in (1, 2, 8, 64):
        pr = pbat.run(net.n, net.arcs, net.p, net.s, net.t, chi, grad=True, processes=4)
        assert pr.count == full.count
        assert _close_rel(pr.R, full.sum, 4 * EPS)
        assert np.allclose(pr.T1, full.T1, rtol=4 * EPS, atol=0)
        assert np.allclose(pr.T0, full.T0, rtol=4 * EPS, atol=0)
    a = pbat.run(net.n, net.arcs, net.p, net.s, net.t, 16, processes=1)
    b = pbat.run(net.n, net.arcs, net.p, net.s, net.t, 16, processes=4)
    assert a.R_hi == b.R_hi and a.R_lo == b.R_lo       # fixed-order combine


@pytest.mark.parametrize("net", [W.grid(2, 3), W.grid(3, 3), W.grid(3, 4), W.figure1(), W.bridge(0.37),
                                 W.random_connected(9, 17, seed=1), W.random_connected(12, 20, seed=2),
                                 W.random_multigraph(6, 12, seed=3, p_lo=0.1, p_hi=0.9)],
                         ids=lambda n: n.name)
def test_frontier_dp_against_oracle(net):
    R, cnt = frontier_dp.reliability(net.n, net.arcs, net.p, net.s, net.t)
    r = oracle.net_reliability(net)
    assert cnt == r.count
    assert _close_rel(R, r.sum, 1e-14)


def test_frontier_dp_against_exact():
    for (n, arcs, p, s, t) in _rand_cases(15, 99):
        R, cnt, *_ = brute(n, arcs, p, s, t)
        Rd, cd = frontier_dp.reliability(n, arcs, p, s, t)
        assert cd == cnt
        assert abs(Rd - float(R)) <= 1e-15 * max(1.0, float(R))


def test_frontier_dp_grid4x4_against_oracle():
    net = W.grid(4, 4).with_p(np.random.default_rng(3).uniform(0.6, 0.99, 24))
    R, cnt = frontier_dp.reliability(net.n, net.arcs, net.p, net.s, net.t)
    pr = pbat.run(net.n, net.arcs, net.p, net.s, net.t, 64, processes=os.cpu_count())
    assert cnt == pr.count
    assert _close_rel(R, pr.R, 1e-14)


# ------------------------------------------------------------- validation

def test_validation_codes():
    arcs = [(0, 1), (1, 2)]
    assert oracle.validate(3, arcs, [0.5, 0.5], 0, 2) == 0
    assert oracle.validate(3, arcs, [0.5, 0.5], 1, 1) == oracle.ORC_EINVAL
    assert oracle.validate(1, [], [], 0, 0) == oracle.ORC_EINVAL
    assert oracle.validate(3, [(0, 3)], [0.5], 0, 2) == oracle.ORC_EINVAL
    assert oracle.validate(3, arcs, [0.5, float("nan")], 0, 2) == oracle.ORC_EINVAL
    assert oracle.validate(3, arcs, [0.5, 1.5], 0, 2) == oracle.ORC_EINVAL
    assert oracle.validate(3, arcs, [-0.1, 0.5], 0, 2) == oracle.ORC_EINVAL
    assert oracle.validate(3, [(0, 1)] * 63, [0.5] * 63, 0, 2) == oracle.ORC_ETOOBIG
