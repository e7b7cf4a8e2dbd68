"""Pins for the multi-state oracle (arcs with sigma_i states, demand d).

The paper sizes the multi-state solution space (Section 4.1) and names the
multi-state problem as future work (Section 6) without defining its
reliability, so these pins come from mathematics, not from printed values:
the binary problem it must reduce to bit for bit, a different max-flow code
(scipy's) with exact rational probabilities, closed forms for series and
parallel arcs, states that merge into the binary case, and invariants.
"""
import itertools
import random
from fractions import Fraction

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import maximum_flow

import bat_workloads as W
import oracle

EPS = 2.0 ** -53


def _scipy_flow(n, arcs, capx, s, t, directed=False):
    rows, cols, vals = [], [], []
    for (u, v), c in zip(arcs, capx):
        if u == v or c == 0:
            continue
        rows.append(u); cols.append(v); vals.append(int(c))
        if not directed:
            rows.append(v); cols.append(u); vals.append(int(c))
    if not vals:
        return 0
    g = csr_matrix((np.array(vals, dtype=np.int32), (rows, cols)), shape=(n, n))
    return int(maximum_flow(g, s, t).flow_value)


def _brute(n, arcs, sigma, cap, w, s, t, d, directed=False):
    """Exact R_d and count: every vector, scipy's max flow, Fractions."""
    R, cnt = Fraction(0), 0
    for x in itertools.product(*[range(k) for k in sigma]):
        capx = [cap[i][x[i]] for i in range(len(arcs))]
        if _scipy_flow(n, arcs, capx, s, t, directed) >= d:
            cnt += 1
            pr = Fraction(1)
            for i in range(len(arcs)):
                pr *= Fraction(float(w[i][x[i]]))
            R += pr
    return R, cnt


def _random_case(rng, n_max=6, m_max=7, s_max=4):
    n = rng.randint(2, n_max)
    m = rng.randint(0, m_max)
    arcs = [(rng.randrange(n), rng.randrange(n)) for _ in range(m)]
    sigma = [rng.randint(1, s_max) for _ in range(m)]
    cap = [[rng.randint(0, 3) for _ in range(k)] for k in sigma]
    w = []
    for k in sigma:
        raw = [rng.random() + 0.05 for _ in range(k)]
        tot = sum(raw)
        w.append([r / tot for r in raw])
    s, t = rng.sample(range(n), 2)
    return n, arcs, sigma, cap, w, s, t


# ------------------------------------------------------------- enumeration

def test_two_states_is_the_binary_bat_order():
    """With two states per arc the generalised update is Rule 1: the same
    64 vectors in the order of Table 2 (Section 3.1)."""
    assert oracle.ms_sequence([2] * 6) == oracle.bat_sequence(6)
    for c in (0, 16, 30, 63):
        assert oracle.ms_decode([2] * 6, c) == oracle.dec_inv(6, c)


def test_mixed_radix_order():
    seq = oracle.ms_sequence([3, 2, 2])
    assert len(seq) == 12 == len(set(seq))
    assert seq[:5] == [(0, 0, 0), (0, 0, 1), (0, 1, 0), (0, 1, 1), (1, 0, 0)]
    assert seq[-1] == (2, 1, 1)
    assert seq == sorted(seq)                       # x_1 most significant
    assert all(oracle.ms_decode([3, 2, 2], c) == x for c, x in enumerate(seq))
    assert oracle.ms_sequence([1, 1]) == [(0, 0)]   # one-state arcs: one vector


# -------------------------------------------------------------- reductions

@pytest.mark.parametrize("seed", range(8))
def test_binary_reduction_is_bit_exact(seed):
    """States (capacity 0, weight 1 - p) and (capacity 1, weight p) with
    d = 1: the same vectors, verdicts and products as the binary oracle, so
    the same bits of R and the same count."""
    rng = random.Random(seed)
    directed = seed % 2 == 1
    net = (W.random_multigraph(rng.randint(3, 7), rng.randint(0, 11), seed=seed, p_lo=0.05, p_hi=0.95)
           if seed % 3 == 0 else W.random_connected(7, 11, seed=seed, p_lo=0.05, p_hi=0.95))
    m = net.m
    w = [[1.0 - float(p), float(p)] for p in net.p]
    ms = oracle.ms_reliability(net.n, net.arcs, [2] * m, [[0, 1]] * m, w, net.s, net.t, 1, directed=directed)
    b = oracle.reliability(net.n, net.arcs, net.p, net.s, net.t, directed=directed)
    assert ms.count == b.count
    assert (ms.sum_hi, ms.sum_lo) == (b.sum_hi, b.sum_lo)


@pytest.mark.parametrize("seed", range(4))
def test_states_with_equal_effect_merge(seed):
    """Demand 1 with capacities 0, 1, 2: states 1 and 2 both carry the one
    unit, so R is the binary R with p_i = w_i(1) + w_i(2); with every
    w_i(k) = 1/3 the count is R_binary(p = 2/3) * 3^m."""
    net = W.random_connected(6, 9, seed=40 + seed)
    rng = np.random.default_rng(seed)
    w = rng.dirichlet([1.0, 1.0, 1.0], size=net.m)
    ms = oracle.ms_reliability(net.n, net.arcs, [3] * net.m, None, w, net.s, net.t, 1)
    b = oracle.reliability(net.n, net.arcs, w[:, 1] + w[:, 2], net.s, net.t)
    assert abs(ms.sum - b.sum) <= 8 * EPS
    third = [[1 / 3] * 3] * net.m
    msu = oracle.ms_reliability(net.n, net.arcs, [3] * net.m, None, third, net.s, net.t, 1)
    bu = oracle.reliability(net.n, net.arcs, [2 / 3] * net.m, net.s, net.t)
    assert msu.count == round(bu.sum * 3 ** net.m)


# ------------------------------------------------------- exact brute force

@pytest.mark.parametrize("seed", range(25))
def test_exact_rational_bruteforce_with_scipy_flow(seed):
    rng = random.Random(1000 + seed)
    n, arcs, sigma, cap, w, s, t = _random_case(rng)
    directed = seed % 4 == 3
    for d in (1, 2, 3):
        R, cnt = _brute(n, arcs, sigma, cap, w, s, t, d, directed)
        r = oracle.ms_reliability(n, arcs, sigma, cap, w, s, t, d, directed=directed)
        assert r.count == cnt, (seed, d)
        assert abs(r.sum - float(R)) <= 4 * EPS * max(1.0, float(R)), (seed, d, r.sum, float(R))


@pytest.mark.parametrize("seed", range(40))
def test_maxflow_against_scipy(seed):
    rng = random.Random(seed)
    n = rng.randint(2, 9)
    arcs = [(rng.randrange(n), rng.randrange(n)) for _ in range(rng.randint(0, 16))]
    capx = [rng.randint(0, 5) for _ in arcs]
    s, t = rng.sample(range(n), 2)
    for directed in (False, True):
        assert oracle.ms_maxflow(n, arcs, capx, s, t, directed) == _scipy_flow(n, arcs, capx, s, t, directed)


# ------------------------------------------------------------ closed forms

def test_series_closed_form():
    """Arcs in series: the flow is the smallest capacity, so
    R_d = prod_i Pr(cap_i >= d)."""
    rng = np.random.default_rng(7)
    k = 5
    w = rng.dirichlet([1.0] * 4, size=k)
    cap = [[0, 1, 2, 3]] * k
    for d in (1, 2, 3, 4):
        r = oracle.ms_reliability(k + 1, [(i, i + 1) for i in range(k)], [4] * k, cap, w, 0, k, d)
        want = float(np.prod([w[i][d:].sum() for i in range(k)]))
        assert abs(r.sum - want) <= 16 * EPS, (d, r.sum, want)
        assert r.count == (4 - d) ** k if d <= 3 else r.count == 0


def test_parallel_closed_form():
    """Arcs in parallel between s and t: the flow is the sum of the
    capacities, so R_d = Pr(sum_i cap_i >= d), an exact convolution."""
    sig = [3, 4, 2]
    cap = [[0, 1, 2], [0, 1, 1, 3], [0, 2]]
    w = [[Fraction(1, 5), Fraction(3, 10), Fraction(1, 2)],
         [Fraction(1, 10), Fraction(1, 5), Fraction(3, 10), Fraction(2, 5)],
         [Fraction(1, 4), Fraction(3, 4)]]
    dist = {0: Fraction(1)}
    for i in range(3):
        nd = {}
        for tot, pr in dist.items():
            for k in range(sig[i]):
                nd[tot + cap[i][k]] = nd.get(tot + cap[i][k], 0) + pr * w[i][k]
        dist = nd
    wf = [[float(x) for x in row] for row in w]
    for d in range(1, 8):
        r = oracle.ms_reliability(2, [(0, 1)] * 3, sig, cap, wf, 0, 1, d)
        want = sum(p for tot, p in dist.items() if tot >= d)
        assert abs(r.sum - float(want)) <= 8 * EPS, (d, r.sum, float(want))


# -------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", range(6))
def test_invariants(seed):
    rng = random.Random(77 + seed)
    n, arcs, sigma, cap, w, s, t = _random_case(rng, n_max=7, m_max=8, s_max=3)
    prev = 2.0
    for d in range(1, 6):
        r = oracle.ms_reliability(n, arcs, sigma, cap, w, s, t, d)
        assert abs(r.sum + r.U - float(np.prod([sum(x) for x in w]) if w else 1.0)) <= 64 * EPS
        assert r.sum <= prev + 1e-15                    # more demand, less reliability
        prev = r.sum
    huge = sum(max(c) for c in cap) + 1
    r = oracle.ms_reliability(n, arcs, sigma, cap, w, s, t, huge)
    assert r.count == 0 and r.sum == 0.0


def test_range_partition_adds_up():
    net = W.random_connected(6, 8, seed=3)
    sigma = [3, 2, 4, 1, 3, 2, 2, 3]
    rng = np.random.default_rng(0)
    w = [rng.dirichlet([1.0] * k) for k in sigma]
    cap = [list(range(k)) for k in sigma]
    N = int(np.prod(sigma))
    full = oracle.ms_reliability(net.n, net.arcs, sigma, cap, w, net.s, net.t, 2)
    cuts = [0, 1, 77, 500, 701, N]
    parts = [oracle.ms_reliability_range(net.n, net.arcs, sigma, cap, w, net.s, net.t, 2, a, b)
             for a, b in zip(cuts, cuts[1:])]
    assert sum(p.count for p in parts) == full.count
    assert abs(sum(p.sum for p in parts) - full.sum) <= 8 * EPS
    assert sum(p.inspections for p in parts) == full.inspections


# ------------------------------------------------------------ work counter

def test_flow_search_work_hand_values():
    """Residual edges the augmenting-path searches examine, worked out by
    hand on the bridge (0-1, 0-2, 1-2, 1-3, 2-3; s = 0, t = 3; every arc in
    its capacity-1 state, the last vector of the space).  Search 1: node 0's
    2 edges, then node 1's 3 edges reach t (path 0-1-3).  Search 2: node 0's
    2 edges (0-1 is saturated), node 2's 3 edges reach t.  Search 3: node
    0's 2 edges, both saturated: no path."""
    b = W.bridge()
    sig = [2] * 5
    w = [[0.5, 0.5]] * 5
    for d, looks in ((1, 5), (2, 10), (3, 12)):
        r = oracle.ms_reliability_range(b.n, b.arcs, sig, [[0, 1]] * 5, w, b.s, b.t, d, 31, 32)
        assert r.inspections == looks, (d, r.inspections)
        assert r.count == (1 if d <= 2 else 0)


# -------------------------------------------------------------- validation

def test_validation_codes():
    arcs = [(0, 1), (1, 2)]
    ok = dict(sigma=[2, 3], cap=[[0, 1], [0, 1, 2]], w=[[0.5, 0.5], [0.2, 0.3, 0.5]])
    assert oracle.ms_validate(3, arcs, ok["sigma"], ok["cap"], ok["w"], 0, 2, 1) == 0
    assert oracle.ms_validate(3, arcs, ok["sigma"], ok["cap"], ok["w"], 0, 2, 0) == oracle.ORC_EINVAL
    assert oracle.ms_validate(3, arcs, ok["sigma"], ok["cap"], ok["w"], 1, 1, 1) == oracle.ORC_EINVAL
    assert oracle.ms_validate(3, arcs, [2, 0], [[0, 1], []], [[0.5, 0.5], []], 0, 2, 1) == oracle.ORC_EINVAL
    assert oracle.ms_validate(3, arcs, ok["sigma"], [[0, 1], [0, -1, 2]], ok["w"], 0, 2, 1) == oracle.ORC_EINVAL
    assert oracle.ms_validate(3, arcs, ok["sigma"], ok["cap"], [[0.5, 0.5], [0.2, 1.3, 0.5]], 0, 2, 1) \
        == oracle.ORC_EINVAL
    big = [(0, 1)] * 40
    assert oracle.ms_validate(3, big, [3] * 40, None, [[1 / 3] * 3] * 40, 0, 2, 1) == oracle.ORC_ETOOBIG
