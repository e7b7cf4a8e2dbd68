"""GPU parity for multi-state arcs: the HIP flow sweep against the oracle.

Bars: counts bit-exact; R within 1e-12 relative (absolute when R = 0).
Parity here is against the multi-state oracle, which the paper does not
pin (it defines only the binary problem); the oracle is pinned by the binary
reduction, scipy's max flow with exact rationals and closed forms
(tests/test_ms_oracle.py).
"""
import os
import sys

import numpy as np
import pytest

import bat_workloads as W
import oracle

pytestmark = pytest.mark.gpu

REL = 1e-12


def _B():
    import paper_2209_09711_amd as B
    return B


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ok(got, want):
    return got == want == 0.0 or abs(got - want) <= REL * abs(want)


def _both(net, directed=False):
    B = _B()
    R, c = B.bat_ms_reliability(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, net.d, directed=directed)
    o = oracle.ms_reliability(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, net.d, directed=directed)
    return R, c, o


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("directed", [False, True])
def test_bridge_three_levels(d, directed):
    net = W.ms_bridge(d)
    say("ms bridge", d, directed)
    R, c, o = _both(net, directed)
    assert c == o.count and _ok(R, o.sum), (R, o.sum, c, o.count)


@pytest.mark.parametrize("seed", range(6))
def test_binary_states_match_binary_path(seed):
    """Two states of capacity 0 and 1 with d = 1 are the binary problem:
    the multi-state sweep equals the binary HIP path and the binary oracle."""
    B = _B()
    net = W.random_connected(9, 15, seed=seed, p_lo=0.1, p_hi=0.95) if seed % 2 else \
        W.random_multigraph(7, 13, seed=seed, p_lo=0.1, p_hi=0.95)
    m = net.m
    w = [[1.0 - float(p), float(p)] for p in net.p]
    say("ms binary", net.name)
    R, c = B.bat_ms_reliability(net.n, net.arcs, [2] * m, [[0, 1]] * m, w, net.s, net.t, 1)
    Rb, cb = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
    o = oracle.reliability(net.n, net.arcs, net.p, net.s, net.t)
    assert c == cb == o.count
    assert _ok(R, o.sum) and _ok(Rb, o.sum)


@pytest.mark.parametrize("seed", range(24))
def test_mixed_states_against_oracle(seed):
    """Multigraphs with self-loops and parallel arcs, 1-4 states per arc,
    capacities 0-3, demands 1-3, both directions of arc reading."""
    rng = np.random.default_rng(seed)
    net = W.ms_mixed(int(rng.integers(2, 9)), int(rng.integers(0, 12)), seed=seed)
    directed = seed % 3 == 2
    say("ms mixed", seed, net.name, net.space, net.d, directed)
    R, c, o = _both(net, directed)
    assert c == o.count and _ok(R, o.sum), (seed, R, o.sum, c, o.count)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_random_three_levels(d):
    net = W.ms_random(8, 13, seed=100 + d, d=d)
    say("ms random", net.name, net.space)
    R, c, o = _both(net)
    assert c == o.count and _ok(R, o.sum)


def test_ranges_against_oracle():
    """Index ranges in the mixed-radix order of the caller's arcs: ragged
    lengths, a single vector, the last vector, an empty range."""
    B = _B()
    net = W.ms_random(9, 14, seed=7, d=2)
    N = net.space
    cases = [(0, N), (0, 1), (N - 1, N), (12345, 12345), (777, 777 + 64 * 37 + 5), (N // 3, N // 3 + 100003)]
    for lo, hi in cases:
        say("ms range", lo, hi)
        r = B.bat_ms_reliability_range(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, net.d, lo, hi)
        o = oracle.ms_reliability_range(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, net.d, lo, hi)
        assert r.count == o.count and _ok(r.R, o.sum), (lo, hi, r.R, o.sum)


@pytest.mark.parametrize("run", [1, 2, 3, 7, 64])
def test_lane_runs(run):
    """Lanes deciding several consecutive vectors: the shortcuts along the
    fastest coordinate (settling its later states at once when a vector meets
    the demand, passing the flow on when it does not) against the oracle,
    with capacities that rise with the state (shortcuts on) and that do not
    (shortcuts off), over whole spaces and ragged ranges."""
    B = _B()
    old = B.bat_get_option("BAT_MS_RUN")
    try:
        B.bat_set_option("BAT_MS_RUN", run)
        for seed in range(6):
            net = W.ms_random(7, 11, seed=300 + seed, d=1 + seed % 3)
            if seed % 2:
                net.cap = [[2, 0, 1]] * net.m           # not monotone in the state
            say("ms run", run, seed)
            R, c, o = _both(net, directed=seed % 3 == 1)
            assert c == o.count and _ok(R, o.sum), (run, seed, R, o.sum)
            N = net.space
            for lo, hi in [(0, N), (5, N - 7), (N // 2, N // 2 + 999)]:
                r = B.bat_ms_reliability_range(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, net.d,
                                               lo, hi)
                oo = oracle.ms_reliability_range(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, net.d,
                                                 lo, hi)
                assert r.count == oo.count and _ok(r.R, oo.sum), (run, seed, lo, hi)
        for seed in range(8):
            net = W.ms_mixed(6, 9, seed=400 + seed)
            R, c, o = _both(net)
            assert c == o.count and _ok(R, o.sum), (run, "mixed", seed)
    finally:
        B.bat_set_option("BAT_MS_RUN", old)


def test_edge_cases():
    B = _B()
    # no arcs: one empty vector, s and t apart
    assert B.bat_ms_reliability(3, [], [], None, [], 0, 2, 1) == (0.0, 0)
    # demand above every capacity sum
    net = W.ms_bridge(11)
    assert B.bat_ms_reliability(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, 11) == (0.0, 0)
    # one-state arcs fix their capacity; 32 arcs and 32 nodes (the limits)
    arcs = [(i, i + 1) for i in range(31)] + [(0, 31)]
    sigma = [1] * 28 + [3] * 4
    cap = [[2]] * 28 + [[0, 1, 2]] * 4
    w = [[1.0]] * 28 + [[0.1, 0.2, 0.7]] * 4
    for d in (1, 2, 3):
        R, c = B.bat_ms_reliability(32, arcs, sigma, cap, w, 0, 17, d)
        o = oracle.ms_reliability(32, arcs, sigma, cap, w, 0, 17, d)
        assert c == o.count and _ok(R, o.sum), (d, R, o.sum)


@pytest.mark.parametrize("m", [16, 17, 20, 21, 24, 25])
def test_slot_instances(m):
    """Arc counts at the edges of the kernel instances (16, 20, 24 and 32
    slots, the rest padded with no-op slots): against the oracle, with
    eight three-level arcs and the rest fixed at one state."""
    B = _B()
    rng = np.random.default_rng(600 + m)
    n = 12
    arcs = [(i, i + 1) for i in range(n - 1)]
    while len(arcs) < m:
        u, v = (int(x) for x in rng.choice(n, 2, replace=False))
        arcs.append((u, v))
    multi = set(int(x) for x in rng.choice(m, 8, replace=False))
    sigma = [3 if i in multi else 1 for i in range(m)]
    cap = [[0, 1, 2] if i in multi else [int(rng.integers(1, 3))] for i in range(m)]
    w = []
    for i in range(m):
        if i in multi:
            q = rng.dirichlet([1.0, 1.0, 1.0])
            w.append([float(x) for x in q])
        else:
            w.append([1.0])
    for d in (1, 2, 3):
        say("ms slots", m, "d", d)
        R, c = B.bat_ms_reliability(n, arcs, sigma, cap, w, 0, n - 1, d)
        o = oracle.ms_reliability(n, arcs, sigma, cap, w, 0, n - 1, d)
        assert c == o.count and _ok(R, o.sum), (m, d, R, o.sum)


def test_workload_full_size_sampled():
    """The benchmark's 3^18-vector workload: the whole sweep (arcs reordered
    for the flow searches) equals the range sweep over the whole counter in
    the caller's order, and spread ranges of it match the oracle."""
    B = _B()
    net = W.config_ms()
    N = net.space
    say("ms workload", net.name, N)
    R, c = B.bat_ms_reliability(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, net.d)
    full = B.bat_ms_reliability_range(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, net.d, 0, N)
    assert c == full.count and _ok(R, full.R)
    assert 0 < c < N
    rng = np.random.default_rng(5)
    for lo in sorted(int(x) for x in rng.integers(0, N - 70001, size=6)):
        hi = lo + 70001
        r = B.bat_ms_reliability_range(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, net.d, lo, hi)
        o = oracle.ms_reliability_range(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, net.d, lo, hi)
        assert r.count == o.count and _ok(r.R, o.sum), (lo, r.R, o.sum)
    # the whole space on the oracle, in 64 equal ranges over the host cores,
    # added in range order
    from oracle import pbat
    cuts = [N * j // 64 for j in range(65)]
    outs, wall = pbat.run_ms_ranges(net, list(zip(cuts, cuts[1:])), processes=min(16, os.cpu_count() or 1))
    hi = lo = 0.0
    for r_, _, _ in outs:
        hi, lo = pbat.dd_add(hi, lo, r_)
    say("ms oracle whole space", wall, "s")
    assert c == sum(o[1] for o in outs) and _ok(R, hi + lo), (R, hi + lo)
    # a lower demand can only be met more often
    R1, c1 = B.bat_ms_reliability(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, 1)
    assert R1 >= R and c1 >= c


def _random_states_net(seed, n, m, states):
    rng = np.random.default_rng(seed)
    arcs = [(i, i + 1) for i in range(n - 1)]
    while len(arcs) < m:
        u, v = (int(x) for x in rng.choice(n, 2, replace=False))
        arcs.append((u, v))
    sigma = [int(rng.choice(states)) for _ in range(m)]
    cap = [[int(rng.integers(0, 3)) for _ in range(k)] for k in sigma]
    w = [[float(x) for x in rng.dirichlet([1.0] * k)] for k in sigma]
    return arcs, sigma, cap, w


@pytest.mark.parametrize("seed", range(8))
def test_bit_sliced_kernel_against_oracle_and_flow(seed):
    """Whole sweeps with demand 1 to 3 run the bit-sliced kernel (the flow
    reaches 1 when t is reachable over arcs of capacity >= 1, 2 when
    besides no single unit-capacity arc separates s and t, 3 when no arc of
    capacity 1 or 2 and no two unit-capacity arcs do): against the
    oracle and against the augmenting-path kernel (option BAT_MS_BITS 0),
    for 1-5 states with capacities 0-2 in any order, both arc readings,
    default runs and runs of at most 3 and 9 uniform steps."""
    B = _B()
    n = 5 + seed % 4
    states = [[2, 3], [1, 2, 3], [3], [2, 4, 5]][seed % 4]
    m = {0: 12, 1: 12, 2: 10, 3: 8}[seed % 4]
    arcs, sigma, cap, w = _random_states_net(700 + seed, n, m, states)
    old_run, old_bits = B.bat_get_option("BAT_MS_RUN"), B.bat_get_option("BAT_MS_BITS")
    try:
        for directed in (False, True):
            for d in (1, 2, 3):
                o = oracle.ms_reliability(n, arcs, sigma, cap, w, 0, n - 1, d, directed=directed)
                B.bat_set_option("BAT_MS_BITS", 0)
                B.bat_set_option("BAT_MS_RUN", 0)
                Rf, cf = B.bat_ms_reliability(n, arcs, sigma, cap, w, 0, n - 1, d, directed=directed)
                assert B.bat_last_launch().specialised == 0
                assert cf == o.count and _ok(Rf, o.sum)
                B.bat_set_option("BAT_MS_BITS", 1)
                for run in (0, 3, 9):
                    B.bat_set_option("BAT_MS_RUN", run)
                    say("ms bits", seed, directed, d, run)
                    R, c = B.bat_ms_reliability(n, arcs, sigma, cap, w, 0, n - 1, d, directed=directed)
                    assert B.bat_last_launch().specialised == 1
                    assert c == o.count and _ok(R, o.sum), (directed, d, run, R, o.sum, c, o.count)
    finally:
        B.bat_set_option("BAT_MS_RUN", old_run)
        B.bat_set_option("BAT_MS_BITS", old_bits)


@pytest.mark.parametrize("states", [2, 32])
def test_bit_sliced_full_words(states):
    """Words of exactly 32 vectors: five two-state arcs, or one arc of 32
    states (capacities 0, 1, 2 repeating)."""
    B = _B()
    n = 6
    arcs = [(0, 1), (1, 5), (0, 2), (2, 5), (1, 2), (0, 3), (3, 4), (4, 5), (3, 1)]
    m = len(arcs)
    rng = np.random.default_rng(states)
    sigma = [states if i == 0 else 2 for i in range(m)]
    cap = [[k % 3 for k in range(s_)] for s_ in sigma]
    w = [[float(x) for x in rng.dirichlet([1.0] * s_)] for s_ in sigma]
    for d in (1, 2, 3):
        say("ms bits full words", states, d)
        R, c = B.bat_ms_reliability(n, arcs, sigma, cap, w, 0, n - 1, d)
        assert B.bat_last_launch().specialised == 1
        o = oracle.ms_reliability(n, arcs, sigma, cap, w, 0, n - 1, d)
        assert c == o.count and _ok(R, o.sum), (d, R, o.sum)


def test_bit_sliced_many_items_against_flow():
    """A 3^16 space (many wavefronts, run slots chosen by the host): the
    bit-sliced kernel against the augmenting-path kernel on the same graph,
    demands 1 to 3, both arc readings."""
    B = _B()
    arcs, sigma, cap, w = _random_states_net(77, 10, 16, [3])
    old = B.bat_get_option("BAT_MS_BITS")
    try:
        for directed in (False, True):
            for d in (1, 2, 3):
                say("ms bits 3^16", directed, d)
                B.bat_set_option("BAT_MS_BITS", 1)
                R, c = B.bat_ms_reliability(10, arcs, sigma, cap, w, 0, 9, d, directed=directed)
                assert B.bat_last_launch().specialised == 1
                B.bat_set_option("BAT_MS_BITS", 0)
                Rf, cf = B.bat_ms_reliability(10, arcs, sigma, cap, w, 0, 9, d, directed=directed)
                assert c == cf and _ok(R, Rf), (directed, d, R, Rf)
                if not directed and d < 3:
                    assert 0 < c < 3 ** 16
    finally:
        B.bat_set_option("BAT_MS_BITS", old)


@pytest.mark.parametrize("seed", range(4))
def test_bit_sliced_ranges(seed):
    """Index ranges with demand 1 to 3 run the bit-sliced kernel in the
    caller's arc order, the words at both ends masked: ranges inside one
    word, across a few words and long ones, against the oracle's range
    sweep; adjacent ranges add up to the whole sweep."""
    B = _B()
    arcs, sigma, cap, w = _random_states_net(800 + seed, 7, 10, [2, 3])
    N = int(np.prod(sigma))
    rng = np.random.default_rng(seed)
    lo = int(rng.integers(0, N // 2))
    cases = [(lo, lo + 1), (lo, lo + 7), (lo, lo + 500), (0, N), (N // 3, N)]
    old = B.bat_get_option("BAT_MS_RUN")
    try:
        for run in (0, 3):
            B.bat_set_option("BAT_MS_RUN", run)
            for directed in (False, True):
                for d in (1, 2, 3):
                    say("ms bits ranges", seed, run, directed, d)
                    for c_lo, c_hi in cases:
                        r = B.bat_ms_reliability_range(7, arcs, sigma, cap, w, 0, 6, d, c_lo, c_hi, directed=directed)
                        assert B.bat_last_launch().specialised == 1
                        o = oracle.ms_reliability_range(7, arcs, sigma, cap, w, 0, 6, d, c_lo, c_hi, directed=directed)
                        assert r.count == o.count and _ok(r.R, o.sum), (run, directed, d, c_lo, c_hi, r.R, o.sum)
                    cut = int(rng.integers(1, N))
                    a_ = B.bat_ms_reliability_range(7, arcs, sigma, cap, w, 0, 6, d, 0, cut, directed=directed)
                    b_ = B.bat_ms_reliability_range(7, arcs, sigma, cap, w, 0, 6, d, cut, N, directed=directed)
                    R, c = B.bat_ms_reliability(7, arcs, sigma, cap, w, 0, 6, d, directed=directed)
                    assert a_.count + b_.count == c and _ok(a_.R + b_.R, R)
    finally:
        B.bat_set_option("BAT_MS_RUN", old)


def test_bit_sliced_range_in_a_huge_space():
    """Short ranges inside and at the top of a 3^32-vector space (32
    three-level arcs, 1.85e15 vectors: large lane-run and word indices),
    demands 1 to 3, against the oracle's range sweep."""
    B = _B()
    n = 12
    rng = np.random.default_rng(32)
    arcs = [(i, i + 1) for i in range(n - 1)]
    while len(arcs) < 32:
        u, v = (int(x) for x in rng.choice(n, 2, replace=False))
        arcs.append((u, v))
    sigma = [3] * 32
    cap = [[0, 1, 2]] * 32
    w = [[float(x) for x in rng.dirichlet([1.0, 1.0, 1.0])] for _ in range(32)]
    N = 3 ** 32
    for d in (1, 2, 3):
        for c_lo in (int(N * 0.37) + 12345, int(N * 0.83) + 12345, N - 40004):
            c_hi = c_lo + 40003
            say("ms bits huge space", d, c_lo, c_hi)
            r = B.bat_ms_reliability_range(n, arcs, sigma, cap, w, 0, n - 1, d, c_lo, c_hi)
            assert B.bat_last_launch().specialised == 1
            o = oracle.ms_reliability_range(n, arcs, sigma, cap, w, 0, n - 1, d, c_lo, c_hi)
            assert r.count == o.count and _ok(r.R, o.sum), (d, c_lo, c_hi, r.R, o.sum)
