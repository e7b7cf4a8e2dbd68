"""GPU parity: the HIP library against the CPU oracle (and the frontier DP).

Bars (the tolerance for a sum of up to 2^40 FP64 terms):
feasible counts bit-exact; R within 1e-12 relative; T1_i and T0_i within
1e-12 relative; dR/dp_i within 1e-12 (T1_i + T0_i) absolute.  Both kernel
instantiations are covered: the generic one (graph read at run time) and the
graph-specialised one (compiled with hiprtc).
"""
import contextlib
import os
import sys

import numpy as np
import pytest

import bat_workloads as W
import oracle
from oracle import frontier_dp, pbat

pytestmark = pytest.mark.gpu

REL = 1e-12


def _B():
    import paper_2209_09711_amd as B
    return B


@contextlib.contextmanager
def options(**kw):
    B = _B()
    old = {k: B.bat_get_option(k) for k in kw}
    try:
        for k, v in kw.items():
            B.bat_set_option(k, v)
        yield
    finally:
        for k, v in old.items():
            B.bat_set_option(k, v)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_ok(got, want, rel=REL):
    if want == 0.0:
        return got == 0.0
    return abs(got - want) <= rel * abs(want)


KERNELS = [pytest.param(0, id="generic"), pytest.param(1, id="specialised")]


# ---------------------------------------------------------------- paper pins

@pytest.mark.parametrize("jit", KERNELS)
@pytest.mark.parametrize("pv", [0.9, 0.5, 0.123, 1.0, 0.0])
def test_bridge(jit, pv):
    B = _B()
    b = W.bridge(pv)
    with options(BAT_JIT=jit):
        R, cnt = B.bat_reliability(b.n, b.arcs, b.p, b.s, b.t)
    assert cnt == 16
    want = 2 * pv**2 + 2 * pv**3 - 5 * pv**4 + 2 * pv**5
    assert abs(R - want) <= 1e-15


@pytest.mark.parametrize("jit", KERNELS)
def test_figure1_and_table4_divisions(jit):
    B = _B()
    f = W.figure1()
    with options(BAT_JIT=jit):
        R, cnt = B.bat_reliability(f.n, f.arcs, f.p, f.s, f.t)
        assert cnt == 25 and abs(R - 0.960175722) <= 0.5e-9
        assert rel_ok(R, 4800878611 / 5000000000, 1e-15)
        want = pbat.run(f.n, f.arcs, f.p, f.s, f.t, 4, processes=1)
        for i in range(1, 5):      # Eq. 6 divisions, chi = 4
            lo, hi = pbat.division_bounds(6, 4, i)
            r = B.bat_reliability_range(f.n, f.arcs, f.p, f.s, f.t, lo, hi)
            assert r.count == want.division_count[i - 1]
            assert rel_ok(r.R, want.division_R[i - 1])


# ----------------------------------------------------------- random parity

def _cases(k, seed, m_max=20, n_max=20):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        kind = i % 4
        if kind == 3:
            n = int(rng.integers(2, 8))
            m = int(rng.integers(0, 14))
            net = W.random_multigraph(n, m, seed=int(rng.integers(1 << 30)), p_lo=0.0, p_hi=1.0)
            if m:
                net.p[rng.random(m) < 0.15] = 1.0
                net.p[rng.random(m) < 0.15] = 0.0
        else:
            n = int(rng.integers(3, n_max + 1))
            mmin, mmax = n - 1, min(m_max, n * (n - 1) // 2)
            m = int(rng.integers(mmin, mmax + 1))
            net = W.random_connected(n, m, seed=int(rng.integers(1 << 30)), p_lo=0.05, p_hi=0.99)
        out.append(net)
    return out


@pytest.mark.parametrize("jit", KERNELS)
def test_random_vs_oracle(jit):
    B = _B()
    nets = _cases(24 if jit == 0 else 10, 1234 + jit)
    with options(BAT_JIT=jit):
        for net in nets:
            say("case", net.name, net.n, net.m, net.s, net.t)
            R, cnt = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
            o = oracle.net_reliability(net)
            assert cnt == o.count, net.name
            assert rel_ok(R, o.sum), (net.name, R, o.sum)


@pytest.mark.parametrize("jit", KERNELS)
@pytest.mark.parametrize("n", [16, 17, 33, 34])
def test_node_count_classes(jit, n):
    """A cycle of n nodes (every node relevant), s and t opposite: R is
    1 - (1 - prod path1)(1 - prod path2) and the count is
    2^n - (2^a - 1)(2^b - 1) for path lengths a, b."""
    B = _B()
    rng = np.random.default_rng(n)
    arcs = [(i, (i + 1) % n) for i in range(n)]
    p = rng.uniform(0.9, 0.999, n)
    s, t = 0, n // 2
    with options(BAT_JIT=jit):
        say("cycle", n)
        R, cnt = B.bat_reliability(n, arcs, p, s, t)
    a, b = t, n - t
    want = 1.0 - (1.0 - np.prod(p[:a])) * (1.0 - np.prod(p[a:]))
    assert cnt == (1 << n) - ((1 << a) - 1) * ((1 << b) - 1)
    assert rel_ok(R, want, 1e-13)


@pytest.mark.parametrize("jit", KERNELS)
def test_edge_cases(jit):
    B = _B()
    with options(BAT_JIT=jit):
        # m = 0: one empty vector, disconnected
        R, cnt = B.bat_reliability(2, np.zeros((0, 2), np.int32), np.zeros(0), 0, 1)
        assert R == 0.0 and cnt == 0
        # s and t in different components
        R, cnt = B.bat_reliability(4, [(0, 1), (2, 3)], [0.9, 0.9], 0, 3)
        assert R == 0.0 and cnt == 0
        # only self-loops and a parallel pair
        arcs = [(0, 0), (0, 1), (0, 1), (1, 1)]
        p = [0.3, 0.6, 0.7, 0.9]
        R, cnt = B.bat_reliability(2, arcs, p, 0, 1)
        assert cnt == 12 and abs(R - (1 - 0.4 * 0.3)) <= 1e-15
        # m = 11 and 12: exactly one word/wave, and one iteration bit
        for m in (5, 10, 11, 12):
            net = W.random_connected(6, m, seed=m, p_lo=0.1, p_hi=0.9)
            R, cnt = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
            o = oracle.net_reliability(net)
            assert cnt == o.count and rel_ok(R, o.sum)


@pytest.mark.parametrize("jit", [0, 1])
def test_max_sizes_ranges(jit):
    """The largest inputs the ABI takes: 62 arcs (a counter reaching 2^62)
    on a 62-node cycle with s and t opposite (62 relevant nodes: the widest
    reach-word class) and on a denser 40-node graph padded to 64 nodes (33
    relevant); ranges at the start, the middle and the very top of the
    counter, with gradients, against the oracle."""
    B = _B()
    cycle = W.Network("cycle62", 62, [(i, (i + 1) % 62) for i in range(62)], 0, 31, np.linspace(0.6, 0.99, 62))
    dense = W.random_connected(40, 62, seed=4062, p_lo=0.3, p_hi=0.95)
    dense.n = 64                       # 24 isolated nodes
    top = 1 << 62
    rng = np.random.default_rng(62)
    spans = [(0, 70000), (top // 2 - 33333, top // 2 + 44444), (top - 100000, top),
             (top - (1 << 31) - 35000, top - (1 << 31) + 35000)]  # mixed verdicts on the cycle
    for _ in range(2):                                             # mixed verdicts on the dense graph
        lo = int(rng.integers(0, top - (1 << 17)))
        spans.append((lo, lo + 70000))
    for net in (cycle, dense):
        say("max sizes", net.name, net.n, net.m, "jit", jit)
        with options(BAT_JIT=jit):
            for lo, hi in spans:
                r = B.bat_reliability_range(net.n, net.arcs, net.p, net.s, net.t, lo, hi, grad=True)
                o = oracle.reliability_range(net.n, net.arcs, net.p, net.s, net.t, lo, hi, grad=True)
                assert r.count == o.count and rel_ok(r.R, o.sum), (net.name, lo, hi)
                assert np.allclose(r.T1, o.T1, rtol=1e-12, atol=1e-300)
                assert np.allclose(r.T0, o.T0, rtol=1e-12, atol=1e-300)


# ------------------------------------------------------ full-size workloads

def test_config1_full_vs_frontier_dp():
    B = _B()
    c = W.config1()
    say("config1", c.n, c.m)
    R, cnt = B.bat_reliability(c.n, c.arcs, c.p, c.s, c.t)
    Rd, cd = frontier_dp.reliability(c.n, c.arcs, c.p, c.s, c.t)
    assert cnt == cd and rel_ok(R, Rd)
    # sampled divisions against the BAT oracle, spread over the counter
    chi = 1 << 10
    for i in pbat.spread_divisions(chi, 3):
        lo, hi = pbat.division_bounds(c.m, chi, i)
        r = B.bat_reliability_range(c.n, c.arcs, c.p, c.s, c.t, lo, hi)
        o = oracle.reliability_range(c.n, c.arcs, c.p, c.s, c.t, lo, hi)
        assert r.count == o.count and rel_ok(r.R, o.sum)


def test_config2_grid_full_vs_frontier_dp():
    """The headline workload (2^40 vectors) in the launch shape bench.py times."""
    B = _B()
    c = W.config2()
    say("config2", c.n, c.m)
    R, cnt = B.bat_reliability(c.n, c.arcs, c.p, c.s, c.t)
    info = B.bat_last_launch()
    say("config2 kernel ms", info.kernel_ms, "specialised", info.specialised)
    Rd, cd = frontier_dp.reliability(c.n, c.arcs, c.p, c.s, c.t)
    assert cnt == cd and rel_ok(R, Rd)
    # ragged sampled ranges against the oracle
    rng = np.random.default_rng(2)
    for _ in range(3):
        lo = int(rng.integers(0, (1 << 40) - (1 << 21)))
        hi = lo + int(rng.integers(1 << 19, 1 << 20))
        r = B.bat_reliability_range(c.n, c.arcs, c.p, c.s, c.t, lo, hi)
        o = oracle.reliability_range(c.n, c.arcs, c.p, c.s, c.t, lo, hi)
        assert r.count == o.count and rel_ok(r.R, o.sum)


def test_config4_grad_full_vs_frontier_dp():
    B = _B()
    c = W.config4()
    say("config4", c.n, c.m)
    g = B.bat_reliability_grad(c.n, c.arcs, c.p, c.s, c.t)
    Rd, cd = frontier_dp.reliability(c.n, c.arcs, c.p, c.s, c.t)
    assert g.count == cd and rel_ok(g.R, Rd)
    T1, T0 = frontier_dp.gradient(c.n, c.arcs, c.p, c.s, c.t)
    for i in range(c.m):
        assert rel_ok(g.T1[i], T1[i]), (i, g.T1[i], T1[i])
        assert rel_ok(g.T0[i], T0[i]), (i, g.T0[i], T0[i])
        assert abs(g.dRdp[i] - (T1[i] - T0[i])) <= REL * (T1[i] + T0[i])
    # the forward-only sweep agrees with the forward+gradient sweep
    R, cnt = B.bat_reliability(c.n, c.arcs, c.p, c.s, c.t)
    assert cnt == g.count and rel_ok(R, g.R)
    # central finite differences (exact up to rounding: R is multilinear)
    h = 1e-6
    for i in (0, 7, 35):
        q = c.p.copy(); q[i] += h
        Rp, _ = B.bat_reliability(c.n, c.arcs, q, c.s, c.t)
        q[i] -= 2 * h
        Rm, _ = B.bat_reliability(c.n, c.arcs, q, c.s, c.t)
        assert abs((Rp - Rm) / (2 * h) - g.dRdp[i]) <= 1e-9


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("jit", KERNELS)
def test_half_probability_bit_exact(jit):
    B = _B()
    with options(BAT_JIT=jit):
        for seed in range(3):
            net = W.random_connected(14, 24 + seed, seed=seed)
            R, cnt = B.bat_reliability(net.n, net.arcs, np.full(net.m, 0.5), net.s, net.t)
            assert R == cnt * 2.0 ** -net.m
            o = oracle.net_reliability(net, p=np.full(net.m, 0.5))
            assert cnt == o.count


def test_p_one_zero_and_complement():
    B = _B()
    net = W.random_connected(12, 20, seed=9)
    R1, c1 = B.bat_reliability(net.n, net.arcs, np.ones(net.m), net.s, net.t)
    R0, c0 = B.bat_reliability(net.n, net.arcs, np.zeros(net.m), net.s, net.t)
    assert R1 == 1.0 and R0 == 0.0 and c1 == c0


def test_determinism_and_launch_variants():
    B = _B()
    net = W.random_connected(16, 26, seed=77, p_lo=0.6, p_hi=0.99)
    base = [B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t) for _ in range(10)]
    assert all(b == base[0] for b in base)          # bitwise
    R0, c0 = base[0]
    for jit in (0, 1):
        for check in (1, 2):
            for clog in (1, 4, 9):
                with options(BAT_JIT=jit, BAT_CHECK_EVERY=check, BAT_CHUNK_LOG2=clog):
                    R, cnt = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
                assert cnt == c0 and rel_ok(R, R0), (jit, check, clog)
    for seg in (0, 3, 8):
        with options(BAT_SEG_LOG2=seg):
            g = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
        assert g.count == c0 and rel_ok(g.R, R0)


def test_arc_permutation_invariance():
    B = _B()
    net = W.random_connected(15, 24, seed=5, p_lo=0.3, p_hi=0.97)
    R0, c0 = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
    rng = np.random.default_rng(0)
    for _ in range(3):
        perm = rng.permutation(net.m)
        arcs = [net.arcs[i] for i in perm]
        R, cnt = B.bat_reliability(net.n, arcs, net.p[perm], net.s, net.t)
        assert cnt == c0 and rel_ok(R, R0)


# ------------------------------------------------------------------ gradient

@pytest.mark.parametrize("jit", KERNELS)
def test_grad_vs_oracle(jit):
    B = _B()
    nets = _cases(12 if jit == 0 else 6, 99 + jit, m_max=18, n_max=14)
    nets.append(W.bridge(0.9).with_p([1.0, 0.0, 0.7, 1.0, 0.0]))
    with options(BAT_JIT=jit):
        for net in nets:
            say("grad case", net.name, net.n, net.m)
            g = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
            o = oracle.net_reliability(net, grad=True)
            assert g.count == o.count and rel_ok(g.R, o.sum)
            for i in range(net.m):
                assert rel_ok(g.T1[i], o.T1[i]), (net.name, i, g.T1[i], o.T1[i])
                assert rel_ok(g.T0[i], o.T0[i]), (net.name, i, g.T0[i], o.T0[i])
                assert abs(g.dRdp[i] - (o.T1[i] - o.T0[i])) <= REL * (o.T1[i] + o.T0[i]) + 1e-300


def test_grad_birnbaum_bruteforce():
    B = _B()
    net = W.random_connected(13, 22, seed=4, p_lo=0.5, p_hi=0.95)
    g = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
    for i in range(net.m):
        q = net.p.copy(); q[i] = 1.0
        R1, _ = B.bat_reliability(net.n, net.arcs, q, net.s, net.t)
        q[i] = 0.0
        R0, _ = B.bat_reliability(net.n, net.arcs, q, net.s, net.t)
        assert abs(g.dRdp[i] - (R1 - R0)) <= 1e-13
        assert g.dRdp[i] >= -1e-15


# --------------------------------------------------------------- range API

@pytest.mark.parametrize("jit", KERNELS)
def test_ranges_compose(jit):
    B = _B()
    net = W.random_connected(14, 27, seed=31, p_lo=0.4, p_hi=0.99)
    with options(BAT_JIT=jit):
        _ranges_compose(B, net)


def _ranges_compose(B, net):
    full = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
    cuts = [0, 1, 2047, 2048, 70001, 1 << 20, (1 << 27) - 5, 1 << 27]
    hi = lo = 0.0
    cnt = 0
    T1 = np.zeros(net.m)
    T0 = np.zeros(net.m)
    for a, b in zip(cuts[:-1], cuts[1:]):
        r = B.bat_reliability_range(net.n, net.arcs, net.p, net.s, net.t, a, b, grad=True)
        o = oracle.reliability_range(net.n, net.arcs, net.p, net.s, net.t, a, b) if b - a < (1 << 21) else None
        if o is not None:
            assert r.count == o.count and rel_ok(r.R, o.sum)
        hi, lo = pbat.dd_add(hi, lo, r.R_hi, r.R_lo)
        cnt += r.count
        T1 += r.T1
        T0 += r.T0
    assert cnt == full.count and rel_ok(hi + lo, full.R)
    assert np.allclose(T1, full.T1, rtol=1e-12, atol=0) and np.allclose(T0, full.T0, rtol=1e-12, atol=0)


@pytest.mark.parametrize("seed", range(3))
def test_ragged_ranges_specialised_vs_oracle(seed):
    """Ranges that start and end inside an 8-iteration chain block (the
    specialised kernel sweeps whole blocks and masks what lies outside)."""
    B = _B()
    rng = np.random.default_rng(seed)
    net = W.random_connected(13, 24 + seed, seed=70 + seed, p_lo=0.3, p_hi=0.99)
    total = 1 << net.m
    with options(BAT_JIT=1):
        for _ in range(4):
            lo = int(rng.integers(0, total - (1 << 18)))
            hi = lo + int(rng.integers(1, 1 << 18))
            say("ragged", net.name, lo, hi)
            r = B.bat_reliability_range(net.n, net.arcs, net.p, net.s, net.t, lo, hi, grad=True)
            o = oracle.reliability_range(net.n, net.arcs, net.p, net.s, net.t, lo, hi, grad=True)
            assert r.count == o.count and rel_ok(r.R, o.sum)
            assert np.allclose(r.T1, o.T1, rtol=1e-12, atol=1e-300)
            assert np.allclose(r.T0, o.T0, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("perm", [0, 1, 2, 3])
def test_arc_to_bit_orders(perm):
    """Every arc -> counter-bit order gives the same count, R and gradient
    (a whole sweep is a sum over all vectors; only the work split changes)."""
    B = _B()
    nets = [W.random_connected(15, 30, seed=90, p_lo=0.4, p_hi=0.99), W.config4(),
            W.random_connected(10, 20, seed=91, p_lo=0.1, p_hi=0.9)]
    nets[2].arcs = nets[2].arcs + [(0, 0), (3, 3)]               # pruned self-loops
    nets[2].p = np.concatenate([nets[2].p, [0.3, 0.8]])
    for net in nets:
        say("perm", perm, net.name)
        with options(BAT_PERM=0, BAT_JIT=1):
            ref = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
        with options(BAT_PERM=perm, BAT_JIT=1):
            g = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
            R, cnt = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
        assert g.count == ref.count == cnt and rel_ok(g.R, ref.R) and rel_ok(R, ref.R)
        assert np.allclose(g.T1, ref.T1, rtol=1e-12, atol=0) and np.allclose(g.T0, ref.T0, rtol=1e-12, atol=0)


@pytest.mark.parametrize("k", [0, 3, 4, 5, 6])
def test_chain_lengths(k):
    """Warm-start chain lengths: whole sweeps agree with the frontier DP, and
    ranges that cut blocks of 2^k iterations agree with the oracle."""
    B = _B()
    rng = np.random.default_rng(k)
    net = W.config4()
    with options(BAT_CHAIN_LOG2=k, BAT_JIT=1):
        say("chain", k, net.name)
        R, cnt = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
        Rd, cd = frontier_dp.reliability(net.n, net.arcs, net.p, net.s, net.t)
        assert cnt == cd and rel_ok(R, Rd)
        small = W.random_connected(13, 26, seed=77 + k, p_lo=0.3, p_hi=0.99)
        for _ in range(3):
            lo = int(rng.integers(0, (1 << small.m) - (1 << 19)))
            hi = lo + int(rng.integers(1, 1 << 19))
            r = B.bat_reliability_range(small.n, small.arcs, small.p, small.s, small.t, lo, hi)
            o = oracle.reliability_range(small.n, small.arcs, small.p, small.s, small.t, lo, hi)
            assert r.count == o.count and rel_ok(r.R, o.sum)


@pytest.mark.parametrize("perm", [0, 3])
@pytest.mark.parametrize("k", [3, 6])
def test_window_test(perm, k):
    """Skipping the chained blocks whose top iteration cannot connect s and t
    even with all 11 word arcs up changes nothing: whole sweeps of a grid
    (where about half the blocks are skipped), with and without the
    gradient, match the unskipped sweeps and the frontier DP; ranges that
    start and end inside windows and blocks agree with the oracle."""
    B = _B()
    net = W.grid(4, 5, p=np.random.default_rng(5).uniform(0.6, 0.99, 31))
    say("window test", perm, k, net.name)
    res, grads = {}, {}
    for wt in (0, 1):
        with options(BAT_WINDOW_TEST=wt, BAT_PERM=perm, BAT_CHAIN_LOG2=k, BAT_JIT=1, BAT_AUTOTUNE=0):
            res[wt] = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
            li = B.bat_last_launch()
            assert li.specialised == 1 and li.window_test == wt
            grads[wt] = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
            assert B.bat_last_launch().window_test == wt
    assert res[0] == res[1]
    g0, g1 = grads[0], grads[1]
    assert g0.count == g1.count == res[1][1] and rel_ok(g1.R, g0.R, 1e-15)
    assert np.allclose(g1.T1, g0.T1, rtol=1e-14, atol=0) and np.allclose(g1.T0, g0.T0, rtol=1e-14, atol=0)
    Rd, cd = frontier_dp.reliability(net.n, net.arcs, net.p, net.s, net.t)
    assert res[1][1] == cd and rel_ok(res[1][0], Rd)
    rng = np.random.default_rng(100 + k + perm)
    with options(BAT_WINDOW_TEST=1, BAT_CHAIN_LOG2=k, BAT_JIT=1, BAT_CHUNK_LOG2=4):
        for _ in range(3):
            lo = int(rng.integers(0, (1 << net.m) - (1 << 20)))
            hi = lo + int(rng.integers(1 << 16, 1 << 20))
            r = B.bat_reliability_range(net.n, net.arcs, net.p, net.s, net.t, lo, hi)
            o = oracle.reliability_range(net.n, net.arcs, net.p, net.s, net.t, lo, hi)
            assert r.count == o.count and rel_ok(r.R, o.sum), (lo, hi)


@pytest.mark.parametrize("waves,super_restart,simd,keep", [
    (1, 0, 6, 1), (1, 1, 6, 1), (2, 0, 6, 1), (2, 1, 6, 1), (4, 0, 6, 1), (4, 1, 6, 1),
    (4, 0, 0, 1), (4, 0, 5, 1), (4, 0, 8, 1), (4, 0, 6, 0), (4, 1, 0, 0), (4, 0, 6, 2), (4, 1, 5, 2),
    (2, 0, 6, 2)])
def test_forward_launch_shapes(waves, super_restart, simd, keep):
    """Blocks of 1, 2 or 4 wavefronts, with or without the super-block store
    and the kept block bottoms (in registers or LDS), compiled for 4 (the
    compiler's budget) to 8
    wavefronts per SIMD, sweep the same vectors: the launch reports the
    shape it ran, whole sweeps agree bit for bit with the default shape and
    with the frontier DP, and ragged ranges agree with the oracle."""
    B = _B()
    nets = [W.grid(4, 5, p=np.random.default_rng(6).uniform(0.6, 0.99, 31)), W.config4()]
    for net in nets:
        say("shape", waves, super_restart, simd, keep, net.name)
        with options(BAT_JIT=1, BAT_AUTOTUNE=0, BAT_PERM=3, BAT_CHAIN_LOG2=3):
            ref = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
            with options(BAT_BLOCK_WAVES=waves, BAT_SUPER_RESTART=super_restart, BAT_SIMD_WAVES=simd,
                         BAT_KEEP_BOTTOM=keep):
                got = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
                li = B.bat_last_launch()
        assert li.specialised == 1 and li.block_waves == waves and li.simd_waves == simd
        assert li.keep_bottom == keep and li.super_restart == (1 if super_restart and keep else 0)
        assert got == ref
        if net.m <= 31:
            Rd, cd = frontier_dp.reliability(net.n, net.arcs, net.p, net.s, net.t)
            assert got[1] == cd and rel_ok(got[0], Rd)
    net = nets[0]
    rng = np.random.default_rng(40 + waves + super_restart + simd + keep)
    with options(BAT_JIT=1, BAT_BLOCK_WAVES=waves, BAT_SUPER_RESTART=super_restart, BAT_SIMD_WAVES=simd,
                 BAT_KEEP_BOTTOM=keep, BAT_CHUNK_LOG2=7):
        for _ in range(2):
            lo = int(rng.integers(0, (1 << net.m) - (1 << 20)))
            hi = lo + int(rng.integers(1 << 17, 1 << 20))
            r = B.bat_reliability_range(net.n, net.arcs, net.p, net.s, net.t, lo, hi)
            o = oracle.reliability_range(net.n, net.arcs, net.p, net.s, net.t, lo, hi)
            assert r.count == o.count and rel_ok(r.R, o.sum), (lo, hi)


def test_series_joining():
    """Joining two arcs in series through a degree-2 node into one relaxation
    (the AND of their masks) changes nothing: R, counts and gradients match
    the plain relaxation list and the oracle, on graphs with many such
    nodes (paths of parallel series, a ladder, random sparse graphs)."""
    B = _B()
    rng = np.random.default_rng(515)
    nets = [W.parallel_paths(4, np.full(8, 0.9)), W.series(12, np.linspace(0.5, 0.99, 12)), W.grid(2, 12),
            W.grid(4, 5, p=rng.uniform(0.6, 0.99, 31))]
    for seed in range(4):
        nets.append(W.random_connected(16, 20, seed=700 + seed, p_lo=0.3, p_hi=0.99))
    for net in nets:
        say("series", net.name, net.n, net.m)
        out = {}
        for sj in (0, 1):
            with options(BAT_JIT=1, BAT_SERIES=sj, BAT_AUTOTUNE=0):
                R, cnt = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
                li = B.bat_last_launch()
                g = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
            out[sj] = (R, cnt, g, li.relaxations)
        assert out[0][1] == out[1][1] == out[1][2].count
        assert rel_ok(out[1][0], out[0][0], 1e-14) and rel_ok(out[1][2].R, out[0][2].R, 1e-14)
        assert np.allclose(out[1][2].T1, out[0][2].T1, rtol=1e-13, atol=0)
        assert np.allclose(out[1][2].T0, out[0][2].T0, rtol=1e-13, atol=0)
        assert out[1][3] <= out[0][3]
        if net.m <= 24:
            o = oracle.net_reliability(net)
            assert out[1][1] == o.count and rel_ok(out[1][0], o.sum)


def test_sparse_graphs_specialised_vs_oracle():
    """Sparse random graphs (a spanning tree plus a few extra arcs: many
    degree-2 nodes, dead ends, long series paths) through the specialised
    kernels, whose plans join series arcs and relax one way at s and t:
    R, counts and gradients against the oracle."""
    B = _B()
    rng = np.random.default_rng(424242)
    for i in range(12):
        n = int(rng.integers(8, 21))
        m = min(22, n - 1 + int(rng.integers(1, 5)))
        net = W.random_connected(n, m, seed=int(rng.integers(1 << 30)), p_lo=0.2, p_hi=0.99)
        say("sparse", i, net.n, net.m)
        with options(BAT_JIT=1):
            R, cnt = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
            assert B.bat_last_launch().specialised == 1
            g = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
        o = oracle.net_reliability(net, grad=True)
        assert cnt == o.count == g.count and rel_ok(R, o.sum) and rel_ok(g.R, o.sum)
        for j in range(net.m):
            assert rel_ok(g.T1[j], o.T1[j]) and rel_ok(g.T0[j], o.T0[j]), (net.name, j)


@pytest.mark.parametrize("order", [0, 1])
def test_item_orders(order):
    """Counter-order and spread work-item orders sweep the same vectors: equal
    counts, R and gradient; ranges (chunk counts that are not powers of two)
    keep agreeing with the oracle."""
    B = _B()
    nets = [W.config4(), W.random_connected(15, 30, seed=92, p_lo=0.4, p_hi=0.99)]
    for net in nets:
        say("item order", order, net.name)
        with options(BAT_ITEM_ORDER=0, BAT_JIT=1, BAT_CHUNK_LOG2=3):
            ref = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
        with options(BAT_ITEM_ORDER=order, BAT_JIT=1, BAT_CHUNK_LOG2=3):
            g = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
            R, cnt = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
            li = B.bat_last_launch()
            assert li.n_chunks > 1
        assert g.count == ref.count == cnt and rel_ok(g.R, ref.R) and rel_ok(R, ref.R)
        assert np.allclose(g.T1, ref.T1, rtol=1e-12, atol=0) and np.allclose(g.T0, ref.T0, rtol=1e-12, atol=0)
    small = W.random_connected(13, 26, seed=93, p_lo=0.3, p_hi=0.99)
    with options(BAT_ITEM_ORDER=order, BAT_CHUNK_LOG2=2):
        for lo, hi in [(12345, 12345 + 3 * (1 << 13) + 77), (0, 1 << 22), (1 << 24, (1 << 24) + (5 << 13))]:
            r = B.bat_reliability_range(small.n, small.arcs, small.p, small.s, small.t, lo, hi)
            o = oracle.reliability_range(small.n, small.arcs, small.p, small.s, small.t, lo, hi)
            assert r.count == o.count and rel_ok(r.R, o.sum)


def test_autotune_choice_keeps_results():
    """After tuning, the tuned forward and gradient launches still match
    the frontier DP (an independent exact method), not just the untuned
    launch."""
    B = _B()
    net = W.random_connected(16, 34, seed=8, p_lo=0.6, p_hi=0.99)
    Rd, cd = frontier_dp.reliability(net.n, net.arcs, net.p, net.s, net.t)
    R0, c0 = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
    assert c0 == cd and rel_ok(R0, Rd)
    ns = B.bat_autotune(net.n, net.arcs, net.p, net.s, net.t)
    say("autotune ns/vector", ns)
    assert 0.0 < ns < 1.0
    R1, c1 = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
    assert c1 == cd and rel_ok(R1, Rd)
    g = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
    assert g.count == cd and rel_ok(g.R, Rd)
    # the tuned gradient launch against per-arc DP runs: T1_i = R|p_i<-1,
    # T0_i = R|p_i<-0, on a spread of arcs
    for i in range(0, net.m, 5):
        q = net.p.copy()
        q[i] = 1.0
        t1 = frontier_dp.reliability(net.n, net.arcs, q, net.s, net.t)[0]
        q[i] = 0.0
        t0 = frontier_dp.reliability(net.n, net.arcs, q, net.s, net.t)[0]
        assert rel_ok(g.T1[i], t1) and rel_ok(g.T0[i], t0), (i, g.T1[i], t1, g.T0[i], t0)


def test_jit_disk_cache(tmp_path, monkeypatch):
    """Specialised kernels persist on disk: a compile writes one entry, a
    flushed process loads it back with bit-identical results, an entry
    whose header does not match is recompiled and rewritten, and
    BAT_JIT_CACHE=0 writes nothing."""
    B = _B()
    monkeypatch.setenv("BAT_JIT_CACHE_DIR", str(tmp_path))
    monkeypatch.delenv("BAT_JIT_CACHE", raising=False)
    net = W.random_connected(11, 20, seed=515, p_lo=0.3, p_hi=0.95)
    with options(BAT_JIT=1):
        B.bat_set_option("BAT_JIT_FLUSH", 1)
        R1, c1 = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
        assert B.bat_last_launch().specialised
        files = sorted(tmp_path.glob("*.co"))
        assert len(files) == 1 and files[0].stat().st_size > 1000
        B.bat_set_option("BAT_JIT_FLUSH", 1)
        R2, c2 = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
        assert (R2, c2) == (R1, c1) and sorted(tmp_path.glob("*.co")) == files
        files[0].write_bytes(b"BATJIT1\n" + bytes(40))       # a header that matches nothing
        B.bat_set_option("BAT_JIT_FLUSH", 1)
        R3, c3 = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
        assert (R3, c3) == (R1, c1) and files[0].stat().st_size > 1000
        monkeypatch.setenv("BAT_JIT_CACHE", "0")
        other = W.random_connected(11, 21, seed=516, p_lo=0.3, p_hi=0.95)
        B.bat_reliability(other.n, other.arcs, other.p, other.s, other.t)
        assert sorted(tmp_path.glob("*.co")) == files
    assert B.bat_get_option("BAT_JIT_FLUSH") == 0


def test_autotune_compiles_side_by_side(tmp_path, monkeypatch):
    """bat_autotune compiles its candidates' specialised kernels in helper
    processes up front: tuning into an empty disk cache leaves an entry for
    every arc order of the forward sweep and two of the gradient's, the
    kernel a launch then runs is the one an in-process compile gives (the
    same identity), and results match the frontier DP."""
    import time
    B = _B()
    monkeypatch.setenv("BAT_JIT_CACHE_DIR", str(tmp_path))
    monkeypatch.delenv("BAT_JIT_CACHE", raising=False)
    net = W.random_connected(14, 28, seed=612, p_lo=0.5, p_hi=0.99)
    Rd, cd = frontier_dp.reliability(net.n, net.arcs, net.p, net.s, net.t)
    B.bat_set_option("BAT_JIT_FLUSH", 1)
    with options(BAT_JIT_PROCS=16):
        t0 = time.perf_counter()
        B.bat_autotune(net.n, net.arcs, net.p, net.s, net.t)
        say("autotune with helper processes: %.2f s" % (time.perf_counter() - t0))
    assert len(list(tmp_path.glob("*.co"))) >= 6
    with options(BAT_AUTOTUNE=0, BAT_JIT=1):
        R1, c1 = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
        id1 = B.bat_last_launch().kernel_id
    assert c1 == cd and rel_ok(R1, Rd)
    monkeypatch.setenv("BAT_JIT_CACHE", "0")
    B.bat_set_option("BAT_JIT_FLUSH", 1)
    with options(BAT_JIT_PROCS=0, BAT_AUTOTUNE=0, BAT_JIT=1):
        R2, c2 = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
        assert B.bat_last_launch().kernel_id == id1
    assert (R2, c2) == (R1, c1)


# ------------------------------------------------------- directed, forward

def _digraph(seed, n, m):
    """A random digraph with a good chance of s -> t paths: a random
    connected graph, each arc oriented at random, plus reversed copies of
    a third of them."""
    rng = np.random.default_rng(seed)
    net = W.random_connected(n, m, seed=seed, p_lo=0.3, p_hi=0.95)
    arcs = [(u, v) if rng.random() < 0.5 else (v, u) for (u, v) in net.arcs]
    extra = [(v, u) for (u, v) in arcs if rng.random() < 1 / 3]
    arcs = arcs + extra
    p = rng.uniform(0.3, 0.95, size=len(arcs))
    return net.n, arcs, p, net.s, net.t


def test_directed_bridge():
    """The directed bridge (arcs as listed, u -> v) at p = 0.9: the oracle's
    pin, R = 0.97119, 15 connected vectors."""
    B = _B()
    arcs = [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)]
    R, c = B.bat_reliability_ex(4, arcs, np.full(5, 0.9), 0, 3, directed=True)
    o = oracle.reliability(4, arcs, np.full(5, 0.9), 0, 3, directed=True)
    assert c == o.count == 15 and rel_ok(R, o.sum) and abs(R - 0.97119) < 5e-6


@pytest.mark.parametrize("jit", [0, 1])
def test_directed_vs_oracle(jit):
    """Directed sweeps (generic and specialised kernels) against the
    directed oracle: whole sweeps with the gradient, and ranges."""
    B = _B()
    for seed, n, m in [(31, 8, 12), (32, 9, 14), (36, 10, 13)]:
        nn, arcs, p, s, t = _digraph(seed, n, m)
        say("directed", seed, len(arcs), "jit", jit)
        with options(BAT_JIT=jit):
            g = B.bat_reliability_ex(nn, arcs, p, s, t, directed=True, grad=True)
            o = oracle.reliability(nn, arcs, p, s, t, grad=True, directed=True)
            assert g.count == o.count and rel_ok(g.R, o.sum)
            assert np.allclose(g.T1, o.T1, rtol=1e-12, atol=1e-300)
            assert np.allclose(g.T0, o.T0, rtol=1e-12, atol=1e-300)
            u = B.bat_reliability_ex(nn, arcs, p, s, t, directed=False)
            ou = oracle.reliability(nn, arcs, p, s, t)
            assert u[1] == ou.count and rel_ok(u[0], ou.sum)
            M = 1 << len(arcs)
            for lo, hi in [(0, M // 3), (M // 3 + 5, M - 7)]:
                r = B.bat_reliability_range(nn, arcs, p, s, t, lo, hi, grad=True, directed=True)
                orr = oracle.reliability_range(nn, arcs, p, s, t, lo, hi, grad=True, directed=True)
                assert r.count == orr.count and rel_ok(r.R, orr.sum)


@pytest.mark.parametrize("k", [0, 3, 5])
def test_directed_chains_large(k):
    """A larger digraph: warm-started chains (one-directional consistency
    test) against ranges of the directed oracle and the exact count split."""
    B = _B()
    nn, arcs, p, s, t = _digraph(80, 14, 22)
    M = 1 << len(arcs)
    with options(BAT_CHAIN_LOG2=k, BAT_JIT=1):
        say("directed chains", k, len(arcs))
        R, c = B.bat_reliability_ex(nn, arcs, p, s, t, directed=True)
        parts = [B.bat_reliability_range(nn, arcs, p, s, t, a, b, directed=True)
                 for a, b in [(0, M // 2), (M // 2, M)]]
        assert sum(x.count for x in parts) == c
        assert rel_ok(sum(x.R for x in parts), R)
        rng = np.random.default_rng(k)
        for _ in range(3):
            lo = int(rng.integers(0, M - (1 << 18)))
            hi = lo + int(rng.integers(1, 1 << 18))
            r = B.bat_reliability_range(nn, arcs, p, s, t, lo, hi, directed=True)
            o = oracle.reliability_range(nn, arcs, p, s, t, lo, hi, directed=True)
            assert r.count == o.count and rel_ok(r.R, o.sum)
    with options(BAT_JIT=0, BAT_CHAIN_LOG2=k):
        R0, c0 = B.bat_reliability_ex(nn, arcs, p, s, t, directed=True)
    assert c0 == c and rel_ok(R0, R)


@pytest.mark.parametrize("directed", [False, True])
def test_forward_order_ranges(directed):
    """Ranges in the forward BAT order (Eq. 4-5) against the oracle's
    forward order, including ranges that split the word, lane and chained
    bits; the two orders' whole sweeps agree."""
    B = _B()
    net = W.random_connected(13, 26, seed=91 + directed, p_lo=0.3, p_hi=0.99)
    arcs, p = net.arcs, net.p
    M = 1 << len(arcs)
    for lo, hi in [(0, 1000), (12345, 12345 + 3 * (1 << 13) + 77), (M // 2 - 999, M // 2 + (1 << 20)), (M - 4097, M)]:
        r = B.bat_reliability_range(net.n, arcs, p, net.s, net.t, lo, hi, grad=True, directed=directed, forward=True)
        o = oracle.reliability_range(net.n, arcs, p, net.s, net.t, lo, hi, grad=True, directed=directed, forward=True)
        assert r.count == o.count and rel_ok(r.R, o.sum), (lo, hi)
        assert np.allclose(r.T1, o.T1, rtol=1e-12, atol=1e-300) and np.allclose(r.T0, o.T0, rtol=1e-12, atol=1e-300)
    f = B.bat_reliability_range(net.n, arcs, p, net.s, net.t, 0, M, directed=directed, forward=True)
    b = B.bat_reliability_range(net.n, arcs, p, net.s, net.t, 0, M, directed=directed)
    assert f.count == b.count and rel_ok(f.R, b.R)


# ------------------------------------------------------------------- torch

def test_torch_autograd_and_async():
    import torch
    from paper_2209_09711_amd.torch_fn import reliability
    B = _B()
    net = W.random_connected(10, 16, seed=12, p_lo=0.3, p_hi=0.95)
    p = torch.tensor(net.p, dtype=torch.float64, device="cuda", requires_grad=True)
    R, cnt = reliability(p, net.n, net.arcs, net.s, net.t)
    R.backward()
    g = B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
    assert R.item() == g.R and int(cnt.item()) == g.count
    assert np.array_equal(p.grad.cpu().numpy(), g.dRdp)
    q = torch.tensor(net.p[:8] * 0 + 0.6, dtype=torch.float64, device="cuda", requires_grad=True)
    small = W.random_connected(6, 8, seed=3)
    fn = lambda x: reliability(x, small.n, small.arcs, small.s, small.t)[0]
    assert torch.autograd.gradcheck(fn, (q,), eps=1e-6, atol=1e-9, rtol=1e-7)


def test_async_invalid_probability():
    import torch
    B = _B()
    net = W.random_connected(6, 8, seed=3)
    p = torch.tensor(net.p, dtype=torch.float64, device="cuda")
    p[2] = 1.5
    R = torch.zeros((), dtype=torch.float64, device="cuda")
    cnt = torch.zeros((), dtype=torch.int64, device="cuda")
    st = torch.zeros((), dtype=torch.int32, device="cuda")
    B.bat_reliability_async(net.n, net.arcs, p.data_ptr(), net.s, net.t, R.data_ptr(), cnt.data_ptr(),
                            st.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert int(st.item()) == B.BAT_EINVAL and np.isnan(R.item())


# ------------------------------------------------------------------ batched

def _batch_inputs(seed, n_graphs, n_pvec):
    rng = np.random.default_rng(seed)
    graphs, pblocks = [], []
    for g in range(n_graphs):
        if g % 5 == 4:
            net = W.random_multigraph(int(rng.integers(2, 7)), int(rng.integers(0, 12)), seed=int(rng.integers(1 << 30)))
        else:
            n = int(rng.integers(3, 15))
            m = int(rng.integers(n - 1, min(24, n * (n - 1) // 2) + 1))
            net = W.random_connected(n, m, seed=int(rng.integers(1 << 30)))
            s, t = (int(x) for x in rng.choice(n, 2, replace=False))
            net.s, net.t = s, t
        graphs.append((net.n, net.arcs, net.s, net.t))
        pb = rng.uniform(0.0, 1.0, size=(n_pvec, len(net.arcs)))
        if pb.size:
            pb[rng.random(pb.shape) < 0.05] = 1.0
        pblocks.append(pb)
    return graphs, pblocks


@pytest.mark.parametrize("n_pvec", [1, 7, 32, 45])
def test_batched_vs_plain_and_oracle(n_pvec):
    B = _B()
    graphs, pblocks = _batch_inputs(500 + n_pvec, 14, n_pvec)
    say("batched", len(graphs), n_pvec)
    R, cnt = B.bat_reliability_batched(graphs, pblocks)
    for g, (n, arcs, s, t) in enumerate(graphs):
        for j in sorted({0, n_pvec // 2, n_pvec - 1}):
            Rp, cp = B.bat_reliability(n, arcs, pblocks[g][j], s, t)
            assert cnt[g] == cp and rel_ok(R[g, j], Rp), (g, j, R[g, j], Rp)
        # every probability vector index against the oracle (or the frontier
        # DP), spread over the graphs
        j = g % n_pvec
        if len(arcs) <= 16:
            o = oracle.reliability(n, arcs, pblocks[g][j], s, t)
            assert cnt[g] == o.count and rel_ok(R[g, j], o.sum), (g, j)
        else:
            Rd, cd = frontier_dp.reliability(n, arcs, pblocks[g][j], s, t)
            assert cnt[g] == cd and rel_ok(R[g, j], Rd), (g, j)


@pytest.mark.parametrize("n_pvec,jit_arcs,window,streams",
                         [(1, 14, 1, 4), (7, 18, 1, 3), (32, 14, 1, 4), (45, 20, 1, 2), (9, 14, 0, 0),
                          (20, 16, 1, 1)])
def test_batched_specialised_kernels(n_pvec, jit_arcs, window, streams):
    """Graphs with at least jit_arcs arcs run graph-specialised batched
    kernels (on up to `streams` side streams, 0: the calling thread's
    stream), the rest the generic launch,
    in the same call: counts equal to the generic launch's, R within
    rounding of it, and every p-vector index against the frontier DP (more
    than 32 p-vectors split into entries)."""
    B = _B()
    graphs, pblocks = _batch_inputs(900 + n_pvec, 10, n_pvec)
    rng = np.random.default_rng(950 + n_pvec)
    for n, m in [(12, 20), (14, 24), (16, 26), (10, 16), (13, 22)]:
        net = W.random_connected(n, m, seed=int(rng.integers(1 << 30)))
        s, t = (int(x) for x in rng.choice(n, 2, replace=False))
        graphs.append((net.n, net.arcs, s, t))
        pblocks.append(rng.uniform(0.3, 1.0, size=(n_pvec, m)))
    with options(BAT_BATCH_JIT_ARCS=0):
        R0, c0 = B.bat_reliability_batched(graphs, pblocks)
        assert B.bat_last_launch().specialised == 0
    with options(BAT_BATCH_JIT_ARCS=jit_arcs, BAT_WINDOW_TEST=window, BAT_BATCH_STREAMS=streams):
        say("batched specialised from", jit_arcs, "arcs,", n_pvec, "p-vectors")
        R, c = B.bat_reliability_batched(graphs, pblocks)
        assert B.bat_last_launch().specialised == 1
        R2, c2 = B.bat_reliability_batched(graphs, pblocks)
    assert np.array_equal(R, R2) and np.array_equal(c, c2)       # deterministic
    assert np.array_equal(c, c0)
    assert np.allclose(R, R0, rtol=1e-12, atol=0)
    for g, (n, arcs, s_, t_) in enumerate(graphs):
        for j in sorted({g % n_pvec, n_pvec - 1}):
            Rd, cd = frontier_dp.reliability(n, arcs, pblocks[g][j], s_, t_)
            assert c[g] == cd and rel_ok(R[g, j], Rd), (g, j, R[g, j], Rd)


@pytest.mark.parametrize("k", [0, 3, 4, 5, 6])
def test_batched_chain_lengths(k):
    """Warm-started chains in the batched launch: counts exact, R equal to the
    unchained launch to rounding, on graphs large enough to chain."""
    B = _B()
    graphs, pblocks = _batch_inputs(700 + k, 20, 5)
    with options(BAT_CHAIN_LOG2=0):
        R0, c0 = B.bat_reliability_batched(graphs, pblocks)
    with options(BAT_CHAIN_LOG2=k):
        say("batched chain", k, len(graphs))
        R, c = B.bat_reliability_batched(graphs, pblocks)
    assert np.array_equal(c, c0)
    assert np.allclose(R, R0, rtol=1e-12, atol=0)
    g = max(range(len(graphs)), key=lambda i: len(graphs[i][1]))
    n, arcs, s_, t_ = graphs[g]
    Rd, cd = frontier_dp.reliability(n, arcs, pblocks[g][0], s_, t_)
    assert c[g] == cd and rel_ok(R[g, 0], Rd)


def test_batched_autotune_keeps_results():
    """The tuned batched launch against the frontier DP on every graph, each
    with another probability vector."""
    B = _B()
    graphs, pblocks = _batch_inputs(777, 12, 9)
    R0, c0 = B.bat_reliability_batched(graphs, pblocks)
    ms = B.bat_autotune_batched(graphs, pblocks)
    say("batched autotune ms", ms)
    assert 0.0 < ms < 1e4
    R1, c1 = B.bat_reliability_batched(graphs, pblocks)
    assert np.array_equal(c1, c0) and np.allclose(R1, R0, rtol=1e-12, atol=0)
    for g, (n, arcs, s_, t_) in enumerate(graphs):
        j = g % 9
        Rd, cd = frontier_dp.reliability(n, arcs, pblocks[g][j], s_, t_)
        assert c1[g] == cd and rel_ok(R1[g, j], Rd), (g, j, R1[g, j], Rd)


def test_batched_config3_workload():
    """256 graphs x 32 probability vectors in one persistent launch."""
    B = _B()
    nets, pvs = W.config3()
    graphs = [(n.n, n.arcs, n.s, n.t) for n in nets]
    say("config3 batched", len(graphs))
    # the launch the benchmark times: tuned on this batch
    B.bat_autotune_batched(graphs, pvs)
    R, cnt = B.bat_reliability_batched(graphs, pvs)
    R2, cnt2 = B.bat_reliability_batched(graphs, pvs)
    assert np.array_equal(R, R2) and np.array_equal(cnt, cnt2)       # deterministic
    for g, net in enumerate(nets):
        # p-vector 0 and p-vector g mod 32 of every graph: every index 0..31
        # is checked against the frontier DP (an independent exact method)
        for j in sorted({0, g % 32}):
            Rd, cd = frontier_dp.reliability(net.n, net.arcs, pvs[g][j], net.s, net.t)
            assert cnt[g] == cd and rel_ok(R[g, j], Rd), (g, j, R[g, j], Rd)
    big = max(range(len(nets)), key=lambda i: (nets[i].m, nets[i].n))
    for j in range(32):
        net = nets[big]
        Rd, cd = frontier_dp.reliability(net.n, net.arcs, pvs[big][j], net.s, net.t)
        assert cnt[big] == cd and rel_ok(R[big, j], Rd), (big, j, R[big, j], Rd)
    for g in range(0, len(nets), 17):
        net = nets[g]
        for j in (5, 31):
            Rp, cp = B.bat_reliability(net.n, net.arcs, pvs[g][j], net.s, net.t)
            assert cp == cnt[g] and rel_ok(R[g, j], Rp)


def test_threads_share_device_and_reuse_resources():
    """Synchronous calls from several host threads at once (each thread has
    its own stream and workspace), with sizes that grow the workspace, then a
    second set of threads that takes over what the first left behind."""
    import threading

    B = _B()
    nets = _cases(12, 4242, m_max=22)
    want = [oracle.net_reliability(net) for net in nets]
    errors = []

    def worker(k):
        try:
            for j in sorted(range(len(nets)), key=lambda j: (nets[j].m + 7 * k) % 23):
                net = nets[j]
                R, cnt = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
                if cnt != want[j].count or not rel_ok(R, want[j].sum):
                    errors.append((k, net.name, R, want[j].sum, cnt, want[j].count))
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append((k, repr(e)))

    for wave in range(2):
        say("thread wave", wave)
        ts = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        assert not errors, errors[:4]


def test_batched_specialised_large_node_counts():
    """Specialised batched kernels for graphs of more than 32 relevant nodes
    (no kept block bottoms there): two cycles of 34 and 40 nodes, whose
    reliability has a closed form, beside a small generic graph."""
    B = _B()
    rng = np.random.default_rng(1500)
    graphs, pblocks, want = [], [], []
    for n in (34, 40):
        arcs = [(i, (i + 1) % n) for i in range(n)]
        t = n // 2
        pv = rng.uniform(0.9, 0.999, size=(3, n))
        graphs.append((n, arcs, 0, t))
        pblocks.append(pv)
        want.append([1.0 - (1.0 - np.prod(p[:t])) * (1.0 - np.prod(p[t:])) for p in pv])
    small = W.random_connected(6, 9, seed=5)
    graphs.append((small.n, small.arcs, small.s, small.t))
    pblocks.append(rng.uniform(0.3, 0.9, size=(3, small.m)))
    with options(BAT_BATCH_JIT_ARCS=30):
        R, c = B.bat_reliability_batched(graphs, pblocks)
        assert B.bat_last_launch().specialised == 1
    for g, n in enumerate((34, 40)):
        t = n // 2
        assert c[g] == (1 << n) - ((1 << t) - 1) * ((1 << (n - t)) - 1)
        for j in range(3):
            assert rel_ok(R[g, j], want[g][j], 1e-13), (n, j, R[g, j], want[g][j])
    for j in range(3):
        o = oracle.reliability(small.n, small.arcs, pblocks[2][j], small.s, small.t)
        assert c[2] == o.count and rel_ok(R[2, j], o.sum)


def test_batched_specialised_terminals_apart():
    """A specialised batched kernel for a graph whose t no arc reaches (no
    relaxation survives the plan): R = 0 and count 0 for every p-vector,
    beside a connected graph checked against the frontier DP."""
    B = _B()
    apart = [(i, j) for i in range(7) for j in range(i + 1, 7)][:16]
    net = W.random_connected(10, 18, seed=77)
    rng = np.random.default_rng(1600)
    graphs = [(9, apart, 0, 8), (net.n, net.arcs, net.s, net.t)]
    pblocks = [rng.uniform(0.1, 1.0, size=(5, 16)), rng.uniform(0.1, 1.0, size=(5, net.m))]
    with options(BAT_BATCH_JIT_ARCS=14):
        R, c = B.bat_reliability_batched(graphs, pblocks)
        assert B.bat_last_launch().specialised == 1
    assert c[0] == 0 and np.all(R[0] == 0.0)
    for j in range(5):
        Rd, cd = frontier_dp.reliability(net.n, net.arcs, pblocks[1][j], net.s, net.t)
        assert c[1] == cd and rel_ok(R[1, j], Rd)


def test_threads_batched_specialised():
    """Batched calls with graph-specialised kernels from several host
    threads at once (each thread has its own stream and side streams; the
    kernels are compiled once and shared), in two waves of threads: every
    result equals the single-threaded one to the bit."""
    import threading

    B = _B()
    batches = []
    for k in range(3):
        graphs, pblocks = _batch_inputs(1300 + k, 8, 6)
        rng = np.random.default_rng(1400 + k)
        for n, m in [(12, 20), (13, 22)]:
            net = W.random_connected(n, m, seed=int(rng.integers(1 << 30)))
            graphs.append((net.n, net.arcs, 0, n - 1))
            pblocks.append(rng.uniform(0.3, 1.0, size=(6, m)))
        batches.append((graphs, pblocks))
    errors = []
    with options(BAT_BATCH_JIT_ARCS=18):
        want = [B.bat_reliability_batched(g, p) for g, p in batches]
        assert B.bat_last_launch().specialised == 1

        def worker(k):
            try:
                for j in range(6):
                    i = (j + k) % len(batches)
                    R, c = B.bat_reliability_batched(*batches[i])
                    if not (np.array_equal(R, want[i][0]) and np.array_equal(c, want[i][1])):
                        errors.append((k, i))
            except Exception as e:  # noqa: BLE001 - reported below
                errors.append((k, repr(e)))

        for wave in range(2):
            say("batched thread wave", wave)
            ts = [threading.Thread(target=worker, args=(k,)) for k in range(3)]
            for t in ts:
                t.start()
            for t in ts:
                t.join()
            assert not errors, errors[:4]


def test_launch_info_names_the_kernel():
    """The launch description names the kernel that ran: the same launch
    twice reports the same identity, the generic and specialised kernels and
    the forward and gradient sweeps report different ones."""
    B = _B()
    net = W.random_connected(9, 16, seed=77)
    ids = {}
    for jit in (0, 1):
        with options(BAT_JIT=jit):
            for grad in (False, True):
                for _ in range(2):
                    if grad:
                        B.bat_reliability_grad(net.n, net.arcs, net.p, net.s, net.t)
                    else:
                        B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
                    li = B.bat_last_launch()
                    assert li.kernel_id != 0
                    assert li.specialised == jit
                    assert li.perm in (0, 1, 2, 3)
                    assert li.check_every in (1, 2) and li.item_order in (0, 1)
                    assert ids.setdefault((jit, grad), li.kernel_id) == li.kernel_id
    assert len(set(ids.values())) == 4


def test_valu_peak_diagnostic():
    """The measured integer VALU rate is positive and below the chip's
    32-bit vector issue limit, 128 lane-operations per CU per clock
    (256 x 128 x 2.4e9 = 7.86e13 /s, the rate behind the vector FP32
    figure), by at most rounding of the clock: the diagnostic's 16 VALU
    instructions per trip were counted with SQ_INSTS_VALU, and it retires
    about 1.9 wave64 instructions per CU per cycle."""
    B = _B()
    say("valu peak")
    r = B.bat_valu_peak()
    limit = 256 * 128 * 2.4e9
    say("lane-ops/s", r, r / limit)
    assert 0.5 * limit < r < 1.05 * limit
