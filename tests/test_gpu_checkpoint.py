"""Checkpointed sweeps on the GPU: a sweep stopped after some chunks and
resumed from its file gives bitwise the same R, count and gradient as the
same chunking run in one call (with or without a file), and both agree
with the oracle (counts exact, R and T1 / T0 within 1e-12 relative).
Each chunk is one part of the whole sweep's work items; the parts must
cover every vector exactly once, which the exact counts check."""
import sys

import numpy as np
import pytest

import bat_workloads as W
import oracle

pytestmark = pytest.mark.gpu


def _B():
    import paper_2209_09711_amd as B
    return B


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b):
    if isinstance(a, tuple):
        return a == b
    return (a.R == b.R and a.count == b.count and np.array_equal(a.dRdp, b.dRdp)
            and np.array_equal(a.T1, b.T1) and np.array_equal(a.T0, b.T0))


@pytest.mark.parametrize("grad", [False, True])
@pytest.mark.parametrize("jit", [0, 1])
def test_resumed_sweep_is_bitwise_the_uninterrupted_one(tmp_path, grad, jit):
    B = _B()
    net = W.random_connected(12, 21, seed=2101, p_lo=0.4, p_hi=0.99)
    old = B.bat_get_option("BAT_JIT")
    try:
        B.bat_set_option("BAT_JIT", jit)
        say("checkpoint", net.name, "m", net.m, "grad", grad, "jit", jit)
        clog = 17                                              # 16 chunks
        whole = B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, clog, None, grad=grad)
        f = str(tmp_path / "run.ckpt")
        steps = []
        for budget in (3, 0, 5, 1):
            r = B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, clog, f, max_chunks=budget,
                                               grad=grad)
            assert r is None
            steps.append(open(f).read().splitlines()[4])
        assert steps == ["done 3", "done 3", "done 8", "done 9"]
        resumed = B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, clog, f, grad=grad)
        assert _same(resumed, whole)
        again = B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, clog, f, grad=grad)
        assert _same(again, whole)                             # the finished file
    finally:
        B.bat_set_option("BAT_JIT", old)
    o = oracle.reliability(net.n, net.arcs, net.p, net.s, net.t, grad=grad)
    R, cnt = (whole.R, whole.count) if grad else whole
    assert cnt == o.count and abs(R - o.sum) <= 1e-12 * o.sum
    if grad:
        assert np.allclose(whole.T1, o.T1, rtol=1e-12, atol=0) and np.allclose(whole.T0, o.T0, rtol=1e-12, atol=0)
        assert np.all(np.abs(whole.dRdp - o.grad) <= 1e-12 * (o.T1 + o.T0))


def test_flags_and_one_chunk(tmp_path):
    """A digraph in the forward index order, chunked and resumed; and a chunk
    size past 2^m, which is one whole sweep."""
    B = _B()
    rng = np.random.default_rng(77)
    n, m = 10, 18
    arcs = [tuple(int(x) for x in rng.choice(n, 2, replace=False)) for _ in range(m)]
    p = rng.uniform(0.5, 0.99, m)
    say("checkpoint digraph forward order")
    whole = B.bat_reliability_checkpointed(n, arcs, p, 0, n - 1, 13, None, grad=True, directed=True, forward=True)
    f = str(tmp_path / "d.ckpt")
    assert B.bat_reliability_checkpointed(n, arcs, p, 0, n - 1, 13, f, max_chunks=20, grad=True, directed=True,
                                          forward=True) is None
    resumed = B.bat_reliability_checkpointed(n, arcs, p, 0, n - 1, 13, f, grad=True, directed=True, forward=True)
    assert _same(resumed, whole)
    o = oracle.reliability(n, arcs, p, 0, n - 1, grad=True, directed=True)
    assert whole.count == o.count and abs(whole.R - o.sum) <= 1e-12 * o.sum
    assert np.all(np.abs(whole.dRdp - o.grad) <= 1e-12 * (o.T1 + o.T0))
    one = B.bat_reliability_checkpointed(n, arcs, p, 0, n - 1, 40, None, directed=True)
    rng_all = B.bat_reliability_range(n, arcs, p, 0, n - 1, 0, 1 << m, directed=True)
    assert one[1] == rng_all.count == o.count and abs(one[0] - rng_all.R) <= 1e-15 * rng_all.R


@pytest.mark.parametrize("perm", [0, 1, 2, 3])
def test_chunks_follow_the_whole_sweep_order(tmp_path, perm):
    """Chunks are divisions of the counter under the arc order a whole
    sweep would take (here forced by BAT_PERM); the file keeps it, and a
    resume keeps it even when the whole-sweep order has changed since."""
    B = _B()
    net = W.random_connected(11, 20, seed=2002 + perm, p_lo=0.3, p_hi=0.99)
    old = B.bat_get_option("BAT_PERM")
    try:
        B.bat_set_option("BAT_PERM", perm)
        say("checkpoint order", perm)
        whole = B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, 16, None, grad=True)
        f = str(tmp_path / "o.ckpt")
        assert B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, 16, f, max_chunks=5,
                                              grad=True) is None
        launch = open(f).read().splitlines()[3]
        assert launch.startswith(f"launch order={perm} ")
        B.bat_set_option("BAT_PERM", (perm + 1) % 4)
        resumed = B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, 16, f, grad=True)
        assert open(f).read().splitlines()[3] == launch
        assert _same(resumed, whole)
    finally:
        B.bat_set_option("BAT_PERM", old)
    o = oracle.reliability(net.n, net.arcs, net.p, net.s, net.t, grad=True)
    assert whole.count == o.count and abs(whole.R - o.sum) <= 1e-12 * o.sum
    assert np.allclose(whole.T1, o.T1, rtol=1e-12, atol=0) and np.allclose(whole.T0, o.T0, rtol=1e-12, atol=0)


def test_tuned_sweep_in_parts_matches_whole():
    """The 30-arc random graph (2^30 vectors), tuned: 16 parts against the
    whole sweep."""
    B = _B()
    net = W.config1()
    say("checkpoint config1")
    B.bat_autotune(net.n, net.arcs, net.p, net.s, net.t)
    R, cnt = B.bat_reliability(net.n, net.arcs, net.p, net.s, net.t)
    whole = B.bat_last_launch()
    got = B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, 26, None)
    part = B.bat_last_launch()
    # the same order and chains; work items no larger, so each part still
    # fills the GPU; together the parts tile the same counter
    assert (part.perm, part.chain_log2) == (whole.perm, whole.chain_log2)
    assert part.chunk_log2 <= whole.chunk_log2
    assert part.n_chunks * 16 == whole.n_chunks << (whole.chunk_log2 - part.chunk_log2)
    assert got[1] == cnt and abs(got[0] - R) <= 1e-12 * R


def test_edge_cases(tmp_path):
    """No arcs; more parts asked for than the sweep has work items (the
    bridge's 32 vectors are one iteration); s and t in different
    components; p at 0 and 1."""
    B = _B()
    say("checkpoint edge cases")
    R, cnt = B.bat_reliability_checkpointed(2, np.zeros((0, 2), np.int32), np.zeros(0), 0, 1, 0, None)
    assert R == 0.0 and cnt == 0
    b = W.bridge(0.9)
    f = str(tmp_path / "b.ckpt")
    R, cnt = B.bat_reliability_checkpointed(b.n, b.arcs, b.p, b.s, b.t, 0, f)
    assert open(f).read().splitlines()[2] == "parts 1"
    assert cnt == 16 and abs(R - (2 * .81 + 2 * .729 - 5 * .6561 + 2 * .59049)) <= 1e-15
    R, cnt = B.bat_reliability_checkpointed(4, [(0, 1), (2, 3)], [0.9, 0.9], 0, 3, 1, None)
    assert R == 0.0 and cnt == 0
    net = W.random_connected(10, 16, seed=44)
    p = np.array(net.p)
    p[::2] = 1.0
    p[1::4] = 0.0
    g = B.bat_reliability_checkpointed(net.n, net.arcs, p, net.s, net.t, 12, None, grad=True)
    o = oracle.reliability(net.n, net.arcs, p, net.s, net.t, grad=True)
    assert g.count == o.count and abs(g.R - o.sum) <= 1e-12 * max(o.sum, 1e-300)
    assert np.all(np.abs(g.dRdp - o.grad) <= 1e-12 * (o.T1 + o.T0) + 1e-300)
