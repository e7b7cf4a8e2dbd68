"""Host side of the bit-sliced multi-state kernel (demands 1 to 3).

For demand d <= 3 the library decides the maximum s-t flow word by word:
flow >= 1 when t is reachable over the arcs of capacity >= 1, flow >= 2
when besides no single arc of capacity exactly 1 separates s from t there,
and flow >= 3 when no single arc of capacity 1 or 2 and no two arcs of
capacity 1 do (max-flow min-cut: the cuts of capacity 1 and 2 besides
arcs of capacity 0).  The constants the host bakes into the kernel (the word
slots' state patterns, the mixed-radix split of a vector's index into word
bits, uniform run steps and lane digits) are read back from the generated
source and the kernel's steps are replayed here on the CPU, on every
vector of small spaces: the counts must equal the oracle's, which decides
each vector by augmenting paths (Edmonds-Karp).  Needs no GPU.
"""
import re
import shutil
import subprocess

import numpy as np
import pytest

import oracle


def _B():
    import paper_2209_09711_amd as B
    return B


FULL32 = 0xFFFFFFFF


def _consts(src):
    g = src[src.index("struct JitMs"):]
    d = {k: int(v) for k, v in re.findall(r"static constexpr unsigned (\w+) = (\d+)u;", g)}
    d["DIR"] = "DIR = true" in g
    for k, v in re.findall(r"static constexpr unsigned (\w+)\[\d+\] = \{([^}]*)\};", g):
        d[k] = [int(x.rstrip("u")) for x in v.split(",")]
    return d


def _closure(G, W, src, need, skip):
    """Reach from s over masks W without slot `skip`: sweeps until t holds
    `need` (tested after each sweep) or a sweep pair changes nothing (the
    kernel's loop, one lane)."""
    r = [0] * G["N"]
    r[G["S"]] = src
    before = 0
    while True:
        for order in (range(G["M"]), range(G["M"] - 1, -1, -1)):
            for j in order:
                if j == skip:
                    continue
                u, v = G["NU"][j], G["NV"][j]
                r[v] |= r[u] & W[j]
                if not G["DIR"]:
                    r[u] |= r[v] & W[j]
            if r[G["T"]] & need == need:
                return r
        tot = sum(bin(x).count("1") for x in r)
        if tot == before:
            return r
        before = tot


def _replay(G, c_lo=None, c_hi=None):
    """Count of the vectors the kernel's steps accept, over the whole space
    or the index range [c_lo, c_hi) (word slots least significant: vector
    c is bit c mod B of word c div B, whose run step and lane run are the
    quotient's low and high digits)."""
    M, KW, KR, B, RUN = G["M"], G["KW"], G["KR"], G["B"], G["RUN"]
    n_out = 1
    for j in range(KW, M):
        n_out *= G["SIG"][j]
    if c_lo is None:
        c_lo, c_hi = 0, n_out * B
    rl_lo = (c_lo // B) // RUN
    rl_hi = (-(-c_hi // B) + RUN - 1) // RUN
    mask = lambda bits, x: FULL32 if (bits >> x) & 1 else 0  # noqa: E731
    count = 0
    for lane_run in range(rl_lo, rl_hi):
        W, U, U2 = [0] * M, [0] * M, [0] * M
        rl = lane_run
        for j in range(M):
            if j < KW:
                W[j], U[j], U2[j] = G["WW1"][j], G["WU1"][j], G["WU12"][j]
            elif j >= KW + KR:
                x = rl % G["SIG"][j]
                rl //= G["SIG"][j]
                W[j], U[j], U2[j] = mask(G["C1"][j], x), mask(G["CE1"][j], x), mask(G["CE12"][j], x)
        xr = [0] * M
        for step in range(RUN):
            for j in range(KW, KW + KR):
                W[j], U[j], U2[j] = mask(G["C1"][j], xr[j]), mask(G["CE1"][j], xr[j]), mask(G["CE12"][j], xr[j])
            c0 = (lane_run * RUN + step) * B
            full = sum(1 << b for b in range(B) if c_lo <= c0 + b < c_hi) & G["FULL"]
            r0 = _closure(G, W, full, full, -1)
            V = r0[G["T"]]
            if G["D"] == 2:
                for j in range(M):
                    need = V & U[j] & r0[G["NU"][j]]
                    if G["CE1"][j] and need:
                        V &= (~need | _closure(G, W, need, need, j)[G["T"]]) & FULL32
            if G["D"] == 3:
                # one arc of capacity 1 or 2, then two arcs of capacity 1
                for j in range(M):
                    need = V & U2[j] & r0[G["NU"][j]]
                    if G["CE12"][j] and need:
                        V &= (~need | _closure(G, W, need, need, j)[G["T"]]) & FULL32
                for j1 in range(M):
                    for j2 in range(j1 + 1, M):
                        if not (G["CE1"][j1] and G["CE1"][j2]):
                            continue
                        need = V & U[j1] & U[j2] & (r0[G["NU"][j1]] | r0[G["NU"][j2]])
                        if need:
                            Wp = [0 if j in (j1, j2) else W[j] for j in range(M)]
                            V &= (~need | _closure(G, Wp, need, need, -1)[G["T"]]) & FULL32
            count += bin(V).count("1")
            for j in range(KW, KW + KR):
                xr[j] += 1
                if xr[j] < G["SIG"][j]:
                    break
                xr[j] = 0
    return count


def _random_net(seed, lo_states=1, hi_states=4):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 7))
    m = int(rng.integers(5, 10))
    arcs = [(i, i + 1) for i in range(n - 1)]
    while len(arcs) < m:
        u, v = (int(x) for x in rng.choice(n, 2, replace=False))
        arcs.append((u, v))
    sigma = [int(rng.integers(lo_states, hi_states + 1)) for _ in range(m)]
    cap = [[int(rng.integers(0, 3)) for _ in range(k)] for k in sigma]
    return n, arcs, sigma, cap


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("run", [0, 3, 9])
def test_bit_sliced_steps_count_like_the_oracle(seed, run):
    """Random graphs, 1-4 states with capacities 0-2 in any order, both arc
    readings, demands 1 to 3, runs of the default length and of at most 3
    and 9 steps (option BAT_MS_RUN, which moves slots from the lanes to the
    uniform run)."""
    B = _B()
    n, arcs, sigma, cap = _random_net(seed, 1 if seed % 2 else 2)
    w = [[1.0 / k] * k for k in sigma]
    old = B.bat_get_option("BAT_MS_RUN")
    try:
        B.bat_set_option("BAT_MS_RUN", run)
        for directed in (False, True):
            for d in (1, 2, 3):
                G = _consts(B.bat_ms_jit_source(n, arcs, sigma, cap, 0, n - 1, d, directed=directed))
                assert G["D"] == d and G["DIR"] == directed
                if run:
                    rl = 1
                    for j in range(G["KW"], G["KW"] + G["KR"]):
                        rl *= G["SIG"][j]
                    assert rl == G["RUN"] <= run
                o = oracle.ms_reliability(n, arcs, sigma, cap, w, 0, n - 1, d, directed=directed)
                assert _replay(G) == o.count, (seed, run, directed, d)
    finally:
        B.bat_set_option("BAT_MS_RUN", old)


@pytest.mark.parametrize("seed", range(6))
def test_bit_sliced_ranges_count_like_the_oracle(seed):
    """Index ranges (the caller's arc order, arc 0 most significant): the
    kernel's steps over [c_lo, c_hi), the words at both ends masked, count
    like the oracle's range sweep, for ranges inside one word, across a few
    words, and from 0 to the end; runs of at most 1, 3 and 9 steps."""
    B = _B()
    n, arcs, sigma, cap = _random_net(40 + seed, 2, 3)
    w = [[1.0 / k] * k for k in sigma]
    N = int(np.prod(sigma))
    rng = np.random.default_rng(seed)
    lo = int(rng.integers(0, N // 2))
    cases = [(lo, lo + 1), (lo, min(N, lo + 5)), (lo, min(N, lo + 200)), (0, N), (int(rng.integers(1, N)), N)]
    old = B.bat_get_option("BAT_MS_RUN")
    try:
        for run in (1, 3, 9):
            B.bat_set_option("BAT_MS_RUN", run)
            for directed in (False, True):
                for d in (1, 2, 3):
                    for c_lo, c_hi in cases:
                        G = _consts(B.bat_ms_jit_source(n, arcs, sigma, cap, 0, n - 1, d, directed=directed,
                                                        c_lo=c_lo, c_hi=c_hi))
                        o = oracle.ms_reliability_range(n, arcs, sigma, cap, w, 0, n - 1, d, c_lo, c_hi,
                                                        directed=directed)
                        assert _replay(G, c_lo, c_hi) == o.count, (seed, run, directed, d, c_lo, c_hi)
    finally:
        B.bat_set_option("BAT_MS_RUN", old)


def test_word_patterns_and_split():
    """The word holds the longest prefix of slots whose state counts
    multiply to at most 32; its patterns say, per vector bit, whether the
    slot's state has capacity >= 1 and exactly 1; the other slots' state
    sets are bit masks over their states."""
    B = _B()
    arcs = [(0, 1), (1, 2), (0, 2), (2, 3), (1, 3)]
    sigma = [2, 4, 3, 5, 2]
    cap = [[0, 1], [2, 0, 1, 1], [2, 2, 0], [0, 0, 1, 2, 3], [3, 1]]
    G = _consts(B.bat_ms_jit_source(4, arcs, sigma, cap, 0, 3, 2))
    # whole sweeps reorder the arcs by breadth-first distance from s: read
    # each slot's states back through its state count and capacity masks
    by_nodes = {tuple(sorted(a)): i for i, a in enumerate(arcs)}
    B_ = 1
    kw = 0
    while kw < G["M"] and B_ * G["SIG"][kw] <= 32:
        B_ *= G["SIG"][kw]
        kw += 1
    assert kw == G["KW"] and G["FULL"] == (1 << B_) - 1
    stride = 1
    for j in range(G["M"]):
        i = by_nodes[tuple(sorted((G["NU"][j], G["NV"][j])))]
        assert G["SIG"][j] == sigma[i]
        assert G["C1"][j] == sum(1 << x for x, c in enumerate(cap[i]) if c >= 1)
        assert G["CE1"][j] == sum(1 << x for x, c in enumerate(cap[i]) if c == 1)
        assert G["CE12"][j] == sum(1 << x for x, c in enumerate(cap[i]) if c in (1, 2))
        assert (G["UPAIR"] >> j) & 1 == (1 in cap[i])
        if j < G["KW"]:
            for b in range(B_):
                x = (b // stride) % sigma[i]
                assert (G["WW1"][j] >> b) & 1 == (cap[i][x] >= 1)
                assert (G["WU1"][j] >> b) & 1 == (cap[i][x] == 1)
                assert (G["WU12"][j] >> b) & 1 == (cap[i][x] in (1, 2))
            stride *= sigma[i]
        else:
            assert G["WW1"][j] == G["WU1"][j] == G["WU12"][j] == 0


def test_only_demands_up_to_three():
    B = _B()
    arcs = [(0, 1), (1, 2)]
    with pytest.raises(B.BatError):
        B.bat_ms_jit_source(3, arcs, [3, 3], None, 0, 2, 4)
    with pytest.raises(B.BatError):
        B.bat_ms_jit_source(3, [], [], None, 0, 2, 1)
    src = B.bat_ms_jit_source(3, arcs, [3, 3], None, 0, 2, 1)
    assert "bat_ms_bits" in src and "MsCut" in src
    assert "D = 3u" in B.bat_ms_jit_source(3, arcs, [3, 3], None, 0, 2, 3)


@pytest.mark.skipif(shutil.which("hipcc") is None and not __import__("os").path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not installed")
@pytest.mark.parametrize("d", [1, 2])
def test_sources_compile_without_scratch(tmp_path, d):
    """The benchmark's 3^18 workload's kernel compiles for gfx950 with no
    scratch memory (registers only)."""
    import bat_workloads as W
    B = _B()
    net = W.config_ms()
    src = B.bat_ms_jit_source(net.n, net.arcs, net.sigma, net.cap, net.s, net.t, d)
    f = tmp_path / "m.hip"
    f.write_text("#include <hip/hip_runtime.h>\n" + src)
    out = tmp_path / "m.s"
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", "-o", str(out), str(f)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    asm = out.read_text()
    assert re.findall(r"\.private_segment_fixed_size:\s+(\d+)", asm) == ["0"]
    assert "scratch_" not in asm
