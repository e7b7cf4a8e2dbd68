"""The allocation-free entry point against the stream-ordered one.

bat_reliability_noalloc runs the forward sweep in the library's fixed
device scratch.  Two calls in a row, the second on a smaller problem, must
each agree with bat_reliability_async on the same inputs (count exact, R
within 1e-12 relative) and with the oracle where it is cheap; a problem too
large for the scratch must be refused before anything runs.
"""
import sys

import numpy as np
import pytest

import bat_workloads as W
import oracle

pytestmark = pytest.mark.gpu

REL = 1e-12


def _run(fn, net, p_dev):
    import torch
    R = torch.full((), -1.0, dtype=torch.float64, device="cuda")
    cnt = torch.zeros((), dtype=torch.int64, device="cuda")
    st = torch.full((), 7, dtype=torch.int32, device="cuda")
    fn(net.n, net.arcs, p_dev.data_ptr(), net.s, net.t, R.data_ptr(), cnt.data_ptr(), st.data_ptr(),
       torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return float(R.item()), int(cnt.item()), int(st.item())


def test_noalloc_matches_async_twice():
    import torch
    import paper_2209_09711_amd as B
    big = W.random_connected(16, 34, seed=71, p_lo=0.6, p_hi=0.99)
    small = W.random_connected(9, 16, seed=72, p_lo=0.2, p_hi=0.95)
    for net in (big, small):
        print(f"noalloc vs async: {net.name} m={net.m}", flush=True)
        p = torch.tensor(net.p, dtype=torch.float64, device="cuda")
        Rn, cn, sn = _run(B.bat_reliability_noalloc, net, p)
        Ra, ca, sa = _run(B.bat_reliability_async, net, p)
        assert sn == 0 and sa == 0
        assert cn == ca
        assert abs(Rn - Ra) <= REL * Ra
    o = oracle.net_reliability(small)
    assert cn == o.count and abs(Rn - o.sum) <= REL * o.sum
    sys.stdout.flush()


def test_noalloc_invalid_probability_and_too_big():
    import torch
    import paper_2209_09711_amd as B
    net = W.random_connected(6, 8, seed=3)
    p = torch.tensor(net.p, dtype=torch.float64, device="cuda")
    p[2] = 1.5
    R, c, st = _run(B.bat_reliability_noalloc, net, p)
    assert st == B.BAT_EINVAL and np.isnan(R)
    # 2^60 vectors: the partial sums would not fit the fixed scratch
    huge = W.random_connected(20, 60, seed=5)
    ph = torch.tensor(huge.p, dtype=torch.float64, device="cuda")
    Rh = torch.full((), -1.0, dtype=torch.float64, device="cuda")
    ch = torch.zeros((), dtype=torch.int64, device="cuda")
    with pytest.raises(B.BatError) as e:
        B.bat_reliability_noalloc(huge.n, huge.arcs, ph.data_ptr(), huge.s, huge.t, Rh.data_ptr(), ch.data_ptr(),
                                  None, torch.cuda.current_stream().cuda_stream)
    assert e.value.code == B.BAT_ETOOBIG and "scratch" in B.bat_last_error()
    torch.cuda.synchronize()
    assert float(Rh.item()) == -1.0 and int(ch.item()) == 0
    # the next call still works
    small = W.random_connected(8, 14, seed=9)
    ps = torch.tensor(small.p, dtype=torch.float64, device="cuda")
    R2, c2, s2 = _run(B.bat_reliability_noalloc, small, ps)
    o = oracle.net_reliability(small)
    assert s2 == 0 and c2 == o.count and abs(R2 - o.sum) <= REL * o.sum
