"""Checkpoint files of bat_reliability_checkpointed, checked on the CPU.

The entry point cuts a sweep into parts and keeps its running sums in a
text file.  A file whose parts are all done returns its result without any
device work, and a call with max_chunks = 0 only reads the file.  So the
file format, the resume bookkeeping, the problem key and the error paths
can be checked here.  The files are written by these tests with the
oracle's own sums over a partition of the counter (the equal divisions of
Section 4, Eq. 6, added as double-doubles), so the stored values are the
oracle's, not the library's.  The resumed sweeps themselves, bitwise
against uninterrupted ones, are GPU tests (test_gpu_checkpoint.py).
"""
import os

import numpy as np
import pytest

import bat_workloads as W
import oracle
from oracle import pbat


def _B():
    import paper_2209_09711_amd as B
    return B


def _fnv(data: bytes) -> int:
    h = 1469598103934665603
    for b in data:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def _problem(net, flags, clog, grad):
    arcs = np.ascontiguousarray(np.asarray(net.arcs, dtype="<i4").reshape(-1, 2)).tobytes()
    p = np.ascontiguousarray(np.asarray(net.p, dtype="<f8")).tobytes()
    return (f"problem n={net.n} m={net.m} s={net.s} t={net.t} flags={flags} chunk_log2={clog} "
            f"grad={int(grad)} arcs={_fnv(arcs):016x} p={_fnv(p):016x}")


def _oracle_file(net, clog, grad, parts, done=None):
    """The checkpoint text after `done` of `parts` parts (default: all), with
    the oracle's sums over the Eq. 6 divisions standing for the parts'."""
    m = net.m
    chunks = parts
    done = chunks if done is None else done
    R = (0.0, 0.0)
    cnt = 0
    T1 = [(0.0, 0.0)] * m
    T0 = [(0.0, 0.0)] * m
    for j in range(done):
        lo, hi = pbat.division_bounds(m, chunks, j + 1)
        r = oracle.reliability_range(net.n, net.arcs, net.p, net.s, net.t, lo, hi, grad=grad)
        R = pbat.dd_add(*R, r.sum_hi, r.sum_lo)
        cnt += r.count
        if grad:
            T1 = [pbat.dd_add(*T1[i], float(r.T1[i])) for i in range(m)]
            T0 = [pbat.dd_add(*T0[i], float(r.T0[i])) for i in range(m)]
    lines = ["bat-checkpoint 1", _problem(net, 0, clog, grad), f"parts {parts}", "launch order=3 items=0 chain=3",
             f"done {done}",
             f"count {cnt}", f"R {R[0].hex()} {R[1].hex()}"]
    if grad:
        lines.append("T1 " + " ".join(f"{h.hex()} {l.hex()}" for h, l in T1))
        lines.append("T0 " + " ".join(f"{h.hex()} {l.hex()}" for h, l in T0))
    return "\n".join(lines) + "\n", R, cnt, T1, T0


@pytest.mark.parametrize("grad", [False, True])
def test_finished_file_returns_its_sums(tmp_path, grad):
    """A file with every division done gives back exactly its sums, and they
    match the whole-sweep oracle (and, for the bridge, the closed form)."""
    B = _B()
    for net, clog, parts in ((W.bridge(0.9), 2, 1), (W.random_connected(8, 15, seed=5, p_lo=0.3, p_hi=0.97), 12, 8)):
        text, R, cnt, T1, T0 = _oracle_file(net, clog, grad, parts)
        f = tmp_path / f"{net.name}.ckpt"
        f.write_text(text)
        out = B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, clog, str(f), grad=grad)
        whole = oracle.reliability(net.n, net.arcs, net.p, net.s, net.t, grad=grad)
        if grad:
            assert out.R == R[0] + R[1] and out.count == cnt
            assert list(out.T1) == [h + l for h, l in T1] and list(out.T0) == [h + l for h, l in T0]
            assert list(out.dRdp) == [(a[0] - b[0]) + (a[1] - b[1]) for a, b in zip(T1, T0)]
            assert np.allclose(out.dRdp, whole.grad, rtol=1e-13, atol=1e-15)
            Rv = out.R
        else:
            assert out == (R[0] + R[1], cnt)
            Rv = out[0]
        assert cnt == whole.count and abs(Rv - whole.sum) <= 1e-14 * whole.sum
        if net.name.startswith("bridge"):
            assert cnt == 16 and abs(Rv - (2 * .81 + 2 * .729 - 5 * .6561 + 2 * .59049)) <= 1e-15
        assert f.read_text() == text          # a finished file is not rewritten


def test_unfinished_file_with_no_chunk_budget_is_pending(tmp_path):
    B = _B()
    net = W.random_connected(8, 15, seed=3)
    text = _oracle_file(net, 12, True, 8, done=5)[0]
    f = tmp_path / "c.ckpt"
    f.write_text(text)
    assert B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, 12, str(f), max_chunks=0,
                                          grad=True) is None
    assert f.read_text() == text
    assert not os.path.exists(str(f) + ".tmp")


def test_file_for_another_problem_is_refused(tmp_path):
    B = _B()
    net = W.random_connected(8, 15, seed=3)
    text = _oracle_file(net, 12, False, 8)[0]
    f = tmp_path / "c.ckpt"
    f.write_text(text)
    p2 = np.array(net.p)
    p2[4] = np.nextafter(p2[4], 0.0)          # one bit of one probability
    others = [dict(p=p2), dict(chunk_log2=11), dict(grad=True), dict(directed=True), dict(t=net.t - 1)]
    for o in others:
        kw = dict(p=net.p, chunk_log2=12, grad=False, directed=False, t=net.t)
        kw.update(o)
        with pytest.raises(B.BatError) as e:
            B.bat_reliability_checkpointed(net.n, net.arcs, kw["p"], net.s, kw["t"], kw["chunk_log2"], str(f),
                                           max_chunks=0, grad=kw["grad"], directed=kw["directed"])
        assert e.value.code == B.BAT_EINVAL and "another problem" in str(e.value), o
    assert f.read_text() == text


@pytest.mark.parametrize("edit", ["magic", "parts", "too_many_parts", "order", "items", "chain", "done", "R",
                                  "truncate", "trailing"])
def test_damaged_files_are_io_errors(tmp_path, edit):
    B = _B()
    net = W.random_connected(8, 15, seed=3)                  # 2^4 iterations of 2048 vectors
    lines = _oracle_file(net, 12, False, 8)[0].splitlines()
    if edit == "magic":
        lines[0] = "bat-checkpoint 2"
    elif edit == "parts":
        lines[2] = "parts 6"                  # not a power of two
    elif edit == "too_many_parts":
        lines[2] = "parts 32"                 # more parts than work items
    elif edit == "order":
        lines[3] = "launch order=4 items=0 chain=3"   # the forward order, without BAT_FORWARD_ORDER
    elif edit == "items":
        lines[3] = "launch order=3 items=2 chain=3"   # 4 work items: fewer than 8 parts
    elif edit == "chain":
        lines[3] = "launch order=3 items=0 chain=2"
    elif edit == "done":
        lines[4] = "done 9"
    elif edit == "R":
        lines[6] = "R 0x1p-1"
    elif edit == "truncate":
        lines = lines[:5]
    else:
        lines[5] += " x"
    f = tmp_path / "c.ckpt"
    f.write_text("\n".join(lines) + "\n")
    with pytest.raises(B.BatError) as e:
        B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, 12, str(f), max_chunks=0)
    assert e.value.code == B.BAT_EIO


def test_argument_checks_without_device(tmp_path):
    B = _B()
    net = W.bridge()
    for clog in (-1, 63):
        with pytest.raises(B.BatError) as e:
            B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, clog, None, max_chunks=0)
        assert e.value.code == B.BAT_EINVAL
    with pytest.raises(B.BatError) as e:
        B.bat_reliability_checkpointed(net.n, net.arcs, [0.5, 0.5, 2.0, 0.5, 0.5], net.s, net.t, 2, None,
                                       max_chunks=0)
    assert e.value.code == B.BAT_EINVAL
    rc = B._lib.bat_reliability_checkpointed(net.n, net.m, B._ptr(B._arcs(net.arcs)), B._ptr(B._p(net.p, net.m)),
                                             net.s, net.t, 4, 2, None, 0, None, None, None, None, None)
    assert rc == B.BAT_EINVAL
    # no file and no chunk budget: nothing runs, nothing is written
    f = tmp_path / "new.ckpt"
    assert B.bat_reliability_checkpointed(net.n, net.arcs, net.p, net.s, net.t, 2, str(f), max_chunks=0) is None
    assert not f.exists()
