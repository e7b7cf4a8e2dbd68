"""CPU oracle for exact two-terminal reliability (BAT + PLSA + Eq. 1).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The HIP
library never imports, links or calls it, and shares no code with it.

``bat_oracle.c`` holds the arithmetic (see its header for the paper passages
it follows); this module is a ctypes wrapper around it plus the build step.
``pbat.py`` runs the oracle over the equal divisions of Section 4 on several
host processes; ``frontier_dp.py`` is a second, independent exact method
(a frontier dynamic programme) used to pin full-size results.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bat_oracle.c")
_SRC_MS = os.path.join(_HERE, "ms_oracle.c")
_LIB = os.path.join(_HERE, "libbat_oracle.so")
_lock = threading.Lock()
_lib = None

ORC_OK = 0
ORC_EINVAL = -1
ORC_ETOOBIG = -2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, single thread)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in (_SRC, _SRC_MS))
    if force or stale:
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, _SRC_MS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = ctypes.CDLL(_LIB)
            i32, u64, i64 = ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64
            P = ctypes.c_void_p
            lib.orc_validate.argtypes = [i32, i32, P, P, i32, i32]
            lib.orc_validate.restype = ctypes.c_int
            lib.orc_dec_inv.argtypes = [i32, u64, P]
            lib.orc_dec_inv.restype = None
            lib.orc_dec.argtypes = [i32, P]
            lib.orc_dec.restype = u64
            lib.orc_bat_next.argtypes = [i32, P]
            lib.orc_bat_next.restype = ctypes.c_int
            lib.orc_plsa.argtypes = [i32, i32, P, P, i32, i32, i32, P, P, P]
            lib.orc_plsa.restype = ctypes.c_int
            lib.orc_pr.argtypes = [i32, P, P]
            lib.orc_pr.restype = ctypes.c_double
            lib.orc_range.argtypes = [i32, i32, P, P, i32, i32, i32, u64, u64, P, P, P, P, P, P]
            lib.orc_range.restype = ctypes.c_int
            lib.orc_range_order.argtypes = [i32, i32, P, P, i32, i32, i32, i32, u64, u64, P, P, P, P, P, P]
            lib.orc_range_order.restype = ctypes.c_int
            lib.orc_dec_inv_fwd.argtypes = [i32, u64, P]
            lib.orc_dec_inv_fwd.restype = None
            lib.orc_bat_next_fwd.argtypes = [i32, P]
            lib.orc_bat_next_fwd.restype = ctypes.c_int
            lib.orc_ms_validate.argtypes = [i32, i32, P, P, P, P, i32, i32, i32]
            lib.orc_ms_validate.restype = ctypes.c_int
            lib.orc_ms_decode.argtypes = [i32, P, u64, P]
            lib.orc_ms_decode.restype = None
            lib.orc_ms_next.argtypes = [i32, P, P]
            lib.orc_ms_next.restype = ctypes.c_int
            lib.orc_ms_range.argtypes = [i32, i32, P, P, P, P, i32, i32, i32, i32, u64, u64, P, P, P, P]
            lib.orc_ms_range.restype = ctypes.c_int
            lib.orc_ms_maxflow.argtypes = [i32, i32, P, P, i32, i32, i32]
            lib.orc_ms_maxflow.restype = i64
            _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _arcs(arcs) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(arcs, dtype=np.int32).reshape(-1, 2))
    return a


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}")
        self.code = code


@dataclass
class RangeResult:
    sum: float          # compensated pair collapsed: sum + comp
    sum_hi: float
    sum_lo: float
    count: int
    U: float            # mass of disconnected vectors (sum + comp)
    T1: Optional[np.ndarray]
    T0: Optional[np.ndarray]
    layers: int
    inspections: int

    @property
    def grad(self) -> Optional[np.ndarray]:
        return None if self.T1 is None else self.T1 - self.T0


def validate(n, arcs, p, s, t) -> int:
    a = _arcs(arcs)
    pv = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
    return _load().orc_validate(n, a.shape[0], _ptr(a), _ptr(pv), s, t)


def dec_inv(m: int, c: int) -> tuple:
    """Eq. 3: the 0-based c-th vector of the backward BAT (paper index c+1)."""
    x = np.zeros(max(m, 1), dtype=np.uint8)
    _load().orc_dec_inv(m, c, _ptr(x))
    return tuple(int(v) for v in x[:m])


def dec(x) -> int:
    """Eq. 2: Dec(X) (0-based; the paper's index is Dec(X) + 1)."""
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.uint8))
    return int(_load().orc_dec(len(xa), _ptr(xa)))


def dec_inv_fwd(m: int, c: int) -> tuple:
    """Eq. 5 (forward BAT): the 0-based c-th vector, x_1 least significant."""
    x = np.zeros(max(m, 1), dtype=np.uint8)
    _load().orc_dec_inv_fwd(m, c, _ptr(x))
    return tuple(int(v) for v in x[:m])


def bat_sequence(m: int, forward: bool = False):
    """All 2^m vectors in the order the BAT of Section 3.1 generates them
    (forward=True: the forward BAT of Section 4.2, updating from x_1)."""
    lib = _load()
    step = lib.orc_bat_next_fwd if forward else lib.orc_bat_next
    x = np.zeros(max(m, 1), dtype=np.uint8)
    out = [tuple(int(v) for v in x[:m])]
    while step(m, _ptr(x)):
        out.append(tuple(int(v) for v in x[:m]))
    return out


def plsa(n, arcs, s, t, x, directed=False):
    """PLSA on G(X): (connected, number of layers, layer index per node)."""
    a = _arcs(arcs)
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.uint8))
    assert xa.shape[0] == a.shape[0]
    L = ctypes.c_int32(0)
    I = ctypes.c_int64(0)
    lay = np.zeros(n, dtype=np.int32)
    rc = _load().orc_plsa(n, a.shape[0], _ptr(a), _ptr(xa), s, t, int(directed),
                          ctypes.byref(L), ctypes.byref(I), _ptr(lay))
    if rc < 0:
        raise OracleError(rc)
    return bool(rc), int(L.value), lay


def plsa_work(n, arcs, s, t, x, directed=False):
    """PLSA on G(X) with its work counters: (connected, layers, arc
    inspections).  These counters are what the range sums' ``layers`` and
    ``inspections`` add up over the vectors of a range."""
    a = _arcs(arcs)
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.uint8))
    assert xa.shape[0] == a.shape[0]
    L = ctypes.c_int32(0)
    I = ctypes.c_int64(0)
    rc = _load().orc_plsa(n, a.shape[0], _ptr(a), _ptr(xa), s, t, int(directed),
                          ctypes.byref(L), ctypes.byref(I), None)
    if rc < 0:
        raise OracleError(rc)
    return bool(rc), int(L.value), int(I.value)


def pr(p, x) -> float:
    pv = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.uint8))
    return float(_load().orc_pr(len(pv), _ptr(pv), _ptr(xa)))


def reliability_range(n, arcs, p, s, t, c_lo, c_hi, grad=False, directed=False, forward=False) -> RangeResult:
    """BAT over backward-order indices [c_lo, c_hi) (forward=True: forward
    BAT indices, Eq. 4-5)."""
    a = _arcs(arcs)
    m = a.shape[0]
    pv = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
    if pv.shape[0] != m:
        raise OracleError(ORC_EINVAL)
    sum2 = np.zeros(2)
    usum2 = np.zeros(2)
    cnt = ctypes.c_uint64(0)
    stats = np.zeros(2, dtype=np.int64)
    T1 = np.zeros(2 * max(m, 1)) if grad else None
    T0 = np.zeros(2 * max(m, 1)) if grad else None
    rc = _load().orc_range_order(n, m, _ptr(a), _ptr(pv), s, t, int(directed), int(forward), int(c_lo),
                                 int(c_hi), _ptr(sum2), ctypes.byref(cnt), _ptr(usum2), _ptr(T1), _ptr(T0),
                                 _ptr(stats))
    if rc != ORC_OK:
        raise OracleError(rc)
    t1 = t0 = None
    if grad:
        t1 = T1[0:2 * m:2] + T1[1:2 * m:2]
        t0 = T0[0:2 * m:2] + T0[1:2 * m:2]
    return RangeResult(float(sum2[0] + sum2[1]), float(sum2[0]), float(sum2[1]), int(cnt.value),
                       float(usum2[0] + usum2[1]), t1, t0, int(stats[0]), int(stats[1]))


def reliability(n, arcs, p, s, t, grad=False, directed=False) -> RangeResult:
    m = len(np.asarray(arcs).reshape(-1, 2))
    return reliability_range(n, arcs, p, s, t, 0, 1 << m, grad=grad, directed=directed)


def net_reliability(net, p=None, grad=False, directed=False) -> RangeResult:
    """Convenience wrapper taking a ``bat_workloads.Network``."""
    return reliability(net.n, net.arc_array(), net.p if p is None else p, net.s, net.t,
                       grad=grad, directed=directed)


# ------------------------------------------------------------ multi-state
# Arcs with sigma_i states, state k of arc i having capacity cap_i(k) and
# probability w_i(k); a vector meets demand d when the maximum s-t flow is at
# least d (ms_oracle.c states the reading).  States are passed per arc, arc
# 0's states first: a list of per-arc sequences or one flat array.

@dataclass
class MsResult:
    sum: float
    sum_hi: float
    sum_lo: float
    count: int
    U: float
    inspections: int


def _flat(per_arc, dtype):
    if per_arc is None:
        return None
    if isinstance(per_arc, np.ndarray) and per_arc.ndim == 1:
        return np.ascontiguousarray(per_arc.astype(dtype))
    return np.ascontiguousarray(np.concatenate([np.asarray(v, dtype=dtype).reshape(-1) for v in per_arc])
                                if len(per_arc) else np.zeros(0, dtype=dtype))


def ms_validate(n, arcs, sigma, cap, w, s, t, d) -> int:
    a = _arcs(arcs)
    sg = np.ascontiguousarray(np.asarray(sigma, dtype=np.int32))
    return _load().orc_ms_validate(n, a.shape[0], _ptr(a), _ptr(sg), _ptr(_flat(cap, np.int32)),
                                   _ptr(_flat(w, np.float64)), s, t, d)


def ms_decode(sigma, c: int) -> tuple:
    sg = np.ascontiguousarray(np.asarray(sigma, dtype=np.int32))
    x = np.zeros(max(len(sg), 1), dtype=np.int32)
    _load().orc_ms_decode(len(sg), _ptr(sg), c, _ptr(x))
    return tuple(int(v) for v in x[:len(sg)])


def ms_sequence(sigma):
    """Every vector in the order the generalised BAT update visits them."""
    lib = _load()
    sg = np.ascontiguousarray(np.asarray(sigma, dtype=np.int32))
    x = np.zeros(max(len(sg), 1), dtype=np.int32)
    out = [tuple(int(v) for v in x[:len(sg)])]
    while lib.orc_ms_next(len(sg), _ptr(sg), _ptr(x)):
        out.append(tuple(int(v) for v in x[:len(sg)]))
    return out


def ms_maxflow(n, arcs, capx, s, t, directed=False) -> int:
    a = _arcs(arcs)
    c = np.ascontiguousarray(np.asarray(capx, dtype=np.int64))
    return int(_load().orc_ms_maxflow(n, a.shape[0], _ptr(a), _ptr(c), s, t, int(directed)))


def ms_reliability_range(n, arcs, sigma, cap, w, s, t, d, c_lo, c_hi, directed=False) -> MsResult:
    a = _arcs(arcs)
    m = a.shape[0]
    sg = np.ascontiguousarray(np.asarray(sigma, dtype=np.int32))
    if sg.shape[0] != m:
        raise OracleError(ORC_EINVAL)
    cf = _flat(cap, np.int32)
    wf = _flat(w, np.float64)
    sum2 = np.zeros(2)
    usum2 = np.zeros(2)
    cnt = ctypes.c_uint64(0)
    stats = np.zeros(1, dtype=np.int64)
    rc = _load().orc_ms_range(n, m, _ptr(a), _ptr(sg), _ptr(cf), _ptr(wf), s, t, d, int(directed), int(c_lo),
                              int(c_hi), _ptr(sum2), ctypes.byref(cnt), _ptr(usum2), _ptr(stats))
    if rc != ORC_OK:
        raise OracleError(rc)
    return MsResult(float(sum2[0] + sum2[1]), float(sum2[0]), float(sum2[1]), int(cnt.value),
                    float(usum2[0] + usum2[1]), int(stats[0]))


def ms_reliability(n, arcs, sigma, cap, w, s, t, d, directed=False) -> MsResult:
    N = 1
    for v in sigma:
        N *= int(v)
    return ms_reliability_range(n, arcs, sigma, cap, w, s, t, d, 0, N, directed=directed)
