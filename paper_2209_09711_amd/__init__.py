"""MI355X-native exact two-terminal reliability by binary-addition-tree
enumeration (BAT, arXiv 2209.09711): Python binding of ``libbat_hip.so``.

Every function here only marshals arguments for the C ABI declared in
``include/bat.h`` (same names); all enumeration, connectivity and
probability arithmetic runs in the HIP kernels.  There is no CPU fallback:
if the library is missing, importing this package raises ``ImportError``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbat_hip.so")

BAT_OK = 0
BAT_EINVAL = -1
BAT_ETOOBIG = -2
BAT_EDEVICE = -3
BAT_ENOMEM = -4
BAT_EIO = -5
BAT_PENDING = 1
BAT_MAX_NODES = 64
BAT_MAX_ARCS = 62
BAT_MAX_PVEC = 1024

# Every entry point of include/bat.h.
EXPORTED = ("bat_version", "bat_last_error", "bat_reliability", "bat_reliability_grad",
            "bat_reliability_range", "bat_reliability_batched", "bat_reliability_async",
            "bat_reliability_grad_async", "bat_set_option", "bat_get_option", "bat_autotune",
            "bat_last_launch", "bat_jit_source", "bat_autotune_batched", "bat_reliability_ex",
            "bat_reliability_range_ex", "bat_reliability_checkpointed", "bat_valu_peak",
            "bat_reliability_noalloc", "bat_ms_reliability", "bat_ms_reliability_range",
            "bat_ms_jit_source")


class bat_arc(ctypes.Structure):
    _fields_ = [("u", ctypes.c_int32), ("v", ctypes.c_int32)]


class bat_launch_info(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("jit_ms", ctypes.c_double), ("vectors", ctypes.c_uint64),
                ("specialised", ctypes.c_int32), ("chunk_log2", ctypes.c_int32),
                ("n_chunks", ctypes.c_int32), ("relaxations", ctypes.c_int32),
                ("kernel_id", ctypes.c_uint64), ("perm", ctypes.c_int32),
                ("chain_log2", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("item_order", ctypes.c_int32), ("block_waves", ctypes.c_int32),
                ("super_restart", ctypes.c_int32), ("window_test", ctypes.c_int32),
                ("simd_waves", ctypes.c_int32), ("keep_bottom", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


def _load():
    # PyTorch wheels bundle their own HIP runtime under the same soname
    # (libamdhip64.so.7) but link it by its unversioned name.  If torch is
    # loaded first, this library's libamdhip64.so.7 dependency binds to that
    # same runtime, so torch tensors and streams are valid here.  If this
    # library came first, torch would load a second runtime and fail to see
    # the GPU.  So load torch first whenever it is installed.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                          f"g.build()'` (the HIP library is required; there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    i32, u64, i64, dbl = ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
    P = ctypes.c_void_p
    sig = {
        "bat_version": ([], ctypes.c_char_p),
        "bat_last_error": ([], ctypes.c_char_p),
        "bat_reliability": ([i32, i32, P, P, i32, i32, P, P], ctypes.c_int),
        "bat_reliability_grad": ([i32, i32, P, P, i32, i32, P, P, P, P, P], ctypes.c_int),
        "bat_reliability_range": ([i32, i32, P, P, i32, i32, u64, u64, P, P, P, P, P], ctypes.c_int),
        "bat_reliability_batched": ([i32, P, P, P, P, P, i32, P, P, P], ctypes.c_int),
        "bat_reliability_async": ([i32, i32, P, P, i32, i32, P, P, P, P], ctypes.c_int),
        "bat_reliability_grad_async": ([i32, i32, P, P, i32, i32, P, P, P, P, P, P, P], ctypes.c_int),
        "bat_reliability_noalloc": ([i32, i32, P, P, i32, i32, P, P, P, P], ctypes.c_int),
        "bat_ms_reliability": ([i32, i32, P, P, P, P, i32, i32, i32, ctypes.c_uint32, P, P], ctypes.c_int),
        "bat_ms_reliability_range": ([i32, i32, P, P, P, P, i32, i32, i32, ctypes.c_uint32, u64, u64, P, P, P],
                                     ctypes.c_int),
        "bat_set_option": ([ctypes.c_char_p, i64], ctypes.c_int),
        "bat_get_option": ([ctypes.c_char_p, P], ctypes.c_int),
        "bat_autotune": ([i32, i32, P, P, i32, i32, P], ctypes.c_int),
        "bat_last_launch": ([P], ctypes.c_int),
        "bat_jit_source": ([i32, i32, P, i32, i32, ctypes.c_uint32, i32, i32, P, P], ctypes.c_int),
        "bat_ms_jit_source": ([i32, i32, P, P, P, i32, i32, i32, ctypes.c_uint32, u64, u64, P, P], ctypes.c_int),
        "bat_autotune_batched": ([i32, P, P, P, P, P, i32, P, P], ctypes.c_int),
        "bat_reliability_ex": ([i32, i32, P, P, i32, i32, ctypes.c_uint32, P, P, P, P, P], ctypes.c_int),
        "bat_reliability_range_ex": ([i32, i32, P, P, i32, i32, ctypes.c_uint32, u64, u64, P, P, P, P, P],
                                     ctypes.c_int),
        "bat_valu_peak": ([P], ctypes.c_int),
        "bat_reliability_checkpointed": ([i32, i32, P, P, i32, i32, ctypes.c_uint32, i32, ctypes.c_char_p, i64,
                                          P, P, P, P, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


class BatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"BAT error {code}: {msg}")
        self.code = code


def _check(rc: int):
    if rc != BAT_OK:
        raise BatError(rc, _lib.bat_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _arcs(arcs) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(arcs, dtype=np.int32).reshape(-1, 2))
    return a


def _p(p, m) -> np.ndarray:
    pv = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(-1))
    if pv.shape[0] != m:
        raise ValueError(f"p has {pv.shape[0]} entries for {m} arcs")
    return pv


# ------------------------------------------------------------ thin C names

def bat_version() -> str:
    return _lib.bat_version().decode()


def bat_last_error() -> str:
    return _lib.bat_last_error().decode()


def bat_reliability(n_nodes: int, arcs, p, s: int, t: int) -> Tuple[float, int]:
    """(R, feasible-vector count) of Eq. 1; arcs as (m, 2) node pairs."""
    a = _arcs(arcs)
    pv = _p(p, a.shape[0])
    R = ctypes.c_double(0.0)
    cnt = ctypes.c_uint64(0)
    _check(_lib.bat_reliability(n_nodes, a.shape[0], _ptr(a), _ptr(pv), s, t, ctypes.byref(R), ctypes.byref(cnt)))
    return R.value, cnt.value


@dataclass
class GradResult:
    R: float
    count: int
    dRdp: np.ndarray
    T1: np.ndarray
    T0: np.ndarray


def bat_reliability_grad(n_nodes: int, arcs, p, s: int, t: int) -> GradResult:
    a = _arcs(arcs)
    m = a.shape[0]
    pv = _p(p, m)
    R = ctypes.c_double(0.0)
    cnt = ctypes.c_uint64(0)
    g = np.zeros(max(m, 1))
    T1 = np.zeros(max(m, 1))
    T0 = np.zeros(max(m, 1))
    _check(_lib.bat_reliability_grad(n_nodes, m, _ptr(a), _ptr(pv), s, t, ctypes.byref(R), ctypes.byref(cnt),
                                     _ptr(g), _ptr(T1), _ptr(T0)))
    return GradResult(R.value, cnt.value, g[:m], T1[:m], T0[:m])


@dataclass
class RangeResult:
    R_hi: float
    R_lo: float
    count: int
    T1: Optional[np.ndarray]
    T0: Optional[np.ndarray]

    @property
    def R(self) -> float:
        return self.R_hi + self.R_lo


BAT_DIRECTED = 1
BAT_FORWARD_ORDER = 2


def _flags(directed: bool, forward: bool = False) -> int:
    return (BAT_DIRECTED if directed else 0) | (BAT_FORWARD_ORDER if forward else 0)


def bat_reliability_range(n_nodes: int, arcs, p, s: int, t: int, c_lo: int, c_hi: int,
                          grad: bool = False, directed: bool = False, forward: bool = False) -> RangeResult:
    """Partial sums over indices [c_lo, c_hi): backward BAT order, or the
    forward order (forward=True); directed=True reads arcs as u -> v."""
    a = _arcs(arcs)
    m = a.shape[0]
    pv = _p(p, m)
    hi = ctypes.c_double(0.0)
    lo = ctypes.c_double(0.0)
    cnt = ctypes.c_uint64(0)
    T1 = np.zeros(max(m, 1)) if grad else None
    T0 = np.zeros(max(m, 1)) if grad else None
    flags = _flags(directed, forward)
    if flags:
        _check(_lib.bat_reliability_range_ex(n_nodes, m, _ptr(a), _ptr(pv), s, t, flags, int(c_lo), int(c_hi),
                                             ctypes.byref(hi), ctypes.byref(lo), ctypes.byref(cnt), _ptr(T1),
                                             _ptr(T0)))
    else:
        _check(_lib.bat_reliability_range(n_nodes, m, _ptr(a), _ptr(pv), s, t, int(c_lo), int(c_hi),
                                          ctypes.byref(hi), ctypes.byref(lo), ctypes.byref(cnt), _ptr(T1), _ptr(T0)))
    return RangeResult(hi.value, lo.value, cnt.value, None if T1 is None else T1[:m], None if T0 is None else T0[:m])


def _ms_args(arcs, n_states, capacity, w):
    a = _arcs(arcs)
    m = a.shape[0]
    sg = np.ascontiguousarray(np.asarray(n_states, dtype=np.int32).reshape(-1))
    if sg.shape[0] != m:
        raise BatError(BAT_EINVAL, f"n_states has {sg.shape[0]} entries for {m} arcs")
    total = int(sg.sum()) if m else 0

    def flat(x, dt):
        if x is None:
            return None
        if isinstance(x, np.ndarray) and x.ndim == 1:
            v = np.ascontiguousarray(x, dtype=dt)
        else:
            v = np.ascontiguousarray(np.concatenate([np.asarray(r, dtype=dt).reshape(-1) for r in x])
                                     if len(x) else np.zeros(0, dtype=dt))
        if v.shape[0] != total:
            raise BatError(BAT_EINVAL, f"{v.shape[0]} per-state entries for {total} states")
        return v

    return a, m, sg, flat(capacity, np.int32), flat(w, np.float64)


def bat_ms_reliability(n_nodes: int, arcs, n_states, capacity, w, s: int, t: int, demand: int,
                       directed: bool = False) -> Tuple[float, int]:
    """Multi-state arcs: R_d and the count of state vectors whose maximum
    s-t flow reaches `demand`.  capacity and w: per arc, its states'
    capacities (None: state k carries k) and probabilities, as a list of
    sequences or one flat array."""
    a, m, sg, cf, wf = _ms_args(arcs, n_states, capacity, w)
    R = ctypes.c_double(0.0)
    cnt = ctypes.c_uint64(0)
    _check(_lib.bat_ms_reliability(n_nodes, m, _ptr(a), _ptr(sg), _ptr(cf), _ptr(wf), s, t, demand,
                                   _flags(directed), ctypes.byref(R), ctypes.byref(cnt)))
    return R.value, cnt.value


def bat_ms_reliability_range(n_nodes: int, arcs, n_states, capacity, w, s: int, t: int, demand: int,
                             c_lo: int, c_hi: int, directed: bool = False) -> RangeResult:
    """Partial sums over mixed-radix indices [c_lo, c_hi) (arc 0 most
    significant)."""
    a, m, sg, cf, wf = _ms_args(arcs, n_states, capacity, w)
    hi = ctypes.c_double(0.0)
    lo = ctypes.c_double(0.0)
    cnt = ctypes.c_uint64(0)
    _check(_lib.bat_ms_reliability_range(n_nodes, m, _ptr(a), _ptr(sg), _ptr(cf), _ptr(wf), s, t, demand,
                                         _flags(directed), int(c_lo), int(c_hi), ctypes.byref(hi),
                                         ctypes.byref(lo), ctypes.byref(cnt)))
    return RangeResult(hi.value, lo.value, cnt.value, None, None)


def bat_reliability_ex(n_nodes: int, arcs, p, s: int, t: int, directed: bool = False, grad: bool = False):
    """bat_reliability / bat_reliability_grad with flags: (R, count) or a
    GradResult."""
    a = _arcs(arcs)
    m = a.shape[0]
    pv = _p(p, m)
    R = ctypes.c_double(0.0)
    cnt = ctypes.c_uint64(0)
    g = np.zeros(max(m, 1)) if grad else None
    T1 = np.zeros(max(m, 1)) if grad else None
    T0 = np.zeros(max(m, 1)) if grad else None
    _check(_lib.bat_reliability_ex(n_nodes, m, _ptr(a), _ptr(pv), s, t, _flags(directed), ctypes.byref(R),
                                   ctypes.byref(cnt), _ptr(g), _ptr(T1), _ptr(T0)))
    if not grad:
        return R.value, cnt.value
    return GradResult(R.value, cnt.value, g[:m], T1[:m], T0[:m])


def bat_reliability_checkpointed(n_nodes: int, arcs, p, s: int, t: int, chunk_log2: int, path=None,
                                 max_chunks: int = -1, grad: bool = False, directed: bool = False,
                                 forward: bool = False):
    """A whole sweep run as chunks of 2^chunk_log2 indices, with the running
    sums kept in the checkpoint file `path` (None: no file).  Returns None
    while chunks remain (BAT_PENDING), else (R, count) or a GradResult."""
    a = _arcs(arcs)
    m = a.shape[0]
    pv = _p(p, m)
    R = ctypes.c_double(0.0)
    cnt = ctypes.c_uint64(0)
    g = np.zeros(max(m, 1)) if grad else None
    T1 = np.zeros(max(m, 1)) if grad else None
    T0 = np.zeros(max(m, 1)) if grad else None
    rc = _lib.bat_reliability_checkpointed(n_nodes, m, _ptr(a), _ptr(pv), s, t, _flags(directed, forward),
                                           int(chunk_log2), None if path is None else os.fsencode(path),
                                           int(max_chunks), ctypes.byref(R), ctypes.byref(cnt), _ptr(g), _ptr(T1),
                                           _ptr(T0))
    if rc == BAT_PENDING:
        return None
    _check(rc)
    if not grad:
        return R.value, cnt.value
    return GradResult(R.value, cnt.value, g[:m], T1[:m], T0[:m])


def _batch_args(graphs, p_blocks):
    G = len(graphs)
    if G == 0:
        raise ValueError("no graphs")
    n_pvec = int(np.asarray(p_blocks[0]).shape[0])
    nn = np.asarray([g[0] for g in graphs], dtype=np.int32)
    arcs_l = [_arcs(g[1]) for g in graphs]
    off = np.zeros(G + 1, dtype=np.int32)
    off[1:] = np.cumsum([a.shape[0] for a in arcs_l])
    arcs = np.ascontiguousarray(np.concatenate(arcs_l, axis=0) if off[-1] else np.zeros((1, 2), np.int32))
    ss = np.asarray([g[2] for g in graphs], dtype=np.int32)
    tt = np.asarray([g[3] for g in graphs], dtype=np.int32)
    blocks = []
    for g, pb in enumerate(p_blocks):
        pb = np.asarray(pb, dtype=np.float64)
        if pb.shape != (n_pvec, arcs_l[g].shape[0]):
            raise ValueError(f"p block {g} has shape {pb.shape}, want {(n_pvec, arcs_l[g].shape[0])}")
        blocks.append(pb.reshape(-1))
    p = np.ascontiguousarray(np.concatenate(blocks) if blocks else np.zeros(1))
    return G, nn, off, arcs, ss, tt, n_pvec, p


def bat_reliability_batched(graphs: Sequence[Tuple[int, object, int, int]], p_blocks: Sequence[np.ndarray]):
    """graphs: [(n_nodes, arcs, s, t)], p_blocks[g]: (n_pvec, m_g) array.
    Returns (R[n_graphs, n_pvec], counts[n_graphs])."""
    G, nn, off, arcs, ss, tt, n_pvec, p = _batch_args(graphs, p_blocks)
    R = np.zeros(G * n_pvec)
    cnt = np.zeros(G, dtype=np.uint64)
    _check(_lib.bat_reliability_batched(G, _ptr(nn), _ptr(off), _ptr(arcs), _ptr(ss), _ptr(tt), n_pvec, _ptr(p),
                                        _ptr(R), _ptr(cnt)))
    return R.reshape(G, n_pvec), cnt


def bat_autotune_batched(graphs: Sequence[Tuple[int, object, int, int]], p_blocks: Sequence[np.ndarray]) -> float:
    """Tune the batched launch for this batch structure; returns the best
    kernel time in ms."""
    G, nn, off, arcs, ss, tt, n_pvec, p = _batch_args(graphs, p_blocks)
    ms = ctypes.c_double(0.0)
    _check(_lib.bat_autotune_batched(G, _ptr(nn), _ptr(off), _ptr(arcs), _ptr(ss), _ptr(tt), n_pvec, _ptr(p),
                                     ctypes.byref(ms)))
    return ms.value


def bat_set_option(key: str, value: int):
    _check(_lib.bat_set_option(key.encode(), int(value)))


def bat_get_option(key: str) -> int:
    v = ctypes.c_int64(0)
    _check(_lib.bat_get_option(key.encode(), ctypes.byref(v)))
    return v.value


def bat_autotune(n_nodes: int, arcs, p, s: int, t: int) -> float:
    """Tune the launch for this graph structure; returns ns per state vector."""
    a = _arcs(arcs)
    pv = _p(p, a.shape[0])
    ns = ctypes.c_double(0.0)
    _check(_lib.bat_autotune(n_nodes, a.shape[0], _ptr(a), _ptr(pv), s, t, ctypes.byref(ns)))
    return ns.value


def bat_jit_source(n_nodes: int, arcs, s: int, t: int, grad: bool = False, perm: int = 0,
                   directed: bool = False, batch_pvec: int = 0) -> str:
    """The hiprtc source of the graph-specialised kernel (diagnostics);
    batch_pvec > 0: the batched sweep of that many p-vectors."""
    a = _arcs(arcs)
    n = ctypes.c_uint64(0)
    f = _flags(directed)
    g = -int(batch_pvec) if batch_pvec else int(grad)
    _check(_lib.bat_jit_source(n_nodes, a.shape[0], _ptr(a), s, t, f, g, perm, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(_lib.bat_jit_source(n_nodes, a.shape[0], _ptr(a), s, t, f, g, perm, buf, ctypes.byref(n)))
    return buf.value.decode()


def bat_ms_jit_source(n_nodes: int, arcs, n_states, capacity, s: int, t: int, demand: int,
                      directed: bool = False, c_lo: int = 0, c_hi: int = 0) -> str:
    """The hiprtc source of the bit-sliced multi-state kernel that a sweep
    with demand 1 to 3 compiles (diagnostics): the whole space when
    c_lo = c_hi = 0, else the range [c_lo, c_hi)."""
    w = [[1.0] * int(k) for k in n_states]
    a, m, sg, cf, _ = _ms_args(arcs, n_states, capacity, w)
    n = ctypes.c_uint64(0)
    f = _flags(directed)
    args = (n_nodes, m, _ptr(a), _ptr(sg), _ptr(cf), s, t, demand, f, int(c_lo), int(c_hi))
    _check(_lib.bat_ms_jit_source(*args, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(_lib.bat_ms_jit_source(*args, buf, ctypes.byref(n)))
    return buf.value.decode()


def bat_valu_peak() -> float:
    """Measured sustained integer VALU rate (32-bit lane-ops/s)."""
    r = ctypes.c_double(0.0)
    _check(_lib.bat_valu_peak(ctypes.byref(r)))
    return r.value


def bat_last_launch() -> bat_launch_info:
    info = bat_launch_info()
    _check(_lib.bat_last_launch(ctypes.byref(info)))
    return info


def bat_reliability_async(n_nodes: int, arcs, p_dev_ptr: int, s: int, t: int, R_dev_ptr: int,
                          count_dev_ptr: int, status_dev_ptr: Optional[int], stream: int):
    a = _arcs(arcs)
    _check(_lib.bat_reliability_async(n_nodes, a.shape[0], _ptr(a), p_dev_ptr, s, t, R_dev_ptr, count_dev_ptr,
                                      status_dev_ptr, stream))


def bat_reliability_noalloc(n_nodes: int, arcs, p_dev_ptr: int, s: int, t: int, R_dev_ptr: int,
                            count_dev_ptr: int, status_dev_ptr: Optional[int], stream: int):
    a = _arcs(arcs)
    _check(_lib.bat_reliability_noalloc(n_nodes, a.shape[0], _ptr(a), p_dev_ptr, s, t, R_dev_ptr, count_dev_ptr,
                                        status_dev_ptr, stream))


def bat_reliability_grad_async(n_nodes: int, arcs, p_dev_ptr: int, s: int, t: int, R_dev_ptr: int,
                               count_dev_ptr: int, dRdp_dev_ptr: int, T1_dev_ptr: Optional[int],
                               T0_dev_ptr: Optional[int], status_dev_ptr: Optional[int], stream: int):
    a = _arcs(arcs)
    _check(_lib.bat_reliability_grad_async(n_nodes, a.shape[0], _ptr(a), p_dev_ptr, s, t, R_dev_ptr,
                                           count_dev_ptr, dRdp_dev_ptr, T1_dev_ptr, T0_dev_ptr, status_dev_ptr,
                                           stream))


# ------------------------------------------------------------ friendly names
reliability = bat_reliability
reliability_grad = bat_reliability_grad
reliability_range = bat_reliability_range
reliability_batched = bat_reliability_batched
autotune = bat_autotune
version = bat_version
