"""PBAT harness: the oracle run over the equal divisions of Sections 4-5.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Equal-division policy (Eq. 6): with chi = 2^d divisions of the 2^m
backward-order indices, division i (1-based) holds the mu = 2^m / chi
vectors with 1-based indices (i-1)*mu + k, k = 1..mu, i.e. the vectors whose
first d coordinates spell i-1 in binary (Eq. 7).  Each division is one
independent oracle call (PBAT STEP 2), run in its own host process; STEP 3
adds the per-division results, here in fixed division order with
double-double arithmetic so the combined value does not depend on which
process finished first.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import reliability_range


def two_sum(a: float, b: float):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def dd_add(hi: float, lo: float, x_hi: float, x_lo: float = 0.0):
    s, e = two_sum(hi, x_hi)
    e += lo + x_lo
    return two_sum(s, e)


def division_bounds(m: int, chi: int, i: int):
    """0-based index range [lo, hi) of the 1-based division i (Eq. 6)."""
    if chi <= 0 or chi & (chi - 1):
        raise ValueError("chi must be a power of two")
    if chi > (1 << m):
        raise ValueError("chi exceeds the number of vectors")
    mu = (1 << m) // chi
    return (i - 1) * mu, i * mu


def division_prefix(m: int, chi: int, i: int):
    """Eq. 7: the first log2(chi) coordinates shared by every vector of
    division i (the i-th vector of B^(log2 chi))."""
    d = chi.bit_length() - 1
    return tuple(((i - 1) >> (d - 1 - k)) & 1 for k in range(d))


def _work(args):
    n, arcs, p, s, t, lo, hi, grad, directed = args
    r = reliability_range(n, arcs, p, s, t, lo, hi, grad=grad, directed=directed)
    return (r.sum_hi, r.sum_lo, r.count, r.T1, r.T0, r.inspections, r.layers)


@dataclass
class PbatResult:
    R: float
    R_hi: float
    R_lo: float
    count: int
    division_R: List[float]
    division_count: List[int]
    T1: Optional[np.ndarray]
    T0: Optional[np.ndarray]
    vectors: int
    inspections: int
    layers: int
    wall_s: float
    processes: int


def run(n, arcs, p, s, t, chi: int, divisions: Optional[Sequence[int]] = None,
        grad: bool = False, directed: bool = False, processes: Optional[int] = None) -> PbatResult:
    """Run the oracle on the given 1-based divisions (default: all chi)."""
    arcs = np.ascontiguousarray(np.asarray(arcs, dtype=np.int32).reshape(-1, 2))
    m = arcs.shape[0]
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
    divs = list(range(1, chi + 1)) if divisions is None else [int(i) for i in divisions]
    jobs = []
    for i in divs:
        lo, hi = division_bounds(m, chi, i)
        jobs.append((n, arcs, p, s, t, lo, hi, grad, directed))
    procs = processes or os.cpu_count() or 1
    t0 = time.perf_counter()
    if procs == 1 or len(jobs) == 1:
        outs = [_work(j) for j in jobs]
    else:
        ctx = mp.get_context("fork")
        with ctx.Pool(min(procs, len(jobs))) as pool:
            outs = pool.map(_work, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    hi = lo = 0.0
    cnt = 0
    T1 = np.zeros(m) if grad else None
    T0 = np.zeros(m) if grad else None
    T1c = np.zeros(m) if grad else None
    T0c = np.zeros(m) if grad else None
    insp = lay = 0
    dR, dC = [], []
    for (sh, sl, c, t1, t0, ins, ly) in outs:  # STEP 3, fixed division order
        hi, lo = dd_add(hi, lo, sh, sl)
        cnt += c
        insp += ins
        lay += ly
        dR.append(sh + sl)
        dC.append(c)
        if grad:
            for k in range(m):
                T1[k], T1c[k] = dd_add(T1[k], T1c[k], float(t1[k]))
                T0[k], T0c[k] = dd_add(T0[k], T0c[k], float(t0[k]))
    if grad:
        T1 = T1 + T1c
        T0 = T0 + T0c
    nvec = sum(division_bounds(m, chi, i)[1] - division_bounds(m, chi, i)[0] for i in divs)
    return PbatResult(hi + lo, hi, lo, cnt, dR, dC, T1, T0, nvec, insp, lay, wall, procs)


def spread_divisions(chi: int, k: int) -> List[int]:
    """k distinct divisions spread over 1..chi (for sampled timing and
    checks: the cost of a vector varies along the counter, so a prefix slice
    is not representative).  Golden-ratio (Weyl) sequence: evenly spread,
    and unlike evenly strided indices it varies every bit of the division
    prefix, i.e. every one of the leading arcs' states."""
    k = max(1, min(k, chi))
    phi = 0.6180339887498949
    out, seen, j = [], set(), 0
    while len(out) < k:
        i = 1 + int(((j + 1) * phi % 1.0) * chi)
        j += 1
        if i not in seen:
            seen.add(i)
            out.append(i)
    return sorted(out)


def run_ranges(jobs, processes: Optional[int] = None):
    """Oracle calls on (n, arcs, p, s, t, lo, hi) index ranges of several
    networks in one process pool; per job: (R, count, inspections, layers),
    plus the pool's wall time (for timing samples that span many graphs)."""
    work = [(n, np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1, 2)),
             np.ascontiguousarray(np.asarray(p, dtype=np.float64)), s, t, lo, hi, False, False)
            for (n, a, p, s, t, lo, hi) in jobs]
    procs = processes or os.cpu_count() or 1
    t0 = time.perf_counter()
    if procs == 1 or len(work) == 1:
        outs = [_work(j) for j in work]
    else:
        ctx = mp.get_context("fork")
        with ctx.Pool(min(procs, len(work))) as pool:
            outs = pool.map(_work, work, chunksize=1)
    wall = time.perf_counter() - t0
    return [(sh + sl, c, ins, ly) for (sh, sl, c, _t1, _t0, ins, ly) in outs], wall


def _ms_work(args):
    from . import ms_reliability_range
    n, arcs, sigma, cap, w, s, t, d, lo, hi = args
    r = ms_reliability_range(n, arcs, sigma, cap, w, s, t, d, lo, hi)
    return r.sum_hi + r.sum_lo, r.count, r.inspections


def run_ms_ranges(net, ranges, processes: Optional[int] = None):
    """The multi-state oracle on index ranges of one network, in one process
    pool: per range (R, count, inspections), plus the wall time."""
    jobs = [(net.n, net.arcs, net.sigma, net.cap, net.w, net.s, net.t, net.d, lo, hi) for lo, hi in ranges]
    procs = processes or os.cpu_count() or 1
    t0 = time.perf_counter()
    if procs == 1 or len(jobs) == 1:
        outs = [_ms_work(j) for j in jobs]
    else:
        ctx = mp.get_context("fork")
        with ctx.Pool(min(procs, len(jobs))) as pool:
            outs = pool.map(_ms_work, jobs, chunksize=1)
    return outs, time.perf_counter() - t0
