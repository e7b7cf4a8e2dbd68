#!/usr/bin/env python3
"""Benchmark: exact two-terminal reliability of the 5x5 grid (m = 40).

One "step" is one complete pass of the hot path over the headline workload:
all 2^40 arc-state vectors of the 5x5 grid enumerated in BAT order, the s-t
connectivity of each decided, and Pr(X) summed in FP64 over the connected
ones, giving the exact R and the feasible-vector count.  The probabilities
are resident in device memory before the timed region starts; R and the
count stay in device memory (stream-ordered entry point).

Printed (one JSON line): vectors/s as the metric value, plus time-to-exact-R
(cold and warm, host call to R on the host), the forward+gradient vs forward
time ratio on the 36-arc differentiation workload, the roofline of the
enumeration kernel (HIP events on its own stream) and the CPU oracle's rate
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs at a 2.4 GHz peak engine clock.  The vector ALUs of a CU
# complete 128 32-bit lane-operations per clock: the chip's vector FP32 rate
# (157.3 TFLOP/s counting an FMA as two) is 256 x 2.4e9 x 128 FMAs, and
# integer add / xor chains issue at that rate too -- the library's VALU-rate
# kernel retires 1.85 wave64 VALU instructions per CU per cycle by its own
# SQ_INSTS_VALU and GRBM_GUI_ACTIVE counters (profiles/k_valu_peak_mi355x.md),
# so one wave64 instruction per CU per clock is not the ceiling.  A
# bit-sliced lane-op decides one arc for 32 state vectors, so the bit-op peak
# is 32x the lane rate.
CUS, CLOCK_HZ = 256, 2.4e9
PEAK_LANE_OPS = CUS * 128 * CLOCK_HZ              # 7.86e13 int32 lane-ops/s
PEAK_BIT_OPS = PEAK_LANE_OPS * 32                 # 2.52e15 bit-ops/s
HOST_CORES_PER_GPU = 16                           # host cores a one-GPU job is given

# Hardware counters of the enumeration kernel on this workload
# (profiles/bat_fwd_jit_grid5x5_m40.md), keyed by the launch they were
# measured on: the kernel identity the library reports (a hash of the exact
# kernel code) and the launch choices.  Any other launch reports null.  The
# profiled runs loaded the kernel an unprofiled run compiled (--jit-cache),
# so the counters are those of this exact code.
#   traffic_bytes: HBM bytes per launch, rocprofv3 FETCH_SIZE x 2.0 +
#     WRITE_SIZE x 1.0 (KiB), the factors of a plain 1 GiB device copy;
#   valu_busy: SQ_INSTS_VALU / (256 CUs x GRBM_GUI_ACTIVE cycles);
#   valu_insts_per_vector: SQ_INSTS_VALU x 64 lanes / 2^40 (lane-ops);
#   salu_busy: SQ_INSTS_SALU / (256 x cycles), the scalar unit's share;
#   lds_busy: SQ_LDS_IDX_ACTIVE / (256 x cycles).
MEASURED = {
    "43a630a3f3b13d07/perm3/chunk12/chain3/check1/order1/waves4/super0/window1/simd6/keep1": {
        "traffic_bytes": (19407.5 * 2.0 + 32203688.0625 * 1.0) * 1024,
        "valu_busy": 0.85,
        "valu_insts_per_vector": 3.58,
        "salu_busy": 0.30,
        "lds_busy": 0.06,
    },
}


def launch_key(li) -> str:
    return (f"{li.kernel_id:016x}/perm{li.perm}/chunk{li.chunk_log2}/chain{li.chain_log2}"
            f"/check{li.check_every}/order{li.item_order}/waves{li.block_waves}/super{li.super_restart}"
            f"/window{li.window_test}/simd{li.simd_waves}/keep{li.keep_bottom}")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the fwd+grad / batched comparisons")
    ap.add_argument("--jit-cache", default=None,
                    help="kernel cache directory to use and keep (default: a fresh temporary one). A profiler "
                         "run pointed at a cache an unprofiled run filled executes the same code objects: "
                         "kernels compiled inside a rocprofv3 process come out with another register allocation. "
                         "The cold time-to-R figure is then not cold.")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--batched-only", action="store_true",
                    help="only tune and time the batched launch on its workload (for profiling runs)")
    ap.add_argument("--batched-pvec", type=int, default=0,
                    help="with --batched-only: use only the first K probability vectors of each graph")
    ap.add_argument("--cpu-sample-log2", type=int, default=30,
                    help="log2 of the state vectors in the oracle's timed sample")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--ms-demand", type=int, default=0,
                    help="with --multistate-only: this demand instead of the workload's")
    ap.add_argument("--multistate-only", action="store_true",
                    help="only time the multi-state workload's sweep (for profiling runs)")
    ap.add_argument("--valu-peak-only", action="store_true",
                    help="only run the sustained integer VALU diagnostic (for counter runs) and exit")
    ap.add_argument("--copy-ref-gib", type=float, default=0.0,
                    help="only run a plain device-to-device copy of this many GiB (the reference kernel "
                         "that scales the HBM byte counters) and exit")
    return ap.parse_args()


def copy_reference(gib: float):
    import torch
    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_reference_bytes_read": 4 * n, "copy_reference_bytes_written": 4 * n}), flush=True)


def host_cpu():
    """CPU model and how many host processes the oracle legs use: the host
    cores a one-GPU job is given (16), fewer if fewer cores are visible."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    visible = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    procs = int(os.environ.get("BAT_BENCH_CPU_PROCS", "0")) or min(visible, HOST_CORES_PER_GPU)
    return model, visible, procs


def oracle_sample(net, sample_log2: int, procs: int, grad: bool = False, chi_log2: int = 17, p=None):
    """The oracle (PBAT equal divisions, Eq. 6) on an evenly spread sample of
    divisions of one network's counter: about 2^sample_log2 vectors."""
    from oracle import pbat
    chi_log2 = min(chi_log2, net.m)
    chi = 1 << chi_log2
    mu_log2 = net.m - chi_log2
    k = max(1, 1 << max(0, sample_log2 - mu_log2))
    divs = pbat.spread_divisions(chi, k)
    r = pbat.run(net.n, net.arcs, net.p if p is None else p, net.s, net.t, chi, divisions=divs, grad=grad,
                 processes=procs)
    return r, len(divs), chi


def cpu_baselines(c2, c4, c3, sample_log2: int):
    """The oracle as it stands, timed on the host cores, on bounded samples of
    each workload, plus the work counters that set each roofline's
    algorithmic work per vector."""
    model, visible, procs = host_cpu()
    out = {"cpu_model": model, "cores_visible": visible, "cores_used": procs}
    # headline: the 5x5 grid, forward, all the host cores the job has
    r, k, chi = oracle_sample(c2, sample_log2, procs)
    out["c2"] = {
        "value": r.vectors / r.wall_s / 1e9, "unit": "Gvec/s", "cores": r.processes, "kind": "oracle",
        "sample": f"{k} of {chi} equal divisions (Eq. 6) spread evenly over the 2^{c2.m} counter, "
                  f"{r.vectors} vectors, {r.wall_s:.1f} s wall on {r.processes} processes ({model})",
        "projected_time_to_R_s": (1 << c2.m) / (r.vectors / r.wall_s),
        "inspections_per_vector": r.inspections / r.vectors, "layers_per_vector": r.layers / r.vectors,
        "connected_fraction": r.count / r.vectors}
    # one core, comparable with the paper's single-thread BAT runs
    r1, k1, chi1 = oracle_sample(c2, sample_log2 - 4, 1)
    out["c2_single_core"] = {
        "value": r1.vectors / r1.wall_s / 1e9, "unit": "Gvec/s", "cores": 1, "kind": "oracle",
        "sample": f"{k1} of {chi1} divisions, {r1.vectors} vectors, {r1.wall_s:.1f} s ({model})",
        "projected_time_to_R_s": (1 << c2.m) / (r1.vectors / r1.wall_s)}
    # the differentiation workload: forward and forward + gradient
    rf, kf, chif = oracle_sample(c4, sample_log2 - 2, procs)
    rg, kg, chig = oracle_sample(c4, sample_log2 - 3, procs, grad=True)
    out["c4"] = {
        "value": rf.vectors / rf.wall_s / 1e9, "unit": "Gvec/s", "cores": rf.processes, "kind": "oracle",
        "sample": f"{kf} of {chif} divisions, {rf.vectors} vectors, {rf.wall_s:.1f} s",
        "inspections_per_vector": rf.inspections / rf.vectors, "connected_fraction": rf.count / rf.vectors}
    out["c4_grad"] = {
        "value": rg.vectors / rg.wall_s / 1e9, "unit": "Gvec/s", "cores": rg.processes, "kind": "oracle",
        "sample": f"{kg} of {chig} divisions with all {c4.m} T1/T0 sums, {rg.vectors} vectors, "
                  f"{rg.wall_s:.1f} s",
        "inspections_per_vector": rg.inspections / rg.vectors}
    # the batched workload: the oracle handles one probability vector per
    # pass, so its rate in (vector, p-vector) pairs is its vector rate.
    # Graphs are drawn with probability proportional to their 2^m vectors
    # (systematic sampling on the cumulative count), so the mean of their
    # counters estimates the workload's mean per vector.
    import numpy as np
    nets, pvs = c3
    sizes = np.array([1 << g.m for g in nets], dtype=np.float64)
    cum = np.cumsum(sizes) / sizes.sum()
    picks = [int(np.searchsorted(cum, (j + 0.5) / 32)) for j in range(32)]
    from oracle import pbat
    jobs = []
    for j, gi in enumerate(picks):
        g = nets[gi]
        chi = 1 << min(10, g.m)
        for i in pbat.spread_divisions(chi, max(1, (1 << max(0, sample_log2 - 8)) >> (g.m - min(10, g.m)))):
            lo, hi = pbat.division_bounds(g.m, chi, i)
            jobs.append((g.n, g.arcs, pvs[gi][j % pvs[gi].shape[0]], g.s, g.t, lo, hi))
    res, wall = pbat.run_ranges(jobs, procs)
    vecs = sum(hi - lo for (*_, lo, hi) in jobs)
    insp = sum(r[2] for r in res)
    cnt = sum(r[1] for r in res)
    out["c3"] = {
        "value": vecs / wall / 1e9, "unit": "G(vector, p-vector) pairs/s", "cores": procs, "kind": "oracle",
        "sample": f"32 of {len(nets)} graphs drawn by size, spread divisions of each, one p-vector each, "
                  f"{vecs} vectors, {wall:.1f} s",
        "inspections_per_vector": insp / vecs, "connected_fraction": cnt / vecs}
    return out


def ms_cpu_baseline(net, sample_log2: int, procs: int):
    """The multi-state oracle on 256 equal ranges spread over the mixed-radix
    counter, about 2^sample_log2 vectors in all."""
    from oracle import pbat
    N = net.space
    per = max(1, (1 << sample_log2) // 256)
    starts = [int((j + 0.5) * N / 256) for j in range(256)]
    ranges = [(lo, min(N, lo + per)) for lo in starts]
    outs, wall = pbat.run_ms_ranges(net, ranges, procs)
    vecs = sum(hi - lo for lo, hi in ranges)
    return {"value": vecs / wall / 1e9, "unit": "Gvec/s", "cores": procs, "kind": "oracle",
            "sample": f"256 ranges of {per} vectors spread over the {N}-vector counter, {wall:.1f} s",
            "projected_time_to_R_s": N / (vecs / wall),
            "inspections_per_vector": sum(o[2] for o in outs) / vecs,
            "connected_fraction": sum(o[1] for o in outs) / vecs}


def roofline_alu(vectors: int, work_per_vector: float, kernel_s: float):
    """Integer-ALU roofline of a bit-sliced sweep: algorithmic bit-operations
    (the oracle's arc inspections per vector) per second against the bit-op
    peak."""
    ach = vectors * work_per_vector / kernel_s
    return {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_BIT_OPS / 1e12, "unit": "Tbitop/s",
            "frac": ach / PEAK_BIT_OPS, "work_per_vector": work_per_vector,
            "work_unit": "PLSA arc inspections (1 bit-op each)", "kernel_ms": kernel_s * 1e3}


def batched_only(pvec: int = 0):
    """The batched workload alone: tune, then time three launches (pvec > 0:
    only each graph's first pvec probability vectors)."""
    import numpy as np
    import torch

    import bat_workloads as W
    import paper_2209_09711_amd as B

    torch.cuda.set_device(0)
    nets, pvs = W.config3()
    if pvec > 0:
        pvs = [np.ascontiguousarray(pv[:pvec]) for pv in pvs]
    graphs = [(g.n, g.arc_array(), g.s, g.t) for g in nets]
    t0 = time.perf_counter()
    B.bat_autotune_batched(graphs, pvs)
    tune_s = time.perf_counter() - t0
    ks = []
    for _ in range(3):
        B.bat_reliability_batched(graphs, pvs)
        li = B.bat_last_launch()
        ks.append(li.kernel_ms)
    vec = sum(1 << g.m for g in nets)
    print(json.dumps({"workload": f"{len(nets)} random graphs x {pvs[0].shape[0]} p-vectors (seed 220909711/3)",
                      "state_vectors": vec, "batched_kernel_ms": float(np.min(ks)),
                      "batched_kernel_ms_all": ks, "specialised": bool(li.specialised),
                      "autotune_s": tune_s}), flush=True)


def main():
    a = parse()
    if a.copy_ref_gib > 0:
        copy_reference(a.copy_ref_gib)
        return
    if a.batched_only:
        batched_only(a.batched_pvec)
        return
    if a.multistate_only:
        import bat_workloads as W
        import paper_2209_09711_amd as B
        msn = W.config_ms()
        dem = a.ms_demand if a.ms_demand > 0 else msn.d

        def calls(k):
            ks = []
            for _ in range(k):
                R, c = B.bat_ms_reliability(msn.n, msn.arcs, msn.sigma, msn.cap, msn.w, msn.s, msn.t, dem)
                ks.append(B.bat_last_launch().kernel_ms)
            return R, c, ks
        R, c, _ = calls(1)
        first_jit_ms = B.bat_last_launch().jit_ms
        R, c, ks = calls(3)
        bits = bool(B.bat_last_launch().specialised)
        # the same sweep on the augmenting-path kernel
        old = B.bat_get_option("BAT_MS_BITS")
        B.bat_set_option("BAT_MS_BITS", 0)
        Rf, cf, kf = calls(2)
        B.bat_set_option("BAT_MS_BITS", old)
        print(json.dumps({"workload": msn.name, "demand": dem, "state_vectors": msn.space, "R": R, "count": c,
                          "kernel_ms_all": ks, "bit_sliced": bits, "first_call_jit_ms": first_jit_ms,
                          "flow_kernel_ms_all": kf, "flow_R": Rf, "flow_count": cf}), flush=True)
        return
    if a.valu_peak_only:
        import paper_2209_09711_amd as B
        print(json.dumps({"valu_peak_lane_ops_per_s": B.bat_valu_peak()}), flush=True)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the enumeration would shard "
              f"by counter ranges across GPUs, which this library does not launch.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import bat_workloads as W
    import paper_2209_09711_amd as B

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    net = W.config2()
    m = net.m
    nvec = 1 << m
    arcs = net.arc_array()

    # cold time-to-R: host call -> R on the host, first call (compiles the
    # graph-specialised kernel: the on-disk kernel cache points at a fresh
    # directory, so nothing compiled earlier is reused)
    import tempfile
    if a.jit_cache:
        os.makedirs(a.jit_cache, exist_ok=True)
        os.environ["BAT_JIT_CACHE_DIR"] = os.path.abspath(a.jit_cache)
    else:
        cache_tmp = tempfile.TemporaryDirectory(prefix="bat-bench-jit-")
        os.environ["BAT_JIT_CACHE_DIR"] = cache_tmp.name
    t0 = time.perf_counter()
    R_cold, cnt_cold = B.bat_reliability(net.n, arcs, net.p, net.s, net.t)
    cold_s = time.perf_counter() - t0
    info = B.bat_last_launch()
    jit_ms = info.jit_ms
    # the same first call in a later process: kernel loaded from the disk cache
    B.bat_set_option("BAT_JIT_FLUSH", 1)
    t0 = time.perf_counter()
    B.bat_reliability(net.n, arcs, net.p, net.s, net.t)
    cold_cached_s = time.perf_counter() - t0
    load_ms = B.bat_last_launch().jit_ms
    # autotune (one-time, reported separately): work-item size, convergence
    # test cadence, kernel kind and arc-to-bit order, timed on spread slices
    t0 = time.perf_counter()
    tune_ns = B.bat_autotune(net.n, arcs, net.p, net.s, net.t)
    tune_s = time.perf_counter() - t0
    R_cold, cnt_cold = B.bat_reliability(net.n, arcs, net.p, net.s, net.t)

    p_dev = torch.tensor(net.p, dtype=torch.float64, device=dev)
    R_dev = torch.zeros((), dtype=torch.float64, device=dev)
    c_dev = torch.zeros((), dtype=torch.int64, device=dev)
    st_dev = torch.zeros((), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def step():
        B.bat_reliability_async(net.n, arcs, p_dev.data_ptr(), net.s, net.t, R_dev.data_ptr(),
                                c_dev.data_ptr(), st_dev.data_ptr(), stream)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    kern_ms = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
        li_step = B.bat_last_launch()
        kern_ms.append(li_step.kernel_ms)   # HIP events on the launch stream
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    R = float(R_dev.item())
    count = int(c_dev.item())
    assert int(st_dev.item()) == 0
    assert count == cnt_cold and R == R_cold, "bench runs disagree"

    # warm time-to-R through the synchronous host entry point
    t0 = time.perf_counter()
    R_w, _ = B.bat_reliability(net.n, arcs, net.p, net.s, net.t)
    warm_s = time.perf_counter() - t0
    li = B.bat_last_launch()

    out = {
        "metric": "arc-state vectors/s (G/s) + time-to-exact-R at m=40; fwd+grad vs fwd",
        "value": nvec / (ms_per_step / 1e3) / 1e9,
        "unit": "Gvec/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 bit-sliced connectivity + f64 accumulation",
        "data": "synthetic",
        "config": {"workload": "5x5 grid, m=40 undirected arcs, corner to corner, p~U[0.85,0.99] "
                               "(seed 220909711/2), 2^40 state vectors, plain forward",
                   "vectors_per_step": nvec},
        "R": R,
        "R_hex": R.hex(),
        "launch": launch_key(li_step),
        "feasible_count": count,
        "time_to_exact_R_s": {"cold_incl_jit": cold_s, "warm": warm_s, "jit_compile_ms": jit_ms,
                              "cold_from_disk_cache": cold_cached_s, "jit_cache_load_ms": load_ms,
                              "autotune_s": tune_s, "autotune_ns_per_vector": tune_ns},
        "kernel_ms_mean": float(np.mean(kern_ms)),
        "specialised_kernel": bool(li.specialised),
        "relaxations_per_sweep": li.relaxations,
    }

    c4 = W.config4()
    c3 = W.config3()
    grad_c2_ms = None
    if not a.no_extras:
        # the same sweep with all 40 gradients (the autotuner tuned it too)
        B.bat_reliability_grad(net.n, arcs, net.p, net.s, net.t)
        g2 = []
        for _ in range(2):
            B.bat_reliability_grad(net.n, arcs, net.p, net.s, net.t)
            g2.append(B.bat_last_launch().kernel_ms)
        grad_c2_ms = min(g2)
        out["fwd_grad_vs_fwd_c2"] = {"workload": "5x5 grid, m=40, R + 40 gradients",
                                     "fwd_kernel_ms": float(np.mean(kern_ms)), "fwd_grad_kernel_ms": grad_c2_ms,
                                     "ratio": grad_c2_ms / float(np.mean(kern_ms)),
                                     "grad_launch": launch_key(B.bat_last_launch())}
        B.bat_autotune(c4.n, c4.arcs, c4.p, c4.s, c4.t)
        B.bat_reliability(c4.n, c4.arcs, c4.p, c4.s, c4.t)          # warm both kernels
        B.bat_reliability_grad(c4.n, c4.arcs, c4.p, c4.s, c4.t)
        fw, gr = [], []
        for _ in range(3):
            B.bat_reliability(c4.n, c4.arcs, c4.p, c4.s, c4.t)
            li_f = B.bat_last_launch()
            fw.append(li_f.kernel_ms)
            B.bat_reliability_grad(c4.n, c4.arcs, c4.p, c4.s, c4.t)
            li_g = B.bat_last_launch()
            gr.append(li_g.kernel_ms)
        out["fwd_grad_vs_fwd"] = {"workload": "random n=18 m=36 (seed 220909711/4), R + 36 gradients",
                                  "fwd_kernel_ms": min(fw), "fwd_grad_kernel_ms": min(gr),
                                  "ratio": min(gr) / min(fw),
                                  "fwd_launch": launch_key(li_f), "grad_launch": launch_key(li_g)}
    if not a.no_extras and not a.no_batched:
        # batched: one persistent launch vs the plain forward on every
        # (graph, probability vector) pair of the same workload
        nets, pvs = c3
        graphs = [(g.n, g.arc_array(), g.s, g.t) for g in nets]
        B.bat_reliability_batched(graphs, pvs)
        # autotune (one-time, reported separately): chain length and
        # segment size of the batched launch on this batch
        t0 = time.perf_counter()
        B.bat_autotune_batched(graphs, pvs)
        btune_s = time.perf_counter() - t0
        bks = []
        for _ in range(3):
            t0 = time.perf_counter()
            Rb, cb = B.bat_reliability_batched(graphs, pvs)
            bw = time.perf_counter() - t0
            bks.append(B.bat_last_launch().kernel_ms)
        bk = min(bks)
        t0 = time.perf_counter()
        pk = 0.0
        worst = 0.0
        for gi, (n_, a_, s_, t_) in enumerate(graphs):
            for j in range(pvs[gi].shape[0]):
                Rp, cp = B.bat_reliability(n_, a_, pvs[gi][j], s_, t_)
                pk += B.bat_last_launch().kernel_ms
                assert cp == cb[gi]
                worst = max(worst, abs(Rp - Rb[gi, j]) / Rp if Rp else abs(Rb[gi, j]))
        pw = time.perf_counter() - t0
        vec = sum(1 << g.m for g in nets)
        out["batched_vs_plain"] = {
            "workload": f"{len(nets)} random graphs, n 8-16, m 16-28 (seed 220909711/3), "
                        f"{pvs[0].shape[0]} p-vectors each, {vec} state vectors x {pvs[0].shape[0]}",
            "batched_wall_ms": bw * 1e3, "batched_kernel_ms": bk, "batched_autotune_s": btune_s,
            "plain_wall_ms": pw * 1e3, "plain_kernel_ms_sum": pk,
            "speedup_wall": pw / bw, "max_rel_diff": worst}

    msn = W.config_ms()
    ms_out = None
    if not a.no_extras:
        # multi-state arcs: three capacity levels per arc, demand 2
        B.bat_ms_reliability(msn.n, msn.arcs, msn.sigma, msn.cap, msn.w, msn.s, msn.t, msn.d)
        mks = []
        for _ in range(3):
            t0 = time.perf_counter()
            Rm, cm = B.bat_ms_reliability(msn.n, msn.arcs, msn.sigma, msn.cap, msn.w, msn.s, msn.t, msn.d)
            mw = time.perf_counter() - t0
            mks.append(B.bat_last_launch().kernel_ms)
        bits = bool(B.bat_last_launch().specialised)
        # the same sweep on the augmenting-path kernel, for comparison
        old_bits = B.bat_get_option("BAT_MS_BITS")
        B.bat_set_option("BAT_MS_BITS", 0)
        Rf, cf = B.bat_ms_reliability(msn.n, msn.arcs, msn.sigma, msn.cap, msn.w, msn.s, msn.t, msn.d)
        fk = B.bat_last_launch().kernel_ms
        # and the same graph at demand 3, on both kernels
        R3f, c3f = B.bat_ms_reliability(msn.n, msn.arcs, msn.sigma, msn.cap, msn.w, msn.s, msn.t, 3)
        fk3 = B.bat_last_launch().kernel_ms
        B.bat_set_option("BAT_MS_BITS", old_bits)
        assert cf == cm
        B.bat_ms_reliability(msn.n, msn.arcs, msn.sigma, msn.cap, msn.w, msn.s, msn.t, 3)
        k3 = []
        for _ in range(3):
            R3, c3_ = B.bat_ms_reliability(msn.n, msn.arcs, msn.sigma, msn.cap, msn.w, msn.s, msn.t, 3)
            k3.append(B.bat_last_launch().kernel_ms)
        assert c3_ == c3f
        ms_out = {"workload": f"random n={msn.n} m={msn.m} (seed 220909711/5), 3 capacity levels per arc, "
                              f"demand {msn.d}, {msn.space} state vectors",
                  "R": Rm, "count": cm, "kernel_ms": min(mks), "wall_ms": mw * 1e3,
                  "value": msn.space / (min(mks) / 1e3) / 1e9, "unit": "Gvec/s",
                  "bit_sliced": bits, "flow_kernel_ms": fk, "flow_R_rel_diff": abs(Rf - Rm) / Rm if Rm else 0.0,
                  "demand3": {"R": R3, "count": c3_, "kernel_ms": min(k3), "flow_kernel_ms": fk3,
                              "flow_R_rel_diff": abs(R3f - R3) / R3 if R3 else 0.0}}
        out["multistate"] = ms_out

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baselines(net, c4, c3, a.cpu_sample_log2)
        h = cpu["c2"]
        out["cpu_baseline"] = {k: h[k] for k in ("value", "unit", "cores", "kind", "sample",
                                                 "projected_time_to_R_s")}
        out["cpu_baseline"]["cpu_model"] = cpu["cpu_model"]
        out["cpu_baseline"]["cores_visible"] = cpu["cores_visible"]
        out["cpu_baseline"]["cores_cap"] = "the host cores a one-GPU job is given (16)"
        out["cpu_baseline_legs"] = {k: {kk: vv for kk, vv in cpu[k].items()
                                        if kk not in ("inspections_per_vector", "layers_per_vector",
                                                      "connected_fraction")}
                                    for k in ("c2_single_core", "c4", "c4_grad", "c3")}

    # rooflines: integer ALU bound (no HBM traffic per vector, no
    # contraction).  Algorithmic work per state vector = the layered
    # search's arc inspections (oracle-measured mean on each sample), one
    # bit-operation each.
    kern_s = float(np.mean(kern_ms)) / 1e3
    # the sustained integer VALU rate this device reaches on independent
    # add / xor chains (library diagnostic)
    lane_peak = B.bat_valu_peak()
    if cpu is not None:
        insp = cpu["c2"]["inspections_per_vector"]
        mk = MEASURED.get(launch_key(li_step), {})
        rl = roofline_alu(nvec, insp, kern_s)
        rl.update({"traffic": mk.get("traffic_bytes"), "valu_busy": mk.get("valu_busy"),
                   "valu_insts_per_vector": mk.get("valu_insts_per_vector"), "salu_busy": mk.get("salu_busy"),
                   "lds_busy": mk.get("lds_busy"), "launch": launch_key(li_step),
                   "valu_rate_measured": lane_peak,
                   "frac_of_measured_rate": nvec * insp / kern_s / (lane_peak * 32) if lane_peak > 0 else None})
        out["roofline"] = rl
        others = {}
        if "fwd_grad_vs_fwd" in out:
            f4 = out["fwd_grad_vs_fwd"]
            n4 = 1 << c4.m
            others["c4_fwd"] = roofline_alu(n4, cpu["c4"]["inspections_per_vector"], f4["fwd_kernel_ms"] / 1e3)
            others["c4_fwd_grad"] = roofline_alu(n4, cpu["c4"]["inspections_per_vector"],
                                                 f4["fwd_grad_kernel_ms"] / 1e3)
        if grad_c2_ms:
            others["c2_fwd_grad"] = roofline_alu(nvec, insp, grad_c2_ms / 1e3)
        if "batched_vs_plain" in out:
            bv = out["batched_vs_plain"]
            nvb = sum(1 << g.m for g in c3[0])
            # one connectivity verdict per vector serves all 32 p-vectors
            others["c3_batched"] = roofline_alu(nvb, cpu["c3"]["inspections_per_vector"],
                                                bv["batched_kernel_ms"] / 1e3)
        if ms_out is not None:
            mc = ms_cpu_baseline(msn, a.cpu_sample_log2 - 4, host_cpu()[2])
            out["cpu_baseline_legs"]["multistate"] = {k: v for k, v in mc.items()
                                                      if k not in ("inspections_per_vector", "connected_fraction")}
            # the work is the oracle's residual-edge looks in its
            # augmenting-path searches: one bit-op each when the kernel is
            # bit-sliced (demand <= 2: up to 32 vectors per 32-bit word),
            # one lane-op each when one lane decides one vector
            ach = msn.space * mc["inspections_per_vector"] / (ms_out["kernel_ms"] / 1e3)
            if ms_out["bit_sliced"]:
                others["multistate"] = {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_BIT_OPS / 1e12,
                                        "unit": "Tbitop/s", "frac": ach / PEAK_BIT_OPS,
                                        "work_per_vector": mc["inspections_per_vector"],
                                        "work_unit": "residual-edge looks of the augmenting-path searches "
                                                     "(1 bit-op each)", "kernel_ms": ms_out["kernel_ms"]}
            else:
                others["multistate"] = {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                                        "unit": "Tlaneop/s", "frac": ach / PEAK_LANE_OPS,
                                        "work_per_vector": mc["inspections_per_vector"],
                                        "work_unit": "residual-edge looks of the augmenting-path searches "
                                                     "(1 lane-op each)", "kernel_ms": ms_out["kernel_ms"]}
        out["rooflines_other"] = others
    line = json.dumps(out)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
