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

# MI355X: 256 CUs, 64 lanes each, 2.4 GHz peak engine clock; one int32
# lane-op per lane per clock on the vector ALUs.  A bit-sliced lane-op
# handles 32 state vectors, so the bit-operation peak is 32x the lane rate.
CUS, LANES, CLOCK_HZ = 256, 64, 2.4e9
PEAK_LANE_OPS = CUS * LANES * CLOCK_HZ            # 3.93e13 int32 lane-ops/s
PEAK_BIT_OPS = PEAK_LANE_OPS * 32                 # 1.26e15 bit-ops/s

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
    ap.add_argument("--cpu-sample-log2", type=int, default=30,
                    help="log2 of the state vectors in the oracle's timed sample")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
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


def cpu_baseline(net, sample_log2: int):
    """The CPU oracle (PBAT equal divisions over the host cores) on an evenly
    spread sample of Eq. 6 divisions of the same workload."""
    from oracle import pbat
    procs = int(os.environ.get("BAT_BENCH_CPU_PROCS", "0")) or min(os.cpu_count() or 1, 16)
    chi = 1 << 17                                  # divisions of 2^23 vectors at m = 40
    mu_log2 = net.m - 17
    k = max(1, 1 << max(0, sample_log2 - mu_log2))
    divs = pbat.spread_divisions(chi, k)
    r = pbat.run(net.n, net.arcs, net.p, net.s, net.t, chi, divisions=divs, processes=procs)
    return {
        "value": r.vectors / r.wall_s / 1e9,
        "unit": "Gvec/s",
        "cores": r.processes,
        "kind": "oracle",
        "sample": f"{len(divs)} of {chi} equal divisions (Eq. 6) spread evenly over the 2^{net.m} "
                  f"counter, {r.vectors} vectors, {r.wall_s:.1f} s wall on {r.processes} processes",
        "inspections_per_vector": r.inspections / r.vectors,
        "layers_per_vector": r.layers / r.vectors,
        "projected_time_to_R_s": (1 << net.m) / (r.vectors / r.wall_s),
    }


def batched_only():
    """The batched workload alone: tune, then time three launches."""
    import numpy as np
    import torch

    import bat_workloads as W
    import paper_2209_09711_amd as B

    torch.cuda.set_device(0)
    nets, pvs = W.config3()
    graphs = [(g.n, g.arc_array(), g.s, g.t) for g in nets]
    B.bat_autotune_batched(graphs, pvs)
    ks = []
    for _ in range(3):
        B.bat_reliability_batched(graphs, pvs)
        ks.append(B.bat_last_launch().kernel_ms)
    vec = sum(1 << g.m for g in nets)
    print(json.dumps({"workload": f"{len(nets)} random graphs x {pvs[0].shape[0]} p-vectors (seed 220909711/3)",
                      "state_vectors": vec, "batched_kernel_ms": float(np.min(ks)),
                      "batched_kernel_ms_all": ks}), flush=True)


def main():
    a = parse()
    if a.copy_ref_gib > 0:
        copy_reference(a.copy_ref_gib)
        return
    if a.batched_only:
        batched_only()
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

    if not a.no_extras:
        c4 = W.config4()
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
        nets, pvs = W.config3()
        graphs = [(g.n, g.arc_array(), g.s, g.t) for g in nets]
        B.bat_reliability_batched(graphs, pvs)
        # autotune (one-time, reported separately): chain length and
        # segment size of the batched launch on this batch
        t0 = time.perf_counter()
        B.bat_autotune_batched(graphs, pvs)
        btune_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        Rb, cb = B.bat_reliability_batched(graphs, pvs)
        bw = time.perf_counter() - t0
        bk = B.bat_last_launch().kernel_ms
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

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(net, a.cpu_sample_log2)
        out["cpu_baseline"] = {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["projected_time_to_R_s"] = cpu["projected_time_to_R_s"]

    # roofline of the enumeration kernel: integer ALU bound (no HBM traffic
    # per vector, no contraction).  Algorithmic work per state vector = the
    # layered search's arc inspections (oracle-measured mean on the sample),
    # one bit-operation each.
    kern_s = float(np.mean(kern_ms)) / 1e3
    insp = cpu["inspections_per_vector"] if cpu else None
    # the sustained integer VALU rate this device reaches on independent
    # add / xor chains (library diagnostic), as a second peak
    lane_peak = B.bat_valu_peak()
    if insp is not None:
        achieved = nvec * insp / kern_s
        out["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_BIT_OPS / 1e12,
                           "unit": "Tbitop/s", "frac": achieved / PEAK_BIT_OPS,
                           "traffic": MEASURED.get(launch_key(li_step), {}).get("traffic_bytes"),
                           "valu_busy": MEASURED.get(launch_key(li_step), {}).get("valu_busy"),
                           "valu_insts_per_vector": MEASURED.get(launch_key(li_step), {}).get("valu_insts_per_vector"),
                           "salu_busy": MEASURED.get(launch_key(li_step), {}).get("salu_busy"),
                           "lds_busy": MEASURED.get(launch_key(li_step), {}).get("lds_busy"),
                           "launch": launch_key(li_step),
                           "peak_measured": lane_peak * 32 / 1e12,
                           "frac_measured": achieved / (lane_peak * 32) if lane_peak > 0 else None,
                           "work_per_vector": insp, "work_unit": "PLSA arc inspections (1 bit-op each)"}
    line = json.dumps(out)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
