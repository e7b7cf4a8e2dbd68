"""Host-side checks of the C ABI that need no GPU.

The library must load, export every function declared in include/bat.h,
and reject bad arguments before touching the device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "bat.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bat_[a-z_]+)\s*\(", txt)))


def test_header_declarations_are_exported():
    import paper_2209_09711_amd as B
    lib = ctypes.CDLL(B.LIB_PATH)
    names = _declared()
    assert "bat_reliability" in names and "bat_reliability_grad" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTED) == names


def test_version_and_options():
    import paper_2209_09711_amd as B
    assert B.bat_version().startswith("bat-mi355x")
    old = B.bat_get_option("BAT_CHECK_EVERY")
    B.bat_set_option("BAT_CHECK_EVERY", 2)
    assert B.bat_get_option("BAT_CHECK_EVERY") == 2
    B.bat_set_option("BAT_CHECK_EVERY", old)
    with pytest.raises(B.BatError) as e:
        B.bat_set_option("NO_SUCH_OPTION", 1)
    assert e.value.code == B.BAT_EINVAL


@pytest.mark.parametrize("args,code", [
    ((1, [], [], 0, 0), -1),                       # n < 2
    ((3, [(0, 1)], [0.5], 1, 1), -1),              # s == t
    ((3, [(0, 1)], [0.5], 0, 3), -1),              # t out of range
    ((3, [(0, 5)], [0.5], 0, 2), -1),              # arc node out of range
    ((3, [(0, 1)], [1.5], 0, 2), -1),              # p > 1
    ((3, [(0, 1)], [-0.25], 0, 2), -1),            # p < 0
    ((3, [(0, 1)], [float("nan")], 0, 2), -1),     # NaN
    ((65, [(0, 1)], [0.5], 0, 2), -2),             # too many nodes
    ((3, [(0, 1)] * 63, [0.5] * 63, 0, 2), -2),    # too many arcs
])
def test_validation_without_device(args, code):
    import paper_2209_09711_amd as B
    with pytest.raises(B.BatError) as e:
        B.bat_reliability(*args)
    assert e.value.code == code
    assert B.bat_last_error() != ""
    with pytest.raises(B.BatError) as e:
        B.bat_reliability_grad(*args)
    assert e.value.code == code


def test_range_argument_checks():
    import paper_2209_09711_amd as B
    with pytest.raises(B.BatError) as e:
        B.bat_reliability_range(3, [(0, 1), (1, 2)], [0.5, 0.5], 0, 2, 3, 2)   # lo > hi
    assert e.value.code == B.BAT_EINVAL
    with pytest.raises(B.BatError) as e:
        B.bat_reliability_range(3, [(0, 1), (1, 2)], [0.5, 0.5], 0, 2, 0, 5)   # hi > 2^m
    assert e.value.code == B.BAT_EINVAL
    # an empty range needs no device work
    r = B.bat_reliability_range(3, [(0, 1), (1, 2)], [0.5, 0.5], 0, 2, 2, 2, grad=True)
    assert r.R == 0.0 and r.count == 0 and list(r.T1) == [0.0, 0.0]


def test_null_outputs_rejected():
    import paper_2209_09711_amd as B
    lib = ctypes.CDLL(B.LIB_PATH)
    lib.bat_reliability.restype = ctypes.c_int
    arcs = (B.bat_arc * 1)(B.bat_arc(0, 1))
    p = (ctypes.c_double * 1)(0.5)
    rc = lib.bat_reliability(2, 1, arcs, p, 0, 1, None, None)
    assert rc == B.BAT_EINVAL


def test_valu_peak_null_output():
    import paper_2209_09711_amd as B
    assert B._lib.bat_valu_peak(None) == B.BAT_EINVAL


def test_no_oracle_in_product_path():
    """The product package never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2209_09711_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h", ".inc")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "bat_oracle" not in txt and "libbat_oracle" not in txt, f


def _hipcc():
    import shutil
    return shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not installed")
@pytest.mark.parametrize("grad", [False, True])
def test_jit_sources_compile(tmp_path, grad):
    """The graph-specialised kernel sources compile for gfx950 (the same text
    hiprtc gets, plus the runtime header hiprtc provides by itself); graphs
    of up to 32 relevant nodes keep their reach words in registers inside
    the convergence loops."""
    import subprocess
    import bat_workloads as W
    import paper_2209_09711_amd as B
    loops = W.random_connected(10, 20, seed=91, p_lo=0.1, p_hi=0.9)
    loops.arcs = loops.arcs + [(0, 0), (3, 3)]
    # a 34-node cycle: more relevant nodes than the register-resident budget
    cycle = W.Network("cycle34", 34, [(i, (i + 1) % 34) for i in range(34)], 0, 17, np.full(34, 0.9))
    cases = [(W.config4(), 3, True, False), (W.config2(), 0, True, False), (loops, 1, True, False),
             (cycle, 2, False, False), (W.config4(), 3, True, True)]
    for k, (net, perm, small, directed) in enumerate(cases):
        src = B.bat_jit_source(net.n, net.arcs, net.s, net.t, grad=grad, perm=perm, directed=directed)
        assert ("DIR = true" in src) == directed
        assert "struct JitGraph" in src and ("bat_grad_jit" if grad else "bat_fwd_jit") in src
        f = tmp_path / f"k{k}.hip"
        f.write_text("#include <hip/hip_runtime.h>\n" + src)
        out = tmp_path / f"k{k}.s"
        r = subprocess.run([_hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                            "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", "-o", str(out), str(f)],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-2000:]
        asm = out.read_text()
        priv = [int(x) for x in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", asm)]
        spill = [int(x) for x in re.findall(r"\.vgpr_spill_count:\s+(\d+)", asm)]
        assert priv and spill
        if small:
            # Both builds ask the compiler for more wavefronts per SIMD than
            # its own register budget gives (gradient 3, forward 6), so both
            # may spill, but not inside the convergence loops: for the
            # gradient nothing below the block loop (depth >= 2), for the
            # forward at most a few reloads inside the sweeps of a chain
            # step (depth >= 3: block loop, chain steps, sweeps), against
            # some 700 instructions there.
            limit = 2 if grad else 3
            depth, inner, deepest = 0, [], 0
            for line in asm.splitlines():
                if re.match(r"^(\.LBB\d+_\d+:|; %bb\.\d+:)", line):  # every block start
                    mm = re.search(r"Depth=(\d+)", line)
                    depth = int(mm.group(1)) if mm else 0
                    deepest = max(deepest, depth)
                if "scratch_" in line and depth >= limit:
                    inner.append(line.strip())
            assert len(inner) <= (0 if grad else 4), (net.name, directed, inner[:4])
            if not grad:
                assert deepest == 3, (net.name, deepest)
    with pytest.raises(B.BatError):
        B.bat_jit_source(3, [(0, 1), (1, 2)], 0, 2, perm=9)


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not installed")
@pytest.mark.parametrize("npv,acc", [(1, 1), (8, 1), (9, 1), (16, 1), (16, 0), (17, 1), (32, 1), (32, 0)])
def test_batch_jit_sources_compile(tmp_path, npv, acc):
    """The graph-specialised batched sweep compiles for gfx950 for 1 to 32
    p-vectors: above 8 with the transposed accumulation (one accumulator
    per lane) in blocks of 16 wavefronts, or (option BAT_BATCH_ACC 0) with
    per-lane accumulators, 32 in blocks of 8 and up to 16 in blocks of 12;
    no scratch access inside the sweep loops."""
    import subprocess
    import bat_workloads as W
    import paper_2209_09711_amd as B
    nets, _ = W.config3(n_graphs=40, n_pvec=1)
    net = max(nets, key=lambda g: (g.m, g.n))
    old = B.bat_get_option("BAT_BATCH_ACC")
    try:
        B.bat_set_option("BAT_BATCH_ACC", acc)
        src = B.bat_jit_source(net.n, net.arcs, net.s, net.t, batch_pvec=npv)
    finally:
        B.bat_set_option("BAT_BATCH_ACC", old)
    transposed = acc == 1 and npv > 8
    assert "bat_batch_jit" in src and (f"LdsBatchT<{npv}>" if transposed else f"LdsBatch<{npv}>") in src
    waves = 16 if transposed else (8 if npv > 16 else 12)
    assert f"__launch_bounds__({64 * waves})" in src
    f = tmp_path / "b.hip"
    f.write_text("#include <hip/hip_runtime.h>\n" + src)
    out = tmp_path / "b.s"
    r = subprocess.run([_hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", "-o", str(out), str(f)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    asm = out.read_text()
    depth, inner = 0, []
    for line in asm.splitlines():
        if re.match(r"^(\.LBB\d+_\d+:|; %bb\.\d+:)", line):
            mm = re.search(r"Depth=(\d+)", line)
            depth = int(mm.group(1)) if mm else 0
        if "scratch_" in line and depth >= 2:
            inner.append(line.strip())
    assert not inner, inner[:4]
    with pytest.raises(B.BatError):
        B.bat_jit_source(net.n, net.arcs, net.s, net.t, batch_pvec=33)
    with pytest.raises(B.BatError):
        B.bat_jit_source(net.n, net.arcs, net.s, net.t, batch_pvec=4, directed=True)


def _loaded_hiprtc():
    """The hiprtc library file this process has mapped (the library's)."""
    import paper_2209_09711_amd  # noqa: F401  (loads the library and its hiprtc)
    with open("/proc/self/maps") as f:
        for line in f:
            path = line.split()[-1]
            if os.path.basename(path).startswith("libhiprtc.so"):
                return path
    return None


def test_jit_helper_matches_in_process_compile(tmp_path):
    """The compile helper the autotuner runs side by side (bat_jitc, built
    beside the library), given the hiprtc library this process uses, gives
    byte for byte the code object of an in-process compile of the same
    source with the same options, so a kernel's identity does not depend on
    where it was compiled; a bad source fails with exit status 1."""
    import subprocess
    import bat_workloads as W
    import paper_2209_09711_amd as B
    rtc = _loaded_hiprtc()
    assert rtc is not None
    helper = os.path.join(os.path.dirname(B.LIB_PATH), "bat_jitc")
    assert os.access(helper, os.X_OK)
    net = W.config0()
    src = B.bat_jit_source(net.n, net.arcs, net.s, net.t, perm=1)
    opts = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    (tmp_path / "k.hip").write_text(src)
    r = subprocess.run([helper, rtc, str(tmp_path / "k.hip"), str(tmp_path / "k.co"), *opts],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    via_helper = (tmp_path / "k.co").read_bytes()
    assert via_helper[:4] == b"\x7fELF"
    assert not (tmp_path / "k.co.part").exists()

    h = ctypes.CDLL(rtc)
    vp = ctypes.c_void_p
    h.hiprtcCreateProgram.argtypes = [ctypes.POINTER(vp), ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int, vp, vp]
    h.hiprtcCompileProgram.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p)]
    h.hiprtcGetCodeSize.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    h.hiprtcGetCode.argtypes = [vp, ctypes.c_char_p]
    h.hiprtcDestroyProgram.argtypes = [ctypes.POINTER(vp)]
    prog = vp()
    assert h.hiprtcCreateProgram(ctypes.byref(prog), src.encode(), b"bat_jit.hip", 0, None, None) == 0
    argv = (ctypes.c_char_p * len(opts))(*[o.encode() for o in opts])
    assert h.hiprtcCompileProgram(prog, len(opts), argv) == 0
    size = ctypes.c_size_t()
    assert h.hiprtcGetCodeSize(prog, ctypes.byref(size)) == 0
    buf = ctypes.create_string_buffer(size.value)
    assert h.hiprtcGetCode(prog, buf) == 0
    h.hiprtcDestroyProgram(ctypes.byref(prog))
    assert buf.raw == via_helper

    (tmp_path / "bad.hip").write_text(src + "\nthis is not C++;\n")
    r = subprocess.run([helper, rtc, str(tmp_path / "bad.hip"), str(tmp_path / "bad.co"), *opts],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and not (tmp_path / "bad.co").exists()
    r = subprocess.run([helper], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    r = subprocess.run([helper, str(tmp_path / "no_such_lib.so"), str(tmp_path / "k.hip"), str(tmp_path / "x.co")],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2


def test_flag_validation_without_device():
    """Unknown flag bits are rejected before any device work."""
    import paper_2209_09711_amd as B
    a = np.asarray([[0, 1], [1, 2]], dtype=np.int32)
    p = np.full(2, 0.5)
    R = ctypes.c_double(0.0)
    cnt = ctypes.c_uint64(0)
    rc = B._lib.bat_reliability_ex(3, 2, B._ptr(a), B._ptr(p), 0, 2, 8, ctypes.byref(R), ctypes.byref(cnt),
                                   None, None, None)
    assert rc == -1 and "flags" in B.bat_last_error()
    hi = ctypes.c_double(0.0)
    lo = ctypes.c_double(0.0)
    rc = B._lib.bat_reliability_range_ex(3, 2, B._ptr(a), B._ptr(p), 0, 2, 4, 0, 4, ctypes.byref(hi),
                                         ctypes.byref(lo), ctypes.byref(cnt), None, None)
    assert rc == -1 and "flags" in B.bat_last_error()
    assert B.BAT_DIRECTED == 1 and B.BAT_FORWARD_ORDER == 2


def test_header_is_plain_c(tmp_path):
    """include/bat.h is a C header: a C99 translation unit that includes it
    and takes the address of every declared function compiles warning-free."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    names = _declared()
    src = ["#include \"bat.h\"", "#include <stddef.h>", "typedef void (*fp)(void);", "fp table[] = {"]
    src += [f"    (fp){n}," for n in names]
    src += ["};", "size_t n_table = sizeof table / sizeof table[0];",
            "int check(void) { bat_arc a = {0, 1}; return a.u + a.v + BAT_OK + BAT_EINVAL + BAT_ETOOBIG"
            " + BAT_EDEVICE + BAT_ENOMEM + BAT_EIO + BAT_PENDING + BAT_MAX_NODES + BAT_MAX_ARCS + BAT_MAX_PVEC + (int)BAT_DIRECTED"
            " + (int)BAT_FORWARD_ORDER; }"]
    f = tmp_path / "abi.c"
    f.write_text("\n".join(src) + "\n")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror",
                        "-I", os.path.join(ROOT, "include"), "-c", str(f), "-o", str(tmp_path / "abi.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.mark.parametrize("kw,code", [
    (dict(demand=0), -1),                                    # demand below 1
    (dict(demand=1025), -1),                                 # demand above the limit
    (dict(n_states=[2, 0]), -1),                             # an arc with no state
    (dict(n_states=[2, 33]), -1),                            # too many states for one arc
    (dict(capacity=[[0, 1], [0, -1]]), -1),                  # negative capacity
    (dict(w=[[0.5, 0.5], [1.5, -0.5]]), -1),                 # probability outside [0, 1]
    (dict(w=[[0.5, 0.5], [float("nan"), 0.5]]), -1),         # NaN
    (dict(s=1, t=1), -1),                                    # s == t
    (dict(n=33), -2),                                        # more nodes than the flow test's masks
])
def test_multistate_validation_without_device(kw, code):
    import paper_2209_09711_amd as B
    args = dict(n=3, arcs=[(0, 1), (1, 2)], n_states=[2, 2], capacity=[[0, 1], [0, 1]], w=[[0.5, 0.5], [0.5, 0.5]],
                s=0, t=2, demand=1)
    args.update(kw)
    if "n_states" in kw and "capacity" not in kw:
        args["capacity"] = None
        args["w"] = [[0.5] * max(k, 0) for k in kw["n_states"]]
    with pytest.raises(B.BatError) as e:
        B.bat_ms_reliability(args["n"], args["arcs"], args["n_states"], args["capacity"], args["w"], args["s"],
                             args["t"], args["demand"])
    assert e.value.code == code
    assert B.bat_last_error() != ""


def test_multistate_size_limits_without_device():
    import paper_2209_09711_amd as B
    with pytest.raises(B.BatError) as e:                     # 33 arcs
        B.bat_ms_reliability(3, [(0, 1)] * 33, [1] * 33, None, [[1.0]] * 33, 0, 2, 1)
    assert e.value.code == B.BAT_ETOOBIG
    with pytest.raises(B.BatError) as e:                     # 32^13 > 2^62 vectors
        B.bat_ms_reliability(3, [(0, 1)] * 13, [32] * 13, None, [[1 / 32] * 32] * 13, 0, 2, 1)
    assert e.value.code == B.BAT_ETOOBIG
    with pytest.raises(B.BatError) as e:                     # a range past the end of the space
        B.bat_ms_reliability_range(3, [(0, 1), (1, 2)], [2, 3], None, [[0.5, 0.5], [0.2, 0.3, 0.5]], 0, 2, 1, 0, 7)
    assert e.value.code == B.BAT_EINVAL
    with pytest.raises(B.BatError) as e:                     # unknown flag bits via a bad n_states length
        B.bat_ms_reliability(3, [(0, 1), (1, 2)], [2], None, [[0.5, 0.5]], 0, 2, 1)
    assert e.value.code == B.BAT_EINVAL
