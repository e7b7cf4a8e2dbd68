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


def test_no_oracle_in_product_path():
    """The product package never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2209_09711_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h", ".inc")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "bat_oracle" not in txt and "libbat_oracle" not in txt, f
