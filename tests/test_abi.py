"""The C ABI without a GPU: libcse.so loads, exports every entry point include/cse.h
declares, and rejects invalid arguments with CSE_EINVAL before touching the device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cse.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cse_[a-z_]+)\s*\(", src)))


def test_header_declarations_exported():
    import paper_2212_10042_amd as cse
    decl = _declared()
    assert "cse_simulate" in decl and "cse_validate" in decl and "cse_calibrate" in decl and "cse_bound" in decl
    out = subprocess.run(["nm", "-D", "--defined-only", cse.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (cse_\w+)", out))
    assert set(decl) <= exported, set(decl) - exported
    for fn in decl:
        assert hasattr(cse.lib(), fn)
    assert set(cse.EXPORTED) == set(decl)


def test_noalloc_workspace_size_matches_header():
    import paper_2212_10042_amd as cse
    src = open(os.path.join(ROOT, "include", "cse.h")).read()
    m = re.search(r"#define CSE_NOALLOC_SCRATCH_BYTES \(\(int64_t\)(\d+) << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == cse.NOALLOC_SCRATCH_BYTES


def test_header_compiles_as_c():
    src = "#include \"cse.h\"\nint main(void){cse_design d={0};(void)d;return 0;}\n"
    r = subprocess.run(["gcc", "-x", "c", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        "-fsyntax-only", "-"], input=src, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def _create(design, theta, radii, sims, flags=0):
    import paper_2212_10042_amd as cse
    h = ctypes.c_void_p()
    th = np.ascontiguousarray(theta, np.float64)
    rd = np.ascontiguousarray(radii, np.float64)
    sm = np.ascontiguousarray(sims, np.int32)
    st = cse.lib().cse_platten_create(ctypes.byref(design), th.shape[0] if th.ndim else 0, cse._ptr(th),
                                      cse._ptr(rd), cse._ptr(sm), flags, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("case", ["zero_boxes", "bad_kind", "bad_arms", "bad_sims", "bad_radius",
                                  "bad_flag", "keep_all_multi", "reserved"])
def test_invalid_arguments_rejected(case):
    import paper_2212_10042_amd as cse
    des = cse.make_design("binom2")
    th = np.array([[0.0, -0.5]])
    rd = np.array([[0.1, 0.1]])
    sm = np.array([100], np.int32)
    flags = 0
    if case == "zero_boxes":
        th = np.zeros((0, 2))
    elif case == "bad_kind":
        des.kind = 99
    elif case == "bad_arms":
        des.n_arms = 3
    elif case == "bad_sims":
        sm = np.array([0], np.int32)
    elif case == "bad_radius":
        rd = np.array([[0.1, -0.1]])
    elif case == "bad_flag":
        flags = 8
    elif case == "keep_all_multi":
        des = cse.make_design("hier4")
        th = np.zeros((1, 4))
        rd = np.full((1, 4), 0.1)
        flags = cse.CSE_PLATTEN_KEEP_ALL
    elif case == "reserved":
        des.reserved = 1
    st, h = _create(des, th, rd, sm, flags)
    assert st in (cse.CSE_EINVAL, cse.CSE_EUNSUPPORTED)
    assert not h.value
    assert len(cse.lib().cse_last_error()) > 0


def test_null_handles_rejected():
    import paper_2212_10042_amd as cse
    L = cse.lib()
    assert L.cse_platten_size(None) < 0
    assert L.cse_platten_destroy(None) == cse.CSE_OK
    assert L.cse_simulate(None, 0, None, None, None, None, None) == cse.CSE_EINVAL
    assert L.cse_bound(None, 0, None, None, 0.01, None, None, None) == cse.CSE_EINVAL


def test_null_handles_rejected_newer_entry_points():
    import paper_2212_10042_amd as cse
    L = cse.lib()
    assert L.cse_validate_lower(None, None, 0.01, None, None, None, None) == cse.CSE_EINVAL
    assert L.cse_confidence_set(None, None, 0, None, None, 0, None, None, None, None, None) == cse.CSE_EINVAL
    assert L.cse_calibrate_tiebreak(None, 0, 0.025, None, None, None, None, None, None, None, None) == cse.CSE_EINVAL
    assert L.cse_calibrate_noalloc(None, 0, 0.025, None, None, None, None, None, 0.01, None, None, None, None, None,
                                   None, None) == cse.CSE_EINVAL
    assert L.cse_taylor(None, None, None, None, None, None, None) == cse.CSE_EINVAL
    assert L.cse_platten_tiles(None, None, None) == cse.CSE_EINVAL
    assert L.cse_adagrid_decide(None, 0, None, None, 0, None, None, None, None, None) == cse.CSE_EINVAL
    assert L.cse_platten_set_option(None, cse.CSE_OPT_B2_MARGIN, 3.0) == cse.CSE_EINVAL
    assert L.cse_work_counters(None, None, None) == cse.CSE_EINVAL


@pytest.mark.parametrize("case", ["basket_theta0_nan", "basket_n_per_arm", "sims_too_many"])
def test_invalid_basket_and_size_arguments(case):
    import paper_2212_10042_amd as cse
    th = np.array([[-1.8, -1.6, -2.0, -1.7]])
    rd = np.full((1, 4), 0.1)
    sm = np.array([100], np.int32)
    des = cse.make_design("basket4")
    if case == "basket_theta0_nan":
        des.theta0[2] = float("nan")
    elif case == "basket_n_per_arm":
        des.n_per_arm = 36
    else:
        sm = np.array([(1 << 24) + 1], np.int32)
    st, h = _create(des, th, rd, sm)
    assert st in (cse.CSE_EINVAL, cse.CSE_EUNSUPPORTED)
    assert not h.value
