"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/lhfmm.h, and rejects bad arguments on the host before any
device work (negative status, thread-local message)."""
import ctypes as C
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_1201_5430_amd as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("liblhfmm.so not built")
    return L, L.load()


def test_exports_match_header():
    L, lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "lhfmm.h")).read()
    declared = set(re.findall(r"\b(lhf_[a-z_]+)\s*\(", hdr))
    assert declared == set(L.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.lhf_version().startswith(b"lhfmm")


def test_argument_validation_is_host_side():
    L, lib = _lib()
    h = C.c_void_p()
    dummy = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    cases = [
        (dict(p=12, depth=4), 0, 0.01, "n must be >= 1"),
        (dict(p=-1, depth=4), 10, 0.01, "p out of range"),
        (dict(p=25, depth=4), 10, 0.01, "p out of range"),
        (dict(p=17, depth=4, precision=L.FP32), 10, 0.01, "p out of range"),
        (dict(p=8, depth=1), 10, 0.01, "depth out of range"),
        (dict(p=8, depth=11), 10, 0.01, "depth out of range"),
        (dict(p=8, depth=3), 10, -1.0, "core radius"),
        (dict(p=8, depth=3), 10, float("nan"), "core radius"),
        (dict(p=8, depth=3, L=0.0), 10, 0.01, "domain_len"),
        (dict(p=8, depth=3, precision=7), 10, 0.01, "precision"),
        (dict(p=8, depth=3, tol=0.0), 10, 0.01, "tol"),
    ]
    for kw, n, a, msg in cases:
        d = L.make_desc(**kw)
        st = lib.lhf_plan_create(C.byref(h), C.byref(d), n, dummy, a, None)
        assert st == -1, (kw, st)
        assert h.value is None
        assert msg in lib.lhf_last_error().decode()
    d = L.make_desc(p=8, depth=3)
    assert lib.lhf_plan_create(C.byref(h), C.byref(d), 10, None, 0.01, None) == -1
    assert lib.lhf_plan_create(None, C.byref(d), 10, dummy, 0.01, None) == -1
    assert lib.lhf_execute(None, dummy, dummy, dummy, None, None) == -1
    assert lib.lhf_plan_destroy(None) == 0
    st = L.Stats()
    assert lib.lhf_plan_stats(None, C.byref(st)) == -1


def test_multi_system_and_batch_validation_is_host_side():
    import numpy as np
    L, lib = _lib()
    h = C.c_void_p()
    dummy = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    d = L.make_desc(p=8, depth=3)
    f64 = lambda a: np.ascontiguousarray(a, np.float64)
    i64 = lambda a: np.ascontiguousarray(a, np.int64)
    P = lambda a, t: a.ctypes.data_as(C.POINTER(t))
    lo, ln, a = f64([[0, 0, 0], [1, 1, 1]]), f64([1.0, 1.0]), f64([0.01, 0.01])
    cases = [
        (i64([1, 5, 9]), ln, a, "sys_offsets[0]"),
        (i64([0, 5, 3]), ln, a, "non-decreasing"),
        (i64([0, 0, 0]), ln, a, "n must be >= 1"),
        (i64([0, 5, 9]), f64([1.0, 0.0]), a, "cube sides"),
        (i64([0, 5, 9]), ln, f64([0.01, -1.0]), "core radius"),
    ]
    for off, lns, aa, msg in cases:
        st = lib.lhf_plan_create_multi(C.byref(h), C.byref(d), 2, P(off, C.c_int64), dummy, P(lo, C.c_double),
                                       P(lns, C.c_double), P(aa, C.c_double), None)
        assert st == -1 and h.value is None, (msg, st)
        assert msg in lib.lhf_last_error().decode()
        st = lib.lhf_batch_create(C.byref(h), C.byref(d), 2, P(off, C.c_int64), dummy, P(lo, C.c_double),
                                  P(lns, C.c_double), P(aa, C.c_double), None, None, None)
        assert st == -1 and h.value is None, (msg, st)
    off = i64([0, 5, 9])
    bad_depth = np.ascontiguousarray([3, 11], np.int32)
    st = lib.lhf_batch_create(C.byref(h), C.byref(d), 2, P(off, C.c_int64), dummy, P(lo, C.c_double),
                              P(ln, C.c_double), P(a, C.c_double), P(bad_depth, C.c_int32), None, None)
    assert st == -1 and "sys_depth" in lib.lhf_last_error().decode()
    assert lib.lhf_batch_execute(None, dummy, dummy, dummy, 1, None) == -1
    assert lib.lhf_batch_destroy(None) == 0
    assert lib.lhf_autotune(8, 7, None, None, None) == -1


def test_descriptor_options_are_checked_on_the_host():
    # new descriptor fields: unknown values are argument errors, valid requests that this
    # library cannot serve are LHF_ERR_UNSUPPORTED; both before any device work
    L, lib = _lib()
    h = C.c_void_p()
    dummy = C.c_void_p(0x1000)
    cases = [
        (dict(p=8, depth=3, flags=0x100), -1, "flag"),
        (dict(p=8, depth=3, translation=7), -1, "translation"),
        (dict(p=8, depth=3, translation=L.TRANS_DIRECT), -6, "LHF_TRANS_DIRECT"),
        (dict(p=8, depth=3, m2l_kernel=9), -1, "m2l_kernel"),
        (dict(p=8, depth=3, mm_kernel=-1), -1, "mm_kernel"),
        (dict(p=6, depth=3, m2l_kernel=L.M2L_HALF), -6, "no instantiation"),
        (dict(p=14, depth=3, m2l_kernel=L.M2L_MFMA), -6, "no instantiation"),
        (dict(p=16, depth=3, m2l_kernel=L.M2L_TILE), -6, "no instantiation"),
        (dict(p=6, depth=3, mm_kernel=L.MM_HALF), -6, "no instantiation"),
        (dict(p=12, depth=3, mm_kernel=L.MM_QUARTER), -6, "no instantiation"),
        (dict(p=16, depth=3, mm_kernel=L.MM_QUARTER, precision=L.FP32), -6, "no instantiation"),
        (dict(p=8, depth=3, mm_kernel=4), -1, "mm_kernel"),
        (dict(p=12, depth=9, m2l_kernel=L.M2L_HALF), -6, "depth <= 8"),
        (dict(p=12, depth=3, m2l_kernel=L.M2L_HALF, flags=L.LHF_DETERMINISTIC), -6, "not deterministic"),
        (dict(p=16, depth=3, m2l_kernel=L.M2L_HALF, flags=L.LHF_DETERMINISTIC), -6, "not deterministic"),
        (dict(p=14, depth=3, m2l_kernel=L.M2L_QUARTER), -6, "no instantiation"),
        (dict(p=16, depth=3, m2l_kernel=L.M2L_QUARTER, precision=L.FP32), -6, "no instantiation"),
        (dict(p=23, depth=3, m2l_kernel=L.M2L_QUARTER, flags=L.LHF_DETERMINISTIC), -6, "not deterministic"),
    ]
    for kw, code, msg in cases:
        d = L.make_desc(**kw)
        st = lib.lhf_plan_create(C.byref(h), C.byref(d), 10, dummy, 0.01, None)
        assert st == code and h.value is None, (kw, st)
        assert msg in lib.lhf_last_error().decode(), (kw, lib.lhf_last_error())
    d = L.make_desc(p=8, depth=3)
    d.reserved = 1
    assert lib.lhf_plan_create(C.byref(h), C.byref(d), 10, dummy, 0.01, None) == -1
    assert "reserved" in lib.lhf_last_error().decode()


def test_output_tensors_are_checked_on_the_host():
    # the binding refuses host tensors and wrong shapes before any pointer crosses the C ABI
    import torch
    L, _ = _lib()
    with pytest.raises(TypeError):
        L._dev_array(torch.zeros(5, 3, dtype=torch.float64), torch.float64, "v")
    with pytest.raises(TypeError):
        L._dev_array(np.zeros((5, 3)), torch.float64, "v")


def test_scalar_entry_point_checks_its_arguments():
    L, lib = _lib()
    assert lib.lhf_execute_scalar(None, C.c_void_p(0x1000), C.c_void_p(0x1000), None, None) == -1
    assert "plan" in lib.lhf_last_error().decode()


def test_filament_entry_points_check_their_arguments():
    L, lib = _lib()
    h = C.c_void_p()
    d = L.make_desc(p=8, depth=3, max_per_leaf=16)
    dummy = C.c_void_p(0x1000)
    assert lib.lhf_filament_create(C.byref(h), C.byref(d), 10, dummy, 5, dummy, None) == -6
    assert "uniform" in lib.lhf_last_error().decode() and h.value is None
    d = L.make_desc(p=8, depth=3)
    assert lib.lhf_filament_create(C.byref(h), C.byref(d), 1, dummy, 5, dummy, None) == -1
    assert lib.lhf_filament_execute(None, dummy, dummy, None) == -1
    assert lib.lhf_filament_destroy(None) == 0


def test_shape_entry_points_check_their_arguments():
    L, lib = _lib()
    sh = L.Shapes()
    assert lib.lhf_plan_set_shapes(None, C.byref(sh)) == -1
    assert lib.lhf_plan_get_shapes(None, C.byref(sh)) == -1
    assert lib.lhf_plan_autotune(None, None, None, C.byref(sh), None) == -1
    assert b"NULL" in lib.lhf_last_error()
