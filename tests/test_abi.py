"""The C-ABI library loads and exports every symbol the header declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2511_13894_amd import pdhg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(pdhg_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("pdhg_create", "pdhg_solve", "pdhg_corner_push", "pdhg_kkt", "pdhg_destroy", "pdhg_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol():
    if not pdhg.LIB_PATH.exists():
        pytest.fail("libpdhg.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(str(pdhg.LIB_PATH))
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(pdhg.EXPORTS) <= set(_declared())


def test_struct_layouts_match_binding():
    lib = pdhg.load()
    assert lib.pdhg_struct_size(0) == ctypes.sizeof(pdhg.Params)
    assert lib.pdhg_struct_size(1) == ctypes.sizeof(pdhg.Result)
    assert lib.pdhg_struct_size(2) == ctypes.sizeof(pdhg.KKTReport)
    assert lib.pdhg_struct_size(3) == ctypes.sizeof(pdhg.PushResult)
    assert lib.pdhg_struct_size(7) == ctypes.sizeof(pdhg.DualPushResult)
    assert lib.pdhg_struct_size(99) == -1


def test_default_params_and_argument_errors_without_gpu():
    """Defaults, and argument checks that fail before any device call."""
    lib = pdhg.load()
    p = pdhg.default_params()
    assert p.eps_rel == 1e-6 and p.check_every == 64 and p.ruiz_iters == 10 and p.power_iters == 4000 and p.power_tol == 1e-3
    assert p.push_compact == 1 and p.record_history == 0
    assert p.push_gate == 0 and p.push_gate_rows == 2.0 and p.push_gate_min == 100000
    assert p.halpern == 1 and p.reflect_gamma == 1.0 and p.push_min_iters == 100
    h = ctypes.c_void_p()
    rp = (ctypes.c_int64 * 2)(0, 1)
    ci = (ctypes.c_int32 * 1)(5)  # column out of range for n = 2
    va = (ctypes.c_double * 1)(1.0)
    b = (ctypes.c_double * 1)(1.0)
    c = (ctypes.c_double * 2)(1.0, 1.0)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.pdhg_create(1, 2, 1, rp, ci, ctypes.cast(va, dp), ctypes.cast(b, dp), ctypes.cast(c, dp), None, None,
                         None, ctypes.byref(p), ctypes.byref(h))
    assert rc == -1 and b"column" in lib.pdhg_last_error()
    ci[0] = 0
    c[1] = float("nan")
    rc = lib.pdhg_create(1, 2, 1, rp, ci, ctypes.cast(va, dp), ctypes.cast(b, dp), ctypes.cast(c, dp), None, None,
                         None, ctypes.byref(p), ctypes.byref(h))
    assert rc == -1 and b"c" in lib.pdhg_last_error()
    c[1] = 1.0
    # the largest model: indices are 32-bit, so nnz >= 2^31 is refused before any array is read
    rc = lib.pdhg_create(1, 2, 1 << 31, rp, ci, ctypes.cast(va, dp), ctypes.cast(b, dp), ctypes.cast(c, dp), None,
                         None, None, ctypes.byref(p), ctypes.byref(h))
    assert rc == -1 and b"2^31" in lib.pdhg_last_error()
    for field, bad in (("push_gate_rows", -1.0), ("push_gate_min", -5), ("push_gate_rows", float("nan"))):
        q = pdhg.default_params()
        setattr(q, field, bad)
        rc = lib.pdhg_create(1, 2, 1, rp, ci, ctypes.cast(va, dp), ctypes.cast(b, dp), ctypes.cast(c, dp), None,
                             None, None, ctypes.byref(q), ctypes.byref(h))
        assert rc == -1 and b"invalid parameter" in lib.pdhg_last_error(), field
    assert lib.pdhg_solve(None, None) == -1
    assert lib.pdhg_kkt(None, None, None, None) == -1
    lib.pdhg_destroy(None)


def test_numeric_parameters_are_validated_without_gpu():
    """Non-finite or out-of-range tolerances, factors and caps are refused
    at create, before any device call: a NaN eps_abs would make every fixing
    test false, a negative push scale would flip the push objective."""
    lib = pdhg.load()
    h = ctypes.c_void_p()
    rp = (ctypes.c_int64 * 2)(0, 1)
    ci = (ctypes.c_int32 * 1)(0)
    va = (ctypes.c_double * 1)(1.0)
    b = (ctypes.c_double * 1)(1.0)
    c = (ctypes.c_double * 2)(1.0, 1.0)
    dp = ctypes.POINTER(ctypes.c_double)
    nan, inf = float("nan"), float("inf")
    bad = [("eps_abs", nan), ("eps_abs", -1e-6), ("eps_abs", inf), ("eps_rel", nan), ("eps_rel", inf),
           ("push_obj_scale", -1.0), ("push_obj_scale", 0.0), ("push_obj_scale", nan), ("push_max_iter", -1),
           ("max_iter", -1), ("reflect_gamma", 1.5), ("reflect_gamma", -0.1), ("reflect_gamma", nan),
           ("pw_smooth", nan), ("pw_smooth", 2.0), ("restart_suff", nan), ("restart_nec", 1.5),
           ("restart_art", -0.1), ("restart_art", nan), ("pc_alpha", nan), ("time_limit", nan),
           ("eta_safety", inf), ("halpern", 2)]
    for field, value in bad:
        q = pdhg.default_params()
        setattr(q, field, value)
        rc = lib.pdhg_create(1, 2, 1, rp, ci, ctypes.cast(va, dp), ctypes.cast(b, dp), ctypes.cast(c, dp), None,
                             None, None, ctypes.byref(q), ctypes.byref(h))
        assert rc == -1, (field, value)
        assert lib.pdhg_last_error(), field
    lg = (ctypes.c_float * 2)(0.0, 0.0)
    assert lib.pdhg_corner_push_logits(None, lg, 0.5, 1, None) == -1
    assert lib.pdhg_batch_corner_push_logits(None, lg, 0.5, None, None) == -1


def test_kernel_codes_are_validated_without_gpu():
    """The dual-half-only kernel codes (sliced ELLPACK -3032, row segments
    -4000) and anything outside the encoding are refused for the primal half,
    and the batch (tiled kernels only) refuses both, before any device call."""
    lib = pdhg.load()
    h = ctypes.c_void_p()
    rp = (ctypes.c_int64 * 2)(0, 1)
    ci = (ctypes.c_int32 * 1)(0)
    va = (ctypes.c_double * 1)(1.0)
    b = (ctypes.c_double * 1)(1.0)
    c = (ctypes.c_double * 2)(1.0, 1.0)
    dp = ctypes.POINTER(ctypes.c_double)
    for field, value in (("lanes_at", -4000), ("lanes_at", -3032), ("lanes_a", 3), ("lanes_a", -4001),
                         ("lanes_at", 128)):
        q = pdhg.default_params()
        setattr(q, field, value)
        rc = lib.pdhg_create(1, 2, 1, rp, ci, ctypes.cast(va, dp), ctypes.cast(b, dp), ctypes.cast(c, dp), None,
                             None, None, ctypes.byref(q), ctypes.byref(h))
        assert rc == -1 and b"lanes" in lib.pdhg_last_error(), (field, value)
    descs = (pdhg.LpDesc * 1)()
    descs[0].m, descs[0].n, descs[0].nnz = 2, 3, 4
    for value in (-4000, -3032):
        q = pdhg.default_params()
        q.lanes_a = value
        assert lib.pdhg_batch_create_device(1, descs, ctypes.byref(q), ctypes.byref(h)) == -1
        assert b"tiled kernels only" in lib.pdhg_last_error(), value


def test_batch_create_device_argument_errors_without_gpu():
    """pdhg_batch_create_device refuses bad counts, NULL arrays, lane
    choices outside the tiled kernels and invalid parameters before it
    touches the device or any LP array."""
    lib = pdhg.load()
    p = pdhg.default_params()
    h = ctypes.c_void_p()
    descs = (pdhg.LpDesc * 1)()
    assert lib.pdhg_batch_create_device(0, descs, ctypes.byref(p), ctypes.byref(h)) == -1
    assert lib.pdhg_batch_create_device(70000, descs, ctypes.byref(p), ctypes.byref(h)) == -1
    assert b"65535" in lib.pdhg_last_error()
    assert lib.pdhg_batch_create_device(1, descs, ctypes.byref(p), None) == -1
    descs[0].m, descs[0].n, descs[0].nnz = 2, 3, 4  # NULL arrays
    assert lib.pdhg_batch_create_device(1, descs, ctypes.byref(p), ctypes.byref(h)) == -1
    assert b"NULL" in lib.pdhg_last_error()
    q = pdhg.default_params()
    q.lanes_a = 8  # a lane-group kernel: the batch runs tiles only
    assert lib.pdhg_batch_create_device(1, descs, ctypes.byref(q), ctypes.byref(h)) == -1
    q = pdhg.default_params()
    q.eps_rel = float("nan")
    assert lib.pdhg_batch_create_device(1, descs, ctypes.byref(q), ctypes.byref(h)) == -1
    assert b"invalid parameter" in lib.pdhg_last_error()
