"""Warm start, checkpoint/resume and the device-pointer solution accessor."""
import ctypes as C

import numpy as np
import pytest

from paper_2511_13894_amd import lpgen, pdhg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_checkpoint_resume_continues_bitwise(prec):
    """Also in the mixed mode, whose anchored data a resumed handle rebuilds
    from the restored anchor with the same products the restart used."""
    lp = lpgen.config1(seed=5, m=800, n=3200)
    a = pdhg.Solver(lp, eps_rel=1e-7, precision=prec)
    a.iterate(100)
    state = a.get_state()
    a.iterate(150)
    xa, ya = a.get_iterate()
    b = pdhg.Solver(lp, eps_rel=1e-7, precision=prec)
    b.set_state(state)
    b.iterate(150)
    xb, yb = b.get_iterate()
    np.testing.assert_array_equal(xa, xb)
    np.testing.assert_array_equal(ya, yb)
    ra, rb = a.solve(), b.solve()
    print(f"[state] {prec} resumed solve: {rb.iters} iterations (uninterrupted {ra.iters})", flush=True)
    assert (ra.status, ra.iters, ra.restarts) == (rb.status, rb.iters, rb.restarts)
    assert ra.pobj == rb.pobj
    pa, pb = a.corner_push(3), b.corner_push(3)
    assert (pa.iters, pa.after.p_off) == (pb.iters, pb.after.p_off)


def test_checkpoint_errors():
    lp = lpgen.config0(1)
    a = pdhg.Solver(lp)
    a.iterate(10)
    state = a.get_state()
    with pytest.raises(pdhg.PdhgError):
        pdhg.Solver(lpgen.tiny(3)).set_state(state)
    with pytest.raises(pdhg.PdhgError):
        a.set_state(b"not a checkpoint" * 8)
    f32 = pdhg.Solver(lp, precision="fp32")
    with pytest.raises(pdhg.PdhgError):
        f32.set_state(state)
    a.solve()
    a.corner_push(1)
    with pytest.raises(pdhg.PdhgError):
        a.get_state()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_warm_start_from_an_optimal_point_stops_at_the_first_check(prec):
    """Also in the mixed mode, where the start point becomes the float64
    anchor with a zero stored difference."""
    lp = lpgen.config0(4)
    a = pdhg.Solver(lp, eps_rel=1e-8)
    ra = a.solve()
    x, y, _ = a.get_solution()
    b = pdhg.Solver(lp, eps_rel=1e-6, precision=prec)
    b.set_start(x, y)
    rb = b.solve()
    print(f"[state] cold solve {ra.iters} iterations; {prec} warm start from its answer {rb.iters}", flush=True)
    assert rb.status == pdhg.PDHG_OPTIMAL and rb.iters <= 128 < ra.iters
    bad = x.copy()
    bad[0] = np.nan
    with pytest.raises(pdhg.PdhgError):
        b.set_start(bad, y)


def test_solution_into_device_buffers():
    lp = lpgen.config0(5)
    s = pdhg.Solver(lp)
    s.solve()
    x, y, z = s.get_solution()
    # the HIP runtime the library itself loaded (the same file, hence the same runtime instance)
    path = next(line.split()[-1] for line in open("/proc/self/maps") if "libamdhip64.so" in line)
    hip = C.CDLL(path)
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipDeviceSynchronize.argtypes = []
    hip.hipFree.argtypes = [C.c_void_p]
    bufs = []
    for k in (lp.n, lp.m, lp.n):
        p = C.c_void_p()
        assert hip.hipMalloc(C.byref(p), 8 * k) == 0
        bufs.append(p)
    try:
        assert s.lib.pdhg_get_solution_device(s.h, bufs[0], bufs[1], bufs[2], None) == 0
        assert hip.hipDeviceSynchronize() == 0
        got = []
        for p, k in zip(bufs, (lp.n, lp.m, lp.n)):
            h = np.zeros(k)
            assert hip.hipMemcpy(h.ctypes.data_as(C.c_void_p), p, 8 * k, 2) == 0  # device to host
            got.append(h)
        for a, b in zip(got, (x, y, z)):
            np.testing.assert_array_equal(a, b)
    finally:
        for p in bufs:
            hip.hipFree(p)


def test_create_from_device_memory_equals_host_create():
    """pdhg_create_device on the same (row-sorted) LP gives the same solve and
    push, bit for bit, as pdhg_create; invalid device models are refused by
    the device's own checks."""
    import copy

    for prec in ("fp64", "fp32"):
        lp = lpgen.config1(seed=3, m=300, n=1200)
        a = pdhg.Solver(lp, precision=prec, eps_rel=1e-6)
        d = pdhg.DeviceLP(lp)
        b = pdhg.Solver(d, precision=prec, eps_rel=1e-6)
        d.free()  # the library holds its own copy
        ra, rb = a.solve(), b.solve()
        assert (ra.status, ra.iters, ra.restarts) == (rb.status, rb.iters, rb.restarts)
        pa, pb = a.corner_push(5), b.corner_push(5)
        assert (pa.status, pa.iters, pa.n_fix_lower, pa.n_fix_upper) == (pb.status, pb.iters, pb.n_fix_lower, pb.n_fix_upper)
        for va, vb in zip(a.get_solution(), b.get_solution()):
            np.testing.assert_array_equal(va, vb)
    lp = lpgen.config0(1)
    bad_cases = []
    x = copy.deepcopy(lp)
    x.col = x.col.copy()
    x.col[x.row_ptr[3]] = lp.n  # a column out of range
    bad_cases.append((x, b"column index out of range"))
    x = copy.deepcopy(lp)
    x.col = x.col.copy()
    r0 = int(x.row_ptr[5])
    x.col[r0], x.col[r0 + 1] = x.col[r0 + 1], x.col[r0]  # unsorted row
    bad_cases.append((x, b"ascending"))
    x = copy.deepcopy(lp)
    x.val = x.val.copy()
    x.val[7] = np.nan
    bad_cases.append((x, b"non-finite matrix value"))
    x = copy.deepcopy(lp)
    x.u = x.u.copy()
    x.u[4] = -1.0  # l > u
    bad_cases.append((x, b"bounds"))
    for x, msg in bad_cases:
        d = pdhg.DeviceLP(x)
        with pytest.raises(pdhg.PdhgError) as e:
            pdhg.Solver(d)
        assert msg.decode() in str(e.value), str(e.value)
        d.free()
