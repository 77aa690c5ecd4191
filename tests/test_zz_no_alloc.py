"""The no-allocation forward of the fix predictor, through the C ABI: the
caller's device buffers in and out, the staging array fixed in the library.
It must give the allocating forward's logits exactly (the same conversion
and kernel), on two calls in a row, the second smaller, and write nothing
past its n."""
import ctypes as C

import numpy as np
import pytest

from paper_2511_13894_amd import pdhg

pytestmark = pytest.mark.gpu


def _features(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, 16)).astype(np.float32)
    f[:, 12:] = 0
    return f


def test_forward_noalloc_equals_the_allocating_forward():
    hip = pdhg._hip_runtime()
    net = pdhg.Mlp(3)
    n_max = 65536
    fdev, ldev = C.c_void_p(), C.c_void_p()
    assert hip.hipMalloc(C.byref(fdev), n_max * 16 * 4) == 0
    assert hip.hipMalloc(C.byref(ldev), n_max * 4) == 0
    try:
        for n, seed in ((50000, 1), (1234, 2)):  # the second call is smaller than the first
            f = np.ascontiguousarray(_features(n, seed))
            assert hip.hipMemcpy(fdev, f.ctypes.data_as(C.c_void_p), f.nbytes, 1) == 0
            sentinel = np.full(n_max, np.nan, dtype=np.float32)
            assert hip.hipMemcpy(ldev, sentinel.ctypes.data_as(C.c_void_p), sentinel.nbytes, 1) == 0
            print(f"[noalloc] forward of {n} variables", flush=True)
            net.forward_noalloc(fdev, n, ldev)
            assert hip.hipDeviceSynchronize() == 0
            got = np.empty(n_max, dtype=np.float32)
            assert hip.hipMemcpy(got.ctypes.data_as(C.c_void_p), ldev, got.nbytes, 2) == 0
            want = net.forward(f)
            np.testing.assert_array_equal(got[:n], want)
            assert np.all(np.isnan(got[n:]))  # nothing written past n
        with pytest.raises(pdhg.PdhgError) as e:
            net.forward_noalloc(fdev, n_max + 1, ldev)
        assert "65536" in str(e.value)
        net.forward_noalloc(fdev, 0, ldev)  # an empty call is a no-op
    finally:
        hip.hipFree(fdev)
        hip.hipFree(ldev)
