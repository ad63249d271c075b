"""The allocation-free FP64 dot product (scratch in a static device array) against prop_dot_f64, which
allocates its partial sums per call: two calls in a row, the second with a smaller input, each
bitwise equal to the allocating call (same kernels, same order) and within 1e-12 of an FP64 numpy dot.
Collected last (the file name) so that a failure here hides no other test."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_noalloc_dot_matches_the_allocating_dot():
    from paper_2004_10519_amd import prop
    L = prop.lib()
    rng = np.random.default_rng(77)
    for n in (3_000_017, 1_001):
        a = rng.standard_normal(n).astype(np.float32)
        b = rng.standard_normal(n).astype(np.float32)
        ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        res = ctypes.c_double()
        rc = L.prop_dot_f64_noalloc(ta.data_ptr(), tb.data_ptr(), n, ctypes.byref(res),
                                    int(torch.cuda.current_stream().cuda_stream))
        assert rc == prop.PROP_OK, L.prop_last_error()
        ref = prop.dot_f64(ta, tb)
        assert res.value == ref, (n, res.value, ref)
        exact = float(np.dot(a.astype(np.float64), b.astype(np.float64)))
        assert abs(res.value - exact) <= 1e-12 * np.abs(a.astype(np.float64) * b).sum()
    res = ctypes.c_double(1.0)
    assert L.prop_dot_f64_noalloc(ta.data_ptr(), tb.data_ptr(), 0, ctypes.byref(res), None) == prop.PROP_OK
    assert res.value == 0.0
    with pytest.raises(prop.PropError) as e:
        L_res = ctypes.c_double()
        prop._check(L.prop_dot_f64_noalloc(ta.data_ptr(), tb.data_ptr(), -1, ctypes.byref(L_res), None))
    assert e.value.code == prop.PROP_EINVAL
