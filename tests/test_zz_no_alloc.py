"""The allocation-free stress average (GPU): ceff_average_stress_noalloc on a
device displacement gives what ceff_average_stress gives on the same values,
on two calls in a row, the second on a smaller grid (the scratch array keeps
the first call's partials, which must not leak into the second)."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_common import announce, need_gpu

pytestmark = pytest.mark.gpu


def _noalloc(p, c, J, u_dev):
    out = np.full(6, np.nan)
    p.ceff_average_stress_noalloc(c.h, J, ctypes.c_void_p(u_dev.data_ptr()), out.ctypes.data_as(
        ctypes.POINTER(ctypes.c_double)))
    return out


def test_noalloc_average_equals_allocating_entry_point():
    p = need_gpu()
    import torch
    with p.Context() as c:
        for shape, seed in (((40, 36, 33), 11), ((17, 18, 20), 12)):
            K, G = synth.random_fields(shape, seed, lo=(2.0, 1e-3), hi=(90.0, 45.0))
            c.set_material(K, G)
            rng = np.random.default_rng(seed)
            u = rng.standard_normal((3,) + K.shape)
            u_dev = torch.tensor(u, dtype=torch.float64, device="cuda")
            for J in range(6):
                announce("noalloc average", shape, J)
                ref = c.average_stress(J, u)
                got = _noalloc(p, c, J, u_dev)
                assert np.all(np.isfinite(got))
                np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_noalloc_rejects_bad_arguments():
    p = need_gpu()
    import torch
    with p.Context() as c:
        out = np.zeros(6)
        op = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        u_dev = torch.zeros(3 * 8, dtype=torch.float64, device="cuda")
        assert p._L.ceff_average_stress_noalloc(c.h, 0, ctypes.c_void_p(u_dev.data_ptr()), op) == p._lib.CEFF_ESTATE
        K, G = synth.random_fields((2, 2, 2), 3, lo=(2.0, 1e-3), hi=(90.0, 45.0))
        c.set_material(K, G)
        assert p._L.ceff_average_stress_noalloc(c.h, 6, ctypes.c_void_p(u_dev.data_ptr()), op) == p._lib.CEFF_EINVAL
        assert p._L.ceff_average_stress_noalloc(c.h, 0, None, op) == p._lib.CEFF_EINVAL
        assert p._L.ceff_average_stress_noalloc(c.h, 0, ctypes.c_void_p(u_dev.data_ptr()), None) == p._lib.CEFF_EINVAL
