"""Grids whose displacement fields exceed 4 GiB (GPU).

The iteration kernel with one load per block reads and writes a field
through a buffer view of one z-plane of one component at a time.  Regression
test of the earlier whole-field views, whose 32-bit byte range silently read
zeros (and wrapped stores) once 3N words passed 4 GiB: FP64 from 564^3 on,
FP32 from 711^3 on.  The iterates of the buffer-view kernel (variant 3, the
default) must equal those of the kernel with 64-bit pointer arithmetic
(variant 1) after ten steps, on a seeded three-phase image.
"""
import ctypes

import numpy as np
import pytest

from gpu_common import announce, need_gpu

pytestmark = pytest.mark.gpu

TAB_K = np.array([70.0, 37.0, 2.2])
TAB_G = np.array([32.0, 44.0, 1e-3])


def _steps(p, c, J, nsteps, precision, n):
    u = np.empty(3 * n ** 3)
    p.ceff_apt_steps(c.h, J, nsteps, precision, 0.95, 3.0, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)
    return u


@pytest.mark.parametrize("n,precision,tol", [(566, "fp64", 1e-12), (712, "mixed", 1e-5)])
def test_one_load_beyond_4gib_matches_pointer_form(monkeypatch, n, precision, tol):
    p = need_gpu()
    word = 8 if precision == "fp64" else 4
    assert 3 * n ** 3 * word > 2 ** 32
    prec = p.CEFF_PREC_FP64 if precision == "fp64" else p.CEFF_PREC_MIXED
    rng = np.random.default_rng(n)
    phase = rng.integers(0, 3, size=(n, n, n), dtype=np.uint8)
    with p.Context() as c:
        c.set_phases(phase, TAB_K, TAB_G)
        del phase
        monkeypatch.delenv("CEFF_TILE", raising=False)
        announce("beyond 4 GiB", n, precision, "default variant 9")
        u3 = _steps(p, c, 2, 10, prec, n)
        st = c.stats()
        assert (st["tile_bx"], st["tile_by"], st["tile_kc"], st["tile_variant"]) == (64, 8, 32, 9)
        monkeypatch.setenv("CEFF_TILE", "34,14,12,1,1")
        announce("beyond 4 GiB", n, precision, "variant 1 (pointer form)")
        u1 = _steps(p, c, 2, 10, prec, n)
        assert c.stats()["tile_variant"] == 1
    N = n ** 3
    # the top planes of u_z lie beyond 4 GiB of the field: they must carry the iterate
    top = u1[3 * N - n * n:]
    assert np.abs(top).max() > 0.0
    scale = np.abs(u1).max()
    err = float(np.abs(u3 - u1).max()) / scale
    print(f"n {n} {precision}: max |u3 - u1| / max |u1| = {err:.3e}", flush=True)
    assert err <= tol
