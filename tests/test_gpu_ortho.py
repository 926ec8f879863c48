"""Orthotropic cells (ceff_set_stiffness with nine constants per cell), GPU.

Step, residual and average parity with the oracle's orthotropic operator and
its stress-state APT iteration (stresses kept as state and relaxed as in the
paper's scheme; on isotropic cells it is the paper-form iteration), C* parity with the oracle's PCG solve,
the textbook laminate averages at full size, and the isotropic special case
against the isotropic path."""
import numpy as np
import pytest

import closed_forms as cf
import oracle
import synth
from gpu_common import announce, matrix_rel, need_gpu

pytestmark = pytest.mark.gpu

SHAPES = [((8, 8, 8), 1), ((12, 10, 9), 2), ((5, 23, 6), 4), ((6, 5, 41), 5), ((70, 9, 5), 3)]


def c9(shape, seed):
    nz, ny, nx = shape[2], shape[1], shape[0]
    return synth.random_orthotropic((nz, ny, nx), seed)


@pytest.mark.parametrize("shape,seed", SHAPES)
def test_ortho_steps_match_oracle(shape, seed):
    p = need_gpu()
    C9 = c9(shape, seed)
    announce("ortho apt_steps", shape, seed)
    with p.Context() as c:
        c.set_stiffness(C9)
        for J in (0, 3, 5):
            for k in (1, 2, 11):
                u, up = c.apt_steps(J, k, "fp64", courant=0.95, strouhal=3.0)
                ref, refp = oracle.apt_stress(J, k, 0.95, 3.0, C9=C9)
                sc = np.abs(ref).max()
                assert np.max(np.abs(u - ref)) <= 1e-11 * sc, (J, k)
                if k > 1:
                    assert np.max(np.abs(up - refp)) <= 1e-11 * sc
        u32, _ = c.apt_steps(1, 9, "mixed", courant=0.95, strouhal=3.0)
    ref, _ = oracle.apt_stress(1, 9, 0.95, 3.0, C9=C9)
    assert np.max(np.abs(u32 - ref)) <= 2e-5 * np.abs(ref).max()


@pytest.mark.parametrize("shape,seed", SHAPES[:3])
def test_ortho_residual_and_averages_match_oracle(shape, seed):
    p = need_gpu()
    C9 = c9(shape, seed)
    nz, ny, nx = C9.shape[1:]
    u = np.stack([synth.random_fields((nx, ny, nz), 40 + q, lo=(0.5, 0.5), hi=(2.0, 2.0))[0] - 1.0
                  for q in range(3)])
    announce("ortho residual", shape)
    with p.Context() as c:
        c.set_stiffness(C9)
        for J in (0, 4):
            r, n2 = c.residual(J, u, "fp64")
            ref = oracle.residual_ortho(C9, oracle.unit_strain(J), u)
            sc = np.abs(ref).max()
            assert np.max(np.abs(r - ref)) <= 1e-12 * sc
            assert n2 == pytest.approx(float(np.sum(ref * ref)), rel=1e-12)
            r32, _ = c.residual(J, u, "mixed")
            assert np.max(np.abs(r32 - ref)) <= 2e-5 * sc
        for J in range(6):
            a = c.average_stress(J, u)
            ref = oracle.average_stress_ortho(C9, oracle.unit_strain(J), u)
            np.testing.assert_allclose(a, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("shape,seed", [((12, 10, 9), 21), ((20, 18, 16), 22)])
def test_ortho_ceff_matches_oracle(shape, seed):
    p = need_gpu()
    C9 = c9(shape, seed)
    Co, _ = oracle.ceff_ortho(C9, rtol=1e-12)
    announce("ortho ceff", shape)
    with p.Context() as c:
        c.set_stiffness(C9)
        for prec, fuse in (("mixed", True), ("mixed", False), ("fp64", False)):
            C, info = c.solve(precision=prec, fuse_loads=fuse, rtol=1e-9)
            assert info["status"] == 0
            assert matrix_rel(C, Co) <= 1e-6, (prec, fuse, matrix_rel(C, Co))


def test_ortho_laminate_full_size():
    """Orthotropic layers stacked along z at 96^3 (three layer types, uneven
    thicknesses): the laminate averages hold exactly for the discrete operator."""
    p = need_gpu()
    lay = synth.random_orthotropic((3, 1, 1), 31)[:, :, 0, 0]
    thick = [40, 24, 32]
    C9 = np.concatenate([np.broadcast_to(lay[:, l, None, None, None], (9, t, 96, 96))
                         for l, t in enumerate(thick)], axis=1).astype(np.float32)
    announce("ortho laminate 96^3")
    with p.Context() as c:
        c.set_stiffness(np.ascontiguousarray(C9))
        C, info = c.solve(precision="mixed", rtol=1e-8)
    Cb = cf.backus_z_ortho(thick, [oracle.voigt_of_c9(lay[:, l].astype(np.float32).astype(np.float64))
                                   for l in range(3)])
    assert matrix_rel(C, Cb) <= 1e-6


def test_isotropic_cells_through_set_stiffness():
    p = need_gpu()
    m = synth.workload_sphere32()
    K, G = m.fields()
    with p.Context() as c:
        c.set_material(K, G)
        Ci, ii = c.solve(precision="mixed", rtol=1e-9)
        c.set_stiffness(oracle.iso_to_c9(K, G))
        Co, io = c.solve(precision="mixed", rtol=1e-9)
    assert matrix_rel(Co, Ci) <= 1e-8


def test_set_stiffness_errors():
    p = need_gpu()
    from paper_2410_20441_amd import _lib
    C9 = c9((6, 5, 4), 3)
    with p.Context() as c:
        c.set_stiffness(C9)
        bad = C9.copy()
        bad[5, 0, 0, 0] = 2.0 * np.sqrt(bad[0, 0, 0, 0] * bad[1, 0, 0, 0])  # C12 beyond the normal block's PD range
        with pytest.raises(p.CeffError) as e:
            c.set_stiffness(bad)
        assert e.value.status == _lib.CEFF_EINVAL
        bad = C9.copy()
        bad[7, 1, 2, 3] = -1.0
        with pytest.raises(p.CeffError):
            c.set_stiffness(bad)
        x = np.ascontiguousarray(np.zeros(21 * C9[0].size))  # general cells, not positive definite
        st = p._L.ceff_set_stiffness(c.h, x.ctypes.data, 21, _lib.CEFF_F64, _lib.CEFF_HOST)
        assert st == _lib.CEFF_EINVAL
        st = p._L.ceff_set_stiffness(c.h, x.ctypes.data, 5, _lib.CEFF_F64, _lib.CEFF_HOST)
        assert st == _lib.CEFF_EINVAL
        c.set_stiffness(C9)
        C, info = c.solve(precision="fp64", rtol=1e-9, keep_fields=True)
        with pytest.raises(p.CeffError) as e:
            c.gradient(np.eye(6))
        assert e.value.status == _lib.CEFF_EUNSUPPORTED
