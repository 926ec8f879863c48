"""General anisotropic (triclinic) cells, ceff_set_stiffness with 21 constants (GPU).

Step, residual and average parity with the oracle's octant reading of the
coupled law and its stress-state APT iteration (stresses kept as state and
relaxed as in the paper's scheme); C* parity with the
oracle's PCG solve (FP64 and mixed precision); the exact layer average of a
rotated laminate; orthotropic cells given as 21 constants against the
orthotropic path; the error paths."""
import numpy as np
import pytest

import closed_forms as cf
import oracle
import synth
from gpu_common import announce, matrix_rel, need_gpu

pytestmark = pytest.mark.gpu

SHAPES = [((6, 6, 6), 1), ((9, 7, 5), 2), ((5, 11, 4), 3), ((4, 5, 13), 4)]


def c21(shape, seed, soft=0.2):
    nx, ny, nz = shape
    return synth.random_triclinic((nz, ny, nx), seed, soft=soft)


@pytest.mark.parametrize("shape,seed", SHAPES)
def test_tri_steps_match_oracle(shape, seed):
    p = need_gpu()
    C21 = c21(shape, seed)
    announce("tri apt_steps", shape, seed)
    with p.Context() as c:
        c.set_stiffness(C21)
        for J in (0, 3, 5):
            for k in (1, 2, 11):
                u, up = c.apt_steps(J, k, "fp64", courant=0.95, strouhal=3.0)
                ref, refp = oracle.apt_stress(J, k, 0.95, 3.0, C21=C21)
                sc = np.abs(ref).max()
                assert np.max(np.abs(u - ref)) <= 1e-11 * sc, (J, k)
                if k > 1:
                    assert np.max(np.abs(up - refp)) <= 1e-11 * sc
        u32, _ = c.apt_steps(2, 9, "mixed", courant=0.95, strouhal=3.0)
    ref, _ = oracle.apt_stress(2, 9, 0.95, 3.0, C21=C21)
    assert np.max(np.abs(u32 - ref)) <= 2e-5 * np.abs(ref).max()


@pytest.mark.parametrize("shape,seed", SHAPES[:3])
def test_tri_residual_and_averages_match_oracle(shape, seed):
    p = need_gpu()
    C21 = c21(shape, seed)
    rng = np.random.default_rng(seed + 50)
    u = rng.standard_normal((3,) + C21.shape[1:])
    announce("tri residual", shape)
    with p.Context() as c:
        c.set_stiffness(C21)
        for J in (1, 4):
            r, n2 = c.residual(J, u, "fp64")
            ref = oracle.residual_tri(C21, oracle.unit_strain(J), u)
            sc = np.abs(ref).max()
            assert np.max(np.abs(r - ref)) <= 1e-12 * sc
            assert n2 == pytest.approx(float(np.sum(ref * ref)), rel=1e-12)
            r32, _ = c.residual(J, u, "mixed")
            assert np.max(np.abs(r32 - ref)) <= 2e-5 * sc
        for J in range(6):
            a = c.average_stress(J, u)
            ref = oracle.average_stress_tri(C21, oracle.unit_strain(J), u)
            np.testing.assert_allclose(a, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tri_ceff_matches_oracle(precision):
    p = need_gpu()
    C21 = c21((12, 10, 9), 7, soft=0.3)
    announce("tri ceff", precision)
    Co, _ = oracle.ceff_tri(C21, rtol=1e-12)
    with p.Context() as c:
        c.set_stiffness(C21)
        C, info = c.solve(precision=precision, rtol=1e-9)
    assert info["status"] == 0
    print(f"tri {precision}: iterations {info['iters'].tolist()}, error {matrix_rel(C, Co):.2e}", flush=True)
    assert matrix_rel(C, Co) <= 1e-6


def test_tri_rotated_laminate_layer_average():
    """Layers of an orthotropic material turned about the stacking axis z (C44 = C55)
    by different angles: C* is the exact anisotropic layer average."""
    p = need_gpu()
    rng = np.random.default_rng(3)
    thick = [5, 3, 8]
    mats = []
    for t in thick:
        C = np.diag([100.0, 60.0, 80.0, 25.0, 25.0, 18.0])
        C[0, 1] = C[1, 0] = 20.0
        C[0, 2] = C[2, 0] = 15.0
        C[1, 2] = C[2, 1] = 25.0
        mats.append(cf.rotate_voigt(C, cf.rotation(2, rng.uniform(0.2, 1.3))))
    nz = sum(thick)
    C21 = np.empty((21, nz, 6, 7))
    pos = 0
    for t, M in zip(thick, mats):
        C21[:, pos:pos + t] = oracle.c21_of_voigt(M)[:, None, None, None]
        pos += t
    with p.Context() as c:
        c.set_stiffness(C21)
        C, info = c.solve(precision="mixed", rtol=1e-10)
    # the yz and xz shears (equal C44 = C55 in every layer) leave the affine state in equilibrium
    assert info["status"] == 0 and info["iters"][3] == 0 and info["iters"][4] == 0
    assert matrix_rel(C, cf.layered_average(thick, mats, 2)) <= 1e-6


def test_orthotropic_cells_as_21_constants():
    p = need_gpu()
    C9 = synth.random_orthotropic((7, 6, 8), 11)
    with p.Context() as c:
        c.set_stiffness(C9)
        C9s, _ = c.solve(precision="fp64", rtol=1e-10)
        c.set_stiffness(oracle.c21_of_c9(C9))
        C21s, _ = c.solve(precision="fp64", rtol=1e-10)
    assert matrix_rel(C21s, C9s) <= 1e-8


def test_tri_errors():
    p = need_gpu()
    from paper_2410_20441_amd import _lib
    C21 = c21((5, 5, 5), 13)
    with p.Context() as c:
        bad = C21.copy()
        bad[15, 1, 1, 1] = -1.0  # C44 < 0: not positive definite
        with pytest.raises(p.CeffError) as e:
            c.set_stiffness(bad)
        assert e.value.status == _lib.CEFF_EINVAL
        bad = C21.copy()
        bad[3, 0, 2, 1] = np.nan
        with pytest.raises(p.CeffError) as e:
            c.set_stiffness(bad)
        assert e.value.status == _lib.CEFF_EINVAL
        c.set_stiffness(C21)
        c.solve(precision="fp64", rtol=1e-8, keep_fields=True)
        with pytest.raises(p.CeffError) as e:
            c.gradient(np.eye(6))
        assert e.value.status == _lib.CEFF_EUNSUPPORTED
        c.set_boundary("walls")
        with pytest.raises(p.CeffError) as e:
            c.solve(loads=(0,), precision="fp64")
        assert e.value.status == _lib.CEFF_EUNSUPPORTED
