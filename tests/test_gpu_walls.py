"""Wall boundaries (ceff_set_boundary(CEFF_BC_WALLS): the paper's direct tests),
GPU.  Loads 0..2 run the normal test (rigid, free-slip walls), loads 3..5 the
simple-shear test (the loaded walls also hold the sheared component through
split half edges).

Step, residual and average parity with the oracle's wall modes for all six
loads (steps against both the displacement form and the paper's (p, tau, v)
form), C* columns against the oracle's wall-mode PCG solve, the paper's layered
Model 1 at its full size against the analytic values (normal block and the
in-plane C66, which the walls do not disturb) and against the oracle's slab
solution for C44 and C55, and the error paths."""
import json
import os

import numpy as np
import pytest

import closed_forms as cf
import oracle
import synth
from gpu_common import announce, need_gpu

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
SHAPES = [((8, 8, 8), 1), ((12, 10, 9), 2), ((70, 9, 5), 3), ((5, 23, 6), 4), ((6, 5, 41), 5)]


def fields(shape, seed):
    return synth.random_fields(shape, seed, lo=(2.0, 1e-3), hi=(90.0, 45.0))


def rel6(C, Co):
    return np.max(np.abs(C - Co)) / np.max(np.abs(Co))


@pytest.mark.parametrize("shape,seed", SHAPES)
def test_walls_steps_match_oracle(shape, seed):
    p = need_gpu()
    K, G = fields(shape, seed)
    announce("walls apt_steps", shape, seed)
    with p.Context() as c:
        c.set_material(K, G)
        c.set_boundary("walls")
        for J in range(6):
            for k in (1, 2, 11):
                u, up = c.apt_steps(J, k, "fp64", courant=0.95, strouhal=3.0)
                ref, refp = oracle.apt_disp(J, k, 0.95, 3.0, K=K, G=G, walls=True)
                sc = np.abs(ref).max()
                assert np.max(np.abs(u - ref)) <= 1e-11 * sc, (J, k)
                if k > 1:
                    assert np.max(np.abs(up - refp)) <= 1e-11 * sc
        u32, _ = c.apt_steps(2, 9, "mixed", courant=0.95, strouhal=3.0)
        v32, _ = c.apt_steps(5, 9, "mixed", courant=0.95, strouhal=3.0)
    ref, _ = oracle.apt_disp(2, 9, 0.95, 3.0, K=K, G=G, walls=True)
    assert np.max(np.abs(u32 - ref)) <= 2e-5 * np.abs(ref).max()
    ref, _ = oracle.apt_disp(5, 9, 0.95, 3.0, K=K, G=G, walls=True)
    assert np.max(np.abs(v32 - ref)) <= 2e-5 * np.abs(ref).max()


@pytest.mark.parametrize("shape,seed", SHAPES[:3])
@pytest.mark.parametrize("use_phases", [False, True])
def test_walls_steps_match_paper_form(shape, seed, use_phases):
    """The iterates under the walls against the oracle's iteration in the paper's own
    variables (pressure, deviatoric and edge stresses, velocity), all six loads, FP64
    and mixed precision, from K and G fields and from a phase image."""
    p = need_gpu()
    if use_phases:
        # three phases, soft to stiff, scattered at random
        ph = np.random.default_rng(seed).integers(0, 3, size=shape).astype(np.uint8)
        K_tab, G_tab = np.array([2.0, 36.0, 90.0]), np.array([1e-3, 44.0, 45.0])
        K, G = K_tab[ph], G_tab[ph]
    else:
        K, G = fields(shape, seed)
    announce("walls apt_steps vs paper form", shape, seed, use_phases)
    with p.Context() as c:
        if use_phases:
            c.set_phases(ph, K_tab, G_tab)
        else:
            c.set_material(K, G)
        c.set_boundary("walls")
        for J in range(6):
            ref = oracle.apt_steps(K, G, J, 11, 0.95, 3.0, walls=True)["v"]
            sc = np.abs(ref).max()
            u, _ = c.apt_steps(J, 11, "fp64", courant=0.95, strouhal=3.0)
            assert np.max(np.abs(u - ref)) <= 1e-11 * sc, J
            u, _ = c.apt_steps(J, 11, "mixed", courant=0.95, strouhal=3.0)
            assert np.max(np.abs(u - ref)) <= 2e-5 * sc, J


@pytest.mark.parametrize("shape,seed", SHAPES[:3])
def test_walls_residual_and_averages_match_oracle(shape, seed):
    p = need_gpu()
    K, G = fields(shape, seed)
    u = np.stack([synth.random_fields(shape, 60 + q, lo=(0.5, 0.5), hi=(2.0, 2.0))[0] - 1.0 for q in range(3)])
    announce("walls residual", shape)
    with p.Context() as c:
        c.set_material(K, G)
        c.set_boundary("walls")
        for J in (0, 2, 3, 4, 5):
            r, n2 = c.residual(J, u, "fp64")
            ref = oracle.residual_walls(K, G, oracle.unit_strain(J), u)
            assert np.max(np.abs(r - ref)) <= 1e-12 * np.abs(ref).max(), J
            assert n2 == pytest.approx(float(np.sum(ref * ref)), rel=1e-12)
        for J in range(6):
            a = c.average_stress(J, u)
            ref = oracle.average_stress_walls(K, G, oracle.unit_strain(J), u)
            np.testing.assert_allclose(a, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("use_phases", [False, True])
def test_walls_ceff_matches_oracle(use_phases):
    p = need_gpu()
    m = synth.gaussian_field_three_phase(20, 0xC4)
    K, G = m.fields()
    Co, _ = oracle.ceff_walls(K, G, rtol=1e-12, loads=range(6))
    announce("walls ceff", use_phases)
    with p.Context() as c:
        if use_phases:
            c.set_phases(m.phase, m.K_tab, m.G_tab)
        else:
            c.set_material(K, G)
        c.set_boundary("walls")
        for prec in ("mixed", "fp64"):
            C, info = c.solve(precision=prec, rtol=1e-9)
            assert info["status"] == 0 and info["stats"]["fused_loads"] == 0
            assert rel6(C, Co) <= 1e-6, (prec, rel6(C, Co))
        # the walls change the result: periodic C* differs
        c.set_boundary("periodic")
        Cp, _ = c.solve(precision="fp64", rtol=1e-9)
    assert rel6(Cp, Co) > 1e-4


def test_walls_homogeneous_is_exact():
    p = need_gpu()
    m = synth.homogeneous((20, 18, 16))
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        c.set_boundary("walls")
        C, info = c.solve(precision="mixed")
    np.testing.assert_allclose(C, cf.c_iso(70.0, 32.0), rtol=1e-14, atol=1e-12)
    assert np.all(info["iters"] == 0)


def test_walls_paper_layered_model_full_size():
    """Model 1 at 191^3 with walls: the normal block and C66 equal the analytic
    values to every printed digit (the paper's numerical column differs by up to
    0.4%: C33 30.419, C12 3.720, C13 2.148, C66 25.376).  C44 and C55 exceed the
    analytic 14.124, as the paper's do (15.307): the walls normal to the sheared
    direction hold the layer-wise displacement.  They equal the oracle's value,
    computed on a one-voxel slab (the solution is uniform along x for C44, along
    y for C55)."""
    p = need_gpu()
    g = json.load(open(os.path.join(GOLD, "table2_layered.json")))
    geo = g["geometry"]
    st, so = g["layers"]["stiff"], g["layers"]["soft"]
    m = synth.laminate_z(191, 191, 191, geo["stiff_layers"], geo["layer_thickness"],
                         stiff=(st["K"], st["G"]), soft=(so["K"], so["G"]))
    announce("walls laminate 191^3")
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        c.set_boundary("walls")
        C, info = c.solve(precision="mixed", rtol=1e-8)
    assert info["status"] == 0
    idx = {"C11": (0, 0), "C22": (1, 1), "C33": (2, 2), "C12": (0, 1), "C13": (0, 2), "C23": (1, 2),
           "C66": (5, 5)}
    for name, (I, J) in idx.items():
        assert round(C[I, J], 3) == pytest.approx(g["analytic_GPa"][name], abs=1e-12), name
    # the paper's own route to the off-diagonal constants: triaxial test + D1-D5
    C12, C13, C23 = p.triaxial_offdiagonals(C)
    for name, v in (("C12", C12), ("C13", C13), ("C23", C23)):
        assert round(v, 3) == pytest.approx(g["analytic_GPa"][name], abs=1e-12), name
    slab = synth.laminate_z(1, 191, 191, geo["stiff_layers"], geo["layer_thickness"],
                            stiff=(st["K"], st["G"]), soft=(so["K"], so["G"]))
    Co, _ = oracle.ceff_walls(*slab.fields(), rtol=1e-12, loads=(3,))
    print("C44 %.6f C55 %.6f oracle slab %.6f, analytic %.3f" % (C[3, 3], C[4, 4], Co[3, 3], g["analytic_GPa"]["C44"]))
    assert C[3, 3] == pytest.approx(Co[3, 3], rel=1e-6)
    assert C[4, 4] == pytest.approx(Co[3, 3], rel=1e-6)


def test_walls_errors():
    p = need_gpu()
    from paper_2410_20441_amd import _lib
    K, G = fields((8, 8, 8), 9)
    with p.Context() as c:
        c.set_material(K, G)
        with pytest.raises(p.CeffError) as e:
            p.ceff_set_boundary(c.h, 7)
        assert e.value.status == _lib.CEFF_EINVAL
        c.set_boundary("walls")
        c.solve(loads=(0, 1, 2), precision="fp64", keep_fields=True)
        with pytest.raises(p.CeffError) as e:
            c.gradient(np.diag([1.0, 0, 0, 0, 0, 0]))
        assert e.value.status == _lib.CEFF_EUNSUPPORTED
        c.set_stiffness(oracle.iso_to_c9(K, G))
        with pytest.raises(p.CeffError) as e:
            c.solve(loads=(0,), precision="fp64")
        assert e.value.status == _lib.CEFF_EUNSUPPORTED


def test_triaxial_offdiagonals_formula():
    """D1-D5 recover the off-diagonal constants of any symmetric normal block from a
    triaxial test with arbitrary nonzero strains; zero or non-finite input is rejected."""
    p = need_gpu()
    from paper_2410_20441_amd import _lib
    import ctypes
    Cn = np.array([[80.0, 31.0, 27.0], [31.0, 66.0, 22.0], [27.0, 22.0, 51.0]])
    eps = np.array([0.7, -1.3, 2.1])
    sig = Cn @ eps
    out = np.empty(3)
    dp = ctypes.POINTER(ctypes.c_double)
    a = lambda x: np.ascontiguousarray(x, np.float64).ctypes.data_as(dp)
    p.ceff_triaxial_offdiagonals(a(sig), a(eps), a(np.diag(Cn)), out.ctypes.data_as(dp))
    np.testing.assert_allclose(out, [31.0, 27.0, 22.0], rtol=1e-13)
    for bad in ([0.7, 0.0, 2.1], [0.7, np.nan, 2.1]):
        assert p._L.ceff_triaxial_offdiagonals(a(sig), a(bad), a(np.diag(Cn)), out.ctypes.data_as(dp)) == \
            _lib.CEFF_EINVAL
