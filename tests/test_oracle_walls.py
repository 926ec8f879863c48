"""Pins of the oracle's wall-boundary modes (the paper's direct tests: the
normal-compression and triaxial tests with rigid, free-slip walls, and the
simple-shear test whose loaded walls also hold the sheared component), CPU.

Checked against an independent dense energy minimisation with the same walls
(all six loads), against the homogeneous medium (exact, no iterations), against
the exact layer averages of a z-laminate (the normal block, whose solution the
walls do not disturb, and the in-plane shear C66, whose uniform-strain solution
they do not disturb either), against the mean shear strain (the walls impose it
exactly) and against the paper's layered-model analytic values.  The iteration in
the paper's own variables under the walls is checked against the displacement form
step by step and against the PCG solution at its fixed point."""
import json
import os

import numpy as np
import pytest

import closed_forms as cf
import oracle
from oracle import dense
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
IDX = {"C11": (0, 0), "C22": (1, 1), "C33": (2, 2), "C12": (0, 1), "C13": (0, 2), "C23": (1, 2)}


def rel(A, B):
    return np.nanmax(np.abs(A - B)) / np.nanmax(np.abs(B))


def test_walls_dense_matches_pcg():
    K, G = synth.random_fields((3, 4, 3), 5, lo=(5.0, 2.0), hi=(90.0, 45.0))
    Cw, _ = oracle.ceff_walls(K, G, rtol=1e-13, loads=range(6))
    Cd = dense.ceff_dense_walls(K, G, loads=range(6))
    assert rel(Cw, Cd) < 1e-10
    # the walls change the answer (they are not the periodic problem)
    Cp, _ = oracle.ceff(K, G, rtol=1e-13, loads=range(3))
    assert rel(Cw[:3, :3], Cp[:3, :3]) > 1e-3


def test_walls_homogeneous_exact():
    m = synth.homogeneous((5, 4, 6))
    Cw, info = oracle.ceff_walls(*m.fields(), loads=range(6))
    np.testing.assert_allclose(Cw, cf.c_iso(70.0, 32.0), rtol=1e-14, atol=1e-12)
    assert all(it == 0 for it, _ in info.values())


def test_walls_laminate_normal_block_exact():
    Ks, Gs, thick = [30.0, 6.0, 80.0], [20.0, 3.0, 40.0], [3, 2, 4]
    K = np.concatenate([np.full((t, 4, 5), k) for t, k in zip(thick, Ks)])
    G = np.concatenate([np.full((t, 4, 5), g) for t, g in zip(thick, Gs)])
    Cw, _ = oracle.ceff_walls(K, G, rtol=1e-13)
    Cb = cf.backus_z(thick, Ks, Gs)
    assert rel(Cw[:3, :3], Cb[:3, :3]) < 1e-10


def test_shear_walls_laminate():
    """Simple-shear tests on a z-laminate: the in-plane shear keeps the uniform
    strain of the exact solution (C66 = the layer average of G, exactly); the
    shears across the layers are stiffened by the walls normal to y (C44) or x
    (C55), which hold the layer-wise displacement of the exact solution."""
    Ks, Gs, thick = [30.0, 6.0, 80.0], [20.0, 3.0, 40.0], [3, 2, 4]
    K = np.concatenate([np.full((t, 4, 5), k) for t, k in zip(thick, Ks)])
    G = np.concatenate([np.full((t, 4, 5), g) for t, g in zip(thick, Gs)])
    Cw, _ = oracle.ceff_walls(K, G, rtol=1e-13, loads=(3, 4, 5))
    Cb = cf.backus_z(thick, Ks, Gs)
    assert Cw[5, 5] == pytest.approx(Cb[5, 5], rel=1e-12)
    assert Cw[3, 3] > Cb[3, 3] * 1.01 and Cw[4, 4] > Cb[4, 4] * 1.01
    np.testing.assert_allclose(Cw[3:, 3:] - np.diag(np.diag(Cw[3:, 3:])), 0.0, atol=1e-9)


@pytest.mark.parametrize("J", [3, 4, 5])
def test_shear_walls_impose_the_mean_strain(J):
    """The loaded walls move by exactly the applied shear, so the volume average
    of the shear strain (split edges counting half on each side) is the load's."""
    K, G = synth.random_fields((5, 4, 6), 3, lo=(10.0, 5.0), hi=(80.0, 40.0))
    u, _, rel_ = oracle.solve_load_walls(K, G, J, rtol=1e-13)
    E = oracle.unit_strain(J)
    eps = dense.strain_field(u, E)
    _, keep = dense.wall_masks(K.shape, J)
    bot, top = dense.split_edge_strains(u, E, J)
    mean = ((eps[J] * keep[J - 3].reshape(K.shape)).sum() + 0.5 * (bot + top).sum()) / K.size
    assert mean == pytest.approx(E[J], rel=1e-12)
    # and the walls do act: the solution is not the affine field
    assert np.max(np.abs(u)) > 1e-3


def test_walls_paper_layered_model_analytic_values():
    """Model 1 (six stiff 15-voxel layers in 191): with walls, the normal block
    still equals the analytic values to every printed digit (a 2 x 2 x 191 prism is
    the same problem, the solution being uniform in x and y)."""
    g = json.load(open(os.path.join(GOLD, "table2_layered.json")))
    geo = g["geometry"]
    m = synth.laminate_z(2, 2, geo["n"], geo["stiff_layers"], geo["layer_thickness"],
                         stiff=(g["layers"]["stiff"]["K"], g["layers"]["stiff"]["G"]),
                         soft=(g["layers"]["soft"]["K"], g["layers"]["soft"]["G"]))
    C, _ = oracle.ceff_walls(*m.fields(), rtol=1e-12)
    for name, (I, J) in IDX.items():
        assert round(C[I, J], g["printed_decimals"]) == pytest.approx(g["analytic_GPa"][name], abs=1e-12), name


def test_shear_walls_paper_layered_model():
    """Model 1 under the simple-shear tests.  C66 (shear in the plane of the
    layers) equals the analytic value to every printed digit.  C44 and C55 (shear
    across the layers) exceed the analytic value: the walls normal to the shear
    direction hold the layer-wise displacement (the paper attributes its C44 and
    C55 excess to the same boundary conditions).  The solution is uniform along
    the third direction, so 1-voxel-thick slabs are the full problem."""
    g = json.load(open(os.path.join(GOLD, "table2_layered.json")))
    geo = g["geometry"]
    lay = dict(stiff=(g["layers"]["stiff"]["K"], g["layers"]["stiff"]["G"]),
               soft=(g["layers"]["soft"]["K"], g["layers"]["soft"]["G"]))
    n = geo["n"]
    C44, _ = oracle.ceff_walls(*synth.laminate_z(1, n, n, geo["stiff_layers"], geo["layer_thickness"], **lay).fields(),
                               rtol=1e-12, loads=(3,))
    C55, _ = oracle.ceff_walls(*synth.laminate_z(n, 1, n, geo["stiff_layers"], geo["layer_thickness"], **lay).fields(),
                               rtol=1e-12, loads=(4,))
    C66, _ = oracle.ceff_walls(*synth.laminate_z(2, 2, n, geo["stiff_layers"], geo["layer_thickness"], **lay).fields(),
                               rtol=1e-12, loads=(5,))
    assert round(C66[5, 5], g["printed_decimals"]) == pytest.approx(g["analytic_GPa"]["C66"], abs=1e-12)
    assert C44[3, 3] == pytest.approx(C55[4, 4], rel=1e-10)
    assert C44[3, 3] > g["analytic_GPa"]["C44"] * 1.03


def test_walls_residual_and_iteration_fixed_point():
    K, G = synth.random_fields((4, 5, 6), 3, lo=(10.0, 5.0), hi=(80.0, 40.0))
    for J in (0, 2, 3, 5):
        u_ref, _, _ = oracle.solve_load_walls(K, G, J, rtol=1e-13)
        r = oracle.residual_walls(K, G, oracle.unit_strain(J), u_ref)
        assert np.max(np.abs(r)) < 1e-9 * np.max(np.abs(oracle.residual_walls(K, G, oracle.unit_strain(J),
                                                                                np.zeros_like(u_ref))))
        # wall faces stay put
        assert np.all(u_ref[0][:, :, 0] == 0) and np.all(u_ref[1][:, 0, :] == 0) and np.all(u_ref[2][0] == 0)
        u, _ = oracle.apt_disp(J, 3000, 0.95, 4.0, K=K, G=G, walls=True)
        assert np.max(np.abs(u - u_ref)) < 1e-9 * np.max(np.abs(u_ref))


def test_walls_paper_form_equals_displacement_form():
    """Under the walls of every load the paper's (p, tau, v) iteration, with the split
    edges' two halves relaxed separately, gives the displacement-form iterates."""
    K, G = synth.random_fields((7, 5, 6), 4, lo=(2.0, 1e-3), hi=(90.0, 45.0))
    for J in range(6):
        for k in (1, 2, 9):
            u, up = oracle.apt_disp(J, k, 0.95, 3.0, K=K, G=G, walls=True)
            v = oracle.apt_steps(K, G, J, k, 0.95, 3.0, walls=True)["v"]
            assert np.max(np.abs(u - v)) <= 1e-12 * np.abs(v).max(), (J, k)
            if k > 1:
                vp = oracle.apt_steps(K, G, J, k - 1, 0.95, 3.0, walls=True)["v"]
                assert np.max(np.abs(up - vp)) <= 1e-12 * np.abs(v).max(), (J, k)


def test_walls_paper_form_fixed_point_and_restart():
    """The paper-form wall iteration converges to the wall-mode PCG solution, keeps the
    wall faces and the free boundary edges' shear stresses at zero, and restarting it
    from a saved state (with the split edges' side-1 halves) continues the same run."""
    K, G = synth.random_fields((4, 5, 6), 3, lo=(10.0, 5.0), hi=(80.0, 40.0))
    for J in (1, 4):
        u_ref, _, _ = oracle.solve_load_walls(K, G, J, rtol=1e-13)
        st = oracle.apt_steps(K, G, J, 3000, courant=0.95, strouhal=4.0, walls=True)
        v = st["v"]
        assert np.max(np.abs(v - u_ref)) < 1e-9 * np.max(np.abs(u_ref))
        assert np.all(v[0][:, :, 0] == 0) and np.all(v[1][:, 0, :] == 0) and np.all(v[2][0] == 0)
        # free-slip edges on the walls: yz-edges with j = 0 or k = 0 carry no stress in the
        # normal test; in the simple-shear test of xz the xy-edges on the x and y walls
        # are free, and the xz-edges on the z walls are split (side 0 in txz, side 1 in half1)
        if J == 1:
            assert np.all(st["tyz"][:, 0, :] == 0) and np.all(st["tyz"][0] == 0)
        else:
            assert np.all(st["txy"][:, :, 0] == 0) and np.all(st["txy"][:, 0, :] == 0)
            assert np.any(st["half1"][0] != 0) and np.all(st["half1"][1:] == 0)
        a = oracle.apt_steps(K, G, J, 7, courant=0.95, strouhal=4.0, walls=True)
        b = oracle.apt_steps(K, G, J, 5, courant=0.95, strouhal=4.0, walls=True, state=a)
        c = oracle.apt_steps(K, G, J, 12, courant=0.95, strouhal=4.0, walls=True)
        assert all(np.array_equal(b[n], c[n]) for n in c)
