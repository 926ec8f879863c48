"""Pins of the oracle for orthotropic cells (nine constants per cell), CPU.

The orthotropic law is the isotropic one written with its 6x6 Voigt matrix;
the pins tie the orthotropic code to the independently pinned isotropic code,
to the dense energy minimisation, to textbook laminate averages and to lattice
symmetries, so that a constant routed to the wrong node fails one of them."""
import numpy as np
import pytest

import closed_forms as cf
import oracle
from oracle import dense
import synth


def rel(A, B):
    return np.max(np.abs(A - B)) / np.max(np.abs(B))


def random_ortho(shape, seed):
    C9 = synth.random_orthotropic(shape, seed)
    for t in range(int(np.prod(shape))):
        assert np.all(np.linalg.eigvalsh(oracle.voigt_of_c9(C9.reshape(9, -1)[:, t])) > 0)
    return C9


def test_isotropic_cells_reduce_to_the_isotropic_oracle():
    K, G = synth.random_fields((5, 4, 6), 3)
    C9 = oracle.iso_to_c9(K, G)
    E = oracle.unit_strain(4)
    u = np.stack([synth.random_fields((5, 4, 6), 10 + c)[0] for c in range(3)])
    np.testing.assert_allclose(oracle.stress_ortho(C9, E, u), oracle.stress(K, G, E, u), rtol=1e-13, atol=1e-11)
    np.testing.assert_allclose(oracle.residual_ortho(C9, E, u), oracle.residual(K, G, E, u), rtol=1e-12, atol=1e-10)
    Ci, _ = oracle.ceff(K, G, rtol=1e-12)
    Co, _ = oracle.ceff_ortho(C9, rtol=1e-12)
    assert rel(Co, Ci) < 1e-10


def test_homogeneous_orthotropic_is_exact():
    c = random_ortho((1, 1, 1), 5)[:, 0, 0, 0]
    C9 = np.broadcast_to(c[:, None, None, None], (9, 4, 5, 6)).copy()
    C, info = oracle.ceff_ortho(C9)
    np.testing.assert_allclose(C, oracle.voigt_of_c9(c), rtol=1e-14, atol=1e-12)
    assert all(it == 0 for it, _ in info.values())


def test_orthotropic_laminate_is_exact():
    """Layers normal to z with their own orthotropic constants: the textbook laminate
    averages hold exactly for the discrete operator (integer layers, harmonic edges)."""
    layers = random_ortho((3, 1, 1), 8)[:, :, 0, 0]          # (9, 3 layers)
    thick = [2, 3, 1]
    C9 = np.concatenate([np.broadcast_to(layers[:, l, None, None, None], (9, t, 4, 5))
                         for l, t in enumerate(thick)], axis=1)
    C, _ = oracle.ceff_ortho(np.ascontiguousarray(C9), rtol=1e-13)
    Cb = cf.backus_z_ortho(thick, [oracle.voigt_of_c9(layers[:, l]) for l in range(3)])
    assert rel(C, Cb) < 1e-10


def test_orthotropic_dense_matches_pcg():
    C9 = random_ortho((2, 3, 3), 11)
    Cd = dense.ceff_dense(None, None, C9=C9)
    Cp, _ = oracle.ceff_ortho(C9, rtol=1e-13)
    assert rel(Cp, Cd) < 1e-9
    assert rel(Cp, Cp.T) < 1e-10


def test_orthotropic_axis_swap():
    """Swapping x and y of the image and of every cell's constants permutes C*."""
    C9 = random_ortho((3, 5, 4), 12)
    C, _ = oracle.ceff_ortho(C9, rtol=1e-13)
    # constants of the swapped cells: C11<->C22, C23<->C13, C44<->C55
    Cs = C9[[1, 0, 2, 4, 3, 5, 7, 6, 8]]
    Cs = np.ascontiguousarray(np.swapaxes(Cs, 2, 3))
    Ct, _ = oracle.ceff_ortho(Cs, rtol=1e-13)
    P = [1, 0, 2, 4, 3, 5]
    assert rel(Ct, C[np.ix_(P, P)]) < 1e-10


def test_displacement_form_equals_paper_form():
    """For isotropic cells the displacement-form iteration is the paper's (p, tau, v) one."""
    K, G = synth.random_fields((7, 5, 6), 4, lo=(2.0, 1e-3), hi=(90.0, 45.0))
    for J in (0, 3):
        for k in (1, 2, 9):
            u, up = oracle.apt_disp(J, k, 0.95, 3.0, K=K, G=G)
            v = oracle.apt_steps(K, G, J, k, 0.95, 3.0)["v"]
            assert np.max(np.abs(u - v)) <= 1e-12 * np.abs(v).max()
            if k > 1:
                vp = oracle.apt_steps(K, G, J, k - 1, 0.95, 3.0)["v"]
                assert np.max(np.abs(up - vp)) <= 1e-12 * np.abs(v).max()


def test_orthotropic_iteration_fixed_point():
    """The displacement-form iteration on orthotropic cells converges to the PCG solution."""
    C9 = random_ortho((4, 5, 6), 13)
    for J in (1, 5):
        u_ref, _, _ = oracle.solve_load_ortho(C9, J, rtol=1e-13)
        u, _ = oracle.apt_disp(J, 3000, 0.95, 4.0, C9=C9)
        u = u - u.reshape(3, -1).mean(1)[:, None, None, None]
        assert np.max(np.abs(u - u_ref)) < 1e-9 * np.max(np.abs(u_ref))


def test_stress_state_iteration_is_the_paper_form_and_converges():
    """The stress-state APT iteration: on isotropic cells it is the paper's (p, tau, v)
    iteration, periodic and under the wall tests; on orthotropic cells it reproduces the
    displacement-form iterates step by step and converges to the PCG solution."""
    K, G = synth.random_fields((7, 5, 6), 4, lo=(2.0, 1e-3), hi=(90.0, 45.0))
    for walls in (False, True):
        for J in range(6):
            for k in (1, 2, 9):
                u, _ = oracle.apt_stress(J, k, 0.95, 3.0, K=K, G=G, walls=walls)
                v = oracle.apt_steps(K, G, J, k, 0.95, 3.0, walls=walls)["v"]
                assert np.max(np.abs(u - v)) <= 1e-12 * np.abs(v).max(), (walls, J, k)
    C9 = random_ortho((4, 5, 6), 14)
    for J in (0, 3, 5):
        for k in (1, 2, 9):
            u, up = oracle.apt_stress(J, k, 0.95, 3.0, C9=C9)
            w, wp = oracle.apt_disp(J, k, 0.95, 3.0, C9=C9)
            assert np.max(np.abs(u - w)) <= 1e-12 * np.abs(w).max(), (J, k)
            assert np.max(np.abs(up - wp)) <= 1e-12 * np.abs(w).max(), (J, k)
    J = 1
    u_ref, _, _ = oracle.solve_load_ortho(C9, J, rtol=1e-13)
    v, _ = oracle.apt_stress(J, 3000, 0.95, 4.0, C9=C9)
    v = v - v.reshape(3, -1).mean(1)[:, None, None, None]
    assert np.max(np.abs(v - u_ref)) < 1e-9 * np.max(np.abs(u_ref))
