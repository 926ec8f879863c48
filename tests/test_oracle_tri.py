"""Pins of the oracle's general anisotropic (triclinic, 21-constant) cells (CPU).

The coupled law on the staggered grid is a reading of the paper's "Future
perspectives" (items 2-3: triclinic local stiffness needs some fields
averaged): eight corner octants per cell, each with the cell's normal strains
and the series-weighted strain of the edge of each shear component meeting
its corner; energy = sum over cells of 1/8 of the octant energies.  Pinned by:

* orthotropic cells written as 21 constants reproduce the orthotropic oracle
  (stresses, residual, C*);
* a homogeneous triclinic medium gives C* = C with zero iterations;
* an independent dense assembly of the octant energy (oracle/dense.py), solved
  directly, equals Jacobi-PCG on random triclinic images, including unequal
  spacings;
* stacks of rotated orthotropic layers whose couplings act only through the
  in-plane shear give the exact anisotropic layer average (Schoenberg-Muir),
  one stack per axis, so each of the nine normal-shear couplings is exercised;
* axis swaps, cyclic permutations and mirrors of image and constants permute
  and flip C* accordingly; C* is symmetric positive definite;
* the displacement-form APT iteration converges to the PCG solution.
"""
import math

import numpy as np
import pytest

import closed_forms as cf
import oracle
import synth
from oracle import dense


def rel(A, B):
    return float(np.max(np.abs(A - B)) / np.max(np.abs(B)))


def ceff_tri(C21, h=(1.0, 1.0, 1.0), rtol=1e-11):
    """The oracle's C*, with an iteration cap so that a broken operator fails instead of hanging."""
    C, info = oracle.ceff_tri(C21, h, rtol=rtol, max_iter=20000)
    assert all(r <= 10 * rtol for _, r in info.values()), info
    return C, info


def test_c21_of_c9_reduces_to_the_orthotropic_oracle():
    shape = (5, 6, 7)
    C9 = synth.random_orthotropic(shape, 31)
    C21 = oracle.c21_of_c9(C9)
    rng = np.random.default_rng(4)
    u = rng.standard_normal((3,) + shape)
    for J in (0, 3, 5):
        E = oracle.unit_strain(J)
        s9 = oracle.stress_ortho(C9, E, u)
        s21 = oracle.stress_tri(C21, E, u)
        assert rel(s21, s9) < 1e-13
        assert rel(oracle.residual_tri(C21, E, u), oracle.residual_ortho(C9, E, u)) < 1e-13
    C9s, _ = oracle.ceff_ortho(C9, rtol=1e-12)
    Ct, _ = ceff_tri(C21, rtol=1e-12)
    assert rel(Ct, C9s) < 1e-9


def test_homogeneous_triclinic_is_exact():
    one = synth.random_triclinic((1, 1, 1), 77)[:, 0, 0, 0]
    C21 = np.broadcast_to(one[:, None, None, None], (21, 4, 5, 6)).copy()
    Cv = oracle.voigt_of_c21(one)
    C, info = ceff_tri(C21)
    assert all(it == 0 for it, _ in info.values())  # the affine state is in equilibrium
    assert rel(C, Cv) < 1e-14


@pytest.mark.parametrize("shape,h,seed", [((3, 3, 3), (1.0, 1.0, 1.0), 5), ((2, 3, 4), (1.0, 0.7, 1.3), 6)])
def test_dense_octant_energy_matches_pcg(shape, h, seed):
    C21 = synth.random_triclinic(shape, seed, soft=0.3)
    Cd = dense.ceff_dense_tri(C21, h)
    Cp, _ = ceff_tri(C21, h, rtol=1e-13)
    assert rel(Cp, Cd) < 1e-9
    assert rel(Cp, Cp.T) < 1e-9
    assert np.linalg.eigvalsh(0.5 * (Cp + Cp.T)).min() > 0


def _rotated_layers(axis, nlayers, seed):
    """Orthotropic materials (equal shear constants in the two planes that contain the
    stacking axis, so no coupling reaches the traction components) turned about the
    stacking axis by a different angle per layer."""
    rng = np.random.default_rng(seed)
    mats = []
    for q in range(nlayers):
        C11, C22, C33 = rng.uniform(40, 120, 3)
        C12, C13, C23 = rng.uniform(5, 30, 3)
        Gs = rng.uniform(10, 40, 3)  # C44 C55 C66
        pair = {0: (4, 5), 1: (3, 5), 2: (3, 4)}[axis]  # shears containing the stacking axis
        Gs[pair[1] - 3] = Gs[pair[0] - 3]
        C = np.array([[C11, C12, C13, 0, 0, 0], [C12, C22, C23, 0, 0, 0], [C13, C23, C33, 0, 0, 0],
                      [0, 0, 0, Gs[0], 0, 0], [0, 0, 0, 0, Gs[1], 0], [0, 0, 0, 0, 0, Gs[2]]])
        mats.append(cf.rotate_voigt(C, cf.rotation(axis, rng.uniform(0.2, 1.3))))
    return mats


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_rotated_laminate_is_the_exact_layer_average(axis):
    thick = [2, 1, 3]
    mats = _rotated_layers(axis, 3, 10 + axis)
    n_ax = sum(thick)
    shape = [3, 3, 3]                # (nz, ny, nx), the stacking axis gets n_ax cells
    shape[2 - axis] = n_ax
    C21 = np.empty((21,) + tuple(shape))
    pos = 0
    for t, M in zip(thick, mats):
        sl = [slice(None)] * 3
        sl[2 - axis] = slice(pos, pos + t)
        C21[(slice(None),) + tuple(sl)] = oracle.c21_of_voigt(M)[(slice(None),) + (None,) * 3]
        pos += t
    # every normal-shear coupling of the in-plane shear is present
    s_in = {0: 3, 1: 4, 2: 5}[axis]
    assert all(abs(M[r, s_in]) > 0.1 for M in mats for r in range(3))
    C, _ = ceff_tri(C21, rtol=1e-13)
    ref = cf.layered_average(thick, mats, axis)
    assert rel(C, ref) < 1e-10


def test_lattice_symmetries_triclinic():
    shape = (3, 5, 4)  # (nz, ny, nx)
    C21 = synth.random_triclinic(shape, 12, soft=0.25)
    C, _ = ceff_tri(C21, rtol=1e-13)
    assert rel(C, C.T) < 1e-9
    M = oracle.voigt_of_c21(C21)  # (6, 6, nz, ny, nx)

    def transformed(P, sgn, arr_axes, flip_x=False):
        Mt = M[np.ix_(P, P)] * np.outer(sgn, sgn)[:, :, None, None, None]
        Mt = np.transpose(Mt, (0, 1) + tuple(2 + a for a in arr_axes))
        if flip_x:
            Mt = Mt[..., ::-1]
        return np.ascontiguousarray(oracle.c21_of_voigt(Mt))

    one = np.ones(6)
    # swap x and y: Voigt indices 1<->2 and 4<->5 for the image and its constants
    P = [1, 0, 2, 4, 3, 5]
    Ct, _ = ceff_tri(transformed(P, one, (0, 2, 1)), rtol=1e-13)
    assert rel(Ct, C[np.ix_(P, P)]) < 1e-9
    # cyclic permutation: array axes (z, y, x) -> (y, x, z)
    Pc = [2, 0, 1, 5, 3, 4]
    Cc, _ = ceff_tri(transformed(Pc, one, (1, 2, 0)), rtol=1e-13)
    assert rel(Cc, C[np.ix_(Pc, Pc)]) < 1e-9
    # mirror x -> -x: constants and C* with one x index change sign
    s = np.array([1, 1, 1, 1, -1, -1])
    Cm, _ = ceff_tri(transformed(list(range(6)), s, (0, 1, 2), flip_x=True), rtol=1e-13)
    assert rel(Cm, C * np.outer(s, s)) < 1e-9


def test_triclinic_apt_converges_to_the_pcg_solution():
    C21 = synth.random_triclinic((5, 4, 6), 21, soft=0.2)
    for J in (1, 4):
        u, _, _ = oracle.solve_load_tri(C21, J, rtol=1e-13)
        v, _ = oracle.apt_disp_tri(C21, J, 4000, courant=0.95, strouhal=2.0)
        v = v - v.reshape(3, -1).mean(1)[:, None, None, None]
        assert np.max(np.abs(v - u)) < 1e-8 * np.max(np.abs(u)), J


def test_stress_state_iteration_matches_and_converges():
    """The stress-state APT iteration (stresses relaxed towards Hooke's law of the current
    strain, as in the paper's scheme) reproduces the displacement-form iterates on general
    cells step by step and converges to the PCG solution."""
    C21 = synth.random_triclinic((5, 4, 6), 22, soft=0.2)
    for J in (0, 3, 5):
        for k in (1, 2, 9):
            u, up = oracle.apt_stress(J, k, 0.95, 3.0, C21=C21)
            w, wp = oracle.apt_disp_tri(C21, J, k, 0.95, 3.0)
            assert np.max(np.abs(u - w)) <= 1e-12 * np.abs(w).max(), (J, k)
            assert np.max(np.abs(up - wp)) <= 1e-12 * np.abs(w).max(), (J, k)
    J = 4
    u_ref, _, _ = oracle.solve_load_tri(C21, J, rtol=1e-13)
    v, _ = oracle.apt_stress(J, 4000, 0.95, 2.0, C21=C21)
    v = v - v.reshape(3, -1).mean(1)[:, None, None, None]
    assert np.max(np.abs(v - u_ref)) < 1e-8 * np.max(np.abs(u_ref))
