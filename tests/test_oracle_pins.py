"""Pins of the CPU oracle against closed forms, invariants, brute force and
the paper's printed worked example (CPU only).

A plausible mistake in the oracle (a wrong neighbour, sign or modulus in the
strain, Hooke's law, the divergence or the averages) fails at least one of:
homogeneous exactness, Backus, Hill's identity, symmetry of C, lattice
symmetries, or agreement with the independently written dense solve.
"""
import json
import os

import numpy as np
import pytest

import closed_forms as cf
import oracle
import synth
from oracle import dense

GOLD = os.path.join(os.path.dirname(__file__), "golden")
IDX = {"C11": (0, 0), "C22": (1, 1), "C33": (2, 2), "C44": (3, 3), "C55": (4, 4), "C66": (5, 5),
       "C12": (0, 1), "C13": (0, 2), "C23": (1, 2)}


def rel(A, B):
    return np.max(np.abs(A - B)) / np.max(np.abs(B))


def test_homogeneous_is_exact():
    K = np.full((5, 6, 7), 70.0); G = np.full((5, 6, 7), 32.0)
    C, info = oracle.ceff(K, G, h=(1.0, 0.5, 2.0))
    np.testing.assert_allclose(C, cf.c_iso(70.0, 32.0), rtol=1e-14, atol=1e-12)
    assert all(it == 0 for it, _ in info.values())


@pytest.mark.parametrize("shape,seed", [((4, 3, 5), 1), ((3, 4, 3), 2)])
def test_pcg_matches_dense_energy_minimisation(shape, seed):
    K, G = synth.random_fields(shape, seed)
    Cd = dense.ceff_dense(K, G)
    Co, _ = oracle.ceff(K, G, rtol=1e-13)
    assert rel(Co, Cd) < 1e-10


def test_pcg_matches_dense_anisotropic_spacing():
    K, G = synth.random_fields((3, 4, 4), 7)
    h = (1.0, 0.7, 1.6)
    Cd = dense.ceff_dense(K, G, h)
    Co, _ = oracle.ceff(K, G, h=h, rtol=1e-13)
    assert rel(Co, Cd) < 1e-10


def test_residual_is_energy_gradient():
    """r = div sigma must equal minus the gradient of the strain energy."""
    K, G = synth.random_fields((3, 4, 3), 11)
    rng = np.random.default_rng(0)
    u = rng.standard_normal((3,) + K.shape)
    E = oracle.unit_strain(4) + 0.3 * oracle.unit_strain(0)
    r = oracle.residual(K, G, E, u)
    _, A = dense.solve_dense(K, G, E)
    e0 = dense.strain_field(np.zeros_like(u), E).reshape(6, -1)
    W = dense._energy_weights(K, G)
    B0 = np.stack([dense.strain_field(np.eye(u.size)[c].reshape(u.shape), np.zeros(6)).ravel()
                   for c in range(u.size)], 1)
    grad = A @ u.ravel() + B0.T @ W(e0).ravel()
    np.testing.assert_allclose(r.ravel(), -grad, rtol=1e-10, atol=1e-10 * np.abs(grad).max())


def test_laminate_is_backus_exact():
    Ks, Gs = [36.0, 7.2, 70.0], [44.0, 8.8, 32.0]
    ph = np.array([0, 0, 1, 2, 2, 2, 1, 0, 1, 1, 2, 0])
    nz = len(ph)
    K = np.broadcast_to(np.array(Ks)[ph][:, None, None], (nz, 3, 4)).copy()
    G = np.broadcast_to(np.array(Gs)[ph][:, None, None], (nz, 3, 4)).copy()
    C, _ = oracle.ceff(K, G, rtol=1e-13)
    f = np.bincount(ph, minlength=3) / nz
    np.testing.assert_allclose(C, cf.backus_z(f, Ks, Gs), rtol=0, atol=1e-9 * 112)


def test_paper_layered_model_analytic_column():
    """The paper's Model 1 geometry (191 voxels, six stiff 15-voxel layers) under
    periodic conditions gives its analytic column to every printed digit; the
    solution is uniform in x and y, so a 2 x 2 x 191 prism is the same problem."""
    g = json.load(open(os.path.join(GOLD, "table2_layered.json")))
    geo = g["geometry"]
    m = synth.laminate_z(2, 2, geo["n"], geo["stiff_layers"], geo["layer_thickness"],
                         stiff=(g["layers"]["stiff"]["K"], g["layers"]["stiff"]["G"]),
                         soft=(g["layers"]["soft"]["K"], g["layers"]["soft"]["G"]))
    assert round(m.info["f_stiff"], 4) == geo["stiff_fraction_printed"]
    K, G = m.fields()
    C, _ = oracle.ceff(K, G, rtol=1e-12)
    for name, val in g["analytic_GPa"].items():
        assert round(C[IDX[name]], g["printed_decimals"]) == pytest.approx(val, abs=1e-12), name


def test_hill_uniform_shear_identity():
    m = synth.centred_sphere(12, 3.5, inclusion=(2.2, 32.0))
    K, G = m.fields()
    C, _ = oracle.ceff(K, G, rtol=1e-12, loads=range(3))
    assert C[:3, :3].sum() / 9.0 == pytest.approx(cf.hill_uniform_shear(K, G), rel=1e-10)


@pytest.fixture(scope="module")
def sphere12():
    m = synth.centred_sphere(12, 3.0)
    K, G = m.fields()
    C, info = oracle.ceff(K, G, rtol=1e-12)
    return K, G, C


def test_symmetric(sphere12):
    _, _, C = sphere12
    assert np.max(np.abs(C - C.T)) < 1e-9 * np.abs(C).max()


def test_symmetric_random_field():
    K, G = synth.random_fields((5, 6, 4), 5)
    C, _ = oracle.ceff(K, G, rtol=1e-12)
    assert np.max(np.abs(C - C.T)) < 1e-9 * np.abs(C).max()


def test_voigt_reuss_bounds(sphere12):
    K, G, C = sphere12
    Cs = 0.5 * (C + C.T)
    w = cf._mandel_weights()
    M = lambda X: X * np.outer(w, w)
    assert np.linalg.eigvalsh(M(cf.voigt_bound(K, G)) - M(Cs)).min() > -1e-10 * np.abs(C).max()
    assert np.linalg.eigvalsh(M(Cs) - M(cf.reuss_bound(K, G))).min() > -1e-10 * np.abs(C).max()


def test_hashin_shtrikman_bulk(sphere12):
    K, G, C = sphere12
    phi = float(np.mean(G < 1.0))
    b = cf.hashin_shtrikman(phi, 70.0, 32.0, 2.2, 1e-3)
    Kp, Gp = cf.isotropic_projection(C)
    assert b["K_lower"] <= Kp <= b["K_upper"]
    assert Gp <= b["G_upper"]


def test_lattice_symmetries():
    K, G = synth.random_fields((4, 5, 3), 9)          # shape (nz, ny, nx) = (3, 5, 4)
    C, _ = oracle.ceff(K, G, rtol=1e-13)
    # periodic roll of the image: C unchanged
    Cr, _ = oracle.ceff(np.roll(K, (1, 2, 3), (0, 1, 2)), np.roll(G, (1, 2, 3), (0, 1, 2)), rtol=1e-13)
    assert rel(Cr, C) < 1e-10
    # scaling both moduli scales C
    Cs, _ = oracle.ceff(2.5 * K, 2.5 * G, rtol=1e-13)
    assert rel(Cs, 2.5 * C) < 1e-10
    # swap the x and y axes: Voigt indices 1<->2 and 4<->5
    Kt = np.ascontiguousarray(np.swapaxes(K, 1, 2)); Gt = np.ascontiguousarray(np.swapaxes(G, 1, 2))
    Ct, _ = oracle.ceff(Kt, Gt, rtol=1e-13)
    P = [1, 0, 2, 4, 3, 5]
    assert rel(Ct, C[np.ix_(P, P)]) < 1e-10
    # cyclic permutation x->y->z->x of the axes
    Kc = np.ascontiguousarray(np.transpose(K, (1, 2, 0))); Gc = np.ascontiguousarray(np.transpose(G, (1, 2, 0)))
    Cc, _ = oracle.ceff(Kc, Gc, rtol=1e-13)
    # array axes (z, y, x) -> (y, x, z): the new x' is the old z, y' the old x,
    # z' the old y; Pc lists the old Voigt index of each new one
    Pc = [2, 0, 1, 5, 3, 4]
    assert rel(Cc, C[np.ix_(Pc, Pc)]) < 1e-10
    # mirror x -> -x (reverse the x axis and shift by one cell so the
    # staggered positions map onto themselves): couplings with one x index flip sign
    Km = np.ascontiguousarray(K[:, :, ::-1]); Gm = np.ascontiguousarray(G[:, :, ::-1])
    Cm, _ = oracle.ceff(Km, Gm, rtol=1e-13)
    s = np.array([1, 1, 1, 1, -1, -1])
    assert rel(Cm, C * np.outer(s, s)) < 1e-10


def test_apt_fixed_point_is_the_solution():
    """The paper-form APT iteration converges to the same displacement as PCG."""
    K, G = synth.random_fields((4, 5, 6), 3, lo=(10.0, 5.0), hi=(80.0, 40.0))
    for J in (0, 4):
        u, it, rel_ = oracle.solve_load(K, G, J, rtol=1e-13)
        st = oracle.apt_steps(K, G, J, 3000, courant=0.95, strouhal=4.0)
        v = st["v"] - st["v"].reshape(3, -1).mean(1)[:, None, None, None]
        assert np.max(np.abs(v - u)) < 1e-9 * np.max(np.abs(u))
        # at the fixed point the APT stresses equal Hooke's law of the displacement
        sig = oracle.stress(K, G, oracle.unit_strain(J), st["v"])
        np.testing.assert_allclose(-st["p"] + st["txx"], sig[0], atol=1e-9 * np.abs(sig).max())
        np.testing.assert_allclose(st["txy"], sig[5], atol=1e-9 * np.abs(sig).max())


def test_apt_homogeneous_stays_put():
    K = np.full((4, 4, 4), 70.0); G = np.full((4, 4, 4), 32.0)
    st = oracle.apt_steps(K, G, 3, 20, courant=0.95, strouhal=10.0)
    assert np.all(st["v"] == 0.0)
    assert np.allclose(st["tyz"], 32.0)


def test_apt_trace_free_deviator():
    K, G = synth.random_fields((5, 4, 3), 4)
    st = oracle.apt_steps(K, G, 0, 25, courant=0.95, strouhal=5.0)
    assert np.max(np.abs(st["txx"] + st["tyy"] + st["tzz"])) < 1e-12 * np.abs(st["txx"]).max()


def _six_fields(K, G, rtol=1e-13):
    C, info, fields = oracle.ceff(K, G, rtol=rtol, return_fields=True)
    return C, fields


def test_gradient_matches_central_differences():
    K, G = synth.random_fields((3, 4, 3), 21, lo=(5.0, 3.0), hi=(60.0, 40.0))
    C, fields = _six_fields(K, G)
    rng = np.random.default_rng(1)
    W = rng.standard_normal((6, 6))
    dK, dG = oracle.gradient(K, G, fields, W)
    J = lambda C_: float(np.sum(W * C_))
    for c in [(0, 0, 0), (1, 2, 1), (2, 3, 2), (1, 0, 2)]:
        for which, grad in (("K", dK), ("G", dG)):
            step = 1e-4 * (K if which == "K" else G)[c]
            vals = []
            for sgn in (+1, -1):
                K2, G2 = K.copy(), G.copy()
                (K2 if which == "K" else G2)[c] += sgn * step
                vals.append(J(oracle.ceff(K2, G2, rtol=1e-13)[0]))
            fd = (vals[0] - vals[1]) / (2 * step)
            assert grad[c] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(J(C))), (which, c)


def test_gradient_euler_homogeneity():
    """C is homogeneous of degree one in the moduli: sum K dC/dK + G dC/dG = C."""
    K, G = synth.random_fields((4, 3, 5), 8)
    C, fields = _six_fields(K, G)
    for (I, Jx) in [(0, 0), (3, 3), (0, 2), (1, 4)]:
        W = np.zeros((6, 6)); W[I, Jx] = 1.0
        dK, dG = oracle.gradient(K, G, fields, W)
        assert np.sum(K * dK + G * dG) == pytest.approx(C[I, Jx], rel=1e-9, abs=1e-10 * np.abs(C).max())


def test_dilute_sphere_contribution_converges_to_eshelby():
    """A voxel sphere of radius r in a periodic box of side 6r (porosity about 2%, so the
    interaction between images is small): its stiffness contribution (C* - C_m)/phi
    approaches Eshelby's dilute sphere value -C_m H C_m (the phi -> 0 slope of the
    non-interacting estimate, paper section 4.2) at first order in 1/r, the order of the
    staircase boundary: the relative error falls with r and r times it stays constant."""
    Cm = cf.c_iso(70.0, 32.0)
    Ci = cf.c_iso(2.2, 1e-3)
    eps = 1e-7
    N_esh = (cf.noninteracting_stiffness(Cm, Ci, 1.0, eps) - Cm) / eps
    radii = (2.0, 3.0, 4.0, 5.0)
    errs = {k: [] for k in ((0, 0), (1, 0), (3, 3))}
    for r in radii:
        m = synth.centred_sphere(int(round(6 * r)), r)
        K, G = m.fields()
        C, _ = oracle.ceff(K, G, rtol=1e-9, loads=[0, 3])
        N = (C - Cm) / m.info["phi"]
        for (i, j) in errs:
            errs[(i, j)].append(N[i, j] / N_esh[i, j] - 1.0)
    for k, e in errs.items():
        e = np.array(e)
        assert np.all(e > 0) and np.all(np.diff(e) < 0), (k, e)  # the staircase sphere is softer, less so as r grows
        re = e * np.array(radii)
        assert re.max() / re.min() < 1.25, (k, re)  # first order in 1/r
