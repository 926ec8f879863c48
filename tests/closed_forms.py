"""Closed-form results used to pin the oracle (test helpers only).

Everything here is written from textbook micromechanics, independently of the
oracle and of the GPU library:

* isotropic stiffness / compliance in Voigt notation;
* Backus (1962) long-wave average of a stack of isotropic layers (paper,
  "Model 1": the analytic column of the layered-media table);
* Voigt and Reuss bounds; Hashin-Shtrikman bounds for two isotropic phases;
* Hill's exact result for the bulk response when all phases share one shear
  modulus;
* rotation of a Voigt stiffness (through the fourth-order tensor) and the
  exact long-wave average of a stack of anisotropic layers (Schoenberg and
  Muir's partition into the components continuous across the layering and the
  rest), which reduces to Backus for isotropic layers;
* Eshelby's tensor of a spheroid (Mura's expressions in terms of the
  ellipsoid I-integrals, evaluated by quadrature) and the compliance
  contribution tensor H = [(S2 - S1)^-1 + Q]^-1, Q = C1 : (I - s)
  (paper, appendix "Property contribution tensor H", eqs. N21-N23), used with
  S* = S1 + phi H (paper, "Model 2").
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import integrate

VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def c_iso(K, G):
    lam = K - 2.0 * G / 3.0
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    for i in range(3):
        C[i, i] = lam + 2.0 * G
        C[3 + i, 3 + i] = G
    return C


def backus_z(fracs, Ks, Gs):
    """Effective Voigt stiffness of isotropic layers stacked along z."""
    f = np.asarray(fracs, float); f = f / f.sum()
    K = np.asarray(Ks, float); G = np.asarray(Gs, float)
    lam = K - 2.0 * G / 3.0
    M = lam + 2.0 * G
    avg = lambda a: float(np.sum(f * a))
    C33 = 1.0 / avg(1.0 / M)
    C13 = avg(lam / M) * C33
    C11 = avg(4.0 * G * (lam + G) / M) + avg(lam / M) ** 2 * C33
    C66 = avg(G)
    C12 = C11 - 2.0 * C66
    C44 = 1.0 / avg(1.0 / G)
    C = np.zeros((6, 6))
    C[0, 0] = C[1, 1] = C11; C[2, 2] = C33
    C[0, 1] = C[1, 0] = C12
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = C13
    C[3, 3] = C[4, 4] = C44; C[5, 5] = C66
    return C


def backus_z_ortho(fracs, Cs):
    """Effective Voigt stiffness of orthotropic layers (axes aligned) stacked along z.
    The in-plane strains (11, 22, 12) and the tractions (33, 13, 23) are the same in every
    layer; eliminating the layer strains eps33, eps13, eps23 gives the averages below."""
    f = np.asarray(fracs, float); f = f / f.sum()
    avg = lambda a: float(np.sum(f * np.asarray(a, float)))
    C = [np.asarray(c, float) for c in Cs]
    g = lambda I, J: np.array([c[I, J] for c in C])
    C33 = 1.0 / avg(1.0 / g(2, 2))
    a13 = avg(g(0, 2) / g(2, 2)); a23 = avg(g(1, 2) / g(2, 2))
    out = np.zeros((6, 6))
    out[2, 2] = C33
    out[0, 2] = out[2, 0] = C33 * a13
    out[1, 2] = out[2, 1] = C33 * a23
    out[0, 0] = avg(g(0, 0) - g(0, 2) ** 2 / g(2, 2)) + C33 * a13 ** 2
    out[1, 1] = avg(g(1, 1) - g(1, 2) ** 2 / g(2, 2)) + C33 * a23 ** 2
    out[0, 1] = out[1, 0] = avg(g(0, 1) - g(0, 2) * g(1, 2) / g(2, 2)) + C33 * a13 * a23
    out[3, 3] = 1.0 / avg(1.0 / g(3, 3))
    out[4, 4] = 1.0 / avg(1.0 / g(4, 4))
    out[5, 5] = avg(g(5, 5))
    return out


def voigt_bound(K, G):
    """Arithmetic mean of the local stiffness (per-voxel fields)."""
    return c_iso(np.mean(K), np.mean(G))


def reuss_bound(K, G):
    """Inverse of the mean local compliance."""
    S = np.zeros((6, 6))
    Ks, Gs = np.ravel(K), np.ravel(G)
    vals, inv = np.unique(np.stack([Ks, Gs], 1), axis=0, return_inverse=True)
    cnt = np.bincount(np.ravel(inv), minlength=len(vals))
    for (k, g), c in zip(vals, cnt):
        S += c * np.linalg.inv(c_iso(k, g))
    return np.linalg.inv(S / Ks.size)


def hashin_shtrikman(f2, K1, G1, K2, G2):
    """HS bounds (lower, upper) on the bulk and shear moduli of two isotropic phases."""
    f1 = 1.0 - f2
    def bounds(Km, Gm, Ki, Gi, fi, fm):
        K = Km if Ki == Km else Km + fi / (1.0 / (Ki - Km) + fm / (Km + 4.0 * Gm / 3.0))
        G = Gm if Gi == Gm else Gm + fi / (1.0 / (Gi - Gm) + 2.0 * fm * (Km + 2.0 * Gm) /
                                           (5.0 * Gm * (Km + 4.0 * Gm / 3.0)))
        return K, G
    # the stiffer phase as reference gives the upper bound (well-ordered phases)
    if K1 >= K2 and G1 >= G2:
        up = bounds(K1, G1, K2, G2, f2, f1); lo = bounds(K2, G2, K1, G1, f1, f2)
    else:
        up = bounds(K2, G2, K1, G1, f1, f2); lo = bounds(K1, G1, K2, G2, f2, f1)
    return {"K_lower": lo[0], "K_upper": up[0], "G_lower": lo[1], "G_upper": up[1]}


def hill_uniform_shear(K, G):
    """Exact mean bulk response when G is uniform: (1/9) sum_{i,j<=3} C_ij."""
    G0 = float(np.ravel(G)[0])
    return 1.0 / np.mean(1.0 / (np.ravel(K) + 4.0 * G0 / 3.0)) - 4.0 * G0 / 3.0


def isotropic_projection(C):
    """Bulk and shear moduli of the isotropic part of a Voigt stiffness."""
    Kp = C[:3, :3].sum() / 9.0
    Gp = (C[0, 0] + C[1, 1] + C[2, 2] - C[0, 1] - C[0, 2] - C[1, 2] + 3.0 * (C[3, 3] + C[4, 4] + C[5, 5])) / 15.0
    return Kp, Gp


# ---- fourth-rank tensor helpers (full 3x3x3x3) ---------------------------------

def _mandel_weights():
    return np.array([1, 1, 1, math.sqrt(2), math.sqrt(2), math.sqrt(2)])


def tensor_to_mandel(T):
    w = _mandel_weights()
    M = np.empty((6, 6))
    for I, (i, j) in enumerate(VOIGT):
        for J, (k, l) in enumerate(VOIGT):
            M[I, J] = w[I] * w[J] * T[i, j, k, l]
    return M


def mandel_to_tensor(M):
    w = _mandel_weights()
    T = np.empty((3, 3, 3, 3))
    for I, (i, j) in enumerate(VOIGT):
        for J, (k, l) in enumerate(VOIGT):
            v = M[I, J] / (w[I] * w[J])
            for a, b in {(i, j), (j, i)}:
                for c, d in {(k, l), (l, k)}:
                    T[a, b, c, d] = v
    return T


def voigt_stiffness_to_mandel(C):
    w = _mandel_weights()
    return C * np.outer(w, w)


def mandel_to_voigt_stiffness(M):
    w = _mandel_weights()
    return M / np.outer(w, w)


def _I_integrals(a):
    """I_i and I_ij for an ellipsoid with semi-axes a (Mura, sect. 11)."""
    a = np.asarray(a, float)
    pref = 2.0 * math.pi * a[0] * a[1] * a[2]
    def delta(s):
        return math.sqrt((a[0] ** 2 + s) * (a[1] ** 2 + s) * (a[2] ** 2 + s))
    # split the half line at the squared semi-axes: the integrands change
    # scale there, which a single adaptive pass misses for flat ellipsoids
    cuts = sorted({0.0, *(float(x) ** 2 for x in a)})
    cuts.append(10.0 * cuts[-1])

    def quad(f):
        tot = 0.0
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            tot += integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-12, limit=500)[0]
        return tot + integrate.quad(f, cuts[-1], np.inf, epsabs=0, epsrel=1e-12, limit=500)[0]
    I = np.empty(3); II = np.empty((3, 3))
    for i in range(3):
        I[i] = pref * quad(lambda s: 1.0 / ((a[i] ** 2 + s) * delta(s)))
        for j in range(3):
            II[i, j] = pref * quad(lambda s: 1.0 / ((a[i] ** 2 + s) * (a[j] ** 2 + s) * delta(s)))
    return I, II


def eshelby_tensor(a, nu):
    """Eshelby's interior tensor s_ijkl of an ellipsoid (semi-axes a) in an isotropic
    matrix of Poisson ratio nu (Mura's formulas; full 3x3x3x3)."""
    a = np.asarray(a, float)
    I, II = _I_integrals(a)
    c1 = 1.0 / (8.0 * math.pi * (1.0 - nu))
    S = np.zeros((3, 3, 3, 3))
    for i, j in itertools.product(range(3), range(3)):
        if i == j:
            S[i, i, i, i] = 3.0 * c1 * a[i] ** 2 * II[i, i] + (1.0 - 2.0 * nu) * c1 * I[i]
        else:
            S[i, i, j, j] = c1 * a[j] ** 2 * II[i, j] - (1.0 - 2.0 * nu) * c1 * I[i]
            val = c1 / 2.0 * (a[i] ** 2 + a[j] ** 2) * II[i, j] + (1.0 - 2.0 * nu) * c1 / 2.0 * (I[i] + I[j])
            S[i, j, i, j] = S[i, j, j, i] = S[j, i, i, j] = S[j, i, j, i] = val
    return S


def compliance_contribution(C1_voigt, C2_voigt, s_tensor):
    """H = [(S2 - S1)^-1 + Q]^-1 with Q = C1 : (I4 - s), all in Mandel form (6x6)."""
    C1 = voigt_stiffness_to_mandel(C1_voigt)
    C2 = voigt_stiffness_to_mandel(C2_voigt)
    S1 = np.linalg.inv(C1); S2 = np.linalg.inv(C2)
    s = tensor_to_mandel(s_tensor)
    Q = C1 @ (np.eye(6) - s)
    return np.linalg.inv(np.linalg.inv(S2 - S1) + Q)


def noninteracting_stiffness(C1_voigt, C2_voigt, aspect, phi, axis=2):
    """C* = (S1 + phi H)^-1 (Voigt) for a spheroid with symmetry axis `axis`."""
    K1 = C1_voigt[:3, :3].sum() / 9.0
    G1 = C1_voigt[3, 3]
    nu = (3.0 * K1 - 2.0 * G1) / (2.0 * (3.0 * K1 + G1))
    a = np.ones(3); a[axis] = aspect
    s = eshelby_tensor(a, nu)
    H = compliance_contribution(C1_voigt, C2_voigt, s)
    S1 = np.linalg.inv(voigt_stiffness_to_mandel(C1_voigt))
    return mandel_to_voigt_stiffness(np.linalg.inv(S1 + phi * H))


def voigt_to_tensor4(C):
    """c_ijkl of a Voigt stiffness with engineering shear."""
    T = np.zeros((3, 3, 3, 3))
    for I, (i, j) in enumerate(VOIGT):
        for J, (k, l) in enumerate(VOIGT):
            for a, b in {(i, j), (j, i)}:
                for c, d in {(k, l), (l, k)}:
                    T[a, b, c, d] = C[I, J]
    return T


def tensor4_to_voigt(T):
    return np.array([[T[i, j, k, l] for (k, l) in VOIGT] for (i, j) in VOIGT])


def rotate_voigt(C, R):
    """Stiffness of a material whose axes are turned by the rotation matrix R:
    c'_ijkl = R_ia R_jb R_kc R_ld c_abcd."""
    return tensor4_to_voigt(np.einsum("ia,jb,kc,ld,abcd->ijkl", R, R, R, R, voigt_to_tensor4(C)))


def rotation(axis, theta):
    c, s = math.cos(theta), math.sin(theta)
    i, j = [(1, 2), (2, 0), (0, 1)][axis]
    R = np.eye(3)
    R[i, i], R[i, j], R[j, i], R[j, j] = c, -s, s, c
    return R


# Voigt components continuous in stress (the traction on the layer planes) for
# layers stacked along x, y, z; the others (the in-plane strains) are continuous
# in strain.
_TRACTION = {0: [0, 4, 5], 1: [1, 3, 5], 2: [2, 3, 4]}


def layered_average(fracs, Cs, axis):
    """Exact effective stiffness (6x6 Voigt) of a periodic stack of homogeneous
    anisotropic layers with volume fractions fracs and stiffnesses Cs, stacked
    along `axis`.  With n the traction components and t the in-plane strain
    components, each layer's eps_t equals the mean and its sigma_n is common:
        C_nn* = <C_nn^-1>^-1,   C_nt* = C_nn* <C_nn^-1 C_nt>,
        C_tt* = <C_tt - C_tn C_nn^-1 C_nt> + <C_tn C_nn^-1> C_nn* <C_nn^-1 C_nt>."""
    n = _TRACTION[axis]
    t = [q for q in range(6) if q not in n]
    f = np.asarray(fracs, float) / np.sum(fracs)
    inv = lambda A: np.linalg.inv(A)
    Snn = sum(fk * inv(C[np.ix_(n, n)]) for fk, C in zip(f, Cs))
    Cnn = inv(Snn)
    A = sum(fk * inv(C[np.ix_(n, n)]) @ C[np.ix_(n, t)] for fk, C in zip(f, Cs))
    B = sum(fk * C[np.ix_(t, n)] @ inv(C[np.ix_(n, n)]) for fk, C in zip(f, Cs))
    T0 = sum(fk * (C[np.ix_(t, t)] - C[np.ix_(t, n)] @ inv(C[np.ix_(n, n)]) @ C[np.ix_(n, t)])
             for fk, C in zip(f, Cs))
    out = np.zeros((6, 6))
    out[np.ix_(n, n)] = Cnn
    out[np.ix_(n, t)] = Cnn @ A
    out[np.ix_(t, n)] = B @ Cnn
    out[np.ix_(t, t)] = T0 + B @ Cnn @ A
    return out
