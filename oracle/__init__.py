"""CPU oracle for periodic voxel-grid elastic homogenisation -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library (the HIP path)
never imports, links or calls it, and it shares no code with it.

Contents
--------
* ``ceff_oracle.c`` (loaded through ctypes): FP64 operator, Jacobi-PCG solve,
  stress averages, the paper-form APT iteration (``apt_steps``, also under the
  wall tests), the stress-state APT iteration for every cell law
  (``apt_stress``), the displacement-form APT iteration (``apt_disp``) and the
  closed-form gradient; isotropic (K, G) cells, orthotropic cells with nine
  constants (``*_ortho``), general cells with 21 constants (``*_tri``) and the
  wall tests (``*_walls``).
* ``dense.py``: brute-force dense solve for tiny grids, assembled from the
  strain energy alone (an independent route to the same discrete problem).

Conventions: fields are numpy arrays shaped (nz, ny, nx) (x fastest);
vector fields (3, nz, ny, nx); Voigt order 11, 22, 33, 23, 13, 12 with
engineering shear strain, so unit load J = 4 sets eps_yz = eps_zy = 1/2.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        L.or_stress.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_residual.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_average_stress.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_pcg.argtypes = [_ip, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int64, _dp, _dp, _dp, ctypes.c_int64]
        L.or_pcg.restype = ctypes.c_int64
        L.or_apt_steps.argtypes = [_ip, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int64, _dp]
        L.or_apt_stress.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, _dp, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int64, _dp, _dp]
        L.or_apt_steps_walls.argtypes = [_ip, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_int64, _dp, _dp, ctypes.c_int]
        L.or_gradient.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_stress_ortho.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
        L.or_residual_ortho.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
        L.or_average_stress_ortho.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
        L.or_pcg_ortho.argtypes = [_ip, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int64, _dp, _dp, _dp,
                                   ctypes.c_int64]
        L.or_pcg_ortho.restype = ctypes.c_int64
        L.or_apt_disp.argtypes = [_ip, _dp, _dp, _dp, _dp, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int64, _dp, _dp]
        L.or_stress_tri.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
        L.or_residual_tri.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
        L.or_average_stress_tri.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
        L.or_pcg_tri.argtypes = [_ip, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int64, _dp, _dp]
        L.or_pcg_tri.restype = ctypes.c_int64
        L.or_apt_disp_tri.argtypes = [_ip, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int64, _dp,
                                      _dp]
        L.or_residual_walls.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
        L.or_average_stress_walls.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
        L.or_pcg_walls.argtypes = [_ip, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int64, _dp, _dp, ctypes.c_int]
        L.or_pcg_walls.restype = ctypes.c_int64
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _prep(K, G, h):
    K = np.ascontiguousarray(K, np.float64)
    G = np.ascontiguousarray(G, np.float64)
    if K.shape != G.shape or K.ndim != 3:
        raise ValueError("K and G must be 3-D arrays of the same shape (nz, ny, nx)")
    if not (np.all(K > 0) and np.all(G > 0)):
        raise ValueError("moduli must be positive")
    nz, ny, nx = K.shape
    dims = np.array([nx, ny, nz], np.int64)
    hh = np.array(h, np.float64)
    return K, G, dims, hh


def unit_strain(J: int) -> np.ndarray:
    """Tensor components (xx, yy, zz, yz, xz, xy) of the J-th unit Voigt strain (J = 0..5)."""
    E = np.zeros(6)
    E[J] = 1.0 if J < 3 else 0.5
    return E


def stress(K, G, E, u, h=(1.0, 1.0, 1.0)):
    """Stresses (6, nz, ny, nx): xx, yy, zz at cells; yz, xz, xy at edges."""
    K, G, dims, hh = _prep(K, G, h)
    u = np.ascontiguousarray(u, np.float64).reshape((3,) + K.shape)
    out = np.empty((6,) + K.shape)
    lib().or_stress(dims.ctypes.data_as(_ip), _d(hh), _d(K), _d(G), _d(np.asarray(E, np.float64)), _d(u), _d(out))
    return out


def residual(K, G, E, u, h=(1.0, 1.0, 1.0)):
    """Out-of-balance force div(C:(E + grad u)) at faces, shape (3, nz, ny, nx)."""
    K, G, dims, hh = _prep(K, G, h)
    u = np.ascontiguousarray(u, np.float64).reshape((3,) + K.shape)
    out = np.empty((3,) + K.shape)
    lib().or_residual(dims.ctypes.data_as(_ip), _d(hh), _d(K), _d(G), _d(np.asarray(E, np.float64)), _d(u), _d(out))
    return out


def average_stress(K, G, E, u, h=(1.0, 1.0, 1.0)):
    """Volume-averaged stress in Voigt order (6,)."""
    K, G, dims, hh = _prep(K, G, h)
    u = np.ascontiguousarray(u, np.float64).reshape((3,) + K.shape)
    out = np.empty(6)
    lib().or_average_stress(dims.ctypes.data_as(_ip), _d(hh), _d(K), _d(G), _d(np.asarray(E, np.float64)), _d(u), _d(out))
    return out


def solve_load(K, G, J, h=(1.0, 1.0, 1.0), rtol=1e-11, max_iter=1_000_000, u0=None, want_hist=False):
    """Jacobi-PCG solve for unit load J.  Returns (u, iters, relres[, hist])."""
    K, G, dims, hh = _prep(K, G, h)
    u = np.zeros((3,) + K.shape) if u0 is None else np.array(u0, np.float64).reshape((3,) + K.shape)
    rel = np.zeros(1)
    cap = 200_000 if want_hist else 0
    hist = np.zeros(max(cap, 1))
    it = lib().or_pcg(dims.ctypes.data_as(_ip), _d(hh), _d(K), _d(G), _d(unit_strain(J)), rtol, max_iter,
                      _d(u), _d(rel), _d(hist) if cap else None, cap)
    if want_hist:
        return u, int(it), float(rel[0]), hist[:min(it + 1, cap)]
    return u, int(it), float(rel[0])


def ceff(K, G, h=(1.0, 1.0, 1.0), rtol=1e-11, loads=range(6), return_fields=False, max_iter=1_000_000):
    """Effective stiffness (6x6, FP64): column J = volume-averaged stress under unit load J."""
    C = np.full((6, 6), np.nan)
    fields = {}
    info = {}
    for J in loads:
        u, it, rel = solve_load(K, G, J, h, rtol, max_iter)
        C[:, J] = average_stress(K, G, unit_strain(J), u, h)
        info[J] = (it, rel)
        if return_fields:
            fields[J] = u
    if return_fields:
        return C, info, fields
    return C, info


def apt_steps(K, G, J, nsteps, courant, strouhal, h=(1.0, 1.0, 1.0), state=None, walls=False):
    """Run `nsteps` APT iterations in the paper's (p, tau, v) variables.

    Returns the state dict {p, txx, tyy, tzz, tyz, txz, txy, v} after the
    steps.  With state=None the iteration starts from the affine initial
    state (v = 0, stresses of the uniform strain).  walls: the wall test of
    load J (normal test for J < 3, simple-shear test for J >= 3); the state
    then also holds "half1", the side-1 halves of the split edges (indexed
    like the edge field)."""
    K, G, dims, hh = _prep(K, G, h)
    N = K.size
    sh = K.shape
    init = 1 if state is None else 0
    buf = np.zeros(10 * N) if state is None else np.concatenate([
        state[k].ravel() for k in ("p", "txx", "tyy", "tzz", "tyz", "txz", "txy")] + [state["v"].ravel()])
    buf = np.ascontiguousarray(buf)
    if walls:
        half1 = np.zeros(N) if state is None else np.ascontiguousarray(state["half1"], np.float64).ravel().copy()
        lib().or_apt_steps_walls(dims.ctypes.data_as(_ip), _d(hh), _d(K), _d(G), _d(unit_strain(J)), courant,
                                 strouhal, init, nsteps, _d(buf), _d(half1), wall_mode(J))
    else:
        lib().or_apt_steps(dims.ctypes.data_as(_ip), _d(hh), _d(K), _d(G), _d(unit_strain(J)), courant, strouhal,
                           init, nsteps, _d(buf))
    names = ("p", "txx", "tyy", "tzz", "tyz", "txz", "txy")
    out = {nm: buf[i * N:(i + 1) * N].reshape(sh).copy() for i, nm in enumerate(names)}
    out["v"] = buf[7 * N:].reshape((3,) + sh).copy()
    if walls:
        out["half1"] = half1.reshape(sh).copy()
    return out


# ---- orthotropic cells (nine constants per cell) -----------------------------------
#
# C9 is shaped (9, nz, ny, nx): C11 C22 C33 C23 C13 C12 C44 C55 C66 of each cell
# (Voigt, engineering shear), axes aligned with the grid.

def iso_to_c9(K, G):
    """The nine orthotropic constants of isotropic cells (K, G)."""
    K = np.asarray(K, np.float64); G = np.asarray(G, np.float64)
    a = K + 4.0 * G / 3.0
    b = K - 2.0 * G / 3.0
    return np.stack([a, a, a, b, b, b, G, G, G])


def voigt_of_c9(c):
    """6x6 Voigt stiffness of one cell's nine constants."""
    C11, C22, C33, C23, C13, C12, C44, C55, C66 = c
    return np.array([[C11, C12, C13, 0, 0, 0], [C12, C22, C23, 0, 0, 0], [C13, C23, C33, 0, 0, 0],
                     [0, 0, 0, C44, 0, 0], [0, 0, 0, 0, C55, 0], [0, 0, 0, 0, 0, C66]], float)


def _prep9(C9, h):
    C9 = np.ascontiguousarray(C9, np.float64)
    if C9.ndim != 4 or C9.shape[0] != 9:
        raise ValueError("C9 must be shaped (9, nz, ny, nx)")
    if not np.all(C9[[0, 1, 2, 6, 7, 8]] > 0):
        raise ValueError("diagonal constants must be positive")
    nz, ny, nx = C9.shape[1:]
    return C9, np.array([nx, ny, nz], np.int64), np.array(h, np.float64)


def stress_ortho(C9, E, u, h=(1.0, 1.0, 1.0)):
    C9, dims, hh = _prep9(C9, h)
    sh = C9.shape[1:]
    u = np.ascontiguousarray(u, np.float64).reshape((3,) + sh)
    out = np.empty((6,) + sh)
    lib().or_stress_ortho(dims.ctypes.data_as(_ip), _d(hh), _d(C9), _d(np.asarray(E, np.float64)), _d(u), _d(out))
    return out


def residual_ortho(C9, E, u, h=(1.0, 1.0, 1.0)):
    C9, dims, hh = _prep9(C9, h)
    sh = C9.shape[1:]
    u = np.ascontiguousarray(u, np.float64).reshape((3,) + sh)
    out = np.empty((3,) + sh)
    lib().or_residual_ortho(dims.ctypes.data_as(_ip), _d(hh), _d(C9), _d(np.asarray(E, np.float64)), _d(u), _d(out))
    return out


def average_stress_ortho(C9, E, u, h=(1.0, 1.0, 1.0)):
    C9, dims, hh = _prep9(C9, h)
    u = np.ascontiguousarray(u, np.float64).reshape((3,) + C9.shape[1:])
    out = np.empty(6)
    lib().or_average_stress_ortho(dims.ctypes.data_as(_ip), _d(hh), _d(C9), _d(np.asarray(E, np.float64)), _d(u),
                                  _d(out))
    return out


def solve_load_ortho(C9, J, h=(1.0, 1.0, 1.0), rtol=1e-11, max_iter=1_000_000):
    C9, dims, hh = _prep9(C9, h)
    u = np.zeros((3,) + C9.shape[1:])
    rel = np.zeros(1)
    it = lib().or_pcg_ortho(dims.ctypes.data_as(_ip), _d(hh), _d(C9), _d(unit_strain(J)), rtol, max_iter, _d(u),
                            _d(rel), None, 0)
    return u, int(it), float(rel[0])


def ceff_ortho(C9, h=(1.0, 1.0, 1.0), rtol=1e-11, loads=range(6), max_iter=1_000_000):
    """Effective stiffness (6x6) of an image of orthotropic cells."""
    C = np.full((6, 6), np.nan)
    info = {}
    for J in loads:
        u, it, rel = solve_load_ortho(C9, J, h, rtol, max_iter)
        C[:, J] = average_stress_ortho(C9, unit_strain(J), u, h)
        info[J] = (it, rel)
    return C, info


def apt_disp(J, nsteps, courant, strouhal, K=None, G=None, C9=None, h=(1.0, 1.0, 1.0), walls=False):
    """Displacement-form APT iterate u^nsteps and u^(nsteps-1) (each (3, nz, ny, nx)) for
    isotropic (K, G) or orthotropic (C9) cells, from u^0 = 0; walls: the wall test of
    load J (normal test for J < 3, simple-shear test for J >= 3)."""
    if C9 is not None:
        C9, dims, hh = _prep9(C9, h)
        sh = C9.shape[1:]
        Kp = Gp = None
        cp = _d(C9)
    else:
        K, G, dims, hh = _prep(K, G, h)
        sh = K.shape
        Kp, Gp, cp = _d(K), _d(G), None
    u = np.empty((3,) + sh)
    up = np.empty((3,) + sh)
    lib().or_apt_disp(dims.ctypes.data_as(_ip), _d(hh), Kp, Gp, cp, wall_mode(J) if walls else 0, _d(unit_strain(J)), courant,
                      strouhal, nsteps, _d(u), _d(up))
    return u, up


# ---- general anisotropic cells (21 constants per cell) ------------------------------
#
# C21 is shaped (21, nz, ny, nx): the upper triangle of each cell's symmetric 6x6
# Voigt stiffness (engineering shear), row by row: C11 C12 C13 C14 C15 C16 C22 C23
# C24 C25 C26 C33 C34 C35 C36 C44 C45 C46 C55 C56 C66.  The coupled law's reading
# on the staggered grid (eight corner octants per cell, series-weighted edge
# strains) is described in ceff_oracle.c.

TRI_PAIRS = [(r, q) for r in range(6) for q in range(r, 6)]


def c21_of_voigt(M):
    """21 constants (upper triangle row by row) of Voigt matrices M shaped (6, 6, ...)."""
    M = np.asarray(M, np.float64)
    return np.stack([M[r, q] for r, q in TRI_PAIRS])


def voigt_of_c21(c):
    """Symmetric 6x6 Voigt matrix (6, 6, ...) of 21 constants shaped (21, ...)."""
    c = np.asarray(c, np.float64)
    M = np.empty((6, 6) + c.shape[1:])
    for n, (r, q) in enumerate(TRI_PAIRS):
        M[r, q] = c[n]
        M[q, r] = c[n]
    return M


def c21_of_c9(C9):
    """21 constants of orthotropic cells given by their nine constants."""
    C9 = np.asarray(C9, np.float64)
    M = np.zeros((6, 6) + C9.shape[1:])
    C11, C22, C33, C23, C13, C12, C44, C55, C66 = C9
    M[0, 0], M[1, 1], M[2, 2] = C11, C22, C33
    M[1, 2] = M[2, 1] = C23
    M[0, 2] = M[2, 0] = C13
    M[0, 1] = M[1, 0] = C12
    M[3, 3], M[4, 4], M[5, 5] = C44, C55, C66
    return c21_of_voigt(M)


def _prep21(C21, h):
    C21 = np.ascontiguousarray(C21, np.float64)
    if C21.ndim != 4 or C21.shape[0] != 21:
        raise ValueError("C21 must be shaped (21, nz, ny, nx)")
    if not np.all(C21[[0, 6, 11, 15, 18, 20]] > 0):
        raise ValueError("diagonal constants must be positive")
    nz, ny, nx = C21.shape[1:]
    return C21, np.array([nx, ny, nz], np.int64), np.array(h, np.float64)


def stress_tri(C21, E, u, h=(1.0, 1.0, 1.0)):
    """Stresses (6, nz, ny, nx): normal at cells, shear at edges."""
    C21, dims, hh = _prep21(C21, h)
    sh = C21.shape[1:]
    u = np.ascontiguousarray(u, np.float64).reshape((3,) + sh)
    out = np.empty((6,) + sh)
    lib().or_stress_tri(dims.ctypes.data_as(_ip), _d(hh), _d(C21), _d(np.asarray(E, np.float64)), _d(u), _d(out))
    return out


def residual_tri(C21, E, u, h=(1.0, 1.0, 1.0)):
    C21, dims, hh = _prep21(C21, h)
    sh = C21.shape[1:]
    u = np.ascontiguousarray(u, np.float64).reshape((3,) + sh)
    out = np.empty((3,) + sh)
    lib().or_residual_tri(dims.ctypes.data_as(_ip), _d(hh), _d(C21), _d(np.asarray(E, np.float64)), _d(u), _d(out))
    return out


def average_stress_tri(C21, E, u, h=(1.0, 1.0, 1.0)):
    C21, dims, hh = _prep21(C21, h)
    u = np.ascontiguousarray(u, np.float64).reshape((3,) + C21.shape[1:])
    out = np.empty(6)
    lib().or_average_stress_tri(dims.ctypes.data_as(_ip), _d(hh), _d(C21), _d(np.asarray(E, np.float64)), _d(u),
                                _d(out))
    return out


def solve_load_tri(C21, J, h=(1.0, 1.0, 1.0), rtol=1e-11, max_iter=1_000_000):
    C21, dims, hh = _prep21(C21, h)
    u = np.zeros((3,) + C21.shape[1:])
    rel = np.zeros(1)
    it = lib().or_pcg_tri(dims.ctypes.data_as(_ip), _d(hh), _d(C21), _d(unit_strain(J)), rtol, max_iter, _d(u),
                          _d(rel))
    return u, int(it), float(rel[0])


def ceff_tri(C21, h=(1.0, 1.0, 1.0), rtol=1e-11, loads=range(6), max_iter=1_000_000):
    """Effective stiffness (6x6) of an image of general anisotropic cells."""
    C = np.full((6, 6), np.nan)
    info = {}
    for J in loads:
        u, it, rel = solve_load_tri(C21, J, h, rtol, max_iter)
        C[:, J] = average_stress_tri(C21, unit_strain(J), u, h)
        info[J] = (it, rel)
    return C, info


def apt_disp_tri(C21, J, nsteps, courant, strouhal, h=(1.0, 1.0, 1.0)):
    """Displacement-form APT iterate u^nsteps and u^(nsteps-1) for general cells, from u^0 = 0."""
    C21, dims, hh = _prep21(C21, h)
    sh = C21.shape[1:]
    u = np.empty((3,) + sh)
    up = np.empty((3,) + sh)
    lib().or_apt_disp_tri(dims.ctypes.data_as(_ip), _d(hh), _d(C21), _d(unit_strain(J)), courant, strouhal,
                          nsteps, _d(u), _d(up))
    return u, up


def apt_stress(J, nsteps, courant, strouhal, K=None, G=None, C9=None, C21=None, h=(1.0, 1.0, 1.0), walls=False):
    """Stress-state APT iterate v^nsteps and v^(nsteps-1) (each (3, nz, ny, nx)) for isotropic
    (K, G), orthotropic (C9) or general (C21) cells, from v = 0 and the stress of the uniform
    strain; the stresses relax towards Hooke's law of the current strain and drive the
    velocity, as in the paper's scheme.  walls: the wall test of load J (K, G or C9 cells)."""
    Kp = Gp = cp = tp = None
    if C21 is not None:
        C21, dims, hh = _prep21(C21, h)
        sh, tp = C21.shape[1:], _d(C21)
    elif C9 is not None:
        C9, dims, hh = _prep9(C9, h)
        sh, cp = C9.shape[1:], _d(C9)
    else:
        K, G, dims, hh = _prep(K, G, h)
        sh, Kp, Gp = K.shape, _d(K), _d(G)
    if walls and C21 is not None:
        raise ValueError("the wall tests are defined for isotropic and orthotropic cells")
    u = np.empty((3,) + sh)
    up = np.empty((3,) + sh)
    lib().or_apt_stress(dims.ctypes.data_as(_ip), _d(hh), Kp, Gp, cp, tp, wall_mode(J) if walls else 0,
                        _d(unit_strain(J)), courant, strouhal, nsteps, _d(u), _d(up))
    return u, up


# ---- wall boundaries (the paper's direct tests) --------------------------------------
#
# The box boundary in direction d is the grid plane of index 0 in d: the
# fluctuation of the d-faces there is held at zero.  Normal test (loads 0..2,
# mode 1): the edges lying in a boundary plane carry no shear stress.
# Simple-shear test of the Voigt shear component J (loads 3..5, mode J): the
# loaded walls also hold the sheared component tangentially, through split half
# edges (see ceff_oracle.c).

def wall_mode(J):
    """Wall test of load J: 1 (normal test) for J < 3, else J (simple-shear test)."""
    return 1 if J < 3 else int(J)


def _mode_of(E):
    E = np.asarray(E, np.float64)
    sh = [s for s in (3, 4, 5) if E[s] != 0.0]
    return sh[0] if len(sh) == 1 else 1


def residual_walls(K, G, E, u, h=(1.0, 1.0, 1.0), mode=None):
    """Residual under the walls of `mode` (default: the simple-shear test of E's one
    shear component if it has exactly one, else the normal test)."""
    mode = _mode_of(E) if mode is None else mode
    K, G, dims, hh = _prep(K, G, h)
    u = np.ascontiguousarray(u, np.float64).reshape((3,) + K.shape)
    out = np.empty((3,) + K.shape)
    lib().or_residual_walls(dims.ctypes.data_as(_ip), _d(hh), _d(K), _d(G), _d(np.asarray(E, np.float64)), _d(u),
                            _d(out), mode)
    return out


def average_stress_walls(K, G, E, u, h=(1.0, 1.0, 1.0), mode=None):
    mode = _mode_of(E) if mode is None else mode
    K, G, dims, hh = _prep(K, G, h)
    u = np.ascontiguousarray(u, np.float64).reshape((3,) + K.shape)
    out = np.empty(6)
    lib().or_average_stress_walls(dims.ctypes.data_as(_ip), _d(hh), _d(K), _d(G), _d(np.asarray(E, np.float64)),
                                  _d(u), _d(out), mode)
    return out


def solve_load_walls(K, G, J, h=(1.0, 1.0, 1.0), rtol=1e-11, max_iter=1_000_000):
    K, G, dims, hh = _prep(K, G, h)
    u = np.zeros((3,) + K.shape)
    rel = np.zeros(1)
    it = lib().or_pcg_walls(dims.ctypes.data_as(_ip), _d(hh), _d(K), _d(G), _d(unit_strain(J)), rtol, max_iter,
                            _d(u), _d(rel), wall_mode(J))
    return u, int(it), float(rel[0])


def ceff_walls(K, G, h=(1.0, 1.0, 1.0), rtol=1e-11, loads=(0, 1, 2)):
    """Columns `loads` of C* from the wall tests (other entries NaN): column J < 3 from
    the normal test of J, column J >= 3 from the simple-shear test of J."""
    C = np.full((6, 6), np.nan)
    info = {}
    for J in loads:
        u, it, rel = solve_load_walls(K, G, J, h, rtol)
        C[:, J] = average_stress_walls(K, G, unit_strain(J), u, h, mode=wall_mode(J))
        info[J] = (it, rel)
    return C, info


def gradient(K, G, fields, W, h=(1.0, 1.0, 1.0)):
    """dJ/dK, dJ/dG for J = sum W_IJ C_IJ, from the six converged fields."""
    K, G, dims, hh = _prep(K, G, h)
    u6 = np.ascontiguousarray(np.stack([np.asarray(fields[J], np.float64).reshape((3,) + K.shape)
                                        for J in range(6)]))
    W = np.ascontiguousarray(np.asarray(W, np.float64).reshape(36))
    dK = np.empty(K.shape); dG = np.empty(K.shape)
    lib().or_gradient(dims.ctypes.data_as(_ip), _d(hh), _d(K), _d(G), _d(u6), _d(W), _d(dK), _d(dG))
    return dK, dG
