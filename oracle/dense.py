"""Brute-force dense solve of the periodic staggered-grid problem on tiny grids.

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is a second, independent route to the discrete problem that
``ceff_oracle.c`` solves.  It never forms a divergence: it writes the strain
of a displacement field with numpy array shifts, assembles the strain matrix
B column by column from unit displacements, weights it with the elastic
energy density (paper, "Theory": the rate form of Hooke's law integrated
with unit time step), and minimises the energy
    W(u) = 1/2 sum_cells [K theta^2 + 2G sum_d (eps_dd - theta/3)^2]
           + sum_edges 2 G_e eps_e^2
by a dense least-squares solve of the normal equations B^T D B u = -B^T D e.
The translations (the only null space) are removed with lstsq's minimum-norm
solution.  C_IJ is then the volume average of stress (same definition as in
the C oracle), so an index or sign mistake in either implementation shows up
as a mismatch.
"""
from __future__ import annotations

import numpy as np


def _fwd(a, axis):   # a[i+1] - a[i] along `axis` (periodic)
    return np.roll(a, -1, axis=axis) - a


def _bwd(a, axis):   # a[i] - a[i-1]
    return a - np.roll(a, 1, axis=axis)


# numpy axis of each Cartesian direction for arrays shaped (nz, ny, nx)
_AX = {"x": 2, "y": 1, "z": 0}


def strain_field(u, E, h=(1.0, 1.0, 1.0)):
    """Tensor strain components (xx, yy, zz at cells; yz, xz, xy at edges)."""
    ux, uy, uz = u
    hx, hy, hz = h
    exx = E[0] + _fwd(ux, _AX["x"]) / hx
    eyy = E[1] + _fwd(uy, _AX["y"]) / hy
    ezz = E[2] + _fwd(uz, _AX["z"]) / hz
    eyz = E[3] + 0.5 * (_bwd(uy, _AX["z"]) / hz + _bwd(uz, _AX["y"]) / hy)
    exz = E[4] + 0.5 * (_bwd(ux, _AX["z"]) / hz + _bwd(uz, _AX["x"]) / hx)
    exy = E[5] + 0.5 * (_bwd(ux, _AX["y"]) / hy + _bwd(uy, _AX["x"]) / hx)
    return np.stack([exx, eyy, ezz, eyz, exz, exy])


def edge_moduli(G):
    """Harmonic mean of G over the four cells around each edge: (yz, xz, xy)."""
    inv = 1.0 / G
    def sh(a, ax):
        return np.roll(a, 1, axis=ax)
    x, y, z = _AX["x"], _AX["y"], _AX["z"]
    g_yz = 4.0 / (inv + sh(inv, y) + sh(inv, z) + sh(sh(inv, y), z))
    g_xz = 4.0 / (inv + sh(inv, x) + sh(inv, z) + sh(sh(inv, x), z))
    g_xy = 4.0 / (inv + sh(inv, x) + sh(inv, y) + sh(sh(inv, x), y))
    return np.stack([g_yz, g_xz, g_xy])


def stress_field(K, G, eps):
    th = eps[0] + eps[1] + eps[2]
    Ge = edge_moduli(G)
    out = np.empty_like(eps)
    for d in range(3):
        out[d] = K * th + 2.0 * G * (eps[d] - th / 3.0)
    for c in range(3):
        out[3 + c] = 2.0 * Ge[c] * eps[3 + c]
    return out


def stress_field_c9(C9, eps):
    """Stresses of orthotropic cells (C9: C11 C22 C33 C23 C13 C12 C44 C55 C66)."""
    C11, C22, C33, C23, C13, C12, C44, C55, C66 = C9
    out = np.empty_like(eps)
    out[0] = C11 * eps[0] + C12 * eps[1] + C13 * eps[2]
    out[1] = C12 * eps[0] + C22 * eps[1] + C23 * eps[2]
    out[2] = C13 * eps[0] + C23 * eps[1] + C33 * eps[2]
    for c, Cs in enumerate((C44, C55, C66)):
        out[3 + c] = 2.0 * edge_moduli(Cs)[c] * eps[3 + c]
    return out


def _energy_weights_c9(C9):
    """As _energy_weights, for W = 1/2 sum_cells e_n . Cn e_n + sum_edges 2 C_e eps_e^2."""
    C11, C22, C33, C23, C13, C12, C44, C55, C66 = [c.ravel() for c in C9]
    Ce = np.stack([edge_moduli(Cs)[c].ravel() for c, Cs in enumerate((C9[6], C9[7], C9[8]))])

    def apply(eps):
        out = np.empty_like(eps)
        out[0] = C11 * eps[0] + C12 * eps[1] + C13 * eps[2]
        out[1] = C12 * eps[0] + C22 * eps[1] + C23 * eps[2]
        out[2] = C13 * eps[0] + C23 * eps[1] + C33 * eps[2]
        for c in range(3):
            out[3 + c] = 4.0 * Ce[c] * eps[3 + c]
        return out
    return apply


def octant_strains(eps, C21):
    """Voigt strains (engineering shear) of the eight corner octants of every cell of
    general anisotropic cells, (8, 6, nz, ny, nx), octant o = a + 2b + 4c at the cell's
    corner (+a, +b, +c): the cell's normal strains, and for each shear component the
    edge strain meeting that corner weighted by (harmonic mean over the edge's four
    cells of the component's diagonal constant) / (the cell's own)."""
    S = (C21[15], C21[18], C21[20])  # C44, C55, C66
    Se = (edge_moduli(S[0])[0], edge_moduli(S[1])[1], edge_moduli(S[2])[2])
    x, y, z = _AX["x"], _AX["y"], _AX["z"]

    def at_corner(f, da, db, dc):  # f at index (i + da, j + db, k + dc)
        return np.roll(np.roll(np.roll(f, -da, axis=x), -db, axis=y), -dc, axis=z)
    out = np.empty((8, 6) + eps.shape[1:])
    for o in range(8):
        a, b, c = o & 1, (o >> 1) & 1, o >> 2
        out[o, :3] = eps[:3]
        # yz edge [i, j+b, k+c], xz edge [i+a, j, k+c], xy edge [i+a, j+b, k]
        for s_, (da, db, dc) in enumerate(((0, b, c), (a, 0, c), (a, b, 0))):
            out[o, 3 + s_] = 2.0 * at_corner(eps[3 + s_] * Se[s_], da, db, dc) / S[s_]
    return out


def _octant_apply(C21):
    """(C_cell / 8) times every octant's strain: the weights of W = sum 1/2 v . (C/8) v."""
    M = np.stack([np.stack([C21[_tri_n(r, q)] for q in range(6)]) for r in range(6)])  # (6, 6, ...)

    def apply(v):
        return np.einsum("rq...,oq...->or...", M, v) / 8.0
    return apply


def _tri_n(r, q):
    a, b = min(r, q), max(r, q)
    return 6 * a - a * (a - 1) // 2 + (b - a)


def solve_dense_tri(C21, E, h=(1.0, 1.0, 1.0)):
    """Displacement fluctuation minimising the octant energy of general cells (3, nz, ny, nx)."""
    shape = C21.shape[1:]
    N = int(np.prod(shape))
    zero = np.zeros(6)
    B = np.empty((48 * N, 3 * N))
    for col in range(3 * N):
        u = np.zeros(3 * N); u[col] = 1.0
        B[:, col] = octant_strains(strain_field(u.reshape((3,) + shape), zero, h), C21).reshape(48 * N)
    D = _octant_apply(C21)
    DB = np.empty_like(B)
    for col in range(3 * N):
        DB[:, col] = D(B[:, col].reshape((8, 6) + shape)).reshape(48 * N)
    A = B.T @ DB
    v0 = octant_strains(strain_field(np.zeros((3,) + shape), E, h), C21)
    rhs = -B.T @ D(v0).reshape(48 * N)
    u, *_ = np.linalg.lstsq(A, rhs, rcond=1e-13)
    return u.reshape((3,) + shape), A


def ceff_dense_tri(C21, h=(1.0, 1.0, 1.0)):
    """6x6 effective stiffness of general cells by dense minimisation of the octant
    energy; <sigma_I> = (1/N) dW/dE_I (E_I engineering for shear)."""
    shape = C21.shape[1:]
    N = int(np.prod(shape))
    D = _octant_apply(C21)
    C = np.empty((6, 6))
    for J in range(6):
        E = np.zeros(6); E[J] = 1.0 if J < 3 else 0.5
        u, _ = solve_dense_tri(C21, E, h)
        Dv = D(octant_strains(strain_field(u, E, h), C21))
        for I in range(6):
            EI = np.zeros(6); EI[I] = 1.0 if I < 3 else 0.5
            dv = octant_strains(strain_field(np.zeros((3,) + shape), EI, h), C21)
            C[I, J] = float(np.sum(dv * Dv)) / N
    return C


def _energy_weights(K, G):
    """Quadratic form of the energy density per node: returns a function that
    maps strains (6, N) to the weighted strains D eps (so W = eps^T D eps / 2)."""
    Ge = edge_moduli(G).reshape(3, -1)
    Kf = K.ravel(); Gf = G.ravel()

    def apply(eps):
        th = eps[0] + eps[1] + eps[2]
        out = np.empty_like(eps)
        for d in range(3):
            # d/d eps_dd of 1/2 [K th^2 + 2G sum (eps_dd - th/3)^2]
            out[d] = Kf * th + 2.0 * Gf * (eps[d] - th / 3.0)
        for c in range(3):
            # d/d eps_e of 2 G_e eps_e^2 (counts both symmetric shear components)
            out[3 + c] = 4.0 * Ge[c] * eps[3 + c]
        return out
    return apply


# Simple-shear wall test of the Voigt shear component s (3 yz, 4 xz, 5 xy): the
# direction d it shears and the normal e of the loaded walls.
SHEAR_PAIR = {3: (1, 2), 4: (0, 2), 5: (0, 1)}


def wall_masks(shape, mode=1):
    """Wall layout on the periodic grid: (free, edge_keep).  free (3N, bool) marks
    face displacements that may move (not the d-faces of the plane of index 0 in
    d).  edge_keep (3, N) (order yz, xz, xy) is 0 for edges lying in a boundary
    plane, whose shear stiffness is dropped (free slip), except, for the
    simple-shear test mode = s, the s-edges lying in the d-wall plane only, which
    keep theirs; the s-edges in the loaded e-wall plane are dropped here and
    replaced by the half edges of split_edge_strains."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    idx = (i, j, k)
    free = np.concatenate([(i != 0).ravel(), (j != 0).ravel(), (k != 0).ravel()])
    keep = []
    for comp, (a, b) in SHEAR_PAIR.items():
        if mode == comp:
            keep.append((idx[b] != 0).ravel())
        else:
            keep.append(((idx[a] != 0) & (idx[b] != 0)).ravel())
    return free, np.stack(keep).astype(float)


def _planes(shape, e):
    ae = _AX["xyz"[e]]
    first = [slice(None)] * 3; first[ae] = slice(0, 1)
    last = [slice(None)] * 3; last[ae] = slice(shape[ae] - 1, shape[ae])
    return tuple(first), tuple(last)


def split_edge_strains(u, E, s, h=(1.0, 1.0, 1.0)):
    """Tensor shear strains of the two halves of every s-edge on the loaded wall
    plane (index 0 in e) of the simple-shear test s: (first, last), the halves in
    the cells of index 0 and n_e - 1 in e.  The wall holds the u_d fluctuation at
    zero, so each half differentiates u_d over half a cell; the tangential
    derivative of u_e is taken between the wall faces."""
    d, e = SHEAR_PAIR[s]
    first, last = _planes(u.shape[1:], e)
    tang = _bwd(u[e], _AX["xyz"[d]])[first] / h[d]
    return (E[s] + 0.5 * (2.0 * u[d][first] / h[e] + tang),
            E[s] + 0.5 * (-2.0 * u[d][last] / h[e] + tang))


def split_edge_moduli(Gs, s):
    """Harmonic mean of the shear constant over the two cells of each half edge."""
    d, e = SHEAR_PAIR[s]
    first, last = _planes(Gs.shape, e)
    ad = _AX["xyz"[d]]
    f, l = 1.0 / Gs[first], 1.0 / Gs[last]
    return 2.0 / (f + np.roll(f, 1, axis=ad)), 2.0 / (l + np.roll(l, 1, axis=ad))


def solve_dense(K, G, E, h=(1.0, 1.0, 1.0), C9=None, walls=False):
    """Displacement fluctuation minimising the discrete strain energy (3, nz, ny, nx).
    Isotropic (K, G) cells, or orthotropic cells when C9 is given.  walls: False
    (periodic), True or 1 (normal-test walls: pinned wall faces, no shear energy on
    boundary edges) or 3..5 (the simple-shear test of that component: as 1, with
    the half edges of the loaded walls, each of half an edge's volume)."""
    shape = K.shape if C9 is None else C9.shape[1:]
    N = int(np.prod(shape))
    zero = np.zeros(6)
    mode = 1 if walls is True else int(walls)
    B = np.empty((6 * N, 3 * N))
    for col in range(3 * N):
        u = np.zeros(3 * N); u[col] = 1.0
        B[:, col] = strain_field(u.reshape((3,) + shape), zero, h).reshape(6 * N)
    Dapply0 = _energy_weights(K, G) if C9 is None else _energy_weights_c9(C9)
    if mode:
        free, keep = wall_masks(shape, mode)

        def Dapply(eps):
            out = Dapply0(eps)
            out[3:] *= keep
            return out
        B[:, ~free] = 0.0
    else:
        Dapply = Dapply0
    DB = np.empty_like(B)
    for col in range(3 * N):
        DB[:, col] = Dapply(B[:, col].reshape(6, N)).reshape(6 * N)
    A = B.T @ DB
    e0 = strain_field(np.zeros((3,) + shape), E, h).reshape(6, N)
    rhs = -B.T @ Dapply(e0).reshape(6 * N)
    if mode >= 3:
        # half edges: energy (1/2) * 2 C_h eps^2 each, so weight 2 C_h
        Gs = G if C9 is None else C9[mode + 3]
        w = np.concatenate([m.ravel() for m in split_edge_moduli(Gs, mode)]) * 2.0
        M = w.size
        Bx = np.empty((M, 3 * N))
        for col in range(3 * N):
            u = np.zeros(3 * N); u[col] = 1.0
            Bx[:, col] = np.concatenate([a.ravel() for a in split_edge_strains(u.reshape((3,) + shape), zero,
                                                                                 mode, h)])
        Bx[:, ~free] = 0.0
        ex = np.concatenate([a.ravel() for a in split_edge_strains(np.zeros((3,) + shape), E, mode, h)])
        A = A + Bx.T @ (w[:, None] * Bx)
        rhs = rhs - Bx.T @ (w * ex)
    u, *_ = np.linalg.lstsq(A, rhs, rcond=1e-13)
    return u.reshape((3,) + shape), A


def average_stress_walls(K, G, u, E, mode, h=(1.0, 1.0, 1.0)):
    """Volume averages of the six stresses under the walls of `mode`: free boundary
    edges carry none; a split edge contributes the mean of its two halves."""
    sig = stress_field(K, G, strain_field(u, E, h))
    _, keep = wall_masks(K.shape, mode)
    sig[3:] *= keep.reshape((3,) + K.shape)
    out = sig.reshape(6, -1).sum(axis=1)
    if mode >= 3:
        (eb, et), (gb, gt) = split_edge_strains(u, E, mode, h), split_edge_moduli(G, mode)
        out[mode] += 0.5 * np.sum(2.0 * gb * eb + 2.0 * gt * et)
    return out / K.size


def ceff_dense_walls(K, G, h=(1.0, 1.0, 1.0), loads=(0, 1, 2)):
    """Columns `loads` of C* from the wall tests by dense energy minimisation: the
    normal test for J < 3, the simple-shear test of J for J >= 3 (others NaN)."""
    C = np.full((6, 6), np.nan)
    for J in loads:
        E = np.zeros(6); E[J] = 1.0 if J < 3 else 0.5
        mode = 1 if J < 3 else J
        u, _ = solve_dense(K, G, E, h, walls=mode)
        C[:, J] = average_stress_walls(K, G, u, E, mode, h)
    return C


def ceff_dense(K, G, h=(1.0, 1.0, 1.0), C9=None):
    """6x6 effective stiffness by dense energy minimisation, Voigt order."""
    C = np.empty((6, 6))
    for J in range(6):
        E = np.zeros(6); E[J] = 1.0 if J < 3 else 0.5
        u, _ = solve_dense(K, G, E, h, C9)
        eps = strain_field(u, E, h)
        sig = stress_field(K, G, eps) if C9 is None else stress_field_c9(C9, eps)
        C[:, J] = sig.reshape(6, -1).mean(axis=1)
    return C
