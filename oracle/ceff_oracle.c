/*
 * CPU oracle for periodic voxel-grid elastic homogenisation (FP64).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it exists so that tests and the benchmark's CPU baseline
 * can check the GPU path against a plain, slow, independent implementation.
 * It shares no code, header or constant with the GPU library.
 *
 * What it computes (paper: "Theory", eqs. 1-3 and the volume averages that
 * define C*; "Numerical solution strategy", the APT equations):
 *
 *   For a macroscopic strain E (a symmetric 3x3 tensor), find a periodic
 *   displacement fluctuation u on the staggered grid such that the stress
 *   sigma = C : (E + grad u) is divergence free.  Then <sigma_I> over the grid
 *   is column J of the effective stiffness when E is the J-th unit Voigt
 *   strain (engineering shear, so E_yz = E_zy = 1/2 for J = 4).
 *
 * Discretisation (staggered grid of the paper's "Discretization" section,
 * read with periodic wrap, see the design notes for the readings):
 *   cell (i,j,k)        : normal strains/stresses, K, G
 *   x-face u_x[i,j,k]   : between cells i-1 and i
 *   xy-edge [i,j,k]     : shared by cells (i-1|i, j-1|j, k); shear modulus is
 *                         the harmonic mean of those four cells
 *   exx = E_xx + (ux[i+1]-ux[i])/hx,   exy = E_xy + ((ux[j]-ux[j-1])/hy + (uy[i]-uy[i-1])/hx)/2
 *   sxx = K*theta + 2G(exx - theta/3),  sxy = 2 G_e exy
 *   (div s)_x[i,j,k] = (sxx[i]-sxx[i-1])/hx + (sxy[j+1]-sxy[j])/hy + (sxz[k+1]-sxz[k])/hz
 *
 * Orthotropic cells (axes aligned with the grid; an extension the paper lists
 * among its perspectives) carry nine constants instead of K and G:
 *   c9[q*N + cell], q = 0..8: C11 C22 C33 C23 C13 C12 C44 C55 C66 (Voigt,
 *   engineering shear), so sxx = C11 exx + C12 eyy + C13 ezz (and alike) at
 *   cells, and at edges syz = 2 C44_e eyz, sxz = 2 C55_e exz, sxy = 2 C66_e exy
 *   with the edge constant the harmonic mean over the four cells, as for G.
 *   With C11 = K + 4G/3, C12 = K - 2G/3 and C44 = G this is the isotropic law.
 *
 * General anisotropic cells (the same perspectives list: triclinic local
 * stiffness, which needs strains shared between cells and edges) carry the full
 * symmetric 6x6 Voigt matrix, 21 constants c21[q*N + cell], the upper triangle
 * row by row: C11 C12 C13 C14 C15 C16 C22 C23 C24 C25 C26 C33 C34 C35 C36 C44
 * C45 C46 C55 C56 C66.  Reading of the coupled law on the staggered grid: each
 * cell is split into eight corner octants.  Octant (a, b, c) of cell (i, j, k),
 * at the corner (i+a, j+b, k+c) of the cell's node box, takes the cell's normal
 * strains and, for each shear component, the strain the cell carries of the
 * edge of that component meeting the corner, when the edge's strain is shared by
 * its four cells in series: w gamma_e with w = S_e / S_cell, S the diagonal
 * shear constant of the component (C44 yz, C55 xz, C66 xy) and S_e its harmonic
 * mean over the edge's four cells.  The energy is sum over cells of
 * 1/8 sum over octants of 1/2 eps_o . C_cell eps_o (Voigt, engineering shear),
 * and the stresses are its derivatives: at a cell the octant mean of the normal
 * rows of C eps_o, at an edge the sum over its four cells and the two octants
 * each has there of w/8 times the shear row.  Without couplings this is exactly
 * the orthotropic law above; for positive definite cells the energy is a sum of
 * positive definite octant terms.
 *
 * Wall boundaries (the paper's direct tests, appendix on boundary conditions:
 * faces of the box are rigid in the normal direction and traction-free in the
 * tangential ones) on the same periodic layout: the box boundary in direction
 * d is the grid plane of index 0 in d (it is both the first and, by the wrap,
 * the last plane).  The displacement fluctuation of the d-faces there is held at
 * zero, so the total displacement of both walls is the macroscopic strain's, and
 * the shear stress of every edge lying in a boundary plane is zero (free slip;
 * those edges would couple the two sides of the box across the wrap).  This is
 * the normal compression test (walls = 1, normal loads).
 *
 * Simple-shear test of the Voigt shear component s (walls = s: 3 yz, 4 xz, 5 xy;
 * the same appendix): the load shears direction d across the walls normal to e,
 * (d, e) = (y, z), (x, z), (x, y).  The faces are held as above.  The loaded
 * e-walls are also held tangentially in d (no slip): each s-edge lying in the
 * e-boundary plane is split into two half edges, one per side of the box, whose
 * strain takes the u_d fluctuation across the half cell to the wall, where it is
 * zero, and whose modulus is the harmonic mean of the two cells on that side;
 * each half counts for half a node in the volume average.  The s-edges lying in
 * the d-boundary plane only are computed as in the periodic medium (the walls
 * normal to d transmit the applied shear).  All other boundary edges are free.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (see oracle/build.py).
 * Arrays: x fastest, linear index i + nx*(j + ny*k); vector fields are stored
 * component-major: f[c*N + idx].  Tensor strain components are passed as
 * E[6] = (xx, yy, zz, yz, xz, xy) (tensor, not engineering, shear).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t nx, ny, nz;
    double hx, hy, hz;
} grid_t;

/* Material: isotropic K, G per cell, or nine orthotropic constants per cell (c9 != NULL);
 * walls: 0 periodic boundaries, 1 the walls of the normal test, 3..5 the walls of the
 * simple-shear test of that Voigt shear component (see the header). */
typedef struct {
    const double *K, *G, *c9;
    int walls;
    const double *c21;  /* general anisotropic cells (21 constants) or NULL */
} mat_t;

static inline int64_t wrap(int64_t a, int64_t n) { a %= n; return a < 0 ? a + n : a; }
static inline int64_t at(const grid_t *g, int64_t i, int64_t j, int64_t k) {
    return wrap(i, g->nx) + g->nx * (wrap(j, g->ny) + g->ny * wrap(k, g->nz));
}

/* Harmonic mean of the shear moduli of the four cells sharing an edge.
 * plane = 0: xy-edge (cells differ in i and j), 1: xz-edge (i and k),
 * 2: yz-edge (j and k). */
static double edge_modulus(const grid_t *g, const double *G, int plane, int64_t i, int64_t j, int64_t k) {
    double s;
    if (plane == 0)
        s = 1.0 / G[at(g, i - 1, j - 1, k)] + 1.0 / G[at(g, i, j - 1, k)] +
            1.0 / G[at(g, i - 1, j, k)] + 1.0 / G[at(g, i, j, k)];
    else if (plane == 1)
        s = 1.0 / G[at(g, i - 1, j, k - 1)] + 1.0 / G[at(g, i, j, k - 1)] +
            1.0 / G[at(g, i - 1, j, k)] + 1.0 / G[at(g, i, j, k)];
    else
        s = 1.0 / G[at(g, i, j - 1, k - 1)] + 1.0 / G[at(g, i, j, k - 1)] +
            1.0 / G[at(g, i, j - 1, k)] + 1.0 / G[at(g, i, j, k)];
    return 4.0 / s;
}

/* Index q of the Voigt constant C_rs (r, s = 0..5) in a cell's 21 constants
 * (upper triangle row by row). */
static int tri_q(int r, int s) {
    const int a = r < s ? r : s, b = r < s ? s : r;
    return 6 * a - a * (a - 1) / 2 + (b - a);
}

/* Diagonal shear constant of edge plane p (0 xy, 1 xz, 2 yz) of every cell:
 * G, or C66 / C55 / C44 of orthotropic or general cells. */
static const double *shear_field(const grid_t *g, const mat_t *m, int plane) {
    const int64_t N = g->nx * g->ny * g->nz;
    if (m->c21) return m->c21 + (int64_t)tri_q(5 - plane, 5 - plane) * N;
    if (m->c9) return m->c9 + (plane == 0 ? 8 : (plane == 1 ? 7 : 6)) * N;
    return m->G;
}

/* Shear constant of an edge for material m: the harmonic mean over the four
 * cells of G (isotropic) or of C66 (xy), C55 (xz), C44 (yz) (orthotropic and
 * general cells). */
static double edge_shear(const grid_t *g, const mat_t *m, int plane, int64_t i, int64_t j, int64_t k) {
    return edge_modulus(g, shear_field(g, m, plane), plane, i, j, k);
}

/* Voigt shear component s = 3, 4, 5 (yz, xz, xy): the direction it shears in the
 * simple-shear test and the normal of the loaded walls. */
static const int pair_d[6] = {0, 0, 0, 1, 0, 0}, pair_e[6] = {0, 0, 0, 2, 2, 1};

/* Treatment of the s-edge with index (i, j, k) under the wall conditions:
 * 0 as in the periodic medium, 1 no shear stress (free slip), 2 split into two
 * half edges (no slip on the loaded walls of the simple-shear test s). */
static int wall_edge(const mat_t *m, int s, int64_t i, int64_t j, int64_t k) {
    if (!m->walls) return 0;
    const int64_t p[3] = {i, j, k};
    const int in_d = p[pair_d[s]] == 0, in_e = p[pair_e[s]] == 0;
    if (!in_d && !in_e) return 0;
    if (m->walls == s) return in_e ? 2 : 0;
    return 1;
}

/* Shear stress of one half of the split s-edge (i, j, k) (index 0 in e) of the
 * simple-shear test s.  side 0: the half in the cells of index 0 in e; side 1:
 * the half in the cells of index n_e - 1.  The derivative of u_d across the half
 * cell to the wall is one-sided, the wall's fluctuation being zero; the
 * tangential derivative of u_e is taken between the wall faces, as inside. */
static double half_edge(const grid_t *g, const mat_t *m, int s, const double E[6], const double *u, int64_t i,
                        int64_t j, int64_t k, int side) {
    const int64_t N = g->nx * g->ny * g->nz;
    const int d = pair_d[s], e = pair_e[s];
    const int64_t n[3] = {g->nx, g->ny, g->nz};
    const double h[3] = {g->hx, g->hy, g->hz};
    int64_t p[3] = {i, j, k}, q[3];
    p[e] = side ? n[e] - 1 : 0;
    memcpy(q, p, sizeof q);
    q[d] -= 1;
    const double *Gs = m->c9 ? m->c9 + (int64_t)(s + 3) * N : m->G;
    const int64_t c0 = at(g, p[0], p[1], p[2]), c1 = at(g, q[0], q[1], q[2]);
    const double Gh = 2.0 / (1.0 / Gs[c0] + 1.0 / Gs[c1]);
    const double dud = (side ? -2.0 : 2.0) * u[d * N + c0] / h[e];
    int64_t w0[3] = {i, j, k}, w1[3];
    w0[e] = 0;
    memcpy(w1, w0, sizeof w1);
    w1[d] -= 1;
    const double due = (u[e * N + at(g, w0[0], w0[1], w0[2])] - u[e * N + at(g, w1[0], w1[1], w1[2])]) / h[d];
    return 2.0 * Gh * (E[s] + 0.5 * (dud + due));
}

/* Total strain (E + grad u) at every cell and edge.
 * eps[0..2] normal strains at cells, eps[3] yz-edge, eps[4] xz-edge,
 * eps[5] xy-edge (tensor components). */
static void strains(const grid_t *g, const double E[6], const double *u, double *eps) {
    const int64_t N = g->nx * g->ny * g->nz;
    const double *ux = u, *uy = u + N, *uz = u + 2 * N;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < g->nz; k++)
        for (int64_t j = 0; j < g->ny; j++)
            for (int64_t i = 0; i < g->nx; i++) {
                int64_t c = at(g, i, j, k);
                eps[0 * N + c] = E[0] + (ux[at(g, i + 1, j, k)] - ux[c]) / g->hx;
                eps[1 * N + c] = E[1] + (uy[at(g, i, j + 1, k)] - uy[c]) / g->hy;
                eps[2 * N + c] = E[2] + (uz[at(g, i, j, k + 1)] - uz[c]) / g->hz;
                eps[3 * N + c] = E[3] + 0.5 * ((uy[c] - uy[at(g, i, j, k - 1)]) / g->hz +
                                               (uz[c] - uz[at(g, i, j - 1, k)]) / g->hy);
                eps[4 * N + c] = E[4] + 0.5 * ((ux[c] - ux[at(g, i, j, k - 1)]) / g->hz +
                                               (uz[c] - uz[at(g, i - 1, j, k)]) / g->hx);
                eps[5 * N + c] = E[5] + 0.5 * ((ux[c] - ux[at(g, i, j - 1, k)]) / g->hy +
                                               (uy[c] - uy[at(g, i - 1, j, k)]) / g->hx);
            }
}

/* Hooke's law.  Isotropic: sigma = K tr(eps) I + 2 G dev(eps) at cells;
 * orthotropic: the normal block of the 6x6 Voigt matrix times the normal
 * strains.  Edges: sigma_e = 2 (edge shear constant) eps_e. */
static void hooke(const grid_t *g, const mat_t *m, const double *eps, double *sig) {
    const int64_t N = g->nx * g->ny * g->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < g->nz; k++)
        for (int64_t j = 0; j < g->ny; j++)
            for (int64_t i = 0; i < g->nx; i++) {
                int64_t c = at(g, i, j, k);
                if (m->c9) {
                    const double *C = m->c9;
                    double exx = eps[c], eyy = eps[N + c], ezz = eps[2 * N + c];
                    double C11 = C[c], C22 = C[N + c], C33 = C[2 * N + c];
                    double C23 = C[3 * N + c], C13 = C[4 * N + c], C12 = C[5 * N + c];
                    sig[c] = C11 * exx + C12 * eyy + C13 * ezz;
                    sig[N + c] = C12 * exx + C22 * eyy + C23 * ezz;
                    sig[2 * N + c] = C13 * exx + C23 * eyy + C33 * ezz;
                } else {
                    double th = eps[c] + eps[N + c] + eps[2 * N + c];
                    for (int d = 0; d < 3; d++)
                        sig[d * N + c] = m->K[c] * th + 2.0 * m->G[c] * (eps[d * N + c] - th / 3.0);
                }
                sig[3 * N + c] = 2.0 * edge_shear(g, m, 2, i, j, k) * eps[3 * N + c];
                sig[4 * N + c] = 2.0 * edge_shear(g, m, 1, i, j, k) * eps[4 * N + c];
                sig[5 * N + c] = 2.0 * edge_shear(g, m, 0, i, j, k) * eps[5 * N + c];
                for (int s = 3; s < 6; s++)  /* free boundary edges carry no shear stress */
                    if (wall_edge(m, s, i, j, k) == 1) sig[s * N + c] = 0.0;
            }
}

/* ---- general anisotropic cells (see the header) ---- */

/* Voigt strain (engineering shear) of octant (a, b, c) of cell (i, j, k) from
 * the tensor strains eps (cells: xx yy zz; edges: yz xz xy). */
static void octant_strain(const grid_t *g, const mat_t *m, const double *eps, int64_t i, int64_t j, int64_t k,
                          int a, int b, int c, double out[6]) {
    const int64_t N = g->nx * g->ny * g->nz, cell = at(g, i, j, k);
    for (int d = 0; d < 3; d++) out[d] = eps[d * N + cell];
    /* the corner's edges: yz [i, j+b, k+c], xz [i+a, j, k+c], xy [i+a, j+b, k] (planes 2, 1, 0) */
    const int64_t e[3][3] = {{i, j + b, k + c}, {i + a, j, k + c}, {i + a, j + b, k}};
    for (int s = 0; s < 3; s++) {
        const int plane = 2 - s;
        const double *S = shear_field(g, m, plane);
        const double Se = edge_modulus(g, S, plane, e[s][0], e[s][1], e[s][2]);
        out[3 + s] = 2.0 * eps[(3 + s) * N + at(g, e[s][0], e[s][1], e[s][2])] * Se / S[cell];
    }
}

/* Row r of cell's C times the Voigt vector v. */
static double tri_row(const grid_t *g, const mat_t *m, int64_t cell, int r, const double v[6]) {
    const int64_t N = g->nx * g->ny * g->nz;
    double s = 0.0;
    for (int q = 0; q < 6; q++) s += m->c21[(int64_t)tri_q(r, q) * N + cell] * v[q];
    return s;
}

/* Stresses of general cells: cells get the octant mean of the normal rows, each
 * edge the w/8-weighted shear rows of the two octants of each of its four
 * cells that meet it. */
static void hooke_tri(const grid_t *g, const mat_t *m, const double *eps, double *sig) {
    const int64_t N = g->nx * g->ny * g->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < g->nz; k++)
        for (int64_t j = 0; j < g->ny; j++)
            for (int64_t i = 0; i < g->nx; i++) {
                const int64_t c = at(g, i, j, k);
                double v[6], acc[3] = {0.0, 0.0, 0.0};
                for (int o = 0; o < 8; o++) {
                    octant_strain(g, m, eps, i, j, k, o & 1, (o >> 1) & 1, o >> 2, v);
                    for (int r = 0; r < 3; r++) acc[r] += tri_row(g, m, c, r, v);
                }
                for (int r = 0; r < 3; r++) sig[r * N + c] = acc[r] / 8.0;
                /* edge (i, j, k) of each plane; its cells are (cell offset, corner) pairs */
                for (int s = 0; s < 3; s++) {
                    const int plane = 2 - s;
                    const double *S = shear_field(g, m, plane);
                    const double Se = edge_modulus(g, S, plane, i, j, k);
                    double t = 0.0;
                    for (int p = 0; p < 4; p++) {
                        const int q0 = p & 1, q1 = p >> 1;  /* the two cell offsets across the edge */
                        int64_t ci = i, cj = j, ck = k;
                        int a = 0, b = 0, cc = 0;
                        if (s == 0) { cj = j - 1 + q0; ck = k - 1 + q1; b = 1 - q0; cc = 1 - q1; }
                        if (s == 1) { ci = i - 1 + q0; ck = k - 1 + q1; a = 1 - q0; cc = 1 - q1; }
                        if (s == 2) { ci = i - 1 + q0; cj = j - 1 + q1; a = 1 - q0; b = 1 - q1; }
                        const int64_t cell = at(g, ci, cj, ck);
                        const double w = Se / S[cell];
                        for (int h2 = 0; h2 < 2; h2++) {  /* the cell's two octants at the edge */
                            int aa = a, bb = b, c2 = cc;
                            if (s == 0) aa = h2; else if (s == 1) bb = h2; else c2 = h2;
                            octant_strain(g, m, eps, ci, cj, ck, aa, bb, c2, v);
                            t += w / 8.0 * tri_row(g, m, cell, 3 + s, v);
                        }
                    }
                    sig[(3 + s) * N + c] = t;
                }
            }
}

/* r = div sigma at the faces (the out-of-balance force of eq. 1). */
static void divergence(const grid_t *g, const double *sig, double *r) {
    const int64_t N = g->nx * g->ny * g->nz;
    const double *sxx = sig, *syy = sig + N, *szz = sig + 2 * N;
    const double *syz = sig + 3 * N, *sxz = sig + 4 * N, *sxy = sig + 5 * N;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < g->nz; k++)
        for (int64_t j = 0; j < g->ny; j++)
            for (int64_t i = 0; i < g->nx; i++) {
                int64_t c = at(g, i, j, k);
                r[c] = (sxx[c] - sxx[at(g, i - 1, j, k)]) / g->hx +
                       (sxy[at(g, i, j + 1, k)] - sxy[c]) / g->hy +
                       (sxz[at(g, i, j, k + 1)] - sxz[c]) / g->hz;
                r[N + c] = (sxy[at(g, i + 1, j, k)] - sxy[c]) / g->hx +
                           (syy[c] - syy[at(g, i, j - 1, k)]) / g->hy +
                           (syz[at(g, i, j, k + 1)] - syz[c]) / g->hz;
                r[2 * N + c] = (sxz[at(g, i + 1, j, k)] - sxz[c]) / g->hx +
                               (syz[at(g, i, j + 1, k)] - syz[c]) / g->hy +
                               (szz[c] - szz[at(g, i, j, k - 1)]) / g->hz;
            }
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t t = 0; t < n; t++) s += a[t] * b[t];
    return s;
}

/* ---- exported entry points ------------------------------------------------ */

/* Loop header over the split edges of the simple-shear test s: the s-edges of
 * index 0 in e. */
#define FOR_SPLIT_EDGES(g, s, i, j, k)                                            \
    for (int64_t k = 0; k < (pair_e[s] == 2 ? 1 : (g)->nz); k++)                   \
        for (int64_t j = 0; j < (pair_e[s] == 1 ? 1 : (g)->ny); j++)               \
            for (int64_t i = 0; i < (g)->nx; i++)

/* Stresses; the s-edges split by a simple-shear test hold their side-0 half. */
static void m_stress(const grid_t *g, const mat_t *m, const double E[6], const double *u, double *sig) {
    const int64_t N = g->nx * g->ny * g->nz;
    double *eps = malloc(sizeof(double) * 6 * N);
    strains(g, E, u, eps);
    if (m->c21)
        hooke_tri(g, m, eps, sig);
    else
        hooke(g, m, eps, sig);
    free(eps);
    const int s = m->walls;
    if (s >= 3) FOR_SPLIT_EDGES(g, s, i, j, k) sig[s * N + at(g, i, j, k)] = half_edge(g, m, s, E, u, i, j, k, 0);
}

/* Zero the entries of a face field (3N) that belong to wall faces (held fixed). */
static void mask_walls(const grid_t *g, double *f) {
    const int64_t N = g->nx * g->ny * g->nz;
    for (int64_t k = 0; k < g->nz; k++)
        for (int64_t j = 0; j < g->ny; j++)
            for (int64_t i = 0; i < g->nx; i++) {
                int64_t c = at(g, i, j, k);
                if (i == 0) f[c] = 0.0;
                if (j == 0) f[N + c] = 0.0;
                if (k == 0) f[2 * N + c] = 0.0;
            }
}

static void m_residual(const grid_t *g, const mat_t *m, const double E[6], const double *u, double *r) {
    const int64_t N = g->nx * g->ny * g->nz;
    double *sig = malloc(sizeof(double) * 6 * N);
    m_stress(g, m, E, u, sig);
    divergence(g, sig, r);
    const int s = m->walls;
    if (s >= 3) {
        /* the u_d faces of index n_e - 1 meet the split edges from their side-1 half */
        const int d = pair_d[s], e = pair_e[s];
        const double he = e == 1 ? g->hy : g->hz;
        FOR_SPLIT_EDGES(g, s, i, j, k) {
            int64_t p[3] = {i, j, k};
            p[e] = (e == 1 ? g->ny : g->nz) - 1;
            const int64_t ce = at(g, i, j, k), cf = at(g, p[0], p[1], p[2]);
            r[d * N + cf] += (half_edge(g, m, s, E, u, i, j, k, 1) - sig[s * N + ce]) / he;
        }
    }
    if (m->walls) mask_walls(g, r); /* a wall face is held, its out-of-balance force is the reaction */
    free(sig);
}

static void m_average_stress(const grid_t *g, const mat_t *m, const double E[6], const double *u, double out[6]) {
    const int64_t N = g->nx * g->ny * g->nz;
    double *sig = malloc(sizeof(double) * 6 * N);
    m_stress(g, m, E, u, sig);
    const int sw = m->walls;
    if (sw >= 3) /* each half of a split edge stands for half a node */
        FOR_SPLIT_EDGES(g, sw, i, j, k) {
            const int64_t c = at(g, i, j, k);
            sig[sw * N + c] = 0.5 * (sig[sw * N + c] + half_edge(g, m, sw, E, u, i, j, k, 1));
        }
    for (int c = 0; c < 6; c++) {
        double s = 0.0;
        for (int64_t t = 0; t < N; t++) s += sig[c * N + t];
        out[c] = s / (double)N;
    }
    free(sig);
}

/* Stresses (6N, order xx yy zz at cells, yz xz xy at edges) for displacement u. */
void or_stress(const int64_t dims[3], const double h[3], const double *K, const double *G,
               const double E[6], const double *u, double *sig) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {K, G, NULL, 0, NULL};
    m_stress(&g, &m, E, u, sig);
}

/* Residual r = div(C : (E + grad u)) at faces (3N). */
void or_residual(const int64_t dims[3], const double h[3], const double *K, const double *G,
                 const double E[6], const double *u, double *r) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {K, G, NULL, 0, NULL};
    m_residual(&g, &m, E, u, r);
}

/* Volume averages of the six stress components (Voigt order 11 22 33 23 13 12),
 * each over its own node set (cells or edges, N points each). */
void or_average_stress(const int64_t dims[3], const double h[3], const double *K, const double *G,
                       const double E[6], const double *u, double out[6]) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {K, G, NULL, 0, NULL};
    m_average_stress(&g, &m, E, u, out);
}

/* The same three for orthotropic cells (c9: 9N constants, see the header). */
void or_stress_ortho(const int64_t dims[3], const double h[3], const double *c9, const double E[6],
                     const double *u, double *sig) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {NULL, NULL, c9, 0, NULL};
    m_stress(&g, &m, E, u, sig);
}

void or_residual_ortho(const int64_t dims[3], const double h[3], const double *c9, const double E[6],
                       const double *u, double *r) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {NULL, NULL, c9, 0, NULL};
    m_residual(&g, &m, E, u, r);
}

void or_average_stress_ortho(const int64_t dims[3], const double h[3], const double *c9, const double E[6],
                             const double *u, double out[6]) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {NULL, NULL, c9, 0, NULL};
    m_average_stress(&g, &m, E, u, out);
}

/* Diagonal of the stiffness operator A = -div C grad (Jacobi preconditioner). */
/* Normal stiffness acting on face displacements of direction d in cell c:
 * K + 4G/3 (isotropic) or C11/C22/C33 (orthotropic). */
static double normal_stiffness(const mat_t *m, int64_t N, int d, int64_t c) {
    if (m->c21) return m->c21[(int64_t)tri_q(d, d) * N + c];
    if (m->c9) return m->c9[d * N + c];
    return m->K[c] + 4.0 * m->G[c] / 3.0;
}

static void diagonal(const grid_t *g, const mat_t *m, double *dg) {
    const int64_t N = g->nx * g->ny * g->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < g->nz; k++)
        for (int64_t j = 0; j < g->ny; j++)
            for (int64_t i = 0; i < g->nx; i++) {
                int64_t c = at(g, i, j, k);
                double Mx = normal_stiffness(m, N, 0, at(g, i - 1, j, k)) + normal_stiffness(m, N, 0, c);
                double My = normal_stiffness(m, N, 1, at(g, i, j - 1, k)) + normal_stiffness(m, N, 1, c);
                double Mz = normal_stiffness(m, N, 2, at(g, i, j, k - 1)) + normal_stiffness(m, N, 2, c);
                double hx2 = g->hx * g->hx, hy2 = g->hy * g->hy, hz2 = g->hz * g->hz;
                dg[c] = Mx / hx2 +
                        (edge_shear(g, m, 0, i, j, k) + edge_shear(g, m, 0, i, j + 1, k)) / hy2 +
                        (edge_shear(g, m, 1, i, j, k) + edge_shear(g, m, 1, i, j, k + 1)) / hz2;
                dg[N + c] = My / hy2 +
                            (edge_shear(g, m, 0, i, j, k) + edge_shear(g, m, 0, i + 1, j, k)) / hx2 +
                            (edge_shear(g, m, 2, i, j, k) + edge_shear(g, m, 2, i, j, k + 1)) / hz2;
                dg[2 * N + c] = Mz / hz2 +
                                (edge_shear(g, m, 1, i, j, k) + edge_shear(g, m, 1, i + 1, j, k)) / hx2 +
                                (edge_shear(g, m, 2, i, j, k) + edge_shear(g, m, 2, i, j + 1, k)) / hy2;
            }
}

static void remove_mean(int64_t N, double *v) {
    for (int c = 0; c < 3; c++) {
        double m = 0.0;
        for (int64_t t = 0; t < N; t++) m += v[c * N + t];
        m /= (double)N;
        for (int64_t t = 0; t < N; t++) v[c * N + t] -= m;
    }
}

/* Jacobi-preconditioned conjugate gradients for A u = div(C:E), A = -div C grad,
 * on the zero-mean subspace (A is singular only on the three rigid translations).
 * u: in = initial guess, out = solution.  Stops when ||b - A u|| <= rtol ||b||.
 * Returns the iteration count; *relres gets the final true relative residual
 * (recomputed from u, not the recursive one).  hist (optional, length hist_cap)
 * receives the recursive relative residual of every iteration. */
static int64_t m_pcg(const grid_t *gp, const mat_t *m, const double E[6], double rtol, int64_t max_iter,
                     double *u, double *relres, double *hist, int64_t hist_cap) {
    const grid_t g = *gp;
    const int64_t N = g.nx * g.ny * g.nz, n3 = 3 * N;
    const double zero[6] = {0, 0, 0, 0, 0, 0};
    double *r = malloc(sizeof(double) * n3), *z = malloc(sizeof(double) * n3);
    double *p = malloc(sizeof(double) * n3), *q = malloc(sizeof(double) * n3);
    double *dg = malloc(sizeof(double) * n3), *b = malloc(sizeof(double) * n3);
    diagonal(&g, m, dg);
    m_residual(&g, m, E, u, r); /* r = div C (E + grad u) = b - A u */
    {
        double *u0 = calloc(n3, sizeof(double));
        m_residual(&g, m, E, u0, b); /* b = div C E */
        free(u0);
    }
    double bnorm = sqrt(dot(n3, b, b));
    int64_t it = 0;
    if (bnorm == 0.0) {
        *relres = 0.0;
        goto done;
    }
    for (int64_t t = 0; t < n3; t++) z[t] = r[t] / dg[t];
    if (m->walls) mask_walls(&g, z); else remove_mean(N, z);
    memcpy(p, z, sizeof(double) * n3);
    double rz = dot(n3, r, z);
    for (it = 0; it < max_iter; it++) {
        double rn = sqrt(dot(n3, r, r)) / bnorm;
        if (hist && it < hist_cap) hist[it] = rn;
        if (rn <= rtol) break;
        /* q = A p = -div C grad p */
        m_residual(&g, m, zero, p, q);
        for (int64_t t = 0; t < n3; t++) q[t] = -q[t];
        double alpha = rz / dot(n3, p, q);
        for (int64_t t = 0; t < n3; t++) {
            u[t] += alpha * p[t];
            r[t] -= alpha * q[t];
        }
        for (int64_t t = 0; t < n3; t++) z[t] = r[t] / dg[t];
        if (m->walls) mask_walls(&g, z); else remove_mean(N, z);
        double rz_new = dot(n3, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t t = 0; t < n3; t++) p[t] = z[t] + beta * p[t];
    }
    if (!m->walls) remove_mean(N, u);
    m_residual(&g, m, E, u, r);
    *relres = sqrt(dot(n3, r, r)) / bnorm;
done:
    free(r); free(z); free(p); free(q); free(dg); free(b);
    return it;
}

int64_t or_pcg(const int64_t dims[3], const double h[3], const double *K, const double *G,
               const double E[6], double rtol, int64_t max_iter, double *u, double *relres,
               double *hist, int64_t hist_cap) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {K, G, NULL, 0, NULL};
    return m_pcg(&g, &m, E, rtol, max_iter, u, relres, hist, hist_cap);
}

int64_t or_pcg_ortho(const int64_t dims[3], const double h[3], const double *c9, const double E[6], double rtol,
                     int64_t max_iter, double *u, double *relres, double *hist, int64_t hist_cap) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {NULL, NULL, c9, 0, NULL};
    return m_pcg(&g, &m, E, rtol, max_iter, u, relres, hist, hist_cap);
}

/* Stiffness that limits the explicit step of face displacements of direction d
 * in cell c: for isotropic cells K + 4G/3; for orthotropic cells the largest of
 * the normal constant and the two shear constants acting on that component
 * (x: C11, C66, C55; y: C22, C66, C44; z: C33, C55, C44), which bounds the
 * diagonal of the operator the same way K + 4G/3 does in the isotropic case. */
static double step_stiffness(const mat_t *m, int64_t N, int d, int64_t c) {
    if (m->c21) {
        /* general cells: the same three rows (x: 11, 66, 55; y: 22, 66, 44; z: 33, 55, 44),
         * each diagonal constant raised by the absolute values of the constants of its row
         * that an orthotropic cell does not have (a Gershgorin bound of the coupled row) */
        static const int rows[3][3] = {{0, 5, 4}, {1, 5, 3}, {2, 4, 3}};
        double best = 0.0;
        for (int t = 0; t < 3; t++) {
            const int r = rows[d][t];
            double v = m->c21[(int64_t)tri_q(r, r) * N + c];
            for (int q = 0; q < 6; q++) {
                const int ortho = (r < 3 && q < 3) || q == r;
                if (!ortho) v += fabs(m->c21[(int64_t)tri_q(r, q) * N + c]);
            }
            best = fmax(best, v);
        }
        return best;
    }
    if (!m->c9) return m->K[c] + 4.0 * m->G[c] / 3.0;
    static const int sh[3][2] = {{8, 7}, {8, 6}, {7, 6}};
    double a = m->c9[d * N + c], b = m->c9[sh[d][0] * N + c], e = m->c9[sh[d][1] * N + c];
    return fmax(a, fmax(b, e));
}

/* The APT iteration written on the displacement fluctuation alone.  With unit
 * physical step and pseudo moduli equal to the local moduli, the stress of the
 * paper's relaxation equations is an exponential average of Hooke's stress, and
 * eliminating it from the momentum equation leaves the two-level recurrence
 *   u^1     = u^0 + (beta / H_f) r(u^0)
 *   u^{n+1} = u^n + a (u^n - u^{n-1}) + (a c beta / H_f) r(u^n)
 * with r = div C:(E + grad u), c = ell St / Lx, beta = ell Lx / St, a = 1/(1+c),
 * ell = courant / sqrt(sum 1/h^2), Lx the largest box edge, and H_f the larger
 * step stiffness of the two cells a face separates.  For isotropic cells this
 * is the same iterate sequence as or_apt_steps (tests check that); for
 * orthotropic cells it is the definition of the iteration.
 * Starts from u^0 = 0 and returns u^nsteps in u (3N) and u^(nsteps-1) in u_prev
 * (3N, may be NULL). */
static void m_apt_disp(const grid_t *g, const mat_t *m, const double E[6], double courant, double strouhal,
                       int64_t nsteps, double *u, double *u_prev) {
    const int64_t N = g->nx * g->ny * g->nz, n3 = 3 * N;
    double Lx = fmax(fmax(g->nx * g->hx, g->ny * g->hy), g->nz * g->hz);
    double ell = courant / sqrt(1.0 / (g->hx * g->hx) + 1.0 / (g->hy * g->hy) + 1.0 / (g->hz * g->hz));
    double c = ell * strouhal / Lx, beta = ell * Lx / strouhal, a = 1.0 / (1.0 + c);
    double *old = calloc(n3, sizeof(double)), *r = malloc(sizeof(double) * n3), *Hf = malloc(sizeof(double) * n3);
    for (int64_t t = 0; t < N; t++) {
        int64_t i = t % g->nx, j = (t / g->nx) % g->ny, k = t / (g->nx * g->ny);
        int64_t nb[3] = {at(g, i - 1, j, k), at(g, i, j - 1, k), at(g, i, j, k - 1)};
        for (int d = 0; d < 3; d++) Hf[d * N + t] = fmax(step_stiffness(m, N, d, t), step_stiffness(m, N, d, nb[d]));
    }
    memset(u, 0, sizeof(double) * n3);
    for (int64_t s = 0; s < nsteps; s++) {
        m_residual(g, m, E, u, r);
        for (int64_t t = 0; t < n3; t++) {
            double nu = s == 0 ? u[t] + beta / Hf[t] * r[t]
                               : u[t] + a * (u[t] - old[t]) + a * c * beta / Hf[t] * r[t];
            old[t] = u[t];
            u[t] = nu;
        }
    }
    if (u_prev) memcpy(u_prev, old, sizeof(double) * n3);
    free(old); free(r); free(Hf);
}

void or_apt_disp(const int64_t dims[3], const double h[3], const double *K, const double *G, const double *c9,
                 int walls, const double E[6], double courant, double strouhal, int64_t nsteps, double *u,
                 double *u_prev) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {K, G, c9, walls, NULL};
    m_apt_disp(&g, &m, E, courant, strouhal, nsteps, u, u_prev);
}

/* General anisotropic cells (c21: 21N constants, see the header): stresses,
 * residual, stress averages, Jacobi-PCG solve and displacement-form APT. */
void or_stress_tri(const int64_t dims[3], const double h[3], const double *c21, const double E[6],
                   const double *u, double *sig) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {NULL, NULL, NULL, 0, c21};
    m_stress(&g, &m, E, u, sig);
}

void or_residual_tri(const int64_t dims[3], const double h[3], const double *c21, const double E[6],
                     const double *u, double *r) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {NULL, NULL, NULL, 0, c21};
    m_residual(&g, &m, E, u, r);
}

void or_average_stress_tri(const int64_t dims[3], const double h[3], const double *c21, const double E[6],
                           const double *u, double out[6]) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {NULL, NULL, NULL, 0, c21};
    m_average_stress(&g, &m, E, u, out);
}

int64_t or_pcg_tri(const int64_t dims[3], const double h[3], const double *c21, const double E[6], double rtol,
                   int64_t max_iter, double *u, double *relres) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {NULL, NULL, NULL, 0, c21};
    return m_pcg(&g, &m, E, rtol, max_iter, u, relres, NULL, 0);
}

void or_apt_disp_tri(const int64_t dims[3], const double h[3], const double *c21, const double E[6], double courant,
                     double strouhal, int64_t nsteps, double *u, double *u_prev) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {NULL, NULL, NULL, 0, c21};
    m_apt_disp(&g, &m, E, courant, strouhal, nsteps, u, u_prev);
}

/* The APT iteration with the stress as its state, for any cell law of this file
 * (isotropic, orthotropic, general) and the wall tests.  It is the paper's
 * relaxation scheme with pseudo moduli equal to the local moduli: split into
 * pressure and deviator, the implicit relaxation of each is
 *   sigma <- (sigma + c * Hooke(E + grad v)) / (1 + c)
 * for the whole stress, so this is or_apt_steps written for a general Hooke map
 * (tests check that they agree on isotropic cells), followed by the momentum
 * update v <- v + (beta / H_f) div sigma with the face step stiffness H_f of the
 * displacement form.  Unlike the displacement form it keeps the stresses and the
 * split edges' side-1 halves as state and eliminates nothing.
 * Starts from v = 0 and sigma = Hooke(E); returns v after nsteps in u (3N) and
 * after nsteps - 1 in u_prev (3N, may be NULL). */
static void m_apt_stress(const grid_t *g, const mat_t *m, const double E[6], double courant, double strouhal,
                         int64_t nsteps, double *u, double *u_prev) {
    const int64_t N = g->nx * g->ny * g->nz, n3 = 3 * N;
    const int ws = m->walls;
    double Lx = fmax(fmax(g->nx * g->hx, g->ny * g->hy), g->nz * g->hz);
    double ell = courant / sqrt(1.0 / (g->hx * g->hx) + 1.0 / (g->hy * g->hy) + 1.0 / (g->hz * g->hz));
    double c = ell * strouhal / Lx, beta = ell * Lx / strouhal;
    double *sig = malloc(sizeof(double) * 6 * N), *hk = malloc(sizeof(double) * 6 * N);
    double *r = malloc(sizeof(double) * n3), *Hf = malloc(sizeof(double) * n3);
    double *half1 = calloc(N, sizeof(double));
    for (int64_t t = 0; t < N; t++) {
        int64_t i = t % g->nx, j = (t / g->nx) % g->ny, k = t / (g->nx * g->ny);
        int64_t nb[3] = {at(g, i - 1, j, k), at(g, i, j - 1, k), at(g, i, j, k - 1)};
        for (int d = 0; d < 3; d++) Hf[d * N + t] = fmax(step_stiffness(m, N, d, t), step_stiffness(m, N, d, nb[d]));
    }
    memset(u, 0, sizeof(double) * n3);
    m_stress(g, m, E, u, sig);
    if (ws >= 3) FOR_SPLIT_EDGES(g, ws, i, j, k) half1[at(g, i, j, k)] = half_edge(g, m, ws, E, u, i, j, k, 1);
    for (int64_t st = 0; st < nsteps; st++) {
        m_stress(g, m, E, u, hk);
        for (int64_t t = 0; t < 6 * N; t++) sig[t] = (sig[t] + c * hk[t]) / (1.0 + c);
        if (ws >= 3) FOR_SPLIT_EDGES(g, ws, i, j, k) {
            const int64_t ce = at(g, i, j, k);
            half1[ce] = (half1[ce] + c * half_edge(g, m, ws, E, u, i, j, k, 1)) / (1.0 + c);
        }
        divergence(g, sig, r);
        if (ws >= 3) {
            const int d = pair_d[ws], e = pair_e[ws];
            const double he = e == 1 ? g->hy : g->hz;
            FOR_SPLIT_EDGES(g, ws, i, j, k) {
                int64_t q[3] = {i, j, k};
                q[e] = (e == 1 ? g->ny : g->nz) - 1;
                const int64_t ce = at(g, i, j, k), cf = at(g, q[0], q[1], q[2]);
                r[d * N + cf] += (half1[ce] - sig[ws * N + ce]) / he;
            }
        }
        if (ws) mask_walls(g, r);
        if (u_prev) memcpy(u_prev, u, sizeof(double) * n3);
        for (int64_t t = 0; t < n3; t++) u[t] += beta / Hf[t] * r[t];
    }
    if (u_prev && nsteps == 0) memset(u_prev, 0, sizeof(double) * n3);
    free(sig); free(hk); free(r); free(Hf); free(half1);
}

void or_apt_stress(const int64_t dims[3], const double h[3], const double *K, const double *G, const double *c9,
                   const double *c21, int walls, const double E[6], double courant, double strouhal, int64_t nsteps,
                   double *u, double *u_prev) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {K, G, c9, walls, c21};
    m_apt_stress(&g, &m, E, courant, strouhal, nsteps, u, u_prev);
}

/* Wall-boundary versions (isotropic cells) of the residual, the stress averages
 * and the PCG solve; mode = 1 (normal test) or 3..5 (simple-shear test). */
void or_residual_walls(const int64_t dims[3], const double h[3], const double *K, const double *G,
                       const double E[6], const double *u, double *r, int mode) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {K, G, NULL, mode, NULL};
    m_residual(&g, &m, E, u, r);
}

void or_average_stress_walls(const int64_t dims[3], const double h[3], const double *K, const double *G,
                             const double E[6], const double *u, double out[6], int mode) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {K, G, NULL, mode, NULL};
    m_average_stress(&g, &m, E, u, out);
}

int64_t or_pcg_walls(const int64_t dims[3], const double h[3], const double *K, const double *G, const double E[6],
                     double rtol, int64_t max_iter, double *u, double *relres, int mode) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {K, G, NULL, mode, NULL};
    return m_pcg(&g, &m, E, rtol, max_iter, u, relres, NULL, 0);
}

/* Accelerated pseudo-transient iterations written in the paper's own variables
 * (pressure p, deviator tau, velocity v; "Solution of the system of equations").
 * Readings (design notes): the physical time step is 1, so v plays the role of
 * the displacement fluctuation; the pseudo moduli are the local moduli
 * (K~ = K, G~ = G), giving K~dt = c K, G~dt = c G with c = ell*St/Lx and
 * dt/rho~ = ell*Lx/(St*H~) at a face, H~ = max of K + 4G/3 over the two cells
 * the face separates; ell = courant / sqrt(1/hx^2 + 1/hy^2 + 1/hz^2); the
 * relaxation terms are taken implicitly; the solid viscosity term is dropped.
 * Initial state: v = 0, p = -K tr E, tau = 2G dev E (cells), tau_e = 2 G_e E_e.
 *
 * state (10N): p, txx, tyy, tzz (cells), tyz, txz, txy (edges), vx, vy, vz (faces).
 * If init != 0 the state is first set to the initial state above.  Runs nsteps.
 *
 * Under the wall conditions of the direct tests (m->walls as in the other wall
 * functions; 0 is the periodic medium) wall faces keep v = 0, the free boundary
 * edges carry no shear stress, and under the simple-shear test s each split edge
 * holds two half-edge stresses, each relaxed towards its own Hooke stress
 * (half_edge) as every other stress is.  The side-0 halves are kept in the edge
 * field, the side-1 halves in half1 (N entries, indexed like the edge; used for
 * s >= 3 only, may be NULL otherwise); their difference enters the u_d faces of
 * index n_e - 1, as in the residual.  Initial halves: half_edge of v = 0. */
static void m_apt_steps(const grid_t *gp, const mat_t *m, const double E[6], double courant, double strouhal,
                        int init, int64_t nsteps, double *state, double *half1) {
    const grid_t g = *gp;
    const double *K = m->K, *G = m->G;
    const int ws = m->walls;
    const int64_t N = g.nx * g.ny * g.nz;
    double *p = state, *txx = state + N, *tyy = state + 2 * N, *tzz = state + 3 * N;
    double *tyz = state + 4 * N, *txz = state + 5 * N, *txy = state + 6 * N;
    double *v = state + 7 * N;
    double *tau_e[6] = {NULL, NULL, NULL, tyz, txz, txy};
    double Lx = fmax(fmax(g.nx * g.hx, g.ny * g.hy), g.nz * g.hz);
    double ell = courant / sqrt(1.0 / (g.hx * g.hx) + 1.0 / (g.hy * g.hy) + 1.0 / (g.hz * g.hz));
    double c = ell * strouhal / Lx;           /* pseudo step / physical step */
    double rho_fac = ell * Lx / strouhal;     /* dt~/rho~ = rho_fac / H~ */
    double *eps = malloc(sizeof(double) * 6 * N);
    if (init) {
        double trE = E[0] + E[1] + E[2];
        for (int64_t t = 0; t < N; t++) {
            int64_t i = t % g.nx, j = (t / g.nx) % g.ny, k = t / (g.nx * g.ny);
            p[t] = -K[t] * trE;
            txx[t] = 2.0 * G[t] * (E[0] - trE / 3.0);
            tyy[t] = 2.0 * G[t] * (E[1] - trE / 3.0);
            tzz[t] = 2.0 * G[t] * (E[2] - trE / 3.0);
            tyz[t] = 2.0 * edge_modulus(&g, G, 2, i, j, k) * E[3];
            txz[t] = 2.0 * edge_modulus(&g, G, 1, i, j, k) * E[4];
            txy[t] = 2.0 * edge_modulus(&g, G, 0, i, j, k) * E[5];
            v[t] = v[N + t] = v[2 * N + t] = 0.0;
            if (ws)
                for (int s = 3; s < 6; s++)
                    if (wall_edge(m, s, i, j, k) == 1) tau_e[s][t] = 0.0;
        }
        if (ws >= 3) FOR_SPLIT_EDGES(&g, ws, i, j, k) {
            const int64_t ce = at(&g, i, j, k);
            tau_e[ws][ce] = half_edge(&g, m, ws, E, v, i, j, k, 0);
            half1[ce] = half_edge(&g, m, ws, E, v, i, j, k, 1);
        }
    }
    double *sig = malloc(sizeof(double) * 6 * N), *r = malloc(sizeof(double) * 3 * N);
    for (int64_t st = 0; st < nsteps; st++) {
        /* strain rates from the current velocities (with the macroscopic strain) */
        strains(&g, E, v, eps);
        for (int64_t t = 0; t < N; t++) {
            int64_t i = t % g.nx, j = (t / g.nx) % g.ny, k = t / (g.nx * g.ny);
            double th = eps[t] + eps[N + t] + eps[2 * N + t];
            double Kdt = c * K[t], Gdt = c * G[t];
            /* (1/K~) dp/dt~ + p/(K dt) = -div v, implicit in p */
            p[t] = (p[t] - Kdt * th) / (1.0 + Kdt / K[t]);
            /* (1/2G~) dtau/dt~ + tau/(2G dt) = dev(strain rate), implicit in tau */
            txx[t] = (txx[t] + 2.0 * Gdt * (eps[t] - th / 3.0)) / (1.0 + Gdt / G[t]);
            tyy[t] = (tyy[t] + 2.0 * Gdt * (eps[N + t] - th / 3.0)) / (1.0 + Gdt / G[t]);
            tzz[t] = (tzz[t] + 2.0 * Gdt * (eps[2 * N + t] - th / 3.0)) / (1.0 + Gdt / G[t]);
            /* edges: pseudo and physical shear modulus are the edge's harmonic G_e; free
             * boundary edges stay at zero, split edges are relaxed below */
            for (int s = 3; s < 6; s++) {
                const int we = ws ? wall_edge(m, s, i, j, k) : 0;
                if (we) continue;
                double Ge = edge_modulus(&g, G, 5 - s, i, j, k), Gedt = c * Ge;
                tau_e[s][t] = (tau_e[s][t] + 2.0 * Gedt * eps[s * N + t]) / (1.0 + Gedt / Ge);
            }
        }
        if (ws >= 3) FOR_SPLIT_EDGES(&g, ws, i, j, k) {
            const int64_t ce = at(&g, i, j, k);
            tau_e[ws][ce] = (tau_e[ws][ce] + c * half_edge(&g, m, ws, E, v, i, j, k, 0)) / (1.0 + c);
            half1[ce] = (half1[ce] + c * half_edge(&g, m, ws, E, v, i, j, k, 1)) / (1.0 + c);
        }
        /* momentum with pseudo inertia: rho~ dv/dt~ = div(-p I + tau) */
        for (int64_t t = 0; t < N; t++) {
            sig[t] = -p[t] + txx[t];
            sig[N + t] = -p[t] + tyy[t];
            sig[2 * N + t] = -p[t] + tzz[t];
            sig[3 * N + t] = tyz[t];
            sig[4 * N + t] = txz[t];
            sig[5 * N + t] = txy[t];
        }
        divergence(&g, sig, r);
        if (ws >= 3) {
            const int d = pair_d[ws], e = pair_e[ws];
            const double he = e == 1 ? g.hy : g.hz;
            FOR_SPLIT_EDGES(&g, ws, i, j, k) {
                int64_t q[3] = {i, j, k};
                q[e] = (e == 1 ? g.ny : g.nz) - 1;
                const int64_t ce = at(&g, i, j, k), cf = at(&g, q[0], q[1], q[2]);
                r[d * N + cf] += (half1[ce] - sig[ws * N + ce]) / he;
            }
        }
        if (ws) mask_walls(&g, r); /* wall faces are held */
        for (int64_t t = 0; t < N; t++) {
            int64_t i = t % g.nx, j = (t / g.nx) % g.ny, k = t / (g.nx * g.ny);
            double Hc = K[t] + 4.0 * G[t] / 3.0;
            int64_t nb[3] = {at(&g, i - 1, j, k), at(&g, i, j - 1, k), at(&g, i, j, k - 1)};
            for (int d = 0; d < 3; d++) {
                double Hn = K[nb[d]] + 4.0 * G[nb[d]] / 3.0;
                double Hf = Hc > Hn ? Hc : Hn;
                v[d * N + t] += rho_fac / Hf * r[d * N + t];
            }
        }
    }
    free(eps); free(sig); free(r);
}

void or_apt_steps(const int64_t dims[3], const double h[3], const double *K, const double *G,
                  const double E[6], double courant, double strouhal, int init, int64_t nsteps,
                  double *state) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {K, G, NULL, 0, NULL};
    m_apt_steps(&g, &m, E, courant, strouhal, init, nsteps, state, NULL);
}

void or_apt_steps_walls(const int64_t dims[3], const double h[3], const double *K, const double *G,
                        const double E[6], double courant, double strouhal, int init, int64_t nsteps,
                        double *state, double *half1, int mode) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    mat_t m = {K, G, NULL, mode, NULL};
    m_apt_steps(&g, &m, E, courant, strouhal, init, nsteps, state, half1);
}

/* Gradient of J = sum_IJ W_IJ C_IJ with respect to per-voxel K and G.
 * u6: the six converged fluctuation fields (6 x 3N, load-major), for unit Voigt
 * loads.  Uses the stationarity of each solution, so only the explicit
 * dependence of the strain energy on the moduli enters:
 *   dC_IJ/dK_c = theta^I theta^J / N
 *   dC_IJ/dG_c = [2 sum_d e'^I_dd e'^J_dd + sum_{edges e at c} (G_e/G_c)^2 eps^I_e eps^J_e] / N
 * where e' is the deviatoric normal strain and the edge sum runs over the 12
 * edges that touch cell c (d G_e / d G_c = G_e^2 / (4 G_c^2); edge energy 2 G_e eps^2
 * counted for both symmetric components). */
void or_gradient(const int64_t dims[3], const double h[3], const double *K, const double *G,
                 const double *u6, const double W[36], double *dK, double *dG) {
    grid_t g = {dims[0], dims[1], dims[2], h[0], h[1], h[2]};
    const int64_t N = g.nx * g.ny * g.nz;
    double *eps = malloc(sizeof(double) * 36 * N);
    for (int J = 0; J < 6; J++) {
        double E[6] = {0, 0, 0, 0, 0, 0};
        E[J] = J < 3 ? 1.0 : 0.5;
        strains(&g, E, u6 + (int64_t)J * 3 * N, eps + (int64_t)J * 6 * N);
    }
    (void)K;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < g.nz; k++)
        for (int64_t j = 0; j < g.ny; j++)
            for (int64_t i = 0; i < g.nx; i++) {
                int64_t c = at(&g, i, j, k);
                double gk = 0.0, gg = 0.0;
                /* the 12 edges touching cell c: (plane, di, dj, dk) offsets of the edge index */
                static const int eoff[12][4] = {
                    {0, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 1, 1, 0},
                    {1, 0, 0, 0}, {1, 1, 0, 0}, {1, 0, 0, 1}, {1, 1, 0, 1},
                    {2, 0, 0, 0}, {2, 0, 1, 0}, {2, 0, 0, 1}, {2, 0, 1, 1}};
                for (int I = 0; I < 6; I++)
                    for (int J = 0; J < 6; J++) {
                        double w = W[I * 6 + J];
                        if (w == 0.0) continue;
                        const double *a = eps + (int64_t)I * 6 * N, *b = eps + (int64_t)J * 6 * N;
                        double tha = a[c] + a[N + c] + a[2 * N + c];
                        double thb = b[c] + b[N + c] + b[2 * N + c];
                        gk += w * tha * thb;
                        double dev = 0.0;
                        for (int d = 0; d < 3; d++)
                            dev += (a[d * N + c] - tha / 3.0) * (b[d * N + c] - thb / 3.0);
                        double ed = 0.0;
                        for (int e = 0; e < 12; e++) {
                            int pl = eoff[e][0];
                            int64_t ei = i + eoff[e][1], ej = j + eoff[e][2], ek = k + eoff[e][3];
                            int64_t ec = at(&g, ei, ej, ek);
                            double Ge = edge_modulus(&g, G, pl, ei, ej, ek);
                            int comp = pl == 0 ? 5 : (pl == 1 ? 4 : 3);
                            double q = Ge / G[c];
                            ed += q * q * a[comp * N + ec] * b[comp * N + ec];
                        }
                        gg += w * (2.0 * dev + ed);
                    }
                dK[c] = gk / (double)N;
                dG[c] = gg / (double)N;
            }
    free(eps);
}
