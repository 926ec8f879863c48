/*
 * ceff -- effective elastic stiffness of a voxel image on one MI355X GPU.
 *
 * Computes the 6x6 effective stiffness C* of a heterogeneous linear-elastic
 * voxel image (paper: "Effective elastic properties", the volume averages of
 * stress and strain and the relation <sigma_ij> = C*_ijkl <eps_kl>).  Each
 * requested column J is the volume-averaged stress of the equilibrium state
 * (paper: eqs. 1-3, "Closed System of Equations") under the J-th unit
 * macroscopic Voigt strain with periodic boundary conditions, found with the
 * accelerated pseudo-transient iteration (paper: "Solution of the system of
 * equations") on the staggered grid of the paper's "Discretization" section.
 *
 * Conventions
 *   - Grid: nx x ny x nz voxels (cells) of size hx x hy x hz.  Per-voxel
 *     arrays have N = nx*ny*nz entries, x fastest: index i + nx*(j + ny*k).
 *   - Voigt order 11, 22, 33, 23, 13, 12 with engineering shear: load J = 3
 *     (0-based; the fourth column) applies eps_yz = eps_zy = 1/2.
 *   - Units: any consistent set; C* comes out in the units of K and G.
 *   - C matrices are row-major doubles: C[I*6 + J].
 *   - Inputs are read during the call only and remain owned by the caller.
 *     Device pointers must live on the context's device; the library waits
 *     for work already queued on the context's stream before reading them.
 *     Outputs are caller-allocated.
 *   - Every entry point returns a status and never aborts; the message of
 *     the last failure is available from ceff_last_error.  A context is not
 *     thread safe: one host thread at a time.
 *   - Nothing here needs a GPU to fail cleanly: argument errors are detected
 *     before any device call, and ceff_create returns CEFF_EDEVICE when no
 *     usable device exists.
 */
#ifndef CEFF_H
#define CEFF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ceff_ctx ceff_ctx;

typedef enum {
  CEFF_OK = 0,
  CEFF_EINVAL = -1,        /* bad argument */
  CEFF_ENOMEM = -2,        /* device or host allocation failed */
  CEFF_EDEVICE = -3,       /* HIP runtime error, or no usable device */
  CEFF_ENOTCONV = -4,      /* max_iter reached; outputs hold the last iterate */
  CEFF_EDIVERGED = -5,     /* residual non-finite or grew by 1e6 */
  CEFF_EUNSUPPORTED = -6,  /* valid request this build does not implement */
  CEFF_ESTATE = -7         /* call out of order (no grid, no material, no kept fields) */
} ceff_status;

enum { CEFF_F32 = 0, CEFF_F64 = 1 };          /* element type of caller arrays */
enum { CEFF_HOST = 0, CEFF_DEVICE = 1 };      /* where caller arrays live */
enum { CEFF_PREC_FP64 = 0, CEFF_PREC_MIXED = 1 };
enum { CEFF_FUSE_AUTO = -1 };                 /* ceff_solve_opts.fuse_loads: let the library choose */
enum { CEFF_BC_PERIODIC = 0, CEFF_BC_WALLS = 1 };  /* ceff_set_boundary */

typedef struct {
  int precision;        /* CEFF_PREC_FP64: all sweeps in FP64.
                           CEFF_PREC_MIXED: sweeps in FP32 on a correction of an FP64
                           displacement; FP64 residuals decide convergence. */
  double rtol;          /* stop when ||div sigma(u)||_2 <= rtol * ||div(C:E)||_2 (FP64) */
  int64_t max_iter;     /* iteration cap per load */
  int check_every;      /* iterations between residual checks (rounded up to even) */
  double courant;       /* CFL number in (0, 1]: ell = courant / sqrt(sum 1/h^2) */
  double strouhal;      /* St of the paper's numerical parameters: > 0, or 0 (the default) for
                           the automatic choice of ceff_auto_strouhal, per sample.  St sets
                           only the damping of the iteration, never its fixed point. */
  int fuse_loads;       /* 1: all requested loads advance in one launch per iteration;
                           0: one load after another;
                           CEFF_FUSE_AUTO: one after another for a phase image in mixed
                           precision (the loads share only the phase id); otherwise one after
                           another when the iteration working set of one load (two displacement
                           buffers + moduli) fits in the GPU's Infinity Cache (256 MiB) and that
                           of all requested loads does not, fused otherwise.  Results do not
                           depend on this choice. */
  int use_graph;        /* 1: replay each block of check_every iterations as a HIP graph */
  int keep_fields;      /* 1: keep the converged FP64 displacements for ceff_gradient */
  int autotune;         /* 1: time candidate launch shapes (block extent, z-chunk, loads per
                           block, kernel variant, occupancy) on the problem first and use the
                           fastest; the iterates do not depend on the shape.  The choice is
                           cached per context by precision, loads, phase-table use, sample
                           dimensions and kernel build, and, when the environment variable
                           CEFF_TUNE_CACHE names a file, appended to that file and read back
                           by later processes.  0: the built-in shapes (no cache lookup). */
  double fold_ratio;    /* MIXED: fold the FP32 correction into the FP64 displacement when
                           the residual fell by this factor since the last fold */
  const double* warm_u; /* optional initial displacement fluctuation (host FP64, 6 x 3N,
                           load-major: load J's u_x, u_y, u_z at warm_u + J*3N, component-
                           major like ceff_residual's u), or NULL for the zero start.  MIXED:
                           it becomes the FP64 displacement and the FP32 sweeps start on a
                           zero correction with its residual as the body force (as after a
                           fold); FP64: it is the first iterate.  Relative residuals stay
                           normalised by the zero start's ||div(C:E)||.  ceff_solve only,
                           periodic boundaries (CEFF_EUNSUPPORTED with walls). */
} ceff_solve_opts;

/* Execution counters of the most recent solve (for roofline accounting). */
typedef struct {
  int64_t step_launches;   /* launches of the iteration kernel */
  double step_time_ms;     /* device time of those launches, from HIP events on the solve stream */
  double step_bytes;       /* algorithmic HBM bytes of those launches: per voxel and active load
                              9 words of displacement (+3 with a body force), plus K and G once
                              (or the 1-byte phase id, see phase_moduli) */
  double voxel_updates;    /* sum over launches of N * active loads */
  int64_t outer_checks;    /* FP64 residual evaluations */
  double solve_ms;         /* host wall time of the solve call */
  int tile_bx, tile_by, tile_kc;  /* tile shape used (block extent incl. ghosts, z-chunk) */
  int tile_group;          /* loads per block */
  int tile_variant;        /* iteration-kernel variant: 0 plain z-march; 1 next plane prefetched into
                              registers; 2 march unrolled by two planes; 3 as 2 with all loads of a block
                              between one barrier pair per plane; 4 as 3 unrolled by three, loads issued
                              one plane ahead; 5 one load per block, in-plane neighbours read through the
                              caches instead of LDS; 6 two iterations per launch (CEFF_TB=1); 9 one load
                              per block in rows of 16, 32 or 64 cells, x-neighbour values exchanged
                              between the lanes of a wave (the default for FP32 and for
                              one-load FP64 solves of periodic isotropic cells) */
  int fused_loads;         /* 1 if the requested loads advanced together, one launch per iteration */
  int phase_moduli;        /* 1: the iteration kernel read each cell's 1-byte phase id and a per-phase
                              table (material set with ceff_set_phases) instead of the K and G fields */
  int tile_occ;            /* 1: the high-occupancy build of the iteration kernel (fewer registers) */
} ceff_stats;

/* Fill *o with the defaults: MIXED, rtol 1e-8, max_iter 2e6, check_every 100,
 * courant 0.95, strouhal 0 (automatic), fuse_loads CEFF_FUSE_AUTO, use_graph 1, keep_fields 0,
 * autotune 0, fold_ratio 1e-3, warm_u NULL. */
void ceff_default_opts(ceff_solve_opts* o);

/* The Strouhal number that strouhal = 0 selects for a box of nx x ny x nz cells
 * of size hx x hy x hz and the given Courant number (paper, "Solution of the
 * system of equations": St sets the damping of the iteration; the paper's
 * optimum is derived for a homogeneous medium).  With ell = courant /
 * sqrt(sum 1/h^2) and Lx = max n_d h_d the damping is c = ell St / Lx, and
 *   St = min(max(0.010 Lx / ell, 2), 8.3),
 * i.e. c = 0.010 (the best damping measured for fluid-filled pore images, which
 * stays nearly constant from 64^3 to 256^3), St at least 2 in small boxes and at
 * most 8.3 (a box-scale mode limits large ones: 703^3 pores converge fastest
 * near St 8).  Host only; CEFF_EINVAL for a bad grid or courant outside (0, 1]. */
ceff_status ceff_auto_strouhal(int64_t nx, int64_t ny, int64_t nz, double hx, double hy, double hz, double courant,
                               double* st_out);

/* Check a grid against this build's limits without a context or a device: each
 * dimension in [2, 2^20], one z-plane nx*ny of at most 2^28 cells (2 GiB of
 * FP64), spacings finite and > 0.  Returns CEFF_OK or CEFF_EINVAL.  The same
 * check guards ceff_set_grid and the batch calls.  There is no limit on the
 * total number of cells beyond device memory: the iteration kernels address a
 * field one z-plane at a time, with a 32-bit offset within the plane.  Host
 * only; needs no device. */
ceff_status ceff_check_grid(int64_t nx, int64_t ny, int64_t nz, double hx, double hy, double hz);

/* Create a context on HIP device `device` (runtime plumbing with no paper
 * counterpart).  hip_stream: a hipStream_t the caller orders its device inputs
 * on (NULL = the null stream).  The library runs its own work on an internal
 * stream of default priority.  CEFF_EDEVICE if the device is not usable. */
ceff_status ceff_create(int device, void* hip_stream, ceff_ctx** out);
void ceff_destroy(ceff_ctx* ctx);
/* Message of the last failure (context-owned; valid until the next call). */
const char* ceff_last_error(const ceff_ctx* ctx);

/* Grid dimensions (each in [2, 2^20], with nx*ny <= 2^28) and voxel spacings
 * (> 0), the cells of the paper's staggered grid ("Discretization").  Clears
 * material and kept fields.  CEFF_EINVAL for a grid outside the limits (see
 * ceff_check_grid). */
ceff_status ceff_set_grid(ceff_ctx* ctx, int64_t nx, int64_t ny, int64_t nz, double hx, double hy, double hz);

/* Per-voxel isotropic moduli K(x), G(x) (paper: each voxel carries the bulk
 * and shear moduli of its material, "Discretization").  N values each, dtype
 * CEFF_F32/CEFF_F64, host or device; copied.  All values must be finite and > 0. */
ceff_status ceff_set_isotropic(ceff_ctx* ctx, const void* K, const void* G, int dtype, int where);

/* Phase image (uint8, N values, host or device) plus per-phase moduli
 * (host doubles, nphase entries, finite and > 0).  Every phase id must be < nphase. */
ceff_status ceff_set_phases(ceff_ctx* ctx, const uint8_t* phase, int where, int nphase, const double* K_tab,
                            const double* G_tab);

/* Anisotropic local stiffness c_ijkl(x) (paper, "Future perspectives", items
 * 2-3).  ncomp = 9: orthotropic cells with axes aligned with the grid, given as
 * 9 x N values, component-major (c[q*N + cell]), q = 0..8:
 *   C11 C22 C33 C23 C13 C12 C44 C55 C66   (Voigt, engineering shear).
 * Normal stresses at a cell are its 3x3 normal block times the normal strains;
 * the shear stress at an edge is 2 eps times the harmonic mean, over the four
 * cells around the edge, of C44 (yz-edges), C55 (xz) or C66 (xy), as for G in
 * the isotropic case (isotropic cells: C11 = K + 4G/3, C12 = K - 2G/3, C44 = G).
 * dtype CEFF_F32/CEFF_F64, host or device; copied.  Every constant must be
 * finite, the diagonal ones > 0 and each normal block positive definite, else
 * CEFF_EINVAL.
 * ncomp = 21: general anisotropic (triclinic) cells, 21 x N values, component-
 * major, the upper triangle of each cell's symmetric 6x6 Voigt matrix row by
 * row: C11 C12 C13 C14 C15 C16 C22 C23 C24 C25 C26 C33 C34 C35 C36 C44 C45 C46
 * C55 C56 C66.  The coupled law needs strains shared between cells and edges
 * (the paper's perspectives: "averaging of some local fields"): each cell is
 * split into eight corner octants, each with the cell's normal strains and, for
 * each shear component, the strain of that component's edge meeting its corner
 * times S_e / S_cell (S: the component's diagonal constant C44, C55 or C66, S_e
 * its harmonic mean over the edge's four cells); the energy is the mean over
 * octants of 1/2 eps : C : eps, summed over cells.  Without couplings this is
 * the orthotropic law above.  Every cell must be finite and positive definite,
 * else CEFF_EINVAL.  Such materials run one load at a time, with four launches
 * per iteration and 24 N words of scratch; CEFF_EUNSUPPORTED with wall
 * boundaries and in ceff_average_stress_noalloc.
 * Replaces any material set before; ceff_gradient is not available for
 * anisotropic materials. */
ceff_status ceff_set_stiffness(ceff_ctx* ctx, const void* c, int ncomp, int dtype, int where);

/* Boundary conditions of the context's problem (default CEFF_BC_PERIODIC).
 * CEFF_BC_WALLS: the paper's direct tests (appendix on boundary conditions).
 * On the periodic grid layout the box boundary in direction d is the grid
 * plane of index 0 in d; there the displacement fluctuation of the d-faces is
 * held at zero, so every face of the box is a rigid wall in its normal
 * direction that moves with the macroscopic strain (e.g. by E_zz * L_z in z).
 *   Loads 0-2 (normal compression and the tests for the off-diagonal
 *   constants): every edge lying in a boundary plane carries no shear stress
 *   (free slip).  Each load gives a column of the confined-compression
 *   stiffness, whose upper 3x3 block is what the paper's C11, C22, C33 and its
 *   formulas for C12, C13, C23 compute.
 *   Loads 3-5 (simple shear of yz, xz, xy): the load shears direction d = y, x,
 *   x across the walls normal to e = z, z, y.  Those loaded walls also hold u_d
 *   (no slip): each of the load's own edges in the e-boundary plane is split
 *   into two half edges, one per side of the box, with the one-sided
 *   derivative to the wall and the harmonic mean of that side's two cells,
 *   each counting as half an edge in the average.  The load's own edges in the
 *   d-boundary plane are computed as inside; all other boundary edges are free.
 *   The mean shear strain is then exactly the load's, and C(J, J) is the
 *   paper's C44, C55, C66.
 * The loads run one after another; orthotropic cells, the batch path and the
 * gradient need periodic boundaries (CEFF_EUNSUPPORTED).  Applies to
 * ceff_solve, ceff_apt_steps, ceff_residual and ceff_average_stress. */
ceff_status ceff_set_boundary(ceff_ctx* ctx, int mode);

/* Solve the unit loads in load_mask (bit J = Voigt column J, 0..5) and write
 * those columns of C_out (other entries untouched).  opts may be NULL
 * (defaults).  hist (optional, 3*hist_cap doubles) receives (iteration, load,
 * relative residual) triples of every check; *hist_len their count.
 * iters_out (optional, 6 entries) gets the iterations per load (0 when the
 * affine guess is already in equilibrium, also up to rounding: its residual
 * below 1e-13 of sqrt(3N) max|<sigma>| 2/h_min).  On CEFF_ENOTCONV/CEFF_EDIVERGED
 * the columns hold the stress averages of the last iterate. */
ceff_status ceff_solve(ceff_ctx* ctx, uint32_t load_mask, const ceff_solve_opts* opts, double C_out[36],
                       double* hist, int64_t hist_cap, int64_t* hist_len, int64_t iters_out[6]);

/* Solve nsamples independent images of (possibly) different sizes together:
 * every iteration is one launch over all unconverged (sample, load) pairs.
 * dims: 3 per sample (nx, ny, nz); h: 3 per sample; K[s], G[s]: per-voxel
 * moduli of sample s (dtype, where as in ceff_set_isotropic).  C_out: 36 per
 * sample; iters_out: 6 per sample (optional).  Does not change the context's
 * grid or material. */
ceff_status ceff_solve_batch(ceff_ctx* ctx, int nsamples, const int64_t* dims, const double* h,
                             const void* const* K, const void* const* G, int dtype, int where, uint32_t load_mask,
                             const ceff_solve_opts* opts, double* C_out, int64_t* iters_out);

/* As ceff_solve_batch for phase images that share one phase table: phase[s]
 * is sample s's uint8 image (N_s values, host or device per `where`), K_tab
 * and G_tab the per-phase moduli (host doubles, nphase entries, finite and
 * > 0; every phase id < nphase, else CEFF_EINVAL).  The FP32 iteration then
 * reads one byte per voxel and the moduli from an on-chip copy of the table,
 * as for ceff_set_phases; the results equal those of ceff_solve_batch on the
 * expanded K and G fields.  Does not change the context's grid or material. */
ceff_status ceff_solve_batch_phases(ceff_ctx* ctx, int nsamples, const int64_t* dims, const double* h,
                                    const uint8_t* const* phase, int where, int nphase, const double* K_tab,
                                    const double* G_tab, uint32_t load_mask, const ceff_solve_opts* opts,
                                    double* C_out, int64_t* iters_out);

/* Gradient of J = sum_IJ W[I*6+J] C_IJ with respect to the per-voxel K and G
 * of the current material (the building block of inverse problems that the
 * paper's "Future perspectives", item 5, names for this solver), from the displacements kept by the last
 * ceff_solve (keep_fields = 1, all loads that W touches; isotropic materials
 * only, else CEFF_EUNSUPPORTED).  The solution is
 * stationary, so only the explicit dependence of the strain energy on the
 * moduli enters (no second solve).  dK, dG: N values each, dtype, host or
 * device. */
ceff_status ceff_gradient(ceff_ctx* ctx, const double W[36], void* dK, void* dG, int dtype, int where);

/* ---- single-step entry points (for step-level checks) --------------------- */

/* Run the first nsteps iterations of load J from the affine initial state
 * (strouhal = 0: the automatic choice)
 * (FP64 or MIXED = FP32 arithmetic, no defect correction) and return the
 * displacement iterate u^nsteps and u^(nsteps-1) as host doubles (3N each,
 * component-major; u_prev_out may be NULL). */
ceff_status ceff_apt_steps(ceff_ctx* ctx, int J, int64_t nsteps, int precision, double courant, double strouhal,
                           double* u_out, double* u_prev_out);

/* Out-of-balance force div(C:(E_J + grad u)) of a host displacement u (3N
 * doubles) at the faces, in FP64 (precision FP64) or FP32 arithmetic
 * (MIXED).  r_out (3N, may be NULL) and *norm2 (sum of squares, may be NULL). */
ceff_status ceff_residual(ceff_ctx* ctx, int J, int precision, const double* u, double* r_out, double* norm2);

/* FP64 volume averages of the six stresses of displacement u (host, 3N) under
 * unit load J, Voigt order (paper: the volume-averaged stress). */
ceff_status ceff_average_stress(ceff_ctx* ctx, int J, const double* u, double out6[6]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): ceff_average_stress
 * of a displacement u that is already on the device (FP64, 3N values,
 * component-major, on the context's device, ordered on its stream), with no
 * allocation in the call.  The kernel's partial sums go to a fixed scratch
 * array of 196,672 bytes that each GPU holds for the life of the process
 * (partials of at most 4096 blocks, enough for every grid, so no grid size is
 * rejected).  All calls on one GPU share that array: calls that overlap on one
 * GPU (several threads, contexts or streams) race and must be serialised by the
 * caller.  Argument and state errors as ceff_average_stress; the result equals
 * ceff_average_stress's on the same u. */
ceff_status ceff_average_stress_noalloc(ceff_ctx* ctx, int J, const double* u, double out6[6]);

/* Counters of the most recent solve (ceff_apt_steps: the launch shape only). */
ceff_status ceff_get_stats(const ceff_ctx* ctx, ceff_stats* out);

/* ---- property contribution tensors (host arithmetic, no context) ------------ */

/* Contribution tensors of inclusions of total volume fraction phi in a host of
 * stiffness C_host, from the effective stiffness C_eff of an image that holds
 * them (paper: "Model 2: validation against an Eshelby solution", the relation
 * S* = S1 + phi H, and the appendix on the property contribution tensor):
 *   H = (C_eff^-1 - C_host^-1) / phi   (compliance contribution: S* = S_host + phi H)
 *   N = (C_eff - C_host) / phi         (stiffness contribution:  C* = C_host + phi N)
 * All matrices are 6x6 row-major Voigt with engineering shear, so H is in the
 * compliance convention of C^-1 (H_44 = 4 H_2323, H_14 = 2 H_1123).  With one
 * inclusion in a periodic box, H tends to the single-inclusion tensor as phi -> 0.
 * H_out or N_out may be NULL.  Returns CEFF_EINVAL if phi is not in (0, 1] or a
 * stiffness matrix is singular (pivot below 1e-12 of its largest entry).
 * Computed on the host in FP64 (Gauss-Jordan with partial pivoting); needs no
 * device. */
ceff_status ceff_contribution_tensors(const double C_eff[36], const double C_host[36], double phi, double H_out[36],
                                      double N_out[36]);

/* The paper's direct test for the off-diagonal constants (appendix on boundary
 * conditions, eqs. D1-D5): from a triaxial wall test (all three pairs of walls
 * moved at once) with volume-averaged normal stresses sig_mean = (<s11>, <s22>,
 * <s33>) and normal strains eps_mean = (<e11>, <e22>, <e33>), and the diagonal
 * constants C_diag = (C11, C22, C33) of the three normal tests, form
 *   sbar_ii = sig_mean_i - C_ii eps_mean_i,   ebar_ii = eps_mean_i
 * and solve  ebar22 C12 + ebar33 C13 = sbar11,  ebar11 C12 + ebar33 C23 = sbar22,
 *            ebar11 C13 + ebar22 C23 = sbar33
 * for out = (C12, C13, C23).  Under CEFF_BC_WALLS the solve is linear and the
 * walls impose the normal strains exactly, so the triaxial test with unit
 * strains is the sum of the columns of loads 0-2 (sig_mean = their summed
 * upper three rows, eps_mean = (1, 1, 1)).  Host FP64; needs no device.
 * CEFF_EINVAL if an input is not finite or a strain is zero. */
ceff_status ceff_triaxial_offdiagonals(const double sig_mean[3], const double eps_mean[3], const double C_diag[3],
                                       double out[3]);

/* The same from the columns of the three normal wall tests: C_walls is a 6x6
 * row-major matrix (as ceff_solve writes under CEFF_BC_WALLS) whose columns 0-2
 * hold loads 0-2.  The triaxial test with unit strains is their sum (linear
 * solve, strains imposed by the walls), so sig_mean_i = sum_J C_walls[i][J]
 * over J = 0..2, eps_mean = (1, 1, 1) and C_diag = (C_walls[0][0],
 * C_walls[1][1], C_walls[2][2]); out = (C12, C13, C23) as above.  Host FP64;
 * needs no device.  CEFF_EINVAL if an input entry used is not finite. */
ceff_status ceff_triaxial_from_walls(const double C_walls[36], double out[3]);

#ifdef __cplusplus
}
#endif

#endif /* CEFF_H */
