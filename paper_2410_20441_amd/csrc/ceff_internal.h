// Internal declarations shared by the HIP kernels and the host driver.
// Not part of the public C ABI (that is include/ceff.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ceff {

constexpr int kMaxLoads = 6;

// One voxel sample as the kernels see it (device-resident table, one entry per
// sample).  Vector fields are component-major: f[c*N + i + nx*(j + ny*k)].
template <typename T>
struct SampleDesc {
  int64_t nx, ny, nz, N;
  T rhx, rhy, rhz;            // 1/h per axis
  T mom;                      // heavy-ball momentum a = 1/(1+c)
  T sfac;                     // step numerator: u += (sfac / H_face) * r
  T sfac_first;               // step numerator of the very first iteration (no momentum yet)
  const T* K;                 // bulk modulus per cell (N)
  const T* G;                 // shear modulus per cell (N)
  // rotating displacement buffers per load (3N each): single iterations use the pair
  // (parity, parity ^ 1); the two-iteration kernel writes the other pair (u[2], u[3] or
  // u[0], u[1]), which is allocated only for it
  T* u[4][kMaxLoads];
  const T* force[kMaxLoads];  // optional constant body force per load (3N) or nullptr
  // Optional phase image: when phase != nullptr and the launch shape asks for it
  // (TileShape::pal), the iteration kernel reads the 1-byte phase id of each cell
  // and takes its moduli from ptab (K of phase p at ptab[p], G at ptab[nphase + p])
  // instead of reading K and G.  All samples of such a launch share one table.
  const uint8_t* phase;
  const T* ptab;
  int nphase;
  // Orthotropic cells: 9N constants C11 C22 C33 C23 C13 C12 C44 C55 C66
  // (component-major) or nullptr; when set, K, G and the phase image are unused
  // and the orthotropic kernels run (TileShape::ortho).
  const T* cst;
  // General anisotropic cells: 21N constants (upper triangle of the 6x6 Voigt
  // matrix, row by row, component-major) or nullptr; tse: the harmonic edge
  // means of C44 / C55 / C66 (3N), tihf: 1/H of every face (3N), tscr: 24N of
  // scratch (strains, stresses, the cells' shares of edge stresses).  One
  // sample, load slot 0 (TileShape::tri).
  const T* c21;
  const T* tse;
  const T* tihf;
  T* tscr;
  // 1: rigid walls instead of periodic boundaries: the d-faces of the grid
  // plane of index 0 in d are held, and edges lying in such a plane carry no
  // shear stress (one load per block; TileShape::walls).  wshear[l] = 3, 4, 5
  // makes load slot l the simple-shear test of that Voigt shear component: its
  // own component's boundary edges are computed as inside on the walls normal
  // to the sheared direction and split into two half edges on the loaded walls.
  int walls;
  int wshear[kMaxLoads];
  T E[kMaxLoads][6];          // macroscopic tensor strain per load: xx yy zz yz xz xy
  unsigned active;            // bit l: load l is iterated
  int work_begin, work_end;   // this sample's work items [begin, end)
  int tiles_x, tiles_y, chunks_z, kc;  // tiling of this sample
};

// One block's worth of work: a (tile_x, tile_y, z-chunk) of one sample and the
// load slots [slot0, slot0 + L) of it.  sample < 0 marks padding.
struct WorkItem {
  int sample;
  int tx, ty, kz;
  int slot0;
};

struct TileShape {
  int bx = 0, by = 0;  // block extent including the one-cell ghost ring (threads = bx*by)
  int kc = 0;      // z-planes per chunk (0 = choose automatically)
  int group = 0;   // loads per block: 1, 2, 3 or 6 (0 = all requested loads in one block)
  int pf = 0;      // 0: plain z-march; 1: prefetch the next plane into registers; 2: z-march unrolled by two;
                   // 3: unrolled, all loads of the group between one pair of barriers per plane;
                   // 4: as 3, unrolled by three with the next plane's data requested one plane ahead;
                   // 5: one load per block, no LDS: neighbours read through the caches;
                   // 9: one load per block, rows of 16, 32 or 64 cells, x-neighbours across lanes
  int order = 0;   // 0: load groups of a tile 8 items apart; 1: each XCD takes a contiguous band
  int occ = 0;     // 1: build that targets more waves per SIMD (fewer registers)
  int pal = 0;     // 1: moduli from the samples' phase image and table (variants 3 and 9)
  int ortho = 0;   // 1: orthotropic cells (one load per block, its own kernel)
  int walls = 0;   // 1: wall boundaries (variant 3, one load per block)
  int tri = 0;     // 1: general anisotropic cells (their own launches, one load)
  int force = 2;   // variant 9, body forces of the launch's active loads: 0 none, 1 all of them,
                   // 2 some (each block checks its own)
  int tb = 0;      // 1: two iterations per launch (one load per block, 2-cell ghost ring; iterations
                   // after the first of a solve come in pairs)
};

// ---- launch wrappers (ceff_kernels.hip) ----------------------------------------

// One heavy-ball iteration for every active (sample, load).  parity selects which
// of the two buffers holds u^n (read) and which holds u^{n-1} (read, then
// overwritten by u^{n+1}).  first != 0 runs the start-up step (no momentum).
// If partials != nullptr the squared residual of u^n is accumulated per work item
// and load into partials[w*kMaxLoads + l] (FP64).
template <typename T, int L>
hipError_t launch_step(const SampleDesc<T>* d_samples, const WorkItem* d_work, int nwork, TileShape ts,
                       int parity, int first, double* partials, hipStream_t s);

// Two heavy-ball iterations from (u^parity, u^{parity^1}) into the other buffer pair:
// u^{n+1} to u[(parity ^ 2) & 2], u^{n+2} to u[((parity ^ 2) & 2) | 1] (one load per
// block, work items tiled with a 2-cell ghost ring).  partials as for launch_step
// (the residual of u^{n+1}).
template <typename T>
hipError_t launch_step_pair(const SampleDesc<T>* d_samples, const WorkItem* d_work, int nwork, TileShape ts,
                            int parity, double* partials, hipStream_t s);
// Dynamic LDS of the two-iteration kernel for shape ts and element size elem.
size_t pair_lds_bytes(TileShape ts, size_t elem);

// Residual only: r = div(C:(E + grad u^parity)) + force, written as float or T to
// rout[l] (3N per load, may be nullptr), norms as above.  No update.
template <typename T, typename R, int L>
hipError_t launch_residual(const SampleDesc<T>* d_samples, const WorkItem* d_work, int nwork, TileShape ts,
                           int parity, R* const* rout, double* partials, hipStream_t s);

// The same two for orthotropic cells (SampleDesc::cst).
template <typename T>
hipError_t launch_step_ortho(const SampleDesc<T>* d_samples, const WorkItem* d_work, int nwork, TileShape ts,
                             int parity, int first, double* partials, hipStream_t s);
template <typename T, typename R>
hipError_t launch_residual_ortho(const SampleDesc<T>* d_samples, const WorkItem* d_work, int nwork, TileShape ts,
                                 int parity, R* const* rout, double* partials, hipStream_t s);
// General anisotropic cells (SampleDesc::c21, sample 0, load slot 0): one
// heavy-ball iteration as four launches (strains, cell stresses and edge
// shares, edge gather, update), or the residual (rout[0], 3N).  The update
// launch has nwork blocks and writes norm partials like the other kernels.
template <typename T>
hipError_t launch_step_tri(const SampleDesc<T>* d_samples, int64_t N, int nwork, int parity, int first,
                           double* partials, hipStream_t s);
template <typename T, typename R>
hipError_t launch_residual_tri(const SampleDesc<T>* d_samples, int64_t N, int nwork, int parity, R* const* rout,
                               double* partials, hipStream_t s);
// FP64 stress averages of general cells for the displacement u[0][0] of the
// one-entry table d (its tscr holds 24N doubles): block partials, then the 6 sums.
hipError_t launch_average_stress_tri(const SampleDesc<double>* d, const double* tscr, int64_t N, double* partials,
                                     int nblocks_cap, double* out6, hipStream_t s);
// Edge means and face step factors of general cells from FP64 constants.
template <typename T>
hipError_t launch_tri_setup(const double* c21, int64_t nx, int64_t ny, int64_t nz, T* se, T* ihf, hipStream_t s);
// Per-block flags (1 = some cell's 21 constants not finite or not positive definite).
hipError_t launch_check_tri(const double* c21, int64_t n, int* bad, int* nblocks, hipStream_t s);
// Dynamic LDS of the orthotropic kernels for shape ts and element size elem.
size_t ortho_lds_bytes(TileShape ts, size_t elem);

// Sum partials of each (sample, load) in fixed order: out[s*kMaxLoads + l].
hipError_t launch_finalize_norms(const int* d_ranges /* 2 per sample */, int nsamples, const double* partials,
                                 double* out, hipStream_t s);

// FP64 volume averages of the six stresses of u (3N) under strain E: writes
// block partials (6 per block) then the final 6 sums (not yet divided by N).
// walls: 0 periodic, 1 the normal-test walls, 3..5 the simple-shear test of
// that Voigt shear component (see SampleDesc::wshear).
hipError_t launch_average_stress(int64_t nx, int64_t ny, int64_t nz, const double h[3], const double* K,
                                 const double* G, const double E[6], const double* u, double* partials,
                                 int nblocks_cap, double* out6, int walls, hipStream_t s);

// The same for orthotropic cells (cst: 9N FP64 constants).
hipError_t launch_average_stress_ortho(int64_t nx, int64_t ny, int64_t nz, const double h[3], const double* cst,
                                       const double E[6], const double* u, double* partials, int nblocks_cap,
                                       double* out6, hipStream_t s);

// Gradient of sum W_IJ C_IJ with respect to per-voxel K and G from six FP64
// displacement fields.  The field pointers (nullptr for loads W does not
// touch) and W travel as a kernel argument, so a call allocates nothing.
struct GradLoads {
  const double* u[6];
  double W[36];
};
template <typename R>
hipError_t launch_gradient(int64_t nx, int64_t ny, int64_t nz, const double h[3], const double* K, const double* G,
                           const GradLoads& g, R* dK, R* dG, hipStream_t s);

// Elementwise helpers.
template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s);
template <typename A, typename B>
hipError_t launch_convert(const A* src, B* dst, int64_t n, hipStream_t s);
// base += (double)prev; cur -= prev; prev = 0   (fold an FP32 iterate into the FP64 base)
hipError_t launch_fold(double* base, float* cur, float* prev, int64_t n, hipStream_t s);
// dst += src (FP64)
hipError_t launch_axpy1(double* dst, const double* src, int64_t n, hipStream_t s);
// K, G from a phase image and per-phase tables
template <typename T>
hipError_t launch_phase_to_fields(const uint8_t* phase, int64_t n, const double* Ktab, const double* Gtab, int nphase,
                                  T* K, T* G, hipStream_t s);
// Per-block flags (1 = some K or G not finite and > 0) into bad[0 .. *nblocks)
// (bad must hold 65536 ints).
template <typename T>
hipError_t launch_check_moduli(const T* K, const T* G, int64_t n, int* bad, int* nblocks, hipStream_t s);
// Per-block flags (1 = some cell's orthotropic constants are not finite, a
// diagonal one is not > 0, or its normal block is not positive definite).
hipError_t launch_check_ortho(const double* c, int64_t n, int* bad, int* nblocks, hipStream_t s);

}  // namespace ceff
