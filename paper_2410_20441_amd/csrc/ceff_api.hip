// Host driver and C ABI (include/ceff.h) of the voxel-grid effective
// stiffness solver.  All arithmetic of the method runs in the kernels of
// ceff_kernels.hip; this file sets numerical parameters, owns device memory,
// schedules launches (optionally replayed as HIP graphs), decides convergence
// and assembles C*.
//
// Numerical parameters (paper, "Solution of the system of equations": CFL
// condition, Strouhal number, the numerical combinations dt~/rho~, H~dt~,
// G~dt~, K~dt~ and their optimal values), read with unit physical time step
// and pseudo moduli equal to the local moduli:
//   ell = courant / sqrt(1/hx^2 + 1/hy^2 + 1/hz^2)     (Vp~ dt~)
//   c   = ell * St / Lx                               (dt~ / dt, so K~dt~ = c K)
//   beta= ell * Lx / St                               (dt~/rho~ = beta / H~ at a face)
//   Lx  = max_d n_d h_d
// The displacement recurrence the kernels run then has momentum a = 1/(1+c)
// and step factor s = c/(1+c) * beta (first step: beta, no momentum).
#include "ceff.h"
#include "ceff_internal.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace ceff;

// Block partials of the stress averages: the kernel strides over the cells
// with at most this many blocks, whatever the grid.
constexpr int kAvgBlocks = 4096;

// Scratch of the allocation-free entry point (ceff_average_stress_noalloc):
// the stress-average kernel's block partials (6 x kAvgBlocks) and the six sums
// at the end, 196,672 bytes.  Each GPU the library runs on holds its own copy
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not a device address: kernels get the per-device address that ceff_create
// looks up with hipGetSymbolAddress (scratch_addr below).
constexpr int kScratchDoubles = 6 * kAvgBlocks + 8;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

struct DevBuf {
  void* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p) { o.p = nullptr; }
  ~DevBuf() { reset(); }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
  }
  hipError_t alloc(size_t bytes) {
    reset();
    return hipMalloc(&p, bytes ? bytes : 16);
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

struct PinnedBuf {
  void* p = nullptr;
  size_t n = 0;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  hipError_t ensure(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e == hipSuccess) n = bytes;
    return e;
  }
};

}  // namespace

struct ceff_ctx {
  int device = 0;
  hipStream_t user = nullptr;
  hipStream_t s = nullptr;
  int64_t nx = 0, ny = 0, nz = 0;
  double h[3] = {1, 1, 1};
  bool grid_set = false, have_material = false;
  DevBuf K64, G64, K32, G32;
  bool have32 = false;
  // material given as a phase image: the image and the per-phase table (K then
  // G), in FP64 and FP32; nphase = 0 when the material came as fields
  DevBuf phase8, ptab64, ptab32;
  int nphase = 0;
  // material given as orthotropic cells: 9N constants (FP64, FP32 copy for the mixed path)
  DevBuf c64, c32;
  bool ortho = false;
  // material given as general anisotropic cells: 21N constants (FP64, FP32 copy), the
  // harmonic edge means of the diagonal shear constants and the face step factors
  DevBuf t64, t32, tse64, tse32, tihf64, tihf32;
  bool tri = false;
  int boundary = CEFF_BC_PERIODIC;
  DevBuf keep[6];
  bool kept[6] = {false, false, false, false, false, false};
  std::string err;
  ceff_stats stats{};
  std::map<std::string, TileShape> tuned;  // autotuned launch shapes of this context, by tune_key
  PinnedBuf pinned;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

ceff_status fail(ceff_ctx* c, ceff_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

#define HIPCK(ctx, ...)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (__VA_ARGS__);                                                               \
    if (e_ != hipSuccess)                                                                        \
      return fail((ctx), e_ == hipErrorOutOfMemory ? CEFF_ENOMEM : CEFF_EDEVICE, "%s failed: %s", \
                  #__VA_ARGS__, hipGetErrorString(e_));                                          \
  } while (0)

#define STCK(...)                   \
  do {                              \
    ceff_status st_ = (__VA_ARGS__); \
    if (st_ != CEFF_OK) return st_; \
  } while (0)

ceff_status validate_opts(ceff_ctx* c, const ceff_solve_opts& o) {
  if (o.precision != CEFF_PREC_FP64 && o.precision != CEFF_PREC_MIXED)
    return fail(c, CEFF_EINVAL, "precision must be CEFF_PREC_FP64 or CEFF_PREC_MIXED");
  if (!(o.rtol > 0.0) || !std::isfinite(o.rtol)) return fail(c, CEFF_EINVAL, "rtol must be finite and > 0");
  if (o.max_iter < 1) return fail(c, CEFF_EINVAL, "max_iter must be >= 1");
  if (o.check_every < 1 || o.check_every > 1000000) return fail(c, CEFF_EINVAL, "check_every out of range");
  if (!(o.courant > 0.0) || !(o.courant <= 1.0)) return fail(c, CEFF_EINVAL, "courant must be in (0, 1]");
  if (!(o.strouhal >= 0.0) || !std::isfinite(o.strouhal))
    return fail(c, CEFF_EINVAL, "strouhal must be > 0, or 0 for the automatic choice");
  if (!(o.fold_ratio > 0.0) || !(o.fold_ratio < 1.0)) return fail(c, CEFF_EINVAL, "fold_ratio must be in (0, 1)");
  return CEFF_OK;
}

// The grid limits of every entry point.  The iteration kernels address a field
// through a view of one z-plane of one component and a thread's 32-bit byte
// offset within it, so the only size limit is that of a plane (below 2 GiB of
// FP64); the total size of a field is limited by device memory alone.
ceff_status validate_grid(ceff_ctx* c, int64_t nx, int64_t ny, int64_t nz, const double* h) {
  if (nx < 2 || ny < 2 || nz < 2) return fail(c, CEFF_EINVAL, "grid dimensions must be >= 2");
  if (nx > (1 << 20) || ny > (1 << 20) || nz > (1 << 20)) return fail(c, CEFF_EINVAL, "grid dimension too large");
  if (nx * ny * (int64_t)sizeof(double) > ((int64_t)1 << 31)) return fail(c, CEFF_EINVAL, "z-plane too large");
  for (int d = 0; d < 3; ++d)
    if (!(h[d] > 0.0) || !std::isfinite(h[d])) return fail(c, CEFF_EINVAL, "spacings must be finite and > 0");
  return CEFF_OK;
}

void unit_strain(int J, double E[6]) {
  for (int q = 0; q < 6; ++q) E[q] = 0.0;
  E[J] = J < 3 ? 1.0 : 0.5;
}

struct Params {
  double mom, sfac, sfac_first;
};

// Automatic Strouhal number (strouhal = 0).  St only sets the damping c =
// ell St / Lx of the iteration (momentum 1/(1+c)), never its fixed point.  Below
// the best damping the iteration count grows as 1/c (the heavy-ball decay rate
// of the underdamped regime), above it faster.  Sweeps on pore, crack and
// three-phase images from 64^3 to 256^3 put the best c near a constant of the
// microstructure family (about 0.010 for fluid-filled pores, 0.008 for penny
// cracks, 0.015 for the three-phase field), and a 703^3 pore image at St 8
// (a box-scale mode then limits it).  Hence c = 0.010, with St kept within
// [2, 8.3]: small boxes keep the previous default St 2.
constexpr double kAutoDamping = 0.010, kAutoStMin = 2.0, kAutoStMax = 8.3;

double auto_strouhal(double Lx, double ell) {
  return std::min(std::max(kAutoDamping * Lx / ell, kAutoStMin), kAutoStMax);
}

Params make_params(int64_t nx, int64_t ny, int64_t nz, const double h[3], double courant, double strouhal) {
  const double Lx = std::max({nx * h[0], ny * h[1], nz * h[2]});
  const double ell = courant / std::sqrt(1.0 / (h[0] * h[0]) + 1.0 / (h[1] * h[1]) + 1.0 / (h[2] * h[2]));
  if (strouhal == 0.0) strouhal = auto_strouhal(Lx, ell);
  const double c = ell * strouhal / Lx;
  const double beta = ell * Lx / strouhal;
  return Params{1.0 / (1.0 + c), c / (1.0 + c) * beta, beta};
}

// Copy caller moduli (F32/F64, host/device) into device FP64 arrays.
ceff_status load_moduli(ceff_ctx* c, const void* src, int dtype, int where, int64_t N, DevBuf& dst) {
  HIPCK(c, dst.alloc(sizeof(double) * N));
  if (dtype == CEFF_F64) {
    HIPCK(c, hipMemcpyAsync(dst.p, src, sizeof(double) * N,
                            where == CEFF_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, c->s));
  } else {
    DevBuf tmp;
    const float* dsrc = static_cast<const float*>(src);
    if (where == CEFF_HOST) {
      HIPCK(c, tmp.alloc(sizeof(float) * N));
      HIPCK(c, hipMemcpyAsync(tmp.p, src, sizeof(float) * N, hipMemcpyHostToDevice, c->s));
      dsrc = tmp.as<float>();
    }
    HIPCK(c, launch_convert<float, double>(dsrc, dst.as<double>(), N, c->s));
    HIPCK(c, hipStreamSynchronize(c->s));
  }
  return CEFF_OK;
}

ceff_status check_positive(ceff_ctx* c, const double* K, const double* G, int64_t N) {
  DevBuf bad;
  int nb = 0;
  HIPCK(c, bad.alloc(sizeof(int) * 65536));
  HIPCK(c, launch_check_moduli<double>(K, G, N, bad.as<int>(), &nb, c->s));
  std::vector<int> h(nb);
  HIPCK(c, hipMemcpyAsync(h.data(), bad.p, sizeof(int) * nb, hipMemcpyDeviceToHost, c->s));
  HIPCK(c, hipStreamSynchronize(c->s));
  for (int v : h)
    if (v) return fail(c, CEFF_EINVAL, "moduli must be finite and > 0");
  return CEFF_OK;
}

void clear_ortho(ceff_ctx* c) {
  c->c64.reset();
  c->c32.reset();
  c->ortho = false;
  c->t64.reset(); c->t32.reset(); c->tse64.reset(); c->tse32.reset(); c->tihf64.reset(); c->tihf32.reset();
  c->tri = false;
}

void clear_phases(ceff_ctx* c) {
  c->phase8.reset();
  c->ptab64.reset();
  c->ptab32.reset();
  c->nphase = 0;
}

void clear_kept(ceff_ctx* c) {
  for (int J = 0; J < 6; ++J) {
    c->keep[J].reset();
    c->kept[J] = false;
  }
}

// ---- the solve engine ------------------------------------------------------------

struct SampleIn {
  int64_t nx, ny, nz;
  double h[3];
  const double* K64;
  const double* G64;
  const float* K32;
  const float* G32;
  const uint8_t* phase = nullptr;  // phase image (or nullptr) and its table, K then G
  const double* ptab64 = nullptr;
  const float* ptab32 = nullptr;
  int nphase = 0;
  const double* c64 = nullptr;  // orthotropic cells (9N) or nullptr
  const float* c32 = nullptr;
  const double* t64 = nullptr;  // general cells (21N), their edge means and face factors, or nullptr
  const float* t32 = nullptr;
  const double* tse64 = nullptr;
  const float* tse32 = nullptr;
  const double* tihf64 = nullptr;
  const float* tihf32 = nullptr;
  int walls = 0;                 // 1: rigid, free-slip walls
};

struct Prob {
  int s = 0, J = 0, slot = 0;
  double r0 = 0.0, relres = INFINITY, relres_base = 1.0;
  int64_t iters = 0;
  bool active = false;
  ceff_status st = CEFF_OK;
  int phase = 0;      // mixed precision: 0 = macroscopic strain, 1 = body force from the FP64 residual
  int sol = 0;        // FP64: displacement buffer holding the solution; mixed: unused (base)
  std::vector<double> recent;
};

// MI355X's Infinity Cache (the memory-side last-level cache in front of HBM).
constexpr double kInfinityCacheBytes = 256.0 * 1024 * 1024;

TileShape default_tile(int64_t nx, int64_t ny, bool fp64, bool single, bool batch, bool plain = true) {
  TileShape t{};
  // CEFF_TILE="bx,by[,kc[,group[,variant[,order[,occ]]]]]" overrides the launch shape (the iterates
  // do not depend on it; tests check that)
  if (const char* env = std::getenv("CEFF_TILE")) {
    int bx = 0, by = 0, kc = 0, grp = 6, pf = 1, ord = 1, occ = 0;
    const int n = std::sscanf(env, "%d,%d,%d,%d,%d,%d,%d", &bx, &by, &kc, &grp, &pf, &ord, &occ);
    if (n >= 2 && bx >= 3 && by >= 3 && ((bx * by + 63) / 64) * 64 <= 512 &&
        (grp == 1 || grp == 2 || grp == 3 || grp == 6))
      return TileShape{bx, by, n >= 3 ? kc : 0, pf == 5 || pf == 9 ? 1 : grp,
                       (pf >= 0 && pf <= 5) || pf == 9 ? pf : 0, ord ? 1 : 0, occ ? 1 : 0, 0};
  }
  // FP32, one load per launch: variant 9 (x-neighbours across lanes), 32 x 8 ghosted block
  // (30 x 6 interior, rows within a wave) with 12-plane chunks, high-occupancy build: 0.051-0.054 ms
  // per launch at 191^3 on every MI355X measured, against 0.0569 for variant 3's best (18 x 14, 12
  // planes).  24-plane chunks (seven blocks per CU in one round) took 0.050-0.051 ms on some GPUs
  // and 0.056-0.057 on others.  A batch of images takes the same blocks with one load each: the
  // 48-sample three-phase batch in 9.7 s against 10.7 s with variant 3 and two loads per block.
  // FP64, one load per launch on one image of periodic isotropic cells (plain): the same blocks at
  // the default occupancy, 0.1227 ms per launch at 191^3 against 0.1326 for variant 3 at 34 x 14 and
  // 0.1536 with the high-occupancy build.
  if (fp64 ? single && !batch && plain : single || batch) {
    t.bx = nx + 2 <= 16 ? 16 : 32;
    t.by = (int)std::min<int64_t>(ny + 2, 8);
    t.kc = 12;
    t.group = 1;
    t.pf = 9;
    t.order = 1;
    t.occ = fp64 ? 0 : 1;
    return t;
  }
  // Fastest shapes of the 191^3 sweeps for the other cases, all with 12-plane chunks and the loads
  // of a block staged between one barrier pair per plane.  FP32, several loads per launch: 66 x 7
  // ghosted block (64 x 5 interior), two loads per block.  FP64: 34 x 14 (32 x 12 interior), one load
  // per block.
  t.bx = (int)std::min<int64_t>(nx + 2, fp64 ? 34 : (single ? 18 : 66));
  t.by = (int)std::min<int64_t>(ny + 2, fp64 || single ? 14 : 7);
  t.kc = 12;
  t.group = fp64 ? 1 : 2;
  t.pf = 3;
  t.order = 1;
  t.occ = !fp64 && single ? 1 : 0;
  return t;
}

ceff_status stress_average(ceff_ctx* c, const SampleIn& s, int J, const double* u, double out6[6]);

#ifndef CEFF_KERNEL_HASH
#define CEFF_KERNEL_HASH "unknown"
#endif

// Autotuned launch shapes: kept per context, and in the file named by the
// environment variable CEFF_TUNE_CACHE when it is set (one line per entry:
// key bx by kc group variant order occ), so they survive the process.
bool lookup_tuned(ceff_ctx* c, const std::string& key, TileShape& out) {
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    out = it->second;
    return true;
  }
  const char* path = std::getenv("CEFF_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512], k[400];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    TileShape t{};
    if (std::sscanf(line, "%399s %d %d %d %d %d %d %d", k, &t.bx, &t.by, &t.kc, &t.group, &t.pf, &t.order, &t.occ) !=
        8)
      continue;
    const int nt = ((t.bx * t.by + 63) / 64) * 64;
    const bool valid = t.bx >= 3 && t.by >= 3 && nt <= 512 && t.kc >= 0 && ((t.pf >= 0 && t.pf <= 5) || t.pf == 9) &&
                       (t.group == 1 || t.group == 2 || t.group == 3 || t.group == 6) && (t.order == 0 || t.order == 1) &&
                       (t.occ == 0 || t.occ == 1);
    if (valid && key == k) {  // the last valid entry of a key wins
      out = t;
      found = true;
    }
  }
  std::fclose(f);
  if (found) c->tuned[key] = out;
  return found;
}

void remember_tuned(ceff_ctx* c, const std::string& key, const TileShape& t) {
  c->tuned[key] = t;
  const char* path = std::getenv("CEFF_TUNE_CACHE");
  if (!path || !*path) return;
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%s %d %d %d %d %d %d %d\n", key.c_str(), t.bx, t.by, t.kc, t.group, t.pf, t.order, t.occ);
    std::fclose(f);
  }
}

template <typename T>
struct Engine {
  ceff_ctx* c;
  std::vector<SampleIn> in;
  ceff_solve_opts o;
  bool mixed;
  int Lk;                       // 1: one load (slot 0); otherwise slot J holds load J
  std::vector<int> Js;          // requested loads
  bool beyond_cache = false;    // a launch's working set exceeds the Infinity Cache
  TileShape ts{};
  // device
  std::vector<std::array<DevBuf, 4 * kMaxLoads>> ubuf;  // per sample: u[b][slot] at index b*6+slot
  std::vector<std::array<DevBuf, kMaxLoads>> base, force;
  DevBuf d_in, d_out, d_work, d_work_o, d_partials, d_norms, d_ranges, d_ranges_o, d_rout;
  DevBuf tscr_in, tscr_out;  // general cells: pipeline scratch of the sweeps and of the FP64 residual
  // two iterations per launch (ts.tb): the single iterations (the first of a solve, odd
  // remainders) run on a work list tiled with the usual one-cell ghost ring
  TileShape ts1{};
  DevBuf d_work_s;
  std::vector<WorkItem> work_s;
  std::vector<int> ranges_s;
  std::vector<SampleDesc<T>> h_in;
  std::vector<SampleDesc<double>> h_out;
  std::vector<WorkItem> work, work_o;  // iteration launches / FP64 residual launches
  std::vector<int> ranges, ranges_o;
  std::vector<Prob> probs;
  int parity = 0;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_m = 0, graph_parity = -1, graph_force = -1;
  // accounting
  double step_ms = 0.0, step_bytes = 0.0, vu = 0.0;
  int64_t launches = 0, outer = 0;
  std::vector<double>* hist = nullptr;

  ~Engine() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
  }

  bool single() const { return Js.size() == 1; }
  // periodic boundaries and isotropic cells
  bool plain_cells() const { return in[0].c64 == nullptr && in[0].t64 == nullptr && !in[0].walls; }
  int slot_of(int J) const { return single() ? 0 : J; }
  int group() const {
    return single() || ts.pf == 5 || ts.pf == 9 || ts.ortho || ts.walls || ts.tri ? 1
                                                                                   : (ts.group > 0 ? ts.group : kMaxLoads);
  }

  // Read the moduli from the phase image when there is one (one sample) and the
  // kernel variant supports it; CEFF_MODULI=fields keeps the K and G fields.
  // Orthotropic cells always take their own kernel (one load per block).
  TileShape with_moduli(TileShape t) const {
    const char* env = std::getenv("CEFF_MODULI");
    const bool fields = env != nullptr && std::strcmp(env, "fields") == 0;
    t.ortho = in[0].c64 != nullptr ? 1 : 0;
    t.tri = in[0].t64 != nullptr ? 1 : 0;
    t.walls = in[0].walls;
    if (t.walls) t.pf = 3;  // the wall-boundary kernels are variant 3, one load per block
    // variant 9 (x-neighbours across lanes) needs rows that tile a wave
    if (t.pf == 9 && t.bx != 16 && t.bx != 32 && t.bx != 64) t.pf = 3;
    // the phase table is staged once per block from the first sample, so every
    // sample of the launch must use that same table
    bool shared = true;
    for (const SampleIn& s : in) shared = shared && s.phase != nullptr && s.ptab64 == in[0].ptab64;
    t.pal = !t.ortho && !t.tri && shared && (t.pf == 3 || t.pf == 9) && !fields ? 1 : 0;
    return t;
  }

  // Work list of one launch.  Each (tile, z-chunk) of a sample is split into
  // load groups of `group` slots; the groups of one tile are placed 8 items apart
  // so that the round-robin dispatch of blocks over the 8 XCDs puts them on the
  // same XCD (they then share that XCD's L2 for the moduli).  Every sample's
  // items stay contiguous (padded with sample = -1) so norms reduce per sample.
  ceff_status build_work(TileShape t, int group, std::vector<WorkItem>& w, std::vector<int>& rg,
                         std::vector<int>& kcs) {
    w.clear();
    rg.clear();
    kcs.clear();
    std::vector<int> slots0;  // first slot of each group that holds a requested load
    if (single()) {
      slots0.push_back(0);
    } else {
      for (int g0 = 0; g0 < kMaxLoads; g0 += group) {
        bool any = false;
        for (int J : Js)
          if (J >= g0 && J < g0 + group) any = true;
        if (any) slots0.push_back(g0);
      }
    }
    const int G = (int)slots0.size();
    int64_t total_xy = 0;
    const int gh = t.tb ? 2 : 1;  // ghost ring of the tiles
    for (auto& s : in)
      total_xy += ((s.nx + t.bx - 2 * gh - 1) / (t.bx - 2 * gh)) * ((s.ny + t.by - 2 * gh - 1) / (t.by - 2 * gh));
    for (size_t si = 0; si < in.size(); ++si) {
      const auto& s = in[si];
      const int tx = (int)((s.nx + t.bx - 2 * gh - 1) / (t.bx - 2 * gh));
      const int ty = (int)((s.ny + t.by - 2 * gh - 1) / (t.by - 2 * gh));
      int kc;
      if (t.kc > 0) {
        kc = t.kc;
      } else {
        int64_t chunks = (2048 + total_xy * G - 1) / (total_xy * G);
        if (chunks > s.nz / 4) chunks = s.nz / 4;
        if (chunks < 1) chunks = 1;
        kc = (int)((s.nz + chunks - 1) / chunks);
      }
      if (kc > s.nz) kc = (int)s.nz;
      if (kc < 1) kc = 1;
      const int cz = (int)((s.nz + kc - 1) / kc);
      const int64_t ntile = (int64_t)tx * ty * cz;
      const size_t base = w.size();
      rg.push_back((int)base);
      if (t.order == 1) {
        // (kz, ty, tx, group) in lexicographic order, cut into 8 contiguous bands of
        // equal work; band x goes to positions x, x+8, x+16, ... (XCD x under
        // round-robin dispatch), so blocks running together on one XCD are spatial
        // neighbours and share halo rows and moduli through that XCD's L2.  An
        // item's work is the planes it marches, its chunk's lead plane included:
        // when the last chunk is short, bands of equal item counts leave the XCD
        // with the short chunks idle early (480^3 in 28-plane chunks: 0.952 ms per
        // launch against 0.906 in 32-plane ones).  Shorter bands are padded with
        // empty items.
        const int64_t n = ntile * G;
        const int64_t slice = (int64_t)tx * ty * G;  // items of one z-chunk
        auto work_of = [&](int64_t kz) { return std::min<int64_t>(kc, s.nz - kz * kc) + 1; };
        int64_t total = 0;
        for (int64_t kz = 0; kz < cz; ++kz) total += work_of(kz) * slice;
        std::vector<uint8_t> band((size_t)n);
        int64_t count[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int64_t acc = 0;
        for (int64_t q = 0; q < n; ++q) {
          const int64_t wq = work_of(q / slice);
          const int64_t bq = std::min<int64_t>(7, (8 * (2 * acc + wq)) / (2 * total));  // band of its midpoint
          band[(size_t)q] = (uint8_t)bq;
          ++count[bq];
          acc += wq;
        }
        const int64_t per = *std::max_element(count, count + 8);
        w.resize(base + (size_t)(per * 8), WorkItem{-1, 0, 0, 0, 0});
        int64_t next[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t q = 0; q < n; ++q) {
          const int64_t tt = q / G;
          const int g = (int)(q % G);
          const int a = (int)(tt % tx), b = (int)((tt / tx) % ty), kz = (int)(tt / ((int64_t)tx * ty));
          const int bq = band[(size_t)q];
          const int64_t pos = 8 * next[bq]++ + bq;
          w[base + (size_t)pos] = WorkItem{(int)si, a, b, kz, slots0[g]};
        }
      } else {
        const int64_t nbatch = (ntile + 7) / 8;
        w.resize(base + (size_t)(nbatch * 8 * G), WorkItem{-1, 0, 0, 0, 0});
        for (int64_t tt = 0; tt < ntile; ++tt) {
          const int a = (int)(tt % tx), b = (int)((tt / tx) % ty), kz = (int)(tt / ((int64_t)tx * ty));
          for (int g = 0; g < G; ++g) {
            const int64_t pos = 8 * G * (tt / 8) + 8 * g + (tt % 8);
            w[base + (size_t)pos] = WorkItem{(int)si, a, b, kz, slots0[g]};
          }
        }
      }
      rg.push_back((int)w.size());
      kcs.push_back(kc);
    }
    if (w.size() > (size_t)INT32_MAX / 8) return fail(c, CEFF_EINVAL, "too many work items");
    return CEFF_OK;
  }

  ceff_status upload_desc() {
    HIPCK(c, hipMemcpyAsync(d_in.p, h_in.data(), sizeof(SampleDesc<T>) * h_in.size(), hipMemcpyHostToDevice, c->s));
    HIPCK(c, hipMemcpyAsync(d_out.p, h_out.data(), sizeof(SampleDesc<double>) * h_out.size(), hipMemcpyHostToDevice,
                            c->s));
    return CEFF_OK;
  }

  // Algorithmic bytes of one launch: per voxel and active load, the state words read and
  // written (single iteration: u^n, u^{n-1} read, u^{n+1} written, 9 words; two iterations:
  // u^n, u^{n-1} read, u^{n+1}, u^{n+2} written, 12 words), 3 words of body force, and the
  // material once.
  double bytes_per_launch(bool single_iteration = false) const {
    double b = 0.0;
    const double state = ts.tb && !single_iteration ? 12.0 : 9.0;
    for (size_t si = 0; si < in.size(); ++si) {
      const double N = (double)in[si].nx * in[si].ny * in[si].nz;
      int nact = 0;
      for (int l = 0; l < kMaxLoads; ++l)
        if (h_in[si].active & (1u << l)) {
          ++nact;
          b += N * sizeof(T) * (state + (h_in[si].force[l] ? 3.0 : 0.0));
        }
      if (nact) b += N * (ts.ortho ? sizeof(T) * 9.0 : (ts.tri ? sizeof(T) * 27.0 : (ts.pal ? 1.0 : sizeof(T) * 2.0)));
    }
    return b;
  }
  double vu_per_launch() const {
    double v = 0.0;
    for (size_t si = 0; si < in.size(); ++si)
      for (int l = 0; l < kMaxLoads; ++l)
        if (h_in[si].active & (1u << l)) v += (double)in[si].nx * in[si].ny * in[si].nz;
    return v;
  }

  hipError_t step_on(const WorkItem* dw, int nw, TileShape t, int grp, int par, int first, double* partials) {
    const SampleDesc<T>* d = d_in.as<SampleDesc<T>>();
    if (t.ortho) return launch_step_ortho<T>(d, dw, nw, t, par, first, partials, c->s);
    if (t.tri) return launch_step_tri<T>(d, in[0].nx * in[0].ny * in[0].nz, nw, par, first, partials, c->s);
    switch (grp) {
      case 1: return launch_step<T, 1>(d, dw, nw, t, par, first, partials, c->s);
      case 2: return launch_step<T, 2>(d, dw, nw, t, par, first, partials, c->s);
      case 3: return launch_step<T, 3>(d, dw, nw, t, par, first, partials, c->s);
      default: return launch_step<T, 6>(d, dw, nw, t, par, first, partials, c->s);
    }
  }
  // Body forces of the active loads, from the host copy of the descriptors: 0 none, 1 all, 2 some.
  // Variant 9 builds the first two cases without the per-block check, for launches whose working set
  // fits in the Infinity Cache: there the 191^3 solve gained 1.7%, while at 480^3 (4.1 GB, from HBM)
  // the build without forces moved 15% more bytes than the per-block test and took 0.934 against
  // 0.903 ms per launch on the same GPU.
  int force_state() const {
    if (beyond_cache) return 2;
    bool any = false, all = true;
    for (const SampleDesc<T>& d : h_in)
      for (int l = 0; l < kMaxLoads; ++l)
        if (d.active & (1u << l)) {
          const bool f = d.force[l] != nullptr;
          any = any || f;
          all = all && f;
        }
    return !any ? 0 : (all ? 1 : 2);
  }
  hipError_t step(int first, double* partials) {
    if (ts.tb) return step_on(d_work_s.as<WorkItem>(), (int)work_s.size(), ts1, 1, parity, first, partials);
    TileShape t = ts;
    t.force = force_state();
    return step_on(d_work.as<WorkItem>(), (int)work.size(), t, group(), parity, first, partials);
  }
  // two iterations (ts.tb); the newest iterate is then in the odd buffer of the other pair
  hipError_t step_pair(double* partials) {
    for (const SampleDesc<T>& d : h_in)
      for (int b = 0; b < 4; ++b)
        if (d.active && d.u[b][0] == nullptr) return hipErrorInvalidValue;
    return launch_step_pair<T>(d_in.as<SampleDesc<T>>(), d_work.as<WorkItem>(), (int)work.size(), ts, parity,
                               partials, c->s);
  }
  static int after_pair(int par) { return (((par >> 1) ^ 1) << 1) | 1; }

  // FP64 residual of the outer (FP64) displacement with the macroscopic strain;
  // writes float residuals to force buffers when rout is set; norms into d_norms.
  hipError_t outer_residual(bool write_force) {
    hipError_t e;
    float* const* rout = write_force ? d_rout.as<float*>() : nullptr;
    if (ts.ortho)
      e = launch_residual_ortho<double, float>(d_out.as<SampleDesc<double>>(), d_work_o.as<WorkItem>(),
                                               (int)work_o.size(), ts, 0, rout, d_partials.as<double>(), c->s);
    else if (ts.tri)
      e = launch_residual_tri<double, float>(d_out.as<SampleDesc<double>>(), in[0].nx * in[0].ny * in[0].nz,
                                             (int)work_o.size(), 0, rout, d_partials.as<double>(), c->s);
    else if (single())
      e = launch_residual<double, float, 1>(d_out.as<SampleDesc<double>>(), d_work_o.as<WorkItem>(),
                                            (int)work_o.size(), ts, 0, rout, d_partials.as<double>(), c->s);
    else
      e = launch_residual<double, float, 6>(d_out.as<SampleDesc<double>>(), d_work_o.as<WorkItem>(),
                                            (int)work_o.size(), ts, 0, rout, d_partials.as<double>(), c->s);
    if (e != hipSuccess) return e;
    return launch_finalize_norms(d_ranges_o.as<int>(), (int)in.size(), d_partials.as<double>(),
                                 d_norms.as<double>(), c->s);
  }

  ceff_status read_norms(std::vector<double>& out) {
    const size_t n = in.size() * kMaxLoads;
    HIPCK(c, c->pinned.ensure(sizeof(double) * n));
    HIPCK(c, hipMemcpyAsync(c->pinned.p, d_norms.p, sizeof(double) * n, hipMemcpyDeviceToHost, c->s));
    HIPCK(c, hipStreamSynchronize(c->s));
    out.assign(static_cast<double*>(c->pinned.p), static_cast<double*>(c->pinned.p) + n);
    return CEFF_OK;
  }

  // When the sweep's working set (all loads of this launch and the phase image)
  // exceeds the Infinity Cache, every iteration streams from HBM and the shapes
  // tuned on cache-resident grids lose to wider rows and longer z-chunks.
  // Measured on a 703^3 sphere pack with the phase table: one load per launch,
  // 18 x 14 with 12-plane chunks 3.84 ms, 66 x 7 with 48-plane chunks and the
  // high-occupancy variant 3.11 ms; six loads fused, two per block, 66 x 7 with
  // 12-plane chunks 3.19 ms and with 48-plane chunks 3.08 ms per load.  One load
  // per launch in variant 9 at 480^3: 64 x 8 blocks with 32-plane chunks
  // 0.903 ms, with 48-plane chunks 0.960 ms, against 1.000 ms for variant 3 at
  // 66 x 7 x 48.  Applied to single-image FP32 solves with the phase table whose
  // grid still yields at least 2048 (tile, chunk) items at that shape.  FP32
  // batches (one (sample, load) pair per block, variant 9) beyond the cache take
  // 64 x 8 blocks with 16-plane chunks: the 48-sample three-phase batch (samples
  // 48 to 128 wide, 5.4 GB for all six loads) ran in 8.85 s against 9.67 s with
  // the cache-resident 32 x 8 x 24 blocks (12-, 24-, 32- and 48-plane chunks
  // 8.85, 8.93, 9.09 and 9.86 s).  FP64 one-load solves of one phase image take the same
  // 64 x 8 x 32 blocks at the default occupancy: 1.757 ms per launch at 480^3 against 1.875 for the
  // 32 x 8 x 12 blocks and 1.936 for variant 3 at 34 x 14 x 12.
  void large_grid_shape() {
    const bool fp64 = sizeof(T) == 8;
    if (ts.ortho || ts.walls || ts.tri) return;
    if (fp64 && !(single() && in.size() == 1 && ts.pf == 9)) return;
    if (in.size() > 1) {
      if (ts.pf != 9 || ts.bx != 32) return;  // the batch default for samples wider than 14 cells
      double ws = 0.0;
      int64_t items = 0;
      for (const SampleIn& s : in) {
        ws += (double)s.nx * s.ny * s.nz * (6.0 * sizeof(T) * (double)Js.size() + (ts.pal ? 1.0 : 2.0 * sizeof(T)));
        items += ((s.nx + 61) / 62) * ((s.ny + 5) / 6) * ((s.nz + 15) / 16) * (int64_t)Js.size();
      }
      if (ws <= kInfinityCacheBytes || items < 2048) return;
      ts.bx = 64;
      ts.by = 8;
      ts.kc = 16;
      ts.occ = 1;
      return;
    }
    if (!ts.pal) return;
    const SampleIn& s = in[0];
    const double ws = (double)s.nx * s.ny * s.nz * (6.0 * sizeof(T) * (double)Js.size() + 1.0);
    if (ws <= kInfinityCacheBytes) return;
    if (single()) {
      const int64_t items = ((s.nx + 61) / 62) * ((s.ny + 5) / 6) * ((s.nz + 31) / 32);
      if (items < 2048) return;
      ts.bx = 64;
      ts.by = 8;
      ts.kc = 32;
      ts.pf = 9;
      ts.occ = fp64 ? 0 : 1;
      return;
    }
    const int64_t items = ((s.nx + 63) / 64) * ((s.ny + 4) / 5) * ((s.nz + 47) / 48);
    if (items < 2048) return;
    ts.bx = 66;
    ts.by = 7;
    ts.kc = 48;
    ts.occ = 0;
  }

  // Pick the launch shape: block extent, loads per block and prefetch.  With
  // autotune, time each candidate over a few iterations on this problem (the
  // iterates do not depend on the shape; only speed does) and cache the best.
  ceff_status tune() {
    const bool fp64 = sizeof(T) == 8;
    // the default block spans the largest sample (a batch's first sample may be small)
    int64_t nxm = 0, nym = 0;
    for (const SampleIn& s : in) {
      nxm = std::max(nxm, s.nx);
      nym = std::max(nym, s.ny);
    }
    if (std::getenv("CEFF_TILE")) {
      ts = with_moduli(default_tile(nxm, nym, fp64, single(), in.size() > 1, plain_cells()));
      return CEFF_OK;
    }
    ts = with_moduli(default_tile(nxm, nym, fp64, single(), in.size() > 1, plain_cells()));
    large_grid_shape();
    if (!o.autotune || ts.ortho || ts.walls || ts.tri || want_tb()) return CEFF_OK;
    const std::string key = tune_key();
    TileShape cached{};
    if (lookup_tuned(c, key, cached)) {
      ts = with_moduli(cached);
      return CEFF_OK;
    }
    std::vector<TileShape> cand;
    const int bxs[] = {18, 34, 66};
    const int bys[] = {6, 7, 10, 14};
    const int groups_fused[] = {6, 3, 2, 1};
    const int groups_single[] = {1};
    const int* groups = single() ? groups_single : groups_fused;
    const int ng = single() ? 1 : 4;
    for (int bx : bxs)
      for (int by : bys) {
        const int nt = ((bx * by + 63) / 64) * 64;
        if (nt > 512 || bx * by < 128 || bx > in[0].nx + 2 + 64 || by > in[0].ny + 2 + 8) continue;
        if ((size_t)11 * nt * sizeof(T) > 64 * 1024) continue;
        for (int gi = 0; gi < ng; ++gi)
          for (int pf = 1; pf < 6; ++pf)
            for (int kc : {0, 12})
              for (int occ = 0; occ < 2; ++occ) {
                if (occ && pf < 3) continue;
                if (pf == 5 && groups[gi] != 1) continue;
                if (pf == 5 && (bx - 2) * (by - 2) < 64) continue;
                const int grp = single() ? 1 : groups[gi];
                const TileShape t = with_moduli(TileShape{bx, by, kc, groups[gi], pf, 1, occ, 0});
                const size_t lds = (size_t)(3 + 8 * grp) * nt * sizeof(T) + (t.pal ? 1024 * sizeof(T) : 0);
                if (pf >= 3 && lds > 64 * 1024) continue;
                cand.push_back(t);
              }
      }
    // variant 9 (one load per block): rows of 16, 32 or 64 cells
    if (single() && !ts.walls && !ts.ortho && !ts.tri)
      for (int bx : {16, 32, 64})
        for (int by : {4, 6, 8, 12, 16})
          for (int kc : {12, 24, 32, 48})
            for (int occ = 0; occ < 2; ++occ) {
              if (bx * by > 512 || bx * by < 128 || bx > in[0].nx + 2 + 64 || by > in[0].ny + 2 + 8) continue;
              cand.push_back(with_moduli(TileShape{bx, by, kc, 1, 9, 1, occ, 0}));
            }
    float best = 1e30f;
    TileShape bt = ts;
    std::vector<unsigned> saved(in.size());
    for (size_t si = 0; si < in.size(); ++si) {
      saved[si] = h_in[si].active;
      for (int J : Js) h_in[si].active |= 1u << slot_of(J);
    }
    for (const TileShape& t : cand) {
      std::vector<WorkItem> w;
      std::vector<int> rg, kcs;
      const int grp = single() || t.pf == 5 || t.pf == 9 ? 1 : t.group;
      STCK(build_work(t, grp, w, rg, kcs));
      DevBuf dw;
      HIPCK(c, dw.alloc(sizeof(WorkItem) * w.size()));
      HIPCK(c, hipMemcpyAsync(dw.p, w.data(), sizeof(WorkItem) * w.size(), hipMemcpyHostToDevice, c->s));
      for (size_t si = 0; si < in.size(); ++si) h_in[si].kc = kcs[si];
      STCK(upload_desc());
      auto run = [&](int n) -> hipError_t {
        for (int q = 0; q < n; ++q) {
          hipError_t e = step_on(dw.as<WorkItem>(), (int)w.size(), t, grp, q & 1, 0, nullptr);
          if (e != hipSuccess) return e;
        }
        return hipSuccess;
      };
      HIPCK(c, run(2));
      HIPCK(c, hipEventRecord(c->ev0, c->s));
      HIPCK(c, run(6));
      HIPCK(c, hipEventRecord(c->ev1, c->s));
      HIPCK(c, hipEventSynchronize(c->ev1));
      float ms = 0.f;
      HIPCK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
      if (std::getenv("CEFF_TUNE_VERBOSE"))
        std::fprintf(stderr, "tune bx=%d by=%d kc=%d group=%d pf=%d order=%d occ=%d: %.4f ms/launch\n", t.bx, t.by,
                     t.kc, grp, t.pf, t.order, t.occ, ms / 6);
      if (ms < best) {
        best = ms;
        bt = t;
      }
    }
    for (size_t si = 0; si < in.size(); ++si) h_in[si].active = saved[si];
    ts = bt;
    remember_tuned(c, key, ts);
    return CEFF_OK;
  }

  // What the best launch shape depends on: the precision, which loads advance
  // together, whether the moduli can come from a shared phase table, the
  // samples' dimensions, and the kernels themselves (a hash of their source,
  // fixed at build time).  Wall boundaries and orthotropic cells are not tuned.
  std::string tune_key() const {
    uint64_t h = 1469598103934665603ull;  // FNV-1a over every sample's dimensions
    for (const SampleIn& s : in)
      for (int64_t d : {s.nx, s.ny, s.nz})
        for (int b = 0; b < 8; ++b) {
          h ^= (uint64_t)((d >> (8 * b)) & 0xff);
          h *= 1099511628211ull;
        }
    unsigned mask = 0;
    for (int J : Js) mask |= 1u << J;
    TileShape probe = default_tile(in[0].nx, in[0].ny, sizeof(T) == 8, single(), in.size() > 1);
    probe.pf = 3;
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s:loads%02x:pal%d:samples%zu:%lldx%lldx%lld:dims%016llx:kernels%s",
                  sizeof(T) == 4 ? "f32" : "f64", mask, with_moduli(probe).pal, in.size(), (long long)in[0].nx,
                  (long long)in[0].ny, (long long)in[0].nz, (unsigned long long)h, CEFF_KERNEL_HASH);
    return buf;
  }

  // Two iterations per launch: one image, one load, FP32, periodic isotropic cells, when
  // CEFF_TB=1 asks for it.
  bool want_tb() const {
    const char* env = std::getenv("CEFF_TB");
    return env != nullptr && std::strcmp(env, "1") == 0 && sizeof(T) == 4 && in.size() == 1 && single() &&
           in[0].c64 == nullptr && in[0].t64 == nullptr && !in[0].walls;
  }

  ceff_status setup() {
    const int ns = (int)in.size();
    const int nbuf = want_tb() ? 4 : 2;
    ubuf.resize(ns);
    base.resize(ns);
    force.resize(ns);
    h_in.assign(ns, SampleDesc<T>{});
    h_out.assign(ns, SampleDesc<double>{});
    for (int si = 0; si < ns; ++si) {
      const SampleIn& s = in[si];
      const int64_t N = s.nx * s.ny * s.nz;
      const Params p = make_params(s.nx, s.ny, s.nz, s.h, o.courant, o.strouhal);
      for (SampleDesc<T>* dsc : {&h_in[si]}) {
        dsc->nx = s.nx; dsc->ny = s.ny; dsc->nz = s.nz; dsc->N = N;
        dsc->rhx = (T)(1.0 / s.h[0]); dsc->rhy = (T)(1.0 / s.h[1]); dsc->rhz = (T)(1.0 / s.h[2]);
        dsc->mom = (T)p.mom; dsc->sfac = (T)p.sfac; dsc->sfac_first = (T)p.sfac_first;
        dsc->K = sizeof(T) == 8 ? (const T*)s.K64 : (const T*)s.K32;
        dsc->G = sizeof(T) == 8 ? (const T*)s.G64 : (const T*)s.G32;
        dsc->phase = s.phase;
        dsc->ptab = sizeof(T) == 8 ? (const T*)s.ptab64 : (const T*)s.ptab32;
        dsc->nphase = s.nphase;
        dsc->cst = sizeof(T) == 8 ? (const T*)s.c64 : (const T*)s.c32;
        dsc->c21 = sizeof(T) == 8 ? (const T*)s.t64 : (const T*)s.t32;
        dsc->tse = sizeof(T) == 8 ? (const T*)s.tse64 : (const T*)s.tse32;
        dsc->tihf = sizeof(T) == 8 ? (const T*)s.tihf64 : (const T*)s.tihf32;
        dsc->walls = s.walls;
      }
      SampleDesc<double>& od = h_out[si];
      od.nx = s.nx; od.ny = s.ny; od.nz = s.nz; od.N = N;
      od.rhx = 1.0 / s.h[0]; od.rhy = 1.0 / s.h[1]; od.rhz = 1.0 / s.h[2];
      od.mom = p.mom; od.sfac = p.sfac; od.sfac_first = p.sfac_first;
      od.K = s.K64; od.G = s.G64;
      od.cst = s.c64;
      od.c21 = s.t64;
      od.tse = s.tse64;
      od.tihf = s.tihf64;
      od.walls = s.walls;
      if (s.t64) {  // general cells: one sample; pipeline scratch (24N) for the sweeps and the FP64 residual
        HIPCK(c, tscr_in.alloc(sizeof(T) * 24 * N));
        h_in[si].tscr = tscr_in.as<T>();
        if (sizeof(T) == 8) {
          od.tscr = (double*)h_in[si].tscr;
        } else {
          HIPCK(c, tscr_out.alloc(sizeof(double) * 24 * N));
          od.tscr = tscr_out.as<double>();
        }
      }
      for (int J : Js) {
        const int l = slot_of(J);
        h_in[si].wshear[l] = od.wshear[l] = s.walls && J >= 3 ? J : 0;
        for (int b = 0; b < nbuf; ++b) {
          HIPCK(c, ubuf[si][b * kMaxLoads + l].alloc(sizeof(T) * 3 * N));
          HIPCK(c, launch_fill<T>(ubuf[si][b * kMaxLoads + l].as<T>(), 3 * N, T(0), c->s));
          h_in[si].u[b][l] = ubuf[si][b * kMaxLoads + l].as<T>();
        }
        double E[6];
        unit_strain(J, E);
        for (int q = 0; q < 6; ++q) {
          h_in[si].E[l][q] = (T)E[q];
          od.E[l][q] = E[q];
        }
        if (mixed) {
          HIPCK(c, base[si][l].alloc(sizeof(double) * 3 * N));
          HIPCK(c, launch_fill<double>(base[si][l].as<double>(), 3 * N, 0.0, c->s));
          HIPCK(c, force[si][l].alloc(sizeof(float) * 3 * N));
          od.u[0][l] = base[si][l].as<double>();
        } else {
          od.u[0][l] = (double*)h_in[si].u[0][l];  // T == double here
        }
        Prob pr;
        pr.s = si; pr.J = J; pr.slot = l;
        probs.push_back(pr);
      }
    }
    HIPCK(c, d_in.alloc(sizeof(SampleDesc<T>) * ns));
    HIPCK(c, d_out.alloc(sizeof(SampleDesc<double>) * ns));
    STCK(tune());
    {
      // both displacement buffers and the body force of every advancing load, and the material
      // (191^3 in mixed precision from the phase image: 258 MB)
      double ws = 0.0;
      for (const SampleIn& s : in)
        ws += (double)s.nx * s.ny * s.nz * (9.0 * sizeof(T) * (double)Js.size() + (ts.pal ? 1.0 : 2.0 * sizeof(T)));
      beyond_cache = ws > kInfinityCacheBytes;
    }
    std::vector<int> kcs, kcs_o;
    ts.tb = nbuf == 4 ? 1 : 0;  // pairs only where the second buffer pair exists
    STCK(build_work(ts, group(), work, ranges, kcs));
    if (ts.tb) {
      // the single iterations share the z-chunk length (SampleDesc::kc) with the pairs
      ts.kc = kcs[0];
      ts1 = ts;
      ts1.tb = 0;
      std::vector<int> kcs_s;
      STCK(build_work(ts1, 1, work_s, ranges_s, kcs_s));
      HIPCK(c, d_work_s.alloc(sizeof(WorkItem) * work_s.size()));
      HIPCK(c, hipMemcpyAsync(d_work_s.p, work_s.data(), sizeof(WorkItem) * work_s.size(), hipMemcpyHostToDevice,
                              c->s));
    }
    TileShape to = ts;
    to.kc = 0;
    to.tb = 0;  // the residual kernel tiles with a one-cell ghost ring
    STCK(build_work(to, single() || ts.ortho || ts.walls ? 1 : kMaxLoads, work_o, ranges_o, kcs_o));
    for (int si = 0; si < ns; ++si) {
      h_in[si].kc = kcs[si];
      h_out[si].kc = kcs_o[si];
      h_in[si].work_begin = ranges[2 * si];
      h_in[si].work_end = ranges[2 * si + 1];
      h_out[si].work_begin = ranges_o[2 * si];
      h_out[si].work_end = ranges_o[2 * si + 1];
    }
    HIPCK(c, d_work.alloc(sizeof(WorkItem) * work.size()));
    HIPCK(c, hipMemcpyAsync(d_work.p, work.data(), sizeof(WorkItem) * work.size(), hipMemcpyHostToDevice, c->s));
    HIPCK(c, d_work_o.alloc(sizeof(WorkItem) * work_o.size()));
    HIPCK(c, hipMemcpyAsync(d_work_o.p, work_o.data(), sizeof(WorkItem) * work_o.size(), hipMemcpyHostToDevice,
                            c->s));
    HIPCK(c, d_partials.alloc(sizeof(double) * kMaxLoads * std::max({work.size(), work_o.size(), work_s.size()})));
    HIPCK(c, d_norms.alloc(sizeof(double) * kMaxLoads * ns));
    HIPCK(c, d_ranges.alloc(sizeof(int) * ranges.size()));
    HIPCK(c, hipMemcpyAsync(d_ranges.p, ranges.data(), sizeof(int) * ranges.size(), hipMemcpyHostToDevice, c->s));
    HIPCK(c, d_ranges_o.alloc(sizeof(int) * ranges_o.size()));
    HIPCK(c, hipMemcpyAsync(d_ranges_o.p, ranges_o.data(), sizeof(int) * ranges_o.size(), hipMemcpyHostToDevice,
                            c->s));
    // per-slot float residual outputs for the outer check (only slot arrays of sample 0 are
    // addressed through rout; batches write forces per sample through the same slot pointers
    // when the batch has one sample, otherwise through per-sample passes below)
    HIPCK(c, d_rout.alloc(sizeof(float*) * kMaxLoads));
    // re-zero displacements (tuning may have run steps on them)
    for (int si = 0; si < ns; ++si)
      for (int J : Js) {
        const int l = slot_of(J);
        const int64_t N = in[si].nx * in[si].ny * in[si].nz;
        for (int b = 0; b < nbuf; ++b) HIPCK(c, launch_fill<T>(h_in[si].u[b][l], 3 * N, T(0), c->s));
      }
    return CEFF_OK;
  }

  // Outer FP64 residual for sample set `which` (by active masks already set in h_out).
  // Force outputs are per sample, so samples are processed one at a time when forces
  // are written.
  ceff_status outer_pass(bool write_force, std::vector<double>& norms) {
    const int ns = (int)in.size();
    norms.assign((size_t)ns * kMaxLoads, 0.0);
    if (!write_force) {
      STCK(upload_desc());
      HIPCK(c, outer_residual(false));
      STCK(read_norms(norms));
      ++outer;
      return CEFF_OK;
    }
    std::vector<unsigned> saved(ns);
    for (int si = 0; si < ns; ++si) saved[si] = h_out[si].active;
    for (int si = 0; si < ns; ++si) {
      if (!saved[si]) continue;
      for (int sj = 0; sj < ns; ++sj) h_out[sj].active = sj == si ? saved[si] : 0u;
      float* ptrs[kMaxLoads] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
      for (int l = 0; l < kMaxLoads; ++l)
        if (saved[si] & (1u << l)) ptrs[l] = force[si][l].as<float>();
      HIPCK(c, hipMemcpyAsync(d_rout.p, ptrs, sizeof ptrs, hipMemcpyHostToDevice, c->s));
      STCK(upload_desc());
      HIPCK(c, outer_residual(true));
      std::vector<double> nn;
      STCK(read_norms(nn));
      for (int l = 0; l < kMaxLoads; ++l) norms[(size_t)si * kMaxLoads + l] = nn[(size_t)si * kMaxLoads + l];
      ++outer;
    }
    for (int si = 0; si < ns; ++si) h_out[si].active = saved[si];
    return CEFF_OK;
  }

  ceff_status run_block(int m) {
    // m iterations: m-1 plain steps and one that also reduces the residual of its input
    // (with two iterations per launch: m/2 launches, the last one reducing the residual of
    // its intermediate iterate)
    const double bpl = bytes_per_launch(), vpl = vu_per_launch();
    const int nl = ts.tb ? m / 2 : m;
    // a captured graph has the buffer parity of its first launch and the launches' body-force
    // case built in
    const int fs = force_state();
    if (o.use_graph && (!gexec || graph_m != m || graph_parity != parity || graph_force != fs)) {
      if (gexec) {
        (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
      }
      if (graph) {
        (void)hipGraphDestroy(graph);
        graph = nullptr;
      }
      HIPCK(c, hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
      const int p0 = parity;
      hipError_t e = hipSuccess;
      for (int q = 0; q < nl && e == hipSuccess; ++q) {
        double* part = q == nl - 1 ? d_partials.as<double>() : nullptr;
        e = ts.tb ? step_pair(part) : step(0, part);
        parity = ts.tb ? after_pair(parity) : parity ^ 1;
      }
      if (e == hipSuccess)
        e = launch_finalize_norms(d_ranges.as<int>(), (int)in.size(), d_partials.as<double>(), d_norms.as<double>(),
                                  c->s);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(c->s, &g);
      parity = p0;
      HIPCK(c, e);
      HIPCK(c, e2);
      graph = g;
      HIPCK(c, hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
      graph_m = m;
      graph_parity = p0;
      graph_force = fs;
    }
    HIPCK(c, hipEventRecord(c->ev0, c->s));
    if (o.use_graph) {
      HIPCK(c, hipGraphLaunch(gexec, c->s));
      for (int q = 0; q < nl; ++q) parity = ts.tb ? after_pair(parity) : parity ^ 1;
    } else {
      for (int q = 0; q < nl; ++q) {
        double* part = q == nl - 1 ? d_partials.as<double>() : nullptr;
        HIPCK(c, ts.tb ? step_pair(part) : step(0, part));
        parity = ts.tb ? after_pair(parity) : parity ^ 1;
      }
      HIPCK(c, launch_finalize_norms(d_ranges.as<int>(), (int)in.size(), d_partials.as<double>(),
                                     d_norms.as<double>(), c->s));
    }
    HIPCK(c, hipEventRecord(c->ev1, c->s));
    HIPCK(c, hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIPCK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    step_ms += ms;
    step_bytes += bpl * nl;
    vu += vpl * m;
    launches += nl;
    return CEFF_OK;
  }

  void record(int64_t it, int J, double rr) {
    if (hist) {
      hist->push_back((double)it);
      hist->push_back((double)J);
      hist->push_back(rr);
    }
  }

  // Initial guess (ceff_solve_opts::warm_u, one image).  MIXED: the guess becomes
  // the FP64 displacement and each problem starts as right after a fold: zero FP32
  // correction, the FP64 residual of the guess as body force, no macroscopic
  // strain in the sweep.  FP64: the guess is the first iterate.
  ceff_status apply_warm() {
    const int64_t N = in[0].nx * in[0].ny * in[0].nz;
    std::vector<Prob*> warm;
    for (auto& p : probs) {
      if (!p.active) continue;
      const double* src = o.warm_u + (int64_t)p.J * 3 * N;
      if (mixed) {
        HIPCK(c, hipMemcpyAsync(base[p.s][p.slot].p, src, sizeof(double) * 3 * N, hipMemcpyHostToDevice, c->s));
        h_out[p.s].active |= 1u << p.slot;
        warm.push_back(&p);
      } else {
        HIPCK(c, hipMemcpyAsync(h_in[p.s].u[0][p.slot], src, sizeof(double) * 3 * N, hipMemcpyHostToDevice, c->s));
      }
    }
    if (!mixed) return CEFF_OK;
    std::vector<double> n64;
    STCK(outer_pass(true, n64));
    for (auto& d : h_out) d.active = 0;
    for (Prob* p : warm) {
      const double rr = std::sqrt(n64[(size_t)p->s * kMaxLoads + p->slot]) / p->r0;
      p->relres = rr;
      record(0, p->J, rr);
      if (!std::isfinite(rr) || rr <= o.rtol) {
        p->active = false;
        p->iters = 0;
        p->st = std::isfinite(rr) ? CEFF_OK : CEFF_EDIVERGED;
        h_in[p->s].active &= ~(1u << p->slot);
        continue;
      }
      p->relres_base = rr;
      p->phase = 1;
      for (int q = 0; q < 6; ++q) h_in[p->s].E[p->slot][q] = T(0);
      h_in[p->s].force[p->slot] = (const T*)force[p->s][p->slot].as<float>();
    }
    return CEFF_OK;
  }

  ceff_status solve() {
    STCK(setup());
    // initial residual norms ||div(C:E)|| in FP64 (all displacements are zero)
    for (size_t si = 0; si < in.size(); ++si) {
      unsigned m = 0;
      for (auto& p : probs)
        if (p.s == (int)si) m |= 1u << p.slot;
      h_out[si].active = m;
      h_in[si].active = 0;
    }
    std::vector<double> nn;
    STCK(outer_pass(false, nn));
    for (auto& p : probs) {
      p.r0 = std::sqrt(nn[(size_t)p.s * kMaxLoads + p.slot]);
      if (p.r0 > 0.0 && std::isfinite(p.r0)) {
        // A load whose affine state is in equilibrium up to rounding (e.g. a shear that every
        // layer of a laminate carries with the same modulus, in constants that are not exact
        // binary numbers) leaves only rounding noise, which no iteration reduces: compare the
        // residual with its rounding scale, sqrt(3N) |sigma| 2/h_min, |sigma| from the affine
        // state's mean stresses, and treat it as zero below 1e-13 of that.
        double a6[6];
        const double* zero = mixed ? base[p.s][p.slot].template as<double>() : (const double*)h_in[p.s].u[0][p.slot];
        STCK(stress_average(c, in[p.s], p.J, zero, a6));
        double smax = 0.0;
        for (double v : a6) smax = std::max(smax, std::fabs(v));
        const SampleIn& sp = in[p.s];
        const double N = (double)sp.nx * sp.ny * sp.nz;
        const double scale = std::sqrt(3.0 * N) * smax * 2.0 / std::min({sp.h[0], sp.h[1], sp.h[2]});
        if (p.r0 <= 1e-13 * scale) p.r0 = 0.0;
      }
      if (p.r0 > 0.0 && std::isfinite(p.r0)) {
        p.active = true;
        h_in[p.s].active |= 1u << p.slot;
      } else if (!std::isfinite(p.r0)) {
        p.st = CEFF_EDIVERGED;
      } else {
        p.relres = 0.0;
        p.sol = 0;  // zero displacement: the affine state is in equilibrium
        record(0, p.J, 0.0);
      }
    }
    for (auto& d : h_out) d.active = 0;
    if (o.warm_u) STCK(apply_warm());
    bool any = false;
    for (auto& p : probs) any |= p.active;
    if (any) {
      STCK(upload_desc());
      // first iteration: u^1 from u^0 (zero, or the initial guess) without momentum
      const double bpl = bytes_per_launch(true) * 6.0 / 9.0, vpl = vu_per_launch();
      HIPCK(c, hipEventRecord(c->ev0, c->s));
      parity = 0;
      HIPCK(c, step(1, nullptr));
      HIPCK(c, hipEventRecord(c->ev1, c->s));
      HIPCK(c, hipEventSynchronize(c->ev1));
      float ms = 0.f;
      HIPCK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
      step_ms += ms; step_bytes += bpl; vu += vpl; launches += 1;
      parity = 1;
      for (auto& p : probs)
        if (p.active) p.iters = 1;
    }
    int m = o.check_every + (o.check_every & 1);
    if (ts.tb) m = (m + 3) / 4 * 4;  // whole pairs, an even number of them
    while (true) {
      bool act = false;
      for (auto& p : probs) act |= p.active;
      if (!act) break;
      STCK(run_block(m));
      std::vector<double> norms;
      STCK(read_norms(norms));
      bool desc_dirty = false;
      std::vector<Prob*> to_fold;
      for (auto& p : probs) {
        if (!p.active) continue;
        const int64_t checked = p.iters + m - 1;  // iterate whose residual was reduced
        p.iters += m;
        const double rr = std::sqrt(norms[(size_t)p.s * kMaxLoads + p.slot]) / p.r0;
        p.relres = rr;
        record(checked, p.J, rr);
        const bool bad = !std::isfinite(rr) || rr > 1e6;
        const bool cap = checked >= o.max_iter;
        if (!mixed) {
          if (rr <= o.rtol || bad || cap) {
            p.active = false;
            p.iters = checked;
            p.sol = parity ^ 1;
            p.st = rr <= o.rtol ? CEFF_OK : (bad ? CEFF_EDIVERGED : CEFF_ENOTCONV);
            h_in[p.s].active &= ~(1u << p.slot);
            desc_dirty = true;
          }
        } else {
          bool stall = false;
          if (p.recent.size() >= 3) {
            const double best = *std::min_element(p.recent.end() - 3, p.recent.end());
            stall = rr > 0.9 * best;
          }
          p.recent.push_back(rr);
          if (bad) {
            p.active = false;
            p.iters = checked;
            p.st = CEFF_EDIVERGED;
            h_in[p.s].active &= ~(1u << p.slot);
            desc_dirty = true;
          } else if (rr <= o.rtol || rr <= o.fold_ratio * p.relres_base || stall || cap) {
            to_fold.push_back(&p);
          }
        }
      }
      if (!to_fold.empty()) {
        // fold u^{n} (in buffer parity^1) into the FP64 displacement, keep the momentum
        for (Prob* p : to_fold) {
          const int64_t N = in[p->s].nx * in[p->s].ny * in[p->s].nz;
          HIPCK(c, launch_fold(base[p->s][p->slot].as<double>(), (float*)h_in[p->s].u[parity][p->slot],
                               (float*)h_in[p->s].u[parity ^ 1][p->slot], 3 * N, c->s));
          h_out[p->s].active |= 1u << p->slot;
        }
        std::vector<double> n64;
        STCK(outer_pass(true, n64));
        for (auto& d : h_out) d.active = 0;
        for (Prob* p : to_fold) {
          const int64_t checked = p->iters - 1;
          const double rr = std::sqrt(n64[(size_t)p->s * kMaxLoads + p->slot]) / p->r0;
          p->relres = rr;
          p->recent.clear();
          record(checked, p->J, rr);
          const bool bad = !std::isfinite(rr) || rr > 1e6;
          if (rr <= o.rtol || bad || checked >= o.max_iter) {
            p->active = false;
            p->iters = checked;
            p->st = rr <= o.rtol ? CEFF_OK : (bad ? CEFF_EDIVERGED : CEFF_ENOTCONV);
            h_in[p->s].active &= ~(1u << p->slot);
          } else {
            p->relres_base = rr;
            if (p->phase == 0) {
              p->phase = 1;
              for (int q = 0; q < 6; ++q) h_in[p->s].E[p->slot][q] = T(0);
              h_in[p->s].force[p->slot] = (const T*)force[p->s][p->slot].as<float>();
            }
          }
        }
        desc_dirty = true;
      }
      if (desc_dirty) STCK(upload_desc());
    }
    return CEFF_OK;
  }

  // FP64 solution of problem p on the device.
  const double* solution(const Prob& p) const {
    if (mixed) return base[p.s][p.slot].as<double>();
    return (const double*)h_in[p.s].u[p.sol][p.slot];
  }
};

// FP64 volume averages of the six stresses of u under unit load J, with the
// kernel's block partials (6 per block, at most cap blocks) in `part` and the
// six sums in `o6` (device memory).
ceff_status stress_average_into(ceff_ctx* c, const SampleIn& s, int J, const double* u, double* part, int cap,
                                double* o6, double out6[6]) {
  const int64_t N = s.nx * s.ny * s.nz;
  double E[6];
  unit_strain(J, E);
  DevBuf tscr, tdesc;  // general cells: the pipeline's scratch and a one-entry sample table
  SampleDesc<double> th{};
  if (s.t64) {
    HIPCK(c, tscr.alloc(sizeof(double) * 24 * N));
    th.nx = s.nx; th.ny = s.ny; th.nz = s.nz; th.N = N;
    th.rhx = 1.0 / s.h[0]; th.rhy = 1.0 / s.h[1]; th.rhz = 1.0 / s.h[2];
    th.u[0][0] = const_cast<double*>(u);
    for (int q = 0; q < 6; ++q) th.E[0][q] = E[q];
    th.active = 1u;
    th.c21 = s.t64; th.tse = s.tse64; th.tihf = s.tihf64; th.tscr = tscr.as<double>();
    HIPCK(c, tdesc.alloc(sizeof th));
    HIPCK(c, hipMemcpyAsync(tdesc.p, &th, sizeof th, hipMemcpyHostToDevice, c->s));
    HIPCK(c, launch_average_stress_tri(tdesc.as<SampleDesc<double>>(), tscr.as<double>(), N, part, cap, o6, c->s));
  } else if (s.c64)
    HIPCK(c, launch_average_stress_ortho(s.nx, s.ny, s.nz, s.h, s.c64, E, u, part, cap, o6, c->s));
  else
    HIPCK(c, launch_average_stress(s.nx, s.ny, s.nz, s.h, s.K64, s.G64, E, u, part, cap, o6,
                                   s.walls ? (J >= 3 ? J : 1) : 0, c->s));
  HIPCK(c, hipMemcpyAsync(out6, o6, sizeof(double) * 6, hipMemcpyDeviceToHost, c->s));
  HIPCK(c, hipStreamSynchronize(c->s));
  for (int q = 0; q < 6; ++q) out6[q] /= (double)N;
  return CEFF_OK;
}

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_addr;  // device ordinal -> address of that GPU's `scratch`

// Look up this GPU's copy of `scratch` once (the device must be current).
ceff_status init_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr.count(device)) return CEFF_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return CEFF_EDEVICE;
  g_scratch_addr[device] = static_cast<double*>(p);
  return CEFF_OK;
}

double* scratch_addr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  return it == g_scratch_addr.end() ? nullptr : it->second;
}

ceff_status stress_average(ceff_ctx* c, const SampleIn& s, int J, const double* u, double out6[6]) {
  DevBuf part, o6;
  HIPCK(c, part.alloc(sizeof(double) * 6 * kAvgBlocks));
  HIPCK(c, o6.alloc(sizeof(double) * 6));
  return stress_average_into(c, s, J, u, part.as<double>(), kAvgBlocks, o6.as<double>(), out6);
}

// The launch shape an engine ran with, into the context's counters.
template <typename T>
void record_shape(ceff_ctx* c, const Engine<T>& e) {
  c->stats.tile_bx = e.ts.bx;
  c->stats.tile_by = e.ts.by;
  c->stats.tile_kc = e.h_in.empty() ? 0 : e.h_in[0].kc;
  c->stats.tile_group = e.group();
  c->stats.tile_variant = e.ts.tb ? 6 : e.ts.pf;
  c->stats.phase_moduli = e.ts.pal;
  c->stats.tile_occ = e.ts.occ;
}

template <typename T>
ceff_status run_engine(ceff_ctx* c, std::vector<SampleIn> samples, std::vector<int> Js, const ceff_solve_opts& o,
                       int Lk, std::vector<std::array<double, 36>>& C, std::vector<std::array<int64_t, 6>>& iters,
                       std::vector<double>* hist, bool keep, ceff_status& worst) {
  Engine<T> e;
  e.c = c;
  e.in = std::move(samples);
  e.o = o;
  e.mixed = sizeof(T) == 4;
  e.Lk = Lk;
  e.Js = std::move(Js);
  e.hist = hist;
  STCK(e.solve());
  for (auto& p : e.probs) {
    double a6[6];
    STCK(stress_average(c, e.in[p.s], p.J, e.solution(p), a6));
    for (int I = 0; I < 6; ++I) C[p.s][I * 6 + p.J] = a6[I];
    iters[p.s][p.J] = p.iters;
    if (p.st != CEFF_OK && (worst == CEFF_OK || p.st == CEFF_EDIVERGED)) worst = p.st;
    if (keep) {
      const int64_t N = e.in[p.s].nx * e.in[p.s].ny * e.in[p.s].nz;
      HIPCK(c, c->keep[p.J].alloc(sizeof(double) * 3 * N));
      HIPCK(c, hipMemcpyAsync(c->keep[p.J].p, e.solution(p), sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, c->s));
      c->kept[p.J] = true;
    }
  }
  HIPCK(c, hipStreamSynchronize(c->s));
  c->stats.step_launches += e.launches;
  c->stats.step_time_ms += e.step_ms;
  c->stats.step_bytes += e.step_bytes;
  c->stats.voxel_updates += e.vu;
  c->stats.outer_checks += e.outer;
  record_shape(c, e);
  return CEFF_OK;
}

ceff_status ensure32(ceff_ctx* c) {
  if (c->have32) return CEFF_OK;
  const int64_t N = c->nx * c->ny * c->nz;
  if (c->tri) {
    HIPCK(c, c->t32.alloc(sizeof(float) * 21 * N));
    HIPCK(c, launch_convert<double, float>(c->t64.as<double>(), c->t32.as<float>(), 21 * N, c->s));
    HIPCK(c, c->tse32.alloc(sizeof(float) * 3 * N));
    HIPCK(c, c->tihf32.alloc(sizeof(float) * 3 * N));
    HIPCK(c, launch_tri_setup<float>(c->t64.as<double>(), c->nx, c->ny, c->nz, c->tse32.as<float>(),
                                     c->tihf32.as<float>(), c->s));
    c->have32 = true;
    return CEFF_OK;
  }
  if (c->ortho) {
    HIPCK(c, c->c32.alloc(sizeof(float) * 9 * N));
    HIPCK(c, launch_convert<double, float>(c->c64.as<double>(), c->c32.as<float>(), 9 * N, c->s));
    c->have32 = true;
    return CEFF_OK;
  }
  HIPCK(c, c->K32.alloc(sizeof(float) * N));
  HIPCK(c, c->G32.alloc(sizeof(float) * N));
  HIPCK(c, launch_convert<double, float>(c->K64.as<double>(), c->K32.as<float>(), N, c->s));
  HIPCK(c, launch_convert<double, float>(c->G64.as<double>(), c->G32.as<float>(), N, c->s));
  c->have32 = true;
  return CEFF_OK;
}

// Wall boundaries are implemented for isotropic cells only.
ceff_status check_walls_material(ceff_ctx* c) {
  if (c->boundary == CEFF_BC_WALLS && (c->ortho || c->tri))
    return fail(c, CEFF_EUNSUPPORTED, "wall boundaries with anisotropic cells");
  return CEFF_OK;
}

ceff_status begin_call(ceff_ctx* c) {
  if (!c) return CEFF_EINVAL;
  c->err.clear();
  HIPCK(c, hipSetDevice(c->device));
  HIPCK(c, hipStreamSynchronize(c->user));
  return CEFF_OK;
}

// Inverse of a 6x6 row-major matrix by Gauss-Jordan elimination with partial
// pivoting (FP64).  False if a pivot falls below 1e-12 of the largest entry.
bool invert6(const double* A, double* X) {
  double a[6][12];
  double amax = 0.0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      a[i][j] = A[i * 6 + j];
      a[i][6 + j] = i == j ? 1.0 : 0.0;
      amax = std::max(amax, std::fabs(A[i * 6 + j]));
    }
  if (!(amax > 0.0)) return false;
  for (int col = 0; col < 6; ++col) {
    int piv = col;
    for (int r = col + 1; r < 6; ++r)
      if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
    if (!(std::fabs(a[piv][col]) > 1e-12 * amax)) return false;
    if (piv != col)
      for (int j = 0; j < 12; ++j) std::swap(a[piv][j], a[col][j]);
    const double d = a[col][col];
    for (int j = 0; j < 12; ++j) a[col][j] /= d;
    for (int r = 0; r < 6; ++r) {
      if (r == col) continue;
      const double f = a[r][col];
      if (f == 0.0) continue;
      for (int j = 0; j < 12; ++j) a[r][j] -= f * a[col][j];
    }
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) X[i * 6 + j] = a[i][6 + j];
  return true;
}


// Automatic load fusion.  One iteration touches, per cell, both displacement
// buffers of every load it advances plus the material.  With a phase image in
// mixed precision the loads share only the 1-byte phase id of a cell (1 of 37
// bytes per voxel-update), and one launch per load is faster at every size
// measured: 191^3, cache-resident, 3.4 s against 4.0 s for six loads; 479^3,
// from HBM, 0.995 against 1.068 ms per load and iteration.  Otherwise, when the
// working set of one load fits in the Infinity Cache but the one of all loads
// does not, running the loads one after another keeps each sweep's data
// cache-resident; beyond that fusion reads the material once for all loads.
bool fuse_by_cache(const ceff_ctx* c, bool mixed, int nloads) {
  if (nloads < 2) return true;
  if (mixed && c->nphase > 0 && !c->ortho) return false;
  const double N = (double)c->nx * c->ny * c->nz;
  const double w = mixed ? 4.0 : 8.0;
  const double mat = c->ortho ? 9.0 * w : (c->nphase > 0 ? 1.0 : 2.0 * w);
  const double one = N * (6.0 * w + mat), all = N * (6.0 * w * nloads + mat);
  return !(one <= kInfinityCacheBytes && all > kInfinityCacheBytes);
}

SampleIn ctx_sample(ceff_ctx* c) {
  SampleIn s;
  s.nx = c->nx; s.ny = c->ny; s.nz = c->nz;
  s.h[0] = c->h[0]; s.h[1] = c->h[1]; s.h[2] = c->h[2];
  s.K64 = c->K64.as<double>(); s.G64 = c->G64.as<double>();
  s.K32 = c->have32 ? c->K32.as<float>() : nullptr;
  s.G32 = c->have32 ? c->G32.as<float>() : nullptr;
  s.walls = c->boundary == CEFF_BC_WALLS ? 1 : 0;
  if (c->ortho) {
    s.c64 = c->c64.as<double>();
    s.c32 = c->have32 ? c->c32.as<float>() : nullptr;
  }
  if (c->tri) {
    s.t64 = c->t64.as<double>();
    s.tse64 = c->tse64.as<double>();
    s.tihf64 = c->tihf64.as<double>();
    s.t32 = c->have32 ? c->t32.as<float>() : nullptr;
    s.tse32 = c->have32 ? c->tse32.as<float>() : nullptr;
    s.tihf32 = c->have32 ? c->tihf32.as<float>() : nullptr;
  }
  if (c->nphase > 0) {
    s.phase = c->phase8.as<uint8_t>();
    s.ptab64 = c->ptab64.as<double>();
    s.ptab32 = c->ptab32.as<float>();
    s.nphase = c->nphase;
  }
  return s;
}

}  // namespace

// ---- C ABI ---------------------------------------------------------------------------

extern "C" {

void ceff_default_opts(ceff_solve_opts* o) {
  if (!o) return;
  o->precision = CEFF_PREC_MIXED;
  o->rtol = 1e-8;
  o->max_iter = 2000000;
  o->check_every = 100;
  o->courant = 0.95;
  o->strouhal = 0.0;
  o->fuse_loads = CEFF_FUSE_AUTO;
  o->use_graph = 1;
  o->keep_fields = 0;
  o->autotune = 0;
  o->fold_ratio = 1e-3;
  o->warm_u = nullptr;
}

ceff_status ceff_check_grid(int64_t nx, int64_t ny, int64_t nz, double hx, double hy, double hz) {
  const double h[3] = {hx, hy, hz};
  return validate_grid(nullptr, nx, ny, nz, h);
}

ceff_status ceff_auto_strouhal(int64_t nx, int64_t ny, int64_t nz, double hx, double hy, double hz, double courant,
                               double* st_out) {
  const double h[3] = {hx, hy, hz};
  if (!st_out) return CEFF_EINVAL;
  STCK(validate_grid(nullptr, nx, ny, nz, h));
  if (!(courant > 0.0) || !(courant <= 1.0)) return CEFF_EINVAL;
  const double Lx = std::max({nx * hx, ny * hy, nz * hz});
  *st_out = auto_strouhal(Lx, courant / std::sqrt(1.0 / (hx * hx) + 1.0 / (hy * hy) + 1.0 / (hz * hz)));
  return CEFF_OK;
}

ceff_status ceff_create(int device, void* hip_stream, ceff_ctx** out) {
  if (!out) return CEFF_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return CEFF_EDEVICE;
  if (device < 0 || device >= n) return CEFF_EINVAL;
  std::unique_ptr<ceff_ctx> c(new (std::nothrow) ceff_ctx());
  if (!c) return CEFF_ENOMEM;
  c->device = device;
  c->user = static_cast<hipStream_t>(hip_stream);
  if (hipSetDevice(device) != hipSuccess) return CEFF_EDEVICE;
  if (init_scratch(device) != CEFF_OK) return CEFF_EDEVICE;
  if (hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking) != hipSuccess) return CEFF_EDEVICE;
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) return CEFF_EDEVICE;
  *out = c.release();
  return CEFF_OK;
}

void ceff_destroy(ceff_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->s) (void)hipStreamSynchronize(c->s);
  c->K64.reset(); c->G64.reset(); c->K32.reset(); c->G32.reset();
  clear_phases(c);
  clear_ortho(c);
  clear_kept(c);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->s) (void)hipStreamDestroy(c->s);
  delete c;
}

const char* ceff_last_error(const ceff_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

ceff_status ceff_set_grid(ceff_ctx* c, int64_t nx, int64_t ny, int64_t nz, double hx, double hy, double hz) {
  if (!c) return CEFF_EINVAL;
  const double h[3] = {hx, hy, hz};
  STCK(validate_grid(c, nx, ny, nz, h));
  c->nx = nx; c->ny = ny; c->nz = nz;
  c->h[0] = hx; c->h[1] = hy; c->h[2] = hz;
  c->grid_set = true;
  c->have_material = false;
  c->have32 = false;
  c->K64.reset(); c->G64.reset(); c->K32.reset(); c->G32.reset();
  clear_phases(c);
  clear_ortho(c);
  clear_kept(c);
  c->err.clear();
  return CEFF_OK;
}

ceff_status ceff_set_isotropic(ceff_ctx* c, const void* K, const void* G, int dtype, int where) {
  if (!c) return CEFF_EINVAL;
  if (!c->grid_set) return fail(c, CEFF_ESTATE, "set the grid first");
  if (!K || !G) return fail(c, CEFF_EINVAL, "null moduli");
  if (dtype != CEFF_F32 && dtype != CEFF_F64) return fail(c, CEFF_EINVAL, "dtype must be CEFF_F32 or CEFF_F64");
  if (where != CEFF_HOST && where != CEFF_DEVICE) return fail(c, CEFF_EINVAL, "where must be CEFF_HOST or CEFF_DEVICE");
  STCK(begin_call(c));
  const int64_t N = c->nx * c->ny * c->nz;
  c->have_material = false;
  c->have32 = false;
  clear_phases(c);
  clear_ortho(c);
  clear_kept(c);
  STCK(load_moduli(c, K, dtype, where, N, c->K64));
  STCK(load_moduli(c, G, dtype, where, N, c->G64));
  STCK(check_positive(c, c->K64.as<double>(), c->G64.as<double>(), N));
  c->have_material = true;
  return CEFF_OK;
}

ceff_status ceff_set_phases(ceff_ctx* c, const uint8_t* phase, int where, int nphase, const double* K_tab,
                            const double* G_tab) {
  if (!c) return CEFF_EINVAL;
  if (!c->grid_set) return fail(c, CEFF_ESTATE, "set the grid first");
  if (!phase || !K_tab || !G_tab) return fail(c, CEFF_EINVAL, "null argument");
  if (nphase < 1 || nphase > 256) return fail(c, CEFF_EINVAL, "nphase must be in [1, 256]");
  if (where != CEFF_HOST && where != CEFF_DEVICE) return fail(c, CEFF_EINVAL, "where must be CEFF_HOST or CEFF_DEVICE");
  for (int p = 0; p < nphase; ++p)
    if (!(K_tab[p] > 0.0) || !(G_tab[p] > 0.0) || !std::isfinite(K_tab[p]) || !std::isfinite(G_tab[p]))
      return fail(c, CEFF_EINVAL, "phase moduli must be finite and > 0");
  const int64_t N = c->nx * c->ny * c->nz;
  std::vector<uint8_t> host;
  const uint8_t* hp = phase;
  STCK(begin_call(c));
  if (where == CEFF_DEVICE) {
    host.resize(N);
    HIPCK(c, hipMemcpy(host.data(), phase, N, hipMemcpyDeviceToHost));
    hp = host.data();
  }
  for (int64_t t = 0; t < N; ++t)
    if (hp[t] >= nphase) return fail(c, CEFF_EINVAL, "phase id %d at voxel %lld >= nphase", hp[t], (long long)t);
  c->have_material = false;
  c->have32 = false;
  clear_phases(c);
  clear_ortho(c);
  clear_kept(c);
  // the table in both precisions; (float)x rounds as the device conversion of
  // the FP64 fields does, so table and fields hold the same values
  std::vector<double> t64(2 * nphase);
  std::vector<float> t32(2 * nphase);
  for (int p = 0; p < nphase; ++p) {
    t64[p] = K_tab[p];
    t64[nphase + p] = G_tab[p];
  }
  for (int q = 0; q < 2 * nphase; ++q) t32[q] = (float)t64[q];
  HIPCK(c, c->phase8.alloc(N));
  HIPCK(c, hipMemcpyAsync(c->phase8.p, hp, N, hipMemcpyHostToDevice, c->s));
  HIPCK(c, c->ptab64.alloc(sizeof(double) * 2 * nphase));
  HIPCK(c, c->ptab32.alloc(sizeof(float) * 2 * nphase));
  HIPCK(c, hipMemcpyAsync(c->ptab64.p, t64.data(), sizeof(double) * 2 * nphase, hipMemcpyHostToDevice, c->s));
  HIPCK(c, hipMemcpyAsync(c->ptab32.p, t32.data(), sizeof(float) * 2 * nphase, hipMemcpyHostToDevice, c->s));
  HIPCK(c, c->K64.alloc(sizeof(double) * N));
  HIPCK(c, c->G64.alloc(sizeof(double) * N));
  HIPCK(c, launch_phase_to_fields<double>(c->phase8.as<uint8_t>(), N, c->ptab64.as<double>(),
                                          c->ptab64.as<double>() + nphase, nphase, c->K64.as<double>(),
                                          c->G64.as<double>(), c->s));
  HIPCK(c, hipStreamSynchronize(c->s));
  c->nphase = nphase;
  c->have_material = true;
  return CEFF_OK;
}

ceff_status ceff_set_stiffness(ceff_ctx* c, const void* cmat, int ncomp, int dtype, int where) {
  if (!c) return CEFF_EINVAL;
  if (!c->grid_set) return fail(c, CEFF_ESTATE, "set the grid first");
  if (ncomp != 9 && ncomp != 21)
    return fail(c, CEFF_EINVAL, "ncomp must be 9 (orthotropic, axes aligned with the grid) or 21 (general)");
  if (!cmat) return fail(c, CEFF_EINVAL, "null stiffness");
  if (dtype != CEFF_F32 && dtype != CEFF_F64) return fail(c, CEFF_EINVAL, "dtype must be CEFF_F32 or CEFF_F64");
  if (where != CEFF_HOST && where != CEFF_DEVICE) return fail(c, CEFF_EINVAL, "where must be CEFF_HOST or CEFF_DEVICE");
  STCK(begin_call(c));
  const int64_t N = c->nx * c->ny * c->nz;
  c->have_material = false;
  c->have32 = false;
  c->K64.reset(); c->G64.reset(); c->K32.reset(); c->G32.reset();
  clear_phases(c);
  clear_ortho(c);
  clear_kept(c);
  DevBuf& dst = ncomp == 21 ? c->t64 : c->c64;
  STCK(load_moduli(c, cmat, dtype, where, ncomp * N, dst));
  {
    DevBuf bad;
    int nb = 0;
    HIPCK(c, bad.alloc(sizeof(int) * 65536));
    if (ncomp == 21)
      HIPCK(c, launch_check_tri(c->t64.as<double>(), N, bad.as<int>(), &nb, c->s));
    else
      HIPCK(c, launch_check_ortho(c->c64.as<double>(), N, bad.as<int>(), &nb, c->s));
    std::vector<int> h(nb);
    HIPCK(c, hipMemcpyAsync(h.data(), bad.p, sizeof(int) * nb, hipMemcpyDeviceToHost, c->s));
    HIPCK(c, hipStreamSynchronize(c->s));
    for (int v : h)
      if (v) {
        dst.reset();
        return ncomp == 21 ? fail(c, CEFF_EINVAL, "every cell's 21 constants must be finite and form a positive "
                                                  "definite 6x6 matrix")
                           : fail(c, CEFF_EINVAL, "orthotropic constants must be finite, with positive diagonal and "
                                                  "a positive definite normal block");
      }
  }
  if (ncomp == 21) {
    HIPCK(c, c->tse64.alloc(sizeof(double) * 3 * N));
    HIPCK(c, c->tihf64.alloc(sizeof(double) * 3 * N));
    HIPCK(c, launch_tri_setup<double>(c->t64.as<double>(), c->nx, c->ny, c->nz, c->tse64.as<double>(),
                                      c->tihf64.as<double>(), c->s));
    HIPCK(c, hipStreamSynchronize(c->s));
    c->tri = true;
  } else {
    c->ortho = true;
  }
  c->have_material = true;
  return CEFF_OK;
}

ceff_status ceff_set_boundary(ceff_ctx* c, int mode) {
  if (!c) return CEFF_EINVAL;
  if (mode != CEFF_BC_PERIODIC && mode != CEFF_BC_WALLS)
    return fail(c, CEFF_EINVAL, "mode must be CEFF_BC_PERIODIC or CEFF_BC_WALLS");
  c->boundary = mode;
  clear_kept(c);
  c->err.clear();
  return CEFF_OK;
}

ceff_status ceff_solve(ceff_ctx* c, uint32_t load_mask, const ceff_solve_opts* opts, double C_out[36], double* hist,
                       int64_t hist_cap, int64_t* hist_len, int64_t iters_out[6]) {
  if (!c) return CEFF_EINVAL;
  ceff_solve_opts o;
  ceff_default_opts(&o);
  if (opts) o = *opts;
  STCK(validate_opts(c, o));
  if (!C_out) return fail(c, CEFF_EINVAL, "C_out is null");
  if (load_mask == 0 || (load_mask & ~0x3Fu)) return fail(c, CEFF_EINVAL, "load_mask must be a nonzero 6-bit mask");
  if (hist_cap < 0 || (hist_cap > 0 && !hist)) return fail(c, CEFF_EINVAL, "bad history buffer");
  if (!c->grid_set || !c->have_material) return fail(c, CEFF_ESTATE, "set the grid and the material first");
  const bool walls = c->boundary == CEFF_BC_WALLS;
  if (walls && (c->ortho || c->tri)) return fail(c, CEFF_EUNSUPPORTED, "wall boundaries with anisotropic cells");
  if (walls && o.warm_u) return fail(c, CEFF_EUNSUPPORTED, "an initial guess with wall boundaries");
  STCK(begin_call(c));
  const auto t0 = std::chrono::steady_clock::now();
  c->stats = ceff_stats{};
  if (o.keep_fields) clear_kept(c);
  const bool mixed = o.precision == CEFF_PREC_MIXED;
  if (mixed) STCK(ensure32(c));
  std::vector<int> Js;
  for (int J = 0; J < 6; ++J)
    if (load_mask & (1u << J)) Js.push_back(J);
  std::vector<std::array<double, 36>> C(1);
  std::vector<std::array<int64_t, 6>> it(1);
  for (int q = 0; q < 36; ++q) C[0][q] = C_out[q];
  for (int q = 0; q < 6; ++q) it[0][q] = 0;
  std::vector<double> hv;
  ceff_status worst = CEFF_OK;
  std::vector<std::vector<int>> groups;
  // wall tests and general cells run one load at a time
  const bool fuse = !walls && !c->tri && (o.fuse_loads == CEFF_FUSE_AUTO ? fuse_by_cache(c, mixed, (int)Js.size())
                                                                         : o.fuse_loads != 0);
  if (fuse && Js.size() > 1)
    groups.push_back(Js);
  else
    for (int J : Js) groups.push_back({J});
  for (auto& g : groups) {
    const int Lk = g.size() == 1 ? 1 : 6;
    std::vector<SampleIn> s{ctx_sample(c)};
    if (mixed)
      STCK(run_engine<float>(c, s, g, o, Lk, C, it, &hv, o.keep_fields != 0, worst));
    else
      STCK(run_engine<double>(c, s, g, o, Lk, C, it, &hv, o.keep_fields != 0, worst));
  }
  for (int J : Js)
    for (int I = 0; I < 6; ++I) C_out[I * 6 + J] = C[0][I * 6 + J];
  if (iters_out)
    for (int q = 0; q < 6; ++q) iters_out[q] = (load_mask & (1u << q)) ? it[0][q] : 0;
  const int64_t nh = (int64_t)hv.size() / 3;
  if (hist && hist_cap > 0) {
    const int64_t w = std::min(nh, hist_cap);
    std::memcpy(hist, hv.data(), sizeof(double) * 3 * w);
  }
  if (hist_len) *hist_len = nh;
  c->stats.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  c->stats.fused_loads = groups.size() == 1 && Js.size() > 1 ? 1 : 0;
  if (worst != CEFF_OK) return fail(c, worst, worst == CEFF_ENOTCONV ? "max_iter reached" : "iteration diverged");
  return CEFF_OK;
}

ceff_status ceff_solve_batch(ceff_ctx* c, int nsamples, const int64_t* dims, const double* h, const void* const* K,
                             const void* const* G, int dtype, int where, uint32_t load_mask,
                             const ceff_solve_opts* opts, double* C_out, int64_t* iters_out) {
  if (!c) return CEFF_EINVAL;
  ceff_solve_opts o;
  ceff_default_opts(&o);
  if (opts) o = *opts;
  STCK(validate_opts(c, o));
  if (nsamples < 1 || nsamples > 100000) return fail(c, CEFF_EINVAL, "nsamples out of range");
  if (o.warm_u) return fail(c, CEFF_EINVAL, "warm_u applies to ceff_solve only");
  if (!dims || !h || !K || !G || !C_out) return fail(c, CEFF_EINVAL, "null argument");
  if (dtype != CEFF_F32 && dtype != CEFF_F64) return fail(c, CEFF_EINVAL, "dtype must be CEFF_F32 or CEFF_F64");
  if (where != CEFF_HOST && where != CEFF_DEVICE) return fail(c, CEFF_EINVAL, "where must be CEFF_HOST or CEFF_DEVICE");
  if (load_mask == 0 || (load_mask & ~0x3Fu)) return fail(c, CEFF_EINVAL, "load_mask must be a nonzero 6-bit mask");
  for (int s = 0; s < nsamples; ++s) {
    STCK(validate_grid(c, dims[3 * s], dims[3 * s + 1], dims[3 * s + 2], h + 3 * s));
    if (!K[s] || !G[s]) return fail(c, CEFF_EINVAL, "null moduli for sample %d", s);
  }
  STCK(begin_call(c));
  const auto t0 = std::chrono::steady_clock::now();
  c->stats = ceff_stats{};
  const bool mixed = o.precision == CEFF_PREC_MIXED;
  std::vector<DevBuf> K64(nsamples), G64(nsamples), K32(nsamples), G32(nsamples);
  std::vector<SampleIn> in(nsamples);
  for (int s = 0; s < nsamples; ++s) {
    const int64_t N = dims[3 * s] * dims[3 * s + 1] * dims[3 * s + 2];
    STCK(load_moduli(c, K[s], dtype, where, N, K64[s]));
    STCK(load_moduli(c, G[s], dtype, where, N, G64[s]));
    STCK(check_positive(c, K64[s].as<double>(), G64[s].as<double>(), N));
    if (mixed) {
      HIPCK(c, K32[s].alloc(sizeof(float) * N));
      HIPCK(c, G32[s].alloc(sizeof(float) * N));
      HIPCK(c, launch_convert<double, float>(K64[s].as<double>(), K32[s].as<float>(), N, c->s));
      HIPCK(c, launch_convert<double, float>(G64[s].as<double>(), G32[s].as<float>(), N, c->s));
    }
    in[s] = SampleIn{dims[3 * s], dims[3 * s + 1], dims[3 * s + 2], {h[3 * s], h[3 * s + 1], h[3 * s + 2]},
                     K64[s].as<double>(), G64[s].as<double>(), mixed ? K32[s].as<float>() : nullptr,
                     mixed ? G32[s].as<float>() : nullptr};
  }
  std::vector<int> Js;
  for (int J = 0; J < 6; ++J)
    if (load_mask & (1u << J)) Js.push_back(J);
  std::vector<std::array<double, 36>> C(nsamples);
  std::vector<std::array<int64_t, 6>> it(nsamples);
  for (int s = 0; s < nsamples; ++s) {
    for (int q = 0; q < 36; ++q) C[s][q] = C_out[36 * s + q];
    for (int q = 0; q < 6; ++q) it[s][q] = 0;
  }
  ceff_status worst = CEFF_OK;
  const int Lk = Js.size() == 1 ? 1 : 6;
  if (mixed)
    STCK(run_engine<float>(c, in, Js, o, Lk, C, it, nullptr, false, worst));
  else
    STCK(run_engine<double>(c, in, Js, o, Lk, C, it, nullptr, false, worst));
  for (int s = 0; s < nsamples; ++s) {
    for (int J : Js)
      for (int I = 0; I < 6; ++I) C_out[36 * s + I * 6 + J] = C[s][I * 6 + J];
    if (iters_out)
      for (int q = 0; q < 6; ++q) iters_out[6 * s + q] = (load_mask & (1u << q)) ? it[s][q] : 0;
  }
  c->stats.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (worst != CEFF_OK) return fail(c, worst, worst == CEFF_ENOTCONV ? "max_iter reached" : "iteration diverged");
  return CEFF_OK;
}

ceff_status ceff_solve_batch_phases(ceff_ctx* c, int nsamples, const int64_t* dims, const double* h,
                                    const uint8_t* const* phase, int where, int nphase, const double* K_tab,
                                    const double* G_tab, uint32_t load_mask, const ceff_solve_opts* opts,
                                    double* C_out, int64_t* iters_out) {
  if (!c) return CEFF_EINVAL;
  ceff_solve_opts o;
  ceff_default_opts(&o);
  if (opts) o = *opts;
  STCK(validate_opts(c, o));
  if (nsamples < 1 || nsamples > 100000) return fail(c, CEFF_EINVAL, "nsamples out of range");
  if (o.warm_u) return fail(c, CEFF_EINVAL, "warm_u applies to ceff_solve only");
  if (!dims || !h || !phase || !K_tab || !G_tab || !C_out) return fail(c, CEFF_EINVAL, "null argument");
  if (nphase < 1 || nphase > 256) return fail(c, CEFF_EINVAL, "nphase must be in [1, 256]");
  if (where != CEFF_HOST && where != CEFF_DEVICE) return fail(c, CEFF_EINVAL, "where must be CEFF_HOST or CEFF_DEVICE");
  if (load_mask == 0 || (load_mask & ~0x3Fu)) return fail(c, CEFF_EINVAL, "load_mask must be a nonzero 6-bit mask");
  for (int p = 0; p < nphase; ++p)
    if (!(K_tab[p] > 0.0) || !(G_tab[p] > 0.0) || !std::isfinite(K_tab[p]) || !std::isfinite(G_tab[p]))
      return fail(c, CEFF_EINVAL, "phase moduli must be finite and > 0");
  for (int s = 0; s < nsamples; ++s) {
    STCK(validate_grid(c, dims[3 * s], dims[3 * s + 1], dims[3 * s + 2], h + 3 * s));
    if (!phase[s]) return fail(c, CEFF_EINVAL, "null phase image for sample %d", s);
  }
  STCK(begin_call(c));
  const auto t0 = std::chrono::steady_clock::now();
  c->stats = ceff_stats{};
  const bool mixed = o.precision == CEFF_PREC_MIXED;
  // one table for all samples, in both precisions ((float)x rounds as the
  // device conversion of the FP64 fields does)
  std::vector<double> t64(2 * nphase);
  std::vector<float> t32(2 * nphase);
  for (int p = 0; p < nphase; ++p) {
    t64[p] = K_tab[p];
    t64[nphase + p] = G_tab[p];
  }
  for (int q = 0; q < 2 * nphase; ++q) t32[q] = (float)t64[q];
  DevBuf tab64, tab32;
  HIPCK(c, tab64.alloc(sizeof(double) * 2 * nphase));
  HIPCK(c, tab32.alloc(sizeof(float) * 2 * nphase));
  HIPCK(c, hipMemcpyAsync(tab64.p, t64.data(), sizeof(double) * 2 * nphase, hipMemcpyHostToDevice, c->s));
  HIPCK(c, hipMemcpyAsync(tab32.p, t32.data(), sizeof(float) * 2 * nphase, hipMemcpyHostToDevice, c->s));
  std::vector<DevBuf> ph(nsamples), K64(nsamples), G64(nsamples), K32(nsamples), G32(nsamples);
  std::vector<SampleIn> in(nsamples);
  std::vector<uint8_t> host;
  for (int s = 0; s < nsamples; ++s) {
    const int64_t N = dims[3 * s] * dims[3 * s + 1] * dims[3 * s + 2];
    const uint8_t* hp = phase[s];
    if (where == CEFF_DEVICE) {
      host.resize(N);
      HIPCK(c, hipMemcpy(host.data(), phase[s], N, hipMemcpyDeviceToHost));
      hp = host.data();
    }
    for (int64_t t = 0; t < N; ++t)
      if (hp[t] >= nphase)
        return fail(c, CEFF_EINVAL, "sample %d: phase id %d at voxel %lld >= nphase", s, hp[t], (long long)t);
    HIPCK(c, ph[s].alloc(N));
    HIPCK(c, hipMemcpyAsync(ph[s].p, hp, N, hipMemcpyHostToDevice, c->s));
    HIPCK(c, K64[s].alloc(sizeof(double) * N));
    HIPCK(c, G64[s].alloc(sizeof(double) * N));
    HIPCK(c, launch_phase_to_fields<double>(ph[s].as<uint8_t>(), N, tab64.as<double>(), tab64.as<double>() + nphase,
                                            nphase, K64[s].as<double>(), G64[s].as<double>(), c->s));
    if (mixed) {  // FP32 fields for launch shapes that do not read the table
      HIPCK(c, K32[s].alloc(sizeof(float) * N));
      HIPCK(c, G32[s].alloc(sizeof(float) * N));
      HIPCK(c, launch_convert<double, float>(K64[s].as<double>(), K32[s].as<float>(), N, c->s));
      HIPCK(c, launch_convert<double, float>(G64[s].as<double>(), G32[s].as<float>(), N, c->s));
    }
    // the host copy is reused by the next sample: finish this one's upload first
    if (where == CEFF_DEVICE) HIPCK(c, hipStreamSynchronize(c->s));
    in[s] = SampleIn{dims[3 * s], dims[3 * s + 1], dims[3 * s + 2], {h[3 * s], h[3 * s + 1], h[3 * s + 2]},
                     K64[s].as<double>(), G64[s].as<double>(), mixed ? K32[s].as<float>() : nullptr,
                     mixed ? G32[s].as<float>() : nullptr};
    in[s].phase = ph[s].as<uint8_t>();
    in[s].ptab64 = tab64.as<double>();
    in[s].ptab32 = tab32.as<float>();
    in[s].nphase = nphase;
  }
  HIPCK(c, hipStreamSynchronize(c->s));
  std::vector<int> Js;
  for (int J = 0; J < 6; ++J)
    if (load_mask & (1u << J)) Js.push_back(J);
  std::vector<std::array<double, 36>> C(nsamples);
  std::vector<std::array<int64_t, 6>> it(nsamples);
  for (int s = 0; s < nsamples; ++s) {
    for (int q = 0; q < 36; ++q) C[s][q] = C_out[36 * s + q];
    for (int q = 0; q < 6; ++q) it[s][q] = 0;
  }
  ceff_status worst = CEFF_OK;
  const int Lk = Js.size() == 1 ? 1 : 6;
  if (mixed)
    STCK(run_engine<float>(c, in, Js, o, Lk, C, it, nullptr, false, worst));
  else
    STCK(run_engine<double>(c, in, Js, o, Lk, C, it, nullptr, false, worst));
  for (int s = 0; s < nsamples; ++s) {
    for (int J : Js)
      for (int I = 0; I < 6; ++I) C_out[36 * s + I * 6 + J] = C[s][I * 6 + J];
    if (iters_out)
      for (int q = 0; q < 6; ++q) iters_out[6 * s + q] = (load_mask & (1u << q)) ? it[s][q] : 0;
  }
  c->stats.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (worst != CEFF_OK) return fail(c, worst, worst == CEFF_ENOTCONV ? "max_iter reached" : "iteration diverged");
  return CEFF_OK;
}

ceff_status ceff_gradient(ceff_ctx* c, const double W[36], void* dK, void* dG, int dtype, int where) {
  if (!c) return CEFF_EINVAL;
  if (!W || !dK || !dG) return fail(c, CEFF_EINVAL, "null argument");
  if (dtype != CEFF_F32 && dtype != CEFF_F64) return fail(c, CEFF_EINVAL, "dtype must be CEFF_F32 or CEFF_F64");
  if (where != CEFF_HOST && where != CEFF_DEVICE) return fail(c, CEFF_EINVAL, "where must be CEFF_HOST or CEFF_DEVICE");
  for (int q = 0; q < 36; ++q)
    if (!std::isfinite(W[q])) return fail(c, CEFF_EINVAL, "W must be finite");
  if (!c->grid_set || !c->have_material) return fail(c, CEFF_ESTATE, "set the grid and the material first");
  if (c->ortho || c->tri)
    return fail(c, CEFF_EUNSUPPORTED, "the gradient is defined for isotropic (K, G) materials only");
  if (c->boundary != CEFF_BC_PERIODIC) return fail(c, CEFF_EUNSUPPORTED, "the gradient needs periodic boundaries");
  GradLoads g{};
  for (int q = 0; q < 36; ++q) g.W[q] = W[q];
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J)
      if (W[I * 6 + J] != 0.0) {
        if (!c->kept[I] || !c->kept[J])
          return fail(c, CEFF_ESTATE, "gradient needs the fields of loads %d and %d (solve with keep_fields=1)", I, J);
        g.u[I] = c->keep[I].as<double>();
        g.u[J] = c->keep[J].as<double>();
      }
  STCK(begin_call(c));
  const int64_t N = c->nx * c->ny * c->nz;
  DevBuf oK, oG;
  const size_t es = dtype == CEFF_F64 ? sizeof(double) : sizeof(float);
  void* tK = dK;
  void* tG = dG;
  if (where == CEFF_HOST) {
    HIPCK(c, oK.alloc(es * N));
    HIPCK(c, oG.alloc(es * N));
    tK = oK.p;
    tG = oG.p;
  }
  if (dtype == CEFF_F64)
    HIPCK(c, launch_gradient<double>(c->nx, c->ny, c->nz, c->h, c->K64.as<double>(), c->G64.as<double>(),
                                     g, (double*)tK, (double*)tG, c->s));
  else
    HIPCK(c, launch_gradient<float>(c->nx, c->ny, c->nz, c->h, c->K64.as<double>(), c->G64.as<double>(),
                                    g, (float*)tK, (float*)tG, c->s));
  if (where == CEFF_HOST) {
    HIPCK(c, hipMemcpyAsync(dK, tK, es * N, hipMemcpyDeviceToHost, c->s));
    HIPCK(c, hipMemcpyAsync(dG, tG, es * N, hipMemcpyDeviceToHost, c->s));
  }
  HIPCK(c, hipStreamSynchronize(c->s));
  return CEFF_OK;
}

ceff_status ceff_apt_steps(ceff_ctx* c, int J, int64_t nsteps, int precision, double courant, double strouhal,
                           double* u_out, double* u_prev_out) {
  if (!c) return CEFF_EINVAL;
  if (J < 0 || J > 5) return fail(c, CEFF_EINVAL, "load index must be in [0, 5]");
  if (nsteps < 1 || nsteps > 100000000) return fail(c, CEFF_EINVAL, "nsteps out of range");
  if (precision != CEFF_PREC_FP64 && precision != CEFF_PREC_MIXED) return fail(c, CEFF_EINVAL, "bad precision");
  if (!(courant > 0.0) || !(courant <= 1.0) || !(strouhal >= 0.0) || !std::isfinite(strouhal))
    return fail(c, CEFF_EINVAL, "bad parameters");
  if (!u_out) return fail(c, CEFF_EINVAL, "u_out is null");
  if (!c->grid_set || !c->have_material) return fail(c, CEFF_ESTATE, "set the grid and the material first");
  STCK(check_walls_material(c));
  STCK(begin_call(c));
  ceff_solve_opts o;
  ceff_default_opts(&o);
  o.courant = courant;
  o.strouhal = strouhal;
  o.use_graph = 0;
  const int64_t N = c->nx * c->ny * c->nz;
  auto run = [&](auto tag) -> ceff_status {
    using T = decltype(tag);
    Engine<T> e;
    e.c = c;
    e.in = {ctx_sample(c)};
    e.o = o;
    e.mixed = false;
    e.Lk = 1;
    e.Js = {J};
    STCK(e.setup());
    c->stats = ceff_stats{};
    record_shape(c, e);
    e.h_in[0].active = 1u;
    STCK(e.upload_desc());
    e.parity = 0;
    HIPCK(c, e.step(1, nullptr));
    e.parity = 1;
    int64_t q = 1;
    if (e.ts.tb)
      for (; q + 2 <= nsteps; q += 2) {
        HIPCK(c, e.step_pair(nullptr));
        e.parity = e.after_pair(e.parity);
      }
    for (; q < nsteps; ++q) {
      HIPCK(c, e.step(0, nullptr));
      e.parity ^= 1;
    }
    DevBuf tmp;
    HIPCK(c, tmp.alloc(sizeof(double) * 3 * N));
    for (int which = 0; which < 2; ++which) {
      double* dst = which == 0 ? u_out : u_prev_out;
      if (!dst) continue;
      const T* src = e.h_in[0].u[which == 0 ? e.parity : e.parity ^ 1][0];
      if (sizeof(T) == 8)
        HIPCK(c, hipMemcpyAsync(tmp.p, src, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, c->s));
      else
        HIPCK(c, launch_convert<float, double>((const float*)src, tmp.as<double>(), 3 * N, c->s));
      HIPCK(c, hipMemcpyAsync(dst, tmp.p, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, c->s));
      HIPCK(c, hipStreamSynchronize(c->s));
    }
    return CEFF_OK;
  };
  if (precision == CEFF_PREC_MIXED) {
    STCK(ensure32(c));
    return run(float{});
  }
  return run(double{});
}

ceff_status ceff_residual(ceff_ctx* c, int J, int precision, const double* u, double* r_out, double* norm2) {
  if (!c) return CEFF_EINVAL;
  if (J < 0 || J > 5) return fail(c, CEFF_EINVAL, "load index must be in [0, 5]");
  if (precision != CEFF_PREC_FP64 && precision != CEFF_PREC_MIXED) return fail(c, CEFF_EINVAL, "bad precision");
  if (!u) return fail(c, CEFF_EINVAL, "u is null");
  if (!c->grid_set || !c->have_material) return fail(c, CEFF_ESTATE, "set the grid and the material first");
  STCK(check_walls_material(c));
  STCK(begin_call(c));
  const int64_t N = c->nx * c->ny * c->nz;
  ceff_solve_opts o;
  ceff_default_opts(&o);
  auto run = [&](auto tag) -> ceff_status {
    using T = decltype(tag);
    Engine<T> e;
    e.c = c;
    e.in = {ctx_sample(c)};
    e.o = o;
    e.mixed = false;
    e.Lk = 1;
    e.Js = {J};
    STCK(e.setup());
    DevBuf d64, r, rp, part, nrm;
    HIPCK(c, d64.alloc(sizeof(double) * 3 * N));
    HIPCK(c, hipMemcpyAsync(d64.p, u, sizeof(double) * 3 * N, hipMemcpyHostToDevice, c->s));
    if (sizeof(T) == 8)
      HIPCK(c, hipMemcpyAsync(e.h_in[0].u[0][0], d64.p, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, c->s));
    else
      HIPCK(c, launch_convert<double, float>(d64.as<double>(), (float*)e.h_in[0].u[0][0], 3 * N, c->s));
    e.h_in[0].active = 1u;
    STCK(e.upload_desc());
    HIPCK(c, r.alloc(sizeof(T) * 3 * N));
    T* rptr[1] = {r.as<T>()};
    HIPCK(c, rp.alloc(sizeof rptr));
    HIPCK(c, hipMemcpyAsync(rp.p, rptr, sizeof rptr, hipMemcpyHostToDevice, c->s));
    if (e.ts.ortho)
      HIPCK(c, launch_residual_ortho<T, T>(e.d_in.template as<SampleDesc<T>>(), e.d_work.template as<WorkItem>(),
                                           (int)e.work.size(), e.ts, 0, rp.as<T*>(),
                                           e.d_partials.template as<double>(), c->s));
    else if (e.ts.tri)
      HIPCK(c, launch_residual_tri<T, T>(e.d_in.template as<SampleDesc<T>>(), N, (int)e.work.size(), 0, rp.as<T*>(),
                                         e.d_partials.template as<double>(), c->s));
    else
      HIPCK(c, launch_residual<T, T, 1>(e.d_in.template as<SampleDesc<T>>(), e.d_work.template as<WorkItem>(),
                                        (int)e.work.size(), e.ts, 0, rp.as<T*>(), e.d_partials.template as<double>(),
                                        c->s));
    HIPCK(c, launch_finalize_norms(e.d_ranges.template as<int>(), 1, e.d_partials.template as<double>(),
                                   e.d_norms.template as<double>(), c->s));
    double nn[kMaxLoads];
    HIPCK(c, hipMemcpyAsync(nn, e.d_norms.p, sizeof nn, hipMemcpyDeviceToHost, c->s));
    if (r_out) {
      if (sizeof(T) == 8)
        HIPCK(c, hipMemcpyAsync(d64.p, r.p, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, c->s));
      else
        HIPCK(c, launch_convert<float, double>((const float*)r.p, d64.as<double>(), 3 * N, c->s));
      HIPCK(c, hipMemcpyAsync(r_out, d64.p, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, c->s));
    }
    HIPCK(c, hipStreamSynchronize(c->s));
    if (norm2) *norm2 = nn[0];
    return CEFF_OK;
  };
  if (precision == CEFF_PREC_MIXED) {
    STCK(ensure32(c));
    return run(float{});
  }
  return run(double{});
}

ceff_status ceff_average_stress(ceff_ctx* c, int J, const double* u, double out6[6]) {
  if (!c) return CEFF_EINVAL;
  if (J < 0 || J > 5) return fail(c, CEFF_EINVAL, "load index must be in [0, 5]");
  if (!u || !out6) return fail(c, CEFF_EINVAL, "null argument");
  if (!c->grid_set || !c->have_material) return fail(c, CEFF_ESTATE, "set the grid and the material first");
  STCK(check_walls_material(c));
  STCK(begin_call(c));
  const int64_t N = c->nx * c->ny * c->nz;
  DevBuf d;
  HIPCK(c, d.alloc(sizeof(double) * 3 * N));
  HIPCK(c, hipMemcpyAsync(d.p, u, sizeof(double) * 3 * N, hipMemcpyHostToDevice, c->s));
  return stress_average(c, ctx_sample(c), J, d.as<double>(), out6);
}

ceff_status ceff_average_stress_noalloc(ceff_ctx* c, int J, const double* u, double out6[6]) {
  if (!c) return CEFF_EINVAL;
  if (J < 0 || J > 5) return fail(c, CEFF_EINVAL, "load index must be in [0, 5]");
  if (!u || !out6) return fail(c, CEFF_EINVAL, "null argument");
  if (!c->grid_set || !c->have_material) return fail(c, CEFF_ESTATE, "set the grid and the material first");
  if (c->tri) return fail(c, CEFF_EUNSUPPORTED, "general anisotropic cells need field-sized scratch");
  double* sc = scratch_addr(c->device);
  if (!sc) return fail(c, CEFF_EDEVICE, "no scratch address for device %d", c->device);
  STCK(begin_call(c));
  // partials of at most kAvgBlocks blocks, then the six sums: the whole scratch, for any grid
  return stress_average_into(c, ctx_sample(c), J, u, sc, kAvgBlocks, sc + 6 * kAvgBlocks, out6);
}

ceff_status ceff_get_stats(const ceff_ctx* c, ceff_stats* out) {
  if (!c || !out) return CEFF_EINVAL;
  *out = c->stats;
  return CEFF_OK;
}

ceff_status ceff_contribution_tensors(const double C_eff[36], const double C_host[36], double phi, double H_out[36],
                                      double N_out[36]) {
  if (!C_eff || !C_host) return CEFF_EINVAL;
  if (!(phi > 0.0) || !(phi <= 1.0)) return CEFF_EINVAL;
  for (int q = 0; q < 36; ++q)
    if (!std::isfinite(C_eff[q]) || !std::isfinite(C_host[q])) return CEFF_EINVAL;
  if (H_out) {
    double Se[36], Sh[36];
    if (!invert6(C_eff, Se) || !invert6(C_host, Sh)) return CEFF_EINVAL;
    for (int q = 0; q < 36; ++q) H_out[q] = (Se[q] - Sh[q]) / phi;
  }
  if (N_out)
    for (int q = 0; q < 36; ++q) N_out[q] = (C_eff[q] - C_host[q]) / phi;
  return CEFF_OK;
}

ceff_status ceff_triaxial_offdiagonals(const double sig_mean[3], const double eps_mean[3], const double C_diag[3],
                                       double out[3]) {
  if (!sig_mean || !eps_mean || !C_diag || !out) return CEFF_EINVAL;
  double sb[3], eb[3];
  for (int d = 0; d < 3; ++d) {
    if (!std::isfinite(sig_mean[d]) || !std::isfinite(eps_mean[d]) || !std::isfinite(C_diag[d]) ||
        eps_mean[d] == 0.0)
      return CEFF_EINVAL;
    eb[d] = eps_mean[d];
    sb[d] = sig_mean[d] - C_diag[d] * eps_mean[d];
  }
  // each combination below isolates one unknown of the three equations
  out[0] = (eb[0] * sb[0] + eb[1] * sb[1] - eb[2] * sb[2]) / (2.0 * eb[0] * eb[1]);
  out[1] = (eb[0] * sb[0] - eb[1] * sb[1] + eb[2] * sb[2]) / (2.0 * eb[0] * eb[2]);
  out[2] = (-eb[0] * sb[0] + eb[1] * sb[1] + eb[2] * sb[2]) / (2.0 * eb[1] * eb[2]);
  return CEFF_OK;
}

ceff_status ceff_triaxial_from_walls(const double C_walls[36], double out[3]) {
  if (!C_walls || !out) return CEFF_EINVAL;
  double sig[3], eps[3] = {1.0, 1.0, 1.0}, diag[3];
  for (int i = 0; i < 3; ++i) {
    // row i of the triaxial test: the sum of the three normal wall columns
    sig[i] = C_walls[i * 6 + 0] + C_walls[i * 6 + 1] + C_walls[i * 6 + 2];
    diag[i] = C_walls[i * 6 + i];
  }
  return ceff_triaxial_offdiagonals(sig, eps, diag, out);
}

}  // extern "C"
