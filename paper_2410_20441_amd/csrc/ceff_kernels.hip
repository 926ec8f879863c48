// HIP kernels for gfx950 (MI355X): periodic staggered-grid elasticity on a voxel
// grid, iterated with the accelerated pseudo-transient (APT) method of the
// paper ("Numerical solution strategy").
//
// The paper updates pressure p, deviator tau and velocity v.  With unit
// physical time step and pseudo moduli equal to the local moduli (K~ = K,
// G~ = G), the pressure and deviator relaxations share one factor 1/(1+c),
// so the stress is an exponential average of Hooke's stress of the current
// iterate, and eliminating it gives an equivalent two-level recurrence on the
// displacement alone:
//
//     u^{n+1} = u^n + a (u^n - u^{n-1}) + (s / H_f) div( C : (E + grad u^n) ),
//     a = 1/(1+c),  s = c/(1+c) * ell*Lx/St,  c = ell*St/Lx,
//
// with the first step u^1 = (ell*Lx/St / H_f) div(C:E).  This is what runs
// here: it is the same iterate sequence (to rounding) with 2 displacement
// buffers instead of 9 stress/velocity fields in ping-pong pairs, so each
// voxel-update reads u^n (with its halo) and u^{n-1} and writes u^{n+1} in
// place of u^{n-1}: 9 words of state traffic instead of 18.
//
// Step kernel layout: a block covers a (bx-2) x (by-2) tile of one z-range
// plus a one-cell ring of ghost threads, and marches up the z-range one plane
// at a time.  Every thread loads its own column's u and moduli; the in-plane
// neighbours come through LDS; the z neighbours stay in registers.  Stresses
// are computed once per node by the thread that owns the node (ghost threads
// compute the halo nodes the tile needs).  Several loads share one launch: the
// moduli and the derived edge/face coefficients are read once per plane for
// all of them.  The residual norm is fused into the sweep on check iterations.
#include "ceff_internal.h"

#include <type_traits>

// The build compiles this file several times, with CEFF_KPART = 0, 1, 2, 3, in
// parallel; each compilation emits one share of the launch wrappers (0: all but
// the iteration kernels, 1: FP32 iteration with 1 or 2 loads per block, 2: FP32
// with 3 or 6, 3: FP64).  Without CEFF_KPART one compilation emits everything.
#ifndef CEFF_KPART
#define CEFF_KPART -1
#endif
#define CEFF_IN_PART(n) (CEFF_KPART < 0 || CEFF_KPART == (n))

namespace ceff {

namespace {

// Pointers read from descriptor tables are generic; without this cast the
// compiler emits FLAT accesses, which also count against the LDS wait counter,
// so every LDS barrier would wait for all outstanding global loads.
#define GLOBAL_AS __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const GLOBAL_AS T* gconst(const T* p) {
  return (const GLOBAL_AS T*)p;
}
template <typename T>
__device__ __forceinline__ GLOBAL_AS T* gmut(T* p) {
  return (GLOBAL_AS T*)p;
}

__device__ __forceinline__ int64_t wrap_idx(int64_t a, int64_t n) {
  a %= n;
  return a < 0 ? a + n : a;
}

template <typename T>
__device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }

// Sum of v over the block; the result is valid on thread 0.  Fixed order
// (wave shuffle tree, then waves in index order) so it is deterministic.
__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

// MODE 0: heavy-ball update; MODE 1: write the residual to rout.
// L: loads handled by one block (slots [slot0, slot0+L) of its work item).
// PF: prefetch the next plane's global data into registers while the current
// plane is processed.
template <typename T>
__device__ __forceinline__ T recip(T x) {
  return T(1) / x;
}
// FP32 sweeps use the hardware reciprocal (1 ulp); FP64 keeps exact division
template <>
__device__ __forceinline__ float recip<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// Minimum waves per SIMD the compiler must allow (it caps registers to fit):
// the FP32 kernels with up to two loads per block, and the FP64 one-load
// kernel, are held to 128 VGPRs so that two 512-thread blocks share a CU.
// HI selects the high-occupancy build (more waves per SIMD, fewer registers,
// possibly some spills); the tuner measures both.
template <typename T, int L, bool HI>
struct MinWaves {
  static constexpr int hi = sizeof(T) == 4 ? (L == 1 ? 6 : (L == 2 ? 6 : (L == 3 ? 4 : 1))) : (L == 1 ? 5 : 1);
  static constexpr int lo = (sizeof(T) == 4 && L <= 2) || (sizeof(T) == 8 && L == 1) ? 4 : 1;
  static constexpr int value = HI ? hi : lo;
};

// Per-cell coefficients of the isotropic Hooke law on the staggered grid:
// lambda = K - 2G/3 and 2G for the normal stresses, 1/H with H = K + 4G/3 for
// the face step (the step of a face takes the smaller 1/H of its two cells,
// i.e. 1/max H), and 1/(8G) for the harmonic edge moduli (twice the harmonic
// mean of four cells is 1 / (sum of their 1/(8G)); the factor is a power of two,
// so this is exactly 8 / (sum of 1/G)).
template <typename T>
struct alignas(16) CellCoef {
  T lam, twoG, iH, iG8;
};

template <typename T>
__device__ __forceinline__ CellCoef<T> cell_coef(T K, T G) {
  CellCoef<T> c;
  c.lam = K - T(2.0 / 3.0) * G;
  c.twoG = T(2) * G;
  c.iH = recip(K + T(4.0 / 3.0) * G);
  c.iG8 = T(0.125) * recip(G);
  return c;
}

// Minimum of two positive finite values.  For FP32 the bit patterns of
// positive floats order like unsigned integers: one v_min_u32.
__device__ __forceinline__ float tmin(float a, float b) {
  return __builtin_bit_cast(float, __builtin_elementwise_min(__builtin_bit_cast(unsigned int, a),
                                                             __builtin_bit_cast(unsigned int, b)));
}
__device__ __forceinline__ double tmin(double a, double b) { return __builtin_fmin(a, b); }

// Raw buffer view of one z-plane of one field component: the descriptor (base
// address of the component's plane, byte range of one plane) is formed on the
// scalar unit from uniform values, and an access takes the thread's 32-bit byte
// offset of its column within the plane.  The vector ALU then does no address
// arithmetic, and no offset spans more than one plane (the host keeps a plane
// below 2 GiB), whatever the size of the field.  Reads outside the plane's
// range return 0.
struct PlaneBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ PlaneBuf(const void* p, uint32_t bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000)) {}
  __device__ __forceinline__ float ldf(uint32_t v) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)v, 0, 0));
  }
  __device__ __forceinline__ double ldd(uint32_t v) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)v, 0, 0));
  }
  __device__ __forceinline__ uint32_t ldb(uint32_t v) const {
    return __builtin_amdgcn_raw_buffer_load_b8(r, (int)v, 0, 0);
  }
  __device__ __forceinline__ void st(uint32_t v, float x) const {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, (int)v, 0, 0);
  }
  __device__ __forceinline__ void st(uint32_t v, double x) const {
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, x), r, (int)v, 0, 0);
  }
  template <typename T>
  __device__ __forceinline__ T ld(uint32_t v) const {
    if constexpr (sizeof(T) == 4)
      return ldf(v);
    else
      return ldd(v);
  }
};

// Where the iteration kernel gets a cell's coefficients.  load() issues the
// global read (so it can be requested a plane ahead), coef() turns what it
// returned into coefficients.  PAL = false: from the K and G fields (2 words per
// cell).  PAL = true: from the 1-byte phase id and a per-phase coefficient table
// staged in LDS; the table entries come from the same cell_coef on the same
// values, so both give identical results.  pk: element offset of the z-plane;
// col, colb: the column's element and byte offset within it.
template <typename T, bool PAL>
struct Moduli {
  struct Raw {
    T K, G;
  };
  const T* Kf;
  const T* Gf;
  uint32_t pbytes;  // bytes of one plane of K (or G)
  __device__ Moduli(const SampleDesc<T>& sd, const CellCoef<T>*)
      : Kf(sd.K), Gf(sd.G), pbytes((uint32_t)(sd.nx * sd.ny * (int64_t)sizeof(T))) {}
  __device__ __forceinline__ Raw load(int64_t pk, uint32_t col, uint32_t colb) const {
    (void)col;
    return Raw{PlaneBuf(Kf + pk, pbytes).template ld<T>(colb), PlaneBuf(Gf + pk, pbytes).template ld<T>(colb)};
  }
  __device__ __forceinline__ CellCoef<T> coef(Raw r) const { return cell_coef(r.K, r.G); }
};

template <typename T>
struct Moduli<T, true> {
  struct Raw {
    uint32_t p;
  };
  const uint8_t* ph;
  const CellCoef<T>* tab;
  uint32_t pbytes;  // bytes of one plane of the phase image
  __device__ Moduli(const SampleDesc<T>& sd, const CellCoef<T>* t)
      : ph(sd.phase), tab(t), pbytes((uint32_t)(sd.nx * sd.ny)) {}
  __device__ __forceinline__ Raw load(int64_t pk, uint32_t col, uint32_t colb) const {
    (void)colb;
    return Raw{PlaneBuf(ph + pk, pbytes).ldb(col)};
  }
  __device__ __forceinline__ CellCoef<T> coef(Raw r) const { return tab[r.p]; }
};

// Fill the 256-entry LDS coefficient table of the launch's phase table (ids
// beyond nphase get a harmless unit entry; the host has checked every id).
template <typename T>
__device__ void stage_coef_table(const SampleDesc<T>& sd, CellCoef<T>* tab) {
  for (int i = threadIdx.x; i < 256; i += blockDim.x)
    tab[i] = i < sd.nphase ? cell_coef(sd.ptab[i], sd.ptab[sd.nphase + i]) : cell_coef(T(1), T(1));
  __syncthreads();
}

template <typename T, int L, int MODE, typename R, bool PF, bool HI, bool WALLS = false>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 512), amdgpu_waves_per_eu(MinWaves<T, L, HI>::value)))
step_kernel(const SampleDesc<T>* __restrict__ samples,
                                                   const WorkItem* __restrict__ work, int nwork, int bx, int by,
                                                   int parity, int first, double* __restrict__ partials,
                                                   R* const* __restrict__ rout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int nt = blockDim.x;  // multiple of 64, >= bx*by
  T* sG0 = reinterpret_cast<T*>(smem_raw);
  T* sG1 = sG0 + nt;
  T* sH = sG1 + nt;
  T* sUx = sH + nt;
  T* sUy = sUx + nt;
  T* sUz = sUy + nt;
  T* sSxx = sUz + nt;
  T* sSyy = sSxx + nt;
  T* sSxy = sSyy + nt;
  T* sSxz = sSxy + nt;
  T* sSyz = sSxz + nt;

  const int tid = threadIdx.x;
  const int tx = tid % bx, ty = tid / bx;
  const int TX = bx - 2, TY = by - 2;
  // LDS neighbours, clamped inside the block (values at clamped ghost
  // positions are never consumed by interior threads)
  const int xm = tid > 0 && tx > 0 ? tid - 1 : tid;
  const int xp = tx < bx - 1 && tid + 1 < nt ? tid + 1 : tid;
  const int ym = ty > 0 ? tid - bx : tid;
  const int yp = ty < by - 1 && tid + bx < nt ? tid + bx : tid;
  const int xmym = ty > 0 ? xm - bx : xm;

  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const WorkItem wi = work[w];
    if (wi.sample < 0) {  // padding of the XCD-aware order
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      continue;
    }
    const SampleDesc<T>& sd = samples[wi.sample];
    const int s0 = wi.slot0;
    const unsigned act = (sd.active >> s0) & ((1u << L) - 1u);
    if (act == 0u) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      continue;  // uniform over the block
    }
    const int64_t nx = sd.nx, ny = sd.ny, nz = sd.nz, N = sd.N, plane = nx * ny;
    const T rhx = sd.rhx, rhy = sd.rhy, rhz = sd.rhz;
    const T mom = first ? T(0) : sd.mom;
    const T sfac = first ? sd.sfac_first : sd.sfac;
    const int64_t gi = (int64_t)wi.tx * TX + tx - 1, gj = (int64_t)wi.ty * TY + ty - 1;
    const int64_t col = wrap_idx(gi, nx) + nx * wrap_idx(gj, ny);
    const bool interior = tx >= 1 && tx <= TX && ty >= 1 && ty <= TY && gi < nx && gj < ny;
    const int64_t k0 = (int64_t)wi.kz * sd.kc;
    const int64_t k1 = k0 + sd.kc < nz ? k0 + sd.kc : nz;
    // wall boundaries: this column lies in the x (y) boundary plane; wsh: the
    // Voigt shear component whose simple-shear test this load is (0: none)
    const bool wx = WALLS && wrap_idx(gi, nx) == 0, wy = WALLS && wrap_idx(gj, ny) == 0;
    const int wsh = WALLS ? sd.wshear[s0] : 0;

    const GLOBAL_AS T* __restrict__ Kf = gconst(sd.K);
    const GLOBAL_AS T* __restrict__ Gf = gconst(sd.G);
    const GLOBAL_AS T* ucur[L];
    GLOBAL_AS T* uold[L];
    const GLOBAL_AS T* frc[L];
    bool hasf[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      ucur[l] = gconst(sd.u[parity][s0 + l]);
      uold[l] = gmut(sd.u[parity ^ 1][s0 + l]);
      hasf[l] = sd.force[s0 + l] != nullptr;
      frc[l] = gconst(sd.force[s0 + l]);
    }

    // registers carried up the z-march, per load
    T ux[L], uy[L], uz[L], szz_p[L], sxz_c[L], syz_c[L];
    double nsum[L];
    {
      const int64_t kw = k0 - 1 < 0 ? k0 - 1 + nz : k0 - 1;
      const int64_t o = col + plane * kw;
#pragma unroll
      for (int l = 0; l < L; ++l) {
        if (act & (1u << l)) {
          ux[l] = ucur[l][o];
          uy[l] = ucur[l][N + o];
          uz[l] = ucur[l][2 * N + o];
        } else {
          ux[l] = uy[l] = uz[l] = T(0);
        }
        szz_p[l] = sxz_c[l] = syz_c[l] = T(0);
        nsum[l] = 0.0;
      }
    }
    T Kc = Kf[col + plane * (k0 - 1 < 0 ? k0 - 1 + nz : k0 - 1)];
    T Gc = Gf[col + plane * (k0 - 1 < 0 ? k0 - 1 + nz : k0 - 1)];
    T Hprev = T(1);
    sG0[tid] = Gc;

    // global data consumed while processing plane k: moduli and u^n at plane
    // k+1, u^{n-1} and the body force at plane k
    T Kn, Gn, unx[L], uny[L], unz[L], uo0[L], uo1[L], uo2[L], f0[L], f1[L], f2[L];
    T pK, pG, pux[L], puy[L], puz[L], po0[L], po1[L], po2[L], pf0[L], pf1[L], pf2[L];
    auto fetch = [&](int64_t k, T& K_, T& G_, T* ax, T* ay, T* az, T* b0, T* b1, T* b2, T* c0, T* c1, T* c2) {
      const int64_t kw = k < 0 ? k + nz : k;
      const int64_t kn = k + 1 >= nz ? k + 1 - nz : k + 1;
      const int64_t oc = col + plane * kw, on = col + plane * kn;
      const bool face = k >= k0 && interior;
      K_ = Kf[on];
      G_ = Gf[on];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        ax[l] = ay[l] = az[l] = b0[l] = b1[l] = b2[l] = c0[l] = c1[l] = c2[l] = T(0);
        if (act & (1u << l)) {
          ax[l] = ucur[l][on];
          ay[l] = ucur[l][N + on];
          az[l] = ucur[l][2 * N + on];
          if (face) {
            if (MODE == 0 && !first) {
              b0[l] = uold[l][oc];
              b1[l] = uold[l][N + oc];
              b2[l] = uold[l][2 * N + oc];
            }
            if (hasf[l]) {
              c0[l] = frc[l][oc];
              c1[l] = frc[l][N + oc];
              c2[l] = frc[l][2 * N + oc];
            }
          }
        }
      }
    };
    if (PF) fetch(k0 - 1, pK, pG, pux, puy, puz, po0, po1, po2, pf0, pf1, pf2);

    for (int64_t k = k0 - 1; k < k1; ++k) {
      const int rel = (int)(k - (k0 - 1));
      const int64_t kw = k < 0 ? k + nz : k;
      const int64_t oc = col + plane * kw;
      const bool face = k >= k0 && interior;

      if (PF) {
        Kn = pK;
        Gn = pG;
#pragma unroll
        for (int l = 0; l < L; ++l) {
          unx[l] = pux[l]; uny[l] = puy[l]; unz[l] = puz[l];
          uo0[l] = po0[l]; uo1[l] = po1[l]; uo2[l] = po2[l];
          f0[l] = pf0[l]; f1[l] = pf1[l]; f2[l] = pf2[l];
        }
        if (k + 1 < k1) fetch(k + 1, pK, pG, pux, puy, puz, po0, po1, po2, pf0, pf1, pf2);
      } else {
        fetch(k, Kn, Gn, unx, uny, unz, uo0, uo1, uo2, f0, f1, f2);
      }

      T* gk = (rel & 1) ? sG1 : sG0;   // plane k
      T* gn = (rel & 1) ? sG0 : sG1;   // plane k+1
      gn[tid] = Gn;
      const T Hk = Kc + T(4.0 / 3.0) * Gc;
      sH[tid] = Hk;

      // per-plane coefficients shared by all loads: edge shear moduli (harmonic
      // mean of the four cells around the edge, times two), Lame lambda, 2G
      // and the face step factors; computed after the first barrier
      T G2xy = T(0), G2xz = T(0), G2yz = T(0), sfx = T(0), sfy = T(0), sfz = T(0);
      const T lam = Kc - T(2.0 / 3.0) * Gc;
      const T twoG = T(2) * Gc;
      bool coef = false;
#pragma unroll
      for (int l = 0; l < L; ++l) {
        if (!(act & (1u << l))) continue;
        sUx[tid] = ux[l];
        sUy[tid] = uy[l];
        sUz[tid] = unz[l];
        __syncthreads();
        if (!coef) {
          const T ik = recip(gk[tid]), ikx = recip(gk[xm]), iky = recip(gk[ym]);
          const T in = recip(gn[tid]), inx = recip(gn[xm]), iny = recip(gn[ym]);
          G2xy = T(8) * recip(recip(gk[xmym]) + iky + ikx + ik);
          G2xz = T(8) * recip(ikx + ik + inx + in);
          G2yz = T(8) * recip(iky + ik + iny + in);
          sfx = sfac * recip(tmax(sH[xm], Hk));
          sfy = sfac * recip(tmax(sH[ym], Hk));
          sfz = sfac * recip(tmax(Hprev, Hk));
          coef = true;
        }
        const T* E = sd.E[s0 + l];
        // stresses owned by this thread: cell (k), xy-edge (k), xz/yz-edges (k+1)
        const T exx = E[0] + (sUx[xp] - ux[l]) * rhx;
        const T eyy = E[1] + (sUy[yp] - uy[l]) * rhy;
        const T ezz = E[2] + (unz[l] - uz[l]) * rhz;
        const T th = exx + eyy + ezz;
        const T sxx = lam * th + twoG * exx;
        const T syy = lam * th + twoG * eyy;
        const T szz = lam * th + twoG * ezz;
        T sxy = G2xy * (E[5] + T(0.5) * ((ux[l] - sUx[ym]) * rhy + (uy[l] - sUy[xm]) * rhx));
        T sxz_n = G2xz * (E[4] + T(0.5) * ((unx[l] - ux[l]) * rhz + (unz[l] - sUz[xm]) * rhx));
        T syz_n = G2yz * (E[3] + T(0.5) * ((uny[l] - uy[l]) * rhz + (unz[l] - sUz[ym]) * rhy));
        // published xy-edge stress and carried xz/yz-edge stresses (they differ
        // from the thread's own only at the split edges of a simple-shear test)
        T sxy_s = sxy, sxz_k = sxz_n, syz_k = syz_n;
        if constexpr (WALLS) {
          // free-slip boundary edges, the simple-shear test's own component
          // computed as inside on the walls normal to the sheared direction and
          // split into one half per side on the loaded walls (one-sided
          // derivative to the wall, harmonic mean of the half's two cells:
          // 2 G = 4 / (1/G + 1/G'))
          const bool wzn = k + 1 == nz || k + 1 == 0;  // xz/yz-edges owned here sit between k and k+1
          if ((wx || wy) && wsh != 5) sxy = T(0);
          if ((wx || wzn) && wsh != 4) sxz_n = T(0);
          if ((wy || wzn) && wsh != 3) syz_n = T(0);
          sxy_s = sxy;
          sxz_k = sxz_n;
          syz_k = syz_n;
          if (wsh == 5 && wy) {  // own half in the cells j = 0, published half in j = ny - 1
            const T t = T(0.5) * (uy[l] - sUy[xm]) * rhx;
            sxy = T(4) * recip(recip(gk[tid]) + recip(gk[xm])) * (E[5] + ux[l] * rhy + t);
            sxy_s = T(4) * recip(recip(gk[ym]) + recip(gk[xmym])) * (E[5] - sUx[ym] * rhy + t);
          }
          if (wsh == 4 && wzn) {  // upper edge of plane nz - 1, carried as the lower edge of plane 0
            const T t = T(0.5) * (unz[l] - sUz[xm]) * rhx;
            sxz_n = T(4) * recip(recip(gk[tid]) + recip(gk[xm])) * (E[4] - ux[l] * rhz + t);
            sxz_k = T(4) * recip(recip(gn[tid]) + recip(gn[xm])) * (E[4] + unx[l] * rhz + t);
          }
          if (wsh == 3 && wzn) {
            const T t = T(0.5) * (unz[l] - sUz[ym]) * rhy;
            syz_n = T(4) * recip(recip(gk[tid]) + recip(gk[ym])) * (E[3] - uy[l] * rhz + t);
            syz_k = T(4) * recip(recip(gn[tid]) + recip(gn[ym])) * (E[3] + uny[l] * rhz + t);
          }
        }
        sSxx[tid] = sxx;
        sSyy[tid] = syy;
        sSxy[tid] = sxy_s;
        sSxz[tid] = sxz_c[l];
        sSyz[tid] = syz_c[l];
        __syncthreads();
        if (face) {
          T rx = (sxx - sSxx[xm]) * rhx + (sSxy[yp] - sxy) * rhy + (sxz_n - sxz_c[l]) * rhz;
          T ry = (sSxy[xp] - sxy) * rhx + (syy - sSyy[ym]) * rhy + (syz_n - syz_c[l]) * rhz;
          T rz = (sSxz[xp] - sxz_c[l]) * rhx + (sSyz[yp] - syz_c[l]) * rhy + (szz - szz_p[l]) * rhz;
          rx += f0[l];
          ry += f1[l];
          rz += f2[l];
          if constexpr (WALLS) {  // held wall faces: no out-of-balance force
            if (wx) rx = T(0);
            if (wy) ry = T(0);
            if (kw == 0) rz = T(0);
          }
          if (partials != nullptr)
            nsum[l] += (double)rx * (double)rx + (double)ry * (double)ry + (double)rz * (double)rz;
          if (MODE == 0) {
            uold[l][oc] = ux[l] + mom * (ux[l] - uo0[l]) + sfx * rx;
            uold[l][N + oc] = uy[l] + mom * (uy[l] - uo1[l]) + sfy * ry;
            uold[l][2 * N + oc] = uz[l] + mom * (uz[l] - uo2[l]) + sfz * rz;
          } else {
            GLOBAL_AS R* ro = rout != nullptr ? gmut(rout[s0 + l]) : nullptr;
            if (ro != nullptr) {
              ro[oc] = (R)rx;
              ro[N + oc] = (R)ry;
              ro[2 * N + oc] = (R)rz;
            }
          }
        }
        szz_p[l] = szz;
        sxz_c[l] = sxz_k;
        syz_c[l] = syz_k;
        ux[l] = unx[l];
        uy[l] = uny[l];
        uz[l] = unz[l];
      }
      Kc = Kn;
      Gc = Gn;
      Hprev = Hk;
    }

    if (partials != nullptr) {
      // every work item writes all six slots (zero for loads it does not own)
      double tot[kMaxLoads] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int l = 0; l < L; ++l) {
        if (!(act & (1u << l))) continue;
        tot[s0 + l] = block_sum(nsum[l], red);
      }
      if (tid == 0)
        for (int q = 0; q < kMaxLoads; ++q) partials[(int64_t)w * kMaxLoads + q] = tot[q];
    }
    __syncthreads();  // LDS is reused by the next work item
  }
}

// Same iteration as step_kernel (MODE 0, no prefetch), with the z-march
// unrolled by two: the register sets of "this plane" and "next plane" swap
// roles at compile time instead of being copied at the end of every plane.
template <typename T, int L, bool HI>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 512), amdgpu_waves_per_eu(MinWaves<T, L, HI>::value)))
step_kernel_u2(const SampleDesc<T>* __restrict__ samples, const WorkItem* __restrict__ work, int nwork, int bx,
               int by, int parity, int first, double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int nt = blockDim.x;
  T* sG[2] = {reinterpret_cast<T*>(smem_raw), reinterpret_cast<T*>(smem_raw) + nt};
  T* sH = sG[1] + nt;
  T* sUx = sH + nt;
  T* sUy = sUx + nt;
  T* sUz = sUy + nt;
  T* sSxx = sUz + nt;
  T* sSyy = sSxx + nt;
  T* sSxy = sSyy + nt;
  T* sSxz = sSxy + nt;
  T* sSyz = sSxz + nt;

  const int tid = threadIdx.x;
  const int tx = tid % bx, ty = tid / bx;
  const int TX = bx - 2, TY = by - 2;
  const int xm = tid > 0 && tx > 0 ? tid - 1 : tid;
  const int xp = tx < bx - 1 && tid + 1 < nt ? tid + 1 : tid;
  const int ym = ty > 0 ? tid - bx : tid;
  const int yp = ty < by - 1 && tid + bx < nt ? tid + bx : tid;
  const int xmym = ty > 0 ? xm - bx : xm;

  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const WorkItem wi = work[w];
    if (wi.sample < 0) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      continue;
    }
    const SampleDesc<T>& sd = samples[wi.sample];
    const int s0 = wi.slot0;
    const unsigned act = (sd.active >> s0) & ((1u << L) - 1u);
    if (act == 0u) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      continue;
    }
    const int64_t nx = sd.nx, ny = sd.ny, nz = sd.nz, N = sd.N, plane = nx * ny;
    const T rhx = sd.rhx, rhy = sd.rhy, rhz = sd.rhz;
    const T mom = first ? T(0) : sd.mom;
    const T sfac = first ? sd.sfac_first : sd.sfac;
    const int64_t gi = (int64_t)wi.tx * TX + tx - 1, gj = (int64_t)wi.ty * TY + ty - 1;
    const int64_t col = wrap_idx(gi, nx) + nx * wrap_idx(gj, ny);
    const bool interior = tx >= 1 && tx <= TX && ty >= 1 && ty <= TY && gi < nx && gj < ny;
    const int64_t k0 = (int64_t)wi.kz * sd.kc;
    const int64_t k1 = k0 + sd.kc < nz ? k0 + sd.kc : nz;

    const GLOBAL_AS T* __restrict__ Kf = gconst(sd.K);
    const GLOBAL_AS T* __restrict__ Gf = gconst(sd.G);
    const GLOBAL_AS T* ucur[L];
    GLOBAL_AS T* uold[L];
    const GLOBAL_AS T* frc[L];
    bool hasf[L];
    T E[L][6];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      ucur[l] = gconst(sd.u[parity][s0 + l]);
      uold[l] = gmut(sd.u[parity ^ 1][s0 + l]);
      hasf[l] = sd.force[s0 + l] != nullptr;
      frc[l] = gconst(sd.force[s0 + l]);
#pragma unroll
      for (int q = 0; q < 6; ++q) E[l][q] = sd.E[s0 + l][q];
    }

    // two register sets, indexed by plane parity
    T Ux[2][L], Uy[2][L], Uz[2][L], Szz[2][L], Sxz[2][L], Syz[2][L], Kc[2], Gc[2], Hh[2];
    double nsum[L];
    {
      const int64_t kw = k0 - 1 < 0 ? k0 - 1 + nz : k0 - 1;
      const int64_t o = col + plane * kw;
#pragma unroll
      for (int l = 0; l < L; ++l) {
        Ux[0][l] = Uy[0][l] = Uz[0][l] = T(0);
        if (act & (1u << l)) {
          Ux[0][l] = ucur[l][o];
          Uy[0][l] = ucur[l][N + o];
          Uz[0][l] = ucur[l][2 * N + o];
        }
        Szz[1][l] = Sxz[1][l] = Syz[1][l] = T(0);
        nsum[l] = 0.0;
      }
      Kc[0] = Kf[o];
      Gc[0] = Gf[o];
      Hh[1] = T(1);
      sG[0][tid] = Gc[0];
    }

    auto plane_step = [&](int64_t k, auto Pc) {
      constexpr int P = decltype(Pc)::value;
      constexpr int Q = 1 - P;
      const int64_t kw = k < 0 ? k + nz : k;
      const int64_t kn = k + 1 >= nz ? k + 1 - nz : k + 1;
      const int64_t oc = col + plane * kw, on = col + plane * kn;
      const bool face = k >= k0 && interior;
      // plane k+1 into the other register set; u^{n-1} and force at plane k
      Kc[Q] = Kf[on];
      Gc[Q] = Gf[on];
      T uo0[L], uo1[L], uo2[L], f0[L], f1[L], f2[L];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        Ux[Q][l] = Uy[Q][l] = Uz[Q][l] = uo0[l] = uo1[l] = uo2[l] = f0[l] = f1[l] = f2[l] = T(0);
        if (act & (1u << l)) {
          Ux[Q][l] = ucur[l][on];
          Uy[Q][l] = ucur[l][N + on];
          Uz[Q][l] = ucur[l][2 * N + on];
          if (face) {
            if (!first) {
              uo0[l] = uold[l][oc];
              uo1[l] = uold[l][N + oc];
              uo2[l] = uold[l][2 * N + oc];
            }
            if (hasf[l]) {
              f0[l] = frc[l][oc];
              f1[l] = frc[l][N + oc];
              f2[l] = frc[l][2 * N + oc];
            }
          }
        }
      }
      T* gk = sG[P];
      T* gn = sG[Q];
      gn[tid] = Gc[Q];
      Hh[P] = Kc[P] + T(4.0 / 3.0) * Gc[P];
      sH[tid] = Hh[P];
      const T lam = Kc[P] - T(2.0 / 3.0) * Gc[P];
      const T twoG = T(2) * Gc[P];
      T G2xy = T(0), G2xz = T(0), G2yz = T(0), sfx = T(0), sfy = T(0), sfz = T(0);
      bool coef = false;
#pragma unroll
      for (int l = 0; l < L; ++l) {
        if (!(act & (1u << l))) continue;
        sUx[tid] = Ux[P][l];
        sUy[tid] = Uy[P][l];
        sUz[tid] = Uz[Q][l];
        __syncthreads();
        if (!coef) {
          const T ik = recip(gk[tid]), ikx = recip(gk[xm]), iky = recip(gk[ym]);
          const T in = recip(gn[tid]), inx = recip(gn[xm]), iny = recip(gn[ym]);
          G2xy = T(8) * recip(recip(gk[xmym]) + iky + ikx + ik);
          G2xz = T(8) * recip(ikx + ik + inx + in);
          G2yz = T(8) * recip(iky + ik + iny + in);
          sfx = sfac * recip(tmax(sH[xm], Hh[P]));
          sfy = sfac * recip(tmax(sH[ym], Hh[P]));
          sfz = sfac * recip(tmax(Hh[Q], Hh[P]));
          coef = true;
        }
        const T ux = Ux[P][l], uy = Uy[P][l], uz = Uz[P][l];
        const T unx = Ux[Q][l], uny = Uy[Q][l], unz = Uz[Q][l];
        const T exx = E[l][0] + (sUx[xp] - ux) * rhx;
        const T eyy = E[l][1] + (sUy[yp] - uy) * rhy;
        const T ezz = E[l][2] + (unz - uz) * rhz;
        const T th = exx + eyy + ezz;
        const T sxx = lam * th + twoG * exx;
        const T syy = lam * th + twoG * eyy;
        const T szz = lam * th + twoG * ezz;
        const T sxy = G2xy * (E[l][5] + T(0.5) * ((ux - sUx[ym]) * rhy + (uy - sUy[xm]) * rhx));
        const T sxz_n = G2xz * (E[l][4] + T(0.5) * ((unx - ux) * rhz + (unz - sUz[xm]) * rhx));
        const T syz_n = G2yz * (E[l][3] + T(0.5) * ((uny - uy) * rhz + (unz - sUz[ym]) * rhy));
        const T sxz_c = Sxz[Q][l], syz_c = Syz[Q][l];
        sSxx[tid] = sxx;
        sSyy[tid] = syy;
        sSxy[tid] = sxy;
        sSxz[tid] = sxz_c;
        sSyz[tid] = syz_c;
        __syncthreads();
        if (face) {
          T rx = (sxx - sSxx[xm]) * rhx + (sSxy[yp] - sxy) * rhy + (sxz_n - sxz_c) * rhz;
          T ry = (sSxy[xp] - sxy) * rhx + (syy - sSyy[ym]) * rhy + (syz_n - syz_c) * rhz;
          T rz = (sSxz[xp] - sxz_c) * rhx + (sSyz[yp] - syz_c) * rhy + (szz - Szz[Q][l]) * rhz;
          rx += f0[l];
          ry += f1[l];
          rz += f2[l];
          if (partials != nullptr)
            nsum[l] += (double)rx * (double)rx + (double)ry * (double)ry + (double)rz * (double)rz;
          uold[l][oc] = ux + mom * (ux - uo0[l]) + sfx * rx;
          uold[l][N + oc] = uy + mom * (uy - uo1[l]) + sfy * ry;
          uold[l][2 * N + oc] = uz + mom * (uz - uo2[l]) + sfz * rz;
        }
        Szz[P][l] = szz;
        Sxz[P][l] = sxz_n;
        Syz[P][l] = syz_n;
      }
    };

    for (int64_t k = k0 - 1; k < k1; k += 2) {
      plane_step(k, std::integral_constant<int, 0>{});
      if (k + 1 < k1) plane_step(k + 1, std::integral_constant<int, 1>{});
    }

    if (partials != nullptr) {
      double tot[kMaxLoads] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int l = 0; l < L; ++l) {
        if (!(act & (1u << l))) continue;
        tot[s0 + l] = block_sum(nsum[l], red);
      }
      if (tid == 0)
        for (int q = 0; q < kMaxLoads; ++q) partials[(int64_t)w * kMaxLoads + q] = tot[q];
    }
    __syncthreads();
  }
}

// Unrolled z-march with all loads of the block's group staged together: one
// barrier after the displacements of every load are in LDS, one after their
// stresses, so two barriers per plane whatever the group size.  LDS holds
// 3 + 8L arrays (and the coefficient table with PAL).  The G arrays hold 1/G,
// computed once per cell by its owner.
template <typename T, int L, bool HI, bool PAL, bool WALLS = false>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 512), amdgpu_waves_per_eu(MinWaves<T, L, HI>::value)))
step_kernel_b(const SampleDesc<T>* __restrict__ samples, const WorkItem* __restrict__ work, int nwork, int bx,
              int by, int parity, int first, double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int nt = blockDim.x;
  T* base = reinterpret_cast<T*>(smem_raw);
  T* sG[2] = {base, base + nt};
  T* sH = base + 2 * nt;
  T* lds_l = base + 3 * nt;  // per load: ux uy uz sxx syy sxy sxz syz
  auto S = [&](int l, int f) { return lds_l + (size_t)(8 * l + f) * nt; };
  CellCoef<T>* tab = reinterpret_cast<CellCoef<T>*>(lds_l + (size_t)8 * L * nt);
  if constexpr (PAL) stage_coef_table(samples[0], tab);

  const int tid = threadIdx.x;
  const int tx = tid % bx, ty = tid / bx;
  const int TX = bx - 2, TY = by - 2;
  const int xm = tid > 0 && tx > 0 ? tid - 1 : tid;
  const int xp = tx < bx - 1 && tid + 1 < nt ? tid + 1 : tid;
  const int ym = ty > 0 ? tid - bx : tid;
  const int yp = ty < by - 1 && tid + bx < nt ? tid + bx : tid;
  const int xmym = ty > 0 ? xm - bx : xm;

  // one work item per block (the grid is the work list): straight-line code, so
  // the per-thread set-up above is not spilled around a loop over items
  {
    const int w = blockIdx.x;
    if (w >= nwork) return;
    const WorkItem wi = work[w];
    if (wi.sample < 0) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      return;
    }
    const SampleDesc<T>& sd = samples[wi.sample];
    const int s0 = wi.slot0;
    const unsigned act = (sd.active >> s0) & ((1u << L) - 1u);
    if (act == 0u) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      return;
    }
    const int64_t nx = sd.nx, ny = sd.ny, nz = sd.nz, N = sd.N, plane = nx * ny;
    const T rhx = sd.rhx, rhy = sd.rhy, rhz = sd.rhz;
    const T mom = first ? T(0) : sd.mom;
    const T sfac = first ? sd.sfac_first : sd.sfac;
    const int64_t gi = (int64_t)wi.tx * TX + tx - 1, gj = (int64_t)wi.ty * TY + ty - 1;
    const int64_t col = wrap_idx(gi, nx) + nx * wrap_idx(gj, ny);
    const bool interior = tx >= 1 && tx <= TX && ty >= 1 && ty <= TY && gi < nx && gj < ny;
    // z indices in 32 bits (nz <= 2^20) so that the march's bookkeeping is scalar
    const int nz32 = (int)nz;
    const int k0 = wi.kz * sd.kc;
    const int k1 = k0 + sd.kc < nz32 ? k0 + sd.kc : nz32;
    // wall boundaries: this column lies in the x (y) boundary plane; wsh: the
    // Voigt shear component whose simple-shear test this load is (0: none)
    const bool wx = WALLS && wrap_idx(gi, nx) == 0, wy = WALLS && wrap_idx(gj, ny) == 0;
    const int wsh = WALLS ? sd.wshear[s0] : 0;

    // every field access: a buffer view of the component's z-plane (see PlaneBuf)
    const Moduli<T, PAL> mod(sd, tab);
    const uint32_t col32 = (uint32_t)col, colb = (uint32_t)col * (uint32_t)sizeof(T);
    const uint32_t pbytes = (uint32_t)(plane * (int64_t)sizeof(T));
    const T* pcur[L];
    T* pold[L];
    const T* pfrc[L];
    bool hasf[L];
    T E[L][6];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      hasf[l] = sd.force[s0 + l] != nullptr;
      pcur[l] = sd.u[parity][s0 + l];
      pold[l] = sd.u[parity ^ 1][s0 + l];
      pfrc[l] = sd.force[s0 + l];
#pragma unroll
      for (int q = 0; q < 6; ++q) E[l][q] = sd.E[s0 + l][q];
    }
    // component c of load l's fields in the z-plane at element offset pk
    auto ldu = [&](int l, int c, int64_t pk) -> T { return PlaneBuf(pcur[l] + (c * N + pk), pbytes).template ld<T>(colb); };
    auto ldo_ = [&](int l, int c, int64_t pk) -> T { return PlaneBuf(pold[l] + (c * N + pk), pbytes).template ld<T>(colb); };
    auto ldf = [&](int l, int c, int64_t pk) -> T { return PlaneBuf(pfrc[l] + (c * N + pk), pbytes).template ld<T>(colb); };
    auto sto_ = [&](int l, int c, int64_t pk, T v) { PlaneBuf(pold[l] + (c * N + pk), pbytes).st(colb, v); };

    T Ux[2][L], Uy[2][L], Uz[2][L], Szz[2][L], Sxz[2][L], Syz[2][L], iHh[2];
    CellCoef<T> Cc[2];
    double nsum[L];
    {
      const int kw = k0 - 1 < 0 ? k0 - 1 + nz32 : k0 - 1;
      const int64_t po = plane * kw;
#pragma unroll
      for (int l = 0; l < L; ++l) {
        Ux[0][l] = Uy[0][l] = Uz[0][l] = T(0);
        if (act & (1u << l)) {
          Ux[0][l] = ldu(l, 0, po);
          Uy[0][l] = ldu(l, 1, po);
          Uz[0][l] = ldu(l, 2, po);
        }
        Szz[1][l] = Sxz[1][l] = Syz[1][l] = T(0);
        nsum[l] = 0.0;
      }
      Cc[0] = mod.coef(mod.load(po, col32, colb));
      iHh[1] = T(1);
      sG[0][tid] = Cc[0].iG8;
    }

    // NORM: accumulate the squared residual (check iterations only)
    auto plane_step = [&](int k, auto Pc, auto Nc) {
      constexpr int P = decltype(Pc)::value;
      constexpr int Q = 1 - P;
      constexpr bool NORM = decltype(Nc)::value;
      const int kw = k < 0 ? k + nz32 : k;
      const int kn = k + 1 >= nz32 ? k + 1 - nz32 : k + 1;
      const int64_t pc = plane * kw, pn = plane * kn;
      const bool face = k >= k0 && interior;
      const auto mr = mod.load(pn, col32, colb);
      // u^{n-1} and the force only where a face is updated (ghost threads
      // reading them costs more memory requests than the masking costs ALU).
      // They are read only under the same conditions (face, not the first
      // iteration, a force present), so they are not zeroed: zeroing cost a
      // dozen vector moves per plane in an issue-bound loop.
      T uo0[L], uo1[L], uo2[L], f0[L], f1[L], f2[L];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        if (act & (1u << l)) {
          Ux[Q][l] = ldu(l, 0, pn);
          Uy[Q][l] = ldu(l, 1, pn);
          Uz[Q][l] = ldu(l, 2, pn);
          if (face) {
            if (!first) {
              uo0[l] = ldo_(l, 0, pc);
              uo1[l] = ldo_(l, 1, pc);
              uo2[l] = ldo_(l, 2, pc);
            }
            if (hasf[l]) {
              f0[l] = ldf(l, 0, pc);
              f1[l] = ldf(l, 1, pc);
              f2[l] = ldf(l, 2, pc);
            }
          }
        } else {
          Ux[Q][l] = Uy[Q][l] = Uz[Q][l] = T(0);
        }
      }
      T* gk = sG[P];
      T* gn = sG[Q];
      Cc[Q] = mod.coef(mr);
      gn[tid] = Cc[Q].iG8;
      iHh[P] = Cc[P].iH;
      sH[tid] = iHh[P];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        S(l, 0)[tid] = Ux[P][l];
        S(l, 1)[tid] = Uy[P][l];
        S(l, 2)[tid] = Uz[Q][l];
      }
      __syncthreads();
      const T lam = Cc[P].lam;
      const T twoG = Cc[P].twoG;
      const T ik = gk[tid], ikx = gk[xm], iky = gk[ym];
      const T in = gn[tid], inx = gn[xm], iny = gn[ym];
      const T G2xy = recip(gk[xmym] + iky + ikx + ik);
      const T G2xz = recip(ikx + ik + inx + in);
      const T G2yz = recip(iky + ik + iny + in);
      const T sfx = sfac * tmin(sH[xm], iHh[P]);
      const T sfy = sfac * tmin(sH[ym], iHh[P]);
      const T sfz = sfac * tmin(iHh[Q], iHh[P]);
      // sxy_s: the xy-edge stress published in LDS; sxz_k, syz_k: the ones
      // carried to the next plane (they differ from the thread's own only at the
      // split edges of a simple-shear test)
      T sxx[L], syy[L], szz[L], sxy[L], sxz_n[L], syz_n[L], sxy_s[L], sxz_k[L], syz_k[L];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        const T ux = Ux[P][l], uy = Uy[P][l], uz = Uz[P][l];
        const T unx = Ux[Q][l], uny = Uy[Q][l], unz = Uz[Q][l];
        const T* sUx = S(l, 0);
        const T* sUy = S(l, 1);
        const T* sUz = S(l, 2);
        const T exx = E[l][0] + (sUx[xp] - ux) * rhx;
        const T eyy = E[l][1] + (sUy[yp] - uy) * rhy;
        const T ezz = E[l][2] + (unz - uz) * rhz;
        const T th = exx + eyy + ezz;
        sxx[l] = lam * th + twoG * exx;
        syy[l] = lam * th + twoG * eyy;
        szz[l] = lam * th + twoG * ezz;
        sxy[l] = G2xy * (E[l][5] + T(0.5) * ((ux - sUx[ym]) * rhy + (uy - sUy[xm]) * rhx));
        sxz_n[l] = G2xz * (E[l][4] + T(0.5) * ((unx - ux) * rhz + (unz - sUz[xm]) * rhx));
        syz_n[l] = G2yz * (E[l][3] + T(0.5) * ((uny - uy) * rhz + (unz - sUz[ym]) * rhy));
        if constexpr (WALLS) {
          // edges in a boundary plane carry no shear stress (free slip), except
          // for the simple-shear test's own component: on the walls normal to
          // the sheared direction it is computed as inside, and on the loaded
          // walls (normal to z for yz and xz, to y for xy) the edge splits into
          // two halves, one per side of the box, each with the one-sided
          // derivative to the wall (where the fluctuation is held at zero) and
          // the harmonic mean of its own two cells (2 G = 0.5 / (iG8 + iG8'))
          if ((wx || wy) && wsh != 5) sxy[l] = T(0);
          if ((wx || kn == 0) && wsh != 4) sxz_n[l] = T(0);
          if ((wy || kn == 0) && wsh != 3) syz_n[l] = T(0);
          sxy_s[l] = sxy[l];
          sxz_k[l] = sxz_n[l];
          syz_k[l] = syz_n[l];
          if (wsh == 5 && wy) {  // own half in the cells j = 0, published half in j = ny - 1
            const T t = T(0.5) * (uy - sUy[xm]) * rhx;
            sxy[l] = T(0.5) * recip(ik + ikx) * (E[l][5] + ux * rhy + t);
            sxy_s[l] = T(0.5) * recip(gk[ym] + gk[xmym]) * (E[l][5] - sUx[ym] * rhy + t);
          }
          if (wsh == 4 && kn == 0) {  // upper edge of plane nz - 1, carried as the lower edge of plane 0
            const T t = T(0.5) * (unz - sUz[xm]) * rhx;
            sxz_n[l] = T(0.5) * recip(ik + ikx) * (E[l][4] - ux * rhz + t);
            sxz_k[l] = T(0.5) * recip(in + inx) * (E[l][4] + unx * rhz + t);
          }
          if (wsh == 3 && kn == 0) {
            const T t = T(0.5) * (unz - sUz[ym]) * rhy;
            syz_n[l] = T(0.5) * recip(ik + iky) * (E[l][3] - uy * rhz + t);
            syz_k[l] = T(0.5) * recip(in + iny) * (E[l][3] + uny * rhz + t);
          }
        } else {
          sxy_s[l] = sxy[l];
          sxz_k[l] = sxz_n[l];
          syz_k[l] = syz_n[l];
        }
        S(l, 3)[tid] = sxx[l];
        S(l, 4)[tid] = syy[l];
        S(l, 5)[tid] = sxy_s[l];
        S(l, 6)[tid] = Sxz[Q][l];
        S(l, 7)[tid] = Syz[Q][l];
      }
      __syncthreads();
#pragma unroll
      for (int l = 0; l < L; ++l) {
        if (face && (act & (1u << l))) {
          const T* sSxx = S(l, 3);
          const T* sSyy = S(l, 4);
          const T* sSxy = S(l, 5);
          const T* sSxz = S(l, 6);
          const T* sSyz = S(l, 7);
          const T sxz_c = Sxz[Q][l], syz_c = Syz[Q][l];
          T rx = (sxx[l] - sSxx[xm]) * rhx + (sSxy[yp] - sxy[l]) * rhy + (sxz_n[l] - sxz_c) * rhz;
          T ry = (sSxy[xp] - sxy[l]) * rhx + (syy[l] - sSyy[ym]) * rhy + (syz_n[l] - syz_c) * rhz;
          T rz = (sSxz[xp] - sxz_c) * rhx + (sSyz[yp] - syz_c) * rhy + (szz[l] - Szz[Q][l]) * rhz;
          if (hasf[l]) {
            rx += f0[l];
            ry += f1[l];
            rz += f2[l];
          }
          if constexpr (WALLS) {  // held wall faces: no out-of-balance force
            if (wx) rx = T(0);
            if (wy) ry = T(0);
            if (kw == 0) rz = T(0);
          }
          if (NORM && (L == 1 || partials != nullptr))
            nsum[l] += (double)rx * (double)rx + (double)ry * (double)ry + (double)rz * (double)rz;
          const T ux = Ux[P][l], uy = Uy[P][l], uz = Uz[P][l];
          if (first) {  // no momentum in the start-up step
            sto_(l, 0, pc, ux + sfx * rx);
            sto_(l, 1, pc, uy + sfy * ry);
            sto_(l, 2, pc, uz + sfz * rz);
          } else {
            sto_(l, 0, pc, ux + mom * (ux - uo0[l]) + sfx * rx);
            sto_(l, 1, pc, uy + mom * (uy - uo1[l]) + sfy * ry);
            sto_(l, 2, pc, uz + mom * (uz - uo2[l]) + sfz * rz);
          }
        }
        Szz[P][l] = szz[l];
        Sxz[P][l] = sxz_k[l];
        Syz[P][l] = syz_k[l];
      }
    };

    auto march = [&](auto Nc) {
      for (int k = k0 - 1; k < k1; k += 2) {
        plane_step(k, std::integral_constant<int, 0>{}, Nc);
        if (k + 1 < k1) plane_step(k + 1, std::integral_constant<int, 1>{}, Nc);
      }
    };
    // one load per block: a march without the norm for the plain iterations;
    // with several loads a second copy of the march costs more registers than
    // the norm's instructions, so the norm is guarded at run time
    if constexpr (L > 1) {
      march(std::true_type{});
    } else {
      if (partials != nullptr)
        march(std::true_type{});
      else
        march(std::false_type{});
    }

    if (partials != nullptr) {
      double tot[kMaxLoads] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int l = 0; l < L; ++l) {
        if (!(act & (1u << l))) continue;
        tot[s0 + l] = block_sum(nsum[l], red);
      }
      if (tid == 0)
        for (int q = 0; q < kMaxLoads; ++q) partials[(int64_t)w * kMaxLoads + q] = tot[q];
    }
    __syncthreads();
  }
}

// ---- one iteration with x-neighbours across lanes (variant 9) ---------------
//
// step_kernel_b for one load per block and periodic isotropic cells, with the
// block's rows exactly 16, 32 or 64 cells wide so that no row crosses a wave:
// the x-neighbour of a thread is then the next or previous lane of its own wave,
// and every x-neighbour value (u, 1/(8G), 1/H, sxx, sxy, the carried sxz) moves
// between lanes with a DPP wave shift instead of a round trip through LDS.  Only
// the y-neighbours go through LDS (9 reads and 8 writes per plane instead of 19
// and 10).  The values and the arithmetic are those of step_kernel_b.  Where a
// shift has no source lane (lane 0 for the previous lane, lane 63 for the next)
// it yields zero, and the first and last lanes of the wave's other rows receive
// the neighbouring row's value: these lanes are ghost columns whose shifted
// values no interior thread reads (as with the clamped index there), and the
// zero fill lets the compiler fold each shift into the instruction that consumes
// it as a DPP operand.  Every sum of 1/(8G) terms stays positive, so ghost lanes
// compute finite values.
__device__ __forceinline__ float lane_prev(float v) {  // value of lane - 1 (lane 0: zero)
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_next(float v) {  // value of lane + 1 (lane 63: zero)
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_prev(double v) {  // both halves moved by one lane
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = (int)(uint32_t)b, hi = (int)(uint32_t)(b >> 32);
  const uint32_t l2 = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);
  const uint32_t h2 = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)h2 << 32) | l2);
}
__device__ __forceinline__ double lane_next(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = (int)(uint32_t)b, hi = (int)(uint32_t)(b >> 32);
  const uint32_t l2 = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);
  const uint32_t h2 = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)h2 << 32) | l2);
}

template <typename T, bool HI, bool PAL, int CAP, int FRC>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, CAP), amdgpu_waves_per_eu(MinWaves<T, 1, HI>::value)))
step_kernel_x(const SampleDesc<T>* __restrict__ samples, const WorkItem* __restrict__ work, int nwork, int bx,
              int by, int parity, int first, double* __restrict__ partials) {
  // rows: 0-1 1/(8G) of two planes, 2 1/H, 3-5 ux, uy of plane k and uz of plane k+1, 6 syy, 7 sxy,
  // 8 the carried syz
  __shared__ __align__(16) T sL[9][CAP];
  __shared__ CellCoef<T> tab[PAL ? 256 : 1];
  __shared__ double red[16];
  if constexpr (PAL) stage_coef_table(samples[0], tab);
  const int nt = blockDim.x;
  T* const sG[2] = {sL[0], sL[1]};
  T* const sH = sL[2];
  T* const sUx = sL[3];
  T* const sUy = sL[4];
  T* const sUz = sL[5];
  T* const sSyy = sL[6];
  T* const sSxy = sL[7];
  T* const sSyz = sL[8];

  const int tid = threadIdx.x;
  const int tx = tid % bx, ty = tid / bx;
  const int TX = bx - 2, TY = by - 2;
  const int ym = ty > 0 ? tid - bx : tid;
  const int yp = ty < by - 1 && tid + bx < nt ? tid + bx : tid;

  const int w = blockIdx.x;  // one work item per block
  if (w >= nwork) return;
  const WorkItem wi = work[w];
  if (wi.sample < 0) {
    if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
    return;
  }
  const SampleDesc<T>& sd = samples[wi.sample];
  const int s0 = wi.slot0;
  if (!((sd.active >> s0) & 1u)) {
    if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
    return;
  }
  const int64_t nx = sd.nx, ny = sd.ny, N = sd.N, plane = nx * ny;
  const T rhx = sd.rhx, rhy = sd.rhy, rhz = sd.rhz;
  const T mom = first ? T(0) : sd.mom;
  const T sfac = first ? sd.sfac_first : sd.sfac;
  const int64_t gi = (int64_t)wi.tx * TX + tx - 1, gj = (int64_t)wi.ty * TY + ty - 1;
  const int64_t col = wrap_idx(gi, nx) + nx * wrap_idx(gj, ny);
  const bool interior = tx >= 1 && tx <= TX && ty >= 1 && ty <= TY && gi < nx && gj < ny;
  const int nz32 = (int)sd.nz;
  const int k0 = wi.kz * sd.kc;
  const int k1 = k0 + sd.kc < nz32 ? k0 + sd.kc : nz32;

  const Moduli<T, PAL> mod(sd, tab);
  const uint32_t col32 = (uint32_t)col, colb = (uint32_t)col * (uint32_t)sizeof(T);
  const uint32_t pbytes = (uint32_t)(plane * (int64_t)sizeof(T));
  const T* pcur = sd.u[parity][s0];
  T* pold = sd.u[parity ^ 1][s0];
  const T* pfrc = sd.force[s0];
  // FRC: the host knows that no active load of the launch has a body force (0) or that all of
  // them have one (1); with 2 each block checks its own
  const bool hasf = FRC == 2 ? pfrc != nullptr : FRC == 1;
  T E[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) E[q] = sd.E[s0][q];
  auto ldu = [&](int c, int64_t pk) -> T { return PlaneBuf(pcur + (c * N + pk), pbytes).template ld<T>(colb); };
  auto ldo_ = [&](int c, int64_t pk) -> T { return PlaneBuf(pold + (c * N + pk), pbytes).template ld<T>(colb); };
  auto ldf = [&](int c, int64_t pk) -> T { return PlaneBuf(pfrc + (c * N + pk), pbytes).template ld<T>(colb); };
  auto sto_ = [&](int c, int64_t pk, T v) { PlaneBuf(pold + (c * N + pk), pbytes).st(colb, v); };

  T Ux[2], Uy[2], Uz[2], Szz[2], Sxz[2], Syz[2], iHh[2];
  CellCoef<T> Cc[2];
  double nsum = 0.0;
  {
    const int kw = k0 - 1 < 0 ? k0 - 1 + nz32 : k0 - 1;
    const int64_t po = plane * kw;
    Ux[0] = ldu(0, po);
    Uy[0] = ldu(1, po);
    Uz[0] = ldu(2, po);
    Szz[1] = Sxz[1] = Syz[1] = T(0);
    Cc[0] = mod.coef(mod.load(po, col32, colb));
    iHh[1] = T(1);
    sG[0][tid] = Cc[0].iG8;
  }

  auto plane_step = [&](int k, auto Pc, auto Nc) {
    constexpr int P = decltype(Pc)::value;
    constexpr int Q = 1 - P;
    constexpr bool NORM = decltype(Nc)::value;
    const int kw = k < 0 ? k + nz32 : k;
    const int kn = k + 1 >= nz32 ? k + 1 - nz32 : k + 1;
    const int64_t pc = plane * kw, pn = plane * kn;
    const bool face = k >= k0 && interior;
    const auto mr = mod.load(pn, col32, colb);
    T uo0, uo1, uo2, f0, f1, f2;
    Ux[Q] = ldu(0, pn);
    Uy[Q] = ldu(1, pn);
    Uz[Q] = ldu(2, pn);
    if (face) {
      if (!first) {
        uo0 = ldo_(0, pc);
        uo1 = ldo_(1, pc);
        uo2 = ldo_(2, pc);
      }
      if (hasf) {
        f0 = ldf(0, pc);
        f1 = ldf(1, pc);
        f2 = ldf(2, pc);
      }
    }
    T* gk = sG[P];
    T* gn = sG[Q];
    Cc[Q] = mod.coef(mr);
    gn[tid] = Cc[Q].iG8;
    iHh[P] = Cc[P].iH;
    sH[tid] = iHh[P];
    sUx[tid] = Ux[P];
    sUy[tid] = Uy[P];
    sUz[tid] = Uz[Q];
    __syncthreads();
    const T lam = Cc[P].lam;
    const T twoG = Cc[P].twoG;
    const T ux = Ux[P], uy = Uy[P], uz = Uz[P];
    const T unx = Ux[Q], uny = Uy[Q], unz = Uz[Q];
    // own values from registers, x-neighbours across lanes, y-neighbours from LDS
    const T ik = Cc[P].iG8, ikx = lane_prev(ik), iky = gk[ym];
    const T in = Cc[Q].iG8, inx = lane_prev(in), iny = gn[ym];
    const T G2xy = recip(lane_prev(iky) + iky + ikx + ik);
    const T G2xz = recip(ikx + ik + inx + in);
    const T G2yz = recip(iky + ik + iny + in);
    const T sfx = sfac * tmin(lane_prev(iHh[P]), iHh[P]);
    const T sfy = sfac * tmin(sH[ym], iHh[P]);
    const T sfz = sfac * tmin(iHh[Q], iHh[P]);
    const T exx = E[0] + (lane_next(ux) - ux) * rhx;
    const T eyy = E[1] + (sUy[yp] - uy) * rhy;
    const T ezz = E[2] + (unz - uz) * rhz;
    const T th = exx + eyy + ezz;
    const T sxx = lam * th + twoG * exx;
    const T syy = lam * th + twoG * eyy;
    const T szz = lam * th + twoG * ezz;
    const T sxy = G2xy * (E[5] + T(0.5) * ((ux - sUx[ym]) * rhy + (uy - lane_prev(uy)) * rhx));
    const T sxz_n = G2xz * (E[4] + T(0.5) * ((unx - ux) * rhz + (unz - lane_prev(unz)) * rhx));
    const T syz_n = G2yz * (E[3] + T(0.5) * ((uny - uy) * rhz + (unz - sUz[ym]) * rhy));
    sSyy[tid] = syy;
    sSxy[tid] = sxy;
    sSyz[tid] = Syz[Q];
    // the x-neighbours' stresses, across lanes (no barrier needed for these)
    const T sxx_m = lane_prev(sxx), sxy_p = lane_next(sxy), sxz_p = lane_next(Sxz[Q]);
    __syncthreads();
    if (face) {
      const T sxz_c = Sxz[Q], syz_c = Syz[Q];
      T rx = (sxx - sxx_m) * rhx + (sSxy[yp] - sxy) * rhy + (sxz_n - sxz_c) * rhz;
      T ry = (sxy_p - sxy) * rhx + (syy - sSyy[ym]) * rhy + (syz_n - syz_c) * rhz;
      T rz = (sxz_p - sxz_c) * rhx + (sSyz[yp] - syz_c) * rhy + (szz - Szz[Q]) * rhz;
      if (hasf) {
        rx += f0;
        ry += f1;
        rz += f2;
      }
      if (NORM) nsum += (double)rx * (double)rx + (double)ry * (double)ry + (double)rz * (double)rz;
      if (first) {  // no momentum in the start-up step
        sto_(0, pc, ux + sfx * rx);
        sto_(1, pc, uy + sfy * ry);
        sto_(2, pc, uz + sfz * rz);
      } else {
        sto_(0, pc, ux + mom * (ux - uo0) + sfx * rx);
        sto_(1, pc, uy + mom * (uy - uo1) + sfy * ry);
        sto_(2, pc, uz + mom * (uz - uo2) + sfz * rz);
      }
    }
    Szz[P] = szz;
    Sxz[P] = sxz_n;
    Syz[P] = syz_n;
  };

  auto march = [&](auto Nc) {
    for (int k = k0 - 1; k < k1; k += 2) {
      plane_step(k, std::integral_constant<int, 0>{}, Nc);
      if (k + 1 < k1) plane_step(k + 1, std::integral_constant<int, 1>{}, Nc);
    }
  };
  if (partials != nullptr)
    march(std::true_type{});
  else
    march(std::false_type{});

  if (partials != nullptr) {
    const double tot = block_sum(nsum, red);
    if (tid == 0)
      for (int q = 0; q < kMaxLoads; ++q) partials[(int64_t)w * kMaxLoads + q] = q == s0 ? tot : 0.0;
  }
}

// Two heavy-ball iterations in one z-march (one load per block, periodic
// boundaries): u^{n+1} from (u^n, u^{n-1}) and u^{n+2} from (u^{n+1}, u^n).
// u^n and u^{n-1} are buffers parity and parity ^ 1; the results go to the
// other pair of buffers, u^{n+1} to the even and u^{n+2} to the odd one, so
// no block overwrites data another block still reads, and u^n, u^{n-1} are read
// once for two iterations: 12 words of state traffic per two voxel-updates
// instead of 18.  The ghost ring is two cells deep: stage 1 (u^{n+1}) is valid
// on the tile and a one-cell ring around it, stage 2 on the tile.  Stage 2 runs
// two planes behind stage 1, so both stages' inputs go to LDS together and a
// plane takes two barriers.  The chunk [k0, k1) of u^{n+2} needs u^{n+1} on
// [k0-1, k1], hence u^n on [k0-2, k1+1]: each stage starts with one plane that
// only computes the stresses carried to the next.  LDS: 1/(8G) of four planes
// (by plane index mod 4), 1/H of each stage's plane, and per stage ux uy uz
// sxx syy sxy sxz syz.  On check iterations the squared residual of u^{n+1}
// (stage 2's input) is reduced.
template <typename T, bool HI>
struct MinWavesT {
  static constexpr int value = HI ? (sizeof(T) == 4 ? 4 : 2) : (sizeof(T) == 4 ? 2 : 1);
};

template <typename T, bool HI, bool PAL>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 512), amdgpu_waves_per_eu(MinWavesT<T, HI>::value)))
step_kernel_t(const SampleDesc<T>* __restrict__ samples, const WorkItem* __restrict__ work, int nwork, int bx,
              int by, int parity, double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int nt = blockDim.x;
  T* base = reinterpret_cast<T*>(smem_raw);
  T* sG[4] = {base, base + nt, base + 2 * nt, base + 3 * nt};
  T* sH[2] = {base + 4 * nt, base + 5 * nt};
  auto S = [&](int st, int f) { return base + (size_t)(6 + 8 * st + f) * nt; };
  CellCoef<T>* tab = reinterpret_cast<CellCoef<T>*>(base + (size_t)22 * nt);
  if constexpr (PAL) stage_coef_table(samples[0], tab);

  const int tid = threadIdx.x;
  const int tx = tid % bx, ty = tid / bx;
  const int TX = bx - 4, TY = by - 4;
  const int xm = tid > 0 && tx > 0 ? tid - 1 : tid;
  const int xp = tx < bx - 1 && tid + 1 < nt ? tid + 1 : tid;
  const int ym = ty > 0 ? tid - bx : tid;
  const int yp = ty < by - 1 && tid + bx < nt ? tid + bx : tid;
  const int xmym = ty > 0 ? xm - bx : xm;

  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const WorkItem wi = work[w];
    const SampleDesc<T>* sdp = wi.sample >= 0 ? &samples[wi.sample] : nullptr;
    if (sdp == nullptr || !((sdp->active >> wi.slot0) & 1u)) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      continue;
    }
    const SampleDesc<T>& sd = *sdp;
    const int s0 = wi.slot0;
    const int64_t nx = sd.nx, ny = sd.ny, N = sd.N, plane = nx * ny;
    const int nz32 = (int)sd.nz;
    const T rhx = sd.rhx, rhy = sd.rhy, rhz = sd.rhz;
    const T mom = sd.mom, sfac = sd.sfac;
    const int64_t gi = (int64_t)wi.tx * TX + tx - 2, gj = (int64_t)wi.ty * TY + ty - 2;
    const int64_t col = wrap_idx(gi, nx) + nx * wrap_idx(gj, ny);
    const bool ring1 = tx >= 1 && tx <= bx - 2 && ty >= 1 && ty <= by - 2;
    const bool own = tx >= 2 && tx <= bx - 3 && ty >= 2 && ty <= by - 3 && gi < nx && gj < ny;
    const int k0 = wi.kz * sd.kc;
    const int k1 = k0 + sd.kc < nz32 ? k0 + sd.kc : nz32;
    auto wz = [&](int k) { return k < 0 ? k + nz32 : (k >= nz32 ? k - nz32 : k); };

    const Moduli<T, PAL> mod(sd, tab);
    const uint32_t col32 = (uint32_t)col, colb = (uint32_t)col * (uint32_t)sizeof(T);
    const uint32_t pbytes = (uint32_t)(plane * (int64_t)sizeof(T));
    const T* pn = sd.u[parity][s0];
    const T* po = sd.u[parity ^ 1][s0];
    const int dset = (parity ^ 2) & 2;
    T* q1 = sd.u[dset][s0];
    T* q2 = sd.u[dset | 1][s0];
    const T* pf = sd.force[s0];
    const bool hasf = pf != nullptr;
    T E[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) E[q] = sd.E[s0][q];
    auto ld = [&](const T* f, int c, int k) -> T {
      return PlaneBuf(f + (c * N + plane * (int64_t)wz(k)), pbytes).template ld<T>(colb);
    };
    auto st = [&](T* f, int c, int k, T v) { PlaneBuf(f + (c * N + plane * (int64_t)wz(k)), pbytes).st(colb, v); };

    // u^n of planes k+1 (un), k (uc), k-1, k-2 (uh1, uh2); u^{n+1} of planes k-1, k-2 (v1, v2);
    // cell coefficients of planes k+1, k, k-1, k-2; stresses carried to the next plane per stage
    T un[3], uc[3], uh1[3], uh2[3], v1[3], v2[3];
    CellCoef<T> cn, cc, ch1, ch2;
    // per stage, carried from its previous plane: the lower cell's szz, the lower edges' sxz and
    // syz, and the lower cell's 1/H (the z-face of a plane separates it from the plane below)
    T szz[2] = {T(0), T(0)}, sxzl[2] = {T(0), T(0)}, syzl[2] = {T(0), T(0)}, iHlo[2] = {T(1), T(1)};
    double nsum = 0.0;
    {
      const int k = k0 - 2;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        uc[c] = ld(pn, c, k);
        uh1[c] = uh2[c] = v1[c] = v2[c] = T(0);
      }
      cc = mod.coef(mod.load(plane * (int64_t)wz(k), col32, colb));
      ch1 = ch2 = cc;
      sG[k & 3][tid] = cc.iG8;
    }

    // one stage's stresses at plane p (own column: u at p and p+1, the cell coefficients of p;
    // in-plane neighbours and the 1/(8G) of planes p and p+1 from LDS), published in LDS;
    // also returns the face step factors
    struct Str {
      T sxx, syy, szz, sxy, sxz, syz, sfx, sfy, sfz;
    };
    auto stresses = [&](int sidx, int p, const T* u, const T* unx, const CellCoef<T>& cp) -> Str {
      const T* gk = sG[p & 3];
      const T* gq = sG[(p + 1) & 3];
      const T* sUx = S(sidx, 0);
      const T* sUy = S(sidx, 1);
      const T* sUz = S(sidx, 2);
      const T ik = gk[tid], ikx = gk[xm], iky = gk[ym];
      const T in_ = gq[tid], inx = gq[xm], iny = gq[ym];
      const T G2xy = recip(gk[xmym] + iky + ikx + ik);
      const T G2xz = recip(ikx + ik + inx + in_);
      const T G2yz = recip(iky + ik + iny + in_);
      Str r;
      r.sfx = sfac * tmin(sH[sidx][xm], cp.iH);
      r.sfy = sfac * tmin(sH[sidx][ym], cp.iH);
      r.sfz = sfac * tmin(iHlo[sidx], cp.iH);
      const T exx = E[0] + (sUx[xp] - u[0]) * rhx;
      const T eyy = E[1] + (sUy[yp] - u[1]) * rhy;
      const T ezz = E[2] + (unx[2] - u[2]) * rhz;
      const T th = exx + eyy + ezz;
      r.sxx = cp.lam * th + cp.twoG * exx;
      r.syy = cp.lam * th + cp.twoG * eyy;
      r.szz = cp.lam * th + cp.twoG * ezz;
      r.sxy = G2xy * (E[5] + T(0.5) * ((u[0] - sUx[ym]) * rhy + (u[1] - sUy[xm]) * rhx));
      r.sxz = G2xz * (E[4] + T(0.5) * ((unx[0] - u[0]) * rhz + (unx[2] - sUz[xm]) * rhx));
      r.syz = G2yz * (E[3] + T(0.5) * ((unx[1] - u[1]) * rhz + (unx[2] - sUz[ym]) * rhy));
      S(sidx, 3)[tid] = r.sxx;
      S(sidx, 4)[tid] = r.syy;
      S(sidx, 5)[tid] = r.sxy;
      S(sidx, 6)[tid] = sxzl[sidx];
      S(sidx, 7)[tid] = syzl[sidx];
      return r;
    };
    // the out-of-balance force at this thread's faces of the stage's plane
    auto residual = [&](int sidx, const Str& r, T* out) {
      const T* sSxx = S(sidx, 3);
      const T* sSyy = S(sidx, 4);
      const T* sSxy = S(sidx, 5);
      const T* sSxz = S(sidx, 6);
      const T* sSyz = S(sidx, 7);
      out[0] = (r.sxx - sSxx[xm]) * rhx + (sSxy[yp] - r.sxy) * rhy + (r.sxz - sxzl[sidx]) * rhz;
      out[1] = (sSxy[xp] - r.sxy) * rhx + (r.syy - sSyy[ym]) * rhy + (r.syz - syzl[sidx]) * rhz;
      out[2] = (sSxz[xp] - sxzl[sidx]) * rhx + (sSyz[yp] - syzl[sidx]) * rhy + (r.szz - szz[sidx]) * rhz;
    };

    auto march = [&](auto Nc) {
      constexpr bool NORM = decltype(Nc)::value;
      for (int k = k0 - 2; k <= k1 + 1; ++k) {
        const int p = k - 2;
        const bool s1 = k <= k1, s2 = p >= k0 - 1;
        // global data: u^n and coefficients of plane k+1, u^{n-1} and force at plane k (stage 1),
        // force at plane p (stage 2)
        T uo[3] = {T(0), T(0), T(0)}, f1[3] = {T(0), T(0), T(0)}, f2[3] = {T(0), T(0), T(0)};
        if (s1) {
          const auto mr = mod.load(plane * (int64_t)wz(k + 1), col32, colb);
#pragma unroll
          for (int c = 0; c < 3; ++c) un[c] = ld(pn, c, k + 1);
          if (ring1 && k >= k0 - 1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) uo[c] = ld(po, c, k);
            if (hasf) {
#pragma unroll
              for (int c = 0; c < 3; ++c) f1[c] = ld(pf, c, k);
            }
          }
          cn = mod.coef(mr);
          sG[(k + 1) & 3][tid] = cn.iG8;
          sH[0][tid] = cc.iH;
          S(0, 0)[tid] = uc[0];
          S(0, 1)[tid] = uc[1];
          S(0, 2)[tid] = un[2];
        }
        if (s2) {
          if (own && hasf && p >= k0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) f2[c] = ld(pf, c, p);
          }
          sH[1][tid] = ch2.iH;
          S(1, 0)[tid] = v2[0];
          S(1, 1)[tid] = v2[1];
          S(1, 2)[tid] = v1[2];
        }
        __syncthreads();
        Str r1{}, r2{};
        if (s1) r1 = stresses(0, k, uc, un, cc);
        if (s2) r2 = stresses(1, p, v2, v1, ch2);
        __syncthreads();
        T w1[3] = {T(0), T(0), T(0)};
        if (s1) {
          if (ring1 && k >= k0 - 1) {
            T r[3];
            residual(0, r1, r);
            w1[0] = uc[0] + mom * (uc[0] - uo[0]) + r1.sfx * (r[0] + f1[0]);
            w1[1] = uc[1] + mom * (uc[1] - uo[1]) + r1.sfy * (r[1] + f1[1]);
            w1[2] = uc[2] + mom * (uc[2] - uo[2]) + r1.sfz * (r[2] + f1[2]);
            if (own && k >= k0 && k < k1) {
#pragma unroll
              for (int c = 0; c < 3; ++c) st(q1, c, k, w1[c]);
            }
          }
          szz[0] = r1.szz;
          sxzl[0] = r1.sxz;
          syzl[0] = r1.syz;
          iHlo[0] = cc.iH;
        }
        if (s2) {
          if (own && p >= k0) {
            T r[3];
            residual(1, r2, r);
#pragma unroll
            for (int c = 0; c < 3; ++c) r[c] += f2[c];
            if (NORM) nsum += (double)r[0] * (double)r[0] + (double)r[1] * (double)r[1] + (double)r[2] * (double)r[2];
            st(q2, 0, p, v2[0] + mom * (v2[0] - uh2[0]) + r2.sfx * r[0]);
            st(q2, 1, p, v2[1] + mom * (v2[1] - uh2[1]) + r2.sfy * r[1]);
            st(q2, 2, p, v2[2] + mom * (v2[2] - uh2[2]) + r2.sfz * r[2]);
          }
          szz[1] = r2.szz;
          sxzl[1] = r2.sxz;
          syzl[1] = r2.syz;
          iHlo[1] = ch2.iH;
        }
        // shift the plane histories by one
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          uh2[c] = uh1[c];
          uh1[c] = uc[c];
          uc[c] = un[c];
          v2[c] = v1[c];
          v1[c] = w1[c];
        }
        ch2 = ch1;
        ch1 = cc;
        cc = cn;
      }
    };
    if (partials != nullptr)
      march(std::true_type{});
    else
      march(std::false_type{});

    if (partials != nullptr) {
      const double tot = block_sum(nsum, red);
      if (tid == 0)
        for (int q = 0; q < kMaxLoads; ++q) partials[(int64_t)w * kMaxLoads + q] = q == s0 ? tot : 0.0;
    }
    __syncthreads();
  }
}

// Batched-barrier z-march unrolled by three with three rotating register sets,
// so that the global data of plane k+2 (u^n), and of plane k+1 (u^{n-1},
// body force), is requested while plane k is processed and first used one
// plane later: load latency overlaps a whole plane of work, with no register
// copies between planes.
// the three register sets need room: 4 waves per SIMD for one FP32 load, 3 for
// two, 2 otherwise (HI asks for one wave more)
template <typename T, int L, bool HI>
struct MinWavesP3 {
  static constexpr int lo = sizeof(T) == 4 ? (L == 1 ? 4 : (L == 2 ? 3 : 1)) : (L == 1 ? 2 : 1);
  static constexpr int value = HI ? lo + 1 : lo;
};

template <typename T, int L, bool HI>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 512), amdgpu_waves_per_eu(MinWavesP3<T, L, HI>::value)))
step_kernel_p3(const SampleDesc<T>* __restrict__ samples, const WorkItem* __restrict__ work, int nwork, int bx,
               int by, int parity, int first, double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int nt = blockDim.x;
  T* base = reinterpret_cast<T*>(smem_raw);
  T* sG[2] = {base, base + nt};
  T* sH = base + 2 * nt;
  T* lds_l = base + 3 * nt;  // per load: ux uy uz sxx syy sxy sxz syz
  auto S = [&](int l, int f) { return lds_l + (size_t)(8 * l + f) * nt; };

  const int tid = threadIdx.x;
  const int tx = tid % bx, ty = tid / bx;
  const int TX = bx - 2, TY = by - 2;
  const int xm = tid > 0 && tx > 0 ? tid - 1 : tid;
  const int xp = tx < bx - 1 && tid + 1 < nt ? tid + 1 : tid;
  const int ym = ty > 0 ? tid - bx : tid;
  const int yp = ty < by - 1 && tid + bx < nt ? tid + bx : tid;
  const int xmym = ty > 0 ? xm - bx : xm;

  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const WorkItem wi = work[w];
    if (wi.sample < 0) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      continue;
    }
    const SampleDesc<T>& sd = samples[wi.sample];
    const int s0 = wi.slot0;
    const unsigned act = (sd.active >> s0) & ((1u << L) - 1u);
    if (act == 0u) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      continue;
    }
    const int64_t nx = sd.nx, ny = sd.ny, nz = sd.nz, N = sd.N, plane = nx * ny;
    const T rhx = sd.rhx, rhy = sd.rhy, rhz = sd.rhz;
    const T mom = first ? T(0) : sd.mom;
    const T sfac = first ? sd.sfac_first : sd.sfac;
    const int64_t gi = (int64_t)wi.tx * TX + tx - 1, gj = (int64_t)wi.ty * TY + ty - 1;
    const int64_t col = wrap_idx(gi, nx) + nx * wrap_idx(gj, ny);
    const bool interior = tx >= 1 && tx <= TX && ty >= 1 && ty <= TY && gi < nx && gj < ny;
    const int64_t k0 = (int64_t)wi.kz * sd.kc;
    const int64_t k1 = k0 + sd.kc < nz ? k0 + sd.kc : nz;

    const GLOBAL_AS T* __restrict__ Kf = gconst(sd.K);
    const GLOBAL_AS T* __restrict__ Gf = gconst(sd.G);
    const GLOBAL_AS T* ucur[L];
    GLOBAL_AS T* uold[L];
    const GLOBAL_AS T* frc[L];
    bool hasf[L];
    T E[L][6];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      ucur[l] = gconst(sd.u[parity][s0 + l]);
      uold[l] = gmut(sd.u[parity ^ 1][s0 + l]);
      hasf[l] = sd.force[s0 + l] != nullptr;
      frc[l] = gconst(sd.force[s0 + l]);
#pragma unroll
      for (int q = 0; q < 6; ++q) E[l][q] = sd.E[s0 + l][q];
    }
    bool anyf = false;
#pragma unroll
    for (int l = 0; l < L; ++l) anyf = anyf || ((act & (1u << l)) && hasf[l]);

    // register sets by plane index mod 3: u^n and moduli of that plane, and
    // u^{n-1} and the body force of that plane
    T Ux[3][L], Uy[3][L], Uz[3][L], Ko[3], Go[3];
    T Vo0[3][L], Vo1[3][L], Vo2[3][L], F0[3][L], F1[3][L], F2[3][L];
    T Szz[2][L], Sxz[2][L], Syz[2][L], Hh[2];
    double nsum[L];

    // u^n and moduli of plane k (global index kk, any integer k0-1 .. k1), and
    // u^{n-1} / force of plane k when it is a face plane; into set R
    auto fetch = [&](int64_t kk, auto Rc) {
      constexpr int R = decltype(Rc)::value;
      const int64_t kw = kk < 0 ? kk + nz : (kk >= nz ? kk - nz : kk);
      const int64_t o = col + plane * kw;
      Ko[R] = Kf[o];
      Go[R] = Gf[o];
      const bool face = kk >= k0 && kk < k1 && interior;
#pragma unroll
      for (int l = 0; l < L; ++l) {
        Ux[R][l] = Uy[R][l] = Uz[R][l] = T(0);
        Vo0[R][l] = Vo1[R][l] = Vo2[R][l] = F0[R][l] = F1[R][l] = F2[R][l] = T(0);
        if (act & (1u << l)) {
          Ux[R][l] = ucur[l][o];
          Uy[R][l] = ucur[l][N + o];
          Uz[R][l] = ucur[l][2 * N + o];
          if (face && !first) {
            Vo0[R][l] = uold[l][o];
            Vo1[R][l] = uold[l][N + o];
            Vo2[R][l] = uold[l][2 * N + o];
          }
          if (face && anyf && hasf[l]) {
            F0[R][l] = frc[l][o];
            F1[R][l] = frc[l][N + o];
            F2[R][l] = frc[l][2 * N + o];
          }
        }
      }
    };

#pragma unroll
    for (int l = 0; l < L; ++l) {
      Szz[1][l] = Sxz[1][l] = Syz[1][l] = T(0);
      nsum[l] = 0.0;
    }
    Hh[1] = T(1);
    fetch(k0 - 1, std::integral_constant<int, 0>{});
    fetch(k0, std::integral_constant<int, 1>{});
    sG[0][tid] = Go[0];
    int par = 0;  // plane parity for the LDS moduli and the carried stresses

    // process plane k whose data is in set A, next plane in set B; request
    // plane k+2 into set C
    auto plane_step = [&](int64_t k, auto Ac, auto Bc, auto Cc, auto Pc) {
      constexpr int A = decltype(Ac)::value;
      constexpr int B = decltype(Bc)::value;
      constexpr int C = decltype(Cc)::value;
      constexpr int P = decltype(Pc)::value;
      constexpr int Q = 1 - P;
      const int64_t kw = k < 0 ? k + nz : k;
      const int64_t oc = col + plane * kw;
      const bool face = k >= k0 && interior;
      if (k + 2 <= k1) fetch(k + 2, std::integral_constant<int, C>{});
      T* gk = sG[P];
      T* gn = sG[Q];
      gn[tid] = Go[B];
      Hh[P] = Ko[A] + T(4.0 / 3.0) * Go[A];
      sH[tid] = Hh[P];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        S(l, 0)[tid] = Ux[A][l];
        S(l, 1)[tid] = Uy[A][l];
        S(l, 2)[tid] = Uz[B][l];
      }
      __syncthreads();
      const T lam = Ko[A] - T(2.0 / 3.0) * Go[A];
      const T twoG = T(2) * Go[A];
      const T ik = recip(gk[tid]), ikx = recip(gk[xm]), iky = recip(gk[ym]);
      const T in = recip(gn[tid]), inx = recip(gn[xm]), iny = recip(gn[ym]);
      const T G2xy = T(8) * recip(recip(gk[xmym]) + iky + ikx + ik);
      const T G2xz = T(8) * recip(ikx + ik + inx + in);
      const T G2yz = T(8) * recip(iky + ik + iny + in);
      const T sfx = sfac * recip(tmax(sH[xm], Hh[P]));
      const T sfy = sfac * recip(tmax(sH[ym], Hh[P]));
      const T sfz = sfac * recip(tmax(Hh[Q], Hh[P]));
      T sxx[L], syy[L], szz[L], sxy[L], sxz_n[L], syz_n[L];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        const T ux = Ux[A][l], uy = Uy[A][l], uz = Uz[A][l];
        const T unx = Ux[B][l], uny = Uy[B][l], unz = Uz[B][l];
        const T* sUx = S(l, 0);
        const T* sUy = S(l, 1);
        const T* sUz = S(l, 2);
        const T exx = E[l][0] + (sUx[xp] - ux) * rhx;
        const T eyy = E[l][1] + (sUy[yp] - uy) * rhy;
        const T ezz = E[l][2] + (unz - uz) * rhz;
        const T th = exx + eyy + ezz;
        sxx[l] = lam * th + twoG * exx;
        syy[l] = lam * th + twoG * eyy;
        szz[l] = lam * th + twoG * ezz;
        sxy[l] = G2xy * (E[l][5] + T(0.5) * ((ux - sUx[ym]) * rhy + (uy - sUy[xm]) * rhx));
        sxz_n[l] = G2xz * (E[l][4] + T(0.5) * ((unx - ux) * rhz + (unz - sUz[xm]) * rhx));
        syz_n[l] = G2yz * (E[l][3] + T(0.5) * ((uny - uy) * rhz + (unz - sUz[ym]) * rhy));
        S(l, 3)[tid] = sxx[l];
        S(l, 4)[tid] = syy[l];
        S(l, 5)[tid] = sxy[l];
        S(l, 6)[tid] = Sxz[Q][l];
        S(l, 7)[tid] = Syz[Q][l];
      }
      __syncthreads();
#pragma unroll
      for (int l = 0; l < L; ++l) {
        if (face && (act & (1u << l))) {
          const T* sSxx = S(l, 3);
          const T* sSyy = S(l, 4);
          const T* sSxy = S(l, 5);
          const T* sSxz = S(l, 6);
          const T* sSyz = S(l, 7);
          const T sxz_c = Sxz[Q][l], syz_c = Syz[Q][l];
          T rx = (sxx[l] - sSxx[xm]) * rhx + (sSxy[yp] - sxy[l]) * rhy + (sxz_n[l] - sxz_c) * rhz;
          T ry = (sSxy[xp] - sxy[l]) * rhx + (syy[l] - sSyy[ym]) * rhy + (syz_n[l] - syz_c) * rhz;
          T rz = (sSxz[xp] - sxz_c) * rhx + (sSyz[yp] - syz_c) * rhy + (szz[l] - Szz[Q][l]) * rhz;
          rx += F0[A][l];
          ry += F1[A][l];
          rz += F2[A][l];
          if (partials != nullptr)
            nsum[l] += (double)rx * (double)rx + (double)ry * (double)ry + (double)rz * (double)rz;
          const T ux = Ux[A][l], uy = Uy[A][l], uz = Uz[A][l];
          uold[l][oc] = ux + mom * (ux - Vo0[A][l]) + sfx * rx;
          uold[l][N + oc] = uy + mom * (uy - Vo1[A][l]) + sfy * ry;
          uold[l][2 * N + oc] = uz + mom * (uz - Vo2[A][l]) + sfz * rz;
        }
        Szz[P][l] = szz[l];
        Sxz[P][l] = sxz_n[l];
        Syz[P][l] = syz_n[l];
      }
    };

    // planes k0-1, k0, ..., k1-1; the data sets rotate with period 3 and the
    // parity with period 2, so the loop body covers six planes
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    (void)par;
    for (int64_t k = k0 - 1; k < k1; k += 6) {
      plane_step(k, I0{}, I1{}, I2{}, I0{});
      if (k + 1 >= k1) break;
      plane_step(k + 1, I1{}, I2{}, I0{}, I1{});
      if (k + 2 >= k1) break;
      plane_step(k + 2, I2{}, I0{}, I1{}, I0{});
      if (k + 3 >= k1) break;
      plane_step(k + 3, I0{}, I1{}, I2{}, I1{});
      if (k + 4 >= k1) break;
      plane_step(k + 4, I1{}, I2{}, I0{}, I0{});
      if (k + 5 >= k1) break;
      plane_step(k + 5, I2{}, I0{}, I1{}, I1{});
    }

    if (partials != nullptr) {
      double tot[kMaxLoads] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int l = 0; l < L; ++l) {
        if (!(act & (1u << l))) continue;
        tot[s0 + l] = block_sum(nsum[l], red);
      }
      if (tid == 0)
        for (int q = 0; q < kMaxLoads; ++q) partials[(int64_t)w * kMaxLoads + q] = tot[q];
    }
    __syncthreads();
  }
}

// One load per block, no LDS and no barriers: every thread is an interior
// column of the tile and reads the in-plane neighbours it needs (8 columns)
// directly through the caches; stresses of neighbouring nodes are recomputed
// instead of exchanged.  Waves never wait for each other, so memory latency is
// hidden by the other waves of the CU.  Same arithmetic, in the same order, as
// the LDS kernels.
template <typename T, bool HI>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 512), amdgpu_waves_per_eu(HI ? 6 : 4)))
step_kernel_c(const SampleDesc<T>* __restrict__ samples, const WorkItem* __restrict__ work, int nwork, int bx,
              int by, int parity, int first, double* __restrict__ partials) {
  __shared__ double red[16];
  const int TX = bx - 2, TY = by - 2;
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;

  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const WorkItem wi = work[w];
    if (wi.sample < 0) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      continue;
    }
    const SampleDesc<T>& sd = samples[wi.sample];
    const int l = wi.slot0;
    if (!((sd.active >> l) & 1u)) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      continue;
    }
    const int64_t nx = sd.nx, ny = sd.ny, nz = sd.nz, N = sd.N, plane = nx * ny;
    const T rhx = sd.rhx, rhy = sd.rhy, rhz = sd.rhz;
    const T mom = first ? T(0) : sd.mom;
    const T sfac = first ? sd.sfac_first : sd.sfac;
    const int64_t gi = (int64_t)wi.tx * TX + tx, gj = (int64_t)wi.ty * TY + ty;
    const bool valid = ty < TY && gi < nx && gj < ny;
    const int64_t k0 = (int64_t)wi.kz * sd.kc;
    const int64_t k1 = k0 + sd.kc < nz ? k0 + sd.kc : nz;
    double nsum = 0.0;

    if (valid) {
      const T E0 = sd.E[l][0], E1 = sd.E[l][1], E2 = sd.E[l][2], E3 = sd.E[l][3], E4 = sd.E[l][4],
              E5 = sd.E[l][5];
      const GLOBAL_AS T* __restrict__ Kf = gconst(sd.K);
      const GLOBAL_AS T* __restrict__ Gf = gconst(sd.G);
      const GLOBAL_AS T* __restrict__ ux_ = gconst(sd.u[parity][l]);
      const GLOBAL_AS T* __restrict__ uy_ = ux_ + N;
      const GLOBAL_AS T* __restrict__ uz_ = ux_ + 2 * N;
      GLOBAL_AS T* __restrict__ ox_ = gmut(sd.u[parity ^ 1][l]);
      GLOBAL_AS T* __restrict__ oy_ = ox_ + N;
      GLOBAL_AS T* __restrict__ oz_ = ox_ + 2 * N;
      const bool hasf = sd.force[l] != nullptr;
      const GLOBAL_AS T* __restrict__ fx_ = gconst(sd.force[l]);
      const GLOBAL_AS T* __restrict__ fy_ = fx_ + N;
      const GLOBAL_AS T* __restrict__ fz_ = fx_ + 2 * N;

      // in-plane column offsets: 0 = (0,0), P = +1, M = -1 (x first, then y)
      const int64_t im = gi == 0 ? nx - 1 : gi - 1, ip = gi + 1 == nx ? 0 : gi + 1;
      const int64_t jm = gj == 0 ? ny - 1 : gj - 1, jp = gj + 1 == ny ? 0 : gj + 1;
      // byte offsets within a plane (a plane is far below 4 GiB), so loads take a
      // scalar base plus a 32-bit vector offset
      constexpr uint32_t W = sizeof(T);
      const uint32_t c00 = (uint32_t)(gi + nx * gj) * W, cP0 = (uint32_t)(ip + nx * gj) * W;
      const uint32_t cM0 = (uint32_t)(im + nx * gj) * W, c0M = (uint32_t)(gi + nx * jm) * W;
      const uint32_t c0P = (uint32_t)(gi + nx * jp) * W, cPM = (uint32_t)(ip + nx * jm) * W;
      const uint32_t cMP = (uint32_t)(im + nx * jp) * W, cMM = (uint32_t)(im + nx * jm) * W;
      auto at = [](const GLOBAL_AS T* p, uint32_t off) -> T {
        return *(const GLOBAL_AS T*)((const GLOBAL_AS char*)p + off);
      };

      // one plane of data: u_x at 00 P0 M0 0M PM 0P; u_y at 00 0P M0 MP 0M P0;
      // u_z at 00 M0 0M P0 0P; K at 00 M0 0M; 1/G at MM 0M M0 00 PM P0 MP 0P
      struct Plane {
        T x00, xP0, xM0, x0M, xPM, x0P;
        T y00, y0P, yM0, yMP, y0M, yP0;
        T z00, zM0, z0M, zP0, z0P;
        T K00, KM0, K0M, G00, GM0, G0M;
        T iMM, i0M, iM0, i00, iPM, iP0, iMP, i0P;
      };
      auto load = [&](int64_t kk, Plane& q) {
        const int64_t kw = kk < 0 ? kk + nz : (kk >= nz ? kk - nz : kk);
        const int64_t po = plane * kw;
        const GLOBAL_AS T* X = ux_ + po;
        const GLOBAL_AS T* Y = uy_ + po;
        const GLOBAL_AS T* Z = uz_ + po;
        const GLOBAL_AS T* Kp = Kf + po;
        const GLOBAL_AS T* Gp = Gf + po;
        q.x00 = at(X, c00); q.xP0 = at(X, cP0); q.xM0 = at(X, cM0); q.x0M = at(X, c0M); q.xPM = at(X, cPM);
        q.x0P = at(X, c0P);
        q.y00 = at(Y, c00); q.y0P = at(Y, c0P); q.yM0 = at(Y, cM0); q.yMP = at(Y, cMP); q.y0M = at(Y, c0M);
        q.yP0 = at(Y, cP0);
        q.z00 = at(Z, c00); q.zM0 = at(Z, cM0); q.z0M = at(Z, c0M); q.zP0 = at(Z, cP0); q.z0P = at(Z, c0P);
        q.K00 = at(Kp, c00); q.KM0 = at(Kp, cM0); q.K0M = at(Kp, c0M);
        q.G00 = at(Gp, c00); q.GM0 = at(Gp, cM0); q.G0M = at(Gp, c0M);
        q.iMM = recip(at(Gp, cMM)); q.i0M = recip(q.G0M); q.iM0 = recip(q.GM0); q.i00 = recip(q.G00);
        q.iPM = recip(at(Gp, cPM)); q.iP0 = recip(at(Gp, cP0)); q.iMP = recip(at(Gp, cMP)); q.i0P = recip(at(Gp, c0P));
      };

      Plane pl[2];
      T szz_p = T(0), sxz00 = T(0), sxzP0 = T(0), syz00 = T(0), syz0P = T(0), Hp = T(1);
      load(k0 - 1, pl[0]);

      auto step = [&](int64_t k, auto Ac) {
        constexpr int A = decltype(Ac)::value;
        constexpr int B = 1 - A;
        const Plane& a = pl[A];
        Plane& b = pl[B];
        load(k + 1, b);
        const bool face = k >= k0;
        // cells of plane k: 00 (all normal stresses), M0 (xx), 0M (yy)
        const T l00 = a.K00 - T(2.0 / 3.0) * a.G00, t00 = T(2) * a.G00;
        const T lM0 = a.KM0 - T(2.0 / 3.0) * a.GM0, tM0 = T(2) * a.GM0;
        const T l0M = a.K0M - T(2.0 / 3.0) * a.G0M, t0M = T(2) * a.G0M;
        const T exx00 = E0 + (a.xP0 - a.x00) * rhx, eyy00 = E1 + (a.y0P - a.y00) * rhy,
                ezz00 = E2 + (b.z00 - a.z00) * rhz;
        const T th00 = exx00 + eyy00 + ezz00;
        const T sxx00 = l00 * th00 + t00 * exx00, syy00 = l00 * th00 + t00 * eyy00, szz00 = l00 * th00 + t00 * ezz00;
        const T exxM0 = E0 + (a.x00 - a.xM0) * rhx, eyyM0 = E1 + (a.yMP - a.yM0) * rhy,
                ezzM0 = E2 + (b.zM0 - a.zM0) * rhz;
        const T sxxM0 = lM0 * (exxM0 + eyyM0 + ezzM0) + tM0 * exxM0;
        const T exx0M = E0 + (a.xPM - a.x0M) * rhx, eyy0M = E1 + (a.y00 - a.y0M) * rhy,
                ezz0M = E2 + (b.z0M - a.z0M) * rhz;
        const T syy0M = l0M * (exx0M + eyy0M + ezz0M) + t0M * eyy0M;
        // xy-edges of plane k at 00, P0, 0P
        const T Gxy00 = T(8) * recip(a.iMM + a.i0M + a.iM0 + a.i00);
        const T GxyP0 = T(8) * recip(a.i0M + a.iPM + a.i00 + a.iP0);
        const T Gxy0P = T(8) * recip(a.iM0 + a.i00 + a.iMP + a.i0P);
        const T sxy00 = Gxy00 * (E5 + T(0.5) * ((a.x00 - a.x0M) * rhy + (a.y00 - a.yM0) * rhx));
        const T sxyP0 = GxyP0 * (E5 + T(0.5) * ((a.xP0 - a.xPM) * rhy + (a.yP0 - a.y00) * rhx));
        const T sxy0P = Gxy0P * (E5 + T(0.5) * ((a.x0P - a.x00) * rhy + (a.y0P - a.yMP) * rhx));
        // xz- and yz-edges of plane k+1
        const T Gxz00 = T(8) * recip(a.iM0 + a.i00 + b.iM0 + b.i00);
        const T GxzP0 = T(8) * recip(a.i00 + a.iP0 + b.i00 + b.iP0);
        const T Gyz00 = T(8) * recip(a.i0M + a.i00 + b.i0M + b.i00);
        const T Gyz0P = T(8) * recip(a.i00 + a.i0P + b.i00 + b.i0P);
        const T nxz00 = Gxz00 * (E4 + T(0.5) * ((b.x00 - a.x00) * rhz + (b.z00 - b.zM0) * rhx));
        const T nxzP0 = GxzP0 * (E4 + T(0.5) * ((b.xP0 - a.xP0) * rhz + (b.zP0 - b.z00) * rhx));
        const T nyz00 = Gyz00 * (E3 + T(0.5) * ((b.y00 - a.y00) * rhz + (b.z00 - b.z0M) * rhy));
        const T nyz0P = Gyz0P * (E3 + T(0.5) * ((b.y0P - a.y0P) * rhz + (b.z0P - b.z00) * rhy));
        const T H00 = a.K00 + T(4.0 / 3.0) * a.G00;
        if (face) {
          const int64_t po = plane * (k < 0 ? k + nz : k);
          T rx = (sxx00 - sxxM0) * rhx + (sxy0P - sxy00) * rhy + (nxz00 - sxz00) * rhz;
          T ry = (sxyP0 - sxy00) * rhx + (syy00 - syy0M) * rhy + (nyz00 - syz00) * rhz;
          T rz = (sxzP0 - sxz00) * rhx + (syz0P - syz00) * rhy + (szz00 - szz_p) * rhz;
          if (hasf) {
            rx += at(fx_ + po, c00);
            ry += at(fy_ + po, c00);
            rz += at(fz_ + po, c00);
          }
          nsum += (double)rx * (double)rx + (double)ry * (double)ry + (double)rz * (double)rz;
          const T HM0 = a.KM0 + T(4.0 / 3.0) * a.GM0, H0M = a.K0M + T(4.0 / 3.0) * a.G0M;
          const T sfx = sfac * recip(tmax(HM0, H00));
          const T sfy = sfac * recip(tmax(H0M, H00));
          const T sfz = sfac * recip(tmax(Hp, H00));
          GLOBAL_AS T* px = (GLOBAL_AS T*)((GLOBAL_AS char*)(ox_ + po) + c00);
          GLOBAL_AS T* py = (GLOBAL_AS T*)((GLOBAL_AS char*)(oy_ + po) + c00);
          GLOBAL_AS T* pz = (GLOBAL_AS T*)((GLOBAL_AS char*)(oz_ + po) + c00);
          T vx = T(0), vy = T(0), vz = T(0);
          if (!first) {
            vx = *px;
            vy = *py;
            vz = *pz;
          }
          *px = a.x00 + mom * (a.x00 - vx) + sfx * rx;
          *py = a.y00 + mom * (a.y00 - vy) + sfy * ry;
          *pz = a.z00 + mom * (a.z00 - vz) + sfz * rz;
        }
        szz_p = szz00;
        sxz00 = nxz00;
        sxzP0 = nxzP0;
        syz00 = nyz00;
        syz0P = nyz0P;
        Hp = H00;
      };

      for (int64_t k = k0 - 1; k < k1; k += 2) {
        step(k, std::integral_constant<int, 0>{});
        if (k + 1 < k1) step(k + 1, std::integral_constant<int, 1>{});
      }
    }

    if (partials != nullptr) {
      const double s = block_sum(nsum, red);
      if (tid == 0)
        for (int q = 0; q < kMaxLoads; ++q) partials[(int64_t)w * kMaxLoads + q] = q == l ? s : 0.0;
    }
    __syncthreads();
  }
}

// Orthotropic cells (nine constants per cell, axes aligned with the grid;
// SampleDesc::cst).  One load per block, same z-march and LDS staging as the
// kernels above.  Normal stresses: the 3x3 normal block of the cell's Voigt
// matrix; edge stresses: twice the harmonic mean of C44 (yz), C55 (xz) or C66
// (xy) over the four cells of the edge, times the tensor strain.  A face's step
// stiffness is the larger over its two cells of max(normal constant, the two
// shear constants acting on that displacement component) -- for isotropic
// cells that is K + 4G/3.  MODE 0: iteration; MODE 1: residual into rout.
constexpr int kOrthoArrays = 15;  // LDS arrays of bx*by (rounded) elements

template <typename T, int MODE, typename R>
__global__ void __launch_bounds__(512)
step_kernel_ortho(const SampleDesc<T>* __restrict__ samples, const WorkItem* __restrict__ work, int nwork, int bx,
                  int by, int parity, int first, double* __restrict__ partials, R* const* __restrict__ rout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int nt = blockDim.x;
  T* base = reinterpret_cast<T*>(smem_raw);
  T* s66 = base;                          // 1/C66 of plane k
  T* s55[2] = {base + nt, base + 2 * nt};  // 1/C55 of two planes
  T* s44[2] = {base + 3 * nt, base + 4 * nt};
  T* sHx = base + 5 * nt;
  T* sHy = base + 6 * nt;
  T* sUx = base + 7 * nt;
  T* sUy = base + 8 * nt;
  T* sUz = base + 9 * nt;
  T* sSxx = base + 10 * nt;
  T* sSyy = base + 11 * nt;
  T* sSxy = base + 12 * nt;
  T* sSxz = base + 13 * nt;
  T* sSyz = base + 14 * nt;

  const int tid = threadIdx.x;
  const int tx = tid % bx, ty = tid / bx;
  const int TX = bx - 2, TY = by - 2;
  const int xm = tid > 0 && tx > 0 ? tid - 1 : tid;
  const int xp = tx < bx - 1 && tid + 1 < nt ? tid + 1 : tid;
  const int ym = ty > 0 ? tid - bx : tid;
  const int yp = ty < by - 1 && tid + bx < nt ? tid + bx : tid;
  const int xmym = ty > 0 ? xm - bx : xm;

  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const WorkItem wi = work[w];
    if (wi.sample < 0) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      continue;
    }
    const SampleDesc<T>& sd = samples[wi.sample];
    const int l = wi.slot0;
    if (!((sd.active >> l) & 1u)) {
      if (partials != nullptr && tid < kMaxLoads) partials[(int64_t)w * kMaxLoads + tid] = 0.0;
      continue;
    }
    const int64_t nx = sd.nx, ny = sd.ny, nz = sd.nz, N = sd.N, plane = nx * ny;
    const T rhx = sd.rhx, rhy = sd.rhy, rhz = sd.rhz;
    const T mom = first ? T(0) : sd.mom;
    const T sfac = first ? sd.sfac_first : sd.sfac;
    const int64_t gi = (int64_t)wi.tx * TX + tx - 1, gj = (int64_t)wi.ty * TY + ty - 1;
    const int64_t col = wrap_idx(gi, nx) + nx * wrap_idx(gj, ny);
    const bool interior = tx >= 1 && tx <= TX && ty >= 1 && ty <= TY && gi < nx && gj < ny;
    const int64_t k0 = (int64_t)wi.kz * sd.kc;
    const int64_t k1 = k0 + sd.kc < nz ? k0 + sd.kc : nz;

    const GLOBAL_AS T* __restrict__ cst = gconst(sd.cst);
    const GLOBAL_AS T* ucur = gconst(sd.u[parity][l]);
    GLOBAL_AS T* uold = gmut(sd.u[parity ^ 1][l]);
    const bool hasf = sd.force[l] != nullptr;
    const GLOBAL_AS T* frc = gconst(sd.force[l]);
    const T* E = sd.E[l];
    auto load9 = [&](int64_t o, T* c) {
#pragma unroll
      for (int q = 0; q < 9; ++q) c[q] = cst[q * N + o];
    };

    T cc[9], cn[9];
    T ux, uy, uz, szz_p = T(0), sxz_c = T(0), syz_c = T(0), Hz_p = T(1);
    double nsum = 0.0;
    {
      const int64_t kw = k0 - 1 < 0 ? k0 - 1 + nz : k0 - 1;
      const int64_t o = col + plane * kw;
      ux = ucur[o];
      uy = ucur[N + o];
      uz = ucur[2 * N + o];
      load9(o, cc);
      s55[0][tid] = recip(cc[7]);
      s44[0][tid] = recip(cc[6]);
    }

    for (int64_t k = k0 - 1; k < k1; ++k) {
      const int P = (int)((k - (k0 - 1)) & 1), Q = P ^ 1;
      const int64_t kw = k < 0 ? k + nz : k;
      const int64_t kn = k + 1 >= nz ? k + 1 - nz : k + 1;
      const int64_t oc = col + plane * kw, on = col + plane * kn;
      const bool face = k >= k0 && interior;
      load9(on, cn);
      const T unx = ucur[on], uny = ucur[N + on], unz = ucur[2 * N + on];
      T uo0 = T(0), uo1 = T(0), uo2 = T(0), f0 = T(0), f1 = T(0), f2 = T(0);
      if (face) {
        if (MODE == 0 && !first) {
          uo0 = uold[oc];
          uo1 = uold[N + oc];
          uo2 = uold[2 * N + oc];
        }
        if (hasf) {
          f0 = frc[oc];
          f1 = frc[N + oc];
          f2 = frc[2 * N + oc];
        }
      }
      // cc: this plane's cell; cn: the next plane's
      const T Hx = tmax(cc[0], tmax(cc[8], cc[7]));
      const T Hy = tmax(cc[1], tmax(cc[8], cc[6]));
      const T Hz = tmax(cc[2], tmax(cc[7], cc[6]));
      s66[tid] = recip(cc[8]);
      s55[Q][tid] = recip(cn[7]);
      s44[Q][tid] = recip(cn[6]);
      sHx[tid] = Hx;
      sHy[tid] = Hy;
      sUx[tid] = ux;
      sUy[tid] = uy;
      sUz[tid] = unz;
      __syncthreads();
      const T C66e2 = T(8) * recip(s66[xmym] + s66[ym] + s66[xm] + s66[tid]);
      const T C55e2 = T(8) * recip(s55[P][xm] + s55[P][tid] + s55[Q][xm] + s55[Q][tid]);
      const T C44e2 = T(8) * recip(s44[P][ym] + s44[P][tid] + s44[Q][ym] + s44[Q][tid]);
      const T sfx = sfac * recip(tmax(sHx[xm], Hx));
      const T sfy = sfac * recip(tmax(sHy[ym], Hy));
      const T sfz = sfac * recip(tmax(Hz_p, Hz));
      const T exx = E[0] + (sUx[xp] - ux) * rhx;
      const T eyy = E[1] + (sUy[yp] - uy) * rhy;
      const T ezz = E[2] + (unz - uz) * rhz;
      const T sxx = cc[0] * exx + cc[5] * eyy + cc[4] * ezz;
      const T syy = cc[5] * exx + cc[1] * eyy + cc[3] * ezz;
      const T szz = cc[4] * exx + cc[3] * eyy + cc[2] * ezz;
      const T sxy = C66e2 * (E[5] + T(0.5) * ((ux - sUx[ym]) * rhy + (uy - sUy[xm]) * rhx));
      const T sxz_n = C55e2 * (E[4] + T(0.5) * ((unx - ux) * rhz + (unz - sUz[xm]) * rhx));
      const T syz_n = C44e2 * (E[3] + T(0.5) * ((uny - uy) * rhz + (unz - sUz[ym]) * rhy));
      sSxx[tid] = sxx;
      sSyy[tid] = syy;
      sSxy[tid] = sxy;
      sSxz[tid] = sxz_c;
      sSyz[tid] = syz_c;
      __syncthreads();
      if (face) {
        T rx = (sxx - sSxx[xm]) * rhx + (sSxy[yp] - sxy) * rhy + (sxz_n - sxz_c) * rhz;
        T ry = (sSxy[xp] - sxy) * rhx + (syy - sSyy[ym]) * rhy + (syz_n - syz_c) * rhz;
        T rz = (sSxz[xp] - sxz_c) * rhx + (sSyz[yp] - syz_c) * rhy + (szz - szz_p) * rhz;
        rx += f0;
        ry += f1;
        rz += f2;
        if (partials != nullptr) nsum += (double)rx * (double)rx + (double)ry * (double)ry + (double)rz * (double)rz;
        if (MODE == 0) {
          uold[oc] = ux + mom * (ux - uo0) + sfx * rx;
          uold[N + oc] = uy + mom * (uy - uo1) + sfy * ry;
          uold[2 * N + oc] = uz + mom * (uz - uo2) + sfz * rz;
        } else {
          GLOBAL_AS R* ro = rout != nullptr ? gmut(rout[l]) : nullptr;
          if (ro != nullptr) {
            ro[oc] = (R)rx;
            ro[N + oc] = (R)ry;
            ro[2 * N + oc] = (R)rz;
          }
        }
      }
      szz_p = szz;
      sxz_c = sxz_n;
      syz_c = syz_n;
      Hz_p = Hz;
      ux = unx;
      uy = uny;
      uz = unz;
#pragma unroll
      for (int q = 0; q < 9; ++q) cc[q] = cn[q];
    }

    if (partials != nullptr) {
      const double s = block_sum(nsum, red);
      if (tid == 0)
        for (int q = 0; q < kMaxLoads; ++q) partials[(int64_t)w * kMaxLoads + q] = q == l ? s : 0.0;
    }
    __syncthreads();
  }
}

__global__ void finalize_norms_kernel(const int* __restrict__ ranges, const double* __restrict__ partials,
                                      double* __restrict__ out) {
  __shared__ double red[16];
  const int s = blockIdx.x / kMaxLoads, l = blockIdx.x % kMaxLoads;
  const int b = ranges[2 * s], e = ranges[2 * s + 1];
  double v = 0.0;
  for (int w = b + threadIdx.x; w < e; w += blockDim.x) v += partials[(int64_t)w * kMaxLoads + l];
  v = block_sum(v, red);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// ---- FP64 volume averages ----------------------------------------------------

__global__ void average_partials_kernel(int64_t nx, int64_t ny, int64_t nz, double rhx, double rhy, double rhz,
                                        const double* __restrict__ K, const double* __restrict__ G, double E0,
                                        double E1, double E2, double E3, double E4, double E5,
                                        const double* __restrict__ u, double* __restrict__ partials, int walls) {
  __shared__ double red[16];
  const int64_t N = nx * ny * nz;
  const double* ux = u;
  const double* uy = u + N;
  const double* uz = u + 2 * N;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    const int64_t ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
    const int64_t jp = j + 1 == ny ? 0 : j + 1, jm = j == 0 ? ny - 1 : j - 1;
    const int64_t kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;
    auto at = [&](int64_t a, int64_t b, int64_t d) { return a + nx * (b + ny * d); };
    const double exx = E0 + (ux[at(ip, j, k)] - ux[c]) * rhx;
    const double eyy = E1 + (uy[at(i, jp, k)] - uy[c]) * rhy;
    const double ezz = E2 + (uz[at(i, j, kp)] - uz[c]) * rhz;
    const double th = exx + eyy + ezz;
    const double lam = K[c] - 2.0 / 3.0 * G[c];
    acc[0] += lam * th + 2.0 * G[c] * exx;
    acc[1] += lam * th + 2.0 * G[c] * eyy;
    acc[2] += lam * th + 2.0 * G[c] * ezz;
    const double gc = 1.0 / G[c];
    double gyz = 8.0 / (gc + 1.0 / G[at(i, jm, k)] + 1.0 / G[at(i, j, km)] + 1.0 / G[at(i, jm, km)]);
    double gxz = 8.0 / (gc + 1.0 / G[at(im, j, k)] + 1.0 / G[at(i, j, km)] + 1.0 / G[at(im, j, km)]);
    double gxy = 8.0 / (gc + 1.0 / G[at(im, j, k)] + 1.0 / G[at(i, jm, k)] + 1.0 / G[at(im, jm, k)]);
    double syz = gyz * (E3 + 0.5 * ((uy[c] - uy[at(i, j, km)]) * rhz + (uz[c] - uz[at(i, jm, k)]) * rhy));
    double sxz = gxz * (E4 + 0.5 * ((ux[c] - ux[at(i, j, km)]) * rhz + (uz[c] - uz[at(im, j, k)]) * rhx));
    double sxy = gxy * (E5 + 0.5 * ((ux[c] - ux[at(i, jm, k)]) * rhy + (uy[c] - uy[at(im, j, k)]) * rhx));
    if (walls) {
      // walls = 1 (normal test): every edge in a boundary plane carries no shear
      // stress.  walls = 3, 4, 5 (simple-shear test of yz, xz, xy): so do the
      // other components' boundary edges; the test's own component is computed
      // as inside on the walls normal to the sheared direction and, on the
      // loaded walls, is the mean of the two half edges (one per side of the
      // box: one-sided derivative to the wall, harmonic mean of the half's two
      // cells, 2 G = 4 / (1/G + 1/G'))
      const int64_t kt = nz - 1, jt = ny - 1;
      if (walls == 3) {
        if (k == 0) {
          const double t = 0.5 * (uz[c] - uz[at(i, jm, 0)]) * rhy;
          syz = 0.5 * (4.0 / (gc + 1.0 / G[at(i, jm, 0)]) * (E3 + uy[c] * rhz + t) +
                       4.0 / (1.0 / G[at(i, j, kt)] + 1.0 / G[at(i, jm, kt)]) * (E3 - uy[at(i, j, kt)] * rhz + t));
        }
      } else if (j == 0 || k == 0) {
        syz = 0.0;
      }
      if (walls == 4) {
        if (k == 0) {
          const double t = 0.5 * (uz[c] - uz[at(im, j, 0)]) * rhx;
          sxz = 0.5 * (4.0 / (gc + 1.0 / G[at(im, j, 0)]) * (E4 + ux[c] * rhz + t) +
                       4.0 / (1.0 / G[at(i, j, kt)] + 1.0 / G[at(im, j, kt)]) * (E4 - ux[at(i, j, kt)] * rhz + t));
        }
      } else if (i == 0 || k == 0) {
        sxz = 0.0;
      }
      if (walls == 5) {
        if (j == 0) {
          const double t = 0.5 * (uy[c] - uy[at(im, 0, k)]) * rhx;
          sxy = 0.5 * (4.0 / (gc + 1.0 / G[at(im, 0, k)]) * (E5 + ux[c] * rhy + t) +
                       4.0 / (1.0 / G[at(i, jt, k)] + 1.0 / G[at(im, jt, k)]) * (E5 - ux[at(i, jt, k)] * rhy + t));
        }
      } else if (i == 0 || j == 0) {
        sxy = 0.0;
      }
    }
    acc[3] += syz;
    acc[4] += sxz;
    acc[5] += sxy;
  }
  for (int q = 0; q < 6; ++q) {
    const double s = block_sum(acc[q], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 6 + q] = s;
  }
}

// FP64 stress averages for orthotropic cells (c: 9N constants).
__global__ void average_partials_ortho_kernel(int64_t nx, int64_t ny, int64_t nz, double rhx, double rhy,
                                              double rhz, const double* __restrict__ cst, double E0, double E1,
                                              double E2, double E3, double E4, double E5,
                                              const double* __restrict__ u, double* __restrict__ partials) {
  __shared__ double red[16];
  const int64_t N = nx * ny * nz;
  const double* ux = u;
  const double* uy = u + N;
  const double* uz = u + 2 * N;
  const double* C44 = cst + 6 * N;
  const double* C55 = cst + 7 * N;
  const double* C66 = cst + 8 * N;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    const int64_t ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
    const int64_t jp = j + 1 == ny ? 0 : j + 1, jm = j == 0 ? ny - 1 : j - 1;
    const int64_t kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;
    auto at = [&](int64_t a, int64_t b, int64_t d) { return a + nx * (b + ny * d); };
    const double exx = E0 + (ux[at(ip, j, k)] - ux[c]) * rhx;
    const double eyy = E1 + (uy[at(i, jp, k)] - uy[c]) * rhy;
    const double ezz = E2 + (uz[at(i, j, kp)] - uz[c]) * rhz;
    const double C11 = cst[c], C22 = cst[N + c], C33 = cst[2 * N + c];
    const double C23 = cst[3 * N + c], C13 = cst[4 * N + c], C12 = cst[5 * N + c];
    acc[0] += C11 * exx + C12 * eyy + C13 * ezz;
    acc[1] += C12 * exx + C22 * eyy + C23 * ezz;
    acc[2] += C13 * exx + C23 * eyy + C33 * ezz;
    const double cyz = 8.0 / (1.0 / C44[c] + 1.0 / C44[at(i, jm, k)] + 1.0 / C44[at(i, j, km)] + 1.0 / C44[at(i, jm, km)]);
    const double cxz = 8.0 / (1.0 / C55[c] + 1.0 / C55[at(im, j, k)] + 1.0 / C55[at(i, j, km)] + 1.0 / C55[at(im, j, km)]);
    const double cxy = 8.0 / (1.0 / C66[c] + 1.0 / C66[at(im, j, k)] + 1.0 / C66[at(i, jm, k)] + 1.0 / C66[at(im, jm, k)]);
    acc[3] += cyz * (E3 + 0.5 * ((uy[c] - uy[at(i, j, km)]) * rhz + (uz[c] - uz[at(i, jm, k)]) * rhy));
    acc[4] += cxz * (E4 + 0.5 * ((ux[c] - ux[at(i, j, km)]) * rhz + (uz[c] - uz[at(im, j, k)]) * rhx));
    acc[5] += cxy * (E5 + 0.5 * ((ux[c] - ux[at(i, jm, k)]) * rhy + (uy[c] - uy[at(im, j, k)]) * rhx));
  }
  for (int q = 0; q < 6; ++q) {
    const double s = block_sum(acc[q], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 6 + q] = s;
  }
}

// Orthotropic constants checks: per-block flag 1 when some cell's diagonal
// constant is not finite and > 0 or its 3x3 normal block is not positive
// definite (leading minors).
template <typename T>
__global__ void check_ortho_kernel(const T* __restrict__ c, int64_t n, int* __restrict__ bad) {
  __shared__ double red[16];
  double b = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const double C11 = c[t], C22 = c[n + t], C33 = c[2 * n + t], C23 = c[3 * n + t], C13 = c[4 * n + t],
                 C12 = c[5 * n + t], C44 = c[6 * n + t], C55 = c[7 * n + t], C66 = c[8 * n + t];
    bool ok = isfinite(C11) && isfinite(C22) && isfinite(C33) && isfinite(C23) && isfinite(C13) && isfinite(C12) &&
              isfinite(C44) && isfinite(C55) && isfinite(C66);
    ok = ok && C11 > 0.0 && C22 > 0.0 && C33 > 0.0 && C44 > 0.0 && C55 > 0.0 && C66 > 0.0;
    const double m2 = C11 * C22 - C12 * C12;
    const double m3 = C11 * (C22 * C33 - C23 * C23) - C12 * (C12 * C33 - C23 * C13) + C13 * (C12 * C23 - C22 * C13);
    ok = ok && m2 > 0.0 && m3 > 0.0;
    if (!ok) b = 1.0;
  }
  b = block_sum(b, red);
  if (threadIdx.x == 0) bad[blockIdx.x] = b > 0.0 ? 1 : 0;
}

// ---- general anisotropic (triclinic) cells ------------------------------------
//
// Reading of the coupled law on the staggered grid (the paper's perspectives,
// items 2-3): each cell is split into eight corner octants; octant (a, b, c),
// at the cell's corner (i+a, j+b, k+c), takes the cell's normal strains and,
// for each shear component, the strain of that component's edge meeting the
// corner weighted by w = S_e / S_cell (S: the component's diagonal constant C44,
// C55 or C66; S_e: its harmonic mean over the edge's four cells).  The energy is
// sum over cells of 1/8 sum over octants of 1/2 eps_o . C eps_o, so a cell's
// normal stresses are the octant mean of C eps_o's normal rows and an edge's
// shear stress sums, over its four cells and their two octants at the edge,
// w/8 times the shear row.  One iteration is four launches over the cells of
// sample 0, load slot 0 (the engine runs such materials one load at a time):
// strains into scratch, stresses (cells) and each cell's share of its twelve
// edges' stresses, the gather of those shares into edge stresses, and the
// update (or residual).  Scratch per sample (SampleDesc::tscr): strains 6N
// (xx yy zz at cells, engineering yz xz xy at edges), stresses 6N, shares 12N.
// The constants are the upper triangle of the 6x6 Voigt matrix, row by row.

__device__ __forceinline__ int tri_q(int r, int q) {
  const int a = r < q ? r : q, b = r < q ? q : r;
  return 6 * a - a * (a - 1) / 2 + (b - a);
}

__device__ __forceinline__ int64_t tri_at(int64_t i, int64_t j, int64_t k, int64_t nx, int64_t ny, int64_t nz) {
  i = i < 0 ? i + nx : (i >= nx ? i - nx : i);
  j = j < 0 ? j + ny : (j >= ny ? j - ny : j);
  k = k < 0 ? k + nz : (k >= nz ? k - nz : k);
  return i + nx * (j + ny * k);
}

// Strains of u^parity (load slot 0) under the slot's macroscopic strain.
template <typename T>
__global__ void tri_strain_kernel(const SampleDesc<T>* __restrict__ samples, int parity) {
  const SampleDesc<T>& sd = samples[0];
  if (!(sd.active & 1u)) return;
  const int64_t nx = sd.nx, ny = sd.ny, nz = sd.nz, N = sd.N;
  const T* ux = sd.u[parity][0];
  const T* uy = ux + N;
  const T* uz = ux + 2 * N;
  T* eps = sd.tscr;
  const T E0 = sd.E[0][0], E1 = sd.E[0][1], E2 = sd.E[0][2];
  const T G3 = T(2) * sd.E[0][3], G4 = T(2) * sd.E[0][4], G5 = T(2) * sd.E[0][5];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    eps[c] = E0 + (ux[tri_at(i + 1, j, k, nx, ny, nz)] - ux[c]) * sd.rhx;
    eps[N + c] = E1 + (uy[tri_at(i, j + 1, k, nx, ny, nz)] - uy[c]) * sd.rhy;
    eps[2 * N + c] = E2 + (uz[tri_at(i, j, k + 1, nx, ny, nz)] - uz[c]) * sd.rhz;
    eps[3 * N + c] = G3 + (uy[c] - uy[tri_at(i, j, k - 1, nx, ny, nz)]) * sd.rhz +
                     (uz[c] - uz[tri_at(i, j - 1, k, nx, ny, nz)]) * sd.rhy;
    eps[4 * N + c] = G4 + (ux[c] - ux[tri_at(i, j, k - 1, nx, ny, nz)]) * sd.rhz +
                     (uz[c] - uz[tri_at(i - 1, j, k, nx, ny, nz)]) * sd.rhx;
    eps[5 * N + c] = G5 + (ux[c] - ux[tri_at(i, j - 1, k, nx, ny, nz)]) * sd.rhy +
                     (uy[c] - uy[tri_at(i - 1, j, k, nx, ny, nz)]) * sd.rhx;
  }
}

// Normal stresses of every cell and its shares of the stresses of its twelve
// edges: share (s, p) of component s (0 yz, 1 xz, 2 xy) at the cell's corner
// pair p (yz: b + 2c, xz: a + 2c, xy: a + 2b) goes to tscr[(12 + 4 s + p) N + cell].
template <typename T>
__global__ void tri_stress_kernel(const SampleDesc<T>* __restrict__ samples) {
  const SampleDesc<T>& sd = samples[0];
  if (!(sd.active & 1u)) return;
  const int64_t nx = sd.nx, ny = sd.ny, nz = sd.nz, N = sd.N;
  const T* eps = sd.tscr;
  T* sig = sd.tscr + 6 * N;
  T* share = sd.tscr + 12 * N;
  const T* se = sd.tse;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    T M[21];
#pragma unroll
    for (int q = 0; q < 21; ++q) M[q] = sd.c21[q * N + c];
    const T en[3] = {eps[c], eps[N + c], eps[2 * N + c]};
    // weights w = S_e / S_cell and weighted strains of the twelve edges
    T wyz[2][2], wxz[2][2], wxy[2][2], gyz[2][2], gxz[2][2], gxy[2][2];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int u0 = p & 1, u1 = p >> 1;
      const int64_t eyz = tri_at(i, j + u0, k + u1, nx, ny, nz);  // yz: (b, c) = (u0, u1)
      const int64_t exz = tri_at(i + u0, j, k + u1, nx, ny, nz);  // xz: (a, c)
      const int64_t exy = tri_at(i + u0, j + u1, k, nx, ny, nz);  // xy: (a, b)
      wyz[u0][u1] = se[eyz] / M[15];
      wxz[u0][u1] = se[N + exz] / M[18];
      wxy[u0][u1] = se[2 * N + exy] / M[20];
      gyz[u0][u1] = wyz[u0][u1] * eps[3 * N + eyz];
      gxz[u0][u1] = wxz[u0][u1] * eps[4 * N + exz];
      gxy[u0][u1] = wxy[u0][u1] * eps[5 * N + exy];
    }
    T sn[3] = {T(0), T(0), T(0)};
    T tyz[2][2] = {{T(0), T(0)}, {T(0), T(0)}}, txz[2][2] = {{T(0), T(0)}, {T(0), T(0)}},
      txy[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int a = o & 1, b = (o >> 1) & 1, cc = o >> 2;
      const T v[6] = {en[0], en[1], en[2], gyz[b][cc], gxz[a][cc], gxy[a][b]};
      T row[6];
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        T acc = T(0);
#pragma unroll
        for (int q = 0; q < 6; ++q) acc += M[tri_q(r, q)] * v[q];
        row[r] = acc;
      }
      sn[0] += row[0];
      sn[1] += row[1];
      sn[2] += row[2];
      tyz[b][cc] += row[3];
      txz[a][cc] += row[4];
      txy[a][b] += row[5];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) sig[r * N + c] = sn[r] * T(0.125);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int u0 = p & 1, u1 = p >> 1;
      share[(0 + p) * N + c] = T(0.125) * wyz[u0][u1] * tyz[u0][u1];
      share[(4 + p) * N + c] = T(0.125) * wxz[u0][u1] * txz[u0][u1];
      share[(8 + p) * N + c] = T(0.125) * wxy[u0][u1] * txy[u0][u1];
    }
  }
}

// Edge stresses: each edge sums the shares of its four cells.
template <typename T>
__global__ void tri_gather_kernel(const SampleDesc<T>* __restrict__ samples) {
  const SampleDesc<T>& sd = samples[0];
  if (!(sd.active & 1u)) return;
  const int64_t nx = sd.nx, ny = sd.ny, nz = sd.nz, N = sd.N;
  T* sig = sd.tscr + 6 * N;
  const T* share = sd.tscr + 12 * N;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    T tyz = T(0), txz = T(0), txy = T(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int q0 = q & 1, q1 = q >> 1;
      const int p = (1 - q0) + 2 * (1 - q1);  // the edge's corner pair in that cell
      tyz += share[(0 + p) * N + tri_at(i, j - 1 + q0, k - 1 + q1, nx, ny, nz)];
      txz += share[(4 + p) * N + tri_at(i - 1 + q0, j, k - 1 + q1, nx, ny, nz)];
      txy += share[(8 + p) * N + tri_at(i - 1 + q0, j - 1 + q1, k, nx, ny, nz)];
    }
    sig[3 * N + c] = tyz;
    sig[4 * N + c] = txz;
    sig[5 * N + c] = txy;
  }
}

// Out-of-balance force at the faces, plus the slot's body force.  MODE 0: the
// heavy-ball update of u^parity into the other buffer (step factor sfac times
// the face's 1/H, SampleDesc::tihf); MODE 1: write the residual to rout[0].
// The grid has one block per work item; block w writes its squared-norm partial
// to partials[w * kMaxLoads] (and zeros for the other slots).
template <typename T, int MODE, typename R>
__global__ void __launch_bounds__(256) tri_update_kernel(const SampleDesc<T>* __restrict__ samples, int parity,
                                                         int first, double* __restrict__ partials,
                                                         R* const* __restrict__ rout) {
  __shared__ double red[16];
  const SampleDesc<T>& sd = samples[0];
  const int64_t nx = sd.nx, ny = sd.ny, nz = sd.nz, N = sd.N;
  double nsum = 0.0;
  if (sd.active & 1u) {
    const T* sig = sd.tscr + 6 * N;
    const T* ucur = sd.u[parity][0];
    T* uold = sd.u[parity ^ 1][0];
    const T* f = sd.force[0];
    const T mom = first ? T(0) : sd.mom;
    const T sfac = first ? sd.sfac_first : sd.sfac;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x) {
      const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
      const T* sxx = sig;
      const T* syy = sig + N;
      const T* szz = sig + 2 * N;
      const T* syz = sig + 3 * N;
      const T* sxz = sig + 4 * N;
      const T* sxy = sig + 5 * N;
      T r[3];
      r[0] = (sxx[c] - sxx[tri_at(i - 1, j, k, nx, ny, nz)]) * sd.rhx +
             (sxy[tri_at(i, j + 1, k, nx, ny, nz)] - sxy[c]) * sd.rhy +
             (sxz[tri_at(i, j, k + 1, nx, ny, nz)] - sxz[c]) * sd.rhz;
      r[1] = (sxy[tri_at(i + 1, j, k, nx, ny, nz)] - sxy[c]) * sd.rhx +
             (syy[c] - syy[tri_at(i, j - 1, k, nx, ny, nz)]) * sd.rhy +
             (syz[tri_at(i, j, k + 1, nx, ny, nz)] - syz[c]) * sd.rhz;
      r[2] = (sxz[tri_at(i + 1, j, k, nx, ny, nz)] - sxz[c]) * sd.rhx +
             (syz[tri_at(i, j + 1, k, nx, ny, nz)] - syz[c]) * sd.rhy +
             (szz[c] - szz[tri_at(i, j, k - 1, nx, ny, nz)]) * sd.rhz;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (f != nullptr) r[d] += f[d * N + c];
        nsum += (double)r[d] * (double)r[d];
        if constexpr (MODE == 0) {
          const T u = ucur[d * N + c];
          uold[d * N + c] = u + mom * (u - uold[d * N + c]) + sfac * sd.tihf[d * N + c] * r[d];
        } else {
          if (rout != nullptr && rout[0] != nullptr) rout[0][d * N + c] = (R)r[d];
        }
      }
    }
  }
  if (partials != nullptr) {
    const double tot = block_sum(nsum, red);
    if (threadIdx.x == 0)
      for (int q = 0; q < kMaxLoads; ++q) partials[(int64_t)blockIdx.x * kMaxLoads + q] = q == 0 ? tot : 0.0;
  }
}

// Per-cell sums of the six stresses into block partials (6 per block).
__global__ void tri_sum_kernel(const double* __restrict__ sig, int64_t N, double* __restrict__ partials) {
  __shared__ double red[16];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x)
    for (int q = 0; q < 6; ++q) acc[q] += sig[q * N + c];
  for (int q = 0; q < 6; ++q) {
    const double v = block_sum(acc[q], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 6 + q] = v;
  }
}

// Material set-up of general cells (FP64 constants c, 21N): the harmonic edge
// means S_e of C44 / C55 / C66 (se: yz, xz, xy edges, 3N), and 1/H of every face
// (ihf, 3N), H the larger over the face's two cells of the step stiffness: for
// direction d the largest of three diagonal constants (x: 11, 66, 55; y: 22,
// 66, 44; z: 33, 55, 44), each raised by the absolute values of the constants
// of its row that an orthotropic cell does not have.
template <typename T>
__global__ void tri_setup_kernel(const double* __restrict__ cst, int64_t nx, int64_t ny, int64_t nz,
                                 T* __restrict__ se, T* __restrict__ ihf) {
  const int64_t N = nx * ny * nz;
  auto C = [&](int r, int q, int64_t cell) { return cst[(int64_t)tri_q(r, q) * N + cell]; };
  auto hstep = [&](int d, int64_t cell) {
    const int rows[3][3] = {{0, 5, 4}, {1, 5, 3}, {2, 4, 3}};
    double best = 0.0;
    for (int t = 0; t < 3; ++t) {
      const int r = rows[d][t];
      double v = C(r, r, cell);
      for (int q = 0; q < 6; ++q)
        if (!((r < 3 && q < 3) || q == r)) v += fabs(C(r, q, cell));
      best = fmax(best, v);
    }
    return best;
  };
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    se[c] = (T)(4.0 / (1.0 / C(3, 3, tri_at(i, j - 1, k - 1, nx, ny, nz)) + 1.0 / C(3, 3, tri_at(i, j, k - 1, nx, ny, nz)) +
                       1.0 / C(3, 3, tri_at(i, j - 1, k, nx, ny, nz)) + 1.0 / C(3, 3, c)));
    se[N + c] = (T)(4.0 / (1.0 / C(4, 4, tri_at(i - 1, j, k - 1, nx, ny, nz)) + 1.0 / C(4, 4, tri_at(i, j, k - 1, nx, ny, nz)) +
                           1.0 / C(4, 4, tri_at(i - 1, j, k, nx, ny, nz)) + 1.0 / C(4, 4, c)));
    se[2 * N + c] = (T)(4.0 / (1.0 / C(5, 5, tri_at(i - 1, j - 1, k, nx, ny, nz)) + 1.0 / C(5, 5, tri_at(i, j - 1, k, nx, ny, nz)) +
                               1.0 / C(5, 5, tri_at(i - 1, j, k, nx, ny, nz)) + 1.0 / C(5, 5, c)));
    const int64_t nb[3] = {tri_at(i - 1, j, k, nx, ny, nz), tri_at(i, j - 1, k, nx, ny, nz),
                           tri_at(i, j, k - 1, nx, ny, nz)};
    for (int d = 0; d < 3; ++d) ihf[d * N + c] = (T)(1.0 / fmax(hstep(d, c), hstep(d, nb[d])));
  }
}

// Per-block flags: 1 if a cell's 21 constants are not finite or its 6x6 matrix
// is not positive definite (Cholesky in FP64).
__global__ void check_tri_kernel(const double* __restrict__ cst, int64_t n, int* __restrict__ bad) {
  __shared__ double red[16];
  double b = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double L[6][6];
    bool ok = true;
    for (int r = 0; r < 6; ++r)
      for (int q = 0; q < 6; ++q) {
        L[r][q] = cst[(int64_t)tri_q(r, q) * n + t];
        ok = ok && isfinite(L[r][q]);
      }
    for (int q = 0; q < 6 && ok; ++q) {
      double d = L[q][q];
      for (int m = 0; m < q; ++m) d -= L[q][m] * L[q][m];
      if (!(d > 0.0)) {
        ok = false;
        break;
      }
      L[q][q] = sqrt(d);
      for (int r = q + 1; r < 6; ++r) {
        double v = L[r][q];
        for (int m = 0; m < q; ++m) v -= L[r][m] * L[q][m];
        L[r][q] = v / L[q][q];
      }
    }
    if (!ok) b = 1.0;
  }
  b = block_sum(b, red);
  if (threadIdx.x == 0) bad[blockIdx.x] = b > 0.0 ? 1 : 0;
}

__global__ void average_finalize_kernel(const double* __restrict__ partials, int nblocks, double* __restrict__ out6) {
  __shared__ double red[16];
  const int q = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += partials[(int64_t)b * 6 + q];
  v = block_sum(v, red);
  if (threadIdx.x == 0) out6[q] = v;
}

// ---- gradient of sum W_IJ C_IJ ------------------------------------------------

template <typename R>
__global__ void gradient_kernel(int64_t nx, int64_t ny, int64_t nz, double rhx, double rhy, double rhz,
                                const double* __restrict__ K, const double* __restrict__ G, const GradLoads g,
                                R* __restrict__ dK, R* __restrict__ dG) {
  const int64_t N = nx * ny * nz;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  (void)K;
  const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
  auto wr = [](int64_t a, int64_t n) { return a >= n ? a - n : (a < 0 ? a + n : a); };
  auto at = [&](int64_t a, int64_t b, int64_t d) { return wr(a, nx) + nx * (wr(b, ny) + ny * wr(d, nz)); };
  // the twelve edges touching cell c: (orientation, di, dj, dk); orientation
  // 0 = yz, 1 = xz, 2 = xy (Voigt 4, 5, 6)
  const int eo[12][4] = {{2, 0, 0, 0}, {2, 1, 0, 0}, {2, 0, 1, 0}, {2, 1, 1, 0}, {1, 0, 0, 0}, {1, 1, 0, 0},
                         {1, 0, 0, 1}, {1, 1, 0, 1}, {0, 0, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}, {0, 0, 1, 1}};
  double qe[12];
  int64_t ei[12];
  for (int e = 0; e < 12; ++e) {
    const int64_t a = i + eo[e][1], b = j + eo[e][2], d = k + eo[e][3];
    double s;
    if (eo[e][0] == 0)
      s = 1.0 / G[at(a, b, d)] + 1.0 / G[at(a, b - 1, d)] + 1.0 / G[at(a, b, d - 1)] + 1.0 / G[at(a, b - 1, d - 1)];
    else if (eo[e][0] == 1)
      s = 1.0 / G[at(a, b, d)] + 1.0 / G[at(a - 1, b, d)] + 1.0 / G[at(a, b, d - 1)] + 1.0 / G[at(a - 1, b, d - 1)];
    else
      s = 1.0 / G[at(a, b, d)] + 1.0 / G[at(a - 1, b, d)] + 1.0 / G[at(a, b - 1, d)] + 1.0 / G[at(a - 1, b - 1, d)];
    const double Ge = 4.0 / s;
    qe[e] = (Ge / G[c]) * (Ge / G[c]);
    ei[e] = at(a, b, d);
  }
  double th[6], dv[6][3], es[6][12];
  for (int J = 0; J < 6; ++J) {
    if (g.u[J] == nullptr) continue;
    const GLOBAL_AS double* u = gconst(g.u[J]);
    const GLOBAL_AS double* ux = u;
    const GLOBAL_AS double* uy = u + N;
    const GLOBAL_AS double* uz = u + 2 * N;
    const double Ev[6] = {J == 0 ? 1.0 : 0.0, J == 1 ? 1.0 : 0.0, J == 2 ? 1.0 : 0.0,
                          J == 3 ? 0.5 : 0.0, J == 4 ? 0.5 : 0.0, J == 5 ? 0.5 : 0.0};
    const double exx = Ev[0] + (ux[at(i + 1, j, k)] - ux[c]) * rhx;
    const double eyy = Ev[1] + (uy[at(i, j + 1, k)] - uy[c]) * rhy;
    const double ezz = Ev[2] + (uz[at(i, j, k + 1)] - uz[c]) * rhz;
    th[J] = exx + eyy + ezz;
    dv[J][0] = exx - th[J] / 3.0;
    dv[J][1] = eyy - th[J] / 3.0;
    dv[J][2] = ezz - th[J] / 3.0;
    for (int e = 0; e < 12; ++e) {
      const int64_t a = i + eo[e][1], b = j + eo[e][2], d = k + eo[e][3];
      const int64_t o = ei[e];
      double eps;
      if (eo[e][0] == 0)
        eps = Ev[3] + 0.5 * ((uy[o] - uy[at(a, b, d - 1)]) * rhz + (uz[o] - uz[at(a, b - 1, d)]) * rhy);
      else if (eo[e][0] == 1)
        eps = Ev[4] + 0.5 * ((ux[o] - ux[at(a, b, d - 1)]) * rhz + (uz[o] - uz[at(a - 1, b, d)]) * rhx);
      else
        eps = Ev[5] + 0.5 * ((ux[o] - ux[at(a, b - 1, d)]) * rhy + (uy[o] - uy[at(a - 1, b, d)]) * rhx);
      es[J][e] = eps;
    }
  }
  double gk = 0.0, gg = 0.0;
  for (int I = 0; I < 6; ++I) {
    if (g.u[I] == nullptr) continue;
    for (int J = 0; J < 6; ++J) {
      const double w = g.W[I * 6 + J];
      if (w == 0.0 || g.u[J] == nullptr) continue;
      gk += w * th[I] * th[J];
      double dev = dv[I][0] * dv[J][0] + dv[I][1] * dv[J][1] + dv[I][2] * dv[J][2];
      double ed = 0.0;
      for (int e = 0; e < 12; ++e) ed += qe[e] * es[I][e] * es[J][e];
      gg += w * (2.0 * dev + ed);
    }
  }
  dK[c] = (R)(gk / (double)N);
  dG[c] = (R)(gg / (double)N);
}

// ---- elementwise helpers ---------------------------------------------------------

template <typename T>
__global__ void fill_kernel(T* p, int64_t n, T v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    p[t] = v;
}

template <typename A, typename B>
__global__ void convert_kernel(const A* __restrict__ src, B* __restrict__ dst, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = (B)src[t];
}

__global__ void fold_kernel(double* __restrict__ base, float* __restrict__ cur, float* __restrict__ prev, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const float p = prev[t];
    base[t] += (double)p;
    cur[t] = cur[t] - p;
    prev[t] = 0.0f;
  }
}

__global__ void axpy1_kernel(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    dst[t] += src[t];
}

template <typename T>
__global__ void phase_kernel(const uint8_t* __restrict__ ph, int64_t n, const double* __restrict__ Kt,
                             const double* __restrict__ Gt, int nphase, T* __restrict__ K, T* __restrict__ G) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    int p = ph[t];
    if (p >= nphase) p = nphase - 1;  // validated on the host before launch
    K[t] = (T)Kt[p];
    G[t] = (T)Gt[p];
  }
}

// per-block count of moduli that are not finite and positive
template <typename T>
__global__ void check_moduli_kernel(const T* __restrict__ K, const T* __restrict__ G, int64_t n, int* bad) {
  __shared__ double red[16];
  double cnt = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const T a = K[t], b = G[t];
    if (!(a > T(0)) || !(b > T(0)) || !(a < T(1e300)) || !(b < T(1e300))) cnt += 1.0;
  }
  cnt = block_sum(cnt, red);
  if (threadIdx.x == 0) bad[blockIdx.x] = cnt > 0.0 ? 1 : 0;
}

inline int grid_for(int64_t n, int block = 256) {
  int64_t g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

// ---- launch wrappers -------------------------------------------------------------

template <typename T, int L, bool HI>
void launch_step_occ(const SampleDesc<T>* d_samples, const WorkItem* d_work, int nwork, TileShape ts, int parity,
                     int first, double* partials, hipStream_t s, int nt, size_t lds) {
  if constexpr (L == 1) {
    if (ts.pf == 9 && !ts.walls) {  // x-neighbours across lanes (one load per block, bx 16, 32 or 64)
      auto go = [&](auto pal, auto cap, auto frc) {
        hipLaunchKernelGGL((step_kernel_x<T, HI, decltype(pal)::value, decltype(cap)::value, decltype(frc)::value>),
                           dim3(nwork), dim3(nt), 0, s, d_samples, d_work, nwork, ts.bx, ts.by, parity, first,
                           partials);
      };
      auto with_cap = [&](auto pal, auto frc) {
        if (nt <= 256)
          go(pal, std::integral_constant<int, 256>{}, frc);
        else
          go(pal, std::integral_constant<int, 512>{}, frc);
      };
      auto with_frc = [&](auto pal) {
        if (ts.force == 0)
          with_cap(pal, std::integral_constant<int, 0>{});
        else if (ts.force == 1)
          with_cap(pal, std::integral_constant<int, 1>{});
        else
          with_cap(pal, std::integral_constant<int, 2>{});
      };
      if (ts.pal)
        with_frc(std::true_type{});
      else
        with_frc(std::false_type{});
      return;
    }
  }
  if (ts.pf == 5) {
    const int ntc = (((ts.bx - 2) * (ts.by - 2) + 63) / 64) * 64;
    hipLaunchKernelGGL((step_kernel_c<T, HI>), dim3(nwork), dim3(ntc), 0, s, d_samples, d_work, nwork, ts.bx, ts.by,
                       parity, first, partials);
  } else if (ts.pf == 4)
    hipLaunchKernelGGL((step_kernel_p3<T, L, HI>), dim3(nwork), dim3(nt), (size_t)(3 + 8 * L) * nt * sizeof(T), s,
                       d_samples, d_work, nwork, ts.bx, ts.by, parity, first, partials);
  else if (ts.walls) {
    // wall boundaries: variant 3, one load per block (the engine guarantees L == 1)
    const size_t lds = (size_t)11 * nt * sizeof(T) + (ts.pal ? 256 * sizeof(CellCoef<T>) : 0);
    if (ts.pal)
      hipLaunchKernelGGL((step_kernel_b<T, 1, HI, true, true>), dim3(nwork), dim3(nt), lds, s, d_samples, d_work,
                         nwork, ts.bx, ts.by, parity, first, partials);
    else
      hipLaunchKernelGGL((step_kernel_b<T, 1, HI, false, true>), dim3(nwork), dim3(nt), lds, s, d_samples, d_work,
                         nwork, ts.bx, ts.by, parity, first, partials);
  } else if (ts.pf == 3 && ts.pal)
    hipLaunchKernelGGL((step_kernel_b<T, L, HI, true>), dim3(nwork), dim3(nt),
                       (size_t)(3 + 8 * L) * nt * sizeof(T) + 256 * sizeof(CellCoef<T>), s, d_samples, d_work, nwork,
                       ts.bx, ts.by, parity, first, partials);
  else if (ts.pf == 3)
    hipLaunchKernelGGL((step_kernel_b<T, L, HI, false>), dim3(nwork), dim3(nt), (size_t)(3 + 8 * L) * nt * sizeof(T),
                       s, d_samples, d_work, nwork, ts.bx, ts.by, parity, first, partials);
  else if (ts.pf == 2)
    hipLaunchKernelGGL((step_kernel_u2<T, L, HI>), dim3(nwork), dim3(nt), lds, s, d_samples, d_work, nwork, ts.bx,
                       ts.by, parity, first, partials);
  else if (ts.pf)
    hipLaunchKernelGGL((step_kernel<T, L, 0, T, true, HI>), dim3(nwork), dim3(nt), lds, s, d_samples, d_work, nwork,
                       ts.bx, ts.by, parity, first, partials, (T* const*)nullptr);
  else
    hipLaunchKernelGGL((step_kernel<T, L, 0, T, false, HI>), dim3(nwork), dim3(nt), lds, s, d_samples, d_work,
                       nwork, ts.bx, ts.by, parity, first, partials, (T* const*)nullptr);
}

template <typename T, int L>
hipError_t launch_step(const SampleDesc<T>* d_samples, const WorkItem* d_work, int nwork, TileShape ts, int parity,
                       int first, double* partials, hipStream_t s) {
  const int nt = ((ts.bx * ts.by + 63) / 64) * 64;
  const size_t lds = (size_t)11 * nt * sizeof(T);
  if (ts.occ)
    launch_step_occ<T, L, true>(d_samples, d_work, nwork, ts, parity, first, partials, s, nt, lds);
  else
    launch_step_occ<T, L, false>(d_samples, d_work, nwork, ts, parity, first, partials, s, nt, lds);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_pair(const SampleDesc<T>* d_samples, const WorkItem* d_work, int nwork, TileShape ts,
                            int parity, double* partials, hipStream_t s) {
  const int nt = ((ts.bx * ts.by + 63) / 64) * 64;
  const size_t lds = pair_lds_bytes(ts, sizeof(T));
  if (ts.occ && ts.pal)
    hipLaunchKernelGGL((step_kernel_t<T, true, true>), dim3(nwork), dim3(nt), lds, s, d_samples, d_work, nwork, ts.bx,
                       ts.by, parity, partials);
  else if (ts.occ)
    hipLaunchKernelGGL((step_kernel_t<T, true, false>), dim3(nwork), dim3(nt), lds, s, d_samples, d_work, nwork,
                       ts.bx, ts.by, parity, partials);
  else if (ts.pal)
    hipLaunchKernelGGL((step_kernel_t<T, false, true>), dim3(nwork), dim3(nt), lds, s, d_samples, d_work, nwork,
                       ts.bx, ts.by, parity, partials);
  else
    hipLaunchKernelGGL((step_kernel_t<T, false, false>), dim3(nwork), dim3(nt), lds, s, d_samples, d_work, nwork,
                       ts.bx, ts.by, parity, partials);
  return hipGetLastError();
}

template <typename T, typename R, int L>
hipError_t launch_residual(const SampleDesc<T>* d_samples, const WorkItem* d_work, int nwork, TileShape ts,
                           int parity, R* const* rout, double* partials, hipStream_t s) {
  const int nt = ((ts.bx * ts.by + 63) / 64) * 64;
  const size_t lds = (size_t)11 * nt * sizeof(T);
  if (ts.walls)
    hipLaunchKernelGGL((step_kernel<T, L, 1, R, false, false, true>), dim3(nwork), dim3(nt), lds, s, d_samples,
                       d_work, nwork, ts.bx, ts.by, parity, 0, partials, rout);
  else
    hipLaunchKernelGGL((step_kernel<T, L, 1, R, false, false>), dim3(nwork), dim3(nt), lds, s, d_samples, d_work,
                       nwork, ts.bx, ts.by, parity, 0, partials, rout);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_ortho(const SampleDesc<T>* d_samples, const WorkItem* d_work, int nwork, TileShape ts,
                             int parity, int first, double* partials, hipStream_t s) {
  const int nt = ((ts.bx * ts.by + 63) / 64) * 64;
  hipLaunchKernelGGL((step_kernel_ortho<T, 0, T>), dim3(nwork), dim3(nt), (size_t)kOrthoArrays * nt * sizeof(T), s,
                     d_samples, d_work, nwork, ts.bx, ts.by, parity, first, partials, (T* const*)nullptr);
  return hipGetLastError();
}

template <typename T, typename R>
hipError_t launch_residual_ortho(const SampleDesc<T>* d_samples, const WorkItem* d_work, int nwork, TileShape ts,
                                 int parity, R* const* rout, double* partials, hipStream_t s) {
  const int nt = ((ts.bx * ts.by + 63) / 64) * 64;
  hipLaunchKernelGGL((step_kernel_ortho<T, 1, R>), dim3(nwork), dim3(nt), (size_t)kOrthoArrays * nt * sizeof(T), s,
                     d_samples, d_work, nwork, ts.bx, ts.by, parity, 0, partials, rout);
  return hipGetLastError();
}

#if CEFF_IN_PART(0)
size_t pair_lds_bytes(TileShape ts, size_t elem) {
  const size_t nt = (size_t)(((ts.bx * ts.by + 63) / 64) * 64);
  return 22 * nt * elem + (ts.pal ? 256 * 4 * elem : 0);  // 22 arrays, and the 256-entry coefficient table
}

size_t ortho_lds_bytes(TileShape ts, size_t elem) {
  return (size_t)kOrthoArrays * (((ts.bx * ts.by + 63) / 64) * 64) * elem;
}

hipError_t launch_finalize_norms(const int* d_ranges, int nsamples, const double* partials, double* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(finalize_norms_kernel, dim3(nsamples * kMaxLoads), dim3(256), 0, s, d_ranges, partials, out);
  return hipGetLastError();
}

hipError_t launch_average_stress(int64_t nx, int64_t ny, int64_t nz, const double h[3], const double* K,
                                 const double* G, const double E[6], const double* u, double* partials,
                                 int nblocks_cap, double* out6, int walls, hipStream_t s) {
  int nb = grid_for(nx * ny * nz, 256);
  if (nb > nblocks_cap) nb = nblocks_cap;
  hipLaunchKernelGGL(average_partials_kernel, dim3(nb), dim3(256), 0, s, nx, ny, nz, 1.0 / h[0], 1.0 / h[1],
                     1.0 / h[2], K, G, E[0], E[1], E[2], E[3], E[4], E[5], u, partials, walls);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(average_finalize_kernel, dim3(6), dim3(256), 0, s, partials, nb, out6);
  return hipGetLastError();
}

hipError_t launch_average_stress_ortho(int64_t nx, int64_t ny, int64_t nz, const double h[3], const double* cst,
                                       const double E[6], const double* u, double* partials, int nblocks_cap,
                                       double* out6, hipStream_t s) {
  int nb = grid_for(nx * ny * nz, 256);
  if (nb > nblocks_cap) nb = nblocks_cap;
  hipLaunchKernelGGL(average_partials_ortho_kernel, dim3(nb), dim3(256), 0, s, nx, ny, nz, 1.0 / h[0], 1.0 / h[1],
                     1.0 / h[2], cst, E[0], E[1], E[2], E[3], E[4], E[5], u, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(average_finalize_kernel, dim3(6), dim3(256), 0, s, partials, nb, out6);
  return hipGetLastError();
}

#endif

template <typename R>
hipError_t launch_gradient(int64_t nx, int64_t ny, int64_t nz, const double h[3], const double* K, const double* G,
                           const GradLoads& g, R* dK, R* dG, hipStream_t s) {
  const int64_t N = nx * ny * nz;
  hipLaunchKernelGGL((gradient_kernel<R>), dim3((unsigned)((N + 127) / 128)), dim3(128), 0, s, nx, ny, nz,
                     1.0 / h[0], 1.0 / h[1], 1.0 / h[2], K, G, g, dK, dG);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s) {
  hipLaunchKernelGGL((fill_kernel<T>), dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

template <typename A, typename B>
hipError_t launch_convert(const A* src, B* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((convert_kernel<A, B>), dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

#if CEFF_IN_PART(0)
hipError_t launch_fold(double* base, float* cur, float* prev, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fold_kernel, dim3(grid_for(n)), dim3(256), 0, s, base, cur, prev, n);
  return hipGetLastError();
}

hipError_t launch_axpy1(double* dst, const double* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpy1_kernel, dim3(grid_for(n)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

#endif

template <typename T>
hipError_t launch_phase_to_fields(const uint8_t* phase, int64_t n, const double* Ktab, const double* Gtab, int nphase,
                                  T* K, T* G, hipStream_t s) {
  hipLaunchKernelGGL((phase_kernel<T>), dim3(grid_for(n)), dim3(256), 0, s, phase, n, Ktab, Gtab, nphase, K, G);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_check_moduli(const T* K, const T* G, int64_t n, int* bad, int* nblocks, hipStream_t s) {
  const int g = grid_for(n);
  *nblocks = g;
  hipLaunchKernelGGL((check_moduli_kernel<T>), dim3(g), dim3(256), 0, s, K, G, n, bad);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_tri(const SampleDesc<T>* d, int64_t N, int nwork, int parity, int first, double* partials,
                           hipStream_t s) {
  const int g = grid_for(N);
  hipLaunchKernelGGL((tri_strain_kernel<T>), dim3(g), dim3(256), 0, s, d, parity);
  hipLaunchKernelGGL((tri_stress_kernel<T>), dim3(g), dim3(256), 0, s, d);
  hipLaunchKernelGGL((tri_gather_kernel<T>), dim3(g), dim3(256), 0, s, d);
  hipLaunchKernelGGL((tri_update_kernel<T, 0, T>), dim3(nwork), dim3(256), 0, s, d, parity, first, partials,
                     (T* const*)nullptr);
  return hipGetLastError();
}

template <typename T, typename R>
hipError_t launch_residual_tri(const SampleDesc<T>* d, int64_t N, int nwork, int parity, R* const* rout,
                               double* partials, hipStream_t s) {
  const int g = grid_for(N);
  hipLaunchKernelGGL((tri_strain_kernel<T>), dim3(g), dim3(256), 0, s, d, parity);
  hipLaunchKernelGGL((tri_stress_kernel<T>), dim3(g), dim3(256), 0, s, d);
  hipLaunchKernelGGL((tri_gather_kernel<T>), dim3(g), dim3(256), 0, s, d);
  hipLaunchKernelGGL((tri_update_kernel<T, 1, R>), dim3(nwork), dim3(256), 0, s, d, parity, 0, partials, rout);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tri_setup(const double* c21, int64_t nx, int64_t ny, int64_t nz, T* se, T* ihf, hipStream_t s) {
  hipLaunchKernelGGL((tri_setup_kernel<T>), dim3(grid_for(nx * ny * nz)), dim3(256), 0, s, c21, nx, ny, nz, se, ihf);
  return hipGetLastError();
}

#if CEFF_IN_PART(0)
hipError_t launch_average_stress_tri(const SampleDesc<double>* d, const double* tscr, int64_t N, double* partials,
                                     int nblocks_cap, double* out6, hipStream_t s) {
  const int g = grid_for(N);
  hipLaunchKernelGGL((tri_strain_kernel<double>), dim3(g), dim3(256), 0, s, d, 0);
  hipLaunchKernelGGL((tri_stress_kernel<double>), dim3(g), dim3(256), 0, s, d);
  hipLaunchKernelGGL((tri_gather_kernel<double>), dim3(g), dim3(256), 0, s, d);
  const int nb = g < nblocks_cap ? g : nblocks_cap;
  hipLaunchKernelGGL(tri_sum_kernel, dim3(nb), dim3(256), 0, s, tscr + 6 * N, N, partials);
  hipLaunchKernelGGL(average_finalize_kernel, dim3(6), dim3(256), 0, s, partials, nb, out6);
  return hipGetLastError();
}

hipError_t launch_check_tri(const double* c, int64_t n, int* bad, int* nblocks, hipStream_t s) {
  const int g = grid_for(n);
  *nblocks = g;
  hipLaunchKernelGGL(check_tri_kernel, dim3(g), dim3(256), 0, s, c, n, bad);
  return hipGetLastError();
}

hipError_t launch_check_ortho(const double* c, int64_t n, int* bad, int* nblocks, hipStream_t s) {
  const int g = grid_for(n);
  *nblocks = g;
  hipLaunchKernelGGL((check_ortho_kernel<double>), dim3(g), dim3(256), 0, s, c, n, bad);
  return hipGetLastError();
}

#endif

// explicit instantiations
#define CEFF_INST_STEP(T, L)                                                                                       \
  template hipError_t launch_step<T, L>(const SampleDesc<T>*, const WorkItem*, int, TileShape, int, int, double*, \
                                        hipStream_t);
#if CEFF_IN_PART(1)
template hipError_t launch_step_pair<float>(const SampleDesc<float>*, const WorkItem*, int, TileShape, int, double*,
                                            hipStream_t);
CEFF_INST_STEP(float, 1)
CEFF_INST_STEP(float, 2)
#endif
#if CEFF_IN_PART(2)
CEFF_INST_STEP(float, 3)
CEFF_INST_STEP(float, 6)
#endif
#if CEFF_IN_PART(3)
template hipError_t launch_step_pair<double>(const SampleDesc<double>*, const WorkItem*, int, TileShape, int, double*,
                                             hipStream_t);
CEFF_INST_STEP(double, 1)
CEFF_INST_STEP(double, 2)
CEFF_INST_STEP(double, 3)
CEFF_INST_STEP(double, 6)
#endif
#if CEFF_IN_PART(0)
template hipError_t launch_step_ortho<float>(const SampleDesc<float>*, const WorkItem*, int, TileShape, int, int,
                                             double*, hipStream_t);
template hipError_t launch_step_ortho<double>(const SampleDesc<double>*, const WorkItem*, int, TileShape, int, int,
                                              double*, hipStream_t);
template hipError_t launch_residual_ortho<double, float>(const SampleDesc<double>*, const WorkItem*, int, TileShape,
                                                         int, float* const*, double*, hipStream_t);
template hipError_t launch_residual_ortho<double, double>(const SampleDesc<double>*, const WorkItem*, int, TileShape,
                                                          int, double* const*, double*, hipStream_t);
template hipError_t launch_residual_ortho<float, float>(const SampleDesc<float>*, const WorkItem*, int, TileShape,
                                                        int, float* const*, double*, hipStream_t);
#define CEFF_INST_RES(T, R, L)                                                                              \
  template hipError_t launch_residual<T, R, L>(const SampleDesc<T>*, const WorkItem*, int, TileShape, int, \
                                               R* const*, double*, hipStream_t);
CEFF_INST_RES(double, float, 1)
CEFF_INST_RES(double, float, 6)
CEFF_INST_RES(double, double, 1)
CEFF_INST_RES(double, double, 6)
CEFF_INST_RES(float, float, 1)
CEFF_INST_RES(float, float, 6)
template hipError_t launch_gradient<float>(int64_t, int64_t, int64_t, const double*, const double*, const double*,
                                           const GradLoads&, float*, float*, hipStream_t);
template hipError_t launch_gradient<double>(int64_t, int64_t, int64_t, const double*, const double*, const double*,
                                            const GradLoads&, double*, double*, hipStream_t);
template hipError_t launch_fill<float>(float*, int64_t, float, hipStream_t);
template hipError_t launch_fill<double>(double*, int64_t, double, hipStream_t);
template hipError_t launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);
template hipError_t launch_phase_to_fields<double>(const uint8_t*, int64_t, const double*, const double*, int,
                                                   double*, double*, hipStream_t);
template hipError_t launch_phase_to_fields<float>(const uint8_t*, int64_t, const double*, const double*, int, float*,
                                                  float*, hipStream_t);
template hipError_t launch_check_moduli<double>(const double*, const double*, int64_t, int*, int*, hipStream_t);
template hipError_t launch_step_tri<float>(const SampleDesc<float>*, int64_t, int, int, int, double*, hipStream_t);
template hipError_t launch_step_tri<double>(const SampleDesc<double>*, int64_t, int, int, int, double*, hipStream_t);
template hipError_t launch_residual_tri<double, float>(const SampleDesc<double>*, int64_t, int, int, float* const*,
                                                       double*, hipStream_t);
template hipError_t launch_residual_tri<double, double>(const SampleDesc<double>*, int64_t, int, int,
                                                        double* const*, double*, hipStream_t);
template hipError_t launch_residual_tri<float, float>(const SampleDesc<float>*, int64_t, int, int, float* const*,
                                                      double*, hipStream_t);
template hipError_t launch_tri_setup<float>(const double*, int64_t, int64_t, int64_t, float*, float*, hipStream_t);
template hipError_t launch_tri_setup<double>(const double*, int64_t, int64_t, int64_t, double*, double*, hipStream_t);
template hipError_t launch_check_moduli<float>(const float*, const float*, int64_t, int*, int*, hipStream_t);

#endif

}  // namespace ceff
