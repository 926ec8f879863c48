"""Seeded synthetic voxel microstructures.

This module only builds inputs: phase images and per-phase moduli.  It holds
none of the homogenisation arithmetic, so both the GPU library and the CPU
oracle can be fed from it without sharing any method code.

Every random draw comes from a project-owned splitmix64 generator (Steele,
Lea & Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014),
so a given seed yields the same image on any machine and numpy version.  The
one exception is the Gaussian random field, which uses numpy's FFT for the
smoothing convolution (pocketfft; deterministic for a given numpy build).

Array layout: ``phase[k, j, i]`` with x (index i) fastest, i.e. linear index
``i + nx * (j + ny * k)``.  Voxel (i, j, k) has centre ((i+1/2)h, (j+1/2)h,
(k+1/2)h).  A voxel belongs to an inclusion iff its centre lies in the closed
body.  Geometry is periodic (minimum-image distances).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1

# Phase moduli used by the workloads, in GPa: (K, G).
MATRIX = (70.0, 32.0)
FLUID_PORE = (2.2, 1e-3)
SECOND_SOLID = (37.0, 44.0)


class SplitMix64:
    """splitmix64: state += golden gamma; output = mix(state)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniform_range(self, lo: float, hi: float) -> float:
        return lo + (hi - lo) * self.uniform()

    def randint(self, lo: int, hi: int) -> int:
        """Integer uniform on {lo, ..., hi} (inclusive), by rejection."""
        span = hi - lo + 1
        limit = (1 << 64) - ((1 << 64) % span)
        while True:
            x = self.next_u64()
            if x < limit:
                return lo + (x % span)

    def u64_array(self, n: int) -> np.ndarray:
        """The next n outputs at once (splitmix64 is counter based: output k
        mixes state + k * gamma), identical to n calls of next_u64."""
        k = np.arange(1, n + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + k * np.uint64(0x9E3779B97F4A7C15)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
        self.state = (self.state + n * 0x9E3779B97F4A7C15) & MASK64
        return z

    def uniform_array(self, n: int) -> np.ndarray:
        return (self.u64_array(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def normals(self, n: int) -> np.ndarray:
        """n standard normal variates by the Box-Muller transform (uniforms drawn
        in pairs: u1 in (0, 1], u2 in [0, 1))."""
        m = (n + 1) // 2
        u = self.uniform_array(2 * m)
        u1 = 1.0 - u[0::2]
        u2 = u[1::2]
        rad = np.sqrt(-2.0 * np.log(u1))
        out = np.empty(2 * m)
        out[0::2] = rad * np.cos(2.0 * math.pi * u2)
        out[1::2] = rad * np.sin(2.0 * math.pi * u2)
        return out[:n]

    def unit_vector(self) -> np.ndarray:
        """Uniform direction on the unit sphere (z uniform in [-1,1], phi uniform)."""
        z = self.uniform_range(-1.0, 1.0)
        phi = self.uniform_range(0.0, 2.0 * math.pi)
        s = math.sqrt(max(0.0, 1.0 - z * z))
        return np.array([s * math.cos(phi), s * math.sin(phi), z])


@dataclass
class Microstructure:
    """A voxel image: per-voxel phase ids plus per-phase (K, G)."""

    phase: np.ndarray                      # uint8, shape (nz, ny, nx)
    K_tab: np.ndarray                      # float64, per phase
    G_tab: np.ndarray                      # float64, per phase
    h: tuple = (1.0, 1.0, 1.0)             # (hx, hy, hz)
    info: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.phase.shape

    @property
    def dims(self):
        nz, ny, nx = self.phase.shape
        return (nx, ny, nz)

    def fields(self, dtype=np.float64):
        """Per-voxel K and G arrays, shape (nz, ny, nx)."""
        return (self.K_tab[self.phase].astype(dtype), self.G_tab[self.phase].astype(dtype))

    def fractions(self):
        cnt = np.bincount(self.phase.ravel(), minlength=len(self.K_tab))
        return cnt / self.phase.size


def _centres(n):
    return np.arange(n) + 0.5


def _periodic_delta(x, c, L):
    d = x - c
    return d - L * np.round(d / L)


def stamp_sphere(mask: np.ndarray, centre, radius: float) -> int:
    """Set mask over voxels whose centre is within `radius` of `centre` (periodic).
    Returns the number of voxels that were not set before."""
    nz, ny, nx = mask.shape
    cx, cy, cz = centre
    r = radius
    # candidate index ranges (may wrap)
    ii = np.arange(int(math.floor(cx - r - 1)), int(math.ceil(cx + r + 1)) + 1)
    jj = np.arange(int(math.floor(cy - r - 1)), int(math.ceil(cy + r + 1)) + 1)
    kk = np.arange(int(math.floor(cz - r - 1)), int(math.ceil(cz + r + 1)) + 1)
    ii = np.unique(ii % nx); jj = np.unique(jj % ny); kk = np.unique(kk % nz)
    dx = _periodic_delta(ii + 0.5, cx, nx)
    dy = _periodic_delta(jj + 0.5, cy, ny)
    dz = _periodic_delta(kk + 0.5, cz, nz)
    d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
    sub = d2 <= r * r
    idx = np.ix_(kk, jj, ii)
    fresh = int(np.count_nonzero(sub & ~mask[idx]))
    mask[idx] |= sub
    return fresh


def homogeneous(n, K=MATRIX[0], G=MATRIX[1]) -> Microstructure:
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    return Microstructure(np.zeros((nz, ny, nx), np.uint8), np.array([K]), np.array([G]))


def centred_sphere(n=32, radius=8.0, matrix=MATRIX, inclusion=FLUID_PORE) -> Microstructure:
    """One sphere centred in an n^3 box (the 32^3, r = 8 workload when defaulted)."""
    mask = np.zeros((n, n, n), bool)
    stamp_sphere(mask, (n / 2, n / 2, n / 2), radius)
    ph = mask.astype(np.uint8)
    m = Microstructure(ph, np.array([matrix[0], inclusion[0]]), np.array([matrix[1], inclusion[1]]))
    m.info = {"generator": "centred_sphere", "n": n, "radius": radius, "phi": float(mask.mean()),
              "n_inclusion": int(mask.sum())}
    return m


def centred_spheroid(n, semi_axes, matrix=MATRIX, inclusion=FLUID_PORE) -> Microstructure:
    """One axis-aligned ellipsoid with semi-axes (ax, ay, az) voxels, centred in a periodic
    box of n = (nx, ny, nz) (or n^3) voxels; a voxel belongs to it iff its centre lies in
    the closed ellipsoid.  info["phi"] is the realised voxel fraction."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    ax, ay, az = semi_axes
    x = (_centres(nx) - nx / 2) / ax
    y = (_centres(ny) - ny / 2) / ay
    z = (_centres(nz) - nz / 2) / az
    inside = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2 <= 1.0
    m = Microstructure(inside.astype(np.uint8), np.array([matrix[0], inclusion[0]]),
                       np.array([matrix[1], inclusion[1]]))
    m.info = {"generator": "centred_spheroid", "n": (nx, ny, nz), "semi_axes": tuple(map(float, semi_axes)),
              "phi": float(inside.mean()), "n_inclusion": int(inside.sum())}
    return m


def random_spheres(n, porosity, seed, rmin=3.0, rmax=9.0, matrix=MATRIX, pore=FLUID_PORE) -> Microstructure:
    """Random sequential addition of non-overlapping spheres (periodic box).

    radius ~ U[rmin, rmax], centre ~ U(box); a candidate is rejected if its
    periodic centre distance to any accepted sphere is below the sum of radii.
    Stops after the first accepted sphere that brings voxel porosity to at
    least `porosity`.
    """
    rng = SplitMix64(seed)
    L = float(n)
    mask = np.zeros((n, n, n), bool)
    nvox = mask.size
    cs = np.zeros((64, 3)); rs = np.zeros(64)  # accepted spheres in [:na], grown by doubling
    na = 0
    filled = 0  # voxels set so far (the porosity is filled / nvox)
    tries = 0
    while filled / nvox < porosity:
        tries += 1
        if tries > 10_000_000:
            raise RuntimeError("sphere packing did not reach the target porosity")
        r = rng.uniform_range(rmin, rmax)
        c = np.array([rng.uniform() * L, rng.uniform() * L, rng.uniform() * L])
        if na:
            d = c[None, :] - cs[:na]
            d -= L * np.round(d / L)
            if np.any(np.sqrt((d * d).sum(1)) < rs[:na] + r):
                continue
        if na == len(rs):
            cs = np.concatenate([cs, np.zeros_like(cs)]); rs = np.concatenate([rs, np.zeros_like(rs)])
        cs[na] = c; rs[na] = r; na += 1
        filled += stamp_sphere(mask, c, r)
    m = Microstructure(mask.astype(np.uint8), np.array([matrix[0], pore[0]]), np.array([matrix[1], pore[1]]))
    m.info = {"generator": "random_spheres", "n": n, "seed": seed, "n_spheres": na,
              "porosity": filled / nvox, "target": porosity}
    return m


def laminate_z(nx, ny, nz, stiff_layers, layer_thickness, stiff=(36.0, 44.0), soft=(7.2, 8.8)) -> Microstructure:
    """z-stacked layers: `stiff_layers` stiff layers of `layer_thickness` voxels,
    spaced evenly over nz, the rest soft (phase 0 = stiff, 1 = soft)."""
    ph = np.ones((nz, ny, nx), np.uint8)
    starts = np.linspace(0, nz, stiff_layers, endpoint=False).astype(int)
    for s in starts:
        ph[s:s + layer_thickness] = 0
    m = Microstructure(ph, np.array([stiff[0], soft[0]]), np.array([stiff[1], soft[1]]))
    m.info = {"generator": "laminate_z", "f_stiff": float((ph == 0).mean())}
    return m


def penny_cracks(n, ncracks, seed, amin=10.0, amax=30.0, aspect=0.05, matrix=MATRIX, fluid=FLUID_PORE) -> Microstructure:
    """Overlapping oblate-ellipsoid cracks: semi-axis a ~ U[amin, amax], half
    thickness c = aspect * a, normal uniform on the sphere, centre ~ U(box)."""
    rng = SplitMix64(seed)
    mask = np.zeros((n, n, n), bool)
    for _ in range(ncracks):
        a = rng.uniform_range(amin, amax)
        c = aspect * a
        nrm = rng.unit_vector()
        ctr = np.array([rng.uniform() * n, rng.uniform() * n, rng.uniform() * n])
        lo = np.floor(ctr - a - 1).astype(int); hi = np.ceil(ctr + a + 1).astype(int)
        ii = np.unique(np.arange(lo[0], hi[0] + 1) % n)
        jj = np.unique(np.arange(lo[1], hi[1] + 1) % n)
        kk = np.unique(np.arange(lo[2], hi[2] + 1) % n)
        dx = _periodic_delta(ii + 0.5, ctr[0], n)[None, None, :]
        dy = _periodic_delta(jj + 0.5, ctr[1], n)[None, :, None]
        dz = _periodic_delta(kk + 0.5, ctr[2], n)[:, None, None]
        dn = dx * nrm[0] + dy * nrm[1] + dz * nrm[2]
        d2 = dx * dx + dy * dy + dz * dz
        inside = (dn * dn) / (c * c) + (d2 - dn * dn) / (a * a) <= 1.0
        mask[np.ix_(kk, jj, ii)] |= inside
    m = Microstructure(mask.astype(np.uint8), np.array([matrix[0], fluid[0]]), np.array([matrix[1], fluid[1]]))
    m.info = {"generator": "penny_cracks", "n": n, "seed": seed, "ncracks": ncracks,
              "crack_fraction": float(mask.mean())}
    return m


def gaussian_field_three_phase(n, seed, sigma=4.0, fractions=(0.70, 0.25, 0.05),
                               phases=(MATRIX, SECOND_SOLID, FLUID_PORE)) -> Microstructure:
    """Periodic Gaussian random field (white noise convolved with an isotropic
    Gaussian of width `sigma` voxels, via FFT), thresholded at its empirical
    quantiles: lowest fractions[0] -> phase 0, next fractions[1] -> phase 1,
    the rest -> phase 2.  Ties are broken by linear index (stable sort)."""
    rng = SplitMix64(seed)
    w = rng.normals(n ** 3).reshape(n, n, n)
    k = np.fft.fftfreq(n)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    filt = np.exp(-2.0 * (math.pi ** 2) * (sigma ** 2) * k2)
    f = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    order = np.argsort(f.ravel(), kind="stable")
    ph = np.empty(n ** 3, np.uint8)
    c0 = int(round(fractions[0] * n ** 3)); c1 = int(round((fractions[0] + fractions[1]) * n ** 3))
    ph[order[:c0]] = 0; ph[order[c0:c1]] = 1; ph[order[c1:]] = 2
    m = Microstructure(ph.reshape(n, n, n), np.array([p[0] for p in phases]), np.array([p[1] for p in phases]))
    m.info = {"generator": "gaussian_field_three_phase", "n": n, "seed": seed}
    return m


def random_fields(shape, seed, lo=(1.0, 0.5), hi=(100.0, 50.0)):
    """Per-voxel K, G drawn independently, log-uniform in [lo, hi] (for step
    and operator tests on arbitrary heterogeneous fields)."""
    nx, ny, nz = shape
    rng = SplitMix64(seed)
    n = nx * ny * nz
    u = np.array([rng.uniform() for _ in range(2 * n)])
    K = np.exp(np.log(lo[0]) + (np.log(hi[0]) - np.log(lo[0])) * u[:n]).reshape(nz, ny, nx)
    G = np.exp(np.log(lo[1]) + (np.log(hi[1]) - np.log(lo[1])) * u[n:]).reshape(nz, ny, nx)
    return K, G


# ---- the five workloads -------------------------------------------------------

def random_orthotropic(shape, seed, normal=(20.0, 120.0), shear=(5.0, 50.0), coupling=(-0.3, 0.6)):
    """Per-cell orthotropic constants (9, nz, ny, nx): C11 C22 C33 C23 C13 C12 C44 C55 C66.
    Normal constants uniform in `normal`, shear constants uniform in `shear`, each
    coupling C_ij = t sqrt(C_ii C_jj) with t uniform in `coupling`; cells whose normal
    block is not positive definite (leading minors) are redrawn by the caller's seed
    change, so the generator raises instead of returning them."""
    rng = SplitMix64(seed)
    n = int(np.prod(shape))
    u = lambda lo, hi: lo + (hi - lo) * rng.uniform_array(n).reshape(shape)
    C11, C22, C33 = u(*normal), u(*normal), u(*normal)
    C23 = u(*coupling) * np.sqrt(C22 * C33)
    C13 = u(*coupling) * np.sqrt(C11 * C33)
    C12 = u(*coupling) * np.sqrt(C11 * C22)
    m2 = C11 * C22 - C12 ** 2
    m3 = C11 * (C22 * C33 - C23 ** 2) - C12 * (C12 * C33 - C23 * C13) + C13 * (C12 * C23 - C22 * C13)
    if not (np.all(m2 > 0) and np.all(m3 > 0)):
        raise ValueError("a normal block is not positive definite; use another seed")
    return np.stack([C11, C22, C33, C23, C13, C12, u(*shear), u(*shear), u(*shear)])


def random_triclinic(shape, seed, scale=(5.0, 40.0), soft=0.0, soft_scale=0.05):
    """Per-cell general anisotropic stiffness, (21, nz, ny, nx): the upper triangle of
    s (B B^T + 2 I) row by row, B a 6x6 matrix of entries uniform in [-1, 1] and s
    uniform in `scale`, so every cell is symmetric positive definite with all 21
    constants nonzero.  A fraction `soft` of the cells (chosen at random) is scaled
    by soft_scale."""
    rng = SplitMix64(seed)
    n = int(np.prod(shape))
    B = (2.0 * rng.uniform_array(36 * n) - 1.0).reshape(n, 6, 6)
    sc = scale[0] + (scale[1] - scale[0]) * rng.uniform_array(n)
    if soft > 0.0:
        sc = np.where(rng.uniform_array(n) < soft, sc * soft_scale, sc)
    M = sc[:, None, None] * (np.einsum("nij,nkj->nik", B, B) + 2.0 * np.eye(6)[None])
    out = np.stack([M[:, r, q] for r in range(6) for q in range(r, 6)])
    return np.ascontiguousarray(out.reshape((21,) + tuple(shape)))


def workload_sphere32() -> Microstructure:
    """32^3, matrix (70, 32), one centred fluid sphere of radius 8."""
    return centred_sphere(32, 8.0)


def workload_spheres191(seed=0xC2, n=191) -> Microstructure:
    """191^3, 10 % porosity of non-overlapping fluid spheres, radius U[3, 9]."""
    return random_spheres(n, 0.10, seed)


def workload_cracks(n=479, seed=0xC3, ncracks=2000) -> Microstructure:
    """n^3 cracked solid: 2000 fluid-filled penny cracks, a ~ U[10, 30], aspect 0.05."""
    return penny_cracks(n, ncracks, seed)


def workload_batch(nsamples=48, seed=0xC4, nmin=48, nmax=128):
    """48 three-phase GRF cubes with sizes drawn uniformly from {48..128}."""
    rng = SplitMix64(seed)
    sizes = [rng.randint(nmin, nmax) for _ in range(nsamples)]
    return [gaussian_field_three_phase(n, seed + s) for s, n in enumerate(sizes)]


def workload_grad128(seed=0xC5, n=128) -> Microstructure:
    """128^3 random fluid spheres at 15 % porosity (gradient workload)."""
    return random_spheres(n, 0.15, seed)


def workload_grad16(seed=0x16, n=16) -> Microstructure:
    """16^3 subcase of the gradient workload (finite-difference checks)."""
    return random_spheres(n, 0.15, seed, rmin=2.0, rmax=4.0)
