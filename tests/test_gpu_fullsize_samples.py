"""Parity at the workloads' full sizes on sampled voxels (GPU).

At 479^3 and 703^3 the oracle cannot iterate the whole grid, but after a few APT
steps a voxel's displacement depends only on the material a few cells around it:
each step reaches one cell further (the stresses of the adjacent cells and edges,
whose moduli reach one cell more).  The oracle's paper-form iteration on a periodic
window of 2R+1 cells cut around a voxel therefore reproduces that voxel's iterate
exactly when R exceeds the reach of the steps, provided the iteration's scalars are
those of the full grid.  They depend on the box only through the damping
c = ell St / L and the step beta = ell L / St (L the largest box length); on a window
of length L_w both stay the same with St_w = St L_w / L.

The GPU runs the library's own launch shape for these grids (variant 9, 64 x 8 blocks,
32-plane chunks), in FP32 as the solves do, from the phase image.  Samples include
crack or pore voxels, matrix voxels and the periodic corners of the box."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import announce, need_gpu

pytestmark = pytest.mark.gpu

STEPS = 3
R = 7  # window half-width; three steps reach about four cells


def _samples(m, n, seed, count=6):
    rng = np.random.default_rng(seed)
    soft = np.argwhere(m.phase == 1)
    hard = np.argwhere(m.phase == 0)
    picks = [soft[i] for i in rng.choice(len(soft), count // 2, replace=False)]
    picks += [hard[i] for i in rng.choice(len(hard), count - count // 2, replace=False)]
    picks += [np.array([0, 0, 0]), np.array([n - 1, n - 1, n - 1]), np.array([0, n - 1, n // 2])]
    return [tuple(int(v) for v in p) for p in picks]  # (k, j, i)


def _window_reference(m, n, kji, J, strouhal):
    k, j, i = kji
    idx = [(np.arange(-R, R + 1) + c) % n for c in (k, j, i)]
    ph = m.phase[np.ix_(*idx)]
    K = np.ascontiguousarray(m.K_tab[ph], dtype=np.float64)
    G = np.ascontiguousarray(m.G_tab[ph], dtype=np.float64)
    w = 2 * R + 1
    ref = oracle.apt_steps(K, G, J, STEPS, courant=0.95, strouhal=strouhal * w / n)["v"]
    return ref[:, R, R, R]


def _check(p, m, n, loads, strouhal, seed):
    samples = _samples(m, n, seed)
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        for J in loads:
            u, _ = c.apt_steps(J, STEPS, "mixed", courant=0.95, strouhal=strouhal)
            st = c.stats()
            assert (st["tile_bx"], st["tile_by"], st["tile_kc"], st["tile_variant"]) == (64, 8, 32, 9)
            # relative to the field's largest value: a voxel whose neighbourhood is homogeneous is
            # already in equilibrium and stays exactly zero
            scale = float(np.abs(u).max())
            assert scale > 0
            worst = 0.0
            largest = 0.0
            for kji in samples:
                ref = _window_reference(m, n, kji, J, strouhal)
                got = u[(slice(None),) + kji]
                err = float(np.abs(got - ref).max()) / scale
                worst = max(worst, err)
                largest = max(largest, float(np.abs(ref).max()) / scale)
                assert err <= 2e-5, (J, kji, got, ref)
            assert largest > 1e-2  # the samples include voxels that moved
            print(f"  load {J}: {len(samples)} voxels, worst relative difference {worst:.2e}, largest sampled "
                  f"value {largest:.2f} of the field's", flush=True)
            del u


def test_cracked_solid_479_sampled_voxels_match_oracle():
    """The 479^3 cracked solid (2000 penny cracks), loads 0 and 4, at the benchmark's St 5.0."""
    p = need_gpu()
    m = synth.workload_cracks()
    n = m.phase.shape[0]
    assert n == 479
    announce("full-size samples, cracked solid", n)
    _check(p, m, n, (0, 4), 5.0, 0x479)


def test_sphere_pack_703_sampled_voxels_match_oracle():
    """The 703^3 sphere pack (the largest grid run), load 0, at its St 8.0."""
    p = need_gpu()
    m = synth.random_spheres(703, 0.10, 0xC2)
    announce("full-size samples, sphere pack", 703)
    _check(p, m, 703, (0,), 8.0, 0x703)
