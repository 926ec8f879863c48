"""Step-level parity of the HIP kernels with the CPU oracle (GPU).

* the iteration kernel (displacement form of the APT update) against the
  oracle's APT iteration in the paper's (p, tau, v) variables, after k steps,
  on grids that span several tiles in x and y, several z chunks and ragged
  tails;
* the residual kernel against the oracle's div(C:(E + grad u));
* the FP64 stress-average kernel against the oracle's averages.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import announce, need_gpu

pytestmark = pytest.mark.gpu

SHAPES = [((8, 8, 8), 1), ((12, 10, 9), 2), ((70, 9, 5), 3), ((5, 23, 6), 4), ((6, 5, 41), 5), ((130, 7, 3), 6)]


def fields(shape, seed):
    return synth.random_fields(shape, seed, lo=(2.0, 1e-3), hi=(90.0, 45.0))


@pytest.mark.parametrize("shape,seed", SHAPES)
@pytest.mark.parametrize("J", [0, 3, 5])
def test_steps_fp64_match_paper_form(shape, seed, J):
    p = need_gpu()
    K, G = fields(shape, seed)
    announce("apt_steps fp64", shape, seed, J)
    with p.Context() as c:
        c.set_material(K, G)
        for k in (1, 2, 11):
            u, up = c.apt_steps(J, k, "fp64", courant=0.95, strouhal=3.0)
            ref = oracle.apt_steps(K, G, J, k, courant=0.95, strouhal=3.0)["v"]
            scale = np.abs(ref).max()
            assert np.max(np.abs(u - ref)) <= 1e-11 * scale, (k, np.max(np.abs(u - ref)) / scale)
            if k > 1:
                refp = oracle.apt_steps(K, G, J, k - 1, courant=0.95, strouhal=3.0)["v"]
                assert np.max(np.abs(up - refp)) <= 1e-11 * scale


@pytest.mark.parametrize("shape,seed", SHAPES[:4])
def test_steps_fp32_match_paper_form(shape, seed):
    p = need_gpu()
    K, G = fields(shape, seed)
    announce("apt_steps fp32", shape, seed)
    with p.Context() as c:
        c.set_material(K, G)
        u, _ = c.apt_steps(1, 9, "mixed", courant=0.95, strouhal=3.0)
    ref = oracle.apt_steps(K, G, 1, 9, courant=0.95, strouhal=3.0)["v"]
    assert np.max(np.abs(u - ref)) <= 2e-5 * np.abs(ref).max()


def test_steps_independent_of_tile_shape(monkeypatch):
    """Every node's arithmetic is fixed, so iterates are bitwise identical for any tiling."""
    p = need_gpu()
    K, G = fields((37, 29, 21), 9)
    outs = []
    for tile in ("66,6", "34,10", "18,18,5", "10,34,3"):
        monkeypatch.setenv("CEFF_TILE", tile)
        announce("tile", tile)
        with p.Context() as c:
            c.set_material(K, G)
            outs.append(c.apt_steps(2, 15, "fp64")[0])
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("shape,seed", SHAPES)
def test_residual_matches_oracle(shape, seed):
    p = need_gpu()
    K, G = fields(shape, seed)
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((3,) + K.shape[::1])
    announce("residual", shape)
    with p.Context() as c:
        c.set_material(K, G)
        for J in (0, 4):
            r, n2 = c.residual(J, u, "fp64")
            ref = oracle.residual(K, G, oracle.unit_strain(J), u)
            sc = np.abs(ref).max()
            assert np.max(np.abs(r - ref)) <= 1e-12 * sc
            assert n2 == pytest.approx(float(np.sum(ref * ref)), rel=1e-12)
            r32, n32 = c.residual(J, u, "mixed")
            assert np.max(np.abs(r32 - ref)) <= 2e-5 * sc


@pytest.mark.parametrize("shape,seed", SHAPES[:3])
def test_average_stress_matches_oracle(shape, seed):
    p = need_gpu()
    K, G = fields(shape, seed)
    rng = np.random.default_rng(seed + 100)
    u = rng.standard_normal((3,) + K.shape)
    with p.Context() as c:
        c.set_material(K, G)
        for J in range(6):
            a = c.average_stress(J, u)
            ref = oracle.average_stress(K, G, oracle.unit_strain(J), u)
            np.testing.assert_allclose(a, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_residual_full_size_sampled():
    """The residual kernel at 191^3 (the benchmark grid) against the oracle."""
    p = need_gpu()
    m = synth.workload_spheres191()
    K, G = m.fields()
    rng = np.random.default_rng(7)
    u = rng.standard_normal((3,) + K.shape)
    announce("residual 191^3")
    with p.Context() as c:
        c.set_material(K, G)
        r, n2 = c.residual(3, u, "fp64")
    ref = oracle.residual(K, G, oracle.unit_strain(3), u)
    assert np.max(np.abs(r - ref)) <= 1e-12 * np.abs(ref).max()
    assert n2 == pytest.approx(float(np.sum(ref * ref)), rel=1e-11)
