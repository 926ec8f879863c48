"""Input generators: reproducibility and the recipes' stated properties (CPU)."""
import numpy as np

import synth


def test_splitmix64_reference_values():
    # first outputs of splitmix64 seeded with 0 (published reference sequence)
    r = synth.SplitMix64(0)
    assert r.next_u64() == 0xE220A8397B1DCDAF
    assert r.next_u64() == 0x6E789E6AA1B965F4
    assert r.next_u64() == 0x06C45D188009454F


def test_vectorised_draws_match_scalar():
    a = synth.SplitMix64(0xC4)
    b = synth.SplitMix64(0xC4)
    v = a.u64_array(1000)
    assert all(int(v[i]) == b.next_u64() for i in range(1000))
    assert a.next_u64() == b.next_u64()


def test_normals_moments():
    z = synth.SplitMix64(7).normals(200001)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01


def test_sphere32_recipe():
    m = synth.workload_sphere32()
    assert m.info["n_inclusion"] == 2176
    assert abs(m.info["phi"] - 0.06640625) < 1e-12


def test_sphere_pack_reaches_porosity_without_overlap():
    m = synth.random_spheres(48, 0.10, 0xC2)
    assert 0.10 <= m.info["porosity"] < 0.13
    assert synth.random_spheres(48, 0.10, 0xC2).phase.tobytes() == m.phase.tobytes()


def test_three_phase_fractions():
    m = synth.gaussian_field_three_phase(24, 0xC4)
    f = m.fractions()
    np.testing.assert_allclose(f, [0.70, 0.25, 0.05], atol=1.0 / 24 ** 3)


def test_batch_sizes_in_range():
    rng = synth.SplitMix64(0xC4)
    sizes = [rng.randint(48, 128) for _ in range(48)]
    assert min(sizes) >= 48 and max(sizes) <= 128


def test_cracks_are_thin_and_fluid():
    m = synth.penny_cracks(64, 6, 0xC3, amin=10.0, amax=20.0)
    assert 0.0 < m.info["crack_fraction"] < 0.05
    assert m.K_tab[1] == 2.2
