"""Materials given as a phase image (GPU).

With ceff_set_phases the iteration kernel reads each cell's 1-byte phase id and
takes its coefficients from a per-phase table in LDS instead of reading the K
and G fields.  The table holds the same values as the fields, so the phase path
must give bitwise the same iterates as the field path (CEFF_MODULI=fields), and
both must match the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import announce, matrix_rel, need_gpu

pytestmark = pytest.mark.gpu


def phase_image(shape, nphase, seed):
    """Random phase ids in [0, nphase) and log-uniform per-phase moduli."""
    rng = synth.SplitMix64(seed)
    nz, ny, nx = shape
    ph = (rng.u64_array(nx * ny * nz) % np.uint64(nphase)).astype(np.uint8).reshape(shape)
    K = np.exp(np.log(2.0) + (np.log(90.0) - np.log(2.0)) * rng.uniform_array(nphase))
    G = np.exp(np.log(1e-3) + (np.log(45.0) - np.log(1e-3)) * rng.uniform_array(nphase))
    return synth.Microstructure(ph, K, G)


CASES = [((9, 10, 70), 3, 1), ((21, 29, 37), 5, 2), ((4, 5, 6), 256, 3), ((33, 14, 12), 256, 4)]


@pytest.mark.parametrize("shape,nphase,seed", CASES)
def test_phase_steps_match_oracle(shape, nphase, seed):
    """Iterates of the phase path against the oracle's paper-form APT iteration."""
    p = need_gpu()
    m = phase_image(shape, nphase, seed)
    K, G = m.fields()
    announce("phase apt_steps", shape, nphase, seed)
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        u64, _ = c.apt_steps(3, 7, "fp64", courant=0.95, strouhal=3.0)
        u32, _ = c.apt_steps(3, 7, "mixed", courant=0.95, strouhal=3.0)
    ref = oracle.apt_steps(K, G, 3, 7, courant=0.95, strouhal=3.0)["v"]
    scale = np.abs(ref).max()
    assert np.max(np.abs(u64 - ref)) <= 1e-11 * scale
    assert np.max(np.abs(u32 - ref)) <= 2e-5 * scale


@pytest.mark.parametrize("shape,nphase,seed", CASES)
def test_phase_path_bitwise_equals_field_path(shape, nphase, seed, monkeypatch):
    p = need_gpu()
    m = phase_image(shape, nphase, seed)
    announce("phase vs fields", shape, nphase, seed)
    for prec, fuse in (("mixed", True), ("fp64", False), ("mixed", False)):
        monkeypatch.delenv("CEFF_MODULI", raising=False)
        with p.Context() as c:
            c.set_phases(m.phase, m.K_tab, m.G_tab)
            Ca, ia = c.solve(precision=prec, fuse_loads=fuse, rtol=1e-9, check_every=20)
        assert ia["stats"]["phase_moduli"] == 1
        monkeypatch.setenv("CEFF_MODULI", "fields")
        with p.Context() as c:
            c.set_phases(m.phase, m.K_tab, m.G_tab)
            Cb, ib = c.solve(precision=prec, fuse_loads=fuse, rtol=1e-9, check_every=20)
        assert ib["stats"]["phase_moduli"] == 0
        assert np.array_equal(ia["iters"], ib["iters"]), prec
        assert np.array_equal(Ca, Cb), (prec, np.max(np.abs(Ca - Cb)))
        # one byte per cell instead of two words of moduli
        assert ia["stats"]["step_bytes"] < ib["stats"]["step_bytes"]


def test_sphere32_phases_match_oracle():
    p = need_gpu()
    m = synth.workload_sphere32()
    K, G = m.fields()
    Co, _ = oracle.ceff(K, G, rtol=1e-12)
    announce("sphere32 phases")
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        for prec in ("mixed", "fp64"):
            C, info = c.solve(precision=prec, rtol=1e-8)
            assert info["stats"]["phase_moduli"] == 1
            assert matrix_rel(C, Co) <= 1e-6, prec


def test_three_phase_field_matches_oracle():
    p = need_gpu()
    m = synth.gaussian_field_three_phase(24, 0xC4)
    K, G = m.fields()
    Co, _ = oracle.ceff(K, G, rtol=1e-12)
    announce("three-phase 24^3 phases")
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        C, info = c.solve(precision="mixed", rtol=1e-8)
    assert matrix_rel(C, Co) <= 1e-6
