"""Iteration kernels with another pipeline than variant 3 (GPU): variant 7
(u^n prefetched into LDS: asynchronous copies of u^n planes into a ring of LDS
slots, completions tracked by hand) and variant 8 (one barrier per plane:
double-buffered LDS inputs and stresses).

Both compute every node with the expressions of variant 3 (the compiler may
contract the momentum update's multiply-adds differently, so iterates agree to
a few ulps).  Checked against variant 3 and the
oracle's APT iteration: iterates after 1, 2 and 11 steps on grids spanning
several tiles with ragged tails, z-chunks of 1 to 7 planes (the ring's start-up
and end-of-chunk paths), grids only 2 or 3 planes thick (plane indices wrapping
more than once), blocks of up to 256 and of up to 512 threads, moduli from K
and G fields and from a phase image; and full mixed-precision solves (body
forces after the folds, residual norms on check iterations) against the
variant-3 solve."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import announce, matrix_rel, need_gpu

pytestmark = pytest.mark.gpu

CASES = [  # (nx, ny, nz), seed, tile "bx,by,kc"
    ((40, 33, 29), 1, "18,14,7"),
    ((70, 9, 31), 2, "34,14,3"),
    ((13, 45, 26), 3, "66,7,1"),
    ((37, 29, 4), 4, "18,14,2"),
    ((21, 17, 2), 5, "34,15,5"),
    ((19, 23, 3), 6, "18,14,12"),
]


def _steps(p, monkeypatch, tile, variant, occ, K=None, G=None, m=None, J=1, n=(1, 2, 11)):
    monkeypatch.setenv("CEFF_TILE", f"{tile},1,{variant},1,{occ}")
    out = {}
    with p.Context() as c:
        if m is not None:
            c.set_phases(m.phase, m.K_tab, m.G_tab)
        else:
            c.set_material(K, G)
        for k in n:
            out[k] = c.apt_steps(J, k, "mixed", courant=0.95, strouhal=3.0)
        assert c.stats()["tile_variant"] == variant
    return out


@pytest.mark.parametrize("shape,seed,tile", CASES)
@pytest.mark.parametrize("occ", [0, 1])
@pytest.mark.parametrize("variant", [7, 8])
def test_variant_steps_equal_variant3(monkeypatch, shape, seed, tile, occ, variant):
    p = need_gpu()
    K, G = synth.random_fields(shape[::-1], seed, lo=(2.0, 1e-3), hi=(90.0, 45.0))
    announce(f"variant {variant} vs 3, fields", shape, tile, occ)
    a = _steps(p, monkeypatch, tile, 3, occ, K=K, G=G)
    b = _steps(p, monkeypatch, tile, variant, occ, K=K, G=G)
    for k in a:
        for x, y in zip(a[k], b[k]):
            sc = np.abs(x).max()
            d = float(np.abs(x - y).max() / sc) if sc > 0 else float(np.abs(y).max())
            print(f"  steps {k}: max rel diff {d:.2e}{' (bitwise)' if np.array_equal(x, y) else ''}", flush=True)
            assert d <= 1e-6, (k, d)
    ref, _ = oracle.apt_disp(1, 11, 0.95, 3.0, K=K, G=G)
    assert np.abs(b[11][0] - ref).max() <= 2e-5 * np.abs(ref).max()


@pytest.mark.parametrize("shape,seed,tile", CASES[:3])
@pytest.mark.parametrize("variant", [7, 8])
def test_variant_phase_image_equals_variant3(monkeypatch, shape, seed, tile, variant):
    p = need_gpu()
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, 3, size=(nz, ny, nx)).astype(np.uint8)
    m = synth.Microstructure(phase, np.array([70.0, 2.2, 35.0]), np.array([32.0, 1e-3, 12.0]))
    announce(f"variant {variant} vs 3, phase image", shape, tile)
    for J in (0, 4):
        a = _steps(p, monkeypatch, tile, 3, 1, m=m, J=J, n=(2, 11))
        b = _steps(p, monkeypatch, tile, variant, 1, m=m, J=J, n=(2, 11))
        for k in a:
            for x, y in zip(a[k], b[k]):
                assert np.abs(x - y).max() <= 1e-6 * np.abs(x).max(), (J, k)


@pytest.mark.parametrize("phases", [False, True])
@pytest.mark.parametrize("variant", [7, 8])
def test_variant_solve_equals_variant3_solve(monkeypatch, phases, variant):
    p = need_gpu()
    m = synth.random_spheres(72, 0.10, 0x7B)
    K, G = m.fields()
    res = {}
    for v in (3, variant):
        monkeypatch.setenv("CEFF_TILE", f"18,14,12,1,{v},1,1")
        with p.Context() as c:
            if phases:
                c.set_phases(m.phase, m.K_tab, m.G_tab)
            else:
                c.set_material(K, G)
            res[v] = c.solve(precision="mixed", rtol=1e-8, loads=(0, 3), fuse_loads=False)
            assert res[v][1]["stats"]["tile_variant"] == v
    (C3, i3), (C7, i7) = res[3], res[variant]
    announce(f"variant {variant} solve", phases, i3["iters"].tolist(), i7["iters"].tolist(),
             matrix_rel(C7[:, [0, 3]], C3[:, [0, 3]]))
    assert i7["status"] == 0
    assert matrix_rel(C7[:, [0, 3]], C3[:, [0, 3]]) <= 1e-9
    assert np.all(np.abs(i7["iters"] - i3["iters"]) <= 100)
