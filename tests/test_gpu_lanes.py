"""Iteration kernel with x-neighbours exchanged across lanes (variant 9, GPU).

Variant 9 is variant 3 for one load per block with rows 16, 32 or 64 cells wide,
so that every row lies within one wave: x-neighbour values move between lanes by
DPP wave shifts instead of through LDS.  Its values and arithmetic are those of
variant 3, so on the same tile the iterates agree to a few ulps (the compiler
may contract the update's multiply-adds differently).  Checked after 1, 2 and
11 steps on grids with ragged tails in x and y, z-chunks of 1 to 12 planes,
grids 2 to 4 planes thick, blocks with padding rows, all three row widths, moduli
from K and G fields and from a phase image, and against the oracle's iteration;
and full solves in mixed precision (folds, body forces, residual norms) and in
FP64, where each double crosses lanes as two 32-bit shifts."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import announce, matrix_rel, need_gpu

pytestmark = pytest.mark.gpu

CASES = [  # (nx, ny, nz), seed, tile "bx,by,kc"
    ((40, 33, 29), 1, "16,8,7"),
    ((70, 9, 31), 2, "32,6,3"),
    ((13, 45, 26), 3, "64,5,1"),
    ((37, 29, 4), 4, "16,14,2"),
    ((21, 17, 2), 5, "32,15,5"),
    ((19, 23, 3), 6, "64,8,12"),
]


def _steps(p, monkeypatch, tile, variant, K=None, G=None, m=None, J=1, n=(1, 2, 11), prec="mixed"):
    monkeypatch.setenv("CEFF_TILE", f"{tile},1,{variant},1,1")
    out = {}
    with p.Context() as c:
        if m is not None:
            c.set_phases(m.phase, m.K_tab, m.G_tab)
        else:
            c.set_material(K, G)
        for k in n:
            out[k] = c.apt_steps(J, k, prec, courant=0.95, strouhal=3.0)
        assert c.stats()["tile_variant"] == variant
    return out


@pytest.mark.parametrize("shape,seed,tile", CASES)
def test_lanes_steps_equal_variant3(monkeypatch, shape, seed, tile):
    p = need_gpu()
    K, G = synth.random_fields(shape[::-1], seed, lo=(2.0, 1e-3), hi=(90.0, 45.0))
    announce("variant 9 vs 3, fields", shape, tile)
    a = _steps(p, monkeypatch, tile, 3, K=K, G=G)
    b = _steps(p, monkeypatch, tile, 9, K=K, G=G)
    for k in a:
        for x, y in zip(a[k], b[k]):
            sc = float(np.abs(x).max())  # the previous iterate after one step is zero
            d = float(np.abs(x - y).max() / sc) if sc > 0 else float(np.abs(y).max())
            print(f"  steps {k}: max rel diff {d:.2e}{' (bitwise)' if np.array_equal(x, y) else ''}", flush=True)
            assert d <= 1e-6, (k, d)
    ref = oracle.apt_steps(K, G, 1, 11, 0.95, 3.0)["v"]
    assert np.abs(b[11][0] - ref).max() <= 2e-5 * np.abs(ref).max()


@pytest.mark.parametrize("shape,seed,tile", CASES[::2])
def test_lanes_fp64_steps_equal_variant3(monkeypatch, shape, seed, tile):
    """The FP64 build moves each double as two 32-bit lane shifts."""
    p = need_gpu()
    K, G = synth.random_fields(shape[::-1], seed + 10, lo=(2.0, 1e-3), hi=(90.0, 45.0))
    announce("variant 9 vs 3, fp64", shape, tile)
    a = _steps(p, monkeypatch, tile, 3, K=K, G=G, prec="fp64")
    b = _steps(p, monkeypatch, tile, 9, K=K, G=G, prec="fp64")
    for k in a:
        for x, y in zip(a[k], b[k]):
            sc = float(np.abs(x).max())
            d = float(np.abs(x - y).max() / sc) if sc > 0 else float(np.abs(y).max())
            print(f"  steps {k}: max rel diff {d:.2e}{' (bitwise)' if np.array_equal(x, y) else ''}", flush=True)
            assert d <= 1e-13, (k, d)
    ref = oracle.apt_steps(K, G, 1, 11, 0.95, 3.0)["v"]
    assert np.abs(b[11][0] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("shape,seed,tile", CASES[:3])
def test_lanes_phase_image_equals_variant3(monkeypatch, shape, seed, tile):
    p = need_gpu()
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, 3, size=(nz, ny, nx)).astype(np.uint8)
    m = synth.Microstructure(phase, np.array([70.0, 2.2, 35.0]), np.array([32.0, 1e-3, 12.0]))
    announce("variant 9 vs 3, phase image", shape, tile)
    for J in (0, 4):
        a = _steps(p, monkeypatch, tile, 3, m=m, J=J, n=(2, 11))
        b = _steps(p, monkeypatch, tile, 9, m=m, J=J, n=(2, 11))
        for k in a:
            for x, y in zip(a[k], b[k]):
                assert np.abs(x - y).max() <= 1e-6 * max(np.abs(x).max(), 1e-30), (J, k)


@pytest.mark.parametrize("phases,prec", [(False, "mixed"), (True, "mixed"), (True, "fp64")])
def test_lanes_solve_equals_variant3_solve(monkeypatch, phases, prec):
    p = need_gpu()
    m = synth.random_spheres(72, 0.10, 0x7B)
    K, G = m.fields()
    res = {}
    for v in (3, 9):
        monkeypatch.setenv("CEFF_TILE", f"16,16,12,1,{v},1,1")
        with p.Context() as c:
            if phases:
                c.set_phases(m.phase, m.K_tab, m.G_tab)
            else:
                c.set_material(K, G)
            res[v] = c.solve(precision=prec, rtol=1e-8, loads=(0, 3), fuse_loads=False)
            assert res[v][1]["stats"]["tile_variant"] == v
    (C3, i3), (C9, i9) = res[3], res[9]
    announce("variant 9 solve", phases, prec, i3["iters"].tolist(), i9["iters"].tolist(),
             matrix_rel(C9[:, [0, 3]], C3[:, [0, 3]]))
    assert i9["status"] == 0
    assert matrix_rel(C9[:, [0, 3]], C3[:, [0, 3]]) <= 1e-9
    assert np.all(np.abs(i9["iters"] - i3["iters"]) <= 100)


@pytest.mark.parametrize("shape", [(2, 3, 5), (3, 2, 4), (2, 2, 2), (70, 2, 3), (2, 40, 6), (17, 2, 2)])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_degenerate_grids_default_shape(monkeypatch, shape, prec):
    """Grids two cells wide in x or y, and two planes deep, on the library's own launch shape
    (variant 9 in both precisions): a row's ghost lanes then wrap onto the
    same two columns, and a block's ghost rows onto the same two rows.  The iterate after 11
    steps matches the oracle's paper-form iteration, and C* its PCG solve."""
    p = need_gpu()
    monkeypatch.delenv("CEFF_TILE", raising=False)
    K, G = synth.random_fields(shape[::-1], sum(shape), lo=(2.0, 1e-3), hi=(90.0, 45.0))
    announce("degenerate grid", shape, prec)
    ref = oracle.apt_steps(K, G, 2, 11, 0.95, 3.0)["v"]
    with p.Context() as c:
        c.set_material(K, G)
        u, _ = c.apt_steps(2, 11, prec, courant=0.95, strouhal=3.0)
        assert c.stats()["tile_variant"] == 9
        C, info = c.solve(precision=prec, rtol=1e-9)
    tol = 2e-5 if prec == "mixed" else 1e-11
    assert np.abs(u - ref).max() <= tol * np.abs(ref).max()
    Co, _ = oracle.ceff(K, G, rtol=1e-12)
    assert info["status"] == 0
    assert matrix_rel(C, Co) <= 1e-6
