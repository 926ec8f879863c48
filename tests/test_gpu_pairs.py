"""Two heavy-ball iterations per launch (GPU): the kernel that advances
(u^n, u^{n-1}) to (u^{n+1}, u^{n+2}) in one z-march gives the iterates of two
single iterations, on grids spanning several tiles and z-chunks with ragged
tails, for odd and even step counts, with the moduli from K and G fields and
from a phase image; a full mixed-precision solve (body forces after the folds,
norms on check iterations) reaches the same C* as the single-iteration path."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import announce, matrix_rel, need_gpu

pytestmark = pytest.mark.gpu

SHAPES = [((40, 33, 29), 1), ((70, 9, 31), 2), ((13, 45, 26), 3)]


@pytest.mark.parametrize("shape,seed", SHAPES)
def test_pairs_equal_single_iterations(monkeypatch, shape, seed):
    p = need_gpu()
    K, G = synth.random_fields(shape[::-1], seed, lo=(2.0, 1e-3), hi=(90.0, 45.0))
    monkeypatch.delenv("CEFF_TILE", raising=False)
    out = {}
    for tb in ("0", "1"):
        monkeypatch.setenv("CEFF_TB", tb)
        monkeypatch.setenv("CEFF_TILE", "18,14,7,1,3")  # several tiles and z-chunks at these sizes
        with p.Context() as c:
            c.set_material(K, G)
            for n in (2, 3, 10, 11):
                out[(tb, n)] = c.apt_steps(4, n, "mixed", courant=0.95, strouhal=3.0)
                if tb == "1":
                    assert c.stats()["tile_variant"] == 6
    for n in (2, 3, 10, 11):
        u0, up0 = out[("0", n)]
        u1, up1 = out[("1", n)]
        d = float(np.abs(u1 - u0).max() / np.abs(u0).max())
        dp = float(np.abs(up1 - up0).max() / np.abs(up0).max())
        announce("pairs vs single", shape, n, d, dp)
        assert d <= 1e-6 and dp <= 1e-6, (n, d, dp)
    # and against the oracle's iteration
    ref = oracle.apt_steps(K, G, 4, 11, 0.95, 3.0)["v"]
    assert np.abs(out[("1", 11)][0] - ref).max() <= 2e-5 * np.abs(ref).max()


@pytest.mark.parametrize("phases", [False, True])
def test_pairs_solve_matches_single_iteration_solve(monkeypatch, phases):
    p = need_gpu()
    monkeypatch.delenv("CEFF_TILE", raising=False)
    m = synth.random_spheres(72, 0.10, 0x7B)
    K, G = m.fields()
    res = {}
    for tb in ("0", "1"):
        monkeypatch.setenv("CEFF_TB", tb)
        with p.Context() as c:
            if phases:
                c.set_phases(m.phase, m.K_tab, m.G_tab)
            else:
                c.set_material(K, G)
            res[tb] = c.solve(precision="mixed", rtol=1e-8, loads=(0, 3), fuse_loads=False, check_every=40)
    (C0, i0), (C1, i1) = res["0"], res["1"]
    announce("pairs solve", phases, i0["iters"].tolist(), i1["iters"].tolist(), matrix_rel(C1[:, [0, 3]], C0[:, [0, 3]]))
    assert i1["status"] == 0 and i1["stats"]["tile_variant"] == 6
    assert matrix_rel(C1[:, [0, 3]], C0[:, [0, 3]]) <= 1e-8
    assert np.all(np.abs(i1["iters"] - i0["iters"]) <= 40)
