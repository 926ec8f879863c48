"""The launch-shape autotuner (GPU): it changes speed only, never the iterates,
and its choices persist in the file named by CEFF_TUNE_CACHE."""
import numpy as np
import pytest

import synth
from gpu_common import announce, matrix_rel, need_gpu

pytestmark = pytest.mark.gpu

OPTS = dict(precision="mixed", rtol=1e-8, fuse_loads=True, strouhal=2.0)


def _shape(info):
    st = info["stats"]
    return st["tile_bx"], st["tile_by"], st["tile_kc"], st["tile_group"], st["tile_variant"]


def _entries(path):
    out = {}
    for line in open(path).read().splitlines():
        f = line.split()
        if len(f) == 8:
            out[f[0]] = tuple(int(v) for v in f[1:])
    return out


def test_autotune_keeps_the_iterates_and_persists_its_choice(tmp_path, monkeypatch):
    p = need_gpu()
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("CEFF_TUNE_CACHE", str(cache))
    monkeypatch.delenv("CEFF_TILE", raising=False)
    m = synth.random_spheres(48, 0.10, 0xA7)
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        announce("autotune: default shape")
        C0, i0 = c.solve(**OPTS)
        assert not cache.exists()  # autotune off: the cache file is neither read nor written
        announce("autotune: tuned")
        C1, i1 = c.solve(autotune=True, **OPTS)
    print("default shape", _shape(i0), "autotuned shape", _shape(i1), flush=True)
    assert i0["status"] == 0 and i1["status"] == 0
    assert matrix_rel(C1, C0) <= 1e-12
    assert np.array_equal(i1["iters"], i0["iters"])
    ent = _entries(cache)
    assert len(ent) == 1
    key, (bx, by, kc, grp, pf, order, occ) = next(iter(ent.items()))
    assert key.startswith("f32:loads3f:pal1:samples1:48x48x48:")
    bx1, by1, _, grp1, pf1 = _shape(i1)
    assert (bx1, by1, pf1) == (bx, by, pf)
    assert grp1 == (1 if pf in (5, 9) else grp)

    # a later process (here: a new context) reads the file: plant a different valid shape
    planted = (34, 10, 8, 3, 3, 1, 0)
    with open(cache, "a") as f:
        f.write(key + " " + " ".join(map(str, planted)) + "\n")
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        announce("autotune: from the cache file")
        C2, i2 = c.solve(autotune=True, **OPTS)
        C3, i3 = c.solve(**OPTS)  # autotune off again: built-in shape
    assert _shape(i2) == (34, 10, 8, 3, 3)
    assert _shape(i3) == _shape(i0)
    assert matrix_rel(C2, C0) <= 1e-12
    assert np.array_equal(i2["iters"], i0["iters"])
