"""Full-size parity of the benchmark workload with the oracle (GPU).

tests/golden/spheres191_oracle.json holds oracle C* columns of the 191^3
sphere pack (Jacobi-PCG to rtol 1e-11), written by
tests/golden/make_spheres191_golden.py, which calls only the oracle.  The GPU
solves the same image in the benchmark's configuration (mixed precision, the library's own choice of
load fusion -- one load after another at this size -- with the moduli read
from the phase image, rtol 1e-8, Strouhal number 3.5, residual checks every
100 iterations), at St 3.0 and 2.0, with the library's automatic Strouhal
number, with the six loads forced into one launch, and in the plain FP64
one-load-at-a-time configuration."""
import hashlib
import json
import os

import numpy as np
import pytest

import synth
from gpu_common import announce, need_gpu

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "spheres191_oracle.json")


@pytest.fixture(scope="module")
def golden():
    if not os.path.exists(GOLD):
        pytest.skip("golden file not generated")
    g = json.load(open(GOLD))
    m = synth.workload_spheres191()
    assert hashlib.sha256(m.phase.tobytes()).hexdigest() == g["phase_sha256"], "generator drifted"
    return m, g


@pytest.mark.parametrize("precision,fuse,strouhal", [("mixed", "auto", 3.5), ("mixed", "auto", 3.0),
                                                     ("mixed", "auto", 2.0), ("mixed", "auto", 0.0),
                                                     ("mixed", True, 2.0), ("fp64", False, 2.0)])
def test_spheres191_matches_oracle_columns(golden, precision, fuse, strouhal):
    p = need_gpu()
    m, g = golden
    announce("spheres191 golden", precision, fuse, strouhal, sorted(g["columns"]))
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        C, info = c.solve(precision=precision, fuse_loads=fuse, rtol=1e-8, strouhal=strouhal)
    assert info["status"] == 0
    if fuse == "auto":
        assert info["stats"]["fused_loads"] == 0 and info["stats"]["phase_moduli"] == 1
    cols = {int(J): np.array(v["C_column"]) for J, v in g["columns"].items()}
    scale = max(np.abs(v).max() for v in cols.values())
    for J, col in cols.items():
        err = np.max(np.abs(C[:, J] - col)) / scale
        print(f"column {J}: max |C - C_oracle| / max|C_oracle| = {err:.2e}")
        assert err <= 1e-6, (J, err)
