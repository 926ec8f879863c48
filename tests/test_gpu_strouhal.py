"""The automatic Strouhal number (strouhal = 0, the default) on the pore
families it was fitted on (GPU): the six-load iteration counts land within 10%
of the best of each family's St sweep (191^3 pack, 10% pores: 27 600
load-iterations at St 3.5; 128^3 pack, 15% pores: 29 500 at St 2.2; both with
checks every 100 iterations, mixed precision, rtol 1e-8)."""
import numpy as np
import pytest

import synth
from gpu_common import announce, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,best", [("spheres191", 27600), ("grad128", 29500)])
def test_automatic_strouhal_near_the_swept_best(name, best):
    p = need_gpu()
    m = synth.workload_spheres191() if name == "spheres191" else synth.workload_grad128()
    n = m.phase.shape[0]
    st = p.ceff_auto_strouhal(n, n, n)
    announce("auto St", name, st)
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        C, info = c.solve(precision="mixed", rtol=1e-8, check_every=100)
        C2, info2 = c.solve(precision="mixed", rtol=1e-8, check_every=100, strouhal=st)
    total = int(info["iters"].sum())
    print(f"{name}: St {st:.3f}, {total} load-iterations (swept best {best})", flush=True)
    assert info["status"] == 0
    assert np.array_equal(info["iters"], info2["iters"])  # strouhal = 0 is that St
    assert abs(total - best) <= 0.10 * best
