"""Workloads against stored oracle goldens (GPU).

tests/golden/make_workload_goldens.py wrote these with the CPU oracle alone
(Jacobi-PCG to rtol 1e-11):
* grad128_oracle.json: C* of the 128^3 15%-pore pack and the oracle's
  gradients of C11, C44 and trace(C) with respect to K(x) and G(x) at 4096
  seeded voxels -- checked against the FP32 gradient of the mixed-precision
  solve (FP64 averages);
* batch_oracle.json: all six C* columns of three samples of the 48-sample
  three-phase batch (n = 51, 57, 128) -- checked against one batch solve of
  all 48;
* cracks128_oracle.json: all six C* columns of the cracked-solid recipe at
  its crack number density (2000 per 479^3) in a 128^3 box.
C* parity is matrix-relative, 1e-6 (the target of the method's FP32 sweeps).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import synth
from gpu_common import announce, matrix_rel, need_gpu

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    return json.load(open(path))


def _digest(m):
    return hashlib.sha256(np.ascontiguousarray(m.phase).tobytes()).hexdigest()


def _columns(g):
    C = np.full((6, 6), np.nan)
    for J, v in g["columns"].items():
        C[:, int(J)] = v["C_column"]
    assert not np.isnan(C).any(), "golden incomplete"
    return C


def test_gradient_128_matches_oracle_gradient():
    p = need_gpu()
    g = _load("grad128_oracle.json")
    if "gradients" not in g:
        pytest.skip("gradient golden incomplete")
    m = synth.workload_grad128()
    assert _digest(m) == g["digest"], "generator drifted"
    K, G = m.fields()
    idx = np.array(g["sample"]["flat_indices"], np.int64)
    Co = _columns(g)
    Ws = {"C11": np.diag([1.0, 0, 0, 0, 0, 0]), "C44": np.diag([0, 0, 0, 1.0, 0, 0]), "trace": np.eye(6)}
    announce("grad128 vs oracle gradient")
    with p.Context() as c:
        c.set_material(K, G)
        C, info = c.solve(precision="mixed", rtol=1e-9, keep_fields=True)
        grads = {k: c.gradient(W, out_dtype="float32") for k, W in Ws.items()}
    assert info["status"] == 0
    print(f"grad128 C*: {matrix_rel(C, Co):.2e}", flush=True)
    assert matrix_rel(C, Co) <= 1e-6
    for k, (dK, dG) in grads.items():
        ref = g["gradients"][k]
        eK = np.abs(dK.ravel()[idx].astype(np.float64) - np.array(ref["dK"])).max() / ref["max_abs_dK"]
        eG = np.abs(dG.ravel()[idx].astype(np.float64) - np.array(ref["dG"])).max() / ref["max_abs_dG"]
        print(f"grad128 {k}: dK {eK:.2e}, dG {eG:.2e} (relative to the field's max)", flush=True)
        assert eK <= 1e-5 and eG <= 1e-5, (k, eK, eG)
        # Euler's identity on the full FP32 field (C is homogeneous of degree one in the moduli)
        J = float(np.sum(Ws[k] * C))
        assert float(np.sum(K * dK.astype(np.float64) + G * dG.astype(np.float64))) == pytest.approx(J, rel=1e-5)


def test_batch_samples_match_oracle_columns():
    p = need_gpu()
    g = _load("batch_oracle.json")
    if "samples" not in g or any(len(sub["columns"]) < 6 for sub in g["samples"].values()):
        pytest.skip("batch golden incomplete")
    ms = synth.workload_batch()
    order = [int(s) for s in g["samples"]]  # the order the digest was formed in
    assert hashlib.sha256("".join(_digest(ms[s]) for s in order).encode()).hexdigest() == g["digest"], "drifted"
    announce("batch48 vs oracle, samples", order)
    C, it, info = p.solve_batch_phases([m.phase for m in ms], ms[0].K_tab, ms[0].G_tab, precision="mixed",
                                       rtol=1e-8)
    assert info["status"] == 0
    for s, sub in g["samples"].items():
        s = int(s)
        assert ms[s].phase.shape[0] == sub["n"]
        e = matrix_rel(C[s], _columns(sub))
        print(f"batch sample {s} (n = {sub['n']}): {e:.2e}", flush=True)
        assert e <= 1e-6, (s, e)


def test_cracked_solid_at_crack_density_matches_oracle_columns():
    p = need_gpu()
    g = _load("cracks128_oracle.json")
    if len(g.get("columns", {})) < 6:
        pytest.skip("cracked-solid golden incomplete")
    m = synth.penny_cracks(128, round(2000 * (128 / 479) ** 3), 0xC3)
    assert _digest(m) == g["digest"], "generator drifted"
    Co = _columns(g)
    announce("cracks128 vs oracle")
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        C, info = c.solve(precision="mixed", rtol=1e-8)
    assert info["status"] == 0
    print(f"cracks128: iterations {info['iters'].tolist()}, {matrix_rel(C, Co):.2e}", flush=True)
    assert matrix_rel(C, Co) <= 1e-6
