"""The remaining workloads at their own sizes (GPU): properties that hold at any
size, plus oracle comparisons on the pieces the oracle can afford."""
import numpy as np
import pytest

import closed_forms as cf
import oracle
import synth
from gpu_common import announce, matrix_rel, need_gpu

pytestmark = pytest.mark.gpu


def loewner_ok(C, K, G, tol=1e-9):
    Cs = 0.5 * (C + C.T)
    w = cf._mandel_weights()
    M = lambda X: X * np.outer(w, w)
    sc = np.abs(C).max()
    return (np.linalg.eigvalsh(M(cf.voigt_bound(K, G)) - M(Cs)).min() > -tol * sc and
            np.linalg.eigvalsh(M(Cs) - M(cf.reuss_bound(K, G))).min() > -tol * sc)


def test_batch_of_48_uneven_three_phase_samples():
    """48 Gaussian-random-field samples, n uniform in 48..128, six loads each,
    one launch per iteration over all unconverged (sample, load) pairs."""
    p = need_gpu()
    announce("batch48 generate")
    ms = synth.workload_batch()
    samples = [m.fields(np.float32) for m in ms]
    announce("batch48 solve", [m.phase.shape[0] for m in ms])
    C, it, info = p.solve_batch(samples, precision="mixed", rtol=1e-8)
    assert info["status"] == 0
    for s, m in enumerate(ms):
        K, G = m.fields()
        assert np.max(np.abs(C[s] - C[s].T)) <= 1e-6 * np.abs(C[s]).max(), s
        assert loewner_ok(C[s], K, G), s
    # the smallest sample against the oracle (all loads), and against a solo GPU solve
    s = int(np.argmin([m.phase.shape[0] for m in ms]))
    K, G = ms[s].fields()
    announce("batch48 oracle check of sample", s, K.shape)
    Co, _ = oracle.ceff(K, G, rtol=1e-10, loads=[0, 4])
    assert np.max(np.abs(C[s][:, [0, 4]] - Co[:, [0, 4]])) <= 1e-6 * np.abs(Co[:, [0, 4]]).max()
    Csolo, _ = p.solve(K, G, precision="mixed", rtol=1e-8)
    assert matrix_rel(C[s], Csolo) <= 1e-7


def test_cracked_solid_small_box_matches_oracle():
    """Penny cracks of the cracked-solid recipe (a in [10, 20], aspect 0.05,
    fluid filled) in a 64^3 box: anisotropic C*, checked on two loads."""
    p = need_gpu()
    m = synth.penny_cracks(64, 8, 0xC3, amin=10.0, amax=20.0)
    K, G = m.fields()
    announce("cracks64", m.info)
    C, info = p.solve(K, G, precision="mixed", rtol=1e-8)
    Co, _ = oracle.ceff(K, G, rtol=1e-10, loads=[2, 3])
    assert np.max(np.abs(C[:, [2, 3]] - Co[:, [2, 3]])) <= 1e-6 * np.abs(Co[:, [2, 3]]).max()
    assert np.max(np.abs(C - C.T)) <= 1e-6 * np.abs(C).max()
    assert loewner_ok(C, K, G)


def test_gradient_workload_128():
    """128^3 sphere pack at 15% porosity: FP32 gradients of C11, C44 and trace(C)
    with FP64 averages, against the FP64 path, Euler's identity and a
    directional finite difference."""
    p = need_gpu()
    m = synth.workload_grad128()
    K, G = m.fields()
    announce("grad128", m.info)
    Ws = {"C11": np.diag([1.0, 0, 0, 0, 0, 0]), "C44": np.diag([0, 0, 0, 1.0, 0, 0]), "trace": np.eye(6)}
    with p.Context() as c:
        c.set_material(K, G)
        C, info = c.solve(precision="mixed", rtol=1e-9, keep_fields=True)
        g32 = {k: c.gradient(W, out_dtype="float32") for k, W in Ws.items()}
    with p.Context() as c:
        c.set_material(K, G)
        C64, _ = c.solve(precision="fp64", rtol=1e-10, keep_fields=True)
        g64 = {k: c.gradient(W, out_dtype="float64") for k, W in Ws.items()}
    assert matrix_rel(C, C64) <= 1e-6
    for k, W in Ws.items():
        dK, dG = g32[k]
        eK, eG = g64[k]
        assert np.max(np.abs(dK - eK)) <= 1e-5 * np.abs(eK).max(), k
        assert np.max(np.abs(dG - eG)) <= 1e-5 * np.abs(eG).max(), k
        J = float(np.sum(W * C64))
        assert float(np.sum(K * eK + G * eG)) == pytest.approx(J, rel=1e-7), k
    # directional derivative: soften a 6^3 block of matrix voxels by 2 %
    sl = (slice(40, 46), slice(50, 56), slice(60, 66))
    dirK = np.zeros_like(K); dirK[sl] = 0.02 * K[sl]
    dirG = np.zeros_like(G); dirG[sl] = 0.02 * G[sl]
    Cp, _ = p.solve(K + dirK, G + dirG, precision="fp64", rtol=1e-11, loads=[0, 3])
    Cm, _ = p.solve(K - dirK, G - dirG, precision="fp64", rtol=1e-11, loads=[0, 3])
    for k, (I, Jx) in (("C11", (0, 0)), ("C44", (3, 3))):
        fd = (Cp[I, Jx] - Cm[I, Jx]) / 2.0
        eK, eG = g64[k]
        ad = float(np.sum(eK * dirK + eG * dirG))
        assert ad == pytest.approx(fd, rel=2e-3), k
