"""Property contribution tensors of inclusions (GPU).

H = (C*^-1 - S_host) / phi and N = (C* - C_host) / phi from the effective
stiffness of an image holding one inclusion (paper: Model 2, the relation
S* = S1 + phi H, and the appendix on the property contribution tensor), solved
through the batch path, checked against

* the same formula applied (with numpy) to the oracle's C* of the same images,
  to the parity tolerance of C* (exact up to the solve);
* Eshelby's single-inclusion tensor (tests/closed_forms.py) as the inclusion is
  resolved more finely at fixed volume fraction: the error must shrink.  The
  staircase boundary makes this a convergence check, not an equality."""
import numpy as np
import pytest

import closed_forms as cf
import oracle
import synth
from gpu_common import announce, need_gpu

pytestmark = pytest.mark.gpu

HOST = (36.0, 44.0)                     # background of the paper's Model 2
INCLUSIONS = {"soft": (7.2, 8.8), "stiff": (180.0, 220.0), "pore": (1e-3, 2e-3)}


def voigt_compliance(H_mandel):
    w = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])
    return H_mandel * np.outer(w, w)


def eshelby_H(semi_axes, inc):
    C1 = cf.c_iso(*HOST)
    K, G = HOST
    nu = (3 * K - 2 * G) / (2 * (3 * K + G))
    a = np.asarray(semi_axes, float)
    return voigt_compliance(cf.compliance_contribution(C1, cf.c_iso(*inc), cf.eshelby_tensor(a / a.max(), nu)))


def test_contribution_tensors_definition():
    p = need_gpu()
    rng = synth.SplitMix64(7)
    A = rng.uniform_array(36).reshape(6, 6)
    Ce = A @ A.T + 6 * np.eye(6)
    Ch = cf.c_iso(36.0, 44.0)
    H, N = p.contribution_tensors(Ce, Ch, 0.25)
    np.testing.assert_allclose(H, (np.linalg.inv(Ce) - np.linalg.inv(Ch)) / 0.25, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(N, (Ce - Ch) / 0.25, rtol=1e-15)
    for bad_phi in (0.0, -0.1, 1.5, float("nan")):
        with pytest.raises(p.CeffError):
            p.contribution_tensors(Ce, Ch, bad_phi)
    with pytest.raises(p.CeffError):
        p.contribution_tensors(np.ones((6, 6)), Ch, 0.5)


def test_batch_contributions_match_oracle():
    """Several single-inclusion images, uneven sizes, in one batch solve."""
    p = need_gpu()
    cases = [((20, 20, 20), (5, 5, 5), "soft"), ((24, 22, 18), (7, 7, 2.5), "pore"),
             ((16, 18, 26), (3, 3, 7.5), "stiff")]
    ms = [synth.centred_spheroid(n, ax, matrix=HOST, inclusion=INCLUSIONS[c]) for n, ax, c in cases]
    announce("contribution batch", [m.phase.shape for m in ms])
    C, it, info = p.solve_batch([m.fields() for m in ms], precision="mixed", rtol=1e-9)
    C1 = cf.c_iso(*HOST)
    for s, m in enumerate(ms):
        Co, _ = oracle.ceff(*m.fields(), rtol=1e-12)
        phi = m.info["phi"]
        H, N = p.contribution_tensors(C[s], C1, phi)
        Ho = (np.linalg.inv(Co) - np.linalg.inv(C1)) / phi
        No = (Co - C1) / phi
        assert np.abs(N - No).max() <= 1e-6 * np.abs(Co).max() / phi, s
        # H amplifies C errors by |S*| |S1|-ish factors; both are O(1/modulus)
        assert np.abs(H - Ho).max() <= 1e-5 * np.abs(Ho).max(), (s, np.abs(H - Ho).max() / np.abs(Ho).max())


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 0.5), (0.5, 0.5, 1)], ids=["sphere", "oblate", "prolate"])
@pytest.mark.parametrize("contrast", ["soft", "stiff", "pore"])
def test_spheroid_contribution_converges_to_eshelby(contrast, shape):
    """Spheroid of largest semi-axis r in a box of 8r (phi fixed as r grows).  The
    staircase boundary gives an O(1/r) error against Eshelby's tensor: it must fall as
    r grows from 8 to 16 voxels, and the first-order extrapolation 2 H(16) - H(8) must
    leave only the small interaction error of the periodic array at this phi."""
    p = need_gpu()
    inc = INCLUSIONS[contrast]
    He = eshelby_H(shape, inc)
    Hs, errs = [], []
    for r in (8, 16):
        m = synth.centred_spheroid(8 * r, tuple(r * f for f in shape), matrix=HOST, inclusion=inc)
        announce("eshelby spheroid", contrast, shape, r)
        C, info = p.solve(*m.fields(np.float32), precision="mixed", rtol=1e-8)
        H, _ = p.contribution_tensors(C, cf.c_iso(*HOST), m.info["phi"])
        Hs.append(H)
        errs.append(np.abs(H - He).max() / np.abs(He).max())
        print(contrast, "r", r, "phi %.5f" % m.info["phi"], "max |H - H_Eshelby| / max |H_Eshelby| = %.4f" % errs[-1])
    ext = np.abs(2 * Hs[1] - Hs[0] - He).max() / np.abs(He).max()
    print(contrast, "extrapolated error %.4f" % ext)
    assert errs[1] < 0.75 * errs[0]
    assert ext < 0.03
