"""End-to-end parity of C* from the HIP path with the CPU oracle (GPU)."""
import json
import os

import numpy as np
import pytest

import closed_forms as cf
import oracle
import synth
from gpu_common import announce, matrix_rel, need_gpu

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def sphere32():
    m = synth.workload_sphere32()
    K, G = m.fields()
    C, info = oracle.ceff(K, G, rtol=1e-11)
    return K, G, C


@pytest.mark.parametrize("precision,fuse", [("fp64", False), ("fp64", True), ("mixed", True), ("mixed", False)])
def test_sphere32_matches_oracle(sphere32, precision, fuse):
    p = need_gpu()
    K, G, Co = sphere32
    announce("sphere32", precision, fuse)
    C, info = p.solve(K, G, precision=precision, fuse_loads=fuse, rtol=1e-8)
    assert info["status"] == 0
    assert matrix_rel(C, Co) <= 1e-6, matrix_rel(C, Co)
    assert np.all(info["iters"] > 0)


@pytest.mark.parametrize("shape,seed", [((13, 11, 9), 1), ((70, 6, 7), 2), ((5, 17, 30), 3)])
def test_random_fields_match_oracle(shape, seed):
    p = need_gpu()
    K, G = synth.random_fields(shape, seed, lo=(2.0, 1.0), hi=(90.0, 45.0))
    Co, _ = oracle.ceff(K, G, rtol=1e-12)
    for prec in ("fp64", "mixed"):
        announce("random", shape, prec)
        C, info = p.solve(K, G, precision=prec, rtol=1e-9)
        assert matrix_rel(C, Co) <= 1e-6


def test_anisotropic_spacing_matches_oracle():
    p = need_gpu()
    K, G = synth.random_fields((9, 12, 10), 4, lo=(5.0, 2.0), hi=(80.0, 40.0))
    h = (1.0, 0.6, 1.7)
    Co, _ = oracle.ceff(K, G, h=h, rtol=1e-12)
    C, _ = p.solve(K, G, h=h, precision="fp64", rtol=1e-9)
    assert matrix_rel(C, Co) <= 1e-6


def test_homogeneous_is_exact_without_iterations():
    p = need_gpu()
    K = np.full((6, 7, 8), 70.0); G = np.full((6, 7, 8), 32.0)
    for prec in ("fp64", "mixed"):
        C, info = p.solve(K, G, precision=prec)
        np.testing.assert_allclose(C, cf.c_iso(70.0, 32.0), rtol=1e-14, atol=1e-12)
        assert np.all(info["iters"] == 0)


def test_paper_layered_model_full_size():
    """Model 1 geometry at its full 191^3 size, six loads fused, mixed precision:
    Backus exactly (periodic), the analytic column to the printed digits."""
    p = need_gpu()
    g = json.load(open(os.path.join(GOLD, "table2_layered.json")))
    geo = g["geometry"]
    st, so = g["layers"]["stiff"], g["layers"]["soft"]
    m = synth.laminate_z(191, 191, 191, geo["stiff_layers"], geo["layer_thickness"],
                         stiff=(st["K"], st["G"]), soft=(so["K"], so["G"]))
    announce("laminate 191^3")
    ctx = p.Context()
    ctx.set_phases(m.phase, m.K_tab, m.G_tab)
    C, info = ctx.solve(precision="mixed", rtol=1e-8)
    ctx.close()
    f = m.info["f_stiff"]
    Cb = cf.backus_z([f, 1 - f], [st["K"], so["K"]], [st["G"], so["G"]])
    assert matrix_rel(C, Cb) <= 1e-6
    idx = {"C11": (0, 0), "C22": (1, 1), "C33": (2, 2), "C44": (3, 3), "C55": (4, 4), "C66": (5, 5),
           "C12": (0, 1), "C13": (0, 2), "C23": (1, 2)}
    for name, val in g["analytic_GPa"].items():
        assert round(C[idx[name]], 3) == pytest.approx(val, abs=1e-12), name


def test_hill_identity_full_size():
    """191^3 sphere pack with one shear modulus: Hill's exact bulk response."""
    p = need_gpu()
    m = synth.workload_spheres191()
    K, G = m.fields()
    G[:] = 32.0
    announce("hill 191^3")
    C, info = p.solve(K, G, loads=range(3), precision="mixed", rtol=1e-8)
    assert C[:3, :3].sum() / 9.0 == pytest.approx(cf.hill_uniform_shear(K, G), rel=1e-6)


def test_graph_and_direct_launches_agree():
    p = need_gpu()
    K, G = synth.random_fields((20, 18, 16), 11, lo=(2.0, 1.0), hi=(90.0, 45.0))
    Ca, ia = p.solve(K, G, precision="fp64", use_graph=True, rtol=1e-9)
    Cb, ib = p.solve(K, G, precision="fp64", use_graph=False, rtol=1e-9)
    assert np.array_equal(Ca, Cb)
    assert np.array_equal(ia["iters"], ib["iters"])


def test_batch_matches_per_sample_oracle():
    p = need_gpu()
    shapes = [(12, 12, 12), (10, 14, 9), (16, 8, 11), (7, 7, 20)]
    samples = [synth.random_fields(s, 20 + i, lo=(2.0, 1.0), hi=(90.0, 45.0)) for i, s in enumerate(shapes)]
    for prec in ("fp64", "mixed"):
        announce("batch", prec)
        C, it, info = p.solve_batch(samples, precision=prec, rtol=1e-9)
        for s, (K, G) in enumerate(samples):
            Co, _ = oracle.ceff(K, G, rtol=1e-12)
            assert matrix_rel(C[s], Co) <= 1e-6, (prec, s)
        assert np.all(it > 0)


def test_batch_mixed_phases_and_sizes():
    p = need_gpu()
    ms = [synth.gaussian_field_three_phase(n, 0xC4 + i) for i, n in enumerate((16, 20))]
    samples = [m.fields() for m in ms]
    C, it, info = p.solve_batch(samples, precision="mixed", rtol=1e-8)
    for s, (K, G) in enumerate(samples):
        Co, _ = oracle.ceff(K, G, rtol=1e-11)
        assert matrix_rel(C[s], Co) <= 1e-6


def test_batch_block_spans_largest_sample():
    """The default block of a batch is sized by its largest sample, not its first
    (32-cell rows for the 70-wide sample; the 8-wide first sample alone gives 16)."""
    p = need_gpu()
    samples = [synth.random_fields(s, 60 + i, lo=(2.0, 1.0), hi=(90.0, 45.0))
               for i, s in enumerate([(8, 8, 8), (70, 9, 6)])]
    announce("batch block extent")
    C, it, info = p.solve_batch(samples, precision="mixed", rtol=1e-9)
    assert info["stats"]["tile_bx"] == 32 and info["stats"]["tile_by"] == 8
    for s, (K, G) in enumerate(samples):
        Co, _ = oracle.ceff(K, G, rtol=1e-12)
        assert matrix_rel(C[s], Co) <= 1e-6, s


def test_batch_of_phase_images_equals_field_batch():
    """ceff_solve_batch_phases (one shared table, the phase-table kernel) gives
    the iterates of ceff_solve_batch on the expanded fields, and the oracle's C*."""
    p = need_gpu()
    ms = [synth.gaussian_field_three_phase(n, 0xC4 + i) for i, n in enumerate((16, 22, 19))]
    announce("batch of phase images", [m.phase.shape for m in ms])
    Cp, itp, infop = p.solve_batch_phases([m.phase for m in ms], ms[0].K_tab, ms[0].G_tab, precision="mixed",
                                          rtol=1e-9)
    assert infop["stats"]["phase_moduli"] == 1
    Cf, itf, infof = p.solve_batch([m.fields() for m in ms], precision="mixed", rtol=1e-9)
    assert infof["stats"]["phase_moduli"] == 0
    assert np.array_equal(itp, itf)
    assert np.max(np.abs(Cp - Cf)) <= 1e-12 * np.abs(Cf).max()
    for s, m in enumerate(ms):
        Co, _ = oracle.ceff(*m.fields(), rtol=1e-12)
        assert matrix_rel(Cp[s], Co) <= 1e-6, s
    bad = ms[0].phase.copy()
    bad[0, 0, 0] = 7
    with pytest.raises(p.CeffError):
        p.solve_batch_phases([bad, ms[1].phase], ms[0].K_tab, ms[0].G_tab, precision="mixed")


def test_gradient_matches_oracle():
    p = need_gpu()
    m = synth.workload_grad16()
    K, G = m.fields()
    Co, info, fields = oracle.ceff(K, G, rtol=1e-12, return_fields=True)
    W = np.zeros((6, 6)); W[0, 0] = 1.0; W[3, 3] = 0.5; W += np.eye(6) * 0.25
    dKo, dGo = oracle.gradient(K, G, fields, W)
    with p.Context() as c:
        c.set_material(K, G)
        C, _ = c.solve(precision="fp64", rtol=1e-11, keep_fields=True)
        dK, dG = c.gradient(W, out_dtype="float64")
    assert np.max(np.abs(dK - dKo)) <= 1e-6 * np.abs(dKo).max()
    assert np.max(np.abs(dG - dGo)) <= 1e-6 * np.abs(dGo).max()
    # Euler homogeneity of degree one
    J = float(np.sum(W * C))
    assert float(np.sum(K * dK + G * dG)) == pytest.approx(J, rel=1e-7)


def test_autograd_function():
    p = need_gpu()
    import torch
    K, G = synth.random_fields((10, 9, 8), 31, lo=(5.0, 2.0), hi=(80.0, 40.0))
    Kt = torch.tensor(K, device="cuda", requires_grad=True)
    Gt = torch.tensor(G, device="cuda", requires_grad=True)
    C = p.EffectiveStiffness.apply(Kt, Gt, {"precision": "fp64", "rtol": 1e-11})
    (C[0, 0] + C[3, 3]).backward()
    Co, info, fields = oracle.ceff(K, G, rtol=1e-12, return_fields=True)
    W = np.zeros((6, 6)); W[0, 0] = 1; W[3, 3] = 1
    dKo, dGo = oracle.gradient(K, G, fields, W)
    assert np.max(np.abs(Kt.grad.cpu().numpy() - dKo)) <= 1e-6 * np.abs(dKo).max()
    assert np.max(np.abs(Gt.grad.cpu().numpy() - dGo)) <= 1e-6 * np.abs(dGo).max()


def test_error_paths():
    p = need_gpu()
    import ctypes
    from paper_2410_20441_amd import _lib
    L = _lib.load()
    c = p.Context()
    h = c.h
    o = p.make_opts()
    C = np.zeros(36)
    dp = C.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.ceff_solve(h, 0x3F, ctypes.byref(o), dp, None, 0, None, None) == _lib.CEFF_ESTATE
    assert L.ceff_set_grid(h, 1, 4, 4, 1.0, 1.0, 1.0) == _lib.CEFF_EINVAL
    assert L.ceff_set_grid(h, 4, 4, 4, 1.0, -1.0, 1.0) == _lib.CEFF_EINVAL
    assert L.ceff_set_grid(h, 4, 4, 4, 1.0, 1.0, 1.0) == 0
    bad = np.full(64, 70.0); bad[5] = np.nan
    good = np.full(64, 32.0)
    assert L.ceff_set_isotropic(h, bad.ctypes.data, good.ctypes.data, 1, 0) == _lib.CEFF_EINVAL
    neg = np.full(64, 32.0); neg[3] = -1.0
    assert L.ceff_set_isotropic(h, good.ctypes.data, neg.ctypes.data, 1, 0) == _lib.CEFF_EINVAL
    ph = np.zeros(64, np.uint8); ph[7] = 3
    kt = np.array([70.0, 2.2]); gt = np.array([32.0, 1e-3])
    dkt = kt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)); dgt = gt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.ceff_set_phases(h, ph.ctypes.data, 0, 2, dkt, dgt) == _lib.CEFF_EINVAL
    assert L.ceff_set_stiffness(h, None, 21, 1, 0) == _lib.CEFF_EINVAL
    K, G = synth.random_fields((4, 4, 4), 1)
    assert L.ceff_set_isotropic(h, K.ctypes.data, G.ctypes.data, 1, 0) == 0
    for field, val in (("courant", 1.5), ("rtol", -1.0), ("check_every", 0), ("strouhal", -1.0),
                       ("strouhal", float("nan")),
                       ("precision", 7), ("max_iter", 0)):
        o2 = p.make_opts()
        setattr(o2, field, val)
        assert L.ceff_solve(h, 0x3F, ctypes.byref(o2), dp, None, 0, None, None) == _lib.CEFF_EINVAL, field
    assert L.ceff_solve(h, 0, ctypes.byref(o), dp, None, 0, None, None) == _lib.CEFF_EINVAL
    assert L.ceff_solve(h, 0x40, ctypes.byref(o), dp, None, 0, None, None) == _lib.CEFF_EINVAL
    W = np.eye(6)
    dK = np.zeros(64); dG = np.zeros(64)
    assert L.ceff_gradient(h, W.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), dK.ctypes.data, dG.ctypes.data,
                           1, 0) == _lib.CEFF_ESTATE
    # max_iter forces non-convergence; C is still filled
    o3 = p.make_opts(precision="fp64", max_iter=2, check_every=2)
    st = L.ceff_solve(h, 0x1, ctypes.byref(o3), dp, None, 0, None, None)
    assert st == _lib.CEFF_ENOTCONV
    assert np.all(np.isfinite(C.reshape(6, 6)[:, 0]))
    assert "max_iter" in p.ceff_last_error(h)
    c.close()


@pytest.mark.parametrize("tile", ["66,6,0,6,1", "66,6,0,3,0", "34,10,0,2,1", "34,14,5,1,1", "18,18,3,6,0"])
def test_fused_solve_independent_of_launch_shape(monkeypatch, tile):
    """Block extent, loads per block, z-chunk and prefetch change only the speed."""
    p = need_gpu()
    K, G = synth.random_fields((23, 19, 17), 41, lo=(2.0, 1.0), hi=(90.0, 45.0))
    monkeypatch.delenv("CEFF_TILE", raising=False)
    Cref, iref = p.solve(K, G, precision="mixed", rtol=1e-9)
    monkeypatch.setenv("CEFF_TILE", tile)
    announce("launch shape", tile)
    C, info = p.solve(K, G, precision="mixed", rtol=1e-9)
    assert info["stats"]["tile_group"] == int(tile.split(",")[3])
    assert np.array_equal(info["iters"], iref["iters"])
    assert np.max(np.abs(C - Cref)) <= 1e-12 * np.abs(Cref).max()


@pytest.mark.parametrize("tile", ["34,14,0,2,2", "34,14,7,6,2", "18,22,0,1,2", "34,14,0,2,3", "34,14,0,2,4", "18,14,5,1,4", "34,7,11,3,4", "66,6,0,1,5", "34,10,7,1,5", "10,66,0,1,5"])
def test_unrolled_march_matches(monkeypatch, tile):
    p = need_gpu()
    K, G = synth.random_fields((23, 19, 17), 41, lo=(2.0, 1.0), hi=(90.0, 45.0))
    monkeypatch.setenv("CEFF_TILE", "34,14,0,2,0")
    Cref, iref = p.solve(K, G, precision="mixed", rtol=1e-9)
    monkeypatch.setenv("CEFF_TILE", tile)
    announce("unrolled", tile)
    C, info = p.solve(K, G, precision="mixed", rtol=1e-9)
    assert np.array_equal(info["iters"], iref["iters"])
    assert np.max(np.abs(C - Cref)) <= 1e-12 * np.abs(Cref).max()
    # FP64, one load at a time: the variants are separate kernels whose compiler
    # may contract multiply-adds differently, so agreement is to rounding
    Cr, ir = p.solve(K, G, precision="fp64", rtol=1e-9, fuse_loads=False)
    monkeypatch.setenv("CEFF_TILE", "34,14,0,1,0")
    Cq, iq = p.solve(K, G, precision="fp64", rtol=1e-9, fuse_loads=False)
    assert np.array_equal(ir["iters"], iq["iters"])
    assert np.max(np.abs(Cr - Cq)) <= 1e-12 * np.abs(Cq).max()


@pytest.mark.parametrize("n,fields,fused", [(32, True, 1), (120, True, 1), (128, True, 0), (208, True, 1),
                                            (32, False, 0), (128, False, 0)])
def test_automatic_load_fusion(n, fields, fused):
    """With a phase image the loads run one after another (they share only the
    1-byte phase id); with K and G fields they run one after another exactly when
    one load's working set fits in the Infinity Cache and all six do not
    (homogeneous images: no iterations needed)."""
    p = need_gpu()
    m = synth.homogeneous(n)
    with p.Context() as c:
        if fields:
            c.set_material(*m.fields())
        else:
            c.set_phases(m.phase, m.K_tab, m.G_tab)
        C, info = c.solve(precision="mixed")
    assert info["stats"]["fused_loads"] == fused
    np.testing.assert_allclose(C, cf.c_iso(70.0, 32.0), rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("fuse", [False, True])
def test_large_grid_launch_shape(monkeypatch, fuse):
    """Beyond the Infinity Cache (a 320^3 pore pack: 0.8 GB for one load) the library
    switches one load per launch to 64 x 8 blocks of variant 9 with 32-plane chunks,
    and fused loads to 66 x 7 blocks with 48-plane chunks; the iterate is the one of
    the cache-resident shape."""
    p = need_gpu()
    m = synth.random_spheres(320, 0.10, 0x320)
    monkeypatch.delenv("CEFF_TILE", raising=False)
    announce("large-grid shape 320^3, fused", fuse)
    opts = dict(loads=range(6) if fuse else [0], precision="mixed", max_iter=400, check_every=200,
                allow_unconverged=True, fuse_loads=fuse)
    with p.Context() as c:
        c.set_phases(m.phase, m.K_tab, m.G_tab)
        C, info = c.solve(**opts)
        st = info["stats"]
        assert (st["tile_bx"], st["tile_by"], st["tile_kc"], st["tile_variant"]) == \
            ((66, 7, 48, 3) if fuse else (64, 8, 32, 9))
        assert st["tile_group"] == (2 if fuse else 1)
        monkeypatch.setenv("CEFF_TILE", "18,14,12,1,3,1,0" if not fuse else "66,7,12,2,3,1,0")
        C2, info2 = c.solve(**opts)
        assert info2["stats"]["tile_kc"] == 12
    cols = list(opts["loads"])
    assert np.max(np.abs(C[:, cols] - C2[:, cols])) <= 1e-12 * np.abs(C[:, cols]).max()
    assert np.array_equal(info["iters"], info2["iters"])


@pytest.mark.parametrize("phases", [True, False])
def test_large_batch_launch_shape(monkeypatch, phases):
    """A batch whose six-load working set exceeds the Infinity Cache (two 160^3 pore packs
    and a 96^3 one: 2.1 GB) takes 64 x 8 blocks of variant 9 with 16-plane chunks, from
    phase images and from K and G fields; a batch inside the cache keeps the 32 x 8 x 12
    default; the iterates and iteration counts are those of the default shape."""
    p = need_gpu()
    ms = [synth.random_spheres(160, 0.10, 0x160), synth.random_spheres(160, 0.12, 0x161),
          synth.random_spheres(96, 0.10, 0x96)]
    monkeypatch.delenv("CEFF_TILE", raising=False)
    announce("large-batch shape", phases)
    opts = dict(precision="mixed", max_iter=300, check_every=100, allow_unconverged=True)

    def run():
        if phases:
            return p.solve_batch_phases([m.phase for m in ms], ms[0].K_tab, ms[0].G_tab, **opts)
        return p.solve_batch([m.fields() for m in ms], **opts)

    C, it, info = run()
    st = info["stats"]
    assert (st["tile_bx"], st["tile_by"], st["tile_kc"], st["tile_variant"]) == (64, 8, 16, 9)
    monkeypatch.setenv("CEFF_TILE", "32,8,24,1,9,1,1")
    C2, it2, info2 = run()
    assert (info2["stats"]["tile_bx"], info2["stats"]["tile_kc"]) == (32, 24)
    assert np.max(np.abs(C - C2)) <= 1e-12 * np.abs(C).max()
    assert np.array_equal(it, it2)
    monkeypatch.delenv("CEFF_TILE")
    _, _, info3 = p.solve_batch_phases([np.ascontiguousarray(m.phase[:48, :48, :48]) for m in ms], ms[0].K_tab,
                                       ms[0].G_tab, **opts)
    st3 = info3["stats"]
    assert (st3["tile_bx"], st3["tile_by"], st3["tile_kc"]) == (32, 8, 12)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_warm_start(precision):
    """An initial guess (ceff_solve_opts::warm_u): the oracle's converged fields need no
    iterations in mixed precision (their residual is already below rtol) and at most one
    check interval in FP64; 90% of them needs fewer iterations than the zero start; C*
    keeps the oracle's value.  With walls the option is refused."""
    p = need_gpu()
    from paper_2410_20441_amd import _lib
    K, G = synth.random_fields((12, 10, 9), 77, lo=(2.0, 1.0), hi=(90.0, 45.0))
    U = np.stack([oracle.solve_load(K, G, J, rtol=1e-13)[0] for J in range(6)])
    Co, _ = oracle.ceff(K, G, rtol=1e-12)
    announce("warm start", precision)
    with p.Context() as c:
        c.set_material(K, G)
        C0, i0 = c.solve(precision=precision, rtol=1e-9)
        C1, i1 = c.solve(precision=precision, rtol=1e-9, warm_u=U)
        C2, i2 = c.solve(precision=precision, rtol=1e-9, warm_u=0.9 * U)
        if precision == "mixed":
            assert np.all(i1["iters"] == 0)
        else:
            assert i1["iters"].max() <= 100
        assert np.all(i2["iters"] < i0["iters"]), (i2["iters"], i0["iters"])
        for C in (C0, C1, C2):
            assert matrix_rel(C, Co) <= 1e-6
        c.set_boundary("walls")
        with pytest.raises(p.CeffError) as e:
            c.solve(loads=(0,), precision=precision, warm_u=U)
        assert e.value.status == _lib.CEFF_EUNSUPPORTED
