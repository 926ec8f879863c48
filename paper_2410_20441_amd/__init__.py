"""Effective elastic stiffness of voxel images on MI355X (gfx950).

Thin Python binding of the C ABI declared in ``include/ceff.h``: the
``ceff_*`` functions below have the same names and arguments as the C entry
points and only marshal arguments; every step of the computation runs in the
HIP kernels of ``libceff.so``.  PyTorch is used for device memory and streams
only.  If the library is missing, importing this package raises.

Convenience layer:
  * :class:`Context` -- owns a ``ceff_ctx``; ``solve``, ``gradient`` etc.
  * :func:`solve` -- one image, returns the 6x6 C* (FP64) and run info.
  * :func:`solve_batch` -- several images of different sizes in one solve.
  * :func:`contribution_tensors` -- compliance/stiffness contribution tensors
    of inclusions from C*.
  * :class:`EffectiveStiffness` -- ``torch.autograd.Function``: C*(K, G) with
    the adjoint gradient on backward.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (CEFF_DEVICE, CEFF_F32, CEFF_F64, CEFF_FUSE_AUTO, CEFF_HOST, CEFF_PREC_FP64, CEFF_PREC_MIXED,
                   ceff_solve_opts, ceff_stats)

_L = _lib.load()

__all__ = ["ceff_default_opts", "ceff_check_grid", "ceff_auto_strouhal", "ceff_create", "ceff_destroy", "ceff_last_error", "ceff_set_grid",
           "ceff_set_isotropic", "ceff_set_phases", "ceff_set_stiffness", "ceff_set_boundary", "ceff_solve",
           "ceff_solve_batch", "ceff_solve_batch_phases", "solve_batch_phases",
           "ceff_gradient", "ceff_apt_steps", "ceff_residual", "ceff_average_stress", "ceff_average_stress_noalloc", "ceff_get_stats",
           "ceff_contribution_tensors", "ceff_triaxial_offdiagonals", "ceff_triaxial_from_walls", "triaxial_offdiagonals", "CeffError", "Context", "solve", "solve_batch", "contribution_tensors",
           "EffectiveStiffness", "library_path"]

library_path = _lib.LIB_PATH


class CeffError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# ---- same-name wrappers of the C entry points ------------------------------------

def ceff_default_opts(o=None):
    o = o if o is not None else ceff_solve_opts()
    _L.ceff_default_opts(ctypes.byref(o))
    return o


def ceff_check_grid(nx, ny, nz, hx=1.0, hy=1.0, hz=1.0):
    """Status of the grid against the library's limits (host only, no device)."""
    return _L.ceff_check_grid(nx, ny, nz, hx, hy, hz)


def ceff_auto_strouhal(nx, ny, nz, hx=1.0, hy=1.0, hz=1.0, courant=0.95):
    """The Strouhal number the solver picks when strouhal = 0 (host only, no device)."""
    st = ctypes.c_double()
    rc = _L.ceff_auto_strouhal(nx, ny, nz, hx, hy, hz, courant, ctypes.byref(st))
    if rc != 0:
        raise CeffError(rc, "bad grid or courant number")
    return st.value


def ceff_create(device=0, hip_stream=None):
    h = ctypes.c_void_p()
    st = _L.ceff_create(int(device), hip_stream, ctypes.byref(h))
    if st != 0:
        raise CeffError(st, "ceff_create failed (no usable HIP device?)")
    return h


def ceff_destroy(ctx):
    _L.ceff_destroy(ctx)


def ceff_last_error(ctx):
    m = _L.ceff_last_error(ctx)
    return m.decode() if m else ""


def _check(ctx, st, allow=()):
    if st != 0 and st not in allow:
        raise CeffError(st, ceff_last_error(ctx))
    return st


def ceff_set_grid(ctx, nx, ny, nz, hx=1.0, hy=1.0, hz=1.0):
    return _check(ctx, _L.ceff_set_grid(ctx, nx, ny, nz, hx, hy, hz))


def ceff_set_isotropic(ctx, K, G, dtype, where):
    return _check(ctx, _L.ceff_set_isotropic(ctx, K, G, dtype, where))


def ceff_set_phases(ctx, phase, where, nphase, K_tab, G_tab):
    return _check(ctx, _L.ceff_set_phases(ctx, phase, where, nphase, K_tab, G_tab))


def ceff_set_stiffness(ctx, c, ncomp, dtype, where):
    return _check(ctx, _L.ceff_set_stiffness(ctx, c, ncomp, dtype, where))


def ceff_set_boundary(ctx, mode):
    return _check(ctx, _L.ceff_set_boundary(ctx, mode))


def ceff_solve(ctx, load_mask, opts, C_out, hist, hist_cap, hist_len, iters_out, allow=()):
    return _check(ctx, _L.ceff_solve(ctx, load_mask, opts, C_out, hist, hist_cap, hist_len, iters_out), allow)


def ceff_solve_batch(ctx, nsamples, dims, h, K, G, dtype, where, load_mask, opts, C_out, iters_out, allow=()):
    return _check(ctx, _L.ceff_solve_batch(ctx, nsamples, dims, h, K, G, dtype, where, load_mask, opts, C_out,
                                           iters_out), allow)


def ceff_solve_batch_phases(ctx, nsamples, dims, h, phase, where, nphase, K_tab, G_tab, load_mask, opts, C_out,
                            iters_out, allow=()):
    return _check(ctx, _L.ceff_solve_batch_phases(ctx, nsamples, dims, h, phase, where, nphase, K_tab, G_tab,
                                                  load_mask, opts, C_out, iters_out), allow)


def ceff_gradient(ctx, W, dK, dG, dtype, where):
    return _check(ctx, _L.ceff_gradient(ctx, W, dK, dG, dtype, where))


def ceff_apt_steps(ctx, J, nsteps, precision, courant, strouhal, u_out, u_prev_out):
    return _check(ctx, _L.ceff_apt_steps(ctx, J, nsteps, precision, courant, strouhal, u_out, u_prev_out))


def ceff_residual(ctx, J, precision, u, r_out, norm2):
    return _check(ctx, _L.ceff_residual(ctx, J, precision, u, r_out, norm2))


def ceff_average_stress(ctx, J, u, out6):
    return _check(ctx, _L.ceff_average_stress(ctx, J, u, out6))


def ceff_average_stress_noalloc(ctx, J, u, out6):
    """u: device pointer (int or c_void_p) to 3N FP64 values on the context's device."""
    return _check(ctx, _L.ceff_average_stress_noalloc(ctx, J, u, out6))


def ceff_get_stats(ctx, out):
    return _check(ctx, _L.ceff_get_stats(ctx, out))


def ceff_triaxial_offdiagonals(sig_mean, eps_mean, C_diag, out):
    st = _L.ceff_triaxial_offdiagonals(sig_mean, eps_mean, C_diag, out)
    if st != 0:
        raise CeffError(st, "inputs must be finite and every mean strain nonzero")
    return st


def ceff_triaxial_from_walls(C_walls, out):
    st = _L.ceff_triaxial_from_walls(C_walls, out)
    if st != 0:
        raise CeffError(st, "the wall columns must be finite")
    return st


def ceff_contribution_tensors(C_eff, C_host, phi, H_out, N_out):
    st = _L.ceff_contribution_tensors(C_eff, C_host, phi, H_out, N_out)
    if st != 0:
        raise CeffError(st, "phi must be in (0, 1] and both stiffness matrices finite and invertible")
    return st


# ---- marshalling helpers ----------------------------------------------------------

def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _array_arg(x, name):
    """(pointer, dtype code, where code, keepalive) for a numpy array or torch tensor."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(x, torch.Tensor):
        if x.dtype not in (torch.float32, torch.float64):
            raise TypeError(f"{name}: dtype must be float32 or float64")
        x = x.contiguous()
        where = CEFF_DEVICE if x.is_cuda else CEFF_HOST
        return ctypes.c_void_p(x.data_ptr()), (CEFF_F64 if x.dtype == torch.float64 else CEFF_F32), where, x
    a = np.ascontiguousarray(x)
    if a.dtype not in (np.float32, np.float64):
        a = a.astype(np.float64)
    return ctypes.c_void_p(a.ctypes.data), (CEFF_F64 if a.dtype == np.float64 else CEFF_F32), CEFF_HOST, a


def _shape3(x):
    if x.ndim != 3:
        raise ValueError("moduli must be 3-D arrays shaped (nz, ny, nx)")
    nz, ny, nx = x.shape
    return int(nx), int(ny), int(nz)


def _torch_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover
        pass
    return None


def make_opts(precision="mixed", rtol=1e-8, max_iter=2_000_000, check_every=100, courant=0.95, strouhal=0.0,
              fuse_loads="auto", use_graph=True, keep_fields=False, autotune=False, fold_ratio=1e-3):
    """Solve options.  fuse_loads: True (one launch per iteration for all loads), False (one load
    after another) or "auto" (the library decides from the working set and the cache size).
    strouhal: 0 picks it from the box (ceff_auto_strouhal)."""
    o = ceff_default_opts()
    o.precision = CEFF_PREC_MIXED if precision == "mixed" else CEFF_PREC_FP64
    o.rtol = rtol
    o.max_iter = max_iter
    o.check_every = check_every
    o.courant = courant
    o.strouhal = strouhal
    o.fuse_loads = CEFF_FUSE_AUTO if isinstance(fuse_loads, str) and fuse_loads == "auto" else int(bool(fuse_loads))
    o.use_graph = int(bool(use_graph))
    o.keep_fields = int(bool(keep_fields))
    o.autotune = int(bool(autotune))
    o.fold_ratio = fold_ratio
    return o


class Context:
    """Owns one ceff_ctx on a device (default: torch's current stream)."""

    def __init__(self, device=0, stream=None):
        self.h = ceff_create(device, stream if stream is not None else _torch_stream())
        self.shape = None

    def close(self):
        if self.h:
            ceff_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_material(self, K, G, h=(1.0, 1.0, 1.0)):
        nx, ny, nz = _shape3(K)
        if tuple(G.shape) != tuple(K.shape):
            raise ValueError("K and G shapes differ")
        ceff_set_grid(self.h, nx, ny, nz, *map(float, h))
        pK, dt, wh, kK = _array_arg(K, "K")
        pG, dt2, wh2, kG = _array_arg(G, "G")
        if dt2 != dt or wh2 != wh:
            raise TypeError("K and G must share dtype and device")
        ceff_set_isotropic(self.h, pK, pG, dt, wh)
        self.shape = (nz, ny, nx)
        self.h_spacing = tuple(map(float, h))

    def set_stiffness(self, C, h=(1.0, 1.0, 1.0)):
        """Anisotropic cells (numpy or torch, float32/float64): C shaped (9, nz, ny, nx), orthotropic
        constants C11 C22 C33 C23 C13 C12 C44 C55 C66; or (21, nz, ny, nx), general cells, the upper
        triangle of the 6x6 Voigt matrix row by row (C11 C12 ... C16 C22 ... C66)."""
        if C.ndim != 4 or C.shape[0] not in (9, 21):
            raise ValueError("C must be shaped (9, nz, ny, nx) or (21, nz, ny, nx)")
        nz, ny, nx = (int(v) for v in C.shape[1:])
        ceff_set_grid(self.h, nx, ny, nz, *map(float, h))
        p, dt, wh, keep = _array_arg(C, "C")
        ceff_set_stiffness(self.h, p, int(C.shape[0]), dt, wh)
        self.shape = (nz, ny, nx)
        self.h_spacing = tuple(map(float, h))

    def set_boundary(self, mode):
        """"periodic" (default) or "walls" (the paper's direct tests: loads 0..2 run the
        normal test with rigid, free-slip walls, loads 3..5 the simple-shear test)."""
        ceff_set_boundary(self.h, {"periodic": _lib.CEFF_BC_PERIODIC, "walls": _lib.CEFF_BC_WALLS}[mode])

    def set_phases(self, phase, K_tab, G_tab, h=(1.0, 1.0, 1.0)):
        ph = np.ascontiguousarray(phase, np.uint8)
        nx, ny, nz = _shape3(ph)
        ceff_set_grid(self.h, nx, ny, nz, *map(float, h))
        Kt = np.ascontiguousarray(K_tab, np.float64)
        Gt = np.ascontiguousarray(G_tab, np.float64)
        ceff_set_phases(self.h, ctypes.c_void_p(ph.ctypes.data), CEFF_HOST, len(Kt), _dptr(Kt), _dptr(Gt))
        self.shape = (nz, ny, nx)
        self.h_spacing = tuple(map(float, h))

    def solve(self, loads=range(6), hist_cap=100000, allow_unconverged=False, warm_u=None, **kw):
        """warm_u: optional initial displacement fluctuation, (6, 3, nz, ny, nx) FP64 (entries of
        loads not solved are ignored), see ceff_solve_opts::warm_u."""
        o = make_opts(**kw)
        if warm_u is not None:
            warm = np.ascontiguousarray(warm_u, np.float64)
            if warm.size != 6 * 3 * int(np.prod(self.shape)):
                raise ValueError("warm_u must hold 6 x 3N values")
            o.warm_u = warm.ctypes.data  # `warm` stays referenced until the call returns
        mask = 0
        for J in loads:
            mask |= 1 << int(J)
        C = np.full(36, np.nan)
        hist = np.zeros(3 * hist_cap)
        hl = ctypes.c_int64(0)
        it = np.zeros(6, np.int64)
        allow = (_lib.CEFF_ENOTCONV, _lib.CEFF_EDIVERGED) if allow_unconverged else ()
        st = ceff_solve(self.h, mask, ctypes.byref(o), _dptr(C), _dptr(hist), hist_cap, ctypes.byref(hl),
                        it.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), allow)
        n = min(hl.value, hist_cap)
        return C.reshape(6, 6), {"status": st, "iters": it, "hist": hist[:3 * n].reshape(n, 3),
                                 "stats": self.stats()}

    def stats(self):
        s = ceff_stats()
        ceff_get_stats(self.h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def gradient(self, W, out_dtype="float32", device=None):
        W = np.ascontiguousarray(W, np.float64).reshape(36)
        if device is not None:
            import torch
            dt = torch.float32 if out_dtype == "float32" else torch.float64
            dK = torch.empty(self.shape, dtype=dt, device=device)
            dG = torch.empty(self.shape, dtype=dt, device=device)
            ceff_gradient(self.h, _dptr(W), ctypes.c_void_p(dK.data_ptr()), ctypes.c_void_p(dG.data_ptr()),
                          CEFF_F32 if dt == torch.float32 else CEFF_F64, CEFF_DEVICE)
            return dK, dG
        npdt = np.float32 if out_dtype == "float32" else np.float64
        dK = np.empty(self.shape, npdt)
        dG = np.empty(self.shape, npdt)
        ceff_gradient(self.h, _dptr(W), ctypes.c_void_p(dK.ctypes.data), ctypes.c_void_p(dG.ctypes.data),
                      CEFF_F32 if npdt == np.float32 else CEFF_F64, CEFF_HOST)
        return dK, dG

    def apt_steps(self, J, nsteps, precision="fp64", courant=0.95, strouhal=2.0):
        n = int(np.prod(self.shape))
        u = np.empty(3 * n)
        up = np.empty(3 * n)
        ceff_apt_steps(self.h, J, nsteps, CEFF_PREC_MIXED if precision == "mixed" else CEFF_PREC_FP64, courant,
                       strouhal, _dptr(u), _dptr(up))
        return u.reshape((3,) + self.shape), up.reshape((3,) + self.shape)

    def residual(self, J, u, precision="fp64"):
        u = np.ascontiguousarray(u, np.float64)
        r = np.empty_like(u)
        n2 = ctypes.c_double()
        ceff_residual(self.h, J, CEFF_PREC_MIXED if precision == "mixed" else CEFF_PREC_FP64, _dptr(u), _dptr(r),
                      ctypes.byref(n2))
        return r, n2.value

    def average_stress(self, J, u):
        u = np.ascontiguousarray(u, np.float64)
        out = np.empty(6)
        ceff_average_stress(self.h, J, _dptr(u), _dptr(out))
        return out


def solve(K, G, h=(1.0, 1.0, 1.0), loads=range(6), device=0, **kw):
    """C* (6x6, FP64) of per-voxel moduli K, G shaped (nz, ny, nx)."""
    with Context(device) as c:
        c.set_material(K, G, h)
        return c.solve(loads=loads, **kw)


def contribution_tensors(C_eff, C_host, phi):
    """Compliance and stiffness contribution tensors (H, N), 6x6 Voigt, of inclusions of
    volume fraction phi: S* = S_host + phi H and C* = C_host + phi N (see ceff.h)."""
    Ce = np.ascontiguousarray(C_eff, np.float64).reshape(36)
    Ch = np.ascontiguousarray(C_host, np.float64).reshape(36)
    H = np.empty(36)
    N = np.empty(36)
    ceff_contribution_tensors(_dptr(Ce), _dptr(Ch), float(phi), _dptr(H), _dptr(N))
    return H.reshape(6, 6), N.reshape(6, 6)


def triaxial_offdiagonals(C_walls):
    """(C12, C13, C23) by the paper's triaxial direct test from the normal wall-test
    columns of C_walls (loads 0-2 solved with walls): the triaxial test with unit
    strains is their sum, and C11, C22, C33 are their diagonal (see ceff.h)."""
    C = np.ascontiguousarray(np.asarray(C_walls, np.float64).reshape(36))
    out = np.empty(3)
    ceff_triaxial_from_walls(_dptr(C), _dptr(out))
    return out


def solve_batch(samples, h=None, loads=range(6), device=0, allow_unconverged=False, **kw):
    """samples: list of (K, G) pairs (numpy or torch, same dtype/device for all).
    Returns C (nsamples, 6, 6), iterations (nsamples, 6), stats."""
    ns = len(samples)
    dims = np.zeros(3 * ns, np.int64)
    hh = np.ones(3 * ns)
    Kp = (ctypes.c_void_p * ns)()
    Gp = (ctypes.c_void_p * ns)()
    keep = []
    dt = wh = None
    for s, (K, G) in enumerate(samples):
        dims[3 * s:3 * s + 3] = _shape3(K)
        if h is not None:
            hh[3 * s:3 * s + 3] = h[s]
        pK, d1, w1, kK = _array_arg(K, "K")
        pG, d2, w2, kG = _array_arg(G, "G")
        if dt is None:
            dt, wh = d1, w1
        if (d1, w1, d2, w2) != (dt, wh, dt, wh):
            raise TypeError("all moduli must share dtype and device")
        Kp[s] = pK
        Gp[s] = pG
        keep += [kK, kG]
    o = make_opts(**kw)
    mask = 0
    for J in loads:
        mask |= 1 << int(J)
    C = np.full(36 * ns, np.nan)
    it = np.zeros(6 * ns, np.int64)
    with Context(device) as c:
        allow = (_lib.CEFF_ENOTCONV, _lib.CEFF_EDIVERGED) if allow_unconverged else ()
        st = ceff_solve_batch(c.h, ns, dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(hh), Kp, Gp, dt,
                              wh, mask, ctypes.byref(o), _dptr(C), it.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              allow)
        stats = c.stats()
    return C.reshape(ns, 6, 6), it.reshape(ns, 6), {"status": st, "stats": stats}


def solve_batch_phases(phases, K_tab, G_tab, h=None, loads=range(6), device=0, allow_unconverged=False, **kw):
    """phases: list of uint8 phase images (numpy, host) sharing the table (K_tab, G_tab).
    Returns C (nsamples, 6, 6), iterations (nsamples, 6), stats."""
    ns = len(phases)
    dims = np.zeros(3 * ns, np.int64)
    hh = np.ones(3 * ns)
    ptrs = (ctypes.c_void_p * ns)()
    keep = []
    for s, ph in enumerate(phases):
        a = np.ascontiguousarray(ph, np.uint8)
        dims[3 * s:3 * s + 3] = _shape3(a)
        if h is not None:
            hh[3 * s:3 * s + 3] = h[s]
        ptrs[s] = ctypes.c_void_p(a.ctypes.data)
        keep.append(a)
    Kt = np.ascontiguousarray(K_tab, np.float64)
    Gt = np.ascontiguousarray(G_tab, np.float64)
    o = make_opts(**kw)
    mask = 0
    for J in loads:
        mask |= 1 << int(J)
    C = np.full(36 * ns, np.nan)
    it = np.zeros(6 * ns, np.int64)
    with Context(device) as c:
        allow = (_lib.CEFF_ENOTCONV, _lib.CEFF_EDIVERGED) if allow_unconverged else ()
        st = ceff_solve_batch_phases(c.h, ns, dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(hh), ptrs,
                                     CEFF_HOST, len(Kt), _dptr(Kt), _dptr(Gt), mask, ctypes.byref(o), _dptr(C),
                                     it.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), allow)
        stats = c.stats()
    return C.reshape(ns, 6, 6), it.reshape(ns, 6), {"status": st, "stats": stats}


def _autograd_function():
    import torch

    class EffectiveStiffness(torch.autograd.Function):
        """C* = EffectiveStiffness.apply(K, G[, opts_dict]) for per-voxel moduli on a GPU.

        Forward solves all six loads and keeps the converged displacements;
        backward evaluates the adjoint gradient in one kernel (no second solve).
        """

        @staticmethod
        def forward(ctx, K, G, opts=None):
            opts = dict(opts or {})
            opts["keep_fields"] = True
            c = Context((K.device.index or 0) if K.is_cuda else 0)
            c.set_material(K.detach(), G.detach())
            C, info = c.solve(**opts)
            ctx.ceff_ctx = c
            ctx.shape = K.shape
            ctx.dtype = K.dtype
            return torch.from_numpy(C).to(device=K.device)

        @staticmethod
        def backward(ctx, grad_C):
            c = ctx.ceff_ctx
            W = grad_C.detach().to("cpu", torch.float64).numpy()
            dev = grad_C.device if grad_C.is_cuda else None
            dK, dG = c.gradient(W, out_dtype="float64" if ctx.dtype == torch.float64 else "float32", device=dev)
            if dev is None:
                dK, dG = torch.from_numpy(dK), torch.from_numpy(dG)
            c.close()
            return dK, dG, None

    return EffectiveStiffness


def __getattr__(name):
    if name == "EffectiveStiffness":
        return _autograd_function()
    raise AttributeError(name)
