"""ctypes declarations of the C ABI in include/ceff.h (argument marshalling only).

Loading fails loudly if the HIP library has not been built: there is no
fallback implementation of any step.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libceff.so")

CEFF_OK, CEFF_EINVAL, CEFF_ENOMEM, CEFF_EDEVICE = 0, -1, -2, -3
CEFF_ENOTCONV, CEFF_EDIVERGED, CEFF_EUNSUPPORTED, CEFF_ESTATE = -4, -5, -6, -7
CEFF_F32, CEFF_F64 = 0, 1
CEFF_HOST, CEFF_DEVICE = 0, 1
CEFF_PREC_FP64, CEFF_PREC_MIXED = 0, 1
CEFF_FUSE_AUTO = -1
CEFF_BC_PERIODIC, CEFF_BC_WALLS = 0, 1

STATUS_NAMES = {0: "CEFF_OK", -1: "CEFF_EINVAL", -2: "CEFF_ENOMEM", -3: "CEFF_EDEVICE", -4: "CEFF_ENOTCONV",
                -5: "CEFF_EDIVERGED", -6: "CEFF_EUNSUPPORTED", -7: "CEFF_ESTATE"}


class ceff_solve_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int64),
                ("check_every", ctypes.c_int), ("courant", ctypes.c_double), ("strouhal", ctypes.c_double),
                ("fuse_loads", ctypes.c_int), ("use_graph", ctypes.c_int), ("keep_fields", ctypes.c_int),
                ("autotune", ctypes.c_int), ("fold_ratio", ctypes.c_double), ("warm_u", ctypes.c_void_p)]


class ceff_stats(ctypes.Structure):
    _fields_ = [("step_launches", ctypes.c_int64), ("step_time_ms", ctypes.c_double),
                ("step_bytes", ctypes.c_double), ("voxel_updates", ctypes.c_double),
                ("outer_checks", ctypes.c_int64), ("solve_ms", ctypes.c_double),
                ("tile_bx", ctypes.c_int), ("tile_by", ctypes.c_int), ("tile_kc", ctypes.c_int),
                ("tile_group", ctypes.c_int), ("tile_variant", ctypes.c_int),
                ("fused_loads", ctypes.c_int), ("phase_moduli", ctypes.c_int),
                ("tile_occ", ctypes.c_int)]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)
_st = ctypes.c_int

# name -> (restype, argtypes); every symbol of include/ceff.h
SIGNATURES = {
    "ceff_default_opts": (None, [ctypes.POINTER(ceff_solve_opts)]),
    "ceff_check_grid": (_st, [_i64, _i64, _i64, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "ceff_auto_strouhal": (_st, [_i64, _i64, _i64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _dp]),
    "ceff_create": (_st, [ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "ceff_destroy": (None, [_vp]),
    "ceff_last_error": (ctypes.c_char_p, [_vp]),
    "ceff_set_grid": (_st, [_vp, _i64, _i64, _i64, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "ceff_set_isotropic": (_st, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int]),
    "ceff_set_phases": (_st, [_vp, _vp, ctypes.c_int, ctypes.c_int, _dp, _dp]),
    "ceff_set_stiffness": (_st, [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "ceff_set_boundary": (_st, [_vp, ctypes.c_int]),
    "ceff_solve": (_st, [_vp, ctypes.c_uint32, ctypes.POINTER(ceff_solve_opts), _dp, _dp, _i64, _i64p, _i64p]),
    "ceff_solve_batch": (_st, [_vp, ctypes.c_int, _i64p, _dp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int,
                               ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(ceff_solve_opts), _dp, _i64p]),
    "ceff_solve_batch_phases": (_st, [_vp, ctypes.c_int, _i64p, _dp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int,
                                      _dp, _dp, ctypes.c_uint32, ctypes.POINTER(ceff_solve_opts), _dp, _i64p]),
    "ceff_gradient": (_st, [_vp, _dp, _vp, _vp, ctypes.c_int, ctypes.c_int]),
    "ceff_apt_steps": (_st, [_vp, ctypes.c_int, _i64, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]),
    "ceff_residual": (_st, [_vp, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]),
    "ceff_average_stress": (_st, [_vp, ctypes.c_int, _dp, _dp]),
    "ceff_average_stress_noalloc": (_st, [_vp, ctypes.c_int, _vp, _dp]),
    "ceff_get_stats": (_st, [_vp, ctypes.POINTER(ceff_stats)]),
    "ceff_contribution_tensors": (_st, [_dp, _dp, ctypes.c_double, _dp, _dp]),
    "ceff_triaxial_offdiagonals": (_st, [_dp, _dp, _dp, _dp]),
    "ceff_triaxial_from_walls": (_st, [_dp, _dp]),
}

_lib = None


def load():
    """Load libceff.so (built in-tree by paper_2410_20441_amd/build.py).

    torch is imported first: torch ships its own HIP runtime with the same
    soname as the system one, and whichever is loaded first serves the whole
    process; loading torch's first keeps one runtime for both."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                              f"g.build()'` (hipcc, gfx950); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
