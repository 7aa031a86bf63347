"""ctypes view of libfo_stokes.so (declarations mirror include/fo_stokes.h).

The library must be built in-tree (python -m paper_2204_04321_amd.build); there is
no fallback: loading fails loudly when the shared object is missing.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfo_stokes.so")

FO_OK, FO_EINVAL, FO_ENOMEM, FO_EDEVICE, FO_EDEGENERATE, FO_ENONFINITE, FO_ENOTCONV = 0, -1, -2, -3, -4, -5, -6
FO_TET4, FO_WEDGE6, FO_HEX8 = 4, 6, 8
FO_F64, FO_F32 = 0, 1
FO_JAC_NEWTON, FO_JAC_PICARD = 0, 1


class FoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [
        ("elem", C.c_int32), ("n_base_verts", C.c_int32), ("n_base_cells", C.c_int32),
        ("n_layers", C.c_int32),
        ("base_xy", C.c_void_p), ("base_cells", C.c_void_p), ("surface", C.c_void_p),
        ("thickness", C.c_void_p), ("beta", C.c_void_p), ("sigma", C.c_void_p),
        ("A", C.c_double), ("n", C.c_double), ("rho", C.c_double), ("g", C.c_double),
        ("eps0", C.c_double),
        ("front_edges", C.c_void_p), ("n_front_edges", C.c_int32), ("rho_w", C.c_double),
    ]


class NewtonOpts(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("max_newton", C.c_int32), ("lin_rtol", C.c_double),
        ("gmres_restart", C.c_int32), ("max_lin", C.c_int32), ("jac_dtype", C.c_int32),
        ("max_backtracks", C.c_int32), ("init", C.c_int32), ("linear_solver", C.c_int32),
        ("mlp_params", C.c_void_p), ("mlp_norm", C.c_void_p), ("learned_fallback", C.c_int32),
        ("learned_smooth", C.c_int32), ("preconditioner", C.c_int32), ("mdsc", C.c_void_p),
    ]


class NewtonReport(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("newton_its", C.c_int32), ("lin_its", C.c_int64),
        ("residual_calls", C.c_int32), ("jacobian_calls", C.c_int32), ("backtracks", C.c_int32),
        ("f0_norm", C.c_double), ("final_norm", C.c_double), ("final_rel", C.c_double),
        ("ms_total_fill", C.c_double), ("ms_prec_construction", C.c_double),
        ("ms_linear_solve", C.c_double), ("ms_total_solve", C.c_double),
        ("res_hist", C.c_double * 64),
        ("init_used", C.c_int32), ("learned_fallbacks", C.c_int32),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "res_hist"}
        d["res_hist"] = [self.res_hist[i] for i in range(min(64, self.newton_its + 1))]
        return d


FO_INIT_USER, FO_INIT_SIA, FO_INIT_LEARNED = 0, 1, 2
FO_LIN_GMRES, FO_LIN_PCG = 0, 1
FO_PREC_COLUMN, FO_PREC_MDSC = 0, 1
FO_MDSC_WEIGHTS, FO_MDSC_PLANE, FO_MDSC_BOUND = 0, 1, 2

_lib = None


def _declare(lib):
    vp, i32, i64p = C.c_void_p, C.c_int32, C.POINTER(C.c_int64)
    sig = {
        "fo_mesh_create": (C.c_int, [C.POINTER(MeshDesc), vp, C.POINTER(vp)]),
        "fo_mesh_destroy": (None, [vp]),
        "fo_mesh_info": (C.c_int, [vp, i64p, i64p, i64p, i64p]),
        "fo_jacobian_pattern": (C.c_int, [vp, vp, vp, vp]),
        "fo_assemble_residual": (C.c_int, [vp, vp, vp, vp]),
        "fo_assemble_jacobian": (C.c_int, [vp, vp, vp, vp, i32, i32, vp]),
        "fo_initial_guess_sia": (C.c_int, [vp, vp, vp]),
        "fo_profile_enable": (C.c_int, [vp, i32]),
        "fo_profile_read": (C.c_int, [vp, C.POINTER(C.c_double), i64p]),
        "fo_newton_default_opts": (None, [C.POINTER(NewtonOpts)]),
        "fo_newton_workspace_bytes": (C.c_size_t, [vp, C.POINTER(NewtonOpts)]),
        "fo_newton_solve": (C.c_int, [vp, vp, C.POINTER(NewtonOpts), C.POINTER(NewtonReport), vp,
                                      C.c_size_t, vp]),
        "fo_ensemble_create": (C.c_int, [C.POINTER(vp), i32, vp, C.POINTER(vp)]),
        "fo_ensemble_destroy": (None, [vp]),
        "fo_ensemble_assemble": (C.c_int, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), i32, i32, vp]),
        "fo_mlp_param_count": (C.c_int32, []),
        "fo_column_features": (C.c_int, [vp, vp, vp, vp]),
        "fo_mlp_forward": (C.c_int, [vp, vp, i32, vp, vp, vp]),
        "fo_mlp_backward": (C.c_int, [vp, vp, i32, vp, vp, vp, vp, vp]),
        "fo_mse_grad": (C.c_int, [vp, vp, C.c_int64, vp, vp, vp]),
        "fo_adam_step": (C.c_int, [vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float, C.c_float, i32, vp]),
        "fo_learned_workspace_bytes": (C.c_size_t, [vp]),
        "fo_initial_guess_learned": (C.c_int, [vp, vp, vp, vp, i32, i32, vp, C.c_size_t, C.POINTER(C.c_int32), vp]),
        "fo_initial_guess_learned_noalloc": (C.c_int, [vp, vp, vp, vp, i32, i32, C.POINTER(C.c_int32), vp]),
        "fo_learned_targets": (C.c_int, [vp, vp, vp, vp, vp]),
        "fo_feature_stats": (C.c_int, [vp, C.c_int64, vp, vp, vp]),
        "fo_mdsc_aggregate_graph": (C.c_int, [i32, vp, vp, vp, C.POINTER(C.c_int32)]),
        "fo_mdsc_create": (C.c_int, [vp, vp, C.POINTER(vp)]),
        "fo_mdsc_destroy": (None, [vp]),
        "fo_mdsc_levels": (C.c_int, [vp, C.POINTER(C.c_int32), vp]),
        "fo_mdsc_graph": (C.c_int, [vp, i32, vp, vp, vp]),
        "fo_mdsc_setup": (C.c_int, [vp, vp, i32, vp]),
        "fo_mdsc_apply": (C.c_int, [vp, vp, vp, vp]),
        "fo_mdsc_export": (C.c_int, [vp, i32, i32, vp, C.c_size_t, vp]),
        "fo_status_string": (C.c_char_p, [C.c_int]),
        "fo_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2204_04321_amd.build`")
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def check(status: int):
    if status != FO_OK:
        L = lib()
        raise FoError(status, L.fo_last_error().decode() or L.fo_status_string(status).decode())
