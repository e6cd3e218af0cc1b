"""ctypes view of libvpp.so (include/vpp.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# VPP_DEBUG_BOUNDS=1 in the environment selects the bounds-checked build of
# the same sources (libvpp_debug.so; see vpp_debug_bounds_violations).
LIB_PATH = os.path.join(HERE, "libvpp_debug.so" if os.environ.get("VPP_DEBUG_BOUNDS") == "1" else "libvpp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vpp.h")

VPP_OK = 0
STATUS_NAMES = {0: "VPP_OK", 1: "VPP_ERR_INVALID_ARG", 2: "VPP_ERR_UNSUPPORTED", 3: "VPP_ERR_OUT_OF_MEMORY",
                4: "VPP_ERR_HIP", 5: "VPP_ERR_NOT_CONVERGED", 6: "VPP_ERR_BREAKDOWN", 7: "VPP_ERR_STATE"}
VPP_FP64, VPP_FP32, VPP_MIXED = 0, 1, 2


class Desc(C.Structure):
    _fields_ = [("ncells", C.c_int32 * 3), ("origin", C.c_double * 3), ("extent", C.c_double * 3),
                ("degree", C.c_int32), ("bc", C.c_int32 * 6), ("rho_l", C.c_double), ("rho_g", C.c_double),
                ("heaviside", C.c_int32), ("device", C.c_int32)]


class CgOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("inner_rtol", C.c_double), ("inner_max_iter", C.c_int32),
                ("check_every", C.c_int32), ("deflate", C.c_int32), ("deflate_history", C.c_int32)]


class CgInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("outer_iterations", C.c_int32), ("status", C.c_int32),
                ("rel_residual", C.c_double), ("true_rel_residual", C.c_double),
                ("deflation_corrections", C.c_int32), ("deflation_first_change", C.c_double)]


class KernelConfig(C.Structure):
    _fields_ = [("tile", C.c_int32 * 3), ("variant", C.c_int32)]


class ReinitOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("dtau", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
                ("max_iter", C.c_int32)]


class CpOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("phi_lim", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("normal_steps", C.c_int32)]


_lib = None
vp = C.c_void_p
PP = C.POINTER(C.c_void_p)


def load() -> C.CDLL:
    """Load libvpp.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    sig = {
        "vpp_create": (C.c_int, [C.POINTER(Desc), PP]),
        "vpp_destroy": (C.c_int, [vp]),
        "vpp_num_dofs": (C.c_int64, [vp]),
        "vpp_num_qpoints": (C.c_int64, [vp]),
        "vpp_set_phi": (C.c_int, [vp, vp, vp]),
        "vpp_set_mass": (C.c_int, [vp, C.c_double, vp]),
        "vpp_closest_points": (C.c_int, [vp, vp, C.c_int64, C.POINTER(CpOpts), vp, vp, vp]),
        "vpp_closest_points_normal": (C.c_int, [vp, vp, C.c_int64, vp, vp, vp, C.POINTER(CpOpts), vp, vp, vp]),
        "vpp_extend": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "vpp_normal_rhs": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "vpp_reinit_step": (C.c_int, [vp, vp, vp, vp, vp, C.POINTER(ReinitOpts), vp, C.POINTER(CgInfo), vp]),
        "vpp_curvature_rhs": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "vpp_reinit_apply": (C.c_int, [vp, vp, vp, vp, C.POINTER(ReinitOpts), vp, vp, vp]),
        "vpp_reinit_diagonal": (C.c_int, [vp, vp, vp, vp, C.POINTER(ReinitOpts), vp, vp]),
        "vpp_reinit_rhs": (C.c_int, [vp, vp, vp, vp, vp, C.POINTER(ReinitOpts), vp, vp]),
        "vpp_apply": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
        "vpp_apply_noalloc": (C.c_int, [C.POINTER(Desc), vp, vp, vp, vp]),
        "vpp_diagonal": (C.c_int, [vp, vp, vp]),
        "vpp_cg_solve": (C.c_int, [vp, vp, vp, C.POINTER(CgOpts), C.POINTER(CgInfo), vp]),
        "vpp_grad_coef": (C.c_int, [vp, vp, vp, vp, vp]),
        "vpp_grad_phi": (C.c_int, [vp, vp, vp, vp]),
        "vpp_get_config": (C.c_int, [vp, C.POINTER(KernelConfig)]),
        "vpp_set_config": (C.c_int, [vp, C.POINTER(KernelConfig)]),
        "vpp_get_config_for": (C.c_int, [vp, C.c_int32, C.POINTER(KernelConfig)]),
        "vpp_set_config_for": (C.c_int, [vp, C.c_int32, C.POINTER(KernelConfig)]),
        "vpp_tune": (C.c_int, [vp, C.c_char_p, vp]),
        "vpp_config_candidates": (C.c_int32, [C.c_int32, C.POINTER(KernelConfig), C.c_int32]),
        "vpp_batch_create": (C.c_int, [PP, C.POINTER(C.c_int32), C.c_int32, C.c_char_p, PP]),
        "vpp_batch_apply": (C.c_int, [vp, PP, PP, vp]),
        "vpp_batch_cg_solve": (C.c_int, [vp, PP, PP, C.POINTER(CgOpts), C.POINTER(CgInfo), vp]),
        "vpp_batch_get_config": (C.c_int, [vp, C.POINTER(KernelConfig)]),
        "vpp_batch_destroy": (C.c_int, [vp]),
        "vpp_amr_create": (C.c_int, [C.POINTER(Desc), C.c_void_p, PP]),
        "vpp_amr_destroy": (C.c_int, [vp]),
        "vpp_amr_num_dofs": (C.c_int64, [vp]),
        "vpp_amr_num_free": (C.c_int64, [vp]),
        "vpp_amr_set_phi": (C.c_int, [vp, vp, vp]),
        "vpp_amr_apply": (C.c_int, [vp, vp, vp, vp]),
        "vpp_amr_diagonal": (C.c_int, [vp, vp, vp]),
        "vpp_amr_cg_solve": (C.c_int, [vp, vp, vp, C.POINTER(CgOpts), C.POINTER(CgInfo), vp]),
        "vpp_last_error": (C.c_char_p, []),
        "vpp_abi_version": (C.c_int32, []),
        "vpp_debug_bounds_violations": (C.c_int64, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def declared_functions() -> list:
    """Names of the functions include/vpp.h declares."""
    import re
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vpp_[a-z_0-9]+)\s*\(", text)))
