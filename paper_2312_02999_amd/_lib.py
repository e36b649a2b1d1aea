"""ctypes binding of libpdipc.so (argument marshalling only).

torch is imported first so that its HIP runtime is the one in the process;
the library's dependency on ``libamdhip64.so.7`` then resolves to that copy
(same soname).  No solver arithmetic happens here, and there is no fallback:
if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime before the library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdipc.so")

PDIPC_OK = 0
ERRORS = {
    -1: "PDIPC_E_INVALID", -2: "PDIPC_E_DEGENERATE", -3: "PDIPC_E_NOT_SPD", -4: "PDIPC_E_NOMEM",
    -5: "PDIPC_E_INTERSECTING", -6: "PDIPC_E_HIP",
}
WARNINGS = {1: "PDIPC_W_LS_FAILED", 2: "PDIPC_W_NOT_CONVERGED"}

EXPORTS = [
    "pdipc_default_options", "pdipc_init_mesh", "pdipc_set_actuation", "pdipc_set_actuation_scalar",
    "pdipc_solve_frame", "pdipc_solve_frame_backward", "pdipc_get_sizes", "pdipc_destroy",
    "pdipc_last_error", "pdipc_debug_local", "pdipc_debug_contacts", "pdipc_debug_step",
    "pdipc_debug_host_factor", "pdipc_kernel_timer", "pdipc_debug_dense", "pdipc_device_bytes",
    "pdipc_debug_trace", "pdipc_dense_spd_noalloc",
]


class MeshDesc(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tets", C.c_int32), ("rest_pos", C.c_void_p),
                ("tets", C.c_void_p), ("dirichlet", C.c_void_p), ("n_surf_tris", C.c_int32),
                ("surf_tris", C.c_void_p), ("region", C.c_void_p), ("youngs", C.c_double),
                ("poisson", C.c_double), ("n_surf_verts", C.c_int32), ("W_rowptr", C.c_void_p),
                ("W_col", C.c_void_p), ("W_val", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("dhat", C.c_double), ("kappa", C.c_double), ("iters", C.c_int32), ("tol", C.c_double),
                ("precision", C.c_int32), ("ccd_eta", C.c_double), ("ccd_steps", C.c_int32),
                ("ls_max_halvings", C.c_int32), ("cinv_updates_max", C.c_int32),
                ("fp32_reduced_min", C.c_int32), ("hinv_rows_mb", C.c_int32), ("stream", C.c_void_p),
                ("global_method", C.c_int32), ("cg_tol", C.c_double), ("cg_max_iters", C.c_int32),
                ("barrier_form", C.c_int32), ("kappa_adapt", C.c_int32)]


class FrameStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("n_pt", C.c_int32), ("n_ee", C.c_int32), ("n_c", C.c_int32),
                ("ls_halvings", C.c_int32), ("ls_failures", C.c_int32), ("refine_steps", C.c_int32),
                ("n_candidates", C.c_int32), ("refine_fallbacks", C.c_int32), ("cinv_rebuilds", C.c_int32),
                ("c_delta_max", C.c_int32), ("c_delta_sum", C.c_int32), ("cinv_updates", C.c_int32),
                ("near_ties", C.c_int32), ("pcg_iters", C.c_int32),
                ("alpha_m_min", C.c_double),
                ("alpha_min", C.c_double),
                ("energy", C.c_double), ("grad_inf", C.c_double), ("ms_ipc", C.c_double),
                ("ms_gstep", C.c_double), ("ms_ccd", C.c_double), ("ms_ls", C.c_double),
                ("ms_misc", C.c_double), ("ms_total", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class IterTrace(C.Structure):
    _fields_ = [("n_pt", C.c_int32), ("n_ee", C.c_int32), ("n_c", C.c_int32), ("n_candidates", C.c_int32),
                ("ls_halvings", C.c_int32), ("ls_ok", C.c_int32), ("near_ties", C.c_int32),
                ("refine_steps", C.c_int32), ("cg_iters", C.c_int32), ("alpha_m", C.c_double), ("alpha", C.c_double),
                ("kappa", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load (once) and return the library; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2312_02999_amd.build.build() first "
                          "(there is no fallback implementation)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
    L.pdipc_default_options.argtypes = [C.POINTER(Options)]
    L.pdipc_default_options.restype = None
    L.pdipc_init_mesh.argtypes = [C.POINTER(MeshDesc), C.POINTER(Options), C.POINTER(vp)]
    L.pdipc_init_mesh.restype = i32
    L.pdipc_set_actuation.argtypes = [vp, dp]
    L.pdipc_set_actuation.restype = i32
    L.pdipc_set_actuation_scalar.argtypes = [vp, dp, dp]
    L.pdipc_set_actuation_scalar.restype = i32
    L.pdipc_solve_frame.argtypes = [vp, dp, dp, C.POINTER(FrameStats)]
    L.pdipc_solve_frame.restype = i32
    L.pdipc_solve_frame_backward.argtypes = [vp, dp, dp]
    L.pdipc_solve_frame_backward.restype = i32
    L.pdipc_get_sizes.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.pdipc_get_sizes.restype = i32
    L.pdipc_destroy.argtypes = [vp]
    L.pdipc_destroy.restype = None
    L.pdipc_dense_spd_noalloc.argtypes = [dp, i64, dp, i32, dp, i32, vp, vp]
    L.pdipc_dense_spd_noalloc.restype = i32
    L.pdipc_last_error.argtypes = [vp]
    L.pdipc_last_error.restype = C.c_char_p
    L.pdipc_debug_local.argtypes = [vp, dp, dp, dp, dp]
    L.pdipc_debug_local.restype = i32
    L.pdipc_debug_contacts.argtypes = [vp, dp, dp, i32, C.POINTER(i32)]
    L.pdipc_debug_contacts.restype = i32
    L.pdipc_debug_step.argtypes = [vp, dp, dp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.pdipc_debug_step.restype = i32
    L.pdipc_debug_host_factor.argtypes = [i32, i32, dp, dp, dp, dp, i32, dp, dp, dp, C.POINTER(i64)]
    L.pdipc_debug_host_factor.restype = i32
    L.pdipc_kernel_timer.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(i64)]
    L.pdipc_kernel_timer.restype = i32
    L.pdipc_debug_dense.argtypes = [dp, i64, dp, i32, dp, i32]
    L.pdipc_debug_dense.restype = i32
    L.pdipc_device_bytes.argtypes = [vp, C.POINTER(i64)]
    L.pdipc_device_bytes.restype = i32
    L.pdipc_debug_trace.argtypes = [vp, C.POINTER(IterTrace), i32, C.POINTER(i32)]
    L.pdipc_debug_trace.restype = i32
    _lib = L
    return L


def hip_runtimes_loaded() -> list[str]:
    """Distinct libamdhip64 files mapped into this process."""
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                paths.add(os.path.realpath(line.split()[-1]))
    return sorted(paths)


class PdipcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def check(code: int, handle=None):
    if code < 0:
        msg = lib().pdipc_last_error(handle)
        raise PdipcError(code, msg.decode() if msg else "")
    return code
