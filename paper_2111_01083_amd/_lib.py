"""ctypes declarations of the libpfmm C ABI (include/pfmm.h).

The binding only marshals arguments; every step of an evaluation runs in
the HIP library. It refuses to work without the built library.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpfmm.so")

PFMM_LAPLACE, PFMM_YUKAWA, PFMM_STOKES = 0, 1, 2
PFMM_FP64, PFMM_MIXED = 0, 1
PFMM_FAR_AUTO, PFMM_FAR_DIRECT, PFMM_FAR_NUFFT = 0, 1, 2
PFMM_NEAR_AUTO, PFMM_NEAR_ONE_SIDED, PFMM_NEAR_MUTUAL, PFMM_NEAR_NONE, PFMM_NEAR_FMM = 0, 1, 2, 3, 4
PFMM_MAX_POINTS = 1 << 30          # largest n_src / n_trg (per cell in a batch)
PFMM_STATIC_WORKSPACE_BYTES = 64 << 20   # the fixed device workspace of pfmm_eval_static
ERRORS = {0: "PFMM_OK", -1: "PFMM_EINVAL", -2: "PFMM_EINVAL_LATTICE", -3: "PFMM_EINVAL_TOL",
          -4: "PFMM_EWORKSPACE", -5: "PFMM_EHIP", -6: "PFMM_ENOT_NEUTRAL", -7: "PFMM_ENOMEM"}

# every function declared in include/pfmm.h
EXPORTS = ["pfmm_plan", "pfmm_plan_upload", "pfmm_plan_get_info", "pfmm_plan_get_quadrature",
           "pfmm_plan_get_log_groups", "pfmm_plan_get_spread_kernel",
           "pfmm_plan_stage_times", "pfmm_plan_fmm_stage_times", "pfmm_fmm_tree",
           "pfmm_workspace_bytes", "pfmm_eval", "pfmm_eval_static", "pfmm_workspace_bytes_adjoint", "pfmm_eval_adjoint",
           "pfmm_workspace_bytes_pressure", "pfmm_eval_pressure",
           "pfmm_batch_create", "pfmm_batch_workspace_bytes", "pfmm_eval_batch", "pfmm_batch_destroy",
           "pfmm_plan_get_tuning", "pfmm_plan_set_tuning", "pfmm_autotune", "pfmm_batch_autotune",
           "pfmm_destroy", "pfmm_strerror"]


class pfmm_opts(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("precision", ctypes.c_int), ("far_mode", ctypes.c_int),
                ("m0", ctypes.c_int), ("n_dens", ctypes.c_int), ("self_exclude", ctypes.c_int),
                ("m_gl", ctypes.c_int), ("check_neutral", ctypes.c_int), ("profile", ctypes.c_int),
                ("near_mode", ctypes.c_int), ("periodic", ctypes.c_int), ("ew_rule", ctypes.c_int)]


class pfmm_plan_info_t(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("precision", ctypes.c_int), ("far_mode_used", ctypes.c_int),
                ("m0", ctypes.c_int), ("n_dens", ctypes.c_int), ("self_exclude", ctypes.c_int),
                ("d", ctypes.c_double), ("xi", ctypes.c_double), ("eta", ctypes.c_double),
                ("rot_cos", ctypes.c_double), ("rot_sin", ctypes.c_double), ("eps", ctypes.c_double),
                ("n_modes", ctypes.c_int), ("n_quad", ctypes.c_int), ("m_gl", ctypes.c_int),
                ("nufft_nf", ctypes.c_int), ("nufft_w", ctypes.c_int), ("n_images", ctypes.c_int),
                ("n_log_groups", ctypes.c_int), ("periodic", ctypes.c_int), ("ew_rotated", ctypes.c_int),
                ("ew_cos", ctypes.c_double),
                ("ew_sin", ctypes.c_double), ("fmm_order", ctypes.c_int), ("fmm_symmetric", ctypes.c_int)]


class pfmm_tuning_t(ctypes.Structure):
    _fields_ = [("near_blocks", ctypes.c_int64), ("nufft_grid", ctypes.c_int), ("fmm_level", ctypes.c_int),
                ("fmm_leaves", ctypes.c_int)]


class pfmm_tune_report_t(ctypes.Structure):
    _fields_ = [("n_tried", ctypes.c_int), ("default_ms", ctypes.c_double), ("best_ms", ctypes.c_double)]


_lib = None


def load():
    """Load libpfmm.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libpfmm.so not found at {LIB_PATH}; build it with "
                           "`python -m paper_2111_01083_amd.build` (there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dp, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    lib.pfmm_plan.argtypes = [c_int, dp, dp, ctypes.c_double, ctypes.POINTER(pfmm_opts), ctypes.POINTER(vp)]
    lib.pfmm_plan.restype = c_int
    lib.pfmm_plan_upload.argtypes = [vp]
    lib.pfmm_plan_upload.restype = c_int
    lib.pfmm_plan_get_info.argtypes = [vp, ctypes.POINTER(pfmm_plan_info_t)]
    lib.pfmm_plan_get_info.restype = c_int
    lib.pfmm_plan_get_quadrature.argtypes = [vp, dp, dp]
    lib.pfmm_plan_get_quadrature.restype = c_int
    lib.pfmm_plan_get_log_groups.argtypes = [vp, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    lib.pfmm_plan_get_log_groups.restype = c_int
    lib.pfmm_plan_get_spread_kernel.argtypes = [vp, dp, ctypes.POINTER(c_int), dp]
    lib.pfmm_plan_get_spread_kernel.restype = c_int
    lib.pfmm_plan_stage_times.argtypes = [vp, dp, dp, ctypes.POINTER(c_int)]
    lib.pfmm_plan_stage_times.restype = c_int
    lib.pfmm_plan_fmm_stage_times.argtypes = [vp, dp, ctypes.POINTER(c_int)]
    lib.pfmm_plan_fmm_stage_times.restype = c_int
    lib.pfmm_fmm_tree.argtypes = [vp, i64, i64, ctypes.POINTER(c_int)]
    lib.pfmm_fmm_tree.restype = c_int
    lib.pfmm_workspace_bytes.argtypes = [vp, i64, i64]
    lib.pfmm_workspace_bytes.restype = ctypes.c_size_t
    lib.pfmm_eval.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.pfmm_eval.restype = c_int
    lib.pfmm_eval_static.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp]
    lib.pfmm_eval_static.restype = c_int
    lib.pfmm_workspace_bytes_adjoint.argtypes = [vp, i64]
    lib.pfmm_workspace_bytes_adjoint.restype = ctypes.c_size_t
    lib.pfmm_eval_adjoint.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.pfmm_eval_adjoint.restype = c_int
    lib.pfmm_workspace_bytes_pressure.argtypes = [vp, i64, i64]
    lib.pfmm_workspace_bytes_pressure.restype = ctypes.c_size_t
    lib.pfmm_eval_pressure.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, ctypes.c_size_t, vp]
    lib.pfmm_eval_pressure.restype = c_int
    lib.pfmm_batch_create.argtypes = [c_int, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                      c_int, ctypes.POINTER(vp)]
    lib.pfmm_batch_create.restype = c_int
    lib.pfmm_batch_workspace_bytes.argtypes = [vp]
    lib.pfmm_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.pfmm_eval_batch.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.pfmm_eval_batch.restype = c_int
    lib.pfmm_batch_destroy.argtypes = [vp]
    lib.pfmm_batch_destroy.restype = None
    lib.pfmm_plan_get_tuning.argtypes = [vp, ctypes.POINTER(pfmm_tuning_t)]
    lib.pfmm_plan_get_tuning.restype = c_int
    lib.pfmm_plan_set_tuning.argtypes = [vp, ctypes.POINTER(pfmm_tuning_t)]
    lib.pfmm_plan_set_tuning.restype = c_int
    lib.pfmm_autotune.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, ctypes.c_size_t, vp,
                                  ctypes.POINTER(pfmm_tune_report_t)]
    lib.pfmm_autotune.restype = c_int
    lib.pfmm_batch_autotune.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp,
                                        ctypes.POINTER(pfmm_tune_report_t)]
    lib.pfmm_batch_autotune.restype = c_int
    lib.pfmm_destroy.argtypes = [vp]
    lib.pfmm_destroy.restype = None
    lib.pfmm_strerror.argtypes = [c_int]
    lib.pfmm_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib
