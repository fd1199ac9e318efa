"""ctypes binding of libinrct.so (argument marshalling only).

Every compute call goes to the HIP library; there is no fallback.  If the
library has not been built, loading raises immediately.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinrct.so")

INRCT_OK = 0
INRCT_EINVAL, INRCT_ENOTSUP, INRCT_EHIP, INRCT_ENOMEM = -1, -2, -3, -4
INRCT_PAR2D, INRCT_CONE3D, INRCT_FAN2D = 1, 2, 3
INRCT_FFN, INRCT_SIREN, INRCT_HASH = 1, 2, 3
INRCT_FP32, INRCT_BF16 = 0, 1
INRCT_LS, INRCT_FLS = 0, 1
INRCT_V_FULL, INRCT_V_AT_I = 0, 1
INRCT_WS_GEOM, INRCT_WS_MODEL, INRCT_WS_CTX = 1, 2, 3
INRCT_ADJ_2D, INRCT_ADJ_DIRECT, INRCT_ADJ_WALK, INRCT_ADJ_WALK2 = 0, 1, 2, 3

c_void_p = ctypes.c_void_p
c_int = ctypes.c_int
c_i64 = ctypes.c_int64
c_u64 = ctypes.c_uint64
c_double = ctypes.c_double
c_float = ctypes.c_float


class InrGrid(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int)]


class CtGeometry(ctypes.Structure):
    _fields_ = [("kind", c_int), ("n_views", c_int), ("n_u", c_int), ("n_v", c_int),
                ("du", c_double), ("dv", c_double), ("sid", c_double), ("idd", c_double),
                ("angles", ctypes.POINTER(c_double))]


class InrArch(ctypes.Structure):
    _fields_ = [("kind", c_int), ("in_dim", c_int), ("n_freq", c_int), ("width", c_int),
                ("depth", c_int), ("omega0", c_float), ("mlp_dtype", c_int),
                ("hash_levels", c_int), ("hash_log2_size", c_int), ("hash_base_res", c_int),
                ("hash_max_res", c_int)]


class StepCfg(ctypes.Structure):
    _fields_ = [("loss", c_int), ("k", c_i64), ("seed", c_u64), ("lr", c_double),
                ("beta1", c_double), ("beta2", c_double), ("eps", c_double),
                ("v_mode", c_int)]


class InrctError(RuntimeError):
    pass


_lib = None


def _proto(lib, name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args


def load():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise InrctError(
            "libinrct.so not found at %s: build it with "
            "`python -m paper_2604_09884_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    _proto(lib, "inrct_last_error", ctypes.c_char_p, [])
    _proto(lib, "inrct_workspace_bytes", c_i64,
           [c_int, ctypes.POINTER(InrArch), ctypes.POINTER(CtGeometry), ctypes.POINTER(InrGrid),
            c_i64, ctypes.POINTER(StepCfg)])
    _proto(lib, "inrct_geom_create", c_int,
           [ctypes.POINTER(CtGeometry), ctypes.POINTER(InrGrid), P, ctypes.c_size_t, P,
            ctypes.POINTER(P)])
    _proto(lib, "inrct_geom_destroy", c_int, [P])
    _proto(lib, "inrct_geom_n_rays", c_i64, [P])
    _proto(lib, "inrct_geom_adjoint_kind", c_int, [P])
    _proto(lib, "ct_project", c_int, [P, P, P, P])
    _proto(lib, "ct_backproject", c_int, [P, P, P, P])
    _proto(lib, "ct_backproject_at", c_int, [P, P, P, c_i64, P, P])
    _proto(lib, "inrct_residual_loss", c_int, [P, c_int, P, P, P, P, P])
    _proto(lib, "inrct_model_create", c_int,
           [ctypes.POINTER(InrArch), ctypes.POINTER(InrGrid), c_i64, P, ctypes.c_size_t, P,
            ctypes.POINTER(P)])
    _proto(lib, "inrct_model_destroy", c_int, [P])
    _proto(lib, "inrct_model_n_params", c_i64, [P])
    _proto(lib, "inrct_model_n_fov", c_i64, [P])
    _proto(lib, "inr_eval_grid", c_int, [P, P, P, P, P])
    _proto(lib, "inr_eval_points", c_int, [P, P, P, P, c_i64, P, P])
    _proto(lib, "inr_vjp_subsampled", c_int,
           [P, P, P, P, c_i64, P, c_int, c_double, P, P])
    _proto(lib, "inrct_sample", c_int, [P, c_u64, c_u64, c_i64, P, P])
    _proto(lib, "inrct_adam", c_int,
           [P, P, P, P, P, c_i64, c_double, c_double, c_double, c_double, P, P])
    _proto(lib, "inrct_adam_noalloc", c_int,
           [P, P, P, P, c_i64, c_i64, c_double, c_double, c_double, c_double, P, P])
    _proto(lib, "inr_ctx_create", c_int,
           [P, P, ctypes.POINTER(StepCfg), P, P, P, P, P, P, ctypes.c_size_t, P,
            ctypes.POINTER(P)])
    _proto(lib, "inr_ctx_destroy", c_int, [P])
    _proto(lib, "inr_grad_step", c_int, [P, c_u64, P, P, P])
    _proto(lib, "inr_grad_step_views", c_int, [P, c_u64, P, P, P, P, P])
    _proto(lib, "inr_ctx_buffer", c_void_p, [P, c_int])
    _proto(lib, "inr_ctx_enable_timing", c_int, [P, c_int])
    _proto(lib, "inr_ctx_stage_ms", c_int, [P, c_int, ctypes.POINTER(c_double)])
    _lib = lib
    return lib


def check(status):
    if status != INRCT_OK:
        msg = load().inrct_last_error().decode(errors="replace")
        raise InrctError("libinrct status %d: %s" % (status, msg))


EXPORTED = [
    "inrct_last_error", "inrct_workspace_bytes", "inrct_geom_create", "inrct_geom_destroy", "inrct_geom_n_rays", "inrct_geom_adjoint_kind",
    "ct_project", "ct_backproject", "ct_backproject_at", "inrct_residual_loss",
    "inrct_model_create", "inrct_model_destroy", "inrct_model_n_params",
    "inrct_model_n_fov", "inr_eval_grid", "inr_eval_points", "inr_vjp_subsampled",
    "inrct_sample", "inrct_adam", "inrct_adam_noalloc", "inr_ctx_create", "inr_ctx_destroy", "inr_grad_step",
    "inr_grad_step_views", "inr_ctx_buffer", "inr_ctx_enable_timing", "inr_ctx_stage_ms",
]
