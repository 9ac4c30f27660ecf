"""ctypes declarations of the C ABI in include/maxwell.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmaxwell.so")

MAXWELL_OK = 0
MAXWELL_ERR_INVALID_ARGUMENT = -1
MAXWELL_ERR_UNSUPPORTED = -2
MAXWELL_ERR_OUT_OF_MEMORY = -3
MAXWELL_ERR_HIP = -4
MAXWELL_ERR_WORKSPACE_TOO_SMALL = -5
MAXWELL_STATIC_WS_BYTES = 64 << 20

MAXWELL_BASIS_DENSE = 0
MAXWELL_BASIS_TUCKER = 1
MAXWELL_FP32 = 0
MAXWELL_BF16_SPLIT = 1
MAXWELL_CARTESIAN = 0
MAXWELL_NONCARTESIAN = 1

STATUS_NAMES = {
    0: "MAXWELL_OK", -1: "MAXWELL_ERR_INVALID_ARGUMENT", -2: "MAXWELL_ERR_UNSUPPORTED",
    -3: "MAXWELL_ERR_OUT_OF_MEMORY", -4: "MAXWELL_ERR_HIP", -5: "MAXWELL_ERR_WORKSPACE_TOO_SMALL",
}

# Every entry point declared in include/maxwell.h.
EXPORTS = [
    "maxwell_plan_create", "maxwell_plan_destroy", "maxwell_plan_workspace_size", "maxwell_plan_path",
    "maxwell_basis_apply", "maxwell_basis_apply_adjoint", "maxwell_encode", "maxwell_adjoint",
    "maxwell_forward_loss", "maxwell_forward_transfer", "maxwell_adjoint_transfer", "maxwell_grad",
    "maxwell_last_error", "maxwell_version", "maxwell_batch_create", "maxwell_batch_workspace_size",
    "maxwell_batch_grad", "maxwell_batch_destroy", "maxwell_jvp", "maxwell_normal", "maxwell_cg",
    "maxwell_sense_encode", "maxwell_sense_adjoint", "maxwell_sense_normal", "maxwell_tv_prox",
    "maxwell_ball_project", "maxwell_sense_admm", "maxwell_multi_encode", "maxwell_multi_grad",
    "maxwell_tucker_compress", "maxwell_batch_grad_shared",
    "maxwell_plan_set_timing", "maxwell_plan_timing", "maxwell_bf16_split", "maxwell_grad_static",
    "maxwell_batch_set_options", "maxwell_tune_counts",
]


class BasisDesc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("K", ctypes.c_int64),
        ("dense", ctypes.c_void_p),
        ("r", ctypes.c_int64 * 3),
        ("U", ctypes.c_void_p * 3),
        ("core", ctypes.c_void_p),
    ]


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("J", ctypes.c_int32),
        ("precision", ctypes.c_int),
        ("sampling", ctypes.c_int),
        ("M", ctypes.c_int64),
        ("mask_idx", ctypes.c_void_p),
        ("traj", ctypes.c_void_p),
        ("weights", ctypes.c_void_p),
        ("kb_width", ctypes.c_int32),
        ("oversamp", ctypes.c_float),
        ("kb_beta", ctypes.c_float),
    ]


class MaxwellError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libmaxwell.so; raise if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2008_09042_amd.build`")
    lib = ctypes.CDLL(path)
    vp, sz, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64
    st = ctypes.c_int
    lib.maxwell_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(BasisDesc), ctypes.POINTER(vp)]
    lib.maxwell_plan_create.restype = st
    lib.maxwell_plan_destroy.argtypes = [vp]
    lib.maxwell_plan_destroy.restype = None
    lib.maxwell_plan_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.maxwell_plan_workspace_size.restype = st
    lib.maxwell_plan_path.argtypes = [vp]
    lib.maxwell_plan_path.restype = ctypes.c_char_p
    lib.maxwell_basis_apply.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.maxwell_basis_apply.restype = st
    lib.maxwell_basis_apply_adjoint.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.maxwell_basis_apply_adjoint.restype = st
    lib.maxwell_encode.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.maxwell_encode.restype = st
    lib.maxwell_adjoint.argtypes = [vp, vp, vp, vp, ctypes.c_float, vp, vp, vp, vp, sz, vp]
    lib.maxwell_adjoint.restype = st
    lib.maxwell_forward_loss.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.maxwell_forward_loss.restype = st
    lib.maxwell_forward_transfer.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.maxwell_forward_transfer.restype = st
    lib.maxwell_adjoint_transfer.argtypes = [vp, vp, vp, vp, ctypes.c_float, vp, vp, vp, vp, sz, vp]
    lib.maxwell_adjoint_transfer.restype = st
    lib.maxwell_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(vp)]
    lib.maxwell_batch_create.restype = st
    lib.maxwell_batch_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.maxwell_batch_workspace_size.restype = st
    pa = ctypes.POINTER(vp)
    lib.maxwell_batch_grad.argtypes = [vp, pa, pa, pa, pa, pa, pa, vp, sz, vp]
    lib.maxwell_batch_grad.restype = st
    lib.maxwell_batch_grad_shared.argtypes = [vp, pa, vp, pa, pa, vp, vp, vp, sz, vp]
    lib.maxwell_batch_grad_shared.restype = st
    lib.maxwell_tune_counts.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.maxwell_tune_counts.restype = st
    lib.maxwell_batch_set_options.argtypes = [vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_double)]
    lib.maxwell_batch_set_options.restype = st
    lib.maxwell_batch_destroy.argtypes = [vp]
    lib.maxwell_batch_destroy.restype = None
    lib.maxwell_grad.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.maxwell_grad.restype = st
    lib.maxwell_jvp.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.maxwell_jvp.restype = st
    lib.maxwell_normal.argtypes = [vp, vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, vp, vp, vp, sz, vp]
    lib.maxwell_normal.restype = st
    lib.maxwell_cg.argtypes = [vp, vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_int32, vp, vp, vp,
                               vp, sz, vp]
    lib.maxwell_cg.restype = st
    for f in ("maxwell_sense_encode", "maxwell_sense_adjoint", "maxwell_sense_normal"):
        getattr(lib, f).argtypes = [vp, vp, vp, vp, vp, sz, vp]
        getattr(lib, f).restype = st
    lib.maxwell_tv_prox.argtypes = [vp, vp, ctypes.c_float, ctypes.c_int32, vp, vp, sz, vp]
    lib.maxwell_tv_prox.restype = st
    lib.maxwell_ball_project.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    lib.maxwell_ball_project.restype = st
    lib.maxwell_sense_admm.argtypes = [vp, vp, vp, vp, ctypes.c_float, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, vp, vp, vp, sz, vp]
    lib.maxwell_sense_admm.restype = st
    lib.maxwell_multi_encode.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, sz, vp]
    lib.maxwell_multi_encode.restype = st
    lib.maxwell_multi_grad.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.maxwell_multi_grad.restype = st
    lib.maxwell_tucker_compress.argtypes = [ctypes.POINTER(i64), i64, vp, ctypes.c_float, vp, vp, vp, vp,
                                            ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double), vp]
    lib.maxwell_tucker_compress.restype = st
    lib.maxwell_plan_set_timing.argtypes = [vp, ctypes.c_int]
    lib.maxwell_plan_set_timing.restype = st
    lib.maxwell_plan_timing.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(i64),
                                        ctypes.POINTER(ctypes.c_double)]
    lib.maxwell_plan_timing.restype = st
    lib.maxwell_last_error.argtypes = []
    lib.maxwell_last_error.restype = ctypes.c_char_p
    lib.maxwell_version.argtypes = []
    lib.maxwell_version.restype = ctypes.c_char_p
    lib.maxwell_grad_static.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.maxwell_grad_static.restype = st
    lib.maxwell_bf16_split.argtypes = [vp, i64, ctypes.c_int32, vp, vp, vp]
    lib.maxwell_bf16_split.restype = st
    _lib = lib
    return lib


def check(status: int):
    if status != MAXWELL_OK:
        msg = _lib.maxwell_last_error().decode() if _lib is not None else ""
        raise MaxwellError(status, msg)
