"""ctypes loader of ``lib/libnfft_mi355x.so`` with the signatures of ``include/nfft_mi355x.h``.

Argument marshalling only: every step of the transforms runs in the HIP library.  If the
library has not been built, loading raises instead of falling back to anything else.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libnfft_mi355x.so")

NFFT_C64 = 1
NFFT_C128 = 2
NFFT_SORT_NODES = 1 << 0
NFFT_KEEP_GRID = 1 << 1
NFFT_DETERMINISTIC = 1 << 5  # always on: results are bitwise reproducible
NFFT_PRE_LIN_PSI = 1 << 6  # window factors from lookup tables (Table 3.2, PRE_LIN_PSI)
NFFT_WINDOW_GAUSSIAN = 1 << 2
NFFT_WINDOW_BSPLINE = 1 << 3
NFFT_WINDOW_SINC = 1 << 4
WINDOW_FLAGS = {"kaiser-bessel": 0, "gaussian": NFFT_WINDOW_GAUSSIAN, "bspline": NFFT_WINDOW_BSPLINE,
                "sinc": NFFT_WINDOW_SINC}

STATUS = {
    0: "NFFT_OK",
    -1: "NFFT_ERR_ARG",
    -2: "NFFT_ERR_STATE",
    -3: "NFFT_ERR_WORKSPACE",
    -4: "NFFT_ERR_HIP",
    -5: "NFFT_ERR_UNSUPPORTED",
}

# every exported entry point of include/nfft_mi355x.h
ABI_SYMBOLS = [
    "nfft_plan_create", "nfft_plan_create_params", "nfft_plan_tune", "nfft_plan_destroy", "nfft_plan_get_info",
    "nfft_workspace_bytes", "nfft_set_workspace", "nfft_set_nodes", "nfft_nodes_finite", "nfft_trafo", "nfft_adjoint", "nfft_fastsum", "ndft_trafo",
    "ndft_adjoint", "nfft_grad_x", "nfft_step_grid", "nfft_step_interp", "nfft_step_spread",
    "nfft_step_coeffs", "nfft_profile_enable", "nfft_profile_read", "nfft_batch_create",
    "nfft_batch_get_info", "nfft_batch_workspace_bytes", "nfft_batch_set_workspace",
    "nfft_batch_autotune", "nfft_batch_get_params", "nfft_batch_set_params", "nfft_batch_trafo", "nfft_batch_trafo_noalloc", "nfft_batch_adjoint", "nfft_batch_destroy", "nfft_status_string",
    "nnfft_plan_create", "nnfft_plan_destroy", "nnfft_plan_get_info", "nnfft_workspace_bytes",
    "nnfft_set_workspace", "nnfft_set_nodes", "nnfft_trafo", "nnfft_adjoint",
]


class NfftError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (what, STATUS.get(status, "?"), status))


class PlanParams(ctypes.Structure):
    """nfft_plan_params: bin edges per dimension and the work-item cap (0: defaults)."""
    _fields_ = [("bin", ctypes.c_int32 * 3), ("chunk_cap", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int),
        ("m", ctypes.c_int),
        ("dtype", ctypes.c_int),
        ("flags", ctypes.c_uint32),
        ("N", ctypes.c_int64 * 3),
        ("n", ctypes.c_int64 * 3),
        ("M", ctypes.c_int64),
        ("bin", ctypes.c_int64 * 3),
        ("nbins", ctypes.c_int64),
        ("chunk_cap", ctypes.c_int64),
        ("max_chunks", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_size_t),
        ("lds_bytes", ctypes.c_size_t),
        ("grid_scale", ctypes.c_double),
        ("window", ctypes.c_int),
        ("own_tiles", ctypes.c_int),
        ("own_tile", ctypes.c_int64 * 3),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int),
        ("groups", ctypes.c_int),
        ("tuned", ctypes.c_int),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class NNPlanInfo(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int),
        ("m", ctypes.c_int),
        ("N", ctypes.c_int64 * 3),
        ("K", ctypes.c_int64),
        ("M", ctypes.c_int64),
        ("N2", ctypes.c_int64 * 3),
        ("NA", ctypes.c_int64 * 3),
        ("sigma1", ctypes.c_double * 3),
        ("workspace_bytes", ctypes.c_size_t),
        ("window", ctypes.c_int),
    ]


NFFT_BATCH_NPARAMS = 8
BATCH_PARAM_NAMES = ("pack_fwd", "k_fwd", "pack_adj", "k_adj", "k_interp", "k_spread", "k_fold", "reserved")

_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "the HIP library %s is missing: build it with paper_1810_09891_amd.build.build() "
            "(there is no fallback path)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    I64 = ctypes.c_int64
    sig = {
        "nfft_plan_create": [ctypes.POINTER(P), I, ctypes.POINTER(I64), I64, ctypes.POINTER(I64), I, I,
                             ctypes.c_uint32],
        "nfft_plan_create_params": [ctypes.POINTER(P), I, ctypes.POINTER(I64), I64, ctypes.POINTER(I64), I, I,
                                    ctypes.c_uint32, ctypes.POINTER(PlanParams)],
        "nfft_plan_tune": [I, ctypes.POINTER(I64), I64, ctypes.POINTER(I64), I, I, ctypes.c_uint32, P,
                           ctypes.c_char_p, P, ctypes.POINTER(PlanParams), ctypes.POINTER(ctypes.c_double)],
        "nfft_plan_destroy": [P],
        "nfft_plan_get_info": [P, ctypes.POINTER(PlanInfo)],
        "nfft_workspace_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
        "nfft_set_workspace": [P, P, ctypes.c_size_t],
        "nfft_set_nodes": [P, P, P],
        "nfft_nodes_finite": [P, ctypes.POINTER(ctypes.c_int), P],
        "nfft_trafo": [P, P, P, P],
        "nfft_adjoint": [P, P, P, P],
        "nfft_fastsum": [P, P, P, P, P, P, P],
        "ndft_trafo": [P, P, P, P],
        "ndft_adjoint": [P, P, P, P],
        "nfft_grad_x": [P, P, P, P],
        "nfft_step_grid": [P, P, P, P],
        "nfft_step_interp": [P, P, P, P],
        "nfft_step_spread": [P, P, P, P],
        "nfft_step_coeffs": [P, P, P, P],
        "nfft_profile_enable": [P, I],
        "nfft_profile_read": [P, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(I64), I, ctypes.POINTER(I)],
        "nfft_batch_create": [ctypes.POINTER(P), I, ctypes.POINTER(P), ctypes.c_char_p],
        "nfft_batch_get_info": [P, ctypes.POINTER(BatchInfo)],
        "nfft_batch_get_params": [P, I, ctypes.POINTER(I), ctypes.POINTER(I)],
        "nfft_batch_set_params": [P, I, ctypes.POINTER(I)],
        "nfft_batch_workspace_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
        "nfft_batch_set_workspace": [P, P, ctypes.c_size_t],
        "nfft_batch_autotune": [P, P],
        "nfft_batch_trafo": [P, ctypes.POINTER(P), ctypes.POINTER(P), P],
        "nfft_batch_trafo_noalloc": [P, ctypes.POINTER(P), ctypes.POINTER(P), P],
        "nfft_batch_adjoint": [P, ctypes.POINTER(P), ctypes.POINTER(P), P],
        "nfft_batch_destroy": [P],
        "nnfft_plan_create": [ctypes.POINTER(P), I, ctypes.POINTER(I64), I64, I64, ctypes.c_double, I, I,
                              ctypes.c_uint32],
        "nnfft_plan_destroy": [P],
        "nnfft_plan_get_info": [P, ctypes.POINTER(NNPlanInfo)],
        "nnfft_workspace_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
        "nnfft_set_workspace": [P, P, ctypes.c_size_t],
        "nnfft_set_nodes": [P, P, P, P],
        "nnfft_trafo": [P, P, P, P],
        "nnfft_adjoint": [P, P, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = I
    lib.nfft_status_string.argtypes = [I]
    lib.nfft_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status, what):
    if status != 0:
        raise NfftError(status, what)
