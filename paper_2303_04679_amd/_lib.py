"""ctypes binding of libmodil (include/modil.h): structs, constants, signatures.

Argument marshalling only.  Loading fails loudly when the shared library has
not been built; there is no fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmodil.so")

# ---- constants (mirror include/modil.h) ---------------------------------
OK, ERR_INVALID_ARG, ERR_SHAPE, ERR_DTYPE, ERR_HIP, ERR_NONFINITE, ERR_STATE = 0, -1, -2, -3, -4, -5, -6
F32, F64 = 0, 1
CELL, NODE = 0, 1
OP_POISSON, OP_BURGERS, OP_HEAT_KX, OP_NS3D, OP_CAVITY = 0, 1, 2, 3, 4
FLAG_CHI_FIXED = 1
FLAG_FUSED_RESTRICT = 2
TERM_PDE, TERM_DATA, TERM_REG, TERM_IC, TERM_BC = 0, 1, 2, 3, 4
N_TERMS = 5
FIELD_FORCING0, FIELD_CHI = 0, 4
SCALAR_RE = 0
OPT_FUSED = 0
OPT_MARCH = 1
OPT_MARCH_TILE = 2
OPT_TAIL = 3
OPT_TILE = 4
OPT_TWO_PASS = 5
MAX_LEVELS, MAX_FIELDS = 8, 5
TERM_NAMES = ("pde", "data", "reg", "ic", "bc")


class Problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("dims", ctypes.c_int32 * 3),
        ("lengths", ctypes.c_double * 3),
        ("n_levels", ctypes.c_int32),
        ("centering", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("op", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("max_meas", ctypes.c_int32),
        ("re", ctypes.c_double),
        ("diam", ctypes.c_double),
        ("lambda_", ctypes.c_double),
        ("chi_shift", ctypes.c_double),
        ("tau_coef", ctypes.c_double),
        ("u_ref", ctypes.c_double),
        ("w_pde", ctypes.c_double),
        ("w_reg", ctypes.c_double),
        ("w_bc", ctypes.c_double),
    ]


class PackLayout(ctypes.Structure):
    _fields_ = [
        ("n_fields", ctypes.c_int32),
        ("n_levels", ctypes.c_int32),
        ("total", ctypes.c_int64),
        ("level_offset", ctypes.c_int64 * MAX_LEVELS),
        ("level_stride", ctypes.c_int64 * MAX_LEVELS),
        ("field_offset", (ctypes.c_int64 * MAX_FIELDS) * MAX_LEVELS),
        ("field_dims", ((ctypes.c_int32 * 3) * MAX_FIELDS) * MAX_LEVELS),
        ("fine_total", ctypes.c_int64),
        ("fine_cells", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class AdamHP(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double)]


class CnnDesc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("size", ctypes.c_int32), ("n_obs", ctypes.c_int32),
                ("width1", ctypes.c_int32), ("width2", ctypes.c_int32), ("width3", ctypes.c_int32),
                ("out_ch", ctypes.c_int32), ("re_center", ctypes.c_double),
                ("re_scale", ctypes.c_double)]


class CnnLayout(ctypes.Structure):
    _fields_ = [("n_params", ctypes.c_int64), ("w_offset", ctypes.c_int64 * 6),
                ("b_offset", ctypes.c_int64 * 6), ("img_size", ctypes.c_int64),
                ("act_size", ctypes.c_int64), ("out_size", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_size_t)]


class LbfgsParams(ctypes.Structure):
    _fields_ = [("history", ctypes.c_int32), ("max_evals", ctypes.c_int32),
                ("c1", ctypes.c_double), ("c2", ctypes.c_double)]


class LbfgsInfo(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_double), ("grad_norm", ctypes.c_double), ("step", ctypes.c_double),
                ("evals", ctypes.c_int32), ("status", ctypes.c_int32), ("pairs", ctypes.c_int32),
                ("iteration", ctypes.c_int32)]


LBFGS_MAX_HISTORY = 64

_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "modil_abi_version": (_I, []),
    "modil_status_str": (ctypes.c_char_p, [_I]),
    "modil_last_error": (ctypes.c_char_p, [_P]),
    "modil_layout": (_I, [ctypes.POINTER(Problem), ctypes.POINTER(PackLayout)]),
    "modil_create": (_I, [ctypes.POINTER(Problem), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "modil_destroy": (_I, [_P]),
    "modil_set_stream": (_I, [_P, _P]),
    "modil_set_measurements": (_I, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    _P, _P, ctypes.c_double]),
    "modil_clear_measurements": (_I, [_P]),
    "modil_set_field": (_I, [_P, ctypes.c_int32, _P]),
    "modil_set_instance_scalar": (_I, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double]),
    "modil_prolong": (_I, [_P, _P, _P]),
    "modil_restrict_adjoint": (_I, [_P, _P, _P]),
    "modil_prolong_noalloc": (_I, [ctypes.POINTER(Problem), _P, _P, _P]),
    "modil_loss": (_I, [_P, _P, _P]),
    "modil_loss_grad": (_I, [_P, _P, _P, _P]),
    "modil_adam": (_I, [_P, _P, _P, _P, _P, _P, ctypes.POINTER(AdamHP), ctypes.c_int64]),
    "modil_step": (_I, [_P, _P, _P, _P, _P, ctypes.POINTER(AdamHP), ctypes.c_int64, _P]),
    "modil_run": (_I, [_P, _P, _P, _P, _P, ctypes.POINTER(AdamHP), ctypes.c_int64, ctypes.c_int32,
                       _P]),
    "modil_residual_metric": (_I, [_P, _P, _P]),
    "modil_check": (_I, [_P]),
    "modil_set_option": (_I, [_P, ctypes.c_int32, ctypes.c_int64]),
    "modil_fused_active": (_I, [_P]),
    "modil_profile": (_I, [_P, ctypes.c_int32]),
    "modil_profile_read": (_I, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_int64)]),
    "modil_cnn_layout": (_I, [ctypes.POINTER(CnnDesc), ctypes.POINTER(CnnLayout)]),
    "modil_cnn_create": (_I, [ctypes.POINTER(CnnDesc), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "modil_cnn_destroy": (_I, [_P]),
    "modil_cnn_rasterize": (_I, [_P, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "modil_cnn_forward": (_I, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "modil_cnn_loss_backward": (_I, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P]),
    "modil_cnn_adam": (_I, [_P, _P, _P, _P, _P, _P, ctypes.POINTER(AdamHP), ctypes.c_int64]),
    "modil_cnn_to_bf16": (_I, [_P, _P, _P]),
    "modil_lbfgs_workspace": (_I, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "modil_lbfgs_create": (_I, [_P, ctypes.POINTER(LbfgsParams), _P, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "modil_lbfgs_destroy": (_I, [_P]),
    "modil_lbfgs_reset": (_I, [_P]),
    "modil_lbfgs_step": (_I, [_P, _P, ctypes.POINTER(LbfgsInfo)]),
}

_lib = None


class ModilError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"modil error {status}: {message}")
        self.status = status


def lib():
    """The loaded libmodil (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2303_04679_amd.build_lib`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status, ctx=None):
    if status != OK:
        msg = lib().modil_last_error(ctx)
        raise ModilError(status, msg.decode() if msg else "")
    return status
