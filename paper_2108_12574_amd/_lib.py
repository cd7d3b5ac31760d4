"""ctypes declarations of libcbd.so (the C ABI in include/cbd.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcbd.so")

GRID_CELL, GRID_NODE = 0, 1
MODE_JACOBI, MODE_SCHWARZ, MODE_CBD = 0, 1, 2
PREC_FP64, PREC_FP32, PREC_BF16GEMM = 0, 1, 2
ROWS_AUTO, ROWS_NEVER, ROWS_ALWAYS = 0, 1, 2
ID_QR, ID_GRAM = 0, 1
OK, EARG, EHIP, ENOTSPD, ENOMEM, EWORKSPACE, EREPLAN, WNOTCONV = 0, -1, -2, -3, -4, -5, -6, 1


class RSOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("n_pxy", ctypes.c_int),
                ("proxy_ratio", ctypes.c_double), ("precision", ctypes.c_int),
                ("exact", ctypes.c_int), ("mlp", ctypes.c_void_p), ("row_compression", ctypes.c_int),
                ("id_sketch", ctypes.c_int), ("sketch_seed", ctypes.c_ulonglong),
                ("workspace_bytes", ctypes.c_size_t), ("apply_rhs", ctypes.c_int), ("id_method", ctypes.c_int),
                ("record", ctypes.c_int)]


# (name, restype, argtypes) of every exported symbol of include/cbd.h
_vp, _ip, _dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
_i, _l, _d, _sz = ctypes.c_int, ctypes.c_long, ctypes.c_double, ctypes.c_size_t
SIGNATURES = [
    ("cbd_last_error", ctypes.c_char_p, []),
    ("ie_assemble", _i, [_i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    ("cbd_problem_free", _i, [_vp]),
    ("dd_partition", _i, [_i, _i, _i, _i, _i, _i, ctypes.POINTER(_vp)]),
    ("cbd_partition_free", _i, [_vp]),
    ("dd_partition_info", _i, [_vp, _ip, _ip, _ip, ctypes.POINTER(_l)]),
    ("dd_subdomain_info", _i, [_vp, _i, _ip, _ip, _ip]),
    ("dd_subdomain_index", _i, [_vp, _i, _ip]),
    ("dd_level_boxes", _i, [_vp, _i, _i, _ip, _ip, _ip]),
    ("rs_factor_rank_count", _i, [_vp, ctypes.POINTER(RSOpts), _ip]),
    ("rs_factor_workspace", _i, [_vp, _vp, ctypes.POINTER(RSOpts), _vp, ctypes.POINTER(_sz)]),
    ("rs_factor_batched", _i, [_vp, _vp, ctypes.POINTER(RSOpts), _vp, _vp, _sz, _vp, ctypes.POINTER(_sz), _vp,
                               ctypes.POINTER(_vp)]),
    ("rs_factor_free", _i, [_vp]),
    ("rs_factor_graph_bytes", _sz, [_vp]),
    ("rs_factor_capture", _i, [_vp, _vp, _sz, _vp]),
    ("rs_factor_replay", _i, [_vp, _vp]),
    ("rs_factor_stats", _i, [_vp, _ip, _ip, ctypes.POINTER(_sz), _dp]),
    ("rs_factor_level", _i, [_vp, _i, _ip, _ip, _ip, _ip]),
    ("rs_factor_box", _i, [_vp, _i, _i, _i, _ip, _ip, _ip, _ip, _dp, _dp, _dp, _dp]),
    ("rs_factor_root", _i, [_vp, _i, _ip, _ip, _dp]),
    ("rs_apply", _i, [_vp, _i, _vp, _vp, _vp]),
    ("rs_apply_sub", _i, [_vp, _i, _i, _vp, _vp, _vp]),
    ("kernel_matvec", _i, [_vp, _i, _vp, _vp, _vp]),
    ("cbd_fft_workspace_bytes", _sz, [_i, _i, _i]),
    ("cbd_fft_prepare", _i, [_vp, _i, _vp, _sz, _vp]),
    ("kernel_matvec_fft", _i, [_vp, _i, _vp, _vp, _vp]),
    ("cbd_autotune_matvec", _i, [_vp, _i, _vp, _vp, _vp, _ip]),
    ("cbd_matvec_set_shape", _i, [_vp, _i, _i]),
    ("cbd_autotune_apply", _i, [_vp, _i, _vp, _vp, _ip]),
    ("cbd_apply_set_shape", _i, [_vp, _i, _i, _i]),
    ("pcg_workspace_bytes", _sz, [_l, _i]),
    ("pcg_solve", _i, [_vp, _vp, _i, _vp, _vp, _d, _i, _i, _vp, _sz, _ip, _dp, _vp]),
    ("rank_mlp_params", _i, []),
    ("rank_mlp_workspace_bytes", _sz, [_i]),
    ("rank_mlp_forward", _i, [_vp, _i, _vp, _vp, _vp]),
    ("rank_mlp_loss_grad", _i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    ("rank_mlp_adam", _i, [_vp, _vp, _vp, _vp, _i, ctypes.c_float, _vp]),
    ("rank_mlp_loss_grad_noalloc", _i, [_vp, _i, _vp, _vp, _vp, _vp, _vp]),
    ("rs_factor_features", _i, [_vp, _i, _ip, ctypes.POINTER(ctypes.c_float), _ip]),
    ("rs_factor_schedule", _i, [_vp, _ip, _ip, _ip, _dp, _ip, _ip, _ip, _ip, _ip, _ip, ctypes.POINTER(_l)]),
    ("cbd_timing_enable", _i, [_i]),
    ("cbd_timing_get", _i, [ctypes.c_char_p, _dp, ctypes.POINTER(_l)]),
    ("cbd_timing_reset", _i, []),
]

_lib = None


class CbdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libcbd error %d: %s" % (code, msg))
        self.code = code


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcbd.so is not built; run __graft_entry__.build() or "
                               "python paper_2108_12574_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc, allow_warning=False):
    if rc < 0 or (rc > 0 and not allow_warning):
        raise CbdError(rc, lib().cbd_last_error().decode())
    return rc
