"""ctypes declarations of the C interface in include/imq.h and include/imq_debug.h.

Loading fails loudly if libimq.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libimq.so")

IMQ_MAX_LEVELS = 31
IMQ_NSTAGES = 10

STATUS = {0: "IMQ_OK", 1: "IMQ_ENOTCONVERGED", -1: "IMQ_EINVAL", -2: "IMQ_EDUPLICATE",
          -3: "IMQ_ENOMEM", -4: "IMQ_EHIP", -5: "IMQ_EUNSUPPORTED"}
F64, F32 = 0, 1
PREC = {"fp64": 0, "fp32": 1}


class TreeParams(ctypes.Structure):
    _fields_ = [("leaf_max", ctypes.c_int), ("order_p", ctypes.c_int), ("max_level", ctypes.c_int),
                ("level_order", ctypes.c_int * (IMQ_MAX_LEVELS + 1)),
                ("direct_max", ctypes.c_int), ("autotune", ctypes.c_int), ("autotune_tol", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iters", ctypes.c_int),
                ("mixed_ir", ctypes.c_int), ("max_outer", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)), ("precond", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("relres_fast64", ctypes.c_double)]


class KernelConfig(ctypes.Structure):
    _fields_ = [("m2l_kc", ctypes.c_int), ("m2l_split", ctypes.c_int),
                ("shift_cols", ctypes.c_int), ("m2l_mode", ctypes.c_int),
                ("p2p_wg", ctypes.c_int), ("p2p_mode", ctypes.c_int),
                ("far_field", ctypes.c_int)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class TreeInfo(ctypes.Structure):
    _fields_ = [("npoints", ctypes.c_int64), ("nboxes", ctypes.c_int64), ("nleaves", ctypes.c_int64),
                ("depth", ctypes.c_int), ("order_p", ctypes.c_int), ("K", ctypes.c_int),
                ("p2p_pairs", ctypes.c_int64), ("m2l_pairs", ctypes.c_int64),
                ("m2p_evals", ctypes.c_int64), ("p2l_evals", ctypes.c_int64),
                ("m2m_pairs", ctypes.c_int64), ("l2l_pairs", ctypes.c_int64),
                ("nlevels", ctypes.c_int),
                ("level_boxes", ctypes.c_int64 * (IMQ_MAX_LEVELS + 1)),
                ("level_m2l_pairs", ctypes.c_int64 * (IMQ_MAX_LEVELS + 1)),
                ("level_K", ctypes.c_int * (IMQ_MAX_LEVELS + 1)),
                ("tuned_prec", ctypes.c_int), ("tuned_err", ctypes.c_double), ("tuned_ms", ctypes.c_double)]


_lib = None

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double
_p = ctypes.POINTER

SIGNATURES = {
    "imq_build_tree": (_int, [_int, _p(_i64), _vp, _p(_dbl), _p(TreeParams), _vp, _p(_vp)]),
    "imq_build_tree_alloc": (_int, [_int, _p(_i64), _vp, _p(_dbl), _p(TreeParams), _p(Allocator), _vp, _p(_vp)]),
    "imq_matvec": (_int, [_vp, _int, _int, _vp, _i64, _vp, _i64, _int, _vp]),
    "imq_matvec_noalloc": (_int, [_vp, _int, _int, _vp, _i64, _vp, _i64, _int, _vp]),
    "imq_matvec_noalloc_max_bytes": (ctypes.c_size_t, []),
    "imq_build_eval_tree": (_int, [_vp, _i64, _vp, _i64, _dbl, _p(TreeParams), _vp, _p(_vp)]),
    "imq_evaluate": (_int, [_vp, _int, _int, _vp, _i64, _vp, _i64, _int, _vp]),
    "imq_rows_exact": (_int, [_vp, _int, _vp, _i64, _i64, _vp, _vp, _i64, _vp]),
    "imq_solve": (_int, [_vp, _int, _vp, _i64, _vp, _i64, _p(SolveOpts), _p(SolveStats), _vp]),
    "imq_matvec_backward": (_int, [_vp, _int, _int, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _int, _vp]),
    "imq_get_tree_info": (_int, [_vp, _p(TreeInfo)]),
    "imq_set_kernel_config": (_int, [_vp, _p(KernelConfig)]),
    "imq_set_level_orders": (_int, [_vp, _int, _p(_int)]),
    "imq_set_stage_timing": (_int, [_vp, _int]),
    "imq_get_stage_times": (_int, [_vp, _p(_dbl)]),
    "imq_stage_name": (ctypes.c_char_p, [_int]),
    "imq_tree_free": (None, [_vp]),
    "imq_status_string": (ctypes.c_char_p, [_int]),
    "imq_last_error": (ctypes.c_char_p, []),
    "imq_debug_table": (_int, [_int, _int, _int, _int, _int, _int, _dbl, _p(_dbl)]),
    "imq_debug_host_tree": (_vp, [_int, _p(_i64), _p(_dbl), _p(_dbl), _p(_dbl), _p(TreeParams), _p(_int)]),
    "imq_debug_host_tree_size": (_i64, [_vp, ctypes.c_char_p]),
    "imq_debug_host_tree_get": (_int, [_vp, ctypes.c_char_p, _vp]),
    "imq_debug_host_tree_free": (None, [_vp]),
    "imq_debug_tree_table": (_int, [_vp, _int, _int, _int, _int, _vp]),
    "imq_debug_device_tree": (_vp, [_int, _p(_i64), _p(_dbl), _p(_dbl), _p(_dbl), _p(TreeParams), _p(_int)]),
    "imq_debug_eval_points": (_i64, [_i64, _p(_dbl), _p(_dbl), _i64, _p(_dbl), _p(_dbl), _p(_i64)]),
}


def load():
    """Load libimq.so (built by __graft_entry__.build() or build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class IMQError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = load().imq_last_error().decode()
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")


def check(status: int, where: str, allow_not_converged: bool = False) -> int:
    if status == 0 or (allow_not_converged and status == 1):
        return status
    raise IMQError(status, where)


def params(leaf: int, p: int, max_level: int = 0, level_order=None, direct_max: int = 0,
           autotune: bool = False, autotune_tol: float = 0.0) -> TreeParams:
    prm = TreeParams()
    prm.leaf_max = int(leaf)
    prm.order_p = int(p)
    prm.max_level = int(max_level)
    prm.direct_max = int(direct_max)
    prm.autotune = 1 if autotune else 0
    prm.autotune_tol = float(autotune_tol)
    for i in range(IMQ_MAX_LEVELS + 1):
        prm.level_order[i] = 0
    if level_order is not None:
        for i, v in enumerate(level_order):
            prm.level_order[i] = int(v)
    return prm
