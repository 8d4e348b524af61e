"""ctypes declarations of the C ABI in include/sthosvd.h.

Loads paper_2010_10131_amd/libsthosvd.so (built in-tree by build.py) and
raises immediately when it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsthosvd.so")

STH_OK, STH_ERR_INVALID, STH_ERR_LAYOUT, STH_ERR_NOMEM, STH_ERR_HIP, STH_ERR_NUMERIC, \
    STH_ERR_UNSUPPORTED = range(7)
STATUS_NAMES = ["OK", "ERR_INVALID", "ERR_LAYOUT", "ERR_NOMEM", "ERR_HIP", "ERR_NUMERIC",
                "ERR_UNSUPPORTED"]

STH_F64, STH_F32 = 0, 1
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
SOLVER = {"eig": 0, "als": 1, "auto": 2, "auto_tree": 3}


class SthError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 7 else status}: {msg}")
        self.status = status


class sth_batch_tiles(ctypes.Structure):
    _fields_ = [
        ("gram_wg_per_cu", ctypes.c_int32),
        ("gram_wt_max", ctypes.c_int32),
        ("ttm_rows_per_wave", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class sth_desc(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("dims", ctypes.POINTER(ctypes.c_int64)),
        ("ranks", ctypes.POINTER(ctypes.c_int64)),
        ("mode_order", ctypes.POINTER(ctypes.c_int32)),
        ("dtype", ctypes.c_int32),
        ("gram_prec", ctypes.c_int32),
        ("ttm_prec", ctypes.c_int32),
        ("solver", ctypes.c_int32),
        ("per_mode", ctypes.POINTER(ctypes.c_int32)),
        ("als_iters", ctypes.c_int32),
        ("eig_max_sweeps", ctypes.c_int32),
        ("workspace_cap", ctypes.c_int64),
        ("mlp_weights", ctypes.POINTER(ctypes.c_float)),
    ]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_vpp = ctypes.POINTER(ctypes.c_void_p)

# name: (restype, argtypes)
SIGNATURES = {
    "sth_last_error": (ctypes.c_char_p, []),
    "sth_version": (ctypes.c_char_p, []),
    "sthosvd_plan": (ctypes.c_int, [ctypes.POINTER(sth_desc), ctypes.POINTER(_vp), ctypes.POINTER(_sz)]),
    "sthosvd_plan_solvers": (ctypes.c_int, [_vp, _i32p]),
    "sthosvd_plan_destroy": (None, [_vp]),
    "sthosvd_run": (ctypes.c_int, [_vp, _vp, _vp, _vpp, _vpp, _vpp, ctypes.c_uint64, _vp, _sz, _vp]),
    "sthosvd_check": (ctypes.c_int, [_vp, _vp, _vp]),
    "gram_mode_n_workspace": (_sz, [_i32, _i64p, _i32, _i32]),
    "gram_mode_n": (ctypes.c_int, [_i32, _i64p, _i32, _i32, _i32, _vp, _vp, _vp, _sz, _vp]),
    "ttt_mode_n": (ctypes.c_int, [_i32, _i64p, _i32, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ttm_mode_n_workspace": (_sz, [_i64, _i64]),
    "ttm_mode_n": (ctypes.c_int, [_i32, _i64p, _i32, _i64, _i32, _i32, _vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    "ttm_mode_n_noalloc_max_bytes": (_sz, []),
    "ttm_mode_n_noalloc": (ctypes.c_int, [_i32, _i64p, _i32, _i64, _i32, _i32, _vp, _vp, _i32, _vp, _vp]),
    "ttm_factor_bytes": (_sz, [_i64, _i64, _i32]),
    "ttm_factor_prepare": (ctypes.c_int, [_i64, _i64, _i32, _vp, _i32, _vp, _sz, _vp]),
    "ttm_mode_n_prepared": (ctypes.c_int, [_i32, _i64p, _i32, _i64, _i32, _i32, _vp, _vp, _sz, _vp, _vp]),
    "eig_leading_workspace": (_sz, [_i64]),
    "eig_leading": (ctypes.c_int, [_i64, _i64, _vp, _vp, _vp, _i32, _vp, _sz, _vp]),
    "eig_leading_ex": (ctypes.c_int, [_i64, _i64, _vp, _vp, _vp, _i32, ctypes.c_double, _vp, _sz, _vp]),
    "tucker_reconstruct_workspace": (_sz, [_i32, _i64p, _i64p, _i32]),
    "tucker_reconstruct": (ctypes.c_int, [_i32, _i64p, _i64p, _i32, _i32, _vp, _vpp, _vp, _vp, _sz, _vp]),
    "tucker_error_workspace": (_sz, [_i32, _i64p, _i64p, _i32]),
    "sth_hooi_workspace": (_sz, [_i32, _i64p, _i64p, _i32, _i32]),
    "sth_hooi": (ctypes.c_int, [_i32, _i64p, _i64p, _i32, _i32, _i32, _vp, _vpp, _vp, _i32, _vp, _sz, _vp]),
    "sth_hooi_check": (ctypes.c_int, [_vp, _vp]),
    "tucker_error": (ctypes.c_int, [_i32, _i64p, _i64p, _i32, _i32, _vp, _vp, _vpp, _vp, _vp, _sz, _vp]),
    "sth_sumsq": (ctypes.c_int, [_i32, _vp, _i64, _vp, _vp, _sz, _vp]),
    "sthosvd_mode_step_workspace": (_sz, [_i32, _i64p, _i32, _i64, _i32, _i32, _i32, _i32, _i32]),
    "sthosvd_mode_step": (ctypes.c_int, [_i32, _i64p, _i32, _i64, _i32, _i32, _i32, _i32, _i32, _vp, _vp,
                                         _vp, _vp, _vp, ctypes.c_uint64, _vp, _sz, _vp]),
    "sthosvd_choose_exhaustive_workspace": (_sz, [_i32, _i64p, _i64p, _i32, _i32, _i32, _i32]),
    "sthosvd_choose_exhaustive": (ctypes.c_int, [_i32, _i64p, _i64p, _i32, _i32, _i32, _i32, _vp, _i32p,
                                                 ctypes.POINTER(ctypes.c_float), _vp, _sz, _vp]),
    "sthosvd_plan_batched": (ctypes.c_int, [ctypes.POINTER(sth_desc), _i32, ctypes.POINTER(_vp),
                                            ctypes.POINTER(_sz)]),
    "sthosvd_plan_batched_tiles": (ctypes.c_int, [ctypes.POINTER(sth_desc), _i32,
                                                  ctypes.POINTER(sth_batch_tiles), ctypes.POINTER(_vp),
                                                  ctypes.POINTER(_sz)]),
    "sthosvd_plan_batched_destroy": (None, [_vp]),
    "sthosvd_run_batched": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "sthosvd_check_batched": (ctypes.c_int, [_vp, _vp, _vp]),
    "sth_selector_num_params": (_i32, []),
    "sth_selector_num_trainable": (_i32, []),
    "sth_selector_features": (ctypes.c_int, [_i64, _i64, _i64, ctypes.POINTER(ctypes.c_float)]),
    "sth_selector_predict": (ctypes.c_int, [ctypes.POINTER(ctypes.c_float), _i64, _i64, _i64,
                                            ctypes.POINTER(ctypes.c_float)]),
    "sth_selector_choose": (ctypes.c_int, [ctypes.POINTER(ctypes.c_float), _i64, _i64, _i64, _i32p]),
    "sth_selector_tree_choose": (ctypes.c_int, [_i64, _i64, _i64, _i32p]),
    "sth_mlp_workspace": (_sz, [_i64]),
    "sth_mlp_forward": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _sz, _vp]),
    "sth_mlp_loss_grad": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "sth_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, _i32, _vp]),
}

_lib = None


def load() -> ctypes.CDLL:
    """The HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with paper_2010_10131_amd/build.py "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != STH_OK:
        raise SthError(status, load().sth_last_error().decode())


def i64arr(vals):
    return (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])


def i32arr(vals):
    return (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])


def ptrarr(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(p) if p else None for p in ptrs])
