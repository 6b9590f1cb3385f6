"""ctypes declarations of the C ABI in include/hh.h (argument marshalling only).

Loading fails loudly when libhh.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhh.so")

HH_OK = 0
STATUS = {0: "HH_OK", 1: "HH_ERR_INVALID_ARG", 2: "HH_ERR_OUT_OF_MEMORY", 3: "HH_ERR_HIP",
          4: "HH_ERR_DUPLICATE_POINTS", 5: "HH_ERR_CAPACITY", 6: "HH_ERR_NOT_CONVERGED"}
HH_FP64, HH_FP32, HH_BF16, HH_BF16_SPLIT = 0, 1, 2, 3
HH_MLP_INPUT_DIRECTION, HH_MLP_INPUT_DISPLACEMENT = 0, 1
HH_MLP_NPARAM = 9161
HH_G3_NPARAM = 9938
LMAX_CAP = 64
HH_NPHASE = 8
PHASES = ("tree", "partition", "aca", "near", "far", "combine", "backward", "short")

# name -> (restype, argtypes); every symbol declared in include/hh.h
_vp, _i32, _i64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_pi64, _pi32, _pd, _pu64 = (C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                            C.POINTER(C.c_uint64))


class BatchParams(C.Structure):
    """hh_batch_params of include/hh.h."""
    _fields_ = [("n_sys", C.c_int32), ("offsets", C.POINTER(C.c_int64)),
                ("c_leafs", C.POINTER(C.c_int32)), ("c_leaf", C.c_int32), ("eta", C.c_double),
                ("eps", C.c_double), ("l_max", C.c_int32), ("prec", C.c_int)]


SIGNATURES = {
    "hh_ctx_create": (C.c_int, [C.c_int, _vp, C.POINTER(_vp)]),
    "hh_ctx_destroy": (None, [_vp]),
    "hh_last_error": (C.c_char_p, [_vp]),
    "hh_ctx_set_stream": (C.c_int, [_vp, _vp]),
    "hh_synchronize": (C.c_int, [_vp]),
    "hh_ctx_set_budget": (C.c_int, [_vp, C.c_size_t]),
    "hh_ctx_set_team_min": (C.c_int, [_vp, C.c_int32]),
    "hh_kernel_create_rpy": (C.c_int, [_vp, _d, _d, C.POINTER(_vp)]),
    "hh_kernel_create_rpy6": (C.c_int, [_vp, _d, _d, C.POINTER(_vp)]),
    "hh_kernel_create_mlp": (C.c_int, [_vp, _pd, C.c_int, _d, _d, C.POINTER(_vp)]),
    "hh_kernel_free": (None, [_vp]),
    "hh_build_tree": (C.c_int, [_vp, _vp, _i64, _i32, C.POINTER(_vp)]),
    "hh_build_tree6": (C.c_int, [_vp, _vp, _i64, _i32, C.POINTER(_vp)]),
    "hh_build_tree_batch": (C.c_int, [_vp, _vp, _pi64, _i32, _i32, C.POINTER(_vp)]),
    "hh_build_tree_batch_leaf": (C.c_int, [_vp, _vp, _pi64, _i32, C.POINTER(_i32),
                                           C.POINTER(_vp)]),
    "hh_partition": (C.c_int, [_vp, _vp, _d, C.c_int, C.POINTER(_vp)]),
    "hh_aca_build": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int, _d, _i32, _vp, C.POINTER(_vp)]),
    "hh_aca_build_pivots": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int, _pi32, _pi32, _pi32, _pi32,
                                      C.POINTER(_vp)]),
    "hh_tree_refit": (C.c_int, [_vp, _vp, _vp]),
    "hh_batch_create": (C.c_int, [_vp, _vp, C.POINTER(BatchParams), _vp, C.POINTER(_vp)]),
    "hh_batch_matvec": (C.c_int, [_vp, _vp, _vp, _vp]),
    "hh_batch_info": (C.c_int, [_vp, _pi64, _pi32, _pi64, _pi64, C.POINTER(_vp),
                                C.POINTER(_vp), C.POINTER(_vp)]),
    "hh_batch_free": (None, [_vp]),
    "hh_short_create": (C.c_int, [_vp, _vp, _pd, _pd, _d, C.POINTER(_vp)]),
    "hh_short_matvec": (C.c_int, [_vp, _vp, C.c_int, _vp, _vp]),
    "hh_short_info": (C.c_int, [_vp, _pi64, _pi64]),
    "hh_short_free": (None, [_vp]),
    "hh_filament_forces": (C.c_int, [_vp, _vp, _i64, _i64, _i32, _d, _d, _d, _pd, C.c_int, _vp]),
    "hh_euler_step": (C.c_int, [_vp, _vp, _vp, _i64, _d, C.c_int]),
    "hh_matvec": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int, _vp, _vp]),
    "hh_matvec_noalloc": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int, _vp, _vp]),
    "hh_matvec_backward": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int, _vp, _vp, _vp, _vp, _vp]),
    "hh_tree_free": (None, [_vp]),
    "hh_part_free": (None, [_vp]),
    "hh_lowrank_free": (None, [_vp]),
    "hh_tree_info": (C.c_int, [_vp, _pi64, _pi64, _pi64]),
    "hh_tree_export": (C.c_int, [_vp, _pi64, _pu64, _pi32, _pd]),
    "hh_part_info": (C.c_int, [_vp, _pi64, _pi64]),
    "hh_part_export": (C.c_int, [_vp, _pi32, _pi32]),
    "hh_part_stats": (C.c_int, [_vp, _pi64, _pi64]),
    "hh_lowrank_info": (C.c_int, [_vp, _pi64, _pi64, _pi64, _pi64, _pi64]),
    "hh_lowrank_export": (C.c_int, [_vp, _pi32, _pi32, _pi32, _pi32]),
    "hh_lowrank_factor": (C.c_int, [_vp, _i64, _i32, _pd, _pd]),
    "hh_ctx_set_profiling": (C.c_int, [_vp, C.c_int]),
    "hh_ctx_phase_times": (C.c_int, [_vp, _pd, _pi64, C.c_int]),
    "hh_device_arch_ok": (C.c_int, []),
}



_lib = None


def load():
    """Load libhh.so and declare every entry point. Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhh.so is not built (run paper_2505_08174_amd.build.build()); "
                          "there is no CPU fallback")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class HHError(RuntimeError):
    def __init__(self, status, text):
        super().__init__("%s: %s" % (STATUS.get(status, status), text))
        self.status = status


def check(ctx_handle, status):
    if status != HH_OK:
        msg = load().hh_last_error(ctx_handle)
        raise HHError(status, msg.decode() if msg else "")
