"""ctypes declarations of libqsim.so (argument marshalling only).

The library is loaded from the package directory. If it is missing the import fails loudly:
there is no CPU fallback for any call.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqsim.so")

QSIM_C64 = 0
QSIM_C128 = 1

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4
_ERRNAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", EUNSUPPORTED: "EUNSUPPORTED"}

OPS = {
    "MATRIX": 0, "H": 1, "X": 2, "Y": 3, "Z": 4, "S": 5, "SDG": 6, "T": 7, "TDG": 8,
    "RX90": 9, "RX90DG": 10, "RY90": 11, "RY90DG": 12, "PHASE": 13, "RZ": 14, "V": 15, "SWAP": 16,
    "RK": 17, "RKDG": 18, "RENORM": 19,
}

PLAN_PLAIN, PLAN_FUSED, PLAN_STAGED, PLAN_AUTO = 0, 1, 2, 3
STAGED_FULL, STAGED_HALF, STAGED_WAVE = 0, 1, 2
KERNEL_NAMES = {0: "general", 1: "phase", 2: "diag", 3: "swap", 4: "fused_valu", 5: "fused_mfma", 6: "staged",
                7: "renorm"}


class QsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Gate(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int32), ("target", ctypes.c_int32), ("target2", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("controls", ctypes.c_uint64), ("theta", ctypes.c_double),
        ("u", ctypes.c_double * 8),
    ]


class PlanOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("fuse_k", ctypes.c_int32), ("lds_qubits", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("lds_regs", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("gates", ctypes.c_int64), ("launches", ctypes.c_int64), ("passes", ctypes.c_int64),
                ("alg_bytes", ctypes.c_double), ("alg_flops", ctypes.c_double), ("method", ctypes.c_int32),
                ("fuse_k", ctypes.c_int32), ("lds_qubits", ctypes.c_int32), ("lds_regs", ctypes.c_int32),
                ("issued_flops", ctypes.c_double), ("renorms", ctypes.c_int64)]


class BatchStats(ctypes.Structure):
    _fields_ = [("launch_ms", ctypes.c_double), ("circuits", ctypes.c_int64), ("gates", ctypes.c_int64)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("circuits", ctypes.c_int64), ("gates", ctypes.c_int64), ("split_circuits", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("launches", ctypes.c_int64), ("lds_qubits", ctypes.c_int32),
                ("lds_regs", ctypes.c_int32)]


assert ctypes.sizeof(Gate) == 96

_lib = None

# name -> (restype, argtypes)
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i32, _i64, _u64, _f64, _sz = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "qsim_last_error": (ctypes.c_char_p, []),
    "qsim_version": (ctypes.c_char_p, []),
    "qsim_alloc": (_i32, [_i32, _i32, _vp, ctypes.POINTER(_vp)]),
    "qsim_wrap": (_i32, [_vp, _i32, _i32, _vp, ctypes.POINTER(_vp)]),
    "qsim_free": (_i32, [_vp]),
    "qsim_data": (_vp, [_vp]),
    "qsim_num_qubits": (_i32, [_vp]),
    "qsim_get_dtype": (_i32, [_vp]),
    "qsim_set_stream": (_i32, [_vp, _vp]),
    "qsim_set_basis": (_i32, [_vp, _u64]),
    "qsim_upload": (_i32, [_vp, _vp, _sz]),
    "qsim_download": (_i32, [_vp, _vp, _sz]),
    "qsim_sync": (_i32, [_vp]),
    "qsim_apply_1q": (_i32, [_vp, _i32, _dp]),
    "qsim_apply_ctrl": (_i32, [_vp, _u64, _i32, _dp]),
    "qsim_apply_phase": (_i32, [_vp, _u64, _i32, _f64]),
    "qsim_apply_swap": (_i32, [_vp, _u64, _i32, _i32]),
    "qsim_apply_fused": (_i32, [_vp, _i32, ctypes.POINTER(_i32), _dp]),
    "qsim_apply_modexp": (_i32, [_vp, _i32, _i32, _i32, _i32, _u64, _u64]),
    "qsim_norm": (_i32, [_vp, _dp]),
    "qsim_probs": (_i32, [_vp, _vp, _i32]),
    "qsim_marginals": (_i32, [_vp, _dp]),
    "qsim_renormalize": (_i32, [_vp, _dp]),
    "qsim_renormalize_noalloc": (_i32, [_vp, _i32, _i32, _vp, _vp]),
    "qsim_sample": (_i32, [_vp, _i64, _dp, ctypes.POINTER(_u64)]),
    "qsim_plan_create": (_i32, [_i32, _i32, ctypes.POINTER(Gate), _i64, ctypes.POINTER(PlanOpts), ctypes.POINTER(_vp)]),
    "qsim_plan_get_info": (_i32, [_vp, ctypes.POINTER(PlanInfo)]),
    "qsim_plan_get_norms": (_i32, [_vp, _dp, _i64]),
    "qsim_plan_execute": (_i32, [_vp, _vp]),
    "qsim_plan_free": (_i32, [_vp]),
    "qsim_plan_launches": (_i32, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "qsim_plan_execute_from_zero": (_i32, [_vp, _vp]),
    "qsim_plan_execute_timed": (_i32, [_vp, _vp, _i32, _dp, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "qsim_plan_tune": (_i32, [_i32, _i32, ctypes.POINTER(Gate), _i64, _vp, _i32, _i32, ctypes.POINTER(PlanOpts), _dp,
                              ctypes.POINTER(PlanOpts), _dp, _i32, ctypes.POINTER(_i32)]),
    "qsim_batch_create": (_i32, [_i32, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(Gate), _i32,
                                 ctypes.POINTER(PlanOpts), _vp, ctypes.POINTER(_vp)]),
    "qsim_batch_run": (_i32, [_vp, ctypes.POINTER(BatchStats)]),
    "qsim_batch_latencies": (_i32, [_vp, _dp]),
    "qsim_batch_get_info": (_i32, [_vp, ctypes.POINTER(BatchInfo)]),
    "qsim_batch_download": (_i32, [_vp, _i32, _vp, _sz]),
    "qsim_batch_free": (_i32, [_vp]),
}


def lib():
    """Load libqsim.so (raises if it has not been built; never falls back to anything else)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libqsim.so not found at {LIB_PATH}: run paper_quant_ph_0608239_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != OK:
        msg = lib().qsim_last_error().decode(errors="replace")
        raise QsimError(rc, msg)
