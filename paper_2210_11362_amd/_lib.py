"""ctypes loader for libtrals.so and the raw C-ABI functions (same names as
include/tr_als.h).  No arithmetic happens here: every step runs in the HIP
library, and a missing library raises instead of falling back."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrals.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tr_als.h")

TR_NE, TR_QR, TR_QRNE = 0, 1, 2
TR_F64, TR_F32, TR_BF16, TR_FP8 = 0, 1, 2, 3
TR_OK, TR_EINVAL, TR_ENOMEM, TR_EHIP, TR_ESINGULAR, TR_ENONFINITE = 0, -1, -2, -3, -4, -5

PREC = {"f64": TR_F64, "f32": TR_F32, "bf16": TR_BF16, "fp8": TR_FP8}
VARIANT = {"ne": TR_NE, "qr": TR_QR, "qrne": TR_QRNE}
TR_SOLVE_FACTOR, TR_SOLVE_PINV = 0, 1
SOLVE = {"factor": TR_SOLVE_FACTOR, "pinv": TR_SOLVE_PINV}

_vp = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "tr_als_init": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _i64p, _i64p, _vp, ctypes.c_int,
                                   ctypes.POINTER(_vp), ctypes.c_int, _vp]),
    "tr_als_sweep": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "tr_als_fit": (ctypes.c_int, [_vp, _dp]),
    "tr_als_destroy": (ctypes.c_int, [_vp]),
    "tr_als_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "tr_als_last_error": (ctypes.c_char_p, [_vp]),
    "tr_als_mttsp": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp]),
    "tr_als_coef": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
    "tr_als_gram": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
    "tr_als_update_mode": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "tr_als_store_cores": (ctypes.c_int, [_vp]),
    "tr_als_xnorm2": (ctypes.c_int, [_vp, _dp]),
    "tr_als_mode_regime": (ctypes.c_int, [_vp, ctypes.c_int]),
    "tr_als_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "tr_als_debug_overruns": (ctypes.c_int, []),
    "tr_als_debug_graphs": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_int]),
    "tr_als_profile_read": (ctypes.c_int, [_vp, _dp, _i64p, _dp]),
    "tr_als_set_solve": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double]),
    "tr_als_run": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  ctypes.POINTER(ctypes.c_int), _dp]),
    "tr_inner": (ctypes.c_int, [ctypes.c_int, _i64p, _i64p, ctypes.POINTER(_vp), _i64p, ctypes.POINTER(_vp), _dp,
                                _vp]),
    "tr_norm": (ctypes.c_int, [ctypes.c_int, _i64p, _i64p, ctypes.POINTER(_vp), _dp, _vp]),
    "tr_als_debug_shadow": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_float),
                                           _i64p]),
}


class JobDesc(ctypes.Structure):
    """tr_job_desc."""
    _fields_ = [("N", ctypes.c_int), ("dims", ctypes.c_int64 * 8), ("ranks", ctypes.c_int64 * 8),
                ("variant", ctypes.c_int), ("prec_mixed", ctypes.c_int), ("nsweeps_mixed", ctypes.c_int),
                ("prec_fin", ctypes.c_int), ("nsweeps_fin", ctypes.c_int), ("refine", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("eta", ctypes.c_double), ("X", _vp), ("x_dtype", ctypes.c_int),
                ("init_cores", ctypes.POINTER(_vp)), ("t_arrival", ctypes.c_double)]


class JobInfo(ctypes.Structure):
    """tr_job_info."""
    _fields_ = [("state", ctypes.c_int), ("status", ctypes.c_int), ("rel_err", ctypes.c_double),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("footprint", ctypes.c_size_t), ("slot", ctypes.c_int), ("batched", ctypes.c_int)]


class SrvStats(ctypes.Structure):
    """tr_srv_stats."""
    _fields_ = [("submitted", ctypes.c_uint64), ("done", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("arena_bytes", ctypes.c_size_t), ("peak_in_use", ctypes.c_size_t), ("slots", ctypes.c_int),
                ("max_running", ctypes.c_int)]


TR_JOB_QUEUED, TR_JOB_RUNNING, TR_JOB_DONE, TR_JOB_FAILED = 0, 1, 2, 3
TR_SRV_BATCH = 1

_SIGS.update({
    "tr_gen_planted": (ctypes.c_int, [ctypes.c_int, _i64p, _i64p, ctypes.c_uint64, ctypes.c_double, _vp,
                                      ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
    "tr_gen_planted_noalloc": (ctypes.c_int, [ctypes.c_int, _i64p, _i64p, ctypes.c_uint64, ctypes.c_double, _vp,
                                              ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
    "tr_srv_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_size_t, ctypes.c_int, ctypes.c_int]),
    "tr_srv_submit": (ctypes.c_int, [_vp, ctypes.POINTER(JobDesc), ctypes.POINTER(ctypes.c_uint64)]),
    "tr_srv_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(JobInfo)]),
    "tr_srv_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(JobInfo)]),
    "tr_srv_result": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "tr_srv_drain": (ctypes.c_int, [_vp]),
    "tr_srv_stats_read": (ctypes.c_int, [_vp, ctypes.POINTER(SrvStats)]),
    "tr_srv_destroy": (ctypes.c_int, [_vp]),
    "tr_srv_job_error": (ctypes.c_char_p, [_vp, ctypes.c_uint64]),
})

_lib = None


def header_symbols(path: str = HEADER):
    """Function names declared in the public header."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tr_[a-z_0-9]+)\s*\(", txt)))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2210_11362_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class TRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def check(code: int, ctx=None, what: str = ""):
    if code != TR_OK:
        L = lib()
        detail = L.tr_als_last_error(ctx).decode() if ctx else ""
        base = L.tr_als_strerror(code).decode()
        raise TRError(code, f"{what}: {base}" + (f" ({detail})" if detail else ""))
    return code


def __getattr__(name):
    if name in _SIGS:
        return getattr(lib(), name)
    raise AttributeError(name)
