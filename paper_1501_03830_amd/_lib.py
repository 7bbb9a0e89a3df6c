"""ctypes view of libbse.so (include/bse.h).  Argument marshalling only."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbse.so")

BSE_OK = 0
BSE_ENOMEM = -1000
BSE_EDEVICE = -1001
BSE_ENOTICKET = -1002
BSE_EUNSUPPORTED = -1003
BSE_EBUSY = -1004
BSE_ENOCONV = -1005

BSE_QUEUED, BSE_RUNNING, BSE_DONE, BSE_FAILED = 0, 1, 2, 3
STATE_NAMES = {0: "queued", 1: "running", 2: "done", 3: "failed"}

BSE_PREC_FP64 = 0
BSE_PREC_FP32_REFINE = 1

BSE_WANT_VECTORS = 1
BSE_WANT_WEIGHTS = 2
BSE_TWO_STAGE = 4
BSE_EIGVEC_TWISTED = 8

BSE_NUM_STAGES = 11
STAGE_NAMES = ["build_M", "potrf", "form_W", "sktrd", "bisect", "invit", "reorth", "apply_U",
               "apply_L", "finish", "refine"]


class BseReport(ctypes.Structure):
    _fields_ = [
        ("total_ms", ctypes.c_double),
        ("stage_ms", ctypes.c_double * BSE_NUM_STAGES),
        ("n", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("workspace_bytes", ctypes.c_size_t),
        ("symv_ms", ctypes.c_double),
        ("symv_bytes", ctypes.c_double),
        ("symv_launches", ctypes.c_longlong),
        ("refine_sweeps", ctypes.c_int),
        ("refine_first_correction", ctypes.c_double),
        ("refine_correction", ctypes.c_double),
        ("graph", ctypes.c_int),
    ]

    def as_dict(self):
        return {
            "total_ms": self.total_ms,
            "stage_ms": {name: self.stage_ms[i] for i, name in enumerate(STAGE_NAMES)},
            "n": self.n,
            "prec": self.prec,
            "workspace_bytes": self.workspace_bytes,
            "symv_ms": self.symv_ms,
            "symv_bytes": self.symv_bytes,
            "symv_launches": self.symv_launches,
            "refine_sweeps": self.refine_sweeps,
            "refine_first_correction": self.refine_first_correction,
            "refine_correction": self.refine_correction,
            "graph": self.graph,
        }


class BseRequest(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("A", ctypes.c_void_p),
        ("lda", ctypes.c_int),
        ("B", ctypes.c_void_p),
        ("ldb", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("flags", ctypes.c_uint),
        ("lambda_", ctypes.c_void_p),
        ("X", ctypes.c_void_p),
        ("ldx", ctypes.c_int),
        ("d_r", ctypes.c_void_p),
        ("d_l", ctypes.c_void_p),
        ("w", ctypes.c_void_p),
    ]


class BseServeCounters(ctypes.Structure):
    _fields_ = [
        ("pool_bytes", ctypes.c_size_t),
        ("used_bytes", ctypes.c_size_t),
        ("peak_used_bytes", ctypes.c_size_t),
        ("queued", ctypes.c_longlong),
        ("inflight", ctypes.c_longlong),
        ("max_inflight", ctypes.c_longlong),
        ("batches", ctypes.c_longlong),
        ("solved", ctypes.c_longlong),
        ("slots", ctypes.c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# (name, restype, argtypes) for every symbol declared in include/bse.h
_P = ctypes.c_void_p
_I = ctypes.c_int
_U = ctypes.c_uint
_D = ctypes.POINTER(ctypes.c_double)
SIGNATURES = [
    ("bse_version", _I, []),
    ("bse_last_error", ctypes.c_char_p, []),
    ("bse_ctx_create", _I, [ctypes.POINTER(_P), _I, _P, ctypes.c_size_t, _P]),
    ("bse_ctx_destroy", _I, [_P]),
    ("bse_ctx_set_timing", _I, [_P, _I]),
    ("bse_ctx_set_graphs", _I, [_P, _I]),
    ("bse_get_tile_table", _I, [ctypes.POINTER(_I)]),
    ("bse_set_tile_table", _I, [_P, ctypes.POINTER(_I)]),
    ("bse_footprint_bytes", ctypes.c_size_t, [_I, _I, _U]),
    ("bse_solve", _I, [_P, _I, _P, _I, _P, _I, _I, _U, _P, _P, _I, _P, _P, _P, ctypes.POINTER(BseReport)]),
    ("bse_solve_real", _I, [_P, _I, _P, _I, _P, _I, _I, _U, _P, _P, _I, _P, _P, _P, ctypes.POINTER(BseReport)]),
    ("bse_solve_tda", _I, [_P, _I, _P, _I, _I, _U, _P, _P, _I, _P, _P, _P, ctypes.POINTER(BseReport)]),
    ("bse_spectra", _I, [_P, _I, _P, _P, _I, ctypes.c_double, ctypes.c_double, ctypes.c_double, _P, _P]),
    ("bse_footprint_batched_bytes", ctypes.c_size_t, [_I, ctypes.POINTER(_I), _I, _U]),
    ("bse_solve_batched", _I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_P), ctypes.POINTER(_I),
                               ctypes.POINTER(_P), ctypes.POINTER(_I), _I, _U, ctypes.POINTER(_P),
                               ctypes.POINTER(_P), ctypes.POINTER(_I), ctypes.POINTER(_P),
                               ctypes.POINTER(_P), ctypes.POINTER(_I), ctypes.POINTER(BseReport)]),
    ("bse_serve_config", _I, [_P, ctypes.c_size_t, _I, _I]),
    ("bse_submit", _I, [_P, ctypes.POINTER(BseRequest), ctypes.POINTER(ctypes.c_uint64)]),
    ("bse_poll", _I, [_P, ctypes.c_uint64, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    ("bse_release", _I, [_P, ctypes.c_uint64]),
    ("bse_ticket_times", _I, [_P, ctypes.c_uint64, _D, _D, _D]),
    ("bse_serve_stats", _I, [_P, ctypes.POINTER(BseServeCounters)]),
    ("bse_noalloc_max_bytes", ctypes.c_size_t, []),
    ("bse_solve_noalloc", _I, [_P, _I, _P, _I, _P, _I, _I, _U, _P, _P, _I, _P, _P, _P]),
    ("bse_plan_check", _I, [_I, ctypes.POINTER(_I), _I, _U, ctypes.c_char_p, ctypes.c_size_t]),
    ("bse_build_M", _I, [_P, _I, _P, _I, _P, _I, _P, _I]),
    ("bse_potrf", _I, [_P, _I, _P, _I]),
    ("bse_form_W", _I, [_P, _I, _P, _I, _P, _I]),
    ("bse_sktrd", _I, [_P, _I, _P, _I, _P, _P]),
    ("bse_sktrd2", _I, [_P, _I, _P, _I, _P]),
    ("bse_tridiag_eig", _I, [_P, _I, _P, _P, _P, _I]),
    ("bse_tridiag_eig_flags", _I, [_P, _I, _P, _P, _P, _I, _U]),
]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libbse.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} not found: build the HIP library first (python -m paper_1501_03830_amd.build)")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    lib = load()
    s = lib.bse_last_error()
    return s.decode() if s else ""


class BseError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what} returned {code}: {last_error()}")


def check(code: int, what: str) -> int:
    """Raise on negative codes; positive codes (leading minor not definite)
    are returned to the caller."""
    if code < 0:
        raise BseError(code, what)
    return code
