"""ctypes binding of libbpmf.so (include/bpmf.h): argument marshalling only.

Every step of the sampler runs in the HIP library; this module converts
Python values and device-pointer integers into the C structs and checks the
returned status.  It raises when the library is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BPMF_LIBRARY") or os.path.join(HERE, "libbpmf.so")

BPMF_FP64, BPMF_FP32, BPMF_BF16 = 0, 1, 2
PRECISIONS = {"fp64": BPMF_FP64, "fp32": BPMF_FP32, "bf16": BPMF_BF16}

P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
F64 = C.c_double
SZ = C.c_size_t


class Ratings(C.Structure):
    _fields_ = [("M", I64), ("N", I64), ("nnz", I64),
                ("d_row_ptr", P), ("d_col_idx", P), ("d_row_val", P),
                ("d_col_ptr", P), ("d_row_idx", P), ("d_col_val", P),
                ("val_is_f64", I32)]


class LaunchShape(C.Structure):
    _fields_ = [("heavy_min_ratings", I32), ("piece_min_ratings", I32), ("heavy_split", I32),
                ("rank1_max_ratings", I32), ("rank1_split", I32), ("kernel_variant", I32)]


class Params(C.Structure):
    _fields_ = [("K", I32), ("precision", I32), ("alpha", F64), ("beta0", F64), ("nu0", F64),
                ("mu0", P), ("W0", P), ("mean_rating", F64), ("seed", C.c_uint64),
                ("burnin", I32), ("use_graph", I32), ("validate", I32),
                ("shape", C.POINTER(LaunchShape))]


class Info(C.Structure):
    _fields_ = [("sweeps_done", I64), ("fallback_rows", I64), ("nonfinite_rows", I64),
                ("mean_rating", F64), ("K", I32), ("precision", I32),
                ("rank1_rows", I64 * 2), ("heavy_rows", I64 * 2), ("pieces", I64 * 2),
                ("kernel_variant", I32)]


class FoldinModel(C.Structure):
    _fields_ = [("S", I32), ("K", I32), ("N", I64), ("alpha", F64), ("mean_rating", F64),
                ("d_V", P), ("d_Lambda", P), ("d_mu", P)]


class ServerStats(C.Structure):
    _fields_ = [("requests_done", I64), ("batches", I64), ("max_batch", I64), ("max_inflight", I64),
                ("max_batch_bytes", I64), ("stream_capacity", I64)]


TIMING_CLASSES = ("stats", "hyper", "rows_users", "rows_movies", "fp64_recompute", "predict", "counter",
                  "rows_rank1", "rows_heavy")


class Timing(C.Structure):
    _fields_ = [("ms", F64 * len(TIMING_CLASSES)), ("launches", I64 * len(TIMING_CLASSES))]


class BpmfError(RuntimeError):
    def __init__(self, status, what, msg):
        super().__init__(f"{what}: {msg} (status {status})")
        self.status = status


_lib = None

EXPORTS = {
    "bpmf_workspace_size": [P, P, I64, P],
    "bpmf_init": [P, P, P, P, P, P, SZ, I64, P, P, P],
    "bpmf_sweep": [P, I32, P, I64, P],
    "bpmf_predict": [P, I64, P, P, P, P],
    "bpmf_test_predictions": [P, P, P, P],
    "bpmf_get_hyper": [P, P, P],
    "bpmf_get_info": [P, P, P],
    "bpmf_snapshot": [P, P, P, P, P],
    "bpmf_state_size": [P, P],
    "bpmf_state_save": [P, P, SZ, P],
    "bpmf_state_restore": [P, P, SZ, P],
    "bpmf_destroy": [P],
    "bpmf_set_timing": [P, I32],
    "bpmf_get_timing": [P, P, I32],
    "bpmf_foldin_workspace_size": [P, I64, P],
    "bpmf_foldin": [P, I64, P, P, P, P, P, I64, P, P, SZ, P],
    "bpmf_foldin_noalloc": [P, I64, P, P, P, P, P, I64, P, P],
    "bpmf_foldin_noalloc_max_partials": [],
    "bpmf_server_create": [P, P, SZ, I32, I32, I32],
    "bpmf_server_create_resident": [P, P, I32, I32, I32, I64],
    "bpmf_server_submit": [P, I64, I32, P, P, I32, P],
    "bpmf_server_poll": [P, I32, P, P, P, I64, P, P],
    "bpmf_server_drain": [P],
    "bpmf_server_get_stats": [P, P],
    "bpmf_server_replay": [P, I64, P, P, P, P, P, P, P, P],
    "bpmf_server_destroy": [P],
    "bpmf_status_string": [I32],
    "bpmf_last_error": [],
    "bpmf_version": [],
}


def load(path: str = LIB_PATH):
    """Load libbpmf.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1705_10633_amd.build`")
    lib = C.CDLL(path)
    for name, args in EXPORTS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = (C.c_char_p if name in ("bpmf_status_string", "bpmf_last_error", "bpmf_version")
                      else I64 if name == "bpmf_foldin_noalloc_max_partials" else I32)
    _lib = lib
    return lib


def check(status: int, what: str):
    if status != 0:
        lib = load()
        raise BpmfError(status, what, lib.bpmf_last_error().decode())


def call(name: str, *args):
    lib = load()
    check(getattr(lib, name)(*args), name)
