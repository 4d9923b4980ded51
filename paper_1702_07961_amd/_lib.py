"""ctypes binding of libmms (argument marshalling only).

Every call maps one-to-one onto an ``extern "C"`` entry point of
``include/mms.h``; all sorting work runs in the library's HIP kernels.  The
library must be built (``paper_1702_07961_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# MMS_LIBRARY names another build of the same library (the sanitizer builds
# of paper_1702_07961_amd.build); by default the in-tree libmms.so
LIB_PATH = os.environ.get("MMS_LIBRARY") or os.path.join(PKG, "libmms.so")
# tuning table written by paper_1702_07961_amd.autotune; MMS_TUNING_FILE
# overrides the path, an empty value keeps the library's built-in default
TUNING_PATH = os.path.join(PKG, "tuning_mi355x.json")

MMS_OK = 0
MMS_PENDING = 1
MMS_EINVAL = -1
MMS_ENOMEM = -2
MMS_EHIP = -3
MMS_ENOENT = -4
MMS_ESHUTDOWN = -5

MMS_PAIRS = 0x1
MMS_KEY_I32 = 0x2
MMS_KEY_I64 = 0x4
MMS_KEYS64 = 0x8
MMS_MERGEPATH = 0x10

# every symbol include/mms.h declares
EXPORTS = [
    "mms_last_error", "mms_version", "mms_plan", "mms_workspace_bytes", "mms_sort_u32",
    "mms_sort_pairs_u32", "mms_sort_u64", "mms_sort_pairs_u64", "mms_sort_mergepath_u32", "mms_sort_u32_noalloc", "mms_partition_u32", "mms_copy_u32", "mms_timing_enable", "mms_timing_kinds",
    "mms_timing_reset", "mms_timing_read", "mms_segmented_workspace_bytes", "mms_segmented_sort",
    "mms_set_tuning", "mms_get_tuning", "mms_server_create", "mms_submit", "mms_poll", "mms_wait",
    "mms_release", "mms_server_get_stats", "mms_server_destroy",
]

MMS_SERVER_MAX_STREAMS = 8
MMS_SERVER_DRY_RUN = 0x1

KERNEL_KINDS = ["tile_sort", "partition", "merge", "copy", "segmented"]

_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32


class MmsPlan(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
        ("tile", ctypes.c_uint32),
        ("lanes_per_tile", ctypes.c_uint32),
        ("fanout", ctypes.c_uint32),
        ("merge_tile", ctypes.c_uint32),
        ("rounds", ctypes.c_uint32),
        ("passes", ctypes.c_uint32),
        ("workspace_bytes", ctypes.c_uint64),
    ]


class MmsTiming(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_uint64 * 5),
        ("total_ms", ctypes.c_double * 5),
    ]


class MmsTuning(ctypes.Structure):
    _fields_ = [
        ("max_log2_n", ctypes.c_uint32),
        ("fanout", ctypes.c_uint32),
        ("merge_tile", ctypes.c_uint32),
        ("variant", ctypes.c_uint32),
        ("base", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
    ]


class MmsServerCfg(ctypes.Structure):
    _fields_ = [
        ("d_arena", ctypes.c_void_p),
        ("arena_bytes", ctypes.c_uint64),
        ("streams", ctypes.c_void_p * 8),
        ("num_streams", ctypes.c_uint32),
        ("max_inflight", ctypes.c_uint32),
        ("max_requests", ctypes.c_uint32),
        ("max_batch_requests", ctypes.c_uint32),
        ("max_batch_keys", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class MmsRequest(ctypes.Structure):
    _fields_ = [
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("n", ctypes.c_uint64),
        ("d_keys", ctypes.c_void_p),
        ("d_vals", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
    ]


class MmsResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("n", ctypes.c_uint64),
        ("d_keys", ctypes.c_void_p),
        ("d_vals", ctypes.c_void_p),
        ("t_submit_us", ctypes.c_double),
        ("t_admit_us", ctypes.c_double),
        ("t_launch_us", ctypes.c_double),
        ("t_done_us", ctypes.c_double),
        ("batch", ctypes.c_uint64),
        ("batch_requests", ctypes.c_uint32),
        ("stream_index", ctypes.c_uint32),
    ]


class MmsServerStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "submitted", "admitted", "completed", "released", "rejected", "batches", "queued", "running",
        "data_budget_bytes", "used_bytes", "peak_used_bytes", "meta_bytes", "max_batch_seen")]


class MmsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mms error {code}: {msg}")
        self.code = code


_lib = None


def _declare(lib):
    lib.mms_last_error.restype = ctypes.c_char_p
    lib.mms_last_error.argtypes = []
    lib.mms_version.restype = ctypes.c_int
    lib.mms_plan.argtypes = [_u64, _u32, ctypes.POINTER(MmsPlan)]
    lib.mms_plan.restype = ctypes.c_int
    lib.mms_workspace_bytes.argtypes = [_u64, _u32]
    lib.mms_workspace_bytes.restype = ctypes.c_size_t
    lib.mms_sort_u32.argtypes = [_vp, _vp, _u64, _vp, ctypes.c_size_t, _u32, _vp]
    lib.mms_sort_u32.restype = ctypes.c_int
    lib.mms_sort_pairs_u32.argtypes = [_vp, _vp, _vp, _vp, _u64, _vp, ctypes.c_size_t, _u32, _vp]
    lib.mms_sort_pairs_u32.restype = ctypes.c_int
    lib.mms_sort_mergepath_u32.argtypes = [_vp, _vp, _u64, _vp, ctypes.c_size_t, _u32, _vp]
    lib.mms_sort_mergepath_u32.restype = ctypes.c_int
    lib.mms_sort_u32_noalloc.argtypes = [_vp, _vp, _u64, _u32, _vp]
    lib.mms_sort_u32_noalloc.restype = ctypes.c_int
    lib.mms_sort_u64.argtypes = [_vp, _vp, _u64, _vp, ctypes.c_size_t, _u32, _vp]
    lib.mms_sort_u64.restype = ctypes.c_int
    lib.mms_sort_pairs_u64.argtypes = [_vp, _vp, _vp, _vp, _u64, _vp, ctypes.c_size_t, _u32, _vp]
    lib.mms_sort_pairs_u64.restype = ctypes.c_int
    lib.mms_partition_u32.argtypes = [_vp, _u64, _u64, _u32, _vp, _vp, _u64, _vp, _u32, _vp]
    lib.mms_partition_u32.restype = ctypes.c_int
    lib.mms_copy_u32.argtypes = [_vp, _vp, _u64, _vp]
    lib.mms_copy_u32.restype = ctypes.c_int
    lib.mms_timing_enable.argtypes = [ctypes.c_int]
    lib.mms_timing_enable.restype = ctypes.c_int
    lib.mms_timing_kinds.argtypes = [ctypes.c_uint32]
    lib.mms_timing_kinds.restype = ctypes.c_int
    lib.mms_timing_reset.argtypes = []
    lib.mms_timing_reset.restype = ctypes.c_int
    lib.mms_timing_read.argtypes = [ctypes.POINTER(MmsTiming)]
    lib.mms_timing_read.restype = ctypes.c_int
    lib.mms_segmented_workspace_bytes.argtypes = [_vp, _u64, _u32]
    lib.mms_segmented_workspace_bytes.restype = ctypes.c_size_t
    lib.mms_segmented_sort.argtypes = [_vp, _vp, _vp, _vp, _vp, _u64, _vp, ctypes.c_size_t, _u32, _vp]
    lib.mms_segmented_sort.restype = ctypes.c_int
    lib.mms_set_tuning.argtypes = [ctypes.POINTER(MmsTuning), _u32]
    lib.mms_set_tuning.restype = ctypes.c_int
    lib.mms_get_tuning.argtypes = [_u64, _u32, ctypes.POINTER(MmsTuning)]
    lib.mms_get_tuning.restype = ctypes.c_int
    lib.mms_server_create.argtypes = [ctypes.POINTER(MmsServerCfg), ctypes.POINTER(_vp)]
    lib.mms_server_create.restype = ctypes.c_int
    lib.mms_submit.argtypes = [_vp, ctypes.POINTER(MmsRequest), ctypes.POINTER(_u64)]
    lib.mms_submit.restype = ctypes.c_int
    lib.mms_poll.argtypes = [_vp, _u64, ctypes.POINTER(MmsResult)]
    lib.mms_poll.restype = ctypes.c_int
    lib.mms_wait.argtypes = [_vp, _u64, ctypes.c_int64, ctypes.POINTER(MmsResult)]
    lib.mms_wait.restype = ctypes.c_int
    lib.mms_release.argtypes = [_vp, _u64, _vp]
    lib.mms_release.restype = ctypes.c_int
    lib.mms_server_get_stats.argtypes = [_vp, ctypes.POINTER(MmsServerStats)]
    lib.mms_server_get_stats.restype = ctypes.c_int
    lib.mms_server_destroy.argtypes = [_vp]
    lib.mms_server_destroy.restype = ctypes.c_int
    return lib


def lib() -> ctypes.CDLL:
    """Load libmms.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1702_07961_amd.build` "
                "(the HIP library is required; there is no CPU fallback)")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
        load_tuning(_lib)
    return _lib


def load_tuning(lib, path: str | None = None) -> int:
    """Install the autotuned table (if present); returns the entry count."""
    if path is None:
        path = os.environ.get("MMS_TUNING_FILE", TUNING_PATH)
    if not path or not os.path.exists(path):
        return 0
    with open(path) as f:
        table = json.load(f)
    entries = [(e, 0) for e in table["entries"]] + [(e, MMS_PAIRS) for e in table.get("pairs_entries", [])]
    arr = (MmsTuning * max(1, len(entries)))()
    for i, (e, kind) in enumerate(entries):
        arr[i] = MmsTuning(int(e["max_log2_n"]), int(e["fanout"]), int(e["merge_tile"]), int(e["variant"]),
                           int(e.get("base", 0)), kind)
    if lib.mms_set_tuning(arr, len(entries)) != MMS_OK:
        raise MmsError(MMS_EINVAL, f"{path}: " + lib.mms_last_error().decode())
    return len(entries)


def check(code: int) -> int:
    if code < 0:
        raise MmsError(code, lib().mms_last_error().decode())
    return code
