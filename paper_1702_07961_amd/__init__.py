"""MI355X multiway mergesort (arXiv 1702.07961) — Python front end.

Thin wrappers over the C ABI in ``include/mms.h``: PyTorch supplies device
memory and the stream, ``libmms.so`` does every step of the sort in HIP
kernels.  Importing this package does not load the library; the first call
does, and fails loudly if it has not been built.
"""
from __future__ import annotations

from . import _lib
from ._lib import MMS_KEY_I32, MMS_KEY_I64, MMS_KEYS64, MMS_MERGEPATH, MMS_PAIRS, MmsError, MmsPlan  # noqa: F401
from .server import Result, Server  # noqa: F401

__all__ = ["sort", "sort_pairs", "sort64", "sort_pairs64", "sort_mergepath", "partition", "copy", "plan", "workspace_bytes", "MmsError",
           "timing_enable", "timing_reset", "timing_read", "segmented_sort", "segmented_workspace_bytes",
           "set_tuning", "get_tuning", "Server", "Result"]


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check_u32(t, name):
    torch = _torch()
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype not in (torch.int32, torch.uint32):
        raise ValueError(f"{name} must be int32/uint32, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def plan(n: int, pairs: bool = False, i32: bool = False, keys64: bool = False,
         mergepath: bool = False) -> MmsPlan:
    """Tile size, fan-out, rounds, passes and workspace for a sort of n elements."""
    p = MmsPlan()
    flags = ((MMS_PAIRS if pairs else 0) | (MMS_KEY_I32 if i32 else 0) | (MMS_KEYS64 if keys64 else 0)
             | (MMS_MERGEPATH if mergepath else 0))
    _lib.check(_lib.lib().mms_plan(int(n), flags, p))
    return p


def workspace_bytes(n: int, pairs: bool = False, keys64: bool = False) -> int:
    flags = (MMS_PAIRS if pairs else 0) | (MMS_KEYS64 if keys64 else 0)
    return int(_lib.lib().mms_workspace_bytes(int(n), flags))


def _workspace(n, pairs, device, workspace, keys64=False):
    torch = _torch()
    need = workspace_bytes(n, pairs, keys64)
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < need:
            raise ValueError(f"workspace needs {need} bytes")
        return workspace, need
    if need == 0:
        return None, 0
    return torch.empty(need, dtype=torch.uint8, device=device), need


def sort(keys, out=None, i32: bool | None = None, workspace=None, stream=None):
    """Sort a 1-D int32/uint32 device tensor ascending; returns ``out``.

    int32 tensors sort in signed order, uint32 in unsigned order, unless
    ``i32`` says otherwise.  ``out`` may be ``keys`` itself (in place).
    """
    torch = _torch()
    _check_u32(keys, "keys")
    if i32 is None:
        i32 = keys.dtype == torch.int32
    n = keys.numel()
    if out is None:
        out = torch.empty_like(keys)
    _check_u32(out, "out")
    if out.numel() != n:
        raise ValueError("out has the wrong size")
    ws, need = _workspace(n, False, keys.device, workspace)
    _lib.check(_lib.lib().mms_sort_u32(keys.data_ptr(), out.data_ptr(), n,
                                       ws.data_ptr() if ws is not None else None, need,
                                       MMS_KEY_I32 if i32 else 0, _stream_ptr(stream)))
    return out


def sort_pairs(keys, values, out_keys=None, out_values=None, i32: bool | None = None,
               workspace=None, stream=None):
    """Stable sort of (key, value) pairs by key; returns (out_keys, out_values)."""
    torch = _torch()
    _check_u32(keys, "keys")
    _check_u32(values, "values")
    if i32 is None:
        i32 = keys.dtype == torch.int32
    n = keys.numel()
    if values.numel() != n:
        raise ValueError("keys and values differ in size")
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if out_values is None:
        out_values = torch.empty_like(values)
    ws, need = _workspace(n, True, keys.device, workspace)
    _lib.check(_lib.lib().mms_sort_pairs_u32(
        keys.data_ptr(), values.data_ptr(), out_keys.data_ptr(), out_values.data_ptr(), n,
        ws.data_ptr() if ws is not None else None, need, MMS_KEY_I32 if i32 else 0,
        _stream_ptr(stream)))
    return out_keys, out_values


def sort_mergepath(keys, out=None, i32: bool | None = None, workspace=None, stream=None):
    """The merge-path baseline (pairwise, per-thread serial merges): sorts a
    1-D int32/uint32 device tensor ascending like :func:`sort`."""
    torch = _torch()
    _check_u32(keys, "keys")
    if i32 is None:
        i32 = keys.dtype == torch.int32
    n = keys.numel()
    if out is None:
        out = torch.empty_like(keys)
    _check_u32(out, "out")
    if out.numel() != n:
        raise ValueError("out has the wrong size")
    need = int(_lib.lib().mms_workspace_bytes(n, MMS_MERGEPATH))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)
    elif workspace.numel() * workspace.element_size() < need:
        raise ValueError(f"workspace needs {need} bytes")
    _lib.check(_lib.lib().mms_sort_mergepath_u32(keys.data_ptr(), out.data_ptr(), n, workspace.data_ptr(), need,
                                                 MMS_KEY_I32 if i32 else 0, _stream_ptr(stream)))
    return out


def _check_u64(t, name):
    torch = _torch()
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype not in (torch.int64, torch.uint64):
        raise ValueError(f"{name} must be int64/uint64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def sort64(keys, out=None, i64: bool | None = None, workspace=None, stream=None):
    """Sort a 1-D int64/uint64 device tensor ascending; returns ``out``.

    int64 tensors sort in signed order, uint64 in unsigned order, unless
    ``i64`` says otherwise.  ``out`` may be ``keys`` itself (in place).
    """
    torch = _torch()
    _check_u64(keys, "keys")
    if i64 is None:
        i64 = keys.dtype == torch.int64
    n = keys.numel()
    if out is None:
        out = torch.empty_like(keys)
    _check_u64(out, "out")
    if out.numel() != n:
        raise ValueError("out has the wrong size")
    ws, need = _workspace(n, False, keys.device, workspace, keys64=True)
    _lib.check(_lib.lib().mms_sort_u64(keys.data_ptr(), out.data_ptr(), n,
                                       ws.data_ptr() if ws is not None else None, need,
                                       MMS_KEY_I64 if i64 else 0, _stream_ptr(stream)))
    return out


def sort_pairs64(keys, values, out_keys=None, out_values=None, i64: bool | None = None,
                 workspace=None, stream=None):
    """Stable sort of (64-bit key, 64-bit value) pairs by key; returns (out_keys, out_values)."""
    torch = _torch()
    _check_u64(keys, "keys")
    _check_u64(values, "values")
    if i64 is None:
        i64 = keys.dtype == torch.int64
    n = keys.numel()
    if values.numel() != n:
        raise ValueError("keys and values differ in size")
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if out_values is None:
        out_values = torch.empty_like(values)
    ws, need = _workspace(n, True, keys.device, workspace, keys64=True)
    _lib.check(_lib.lib().mms_sort_pairs_u64(
        keys.data_ptr(), values.data_ptr(), out_keys.data_ptr(), out_values.data_ptr(), n,
        ws.data_ptr() if ws is not None else None, need, MMS_KEY_I64 if i64 else 0,
        _stream_ptr(stream)))
    return out_keys, out_values


def partition(keys, run_len: int, K: int, groups, ranks, i32: bool = False, stream=None):
    """§4.1 split indices; returns a (nqueries, K) uint32 device tensor."""
    torch = _torch()
    _check_u32(keys, "keys")
    g = torch.as_tensor(groups, dtype=torch.int64, device=keys.device).contiguous()
    r = torch.as_tensor(ranks, dtype=torch.int64, device=keys.device).contiguous()
    nq = g.numel()
    out = torch.empty((nq, K), dtype=torch.int32, device=keys.device)
    _lib.check(_lib.lib().mms_partition_u32(keys.data_ptr(), keys.numel(), int(run_len), int(K),
                                            g.data_ptr(), r.data_ptr(), nq, out.data_ptr(),
                                            MMS_KEY_I32 if i32 else 0, _stream_ptr(stream)))
    return out


def copy(src, dst, stream=None):
    _check_u32(src, "src")
    _check_u32(dst, "dst")
    _lib.check(_lib.lib().mms_copy_u32(src.data_ptr(), dst.data_ptr(), src.numel(),
                                       _stream_ptr(stream)))
    return dst


def timing_enable(on: bool = True, kinds=None):
    """Bracket library kernel launches with HIP events on their streams: all
    kinds, or those named in `kinds` (names of timing_read's keys)."""
    if kinds is not None:
        mask = 0
        for k in kinds:
            mask |= 1 << _lib.KERNEL_KINDS.index(k)
        _lib.check(_lib.lib().mms_timing_kinds(mask))
    elif on:
        _lib.check(_lib.lib().mms_timing_kinds((1 << len(_lib.KERNEL_KINDS)) - 1))
    _lib.check(_lib.lib().mms_timing_enable(1 if on else 0))


def timing_reset():
    _lib.check(_lib.lib().mms_timing_reset())


def timing_read() -> dict:
    """{kind: (launches, total_ms)} since the last reset; waits for the events."""
    t = _lib.MmsTiming()
    _lib.check(_lib.lib().mms_timing_read(t))
    return {k: (int(t.launches[i]), float(t.total_ms[i])) for i, k in enumerate(_lib.KERNEL_KINDS)}


def segmented_workspace_bytes(offsets, pairs: bool = False) -> int:
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    return int(_lib.lib().mms_segmented_workspace_bytes(off.ctypes.data, off.size - 1,
                                                        MMS_PAIRS if pairs else 0))


def segmented_sort(keys, offsets, values=None, out_keys=None, out_values=None, i32: bool | None = None,
                   workspace=None, stream=None):
    """Sort every segment [offsets[s], offsets[s+1]) of a device tensor on its own.

    ``offsets`` is a host sequence of num_segs+1 non-decreasing element
    offsets.  With ``values`` the sort is stable by key.  Returns ``out_keys``
    (and ``out_values``).  The batch runs as one hipGraph launch per call once
    the offsets and buffers repeat.
    """
    import numpy as np
    torch = _torch()
    _check_u32(keys, "keys")
    if i32 is None:
        i32 = keys.dtype == torch.int32
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    if off.ndim != 1 or off.size < 1:
        raise ValueError("offsets must hold num_segs + 1 entries")
    if int(off[-1]) > keys.numel():
        raise ValueError("offsets exceed the keys tensor")
    pairs = values is not None
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if pairs:
        _check_u32(values, "values")
        if out_values is None:
            out_values = torch.empty_like(values)
    need = segmented_workspace_bytes(off, pairs)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)
    elif workspace.numel() * workspace.element_size() < need:
        raise ValueError(f"workspace needs {need} bytes")
    _lib.check(_lib.lib().mms_segmented_sort(
        keys.data_ptr(), out_keys.data_ptr(), values.data_ptr() if pairs else None,
        out_values.data_ptr() if pairs else None, off.ctypes.data, off.size - 1,
        workspace.data_ptr(), need, MMS_KEY_I32 if i32 else 0, _stream_ptr(stream)))
    return (out_keys, out_values) if pairs else out_keys


def set_tuning(entries):
    """Install a tuning table: iterable of (max_log2_n, fanout, merge_tile,
    variant[, base[, flags]]), flags MMS_PAIRS for key-value entries."""
    entries = list(entries)
    arr = (_lib.MmsTuning * max(1, len(entries)))()
    for i, e in enumerate(entries):
        l2, k, t, v = e[:4]
        arr[i] = _lib.MmsTuning(int(l2), int(k), int(t), int(v), int(e[4]) if len(e) > 4 else 0,
                                int(e[5]) if len(e) > 5 else 0)
    _lib.check(_lib.lib().mms_set_tuning(arr, len(entries)))


def get_tuning(n: int, pairs: bool = False):
    t = _lib.MmsTuning()
    _lib.check(_lib.lib().mms_get_tuning(int(n), MMS_PAIRS if pairs else 0, t))
    return (t.max_log2_n, t.fanout, t.merge_tile, t.variant, t.base)
