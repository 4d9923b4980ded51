"""CPU oracle for the multiway mergesort — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct sequential heap-based K-way mergesort
(§4 of Casanova et al., arXiv 1702.07961: K lists merged per round, the
merge done with a min-heap and an output buffer), plus brute-force
definitions of the §4.1 partition and of the i-th sorted element.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never loads it, and it
shares no code with the GPU path.  The C source is ``oracle.c``; ``build()``
compiles it with gcc into ``liboracle.so`` next to this file.

``cpu_parallel.cpp`` (``parallel_sort*`` below) is not part of the oracle: it
is a multi-core CPU sort (libstdc++ parallel mode) that the benchmark's
CPU-baseline leg times as context beside the oracle; no check relies on it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KEY_I32 = 1

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


_PAR_SRC = os.path.join(_HERE, "cpu_parallel.cpp")
_PAR_LIB = os.path.join(_HERE, "libcpuparallel.so")


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (no vector intrinsics, plain C); when
    building the default library, also the multi-core context sort."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared",
                           "-fPIC", src, "-o", tmp])
    os.replace(tmp, out)
    if src == _SRC:
        build_parallel()
    return out


def build_parallel() -> str:
    tmp = _PAR_LIB + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-Wall", "-shared", "-fPIC",
                           _PAR_SRC, "-o", tmp])
    os.replace(tmp, _PAR_LIB)
    return _PAR_LIB


_par = None


def _get_parallel():
    global _par
    if _par is None:
        if not os.path.exists(_PAR_LIB):
            build_parallel()
        lib = ctypes.CDLL(_PAR_LIB)
        lib.cpu_parallel_threads.restype = ctypes.c_int
        lib.cpu_parallel_sort_u32.argtypes = [_u32p, ctypes.c_uint64, ctypes.c_uint32]
        lib.cpu_parallel_sort_pairs_u32.argtypes = [_u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32]
        lib.cpu_parallel_sort_u64.argtypes = [_u64p, ctypes.c_uint64]
        _par = lib
    return _par


def parallel_threads() -> int:
    """OpenMP threads the multi-core context sort runs on."""
    return int(_get_parallel().cpu_parallel_threads())


def parallel_sort(keys, vals=None, i32: bool = False):
    """Multi-core context sort (not the oracle): sorts copies, returns them."""
    lib = _get_parallel()
    if keys.dtype == np.uint64:
        k = np.array(keys, dtype=np.uint64, copy=True)
        lib.cpu_parallel_sort_u64(_p64(k), k.size)
        return k
    k = np.array(keys, dtype=np.uint32, copy=True)
    if vals is None:
        lib.cpu_parallel_sort_u32(_p32(k), k.size, KEY_I32 if i32 else 0)
        return k
    v = np.array(vals, dtype=np.uint32, copy=True)
    lib.cpu_parallel_sort_pairs_u32(_p32(k), _p32(v), k.size, KEY_I32 if i32 else 0)
    return k, v


_lib = None


def load(path: str = _LIB) -> ctypes.CDLL:
    lib = ctypes.CDLL(path)
    lib.oracle_sort.argtypes = [_u32p, _u32p, _u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32]
    lib.oracle_sort.restype = ctypes.c_int
    lib.oracle_sort_segments.argtypes = [_u32p, _u32p, _u32p, _u32p, _u64p,
                                         ctypes.c_uint64, ctypes.c_uint32]
    lib.oracle_sort_segments.restype = ctypes.c_int
    lib.oracle_partition.argtypes = [_u32p, _u64p, ctypes.c_uint32, ctypes.c_uint64,
                                     ctypes.c_uint32, _u64p]
    lib.oracle_partition.restype = ctypes.c_int
    lib.oracle_select.argtypes = [_u32p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                  _u32p, _u64p]
    lib.oracle_select.restype = ctypes.c_int
    lib.oracle_sort_u64.argtypes = [_u64p, _u64p, _u64p, _u64p, ctypes.c_uint64, ctypes.c_uint32]
    lib.oracle_sort_u64.restype = ctypes.c_int
    return lib


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = load()
    return _lib


def _p32(a):
    return None if a is None else a.ctypes.data_as(_u32p)


def _p64(a):
    return a.ctypes.data_as(_u64p)


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def sort(keys, vals=None, i32: bool = False, lib=None):
    """Stable ascending sort; returns keys (and values when given)."""
    lib = lib or _get()
    k = _u32(keys)
    ok = np.empty_like(k)
    v = ov = None
    if vals is not None:
        v = _u32(vals)
        assert v.shape == k.shape
        ov = np.empty_like(v)
    rc = lib.oracle_sort(_p32(k), _p32(v), _p32(ok), _p32(ov), k.size, KEY_I32 if i32 else 0)
    if rc:
        raise RuntimeError(f"oracle_sort failed: {rc}")
    return ok if vals is None else (ok, ov)


KEY_I64 = 2


def sort_u64(keys, vals=None, i64: bool = False, lib=None):
    """Stable ascending sort of 64-bit keys (and 64-bit values when given)."""
    lib = lib or _get()
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    ok = np.empty_like(k)
    v = ov = None
    if vals is not None:
        v = np.ascontiguousarray(vals, dtype=np.uint64)
        assert v.shape == k.shape
        ov = np.empty_like(v)
    rc = lib.oracle_sort_u64(_p64(k), None if v is None else _p64(v), _p64(ok),
                             None if ov is None else _p64(ov), k.size, KEY_I64 if i64 else 0)
    if rc:
        raise RuntimeError(f"oracle_sort_u64 failed: {rc}")
    return ok if vals is None else (ok, ov)


def sort_segments(keys, offsets, vals=None, i32: bool = False, lib=None):
    """Sort each segment [offsets[s], offsets[s+1]) on its own."""
    lib = lib or _get()
    k = _u32(keys)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    ok = np.empty_like(k)
    v = ov = None
    if vals is not None:
        v = _u32(vals)
        ov = np.empty_like(v)
    rc = lib.oracle_sort_segments(_p32(k), _p32(v), _p32(ok), _p32(ov), _p64(off),
                                  off.size - 1, KEY_I32 if i32 else 0)
    if rc:
        raise RuntimeError(f"oracle_sort_segments failed: {rc}")
    return ok if vals is None else (ok, ov)


def partition(keys, run_offsets, r: int, i32: bool = False, lib=None) -> np.ndarray:
    """§4.1 split indices c_k of K sorted runs at rank r (brute-force merge-and-count)."""
    lib = lib or _get()
    k = _u32(keys)
    off = np.ascontiguousarray(run_offsets, dtype=np.uint64)
    K = off.size - 1
    c = np.zeros(max(K, 1), dtype=np.uint64)
    rc = lib.oracle_partition(_p32(k), _p64(off), K, int(r), KEY_I32 if i32 else 0, _p64(c))
    if rc:
        raise RuntimeError(f"oracle_partition failed: {rc}")
    return c[:K]


def select(keys, i: int, i32: bool = False, lib=None):
    """(key, input index) of the element at position i of the stable sorted order."""
    lib = lib or _get()
    k = _u32(keys)
    ko = ctypes.c_uint32()
    io = ctypes.c_uint64()
    rc = lib.oracle_select(_p32(k), k.size, int(i), KEY_I32 if i32 else 0,
                           ctypes.byref(ko), ctypes.byref(io))
    if rc:
        raise RuntimeError(f"oracle_select failed: {rc}")
    return ko.value, io.value
