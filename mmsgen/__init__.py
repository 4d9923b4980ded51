"""Seeded synthetic inputs for the multiway mergesort workloads.

The recipes live in ``gen.c`` (splitmix64 plus Lemire's bounded draw); this
module only marshals arrays.  It contains none of the sort's arithmetic and is
the one module that both the GPU tests and the oracle tests draw inputs from.

Seeds follow one convention: workload ``c``'s trial ``t`` uses
``SEED_BASE + 16 * c + t``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libmmsgen.so")

SEED_BASE = 0x4D4D5300

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_f64p = ctypes.POINTER(ctypes.c_double)


def seed_for(workload: int, trial: int = 0) -> int:
    return SEED_BASE + 16 * workload + trial


def build(src: str = _SRC, out: str = _LIB) -> str:
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", src,
                           "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


_lib = None


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        for name, args in [
            ("mmsgen_splitmix64", [ctypes.c_uint64, _u64p, ctypes.c_uint64]),
            ("mmsgen_uniform_u32", [ctypes.c_uint64, _u32p, ctypes.c_uint64]),
            ("mmsgen_nearly_sorted_u32", [ctypes.c_uint64, _u32p, ctypes.c_uint64, ctypes.c_uint64]),
            ("mmsgen_sixteen_u32", [ctypes.c_uint64, _u32p, ctypes.c_uint64]),
            ("mmsgen_stride64_u32", [_u32p, ctypes.c_uint64]),
            ("mmsgen_permutation_u32", [ctypes.c_uint64, _u32p, ctypes.c_uint64]),
            ("mmsgen_iota_u32", [_u32p, ctypes.c_uint64]),
            ("mmsgen_loguniform_sizes", [ctypes.c_uint64, _u64p, ctypes.c_uint64,
                                         ctypes.c_double, ctypes.c_double]),
            ("mmsgen_unit_doubles", [ctypes.c_uint64, _f64p, ctypes.c_uint64]),
            ("mmsgen_mergepath_adversary_u32", [_u32p, _u32p, ctypes.c_uint64, ctypes.c_uint64]),
        ]:
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int if name in ("mmsgen_stride64_u32", "mmsgen_mergepath_adversary_u32") else None
        _lib = lib
    return _lib


def _empty32(n):
    return np.empty(int(n), dtype=np.uint32)


def splitmix64(seed: int, n: int) -> np.ndarray:
    out = np.empty(int(n), dtype=np.uint64)
    _get().mmsgen_splitmix64(seed, out.ctypes.data_as(_u64p), out.size)
    return out


def uniform_u32(seed: int, n: int) -> np.ndarray:
    out = _empty32(n)
    _get().mmsgen_uniform_u32(seed, out.ctypes.data_as(_u32p), out.size)
    return out


def nearly_sorted_u32(seed: int, n: int, swaps: int) -> np.ndarray:
    if n > 1 << 32:
        raise ValueError("n must fit 32-bit keys")
    out = _empty32(n)
    _get().mmsgen_nearly_sorted_u32(seed, out.ctypes.data_as(_u32p), out.size, int(swaps))
    return out


def sixteen_u32(seed: int, n: int) -> np.ndarray:
    out = _empty32(n)
    _get().mmsgen_sixteen_u32(seed, out.ctypes.data_as(_u32p), out.size)
    return out


def stride64_u32(n: int) -> np.ndarray:
    out = _empty32(n)
    if _get().mmsgen_stride64_u32(out.ctypes.data_as(_u32p), out.size):
        raise ValueError("stride-64 family needs n divisible by 64")
    return out


def permutation_u32(seed: int, n: int) -> np.ndarray:
    out = _empty32(n)
    _get().mmsgen_permutation_u32(seed, out.ctypes.data_as(_u32p), out.size)
    return out


def iota_u32(n: int) -> np.ndarray:
    out = _empty32(n)
    _get().mmsgen_iota_u32(out.ctypes.data_as(_u32p), out.size)
    return out


def loguniform_sizes(seed: int, count: int, lo_exp: float, hi_exp: float) -> np.ndarray:
    out = np.empty(int(count), dtype=np.uint64)
    _get().mmsgen_loguniform_sizes(seed, out.ctypes.data_as(_u64p), out.size,
                                   float(lo_exp), float(hi_exp))
    return out


def unit_doubles(seed: int, count: int) -> np.ndarray:
    out = np.empty(int(count), dtype=np.float64)
    _get().mmsgen_unit_doubles(seed, out.ctypes.data_as(_f64p), out.size)
    return out


def poisson_arrivals(seed: int, count: int, rate: float) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process: exponential gaps -ln(1-u)/rate."""
    u = unit_doubles(seed, count)
    return np.cumsum(-np.log1p(-u) / rate)


MERGEPATH_ITEMS = 15     # outputs per thread of the merge-path baseline


def mergepath_adversary_u32(n: int, vt: int = MERGEPATH_ITEMS) -> np.ndarray:
    """Conflict-heavy permutation of 0..n-1 against a merge-path sort whose
    threads merge vt outputs each (n = vt * 2^k); recipe in gen.c."""
    out = _empty32(n)
    tmp = _empty32(n)
    if _get().mmsgen_mergepath_adversary_u32(out.ctypes.data_as(_u32p), tmp.ctypes.data_as(_u32p), out.size, vt):
        raise ValueError("the merge-path adversary needs n = vt * 2^k")
    return out


def family(name: str, seed: int, n: int, swaps: int = 0) -> np.ndarray:
    """Keys of one named input family."""
    if name == "uniform":
        return uniform_u32(seed, n)
    if name == "nearly":
        return nearly_sorted_u32(seed, n, swaps)
    if name == "sixteen":
        return sixteen_u32(seed, n)
    if name == "stride64":
        return stride64_u32(n)
    if name == "permutation":
        return permutation_u32(seed, n)
    if name == "sorted":
        return iota_u32(n)
    if name == "reverse":
        return iota_u32(n)[::-1].copy()
    if name == "equal":
        return np.full(int(n), 0x5A5A5A5A, dtype=np.uint32)
    if name == "mp_adversary":
        return mergepath_adversary_u32(n)
    raise ValueError(f"unknown family {name!r}")


def loguniform_mean(lo_exp: float, hi_exp: float) -> float:
    """Mean of 2^(lo + (hi-lo) u), u uniform: (2^hi - 2^lo) / ((hi-lo) ln 2)."""
    return (2.0 ** hi_exp - 2.0 ** lo_exp) / ((hi_exp - lo_exp) * math.log(2.0))
