"""The C ABI on the CPU: the library loads, exports what include/mms.h
declares, plans as §6.2 prescribes, and rejects bad arguments before any
device work (no GPU is touched by these tests)."""
import ctypes
import math
import os
import re

import pytest

from paper_1702_07961_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mms.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1702_07961_amd import build
        build.build()
    lib = _lib.lib()
    lib.mms_set_tuning(None, 0)     # the built-in default, whatever table was loaded
    yield lib
    _lib.load_tuning(lib)


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mms_[a-z0-9_]+)\s*\(", text)))


def test_header_matches_binding_list():
    assert header_functions() == sorted(_lib.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def test_version_and_error_string(lib):
    assert lib.mms_version() >= 100
    assert isinstance(lib.mms_last_error(), bytes)


def expected_rounds(n, T, K):
    """§6.2: ceil(log_K(ceil(n/T))) merge rounds, computed with integers."""
    runs = -(-n // T)
    r = 0
    while runs > 1:
        runs = -(-runs // K)
        r += 1
    return r


@pytest.mark.parametrize("pairs", [False, True])
def test_plan_pass_count(lib, pairs):
    p0 = _lib.MmsPlan()
    assert lib.mms_plan(1, _lib.MMS_PAIRS if pairs else 0, p0) == 0
    T, K = p0.tile, p0.fanout
    assert T == 64 * 8 * 4 and K == 16
    for n in [1, 2, T - 1, T, T + 1, T * K, T * K + 1, T * K * K, T * K * K + 7, 10**8, 2**27, 2**32 - 1]:
        p = _lib.MmsPlan()
        assert lib.mms_plan(n, _lib.MMS_PAIRS if pairs else 0, p) == 0
        assert p.rounds == expected_rounds(n, T, K), n
        assert p.passes == 1 + p.rounds
        # ceil(log_K(ceil(n/T))) by floating point, away from exact powers
        if n > T and math.log(-(-n // T), K) % 1 > 1e-9:
            assert p.rounds == math.ceil(math.log(-(-n // T), K))
        ws = lib.mms_workspace_bytes(n, _lib.MMS_PAIRS if pairs else 0)
        assert ws == p.workspace_bytes
        if p.rounds:
            assert ws >= n * 4 * (2 if pairs else 1)
        else:
            assert ws == 0


def test_plan_headline_size(lib):
    p = _lib.MmsPlan()
    assert lib.mms_plan(10**8, 0, p) == 0
    assert (p.rounds, p.passes) == (4, 5)


def test_plan_rejects(lib):
    p = _lib.MmsPlan()
    assert lib.mms_plan(1 << 32, 0, p) == _lib.MMS_EINVAL
    assert b"2^32" in lib.mms_last_error()
    assert lib.mms_plan(5, 0x80, p) == _lib.MMS_EINVAL
    assert lib.mms_plan(5, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_workspace_bytes(0, 0) == 0


FAKE = 0x7F0000000000   # never dereferenced: every call below fails its checks first


def test_sort_argument_errors(lib):
    n = 100_000
    ws = lib.mms_workspace_bytes(n, 0)
    assert lib.mms_sort_u32(FAKE, FAKE + 4, n, FAKE + 2**30, ws, 0, None) == _lib.MMS_EINVAL
    assert b"overlap" in lib.mms_last_error()
    assert lib.mms_sort_u32(None, FAKE, n, FAKE + 2**30, ws, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_sort_u32(FAKE, FAKE + 2**28, 1 << 32, FAKE + 2**30, ws, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_sort_u32(FAKE, FAKE + 2**28, n, FAKE + 2**30, ws - 1, 0, None) == _lib.MMS_EINVAL
    assert b"too small" in lib.mms_last_error()
    assert lib.mms_sort_u32(FAKE, FAKE + 2**28, n, FAKE + 2**30 + 4, ws, 0, None) == _lib.MMS_EINVAL
    assert b"aligned" in lib.mms_last_error()
    assert lib.mms_sort_u32(FAKE, FAKE + 2**28, n, FAKE + 2**28, ws, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_sort_u32(FAKE, FAKE + 2**28, n, None, 0, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_sort_u32(FAKE, FAKE + 2**28, n, FAKE + 2**30, ws, 0x40, None) == _lib.MMS_EINVAL
    assert lib.mms_sort_u32(FAKE, FAKE + 2**28, n, FAKE + 2**30, ws, _lib.MMS_PAIRS, None) == _lib.MMS_EINVAL
    assert lib.mms_sort_u32(FAKE, FAKE, 0, None, 0, 0, None) == _lib.MMS_OK


def test_noalloc_argument_errors(lib):
    """Rejections of the no-workspace sort happen before any device call."""
    limit = 64 << 20
    big = 1
    while lib.mms_workspace_bytes(big, 0) <= limit:
        big *= 2
    assert lib.mms_sort_u32_noalloc(FAKE, FAKE + 2**34, big, 0, None) == _lib.MMS_EINVAL
    assert b"scratch" in lib.mms_last_error()
    assert lib.mms_sort_u32_noalloc(FAKE, FAKE + 2**34, 1 << 32, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_sort_u32_noalloc(FAKE, FAKE + 2**34, 1000, _lib.MMS_PAIRS, None) == _lib.MMS_EINVAL
    assert lib.mms_sort_u32_noalloc(FAKE, FAKE, 0, 0, None) == _lib.MMS_OK


def test_pairs_argument_errors(lib):
    n = 100_000
    ws = lib.mms_workspace_bytes(n, _lib.MMS_PAIRS)
    K, V, KO, VO, W = FAKE, FAKE + 2**26, FAKE + 2**27, FAKE + 3 * 2**26, FAKE + 2**30
    assert lib.mms_sort_pairs_u32(K, V, KO, VO, n, W, ws - 256, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_sort_pairs_u32(K, None, KO, VO, n, W, ws, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_sort_pairs_u32(K, K + 8, KO, VO, n, W, ws, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_sort_pairs_u32(K, V, KO, KO, n, W, ws, 0, None) == _lib.MMS_EINVAL


def test_partition_argument_errors(lib):
    assert lib.mms_partition_u32(FAKE, 100, 10, 0, FAKE, FAKE, 1, FAKE, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_partition_u32(FAKE, 100, 10, 17, FAKE, FAKE, 1, FAKE, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_partition_u32(FAKE, 100, 0, 4, FAKE, FAKE, 1, FAKE, 0, None) == _lib.MMS_EINVAL
    assert lib.mms_partition_u32(FAKE, 100, 10, 4, FAKE, FAKE, 0, FAKE, 0, None) == _lib.MMS_OK


def test_copy_argument_errors(lib):
    assert lib.mms_copy_u32(FAKE, FAKE + 8, 100, None) == _lib.MMS_EINVAL
    assert lib.mms_copy_u32(FAKE, FAKE, 0, None) == _lib.MMS_OK


def test_timing_kinds(lib):
    """The timed kernel kinds are a bit mask over the known kinds; a mask that
    selects none of them is an argument error."""
    all_kinds = (1 << len(_lib.KERNEL_KINDS)) - 1
    assert lib.mms_timing_kinds(0) == _lib.MMS_EINVAL
    assert lib.mms_timing_kinds(1 << len(_lib.KERNEL_KINDS)) == _lib.MMS_EINVAL
    assert lib.mms_timing_kinds(all_kinds | (1 << 31)) == _lib.MMS_EINVAL
    assert lib.mms_timing_kinds(1 << _lib.KERNEL_KINDS.index("merge")) == _lib.MMS_OK
    assert lib.mms_timing_kinds(all_kinds) == _lib.MMS_OK


def test_last_error_is_per_thread(lib):
    import threading
    lib.mms_plan(1 << 33, 0, _lib.MmsPlan())
    seen = {}

    def other():
        seen["msg"] = lib.mms_last_error()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["msg"] == b""
    assert lib.mms_last_error() != b""


def test_segmented_workspace_and_errors(lib):
    import numpy as np
    off = np.array([0, 10, 10, 5000, 100_000], dtype=np.uint64)
    ws = lib.mms_segmented_workspace_bytes(off.ctypes.data, 4, 0)
    wsp = lib.mms_segmented_workspace_bytes(off.ctypes.data, 4, _lib.MMS_PAIRS)
    assert ws >= 100_000 * 4 and wsp >= 2 * 100_000 * 4
    bad = np.array([0, 10, 5], dtype=np.uint64)
    assert lib.mms_segmented_workspace_bytes(bad.ctypes.data, 2, 0) == 0
    # decreasing offsets are rejected before any device work
    assert lib.mms_segmented_sort(FAKE, FAKE + 2**28, None, None, bad.ctypes.data, 2,
                                  FAKE + 2**30, 1 << 20, 0, None) == _lib.MMS_EINVAL
    assert b"decrease" in lib.mms_last_error()
    # values need both sides
    assert lib.mms_segmented_sort(FAKE, FAKE + 2**28, FAKE + 2**29, None, off.ctypes.data, 4,
                                  FAKE + 2**30, 1 << 30, 0, None) == _lib.MMS_EINVAL
    # zero segments is a no-op
    assert lib.mms_segmented_sort(FAKE, FAKE, None, None, off.ctypes.data, 0, None, 0, 0, None) == 0


def test_tuning_table(lib):
    t = _lib.MmsTuning()
    assert lib.mms_get_tuning(10**8, 0, t) == 0
    default = (t.fanout, t.merge_tile, t.variant)
    table = (_lib.MmsTuning * 2)(_lib.MmsTuning(20, 8, 4096, 1), _lib.MmsTuning(32, 16, 7168, 2))
    assert lib.mms_set_tuning(table, 2) == 0
    assert lib.mms_get_tuning(1 << 18, 0, t) == 0 and (t.fanout, t.merge_tile, t.variant) == (8, 4096, 1)
    assert lib.mms_get_tuning(10**8, 0, t) == 0 and (t.fanout, t.merge_tile, t.variant) == (16, 7168, 2)
    p = _lib.MmsPlan()
    lib.mms_plan(1 << 18, 0, p)
    assert p.fanout == 8 and p.rounds == expected_rounds(1 << 18, 2048, 8)
    bad = (_lib.MmsTuning * 1)(_lib.MmsTuning(20, 3, 4096, 0))
    assert lib.mms_set_tuning(bad, 1) == _lib.MMS_EINVAL
    bad = (_lib.MmsTuning * 1)(_lib.MmsTuning(20, 8, 4096, 0, 7))     # no base-case shape 7
    assert lib.mms_set_tuning(bad, 1) == _lib.MMS_EINVAL
    shaped = (_lib.MmsTuning * 1)(_lib.MmsTuning(32, 8, 4096, 1, 2))
    assert lib.mms_set_tuning(shaped, 1) == 0
    assert lib.mms_get_tuning(1 << 20, 0, t) == 0 and (t.fanout, t.base) == (8, 2)
    p = _lib.MmsPlan()
    assert lib.mms_plan(1 << 20, 0, p) == 0 and p.lanes_per_tile == 128      # 16 keys x 2 waves
    assert lib.mms_plan(1 << 20, _lib.MMS_PAIRS, p) == 0 and p.lanes_per_tile == 256
    big = (_lib.MmsTuning * 1)(_lib.MmsTuning(32, 16, 7168, 3, 4))      # 8 x 16: 8192-key tiles
    assert lib.mms_set_tuning(big, 1) == 0
    assert lib.mms_plan(10**8, 0, p) == 0
    assert (p.tile, p.lanes_per_tile, p.rounds) == (8192, 1024, 4)       # 12208 runs: 16^3 < 12208
    assert lib.mms_plan(8192, 0, p) == 0 and p.rounds == 0
    assert lib.mms_plan(8193, 0, p) == 0 and p.rounds == 1
    assert lib.mms_plan(10**8, _lib.MMS_PAIRS, p) == 0 and (p.tile, p.lanes_per_tile) == (4096, 512)   # 8 x 8
    kinds = (_lib.MmsTuning * 3)(_lib.MmsTuning(32, 16, 7168, 3, 4, 0),
                                 _lib.MmsTuning(20, 4, 4096, 0, 0, _lib.MMS_PAIRS),
                                 _lib.MmsTuning(32, 8, 4096, 0, 3, _lib.MMS_PAIRS))
    assert lib.mms_set_tuning(kinds, 3) == 0                              # entries of both kinds
    assert lib.mms_get_tuning(10**8, 0, t) == 0 and (t.fanout, t.base, t.flags) == (16, 4, 0)
    assert lib.mms_get_tuning(1 << 18, _lib.MMS_PAIRS, t) == 0 and (t.fanout, t.base) == (4, 0)
    assert lib.mms_get_tuning(10**8, _lib.MMS_PAIRS, t) == 0 and (t.fanout, t.base, t.flags) == (8, 3, 1)
    assert lib.mms_plan(10**8, _lib.MMS_PAIRS, p) == 0 and (p.fanout, p.tile) == (8, 4096)
    bad = (_lib.MmsTuning * 1)(_lib.MmsTuning(32, 16, 7168, 3, 4, 2))   # unknown kind flag
    assert lib.mms_set_tuning(bad, 1) == _lib.MMS_EINVAL
    wide = (_lib.MmsTuning * 1)(_lib.MmsTuning(32, 16, 7168, 3, 6))     # 16 x 8: keys only
    assert lib.mms_set_tuning(wide, 1) == 0
    assert lib.mms_plan(10**8, 0, p) == 0 and p.tile == 8192
    assert lib.mms_plan(10**8, _lib.MMS_PAIRS, p) == 0 and (p.tile, p.lanes_per_tile) == (2048, 256)
    assert lib.mms_set_tuning(None, 0) == 0
    assert lib.mms_get_tuning(10**8, 0, t) == 0 and (t.fanout, t.merge_tile, t.variant) == default
