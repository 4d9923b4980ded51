"""The oracle's pins catch plausible mistakes.

Each mutant is the oracle source with one plausible slip planted in it (a
flipped tie-break, a dropped run, an unsigned compare, an off-by-one in the
heap or in counting, values left behind).  It is compiled to a temporary
library on the CPU and run through a battery of the pins from
test_oracle.py; every mutant must fail at least one of them.
"""
import itertools
import os

import numpy as np
import pytest

import mmsgen
import oracle
from golden_io import partition_cases, sort_cases, sort_cases_u64

with open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")) as _f:
    SOURCE = _f.read()

MUTANTS = {
    "tie_break_reversed": ("return a.run < b.run;", "return a.run > b.run;"),
    "last_run_dropped": ("nruns = j + 1;", "nruns = j;"),
    "signed_as_unsigned": ("if (i32) return (int32_t)a < (int32_t)b;", "if (i32) return a < b;"),
    "heap_right_child_skipped": ("if (r < h->size && hnode_less", "if (r < h->size - 1 && hnode_less"),
    "values_left_behind": ("if (dst_v) dst_v[out] = src_v[next[j]];", "if (dst_v) dst_v[out] = src_v[out];"),
    "groups_overlap": ("g += len * ORACLE_FANOUT)", "g += len * (ORACLE_FANOUT - 1))"),
    "partition_short_by_one": ("for (uint64_t t = 0; t < r; ++t)", "for (uint64_t t = 0; t + 1 < r; ++t)"),
    "select_off_by_one": ("while (below + cnt[lo] <= i)", "while (below + cnt[lo] < i)"),
    "select_wrong_occurrence": ("uint64_t want = i - below;", "uint64_t want = 0;"),
    # the 64-bit sort
    "u64_low_half_only": ("if (i64) return (int64_t)a < (int64_t)b;\n    return a < b;",
                          "if (i64) return (int64_t)a < (int64_t)b;\n    return (uint32_t)a < (uint32_t)b;"),
    "u64_signed_as_unsigned": ("if (i64) return (int64_t)a < (int64_t)b;", "if (i64) return a < b;"),
    "u64_tie_break_reversed": ("if (key64_less(b.key, a.key, i64)) return 0;\n    return a.run < b.run;",
                               "if (key64_less(b.key, a.key, i64)) return 0;\n    return a.run > b.run;"),
    "u64_values_left_behind": ("heap64_pop(&h);\n        int j = (int)x.run;\n        dst_k[out] = src_k[next[j]];\n"
                               "        if (dst_v) dst_v[out] = src_v[next[j]];",
                               "heap64_pop(&h);\n        int j = (int)x.run;\n        dst_k[out] = src_k[next[j]];\n"
                               "        if (dst_v) dst_v[out] = src_v[out];"),
    "u64_last_run_dropped": ("nruns = j + 1;\n            merge_runs64", "nruns = j;\n            merge_runs64"),
    "u64_key_truncated_in_heap": ("hnode64_t x = { src_k[next[j]], (uint32_t)j };",
                                  "hnode64_t x = { (uint32_t)src_k[next[j]], (uint32_t)j };"),
}


def _battery(lib):
    """Return the list of pin names that fail for this library."""
    failed = []
    for name, i32, keys, out, idx in sort_cases():
        k, v = oracle.sort(keys, np.arange(keys.size, dtype=np.uint32), i32=i32, lib=lib)
        if k.tolist() != out.tolist() or v.tolist() != idx.tolist():
            failed.append("hand:" + name)
    keys, offs, splits = partition_cases()
    for r, want in splits:
        if oracle.partition(keys, offs, r, lib=lib).tolist() != want:
            failed.append(f"partition:r={r}")
            break
    for n in range(1, 7):
        for p in itertools.permutations(range(n)):
            k, v = oracle.sort(np.array(p, np.uint32), np.arange(n, dtype=np.uint32), lib=lib)
            inv = np.empty(n, np.uint32)
            inv[list(p)] = np.arange(n, dtype=np.uint32)
            if k.tolist() != list(range(n)) or not np.array_equal(v, inv):
                failed.append(f"perm:{p}")
                break
    for n in [30, 1000]:
        x = mmsgen.sixteen_u32(5, n)
        k, v = oracle.sort(x, np.arange(n, dtype=np.uint32), lib=lib)
        perm = np.argsort(x, kind="stable").astype(np.uint32)
        if not np.array_equal(v, perm):
            failed.append(f"stable:{n}")
    x = mmsgen.uniform_u32(3, 2000)
    perm = np.argsort(x.view(np.int32), kind="stable")
    k, v = oracle.sort(x, np.arange(x.size, dtype=np.uint32), i32=True, lib=lib)
    if not np.array_equal(v, perm.astype(np.uint32)):
        failed.append("signed")
    for x in (mmsgen.sixteen_u32(7, 3001), mmsgen.uniform_u32(8, 200) % np.uint32(8)):
        perm = np.argsort(x, kind="stable")
        for i in range(0, x.size, max(1, x.size // 200)):
            try:
                got = oracle.select(x, i, lib=lib)
            except RuntimeError:
                got = None
            if got != (int(x[perm[i]]), int(perm[i])):
                failed.append(f"select:{i}")
                break
    return failed


def _battery64(lib):
    """Pins of the 64-bit sort (test_oracle_u64.py) that a mutant must fail."""
    failed = []
    for name, i64, keys, out, idx in sort_cases_u64():
        k, v = oracle.sort_u64(keys, np.arange(keys.size, dtype=np.uint64), i64=i64, lib=lib)
        if k.tolist() != out.tolist() or v.tolist() != idx.tolist():
            failed.append("hand64:" + name)
    for n in range(1, 7):
        for p in itertools.permutations(range(n)):
            keys = np.array([(t << 32) | (~t & 0xFFFFFFFF) for t in p], dtype=np.uint64)
            k, v = oracle.sort_u64(keys, np.arange(n, dtype=np.uint64), lib=lib)
            inv = np.empty(n, np.uint64)
            inv[list(p)] = np.arange(n, dtype=np.uint64)
            if not np.array_equal(k, np.sort(keys)) or not np.array_equal(v, inv):
                failed.append(f"perm64:{p}")
                break
    x = mmsgen.splitmix64(11, 3000) >> np.uint64(52)
    for i64 in (False, True):
        perm = np.argsort(x.view(np.int64) if i64 else x, kind="stable").astype(np.uint64)
        k, v = oracle.sort_u64(x, np.arange(x.size, dtype=np.uint64), i64=i64, lib=lib)
        if not np.array_equal(v, perm):
            failed.append(f"stable64:{i64}")
    return failed


def test_unmutated_oracle_passes_battery():
    assert _battery(oracle._get()) == []
    assert _battery64(oracle._get()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    # the 64-bit sort repeats some lines of the 32-bit one: a 32-bit site is
    # its first occurrence, which lies before the 64-bit section; a 64-bit
    # site is unique
    at = SOURCE.find(old)
    assert at >= 0, f"mutation site for {name} not found"
    if name.startswith("u64_"):
        assert SOURCE.count(old) == 1, f"mutation site for {name} not unique"
    else:
        assert at < SOURCE.index("#define ORACLE_KEY_I64"), f"mutation site for {name} not in the 32-bit code"
    src = tmp_path / "oracle_mut.c"
    src.write_text(SOURCE[:at] + new + SOURCE[at + len(old):])
    lib = oracle.load(oracle.build(str(src), str(tmp_path / "liboracle_mut.so")))
    assert _battery(lib) + _battery64(lib), f"mutant {name} survived every pin"
