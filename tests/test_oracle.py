"""Pins of the CPU oracle against facts that do not come from the oracle.

Every check compares the oracle with something the definition of sorting or
the paper fixes independently: hand-worked fixtures, closed forms of the
input families, brute force over all small inputs, invariants, and library
routines (Python's stable ``sorted``, NumPy's stable ``argsort``) for the
special case where the method's result is exactly a stable sort.
"""
import itertools
import math

import numpy as np
import pytest

import mmsgen
import oracle
from golden_io import partition_cases, sort_cases

I32_MAP = np.array([0x80000000, 0xFFFFFFFF, 0x00000000], dtype=np.uint32)


# -- hand-worked fixtures ----------------------------------------------------

@pytest.mark.parametrize("case", sort_cases(), ids=lambda c: c[0])
def test_hand_cases(case):
    name, i32, keys, out, idx = case
    k, v = oracle.sort(keys, np.arange(keys.size, dtype=np.uint32), i32=i32)
    assert k.tolist() == out.tolist()
    assert v.tolist() == idx.tolist()
    assert oracle.sort(keys, i32=i32).tolist() == out.tolist()


def test_hand_partitions():
    keys, offs, splits = partition_cases()
    for r, want in splits:
        assert oracle.partition(keys, offs, r).tolist() == want, r


# -- brute force over all small inputs ----------------------------------------

def _all_segments(inputs):
    lens = [len(x) for x in inputs]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    flat = np.array([v for x in inputs for v in x], dtype=np.uint32)
    local = np.concatenate([np.arange(n, dtype=np.uint32) for n in lens]) if lens else flat
    return flat, offs, local


def test_all_permutations_up_to_8():
    perms = [p for n in range(0, 9) for p in itertools.permutations(range(n))]
    assert len(perms) == sum(math.factorial(n) for n in range(9))
    flat, offs, local = _all_segments(perms)
    k, v = oracle.sort_segments(flat, offs, vals=local)
    for s, p in enumerate(perms):
        a, b = int(offs[s]), int(offs[s + 1])
        n = len(p)
        assert k[a:b].tolist() == list(range(n))
        inv = [0] * n
        for i, x in enumerate(p):
            inv[x] = i
        assert v[a:b].tolist() == inv


@pytest.mark.parametrize("i32", [False, True])
def test_all_ternary_up_to_7_against_stable_sorted(i32):
    seqs = [s for n in range(0, 8) for s in itertools.product(range(3), repeat=n)]
    mapped = [[int(I32_MAP[x]) for x in s] for s in seqs] if i32 else seqs
    flat, offs, local = _all_segments(mapped)
    k, v = oracle.sort_segments(flat, offs, vals=local, i32=i32)
    for s, seq in enumerate(seqs):
        a, b = int(offs[s]), int(offs[s + 1])
        # in the signed mapping 0x80000000 < 0xFFFFFFFF < 0 mirrors 0 < 1 < 2
        want = sorted(range(len(seq)), key=lambda i: (seq[i], i))
        assert v[a:b].tolist() == want
        assert k[a:b].tolist() == [mapped[s][i] for i in want]


def test_unsigned_order_of_signed_patterns():
    # the same bit patterns as unsigned: 0 < 0x80000000 < 0xFFFFFFFF
    keys = np.array([0xFFFFFFFF, 0, 0x80000000, 0, 0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    k, v = oracle.sort(keys, np.arange(6, dtype=np.uint32))
    assert v.tolist() == [1, 3, 2, 5, 0, 4]


# -- library routine for the exact special case -------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 24, 25, 26, 125, 126, 1000, 12345, 1 << 20])
def test_random_against_numpy_stable_argsort(n):
    x = mmsgen.uniform_u32(mmsgen.seed_for(0, n % 16), n)
    k, v = oracle.sort(x, np.arange(n, dtype=np.uint32))
    perm = np.argsort(x, kind="stable")
    assert np.array_equal(v, perm.astype(np.uint32))
    assert np.array_equal(k, x[perm])
    assert np.array_equal(oracle.sort(x), k)


@pytest.mark.parametrize("n", [7, 1000, 65536 + 3])
def test_signed_against_numpy(n):
    x = mmsgen.uniform_u32(mmsgen.seed_for(1, 3), n)
    k, v = oracle.sort(x, np.arange(n, dtype=np.uint32), i32=True)
    perm = np.argsort(x.view(np.int32), kind="stable")
    assert np.array_equal(v, perm.astype(np.uint32))
    assert np.array_equal(k, x[perm])


# -- invariants -----------------------------------------------------------------

def test_invariants_tie_heavy():
    n = 200_003
    x = mmsgen.sixteen_u32(mmsgen.seed_for(2, 1), n)
    k, v = oracle.sort(x, np.arange(n, dtype=np.uint32))
    assert np.all(k[1:] >= k[:-1])                              # sorted
    assert np.array_equal(np.bincount(np.searchsorted(np.unique(x), x)),
                          np.bincount(np.searchsorted(np.unique(x), k)))  # same multiset
    eq = k[1:] == k[:-1]
    assert np.all(v[1:][eq] > v[:-1][eq])                       # stable
    assert np.array_equal(x[v], k)                              # values are a permutation carrying keys
    assert np.array_equal(np.sort(v), np.arange(n, dtype=np.uint32))


# -- closed forms of the input families -----------------------------------------

@pytest.mark.parametrize("swaps", [0, 1, 1000, 100_000])
def test_nearly_sorted_closed_form(swaps):
    n = 100_000
    x = mmsgen.nearly_sorted_u32(mmsgen.seed_for(2, 2), n, swaps)
    k, v = oracle.sort(x, np.arange(n, dtype=np.uint32))
    assert np.array_equal(k, np.arange(n, dtype=np.uint32))
    inv = np.empty(n, dtype=np.uint32)
    inv[x] = np.arange(n, dtype=np.uint32)
    assert np.array_equal(v, inv)


def test_stride64_closed_form():
    n = 64 * 1000
    x = mmsgen.stride64_u32(n)
    k, v = oracle.sort(x, np.arange(n, dtype=np.uint32))
    j = np.arange(n, dtype=np.uint64)
    rows = n // 64
    assert np.array_equal(k, j.astype(np.uint32))
    assert np.array_equal(v, ((j % rows) * 64 + j // rows).astype(np.uint32))


def test_sixteen_closed_form():
    n = 50_000
    x = mmsgen.sixteen_u32(mmsgen.seed_for(3, 1), n)
    k, v = oracle.sort(x, np.arange(n, dtype=np.uint32))
    values = np.arange(16, dtype=np.uint64) * 0x11111111
    pos = 0
    for val in values:
        cnt = int(np.count_nonzero(x == val))
        assert np.all(k[pos:pos + cnt] == val)
        assert np.array_equal(v[pos:pos + cnt], np.flatnonzero(x == val).astype(np.uint32))
        pos += cnt
    assert pos == n


# -- §4.1 partition: brute force against its defining property ---------------

def _composite(keys, offs):
    """(key, run, pos) triples of the concatenated runs."""
    out = []
    for r in range(len(offs) - 1):
        for p in range(int(offs[r]), int(offs[r + 1])):
            out.append((int(keys[p]), r, p))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_partition_defining_property(seed):
    rng = np.random.default_rng(seed)
    K = int(rng.integers(1, 9))
    lens = rng.integers(0, 40, size=K)
    vals = 4 if seed % 2 else 1 << 30          # tie-heavy and distinct-ish
    runs = [np.sort(rng.integers(0, vals, size=int(L))).astype(np.uint32) for L in lens]
    keys = np.concatenate(runs) if runs else np.zeros(0, np.uint32)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    trip = _composite(keys, offs)
    total = len(trip)
    for r in range(total + 1):
        c = oracle.partition(keys, offs, r)
        assert int(c.sum()) == r
        assert all(0 <= int(c[k]) <= int(lens[k]) for k in range(K))
        pre = [(int(keys[int(offs[k]) + i]), k, int(offs[k]) + i) for k in range(K) for i in range(int(c[k]))]
        suf = [(int(keys[int(offs[k]) + i]), k, int(offs[k]) + i) for k in range(K)
               for i in range(int(c[k]), int(lens[k]))]
        if pre and suf:
            assert max(pre) < min(suf)
        assert sorted(pre) == sorted(trip)[:r]


# -- selection by counting ------------------------------------------------------

@pytest.mark.parametrize("family,i32", [("uniform", False), ("uniform", True), ("sixteen", False)])
def test_select_against_stable_argsort(family, i32):
    n = 30_001
    x = mmsgen.family(family, mmsgen.seed_for(4, 1), n)
    perm = np.argsort(x.view(np.int32) if i32 else x, kind="stable")
    for i in [0, 1, 2, n // 3, n // 2, n - 2, n - 1]:
        key, idx = oracle.select(x, i, i32=i32)
        assert idx == int(perm[i])
        assert key == int(x[perm[i]])


def test_select_every_rank_small_keys():
    # many distinct low halves inside one upper-half bucket, every rank
    x = mmsgen.uniform_u32(mmsgen.seed_for(4, 2), 300) % np.uint32(9)
    perm = np.argsort(x, kind="stable")
    for i in range(x.size):
        assert oracle.select(x, i) == (int(x[perm[i]]), int(perm[i]))
