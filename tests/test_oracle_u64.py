"""Pins of the oracle's 64-bit sort (§6.3 also sorts 8-byte integers)
against facts that do not come from the oracle: hand-worked fixtures, brute
force over all small inputs, closed forms, and library routines (Python's
stable ``sorted``, NumPy's stable ``argsort``) for the special case where the
method's result is exactly a stable sort.  Keys are mapped so that both
32-bit halves of a key matter."""
import itertools
import math

import numpy as np
import pytest

import mmsgen
import oracle
from golden_io import sort_cases_u64

M32 = 0xFFFFFFFF


def hi_map(v):
    """Increasing in v; the low half decreases, so comparing only the low
    halves reverses the order."""
    return np.array([(int(t) << 32) | (~int(t) & M32) for t in v], dtype=np.uint64)


def lo_map(v):
    """Increasing in v with a common high half: only the low halves decide."""
    return np.array([0xDEADBEEF00000000 | int(t) for t in v], dtype=np.uint64)


@pytest.mark.parametrize("case", sort_cases_u64(), ids=lambda c: c[0])
def test_hand_cases_u64(case):
    name, i64, keys, out, idx = case
    k, v = oracle.sort_u64(keys, np.arange(keys.size, dtype=np.uint64), i64=i64)
    assert k.tolist() == out.tolist()
    assert v.tolist() == idx.tolist()
    assert oracle.sort_u64(keys, i64=i64).tolist() == out.tolist()


@pytest.mark.parametrize("fmap", [hi_map, lo_map], ids=["high_half", "low_half"])
def test_all_permutations_up_to_7(fmap):
    n_inputs = 0
    for n in range(0, 8):
        for p in itertools.permutations(range(n)):
            keys = fmap(p)
            k, v = oracle.sort_u64(keys, np.arange(n, dtype=np.uint64))
            assert k.tolist() == fmap(range(n)).tolist()
            inv = [0] * n
            for i, x in enumerate(p):
                inv[x] = i
            assert v.tolist() == inv
            n_inputs += 1
    assert n_inputs == sum(math.factorial(n) for n in range(8))


# three values whose unsigned order (0 < 2^63 < 2^64-1) and signed order
# (-2^63 < -1 < 0) differ
VALS = np.array([0x8000000000000000, 0xFFFFFFFFFFFFFFFF, 0x0000000000000000], dtype=np.uint64)


@pytest.mark.parametrize("signed", [False, True])
def test_all_ternary_sequences_up_to_6(signed):
    def key(x):
        x = int(x)
        return x - (1 << 64) if signed and x >> 63 else x
    for n in range(0, 7):
        for seq in itertools.product(range(3), repeat=n):
            keys = VALS[list(seq)] if n else np.zeros(0, np.uint64)
            k, v = oracle.sort_u64(keys, np.arange(n, dtype=np.uint64), i64=signed)
            want = sorted(range(n), key=lambda i: key(keys[i]))     # Python's sort is stable
            assert v.tolist() == want
            assert k.tolist() == [int(keys[i]) for i in want]


@pytest.mark.parametrize("n", [1, 2, 1000, 65_537, 1 << 20])
def test_numpy_stable_argsort(n):
    x = mmsgen.splitmix64(mmsgen.seed_for(14, n % 7), n)
    x[n // 2:] = x[: n - n // 2]                                     # every key twice: ties
    idx = np.arange(n, dtype=np.uint64)
    k, v = oracle.sort_u64(x, idx)
    perm = np.argsort(x, kind="stable")
    assert np.array_equal(v, perm.astype(np.uint64))
    assert np.array_equal(k, x[perm])
    ks, vs = oracle.sort_u64(x, idx, i64=True)
    perm = np.argsort(x.view(np.int64), kind="stable")
    assert np.array_equal(vs, perm.astype(np.uint64))
    assert np.array_equal(ks, x[perm])


def test_values_travel_with_keys():
    n = 30_001
    x = mmsgen.splitmix64(mmsgen.seed_for(14, 9), n) >> np.uint64(50)      # many ties
    payload = mmsgen.splitmix64(mmsgen.seed_for(14, 10), n)
    k, v = oracle.sort_u64(x, payload)
    perm = np.argsort(x, kind="stable")
    assert np.array_equal(v, payload[perm])


def test_closed_forms():
    n = 200_000
    # nearly sorted 0..n-1 in both halves: sorts to the identity map
    base = mmsgen.nearly_sorted_u32(mmsgen.seed_for(14, 11), n, 5000).astype(np.uint64)
    keys = (base << np.uint64(32)) | base
    want = (np.arange(n, dtype=np.uint64) << np.uint64(32)) | np.arange(n, dtype=np.uint64)
    assert np.array_equal(oracle.sort_u64(keys), want)
    # stride-64 interleave: values follow the inverse interleave
    s = mmsgen.stride64_u32(64 * 3000).astype(np.uint64) << np.uint64(20)
    k, v = oracle.sort_u64(s, np.arange(s.size, dtype=np.uint64))
    j = np.arange(s.size, dtype=np.uint64)
    rows = np.uint64(s.size // 64)
    assert np.array_equal(k, j << np.uint64(20))
    assert np.array_equal(v, (j % rows) * np.uint64(64) + j // rows)
