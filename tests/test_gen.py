"""Input generators: determinism, published constants and closed forms."""
import numpy as np
import pytest

import mmsgen


def test_splitmix64_published_values():
    # splitmix64 seeded with 0: first outputs as published with the algorithm
    # (Vigna's reference implementation of Steele-Lea-Flood)
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert mmsgen.splitmix64(0, 3).tolist() == want


def test_uniform_is_top_half_of_splitmix():
    assert np.array_equal(mmsgen.uniform_u32(7, 1000),
                          (mmsgen.splitmix64(7, 1000) >> np.uint64(32)).astype(np.uint32))


def test_determinism_per_seed():
    a = mmsgen.uniform_u32(mmsgen.seed_for(1, 0), 5000)
    b = mmsgen.uniform_u32(mmsgen.seed_for(1, 0), 5000)
    c = mmsgen.uniform_u32(mmsgen.seed_for(1, 1), 5000)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_nearly_sorted_zero_swaps_is_identity():
    assert np.array_equal(mmsgen.nearly_sorted_u32(1, 1000, 0), np.arange(1000, dtype=np.uint32))


def test_nearly_sorted_is_permutation():
    x = mmsgen.nearly_sorted_u32(3, 4096, 10_000)
    assert np.array_equal(np.bincount(x, minlength=4096), np.ones(4096, dtype=np.int64))


def test_stride64_definition():
    n = 64 * 8
    x = mmsgen.stride64_u32(n)
    i = np.arange(n)
    assert np.array_equal(x, ((i % 64) * (n // 64) + i // 64).astype(np.uint32))
    assert np.all(np.diff(x.reshape(8, 64), axis=1) == n // 64)   # each 64-chunk ascends
    assert np.array_equal(np.sort(x), np.arange(n, dtype=np.uint32))


def test_sixteen_values():
    x = mmsgen.sixteen_u32(5, 100_000)
    vals = set(np.unique(x).tolist())
    assert vals == {v * 0x11111111 for v in range(16)}
    assert 0 in vals and 0xFFFFFFFF in vals


def test_permutation():
    x = mmsgen.permutation_u32(9, 10_000)
    assert np.array_equal(np.sort(x), np.arange(10_000, dtype=np.uint32))
    assert not np.array_equal(x, np.arange(10_000, dtype=np.uint32))


def test_loguniform_sizes_range_and_mean():
    s = mmsgen.loguniform_sizes(11, 4096, 8, 20)
    assert s.min() >= 256 and s.max() < (1 << 20)
    mean = mmsgen.loguniform_mean(8, 20)
    assert abs(s.mean() / mean - 1) < 0.1


def test_poisson_arrivals_rate():
    t = mmsgen.poisson_arrivals(13, 20000, rate=1000.0)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 20.0 - 1) < 0.05


def test_mergepath_adversary_is_a_permutation_with_its_pattern():
    """Every merge of two runs of h keys (runs at every level, h >= 15) takes,
    in the first half of its 15-output thread windows, 15, 15 and 2 outputs
    of every three from its first run, and mirrors that in the second half."""
    vt = 15
    n = vt * 2**9
    x = mmsgen.mergepath_adversary_u32(n)
    assert np.array_equal(np.sort(x), np.arange(n, dtype=np.uint32))
    length = n
    while length > vt:
        h = length // 2
        for s in range(0, n, length):
            a = set(x[s:s + h].tolist())
            merged = np.sort(x[s:s + length])
            from_a = np.array([v in a for v in merged.tolist()])
            per_thread = from_a.reshape(-1, vt).sum(1)
            t = per_thread.size
            head = per_thread[: max(0, t // 2 - 3)]
            want = np.tile([15, 15, 2], head.size // 3 + 1)[: head.size]
            assert np.array_equal(head, want), (length, s)
            assert from_a.sum() == h
        length = h
    # runs of vt keys descend
    assert np.all(np.diff(x[:vt].astype(np.int64)) < 0)
    with pytest.raises(ValueError):
        mmsgen.mergepath_adversary_u32(vt * 3)
