"""GPU parity of the 64-bit sorts (§6.3 also sorts 8-byte integers) through
the C ABI against the oracle's 64-bit sort, element by element.

Sizes span one base tile (4096 keys, 2048 pairs), several tiles, several
merge groups and ragged tails; keys are drawn so that both 32-bit halves
matter (full 64-bit uniform, keys that tie in the high half, keys that tie
everywhere, the maximum key that the merge's sentinel equals) in unsigned
and signed order; every fan-out the sort accepts is run.
"""
import os

import numpy as np
import pytest

import mmsgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TK, TP = 4096, 2048     # base tiles: keys, pairs
SIZES = [1, 2, 63, 64, 65, 511, TP - 1, TP, TP + 1, TK - 1, TK, TK + 1, 3 * TK + 5, 16 * TK - 1, 16 * TK + 1,
         16 * TK * 2 + 77, 16 * 16 * TK + 7, 99_991, 1 << 20]


@pytest.fixture(scope="module")
def mms():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_07961_amd as m
    m._lib.lib()
    yield m
    os.environ.pop("MMS64_FANOUT", None)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint64)


def keys64(family, n, seed):
    x = mmsgen.splitmix64(seed, n)
    if family == "uniform":
        return x
    if family == "high_ties":       # 16 high halves: the low half decides among ties
        return (x >> np.uint64(60) << np.uint64(32)) | (x & np.uint64(0xFFFFFFFF))
    if family == "few":             # 8 distinct keys spread over both halves
        return (x >> np.uint64(61)) * np.uint64(0x2000000020000001)
    if family == "max_heavy":       # many keys equal to the all-ones sentinel
        u = mmsgen.unit_doubles(seed + 1, n)
        return np.where(u < 0.4, np.uint64(0xFFFFFFFFFFFFFFFF), x).astype(np.uint64)
    if family == "sorted":
        return np.arange(n, dtype=np.uint64) * np.uint64(0x100000001)
    if family == "reverse":
        return (np.arange(n, dtype=np.uint64) * np.uint64(0x100000001))[::-1].copy()
    raise ValueError(family)


@pytest.mark.parametrize("n", SIZES)
def test_keys64_uniform_sizes(mms, n):
    x = keys64("uniform", n, mmsgen.seed_for(15, n % 16))
    assert np.array_equal(host(mms.sort64(dev(x), i64=False)), oracle.sort_u64(x))
    assert np.array_equal(host(mms.sort64(dev(x), i64=True)), oracle.sort_u64(x, i64=True))


@pytest.mark.parametrize("family", ["high_ties", "few", "max_heavy", "sorted", "reverse"])
@pytest.mark.parametrize("n", [16 * TK + 1, 300_007])
def test_keys64_families(mms, family, n):
    x = keys64(family, n, mmsgen.seed_for(15, 20))
    assert np.array_equal(host(mms.sort64(dev(x), i64=False)), oracle.sort_u64(x))
    assert np.array_equal(host(mms.sort64(dev(x), i64=True)), oracle.sort_u64(x, i64=True))


@pytest.mark.parametrize("n", SIZES)
def test_pairs64_stable(mms, n):
    x = keys64("few" if n % 2 else "high_ties", n, mmsgen.seed_for(15, 30 + n % 7))
    v = np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)      # payload in both halves
    gk, gv = mms.sort_pairs64(dev(x), dev(v), i64=False)
    ok, ov = oracle.sort_u64(x, v)
    assert np.array_equal(host(gk), ok) and np.array_equal(host(gv), ov)
    gk, gv = mms.sort_pairs64(dev(x), dev(v), i64=True)
    ok, ov = oracle.sort_u64(x, v, i64=True)
    assert np.array_equal(host(gk), ok) and np.array_equal(host(gv), ov)


@pytest.mark.parametrize("K", [2, 4, 8, 16])
def test_every_fanout(mms, K):
    os.environ["MMS64_FANOUT"] = str(K)
    try:
        n = 16 * 16 * TK + 12_345
        assert mms.plan(n, keys64=True).fanout == K
        x = keys64("max_heavy", n, mmsgen.seed_for(15, 40 + K))
        assert np.array_equal(host(mms.sort64(dev(x), i64=False)), oracle.sort_u64(x))
        v = np.arange(n, dtype=np.uint64)
        y = keys64("few", n, mmsgen.seed_for(15, 50 + K))
        gk, gv = mms.sort_pairs64(dev(y), dev(v), i64=True)
        ok, ov = oracle.sort_u64(y, v, i64=True)
        assert np.array_equal(host(gk), ok) and np.array_equal(host(gv), ov)
    finally:
        os.environ.pop("MMS64_FANOUT", None)


def test_keys64_in_place_and_empty(mms):
    n = 16 * TK * 3 + 11
    x = keys64("uniform", n, 77)
    t = dev(x)
    mms.sort64(t, out=t, i64=False)
    assert np.array_equal(host(t), oracle.sort_u64(x))
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    assert mms.sort64(e).numel() == 0


def test_keys64_fullsize(mms):
    """10^8 uniform 64-bit keys (the 8-byte workload at the headline's size),
    compared with the oracle element by element."""
    n = 10**8
    x = mmsgen.splitmix64(mmsgen.seed_for(15, 60), n)
    got = host(mms.sort64(dev(x), i64=False))
    assert np.array_equal(got, oracle.sort_u64(x))


def test_pairs64_fullsize_closed_form(mms):
    """2^26 stable pairs of a stride-64 interleave of 0..n-1 (shifted into the
    high half): keys sort to the identity and the values (input indices)
    follow the inverse interleave."""
    n = 1 << 26
    s = mmsgen.stride64_u32(n).astype(np.uint64) << np.uint64(31)
    k, v = mms.sort_pairs64(dev(s), torch.arange(n, dtype=torch.int64, device="cuda"), i64=False)
    j = torch.arange(n, dtype=torch.int64, device="cuda")
    rows = n // 64
    assert torch.equal(k, j << 31)
    assert torch.equal(v, (j % rows) * 64 + j // rows)
