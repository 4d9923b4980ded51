"""Full-size GPU checks in the launch configuration the benchmark times.

The uniform workloads (10^8 keys, unsigned and signed, and 2^27 uniform
pairs) are compared with the oracle's whole sort element by element (about
15-30 s of oracle each).  The others are checked by properties that hold at
any size —
sortedness, equality of the key multiset (histogram of the input vs the
output), stability — by closed forms of the input families (nearly-sorted
and stride-64 inputs sort to 0..n-1; stride-64 values follow the inverse
interleave), and at sampled positions against order statistics the oracle
computes one by one by counting.
"""
import numpy as np
import pytest

import mmsgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_KEYS = 10**8
N_PAIRS = 2**27


@pytest.fixture(scope="module")
def mms():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_07961_amd as m
    m._lib.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def sample_positions(n, seed, count=6):
    rng = np.random.default_rng(seed)
    return sorted({0, n - 1, n // 2, *rng.integers(0, n, count).tolist()})


def check_sorted_permutation(x_dev, out_dev, signed=False):
    a = out_dev.to(torch.int64)
    if not signed:
        a = a & 0xFFFFFFFF
    assert bool((a[1:] >= a[:-1]).all())
    # same multiset: per-key counts of the input equal those of the output
    xs = torch.sort(x_dev.to(torch.int64) & 0xFFFFFFFF).values
    os_ = torch.sort(out_dev.to(torch.int64) & 0xFFFFFFFF).values
    assert torch.equal(xs, os_)


def test_headline_uniform_u32(mms):
    """The benchmark's workload in its launch configuration (loaded tuning
    table), compared with the oracle's sort element by element."""
    x = mmsgen.uniform_u32(mmsgen.seed_for(2, 0), N_KEYS)
    xd = dev(x)
    out = mms.sort(xd, i32=False)
    torch.cuda.synchronize()
    check_sorted_permutation(xd, out)
    got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.sort(x))


@pytest.mark.parametrize("swaps", [0, 10**3, 10**6, 10**8])
def test_nearly_sorted_int32(mms, swaps):
    x = mmsgen.nearly_sorted_u32(mmsgen.seed_for(2, 1), N_KEYS, swaps)
    out = mms.sort(dev(x), i32=True)
    assert torch.equal(out, torch.arange(N_KEYS, dtype=torch.int32, device="cuda"))


def test_uniform_int32_full(mms):
    x = mmsgen.uniform_u32(mmsgen.seed_for(2, 2), N_KEYS)
    xd = dev(x)
    out = mms.sort(xd, i32=True)
    check_sorted_permutation(xd, out, signed=True)
    got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.sort(x, i32=True))


def test_pairs_stride64_closed_form(mms):
    x = mmsgen.stride64_u32(N_PAIRS)
    v = mmsgen.iota_u32(N_PAIRS)
    k, val = mms.sort_pairs(dev(x), dev(v), i32=False)
    j = torch.arange(N_PAIRS, dtype=torch.int64, device="cuda")
    rows = N_PAIRS // 64
    assert torch.equal(k.to(torch.int64), j)
    assert torch.equal(val.to(torch.int64), (j % rows) * 64 + j // rows)


def test_pairs_sixteen_closed_form(mms):
    x = mmsgen.sixteen_u32(mmsgen.seed_for(3, 1), N_PAIRS)
    k, val = mms.sort_pairs(dev(x), dev(mmsgen.iota_u32(N_PAIRS)), i32=False)
    kk = k.to(torch.int64) & 0xFFFFFFFF
    assert bool((kk[1:] >= kk[:-1]).all())
    counts = torch.bincount((dev(x).to(torch.int64) & 0xFFFFFFFF) // 0x11111111, minlength=16)
    assert torch.equal(torch.bincount(kk // 0x11111111, minlength=16), counts)
    vv = val.to(torch.int64)
    same = kk[1:] == kk[:-1]
    assert bool((vv[1:][same] > vv[:-1][same]).all())          # stable inside each run
    assert torch.equal(dev(x)[val.to(torch.int64)], k)         # values point at their keys


def test_pairs_uniform_sampled(mms):
    x = mmsgen.uniform_u32(mmsgen.seed_for(3, 0), N_PAIRS)
    k, val = mms.sort_pairs(dev(x), dev(mmsgen.iota_u32(N_PAIRS)), i32=False)
    kk = k.to(torch.int64) & 0xFFFFFFFF
    assert bool((kk[1:] >= kk[:-1]).all())
    vv = val.to(torch.int64)
    same = kk[1:] == kk[:-1]
    assert bool((vv[1:][same] > vv[:-1][same]).all())
    assert torch.equal(dev(x)[vv], k)
    assert torch.equal(torch.sort(vv).values, torch.arange(N_PAIRS, device="cuda"))
    kh, vh = k.cpu().numpy().view(np.uint32), val.cpu().numpy().view(np.uint32)
    for i in sample_positions(N_PAIRS, 3, count=3):
        key, idx = oracle.select(x, i)
        assert (int(kh[i]), int(vh[i])) == (key, idx), i
    ok, ov = oracle.sort(x, mmsgen.iota_u32(N_PAIRS))
    assert np.array_equal(kh, ok) and np.array_equal(vh, ov)


def test_batched_fullsize(mms):
    """The batched workload the benchmark times: 4096 uint32 arrays with sizes
    log-uniform in [2^8, 2^20] (about 5.3e8 keys), one call.  Every segment
    must equal its own sorted input: checked for all segments at once by
    sorting (segment, key) composites with torch, and for a sample of
    segments against the oracle."""
    sizes = mmsgen.loguniform_sizes(mmsgen.seed_for(4, 0), 4096, 8, 20).astype(np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = int(off[-1])
    x = mmsgen.uniform_u32(mmsgen.seed_for(4, 2), total)
    xd = dev(x)
    out = mms.segmented_sort(xd, off, i32=False)
    seg = torch.repeat_interleave(torch.arange(sizes.size, device="cuda", dtype=torch.int64),
                                  torch.from_numpy(sizes).cuda())
    want = torch.sort((seg << 32) | (xd.to(torch.int64) & 0xFFFFFFFF)).values
    got = (seg << 32) | (out.to(torch.int64) & 0xFFFFFFFF)
    assert torch.equal(got, want)
    del want, got, seg
    oh = out.cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(7)
    for s in sorted({0, int(np.argmax(sizes)), *rng.integers(0, sizes.size, 6).tolist()}):
        a, b = int(off[s]), int(off[s + 1])
        assert np.array_equal(oh[a:b], oracle.sort(x[a:b])), s


def test_keys_near_2_32(mms):
    """The largest sizes the 32-bit positions allow: 2^32 - 778 keys (five
    rounds), checked by sortedness and the histogram of the top 16 bits."""
    n = (1 << 32) - 778
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    x = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device="cuda", generator=g)
    out = mms.sort(x, i32=False)
    a = out.to(torch.int64) & 0xFFFFFFFF
    assert bool((a[1:] >= a[:-1]).all())
    del a
    hx = torch.bincount((x.to(torch.int64) & 0xFFFFFFFF) >> 16, minlength=65536)
    ho = torch.bincount((out.to(torch.int64) & 0xFFFFFFFF) >> 16, minlength=65536)
    assert torch.equal(hx, ho)


def test_pairs_above_2_31(mms):
    """2^31 + 4097 stable pairs with 1024 distinct keys: sorted keys, values a
    permutation that increases inside every run of equal keys."""
    n = (1 << 31) + 4097
    g = torch.Generator(device="cuda")
    g.manual_seed(6)
    x = torch.randint(0, 1024, (n,), dtype=torch.int32, device="cuda", generator=g)
    v = torch.arange(n, dtype=torch.int64, device="cuda").to(torch.int32)
    k, val = mms.sort_pairs(x, v, i32=False)
    vv = val.to(torch.int64) & 0xFFFFFFFF
    # (key, value) strictly increasing: keys sorted, equal keys in input order
    c = (k.to(torch.int64) << 32) | vv
    assert bool((c[1:] > c[:-1]).all())
    del c
    assert torch.equal(torch.bincount(x, minlength=1024), torch.bincount(k, minlength=1024))
    assert torch.equal(x[vv], k)
