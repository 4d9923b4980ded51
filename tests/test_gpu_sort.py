"""GPU parity: the HIP sort through the C ABI against the CPU oracle.

Sizes span one base tile, several tiles, several merge groups and ragged
tails; bit-exact equality is the only acceptance (integer sorting).
Full-size workloads are checked by closed forms of their input families and
by order statistics the oracle computes one at a time.
"""
import numpy as np
import pytest

import mmsgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mms():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_07961_amd as m
    m._lib.lib()
    return m


def dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


T = 2048            # base tile
K = 16              # fan-out
SIZES = [1, 2, 3, 63, 64, 65, 511, 512, 513, T - 1, T, T + 1, 3 * T + 5, T * K - 1, T * K, T * K + 1,
         T * K * 2 + 77, T * K * K + 7, 99_991, 1 << 20]
FAMILIES = ["uniform", "sorted", "reverse", "equal", "sixteen", "nearly"]


def gen(family, n, seed):
    return mmsgen.family(family, seed, n, swaps=max(1, n // 100))


@pytest.mark.parametrize("n", SIZES)
def test_keys_uniform_sizes(mms, n):
    x = mmsgen.uniform_u32(mmsgen.seed_for(1, n % 16), n)
    got = host(mms.sort(dev(x), i32=False))
    assert np.array_equal(got, oracle.sort(x))


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("n", [T * K + 1, 123_457])
def test_keys_families(mms, family, n):
    x = gen(family, n, mmsgen.seed_for(2, 3))
    got = host(mms.sort(dev(x), i32=False))
    assert np.array_equal(got, oracle.sort(x))


def test_keys_extreme_values(mms):
    n = 50_001
    x = mmsgen.uniform_u32(5, n) % np.uint32(4)
    x = np.choose(x, [np.uint32(0), np.uint32(0xFFFFFFFF), np.uint32(0x80000000), np.uint32(0x7FFFFFFF)])
    x = x.astype(np.uint32)
    assert np.array_equal(host(mms.sort(dev(x), i32=False)), oracle.sort(x))
    assert np.array_equal(host(mms.sort(dev(x), i32=True)), oracle.sort(x, i32=True))


@pytest.mark.parametrize("base", [0, 1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("n", [1, T - 1, T, T + 1, 4 * T - 1, 4 * T + 1, T * K * 2 + 77, 300_001])
def test_keys_base_shapes(mms, base, n):
    """Every keys-only base-case shape the tuner can choose (8 x 4, 4 x 8,
    16 x 2 keys per lane x waves on 2048-key tiles, 8 x 8 and 16 x 4 on 4096,
    8 x 16 and 16 x 8 on 8192) sorts, unsigned and signed."""
    x = mmsgen.family("sixteen" if n % 2 else "uniform", mmsgen.seed_for(11, n % 13), n)
    try:
        mms.set_tuning([(64, K, 4096, 2, base)])
        assert np.array_equal(host(mms.sort(dev(x), i32=False)), oracle.sort(x))
        assert np.array_equal(host(mms.sort(dev(x), i32=True)), oracle.sort(x, i32=True))
        # key-value sorts map the shape to 8 x 4 or 8 x 8
        v = np.arange(n, dtype=np.uint32)[::-1].copy()
        gk, gv = mms.sort_pairs(dev(x), dev(v), i32=True)
        ok, ov = oracle.sort(x, v, i32=True)
        assert np.array_equal(host(gk), ok) and np.array_equal(host(gv), ov)
    finally:
        mms.set_tuning([])
        mms._lib.load_tuning(mms._lib.lib())


@pytest.mark.parametrize("K,n,family", [(16, 2048 * 16 * 3 + 4321, "sixteen"), (16, 2048 * 16 * 16 * 2 - 7, "uniform"),
                                         (4, 2048 * 4 ** 4 * 2 + 999, "sixteen"), (2, 2048 * 2 ** 6 * 3 + 5, "uniform"),
                                         (2, 2048 * 2 ** 5 + 1, "sixteen")])
def test_fanouts_ragged_groups(mms, K, n, family):
    """Fan-outs 16, 4 and 2 on 2048-key base tiles and 4096-key merge tiles:
    groups of 8 to 64 merge tiles, partitions refining one bit per round (16
    runs) and several (at most 9 runs, also 3-run last rounds), ragged last
    groups, runs of 2^11 to 2^17 keys, many equal keys; keys and stable pairs
    against the oracle."""
    x = mmsgen.family(family, mmsgen.seed_for(31, K * 1000 + n % 1000), n)
    v = np.arange(n, dtype=np.uint32)
    try:
        mms.set_tuning([(64, K, 4096, 2, 0), (64, K, 4096, 0, 0, mms.MMS_PAIRS)])
        assert np.array_equal(host(mms.sort(dev(x), i32=False)), oracle.sort(x))
        gk, gv = mms.sort_pairs(dev(x), dev(v), i32=True)
        ok, ov = oracle.sort(x, v, i32=True)
        assert np.array_equal(host(gk), ok) and np.array_equal(host(gv), ov)
    finally:
        mms.set_tuning([])
        mms._lib.load_tuning(mms._lib.lib())


@pytest.mark.parametrize("pk,pbase", [(4, 0), (8, 3), (2, 3)])
def test_pairs_own_tuning_entries(mms, pk, pbase):
    """Key-value sorts follow their own tuning entries while keys-only sorts
    keep theirs; both stay exact."""
    n = T * 16 * 3 + 77
    x = mmsgen.sixteen_u32(mmsgen.seed_for(12, pk), n)
    v = np.arange(n, dtype=np.uint32)
    try:
        mms.set_tuning([(64, 16, 7168, 3, 4, 0), (64, pk, 4096, 0, pbase, mms.MMS_PAIRS)])
        assert mms.get_tuning(n, pairs=True)[1] == pk and mms.get_tuning(n)[1] == 16
        gk, gv = mms.sort_pairs(dev(x), dev(v), i32=False)
        ok, ov = oracle.sort(x, v)
        assert np.array_equal(host(gk), ok) and np.array_equal(host(gv), ov)
        assert np.array_equal(host(mms.sort(dev(x), i32=False)), oracle.sort(x))
    finally:
        mms.set_tuning([])
        mms._lib.load_tuning(mms._lib.lib())


@pytest.mark.parametrize("n,frac", [(T, 0.5), (T * K * 3 + 5, 0.25), (300_001, 0.9), (T * K * K + 11, 0.6)])
def test_keys_bulk_sentinel_valued(mms, n, frac):
    """Many keys equal to the merge's sentinel (0xFFFFFFFF unsigned, INT32_MAX
    signed): a run that ends beside a run of such keys must not let the merge
    cursors run past it."""
    u = mmsgen.unit_doubles(mmsgen.seed_for(9, n % 7), n)
    x = mmsgen.uniform_u32(mmsgen.seed_for(10, n % 7), n)
    xu = np.where(u < frac, np.uint32(0xFFFFFFFF), x).astype(np.uint32)
    assert np.array_equal(host(mms.sort(dev(xu), i32=False)), oracle.sort(xu))
    xs = np.where(u < frac, np.uint32(0x7FFFFFFF), x).astype(np.uint32)
    assert np.array_equal(host(mms.sort(dev(xs), i32=True)), oracle.sort(xs, i32=True))


@pytest.mark.parametrize("n", [1000, T * K + 3, 300_001])
def test_keys_signed(mms, n):
    x = mmsgen.uniform_u32(mmsgen.seed_for(2, 5), n)
    got = host(mms.sort(dev(x), i32=True))
    assert np.array_equal(got, oracle.sort(x, i32=True))


def test_keys_in_place(mms):
    n = T * K * 3 + 11
    x = mmsgen.uniform_u32(77, n)
    t = dev(x)
    mms.sort(t, out=t, i32=False)
    assert np.array_equal(host(t), oracle.sort(x))


def test_empty(mms):
    t = torch.empty(0, dtype=torch.int32, device="cuda")
    assert mms.sort(t).numel() == 0


@pytest.mark.parametrize("n", [1, 64, 4097, T * K - 1, T * K * 2 + 77, 200_003])
@pytest.mark.parametrize("family", ["uniform", "sixteen", "equal"])
def test_pairs_stable(mms, n, family):
    x = gen(family, n, mmsgen.seed_for(3, n % 16))
    v = np.arange(n, dtype=np.uint32)
    gk, gv = mms.sort_pairs(dev(x), dev(v), i32=False)
    ok, ov = oracle.sort(x, v)
    assert np.array_equal(host(gk), ok)
    assert np.array_equal(host(gv), ov)


def test_pairs_stride64(mms):
    n = 64 * 5000
    x = mmsgen.stride64_u32(n)
    v = mmsgen.uniform_u32(9, n)             # arbitrary payload travels with its key
    gk, gv = mms.sort_pairs(dev(x), dev(v), i32=False)
    ok, ov = oracle.sort(x, v)
    assert np.array_equal(host(gk), ok)
    assert np.array_equal(host(gv), ov)


def test_pairs_signed(mms):
    n = 70_001
    x = mmsgen.uniform_u32(11, n) % np.uint32(64) - np.uint32(32)   # small signed range, many ties
    v = np.arange(n, dtype=np.uint32)
    gk, gv = mms.sort_pairs(dev(x), dev(v), i32=True)
    ok, ov = oracle.sort(x, v, i32=True)
    assert np.array_equal(host(gk), ok)
    assert np.array_equal(host(gv), ov)


@pytest.mark.parametrize("Kq,L,n,tie", [(16, 2048, 16 * 2048 * 2 + 999, False), (4, 100, 1000, True),
                                        (16, 37, 16 * 37 * 3 - 5, True), (2, 5000, 12_000, False),
                                        (1, 64, 200, False), (7, 333, 7 * 333 + 5, True),
                                        (9, 4096, 9 * 4096 * 2 - 17, False), (8, 777, 8 * 777 * 2 + 3, True),
                                        (10, 1000, 10 * 1000 + 1, True), (3, 8192, 3 * 8192 * 2 + 1234, False),
                                        (5, 500, 5 * 500 * 3 - 1, True)])
def test_partition_against_oracle(mms, Kq, L, n, tie):
    x = (mmsgen.uniform_u32(21, n) % np.uint32(3)) if tie else mmsgen.uniform_u32(22, n)
    for s in range(0, n, L):
        x[s:s + L] = oracle.sort(x[s:s + L])
    span = Kq * L
    groups, ranks, want = [], [], []
    rng = np.random.default_rng(4)
    for g in range(-(-n // span)):
        gb, glen = g * span, min(span, n - g * span)
        offs = np.array([min(k * L, glen) for k in range(-(-glen // L))] + [glen], dtype=np.uint64)
        sub = x[gb:gb + glen]
        for r in sorted({0, 1, glen // 2, glen - 1, glen, *rng.integers(0, glen + 1, 6).tolist()}):
            c = np.zeros(Kq, dtype=np.uint32)
            c[:offs.size - 1] = oracle.partition(sub, offs, int(r))
            groups.append(g)
            ranks.append(int(r))
            want.append(c)
    got = host(mms.partition(dev(x), L, Kq, groups, ranks))
    assert np.array_equal(got, np.array(want, dtype=np.uint32))


def test_copy(mms):
    # up to several grid-stride trips per workgroup (16384 x 256 lanes x 8 chunks of 4 keys per trip)
    for n in [1, 3, 4, 1000, 1 << 20, (1 << 20) + 3, (3 << 27) + 5]:
        x = mmsgen.uniform_u32(n, n)
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        mms.copy(dev(x), out)
        assert np.array_equal(host(out), x)
