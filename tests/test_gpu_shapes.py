"""GPU parity of every keys-only merge shape the library ships, against the
oracle, element by element.

The keys merge has five kernel shapes (variant 0: 64x16-key blocks with 8
waves, the built-in default; 1: 64x8-key blocks with 16 waves; 2: 64x8 with
8 waves; 3: as 2 with two workgroups per compute unit; 4: the minBlockHeap
merge, one heap of 64-key nodes per wave).  Each is run under
every fan-out K in {2, 4, 8, 16} and merge tiles of 2048, 6144, 7424 and 8192 keys,
on unsigned and signed keys, at a size where every workgroup of the
persistent grid walks several tiles per round (so the pipeline's prefetch,
its four-table ring and the buffer swap all run) and the last merge group is
ragged.  The oracle sorts each input once; every shape must reproduce it.
"""
import numpy as np
import pytest

import mmsgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# 2^23 + 12345 keys: with 8192-key merge tiles a round has 1026 tiles, at
# least 4 per workgroup of any shape's persistent grid (at most 256 compute
# units x 4 workgroups for the smallest LDS footprint at 2048-key tiles,
# which has 4102 tiles); the last group of every round is partial.
N_SWEEP = (1 << 23) + 12345
VARIANTS = [0, 1, 2, 3, 4]
FANOUTS = [2, 4, 8, 16]
TOUTS = [2048, 6144, 7424, 8192]
# base-case shape per variant (2048-, 4096- and 8192-key tiles all appear)
BASE_OF_VARIANT = {0: 0, 1: 4, 2: 3, 3: 6, 4: 3}


@pytest.fixture(scope="module")
def mms():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_07961_amd as m
    m._lib.lib()
    yield m
    m.set_tuning([])
    m._lib.load_tuning(m._lib.lib())


@pytest.fixture(scope="module")
def sweep_input():
    x = mmsgen.uniform_u32(mmsgen.seed_for(13, 0), N_SWEEP)
    # a tenth of the keys from a 64-value range: long runs of ties cross tiles
    u = mmsgen.unit_doubles(mmsgen.seed_for(13, 1), N_SWEEP)
    few = (mmsgen.uniform_u32(mmsgen.seed_for(13, 2), N_SWEEP) % np.uint32(64)) * np.uint32(0x04000001)
    x = np.where(u < 0.1, few, x).astype(np.uint32)
    return x, oracle.sort(x), oracle.sort(x, i32=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("variant", VARIANTS)
def test_merge_shape_sweep(mms, sweep_input, variant):
    x, want_u, want_s = sweep_input
    xd = dev(x)
    out = torch.empty_like(xd)
    base = BASE_OF_VARIANT[variant]
    for K in FANOUTS:
        for tout in TOUTS:
            mms.set_tuning([(64, K, tout, variant, base)])
            assert mms.get_tuning(N_SWEEP)[1:4] == (K, tout, variant)
            p = mms.plan(N_SWEEP)
            assert p.rounds >= 2
            mms.sort(xd, out=out, i32=False)
            assert np.array_equal(host(out), want_u), (variant, K, tout, "u32")
            mms.sort(xd, out=out, i32=True)
            assert np.array_equal(host(out), want_s), (variant, K, tout, "i32")


def test_builtin_default_through_c_abi(mms, sweep_input):
    """With no tuning table the C ABI uses its built-in default (K = 16,
    8192-key merge tiles, merge shape 0, base shape 0): the entry point a C
    caller gets without mms_set_tuning."""
    x, want_u, want_s = sweep_input
    mms.set_tuning([])
    t = mms.get_tuning(N_SWEEP)
    assert t[1:5] == (16, 8192, 0, 0)
    xd = dev(x)
    assert np.array_equal(host(mms.sort(xd, i32=False)), want_u)
    assert np.array_equal(host(mms.sort(xd, i32=True)), want_s)
    for n in [1, 2047, 2049, 16 * 2048 + 1, 300_001, 3_000_017]:
        y = x[:n].copy()
        assert np.array_equal(host(mms.sort(dev(y), i32=False)), oracle.sort(y)), n


def test_loaded_table_between_buckets(mms):
    """Plain sorts under the shipped table at sizes whose buckets pick the
    16-wave merge shape (2^21) and the two-workgroup shape (2^22 and up)."""
    mms.set_tuning([])
    mms._lib.load_tuning(mms._lib.lib())
    for n in [1_500_007, (1 << 21) - 3, (1 << 22) + 1001]:
        x = mmsgen.uniform_u32(mmsgen.seed_for(13, 3 + n % 5), n)
        assert np.array_equal(host(mms.sort(dev(x), i32=False)), oracle.sort(x)), n


# key-value sorts: every fan-out and both key-value base shapes (8 x 4 on
# 2048-pair tiles, 8 x 8 on 4096) on a tie-heavy input at a size where every
# fan-out runs two or more merge rounds of many 3840-pair tiles, the last
# group ragged; values are arbitrary words, so a misplaced value shows.
N_PAIRS_SWEEP = (1 << 22) + 12345


@pytest.fixture(scope="module")
def pairs_input():
    n = N_PAIRS_SWEEP
    x = mmsgen.uniform_u32(mmsgen.seed_for(21, 0), n)
    few = (mmsgen.uniform_u32(mmsgen.seed_for(21, 2), n) % np.uint32(16)) * np.uint32(0x10000001)
    u = mmsgen.unit_doubles(mmsgen.seed_for(21, 1), n)
    x = np.where(u < 0.3, few, x).astype(np.uint32)
    v = mmsgen.uniform_u32(mmsgen.seed_for(21, 3), n)
    return x, v, oracle.sort(x, v), oracle.sort(x, v, i32=True)


@pytest.mark.parametrize("base", [0, 3])
def test_pairs_shape_sweep(mms, pairs_input, base):
    x, v, (wku, wvu), (wks, wvs) = pairs_input
    xd, vd = dev(x), dev(v)
    for K in FANOUTS:
        mms.set_tuning([(64, 16, 7168, 3, 4, 0), (64, K, 3840, 0, base, mms.MMS_PAIRS)])
        p = mms.plan(N_PAIRS_SWEEP, pairs=True)
        assert p.rounds >= 2 and p.merge_tile == 3840
        gk, gv = mms.sort_pairs(xd, vd, i32=False)
        assert np.array_equal(host(gk), wku) and np.array_equal(host(gv), wvu), (K, base, "u32")
        gk, gv = mms.sort_pairs(xd, vd, i32=True)
        assert np.array_equal(host(gk), wks) and np.array_equal(host(gv), wvs), (K, base, "i32")


# One-read merges of short pairs: a wave that owns a whole pair of runs of at
# most one block each (N = 512 keys for the 64x8 shapes) merges it from a
# single read.  At the first level of a 16-way tile each of the 8 pairs goes
# to one wave, and the inputs fix how a tile's keys divide among the group's
# 16 runs: evenly (every piece exactly N at 8192-key tiles, both runs of a
# pair a full block), 2:1 and 1:2 within each pair (one piece a full block at
# 6144-key tiles), a random division, the same keys in every run (ties
# across the runs), and disjoint ranges (tiles drawing on one or two runs).
def _group_pattern_input(base_tile, n_groups, seed):
    """Groups of 16 base tiles (the runs of the first merge round), each
    group over its own range of 16 * base_tile consecutive keys divided
    among the runs by a pattern, every run holding base_tile keys in
    shuffled order."""
    K, bt = 16, base_tile
    m = K * bt
    perm_src = mmsgen.uniform_u32(mmsgen.seed_for(seed, 1), n_groups * m)
    rnd = mmsgen.uniform_u32(mmsgen.seed_for(seed, 2), n_groups * m)
    out = []
    for j in range(n_groups):
        kind = j % 6
        base_val = np.uint64(j) * np.uint64(2 * m)
        i = np.arange(m)
        vals = i.astype(np.uint64) + base_val
        if kind == 0:      # round robin: every run gets every 16th key
            run = i % K
        elif kind in (1, 2):
            # per 24 keys: 2 to each heavier run of a pair, 1 to the other,
            # until the heavier runs are full; the rest to the lighter ones
            heavy = 0 if kind == 1 else 1
            cyc, r = i // 24, i % 24
            pair, slot = r // 3, r % 3
            first = np.where(slot < 2, 2 * pair + heavy, 2 * pair + 1 - heavy)
            cut = 12 * bt
            rest = (i - cut) % (K // 2)
            run = np.where(i < cut, first, 2 * rest + 1 - heavy)
        elif kind == 3:    # a random division, bt keys per run
            run = np.empty(m, dtype=np.int64)
            run[np.argsort(rnd[j * m:(j + 1) * m], kind="stable")] = np.repeat(np.arange(K), bt)
        elif kind == 4:    # the same keys in every run
            vals = (i // K).astype(np.uint64) + base_val
            run = i % K
        else:              # disjoint ranges
            run = i // bt
        for k in range(K):
            t = vals[run == k]
            assert t.size == bt, (kind, k, t.size)
            order = np.argsort(perm_src[j * m + k * bt:j * m + (k + 1) * bt], kind="stable")
            out.append(t[order].astype(np.uint32))
    return np.concatenate(out)


@pytest.mark.parametrize("variant,base,touts", [(2, 3, [8192, 6144]), (3, 6, [6144, 7424]), (1, 4, [8192])])
def test_one_read_short_pairs(mms, variant, base, touts):
    for tout in touts:
        mms.set_tuning([(64, 16, tout, variant, base)])
        bt = mms.plan(1 << 20).tile
        x = _group_pattern_input(bt, 6, 40 + tout % 97)
        x = np.concatenate([x, mmsgen.uniform_u32(mmsgen.seed_for(41, tout), 5001)])   # a ragged group
        p = mms.plan(x.size)
        assert p.fanout == 16 and p.merge_tile == tout and p.tile == bt
        want = oracle.sort(x)
        got = host(mms.sort(dev(x), i32=False))
        assert np.array_equal(got, want), (variant, base, tout)
