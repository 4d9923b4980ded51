"""GPU parity of the batched segmented sort against the oracle, segment by
segment (each segment must equal its own oracle sort, bit for bit)."""
import numpy as np
import pytest

import mmsgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

T = 2048
K = 16


@pytest.fixture(scope="module")
def mms():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_07961_amd as m
    m._lib.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


def ragged_sizes():
    # empty, tiny, around one tile, around one group, several rounds
    return [0, 1, 2, 63, 64, 65, 0, T - 1, T, T + 1, 3 * T + 5, 0, T * K - 1, T * K, T * K + 1,
            T * K * 2 + 77, 1, 5000, T * K * K + 7, 0]


def offsets_of(sizes, start=0):
    return np.concatenate([[start], start + np.cumsum(sizes)]).astype(np.uint64)


@pytest.mark.parametrize("family", ["uniform", "sixteen", "sorted", "reverse"])
def test_segmented_keys_ragged(mms, family):
    sizes = ragged_sizes()
    off = offsets_of(sizes)
    x = mmsgen.family(family, mmsgen.seed_for(4, 1), int(off[-1]))
    got = host(mms.segmented_sort(dev(x), off, i32=False))
    assert np.array_equal(got, oracle.sort_segments(x, off))


@pytest.mark.parametrize("sizes", [[T * K * 3 + 11], [0, 0, 0], [1] * 300, [T] * 40, [T * K] * 5,
                                   [0, T * K * K, 0]])
def test_segmented_degenerate_batches(mms, sizes):
    """One segment (the plain sort's plan), only empty segments, 300 one-key
    segments, and segments that end exactly on base-tile and group
    boundaries: keys and stable pairs equal their oracle segment by segment;
    the keys past the last offset are not touched."""
    off = offsets_of(sizes)
    n = int(off[-1])
    x = mmsgen.family("sixteen", mmsgen.seed_for(4, 20 + len(sizes)), n + 8)
    guard = np.full(x.size, 0xA5A5A5A5, dtype=np.uint32)
    out = dev(guard)
    got = host(mms.segmented_sort(dev(x), off, out_keys=out, i32=False))
    assert np.array_equal(got[:n], oracle.sort_segments(x[:n], off))
    assert np.array_equal(got[n:], guard[n:])
    v = np.arange(x.size, dtype=np.uint32)
    gk, gv = mms.segmented_sort(dev(x), off, values=dev(v), i32=True)
    ok, ov = oracle.sort_segments(x[:n], off, vals=v[:n], i32=True)
    assert np.array_equal(host(gk)[:n], ok) and np.array_equal(host(gv)[:n], ov)


def test_segmented_pairs_stable(mms):
    sizes = ragged_sizes()
    off = offsets_of(sizes)
    x = mmsgen.sixteen_u32(mmsgen.seed_for(4, 2), int(off[-1]))
    v = np.arange(x.size, dtype=np.uint32)
    gk, gv = mms.segmented_sort(dev(x), off, values=dev(v), i32=False)
    ok, ov = oracle.sort_segments(x, off, vals=v)
    assert np.array_equal(host(gk), ok)
    assert np.array_equal(host(gv), ov)


def test_segmented_signed(mms):
    sizes = [1000, 0, T * K + 3, 17]
    off = offsets_of(sizes)
    x = mmsgen.uniform_u32(mmsgen.seed_for(4, 3), int(off[-1]))
    got = host(mms.segmented_sort(dev(x), off, i32=True))
    assert np.array_equal(got, oracle.sort_segments(x, off, i32=True))


def test_segmented_offset_start_leaves_prefix(mms):
    sizes = [300, 4000, 70_000]
    off = offsets_of(sizes, start=123)
    n = int(off[-1]) + 50
    x = mmsgen.uniform_u32(mmsgen.seed_for(4, 4), n)
    xd = dev(x)
    out = torch.full_like(xd, 7)
    mms.segmented_sort(xd, off, out_keys=out, i32=False)
    got = host(out)
    assert np.all(got[:123] == 7) and np.all(got[int(off[-1]):] == 7)
    want = oracle.sort_segments(x, off)
    assert np.array_equal(got[123:int(off[-1])], want[123:int(off[-1])])


def test_segmented_graph_replay_new_data(mms):
    # same offsets and buffers: the second call replays the captured graph
    sizes = mmsgen.loguniform_sizes(mmsgen.seed_for(4, 5), 300, 8, 16).astype(np.int64)
    off = offsets_of(sizes)
    n = int(off[-1])
    kin = torch.empty(n, dtype=torch.int32, device="cuda")
    out = torch.empty_like(kin)
    ws = torch.empty(mms.segmented_workspace_bytes(off), dtype=torch.uint8, device="cuda")
    for trial in range(3):
        x = mmsgen.uniform_u32(mmsgen.seed_for(4, 6 + trial), n)
        kin.copy_(dev(x))
        mms.segmented_sort(kin, off, out_keys=out, workspace=ws, i32=False)
        assert np.array_equal(host(out), oracle.sort_segments(x, off)), trial


def test_segmented_matches_plain_calls(mms):
    sizes = [5, T * K + 9, 40_000, 3]
    off = offsets_of(sizes)
    x = mmsgen.uniform_u32(mmsgen.seed_for(4, 9), int(off[-1]))
    seg = host(mms.segmented_sort(dev(x), off, i32=False))
    for s in range(len(sizes)):
        a, b = int(off[s]), int(off[s + 1])
        plain = host(mms.sort(dev(x[a:b]), i32=False)) if b > a else np.zeros(0, np.uint32)
        assert np.array_equal(seg[a:b], plain)


def test_segmented_batch_workload_sampled(mms):
    """4096 segments with log-uniform sizes in [2^8, 2^20] (the batched
    workload): every segment sorted and a permutation of its input (checked
    on the GPU for all segments), and 24 sampled segments equal to the oracle."""
    sizes = mmsgen.loguniform_sizes(mmsgen.seed_for(3, 0), 4096, 8, 20).astype(np.int64)
    off = offsets_of(sizes)
    n = int(off[-1])
    x = mmsgen.uniform_u32(mmsgen.seed_for(3, 1), n)
    xd = dev(x)
    out = mms.segmented_sort(xd, off, i32=False)
    torch.cuda.synchronize()
    seg_id = torch.repeat_interleave(torch.arange(4096, device="cuda"),
                                     torch.from_numpy(sizes).cuda())
    o = out.to(torch.int64) & 0xFFFFFFFF
    same_seg = seg_id[1:] == seg_id[:-1]
    assert bool((o[1:][same_seg] >= o[:-1][same_seg]).all())
    composite_in = torch.sort((seg_id << 32) | (xd.to(torch.int64) & 0xFFFFFFFF)).values
    composite_out = (seg_id << 32) | o
    assert torch.equal(composite_in, composite_out)
    got = host(out)
    rng = np.random.default_rng(7)
    for s in rng.choice(4096, 24, replace=False):
        a, b = int(off[s]), int(off[s + 1])
        assert np.array_equal(got[a:b], oracle.sort(x[a:b])), s


@pytest.mark.parametrize("base", [0, 3, 4, 6])
def test_segmented_base_tiles(mms, base):
    """Batches under every base tile (2048, 4096, 8192 keys): many small
    segments (the batch caps its base tile at the mean segment) and a mix
    around the larger tiles; keys and stable pairs."""
    small = [0, 1, 3, 100, 257, 999, 2048, 2049] * 40
    mixed = [4095, 4096, 4097, 8191, 8192, 8193, 3 * 8192 + 5, 16 * 8192 + 1, 70_001]
    try:
        mms.set_tuning([(64, K, 4096, 3, base)])
        for sizes in (small, mixed, small + mixed):
            off = offsets_of(sizes)
            x = mmsgen.sixteen_u32(mmsgen.seed_for(4, 5 + base), int(off[-1]))
            got = host(mms.segmented_sort(dev(x), off, i32=True))
            assert np.array_equal(got, oracle.sort_segments(x, off, i32=True))
            v = np.arange(x.size, dtype=np.uint32)
            gk, gv = mms.segmented_sort(dev(x), off, values=dev(v), i32=False)
            ok, ov = oracle.sort_segments(x, off, vals=v)
            assert np.array_equal(host(gk), ok) and np.array_equal(host(gv), ov)
    finally:
        mms.set_tuning([])
        mms._lib.load_tuning(mms._lib.lib())


def test_segmented_workspace_reused_between_replays(mms):
    """The batch metadata lives in the caller's workspace and is copied in
    on every call: clobbering the whole workspace between graph replays must
    not change the results."""
    sizes = mmsgen.loguniform_sizes(mmsgen.seed_for(4, 20), 200, 8, 17).astype(np.int64)
    off = offsets_of(sizes)
    n = int(off[-1])
    ws = torch.empty(mms.segmented_workspace_bytes(off), dtype=torch.uint8, device="cuda")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    for trial in range(4):
        x = mmsgen.uniform_u32(mmsgen.seed_for(4, 21 + trial), n)
        ws.fill_(0xA5 + trial)
        mms.segmented_sort(dev(x), off, out_keys=out, workspace=ws, i32=False)
        assert np.array_equal(host(out), oracle.sort_segments(x, off)), trial


def test_segmented_signature_cache_eviction(mms):
    """More distinct offset signatures than the library caches (8), enqueued
    back to back on one stream with no synchronisation in between: evicting
    an entry must wait for its launches, and every result must be exact."""
    cases = []
    for i in range(11):
        sizes = [300 + 97 * i, 0, 2048 * (i + 1) + 5, 40_000 + 1000 * i]
        off = offsets_of(sizes)
        x = mmsgen.uniform_u32(mmsgen.seed_for(4, 40 + i), int(off[-1]))
        xd = dev(x)
        out = torch.empty_like(xd)
        ws = torch.empty(mms.segmented_workspace_bytes(off), dtype=torch.uint8, device="cuda")
        cases.append((x, off, xd, out, ws))
    torch.cuda.synchronize()
    for rep in range(2):
        for x, off, xd, out, ws in cases:
            mms.segmented_sort(xd, off, out_keys=out, workspace=ws, i32=False)
    for x, off, xd, out, ws in cases:
        assert np.array_equal(host(out), oracle.sort_segments(x, off))
