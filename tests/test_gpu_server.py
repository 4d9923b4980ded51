"""GPU tests of the serving loop: every request served in a mixed stream
(keys and pairs, uint32 and int32, sizes from one element to several merge
rounds) is bit-identical to the same request sorted alone by the plain
entry points, and to the oracle; admission under a small arena; inputs
produced on a torch stream right before submission."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


SIZES = [1, 2, 63, 2047, 2048, 2049, 5000, 32768, 32769, 100_003, 1 << 20, 3 * (1 << 20) + 11]


def mixed_requests(seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i, n in enumerate(SIZES * 2):
        kind = ("keys", "pairs")[i % 2]
        fam = ("uniform", "sixteen", "sorted", "reverse")[rng.integers(4)]
        i32 = bool(rng.integers(2))
        x = mmsgen.family(fam, mmsgen.seed_for(5, i), n)
        v = np.arange(n, dtype=np.uint32) if kind == "pairs" else None
        reqs.append((x, v, i32))
    order = rng.permutation(len(reqs))
    return [reqs[j] for j in order]


def alone(mms, x, v, i32):
    if v is None:
        return host(mms.sort(dev(x), i32=i32)), None
    k, vv = mms.sort_pairs(dev(x), dev(v), i32=i32)
    return host(k), host(vv)


def test_mixed_stream_matches_alone_and_oracle(mms):
    reqs = mixed_requests(11)
    inputs = [(dev(x), dev(v) if v is not None else None, i32) for x, v, i32 in reqs]
    torch.cuda.synchronize()
    with mms.Server(budget_bytes=1 << 30, max_batch_keys=1 << 24) as srv:
        tickets = [srv.submit(k, vv, i32=i32) for k, vv, i32 in inputs]
        results = [srv.wait(t, 60_000) for t in tickets]
        assert all(r is not None and r.status == 0 for r in results)
        assert max(r.batch_requests for r in results) > 1, "no coalescing happened"
        for (x, v, i32), r, t in zip(reqs, results, tickets):
            ak, av = alone(mms, x, v, i32)
            gk = host(r.keys)
            assert np.array_equal(gk, ak), (x.size, i32)
            if v is not None:
                assert np.array_equal(host(r.values), av)
            if v is None:
                assert np.array_equal(gk, oracle.sort(x, i32=i32))
            else:
                ok, ov = oracle.sort(x, vals=v, i32=i32)
                assert np.array_equal(gk, ok) and np.array_equal(host(r.values), ov)
            srv.release(t)
        st = srv.stats()
        assert st["used_bytes"] == 0 and st["completed"] == len(reqs)


def test_small_arena_admits_as_results_are_released(mms):
    n = 1 << 20
    xs = [mmsgen.uniform_u32(mmsgen.seed_for(5, 40 + i), n) for i in range(6)]
    inputs = [dev(x) for x in xs]
    torch.cuda.synchronize()
    # room for about two requests (result + workspace) at a time
    with mms.Server(budget_bytes=(20 << 20) + (2 << 20), max_batch_keys=1 << 21,
                    max_batch_requests=8) as srv:
        budget = srv.stats()["data_budget_bytes"]
        assert 16 * n < budget < 24 * n
        tickets = [srv.submit(k) for k in inputs]
        for i, t in enumerate(tickets):
            r = srv.wait(t, 60_000)
            assert r is not None and r.status == 0
            assert np.array_equal(host(r.keys), oracle.sort(xs[i])), i
            srv.release(t, stream=torch.cuda.current_stream())
        st = srv.stats()
        assert st["peak_used_bytes"] <= budget
        assert st["completed"] == 6


def test_input_ready_on_caller_stream(mms):
    n = 3 << 20
    with mms.Server(budget_bytes=1 << 30) as srv:
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            g = torch.Generator(device="cuda")
            g.manual_seed(5)
            x = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device="cuda", generator=g)
            x.add_(7)             # more work queued on the side stream before the submit
            t = srv.submit(x, i32=True, stream=side)
        r = srv.wait(t, 60_000)
        assert r.status == 0
        side.synchronize()
        xh = x.cpu().numpy().view(np.uint32)
        assert np.array_equal(host(r.keys), oracle.sort(xh, i32=True))
        srv.release(t)


def test_caller_streams(mms):
    streams = [torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()]
    xs = [mmsgen.uniform_u32(mmsgen.seed_for(5, 60 + i), 70_000 + 1000 * i) for i in range(9)]
    inputs = [dev(x) for x in xs]
    torch.cuda.synchronize()
    with mms.Server(budget_bytes=1 << 28, streams=streams) as srv:
        tickets = [srv.submit(k) for k in inputs]
        used = set()
        for x, t in zip(xs, tickets):
            r = srv.wait(t, 60_000)
            assert np.array_equal(host(r.keys), oracle.sort(x))
            used.add(r.stream_index)
            srv.release(t)
        assert used <= {0, 1, 2}
