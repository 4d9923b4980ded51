"""Admission logic of the serving loop on the CPU: the server runs in dry-run
mode (scheduler and completion bookkeeping with no device work), so these
tests check budget accounting, first-come first-served admission, limits,
rejection and ticket errors without a GPU."""
import time

import pytest

from paper_1702_07961_amd import _lib

T1 = 2048


@pytest.fixture(scope="module")
def mms():
    import os
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1702_07961_amd import build
        build.build()
    import paper_1702_07961_amd as m
    return m


def half(n):
    return -(-n * 4 // 256) * 256


def footprint(n, pairs):
    res = half(n) * (2 if pairs else 1)
    return res, (res if n > T1 else 0)


def wait_for(pred, timeout=5.0):
    end = time.time() + timeout
    while time.time() < end:
        if pred():
            return True
        time.sleep(0.002)
    return False


def make(mms, budget=1 << 24, **kw):
    kw.setdefault("max_batch_keys", 1 << 20)
    kw.setdefault("max_batch_requests", 16)
    return mms.Server(budget_bytes=budget, dry_run=True, **kw)


def test_budget_accounting(mms):
    with make(mms) as s:
        st = s.stats()
        assert st["data_budget_bytes"] + st["meta_bytes"] <= 1 << 24
        assert st["used_bytes"] == 0
        a = s.submit(n=100_000)
        b = s.submit(n=5000, values=True)
        c = s.submit(n=T1, values=True)       # one tile: no workspace
        for t in (a, b, c):
            assert s.wait(t, 5000).status == 0
        res = sum(footprint(n, p)[0] for n, p in [(100_000, False), (5000, True), (T1, True)])
        # workspaces are returned at completion, results stay until release
        assert s.stats()["used_bytes"] == res
        peak = sum(sum(footprint(n, p)) for n, p in [(100_000, False), (5000, True), (T1, True)])
        assert s.stats()["peak_used_bytes"] <= peak
        s.release(a)
        assert s.stats()["used_bytes"] == res - footprint(100_000, False)[0]
        s.release(b)
        s.release(c)
        st = s.stats()
        assert st["used_bytes"] == 0
        assert (st["submitted"], st["admitted"], st["completed"], st["released"]) == (3, 3, 3, 3)


def test_fifo_head_of_line(mms):
    with make(mms, budget=1 << 23) as s:
        budget = s.stats()["data_budget_bytes"]
        # A's result holds 45% of the budget; B (result + workspace, 90%)
        # cannot fit beside it; C could, but must not overtake B
        n_a = (budget * 45 // 100) // 4
        n_b = n_a
        a = s.submit(n=n_a)
        assert s.wait(a, 5000).status == 0        # A's workspace is back, its result stays
        b = s.submit(n=n_b)
        c = s.submit(n=1000)
        time.sleep(0.05)
        assert s.poll(b) is None and s.poll(c) is None
        st = s.stats()
        assert st["queued"] == 2 and st["admitted"] == 1
        s.release(a)
        rb = s.wait(b, 5000)
        rc = s.wait(c, 5000)
        assert rb.status == 0 and rc.status == 0
        assert rb.t_admit_us <= rc.t_admit_us
        s.release(b)
        s.release(c)


def test_request_limit(mms):
    with make(mms, max_requests=2) as s:
        t = [s.submit(n=500) for _ in range(3)]
        assert s.wait(t[0], 5000) is not None and s.wait(t[1], 5000) is not None
        time.sleep(0.05)
        assert s.poll(t[2]) is None                # two admitted and unreleased
        s.release(t[0])
        assert s.wait(t[2], 5000).status == 0
        s.release(t[1])
        s.release(t[2])


def test_rejections_and_ticket_errors(mms):
    with make(mms, budget=1 << 26, max_batch_keys=1 << 24) as s:
        budget = s.stats()["data_budget_bytes"]
        assert budget // 4 <= 1 << 24
        with pytest.raises(_lib.MmsError) as e:
            s.submit(n=budget // 4)                 # result + workspace exceed the budget
        assert e.value.code == _lib.MMS_ENOMEM
        with pytest.raises(_lib.MmsError) as e:
            s.submit(n=0)
        assert e.value.code == _lib.MMS_EINVAL
        with pytest.raises(_lib.MmsError) as e:
            s.submit(n=(1 << 24) + 1)              # above max_batch_keys
        assert e.value.code == _lib.MMS_EINVAL
        assert s.stats()["rejected"] == 2
        with pytest.raises(_lib.MmsError) as e:
            s.poll(12345)
        assert e.value.code == _lib.MMS_ENOENT
        t = s.submit(n=10)
        assert s.wait(t, 5000).status == 0
        s.release(t)
        with pytest.raises(_lib.MmsError) as e:
            s.release(t)                            # double release
        assert e.value.code == _lib.MMS_ENOENT
        with pytest.raises(_lib.MmsError) as e:
            s.release(999)
        assert e.value.code == _lib.MMS_ENOENT


def test_release_of_pending_request_is_refused(mms):
    with make(mms, max_requests=1) as s:
        a = s.submit(n=100)
        b = s.submit(n=100)                         # waits for a's release
        assert s.wait(a, 5000) is not None
        time.sleep(0.02)
        with pytest.raises(_lib.MmsError) as e:
            s.release(b)
        assert e.value.code == _lib.MMS_EINVAL
        s.release(a)
        assert s.wait(b, 5000).status == 0
        s.release(b)


def test_batches_hold_one_kind(mms):
    with make(mms, max_requests=64) as s:
        kinds = [(n, p, i) for n in (100, 3000, 70_000) for p in (False, True) for i in (False, True)]
        tickets = [(s.submit(n=n, values=p, i32=i), p, i) for n, p, i in kinds * 3]
        batches = {}
        for t, p, i in tickets:
            r = s.wait(t, 5000)
            assert r.status == 0
            batches.setdefault(r.batch, set()).add((p, i))
        assert all(len(v) == 1 for v in batches.values())
        for t, _, _ in tickets:
            s.release(t)
        assert s.stats()["used_bytes"] == 0


def test_batches_hold_one_size_class(mms):
    """A batch holds requests of one size class (ceil(log2 n) // 4: sizes
    within a factor of 16), so small requests never wait in a batch for a
    large one's sort."""
    def cls(n):
        return (max(n, 1) - 1).bit_length() // 4
    with make(mms, max_requests=64, budget=1 << 26) as s:
        sizes = [100, 900, 5000, 20_000, 70_000, 300_000, 1 << 20]
        tickets = [(s.submit(n=n), n) for n in sizes * 4]
        batches = {}
        for t, n in tickets:
            r = s.wait(t, 5000)
            assert r.status == 0
            batches.setdefault(r.batch, set()).add(cls(n))
        assert all(len(v) == 1 for v in batches.values())
        assert len(batches) >= len({cls(n) for n in sizes})
        for t, _ in tickets:
            s.release(t)


def test_shutdown_fails_queued_requests(mms):
    s = make(mms, max_requests=1)
    a = s.submit(n=100)
    s.submit(n=100)
    assert s.wait(a, 5000) is not None
    s.close()                                       # the queued one is dropped
    with pytest.raises(Exception):
        s.submit(n=5)


def test_arena_too_small_for_metadata(mms):
    with pytest.raises(_lib.MmsError) as e:
        mms.Server(budget_bytes=4096, dry_run=True, max_batch_keys=1 << 20)
    assert e.value.code == _lib.MMS_EINVAL
