"""GPU parity of the merge-path baseline (pairwise merges, per-thread serial
merges in LDS; the kind of sort §6.4 compares against) through the C ABI
against the oracle, element by element: sizes around its 3840-key tile and
many merge passes, ragged tails, every input family including the
conflict-heavy one built against it, unsigned and signed keys."""
import numpy as np
import pytest

import mmsgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TILE = 3840
SIZES = [1, 2, 15, 16, 255, 3839, TILE, TILE + 1, 2 * TILE - 1, 2 * TILE + 1, 7 * TILE + 13, 64 * TILE + 5,
         99_991, 1 << 20, 3_000_017]


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


@pytest.mark.parametrize("n", SIZES)
def test_mergepath_sizes(mms, n):
    x = mmsgen.uniform_u32(mmsgen.seed_for(16, n % 11), n)
    assert np.array_equal(host(mms.sort_mergepath(dev(x), i32=False)), oracle.sort(x))
    assert np.array_equal(host(mms.sort_mergepath(dev(x), i32=True)), oracle.sort(x, i32=True))


@pytest.mark.parametrize("family", ["sorted", "reverse", "equal", "sixteen", "nearly", "stride64", "mp_adversary"])
def test_mergepath_families(mms, family):
    n = TILE * 2**7
    x = mmsgen.family(family, mmsgen.seed_for(16, 20), n, swaps=n // 100)
    assert np.array_equal(host(mms.sort_mergepath(dev(x), i32=False)), oracle.sort(x))


def test_mergepath_plan(mms):
    p = mms.plan(TILE * 2**10 + 1, mergepath=True)
    assert (p.tile, p.fanout, p.rounds) == (TILE, 2, 11)
