"""The sort for callers that cannot allocate (mms_sort_u32_noalloc, whose
workspace is a fixed device array inside the library), called through the
C ABI and compared bit for bit with mms_sort_u32 on a caller workspace: two
calls in a row, the second smaller (the array keeps the first call's
contents), then sizes at the array's limit and past it."""
import ctypes

import numpy as np
import pytest

import mmsgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SCRATCH_BYTES = 64 << 20


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_07961_amd import _lib
    return _lib.lib()


def sort_with_workspace(lib, xd, flags):
    n = xd.numel()
    out = torch.empty_like(xd)
    wsb = lib.mms_workspace_bytes(n, flags)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=xd.device)
    s = torch.cuda.current_stream().cuda_stream
    assert lib.mms_sort_u32(ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(out.data_ptr()), n,
                            ctypes.c_void_p(ws.data_ptr() if wsb else 0), wsb, flags, ctypes.c_void_p(s)) == 0
    return out


def sort_noalloc(lib, xd, flags):
    out = torch.empty_like(xd)
    s = torch.cuda.current_stream().cuda_stream
    rc = lib.mms_sort_u32_noalloc(ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(out.data_ptr()), xd.numel(),
                                  flags, ctypes.c_void_p(s))
    assert rc == 0, lib.mms_last_error().decode()
    return out


def host(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("flags", [0, 0x2])
def test_noalloc_matches_workspace_sort(lib, flags):
    for n in [3_000_017, 70_001]:     # the second call is smaller than the first
        x = mmsgen.uniform_u32(mmsgen.seed_for(31, n % 7), n)
        xd = torch.from_numpy(x.view(np.int32)).cuda()
        got = host(sort_noalloc(lib, xd, flags))
        ref = host(sort_with_workspace(lib, xd, flags))
        assert np.array_equal(got, ref), n
        assert np.array_equal(got, oracle.sort(x, i32=bool(flags))), n


def test_noalloc_limit(lib):
    # the largest n whose workspace fits the array, then one past the limit
    lo, hi = 1, 1 << 26
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if lib.mms_workspace_bytes(mid, 0) <= SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid
    x = mmsgen.uniform_u32(mmsgen.seed_for(31, 9), lo + 1)
    xd = torch.from_numpy(x.view(np.int32)).cuda()
    got = host(sort_noalloc(lib, xd[:lo], 0))
    assert np.array_equal(got, host(sort_with_workspace(lib, xd[:lo], 0)))
    out = torch.empty_like(xd)
    rc = lib.mms_sort_u32_noalloc(ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(out.data_ptr()), lo + 1, 0,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1 and b"scratch" in lib.mms_last_error()
