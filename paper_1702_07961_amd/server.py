"""Python front end of the serving loop (``mms_server_*``, ``mms_submit``,
``mms_poll``, ``mms_wait``, ``mms_release`` in include/mms.h).

The arena is one torch allocation owned by the :class:`Server`; results are
returned as tensor views into it and stay valid until :meth:`Server.release`.
All admission, batching and sorting happens in libmms.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import _lib

# a 256-byte-aligned address that the dry-run server is given as its arena;
# the library never dereferences it in that mode
_DRY_ARENA = 1 << 40


@dataclass
class Result:
    ticket: int
    status: int
    n: int
    keys: object            # torch view into the arena (None in dry-run mode)
    values: object
    t_submit_us: float
    t_admit_us: float
    t_launch_us: float
    t_done_us: float
    batch: int
    batch_requests: int
    stream_index: int

    @property
    def latency_us(self) -> float:
        return self.t_done_us - self.t_submit_us


class Server:
    """Admits sort requests by arena budget and serves them in coalesced
    batches on ``num_streams`` streams (the library creates them unless
    ``streams`` lists torch streams)."""

    def __init__(self, budget_bytes: int = 64 << 30, *, streams=None, max_inflight: int = 0,
                 max_requests: int = 0, max_batch_requests: int = 0, max_batch_keys: int = 0,
                 dry_run: bool = False, device=None):
        self._lib = _lib.lib()
        self._torch = None
        self._arena = None
        cfg = _lib.MmsServerCfg()
        if dry_run:
            cfg.d_arena = _DRY_ARENA
            cfg.flags = _lib.MMS_SERVER_DRY_RUN
            self._arena_ptr = _DRY_ARENA
        else:
            import torch
            self._torch = torch
            self._arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device=device or "cuda")
            cfg.d_arena = self._arena.data_ptr()
            self._arena_ptr = self._arena.data_ptr()
        cfg.arena_bytes = int(budget_bytes)
        streams = list(streams or [])
        if len(streams) > _lib.MMS_SERVER_MAX_STREAMS:
            raise ValueError(f"at most {_lib.MMS_SERVER_MAX_STREAMS} streams")
        for i, st in enumerate(streams):
            cfg.streams[i] = st.cuda_stream
        self._streams = streams          # keep the torch streams alive
        cfg.num_streams = len(streams)
        cfg.max_inflight = max_inflight
        cfg.max_requests = max_requests
        cfg.max_batch_requests = max_batch_requests
        cfg.max_batch_keys = max_batch_keys
        h = ctypes.c_void_p()
        _lib.check(self._lib.mms_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._dry = dry_run
        self._inputs = {}               # ticket -> input tensors kept alive until done

    # -- requests ---------------------------------------------------------
    def submit(self, keys=None, values=None, *, i32: bool = False, n: int | None = None, stream=None) -> int:
        """Queue a sort of ``keys`` (and ``values``, stable by key); returns
        the ticket.  The input is read after the work already enqueued on
        ``stream`` (default: torch's current stream).  In dry-run mode pass
        ``n`` (and values=True for pairs) instead of tensors."""
        r = _lib.MmsRequest()
        pairs = values is not None and values is not False
        r.flags = (_lib.MMS_PAIRS if pairs else 0) | (_lib.MMS_KEY_I32 if i32 else 0)
        if self._dry:
            r.n = int(n)
            r.d_keys = 0x1000
            r.d_vals = 0x2000 if pairs else None
        else:
            torch = self._torch
            for t, name in ((keys, "keys"), (values if pairs else None, "values")):
                if t is None:
                    continue
                if not t.is_cuda or t.dtype not in (torch.int32, torch.uint32) or not t.is_contiguous():
                    raise ValueError(f"{name} must be a contiguous int32/uint32 device tensor")
            if pairs and values.numel() != keys.numel():
                raise ValueError("keys and values differ in length")
            r.n = keys.numel()
            r.d_keys = keys.data_ptr()
            r.d_vals = values.data_ptr() if pairs else None
            st = stream if stream is not None else torch.cuda.current_stream()
            r.stream = st.cuda_stream
        t = ctypes.c_uint64()
        _lib.check(self._lib.mms_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        if not self._dry:
            self._inputs[t.value] = (keys, values if pairs else None)
        return t.value

    def _result(self, ticket, code, res) -> Result:
        keys = values = None
        if code == _lib.MMS_OK and not self._dry:
            torch = self._torch
            words = self._arena.view(torch.int32)
            k0 = (res.d_keys - self._arena_ptr) // 4
            keys = words[k0:k0 + res.n]
            if res.d_vals:
                v0 = (res.d_vals - self._arena_ptr) // 4
                values = words[v0:v0 + res.n]
        return Result(ticket, code, res.n, keys, values, res.t_submit_us, res.t_admit_us, res.t_launch_us,
                      res.t_done_us, res.batch, res.batch_requests, res.stream_index)

    def poll(self, ticket: int):
        """The :class:`Result` when the request is done, else None."""
        res = _lib.MmsResult()
        code = self._lib.mms_poll(self._h, int(ticket), ctypes.byref(res))
        if code == _lib.MMS_PENDING:
            return None
        self._inputs.pop(int(ticket), None)
        _lib.check(code)
        return self._result(int(ticket), code, res)

    def wait(self, ticket: int, timeout_ms: int = -1):
        """Block until the request is done (None on timeout)."""
        res = _lib.MmsResult()
        code = self._lib.mms_wait(self._h, int(ticket), int(timeout_ms), ctypes.byref(res))
        if code == _lib.MMS_PENDING:
            return None
        self._inputs.pop(int(ticket), None)
        _lib.check(code)
        return self._result(int(ticket), code, res)

    def release(self, ticket: int, stream=None) -> None:
        """Return the result's arena space.  Work already enqueued on
        ``stream`` (readers of the result) finishes before it is reused."""
        sp = stream.cuda_stream if stream is not None else None
        _lib.check(self._lib.mms_release(self._h, int(ticket), sp))

    def stats(self) -> dict:
        st = _lib.MmsServerStats()
        _lib.check(self._lib.mms_server_get_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in st._fields_}

    def close(self) -> None:
        if self._h:
            _lib.check(self._lib.mms_server_destroy(self._h))
            self._h = None
            self._inputs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
