"""Autotuner of the sort's run-time parameters (§6.2 tunes the fan-out K and
the number of workers per platform; here per size bucket on this GPU).

For every size bucket n = 2^b it times the plain keys-only sort of n uniform
uint32 keys under each candidate (fan-out K, merge output tile, merge kernel
shape) with HIP events and keeps the fastest; with those fixed it then times
each base-case shape (keys per lane x waves, and with it the base tile of
2048, 4096 or 8192 keys).  Key-value sorts get entries of their own: the
stable sort of n (uint32 key, index) pairs under every fan-out and key-value
base shape (8 x 4, 8 x 8).  The table is written as JSON.
The package loads that table into the library (mms_set_tuning) the first
time the library is used.

    python -m paper_1702_07961_amd.autotune [--out FILE] [--min-log2 8]
                                            [--max-log2 27] [--reps 5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(PKG, "tuning_mi355x.json")

FANOUTS = [2, 4, 8, 16]   # 32 would need more than 64 probe lanes in the partition
TILES = [2048, 4096, 6144, 7168, 7424, 8192]
VARIANTS = [0, 1, 2, 3, 4]   # 4: the minBlockHeap merge
# keys per lane x waves: 8x4, 4x8, 16x2 (2048-key tiles), 8x8, 16x4 (4096), 8x16, 16x8 (8192)
BASES = [0, 1, 2, 3, 4, 5, 6]
PAIR_BASES = [0, 3]        # key-value base cases: 8x4, 8x8
MMS_PAIRS = 0x1


def candidates(log2n: int):
    """Every (K, Tout, variant) to time for n = 2^log2n (a single tile has
    no merge round, so nothing to choose)."""
    if (1 << log2n) <= 2048:
        yield 16, 8192, 0
        return
    for K in FANOUTS:
        for T in TILES:
            for v in VARIANTS:
                yield K, T, v


def time_sort(mms, torch, x, out, ws, reps: int) -> float:
    stream = torch.cuda.current_stream()
    mms.sort(x, out=out, i32=False, workspace=ws)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        mms.sort(x, out=out, i32=False, workspace=ws)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def time_pairs(mms, torch, x, v, ok, ov, ws, reps: int) -> float:
    stream = torch.cuda.current_stream()
    mms.sort_pairs(x, v, out_keys=ok, out_values=ov, i32=False, workspace=ws)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        mms.sort_pairs(x, v, out_keys=ok, out_values=ov, i32=False, workspace=ws)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_pairs(mms, torch, x_all, min_log2: int, max_log2: int, reps: int, log=print) -> list:
    """Key-value entries: every fan-out and key-value base shape per bucket."""
    v_all = torch.arange(x_all.numel(), dtype=torch.int32, device="cuda")
    ok_all, ov_all = torch.empty_like(x_all), torch.empty_like(v_all)
    entries = []
    for b in range(min_log2, max_log2 + 1):
        n = 1 << b
        x, v, ok, ov = x_all[:n], v_all[:n], ok_all[:n], ov_all[:n]
        best = None
        for K in FANOUTS:
            for base in PAIR_BASES:
                mms.set_tuning([(64, K, 3840, 0, base, MMS_PAIRS)])
                ws = torch.empty(max(mms.workspace_bytes(n, pairs=True), 256), dtype=torch.uint8, device="cuda")
                ms = time_pairs(mms, torch, x, v, ok, ov, ws, max(reps, int(2e6 // n)))
                if best is None or ms < best[0]:
                    best = (ms, K, base)
        ms, K, base = best
        mms.set_tuning([(64, K, 3840, 0, base, MMS_PAIRS)])
        ws = torch.empty(max(mms.workspace_bytes(n, pairs=True), 256), dtype=torch.uint8, device="cuda")
        mms.sort_pairs(x, v, out_keys=ok, out_values=ov, i32=False, workspace=ws)
        kk = ok.to(torch.int64) & 0xFFFFFFFF
        if not bool((kk[1:] >= kk[:-1]).all()):
            raise RuntimeError(f"tuned key-value sort of 2^{b} is not sorted")
        entries.append({"max_log2_n": b, "fanout": K, "merge_tile": 3840, "variant": 0, "base": base,
                        "ms": round(ms, 5), "gpairs_per_s": round(n / ms / 1e6, 3)})
        log(f"pairs 2^{b}: K={K} base={base} {ms:.4f} ms ({n / ms / 1e6:.2f} Gpairs/s)")
    return entries


def tune(min_log2: int = 8, max_log2: int = 27, reps: int = 5, log=print, keys_from: dict | None = None) -> dict:
    """The whole table; with keys_from (a table) only the key-value entries
    are timed and the keys-only entries are taken from it."""
    import numpy as np
    import torch

    import mmsgen
    import paper_1702_07961_amd as mms

    n_max = 1 << max_log2
    x_all = torch.from_numpy(mmsgen.uniform_u32(mmsgen.seed_for(6, 0), n_max).view(np.int32)).cuda()
    out_all = torch.empty_like(x_all)
    entries = list(keys_from["entries"]) if keys_from else []
    for b in range(min_log2, max_log2 + 1) if not keys_from else ():
        n = 1 << b
        x, out = x_all[:n], out_all[:n]
        best = None
        for K, T, v in candidates(b):
            mms.set_tuning([(64, K, T, v)])
            ws_bytes = mms.workspace_bytes(n)
            ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device="cuda")
            r = max(reps, int(2e6 // n))
            ms = time_sort(mms, torch, x, out, ws, r)
            if best is None or ms < best[0]:
                best = (ms, K, T, v)
        ms, K, T, v = best
        base = BASES[0]
        for bs in BASES[1:]:
            mms.set_tuning([(64, K, T, v, bs)])
            ws = torch.empty(max(mms.workspace_bytes(n), 256), dtype=torch.uint8, device="cuda")
            ms_b = time_sort(mms, torch, x, out, ws, max(reps, int(2e6 // n)))
            if ms_b < ms:
                ms, base = ms_b, bs
        # the fastest candidate must still sort
        mms.set_tuning([(64, K, T, v, base)])
        ws = torch.empty(max(mms.workspace_bytes(n), 256), dtype=torch.uint8, device="cuda")
        mms.sort(x, out=out, i32=False, workspace=ws)
        o = out.to(torch.int64) & 0xFFFFFFFF
        if not bool((o[1:] >= o[:-1]).all()):
            raise RuntimeError(f"tuned sort of 2^{b} is not sorted")
        entries.append({"max_log2_n": b, "fanout": K, "merge_tile": T, "variant": v, "base": base,
                        "ms": round(ms, 5), "gkeys_per_s": round(n / ms / 1e6, 3)})
        log(f"2^{b}: K={K} Tout={T} variant={v} base={base} {ms:.4f} ms ({n / ms / 1e6:.2f} Gkeys/s)")
    pairs_entries = tune_pairs(mms, torch, x_all, min_log2, max_log2, reps, log)
    mms.set_tuning([])
    props = torch.cuda.get_device_properties(0)
    return {"device": props.name, "gcn_arch": getattr(props, "gcnArchName", ""),
            "cus": props.multi_processor_count, "created": time.strftime("%Y-%m-%d %H:%M:%S"),
            "method": "plain sort of 2^b uniform uint32 keys (entries) and stable sort of 2^b "
                      "(uint32 key, index) pairs (pairs_entries), HIP-event mean over reps",
            "entries": entries, "pairs_entries": pairs_entries}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--min-log2", type=int, default=8)
    ap.add_argument("--max-log2", type=int, default=27)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--pairs-only", action="store_true",
                    help="time the key-value entries only; keep the keys-only entries of --out")
    args = ap.parse_args(argv)
    keys_from = None
    if args.pairs_only:
        with open(args.out) as f:
            keys_from = json.load(f)
    table = tune(args.min_log2, args.max_log2, args.reps, log=lambda s: print(s, flush=True), keys_from=keys_from)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"wrote {args.out}", file=sys.stderr)


if __name__ == "__main__":
    main()
