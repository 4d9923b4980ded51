"""Benchmark: sort 10^8 uniform uint32 keys on one MI355X with libmms.

One step = one complete sort (base-case pass, then every partition and merge
round) of 10^8 keys drawn uniformly from [0, 2^32), read from a device
buffer and written to another, workspace preallocated.  Prints one JSON line:

  value      Gkeys/s = 10^8 / (mean time per step)
  roofline   the merge kernel (the dominant one): algorithmic bytes per launch
             (read + write of every key: 2 * 4 * n) over its mean launch time
             from HIP events on its stream, against the 8 TB/s HBM peak;
             "traffic" is the measured HBM bytes per launch from the committed
             rocprofv3 counter summary, or null when the kernel source has
             changed since the counters were taken
  cpu_baseline  the CPU oracle (sequential heap-based mergesort, 1 thread)
             timed on the same input (at most 1e8 keys), the host's core
             counts and model, and a multi-core CPU sort as context
  configs    the other workloads timed the same way (2^20 uniform keys; 1e8
             int32 keys uniform and nearly sorted with 0, 1e3, 1e6, 1e8 swaps;
             2^27 stable pairs with uniform, 16-distinct and stride-64 keys;
             1e8 uniform 64-bit keys and 2^26 64-bit pairs; the merge-path
             baseline beside the multiway sort on uniform, sorted,
             stride-64 and conflict-heavy inputs), each with its dominant
             kernel's mean launch time and fraction of the HBM peak
  paper_context  the paper's reported speedups with the GPUs they were
             measured on (context, not a target)
  batched    4096 uint32 arrays, sizes log-uniform in [2^8, 2^20]: one
             batched (segmented) sort vs 4096 plain calls on one stream
  serving    a Poisson stream of requests (sizes log-uniform in [2^10, 2^26],
             half keys-only, half pairs) at 70% of the measured saturated
             throughput through the serving loop (64 GB arena), vs the same
             trace served by a first-come first-served loop of plain calls:
             p50/p99 latency and keys/s of each

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--no-configs] [--no-batched] [--no-serving]
       one other workload instead of the headline: [--n N] [--family F]
       [--swaps S] [--i32] [--pairs] [--u64] [--mergepath]; its line names
       that workload in "metric" (Gpairs/s for pairs) and has no configs,
       batched or serving legs
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_KEYS = 10**8
N_PAIRS = 2**27
HBM_PEAK_GBS = 8000.0
METRIC = "Gkeys/s sorting 1e8 uint32, % HBM roofline; p99 latency served vs per-call"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "merge_u32_1e8_traffic.json")
KERNEL_SOURCES = ["paper_1702_07961_amd/csrc/mms_merge_keys.hip", "paper_1702_07961_amd/csrc/mms_device.h",
                  "paper_1702_07961_amd/csrc/mms_internal.h", "paper_1702_07961_amd/csrc/mms_tile_plan.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per merge launch from the committed counter summary, if current."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def host_info() -> dict:
    """Host CPU of the run: core counts and the model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def cpu_baseline(x_host, i32: bool = False):
    """The oracle (1 thread) on the workload's input, plus a multi-core CPU
    sort (libstdc++ parallel mode, all usable cores) as context."""
    import oracle
    sample = min(x_host.size, 10**8)
    xs = x_host[:sample].copy()
    t0 = time.perf_counter()
    oracle.sort(xs, i32=i32)
    dt = time.perf_counter() - t0
    rec = {"value": round(sample / dt / 1e9, 6), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
           "sample": f"first {sample} keys of the same input, sequential heap-based "
                     f"5-way mergesort, {dt:.2f} s"}
    rec["host"] = host_info()
    try:
        oracle.parallel_sort(xs[:1 << 20], i32=i32)      # warm the thread pool
        t0 = time.perf_counter()
        oracle.parallel_sort(xs, i32=i32)
        dp = time.perf_counter() - t0
        rec["parallel_context"] = {
            "value": round(sample / dp / 1e9, 6), "unit": "Gkeys/s", "threads": oracle.parallel_threads(),
            "kind": "libstdc++ parallel-mode stable sort (OpenMP), not the oracle",
            "sample": f"the same {sample} keys, {dp:.3f} s"}
    except (OSError, RuntimeError) as e:
        rec["parallel_context"] = {"error": str(e)}
    return rec


# The paper's own results (§6.4): maximum speedups of its multiway mergesort
# on conflict-heavy 4-byte integer inputs, on the GPUs it names.  Context only.
PAPER_CONTEXT = [
    {"over": "Thrust 1.8.1", "max_speedup_pct": 44.3, "gpu": "GTX 770 (Kepler)", "input": "conflict-heavy"},
    {"over": "MGPU 2.10", "max_speedup_pct": 37.6, "gpu": "GTX 770 (Kepler)", "input": "conflict-heavy"},
    {"over": "MGPU 2.10", "max_speedup_pct": 41.2, "gpu": "Tesla K40m (Kepler)", "input": "conflict-heavy"},
    {"over": "Thrust 1.8.1", "max_speedup_pct": 36.8, "gpu": "Tesla K40m (Kepler)", "input": "conflict-heavy"},
    {"over": "MGPU 2.10", "max_speedup_pct": 31.9, "gpu": "Quadro M4000 (Maxwell)", "input": "conflict-heavy"},
    {"over": "Thrust 1.8.1", "max_speedup_pct": 29.4, "gpu": "Quadro M4000 (Maxwell)", "input": "conflict-heavy"},
]


def bench_batched(mms, torch, np, mmsgen, reps: int = 5) -> dict:
    """One batched sort of 4096 arrays vs 4096 plain calls (same stream)."""
    import ctypes
    sizes = mmsgen.loguniform_sizes(mmsgen.seed_for(4, 0), 4096, 8, 20).astype(np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = int(off[-1])
    x = torch.from_numpy(mmsgen.uniform_u32(mmsgen.seed_for(4, 2), total).view(np.int32)).cuda()
    out = torch.empty_like(x)
    ws = torch.empty(mms.segmented_workspace_bytes(off), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    mms.segmented_sort(x, off, out_keys=out, workspace=ws, i32=False)     # captures the graph
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        mms.segmented_sort(x, off, out_keys=out, workspace=ws, i32=False)
    b.record(stream)
    torch.cuda.synchronize()
    seg_ms = a.elapsed_time(b) / reps
    seg_out = out.clone()

    lib = mms._lib.lib()
    wsp = torch.empty(max(mms.workspace_bytes(int(sizes.max())), 256), dtype=torch.uint8, device="cuda")
    xp, op, wp, sp = x.data_ptr(), out.data_ptr(), wsp.data_ptr(), stream.cuda_stream
    wbytes = wsp.numel()
    calls = [(xp + 4 * int(o), op + 4 * int(o), int(n)) for o, n in zip(off[:-1], sizes)]

    def plain_all():
        for i_ptr, o_ptr, n in calls:
            rc = lib.mms_sort_u32(i_ptr, o_ptr, n, wp, wbytes, 0, sp)
            if rc:
                mms._lib.check(rc)
    plain_all()
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(2):
        plain_all()
    b.record(stream)
    torch.cuda.synchronize()
    plain_ms = a.elapsed_time(b) / 2
    if not torch.equal(seg_out, out):
        raise RuntimeError("batched and plain results differ")
    del ctypes
    import oracle
    nseg = 256
    xh = x[:int(off[nseg])].cpu().numpy().view(np.uint32)
    t0 = time.perf_counter()
    oracle.sort_segments(xh, off[:nseg + 1])
    dt = time.perf_counter() - t0
    cpu = {"value": round(int(off[nseg]) / dt / 1e9, 6), "unit": "Gkeys/s", "cores": 1,
           "sample": f"first {nseg} segments ({int(off[nseg])} keys) of the same batch, {dt:.2f} s"}
    return {"workload": "4096 uint32 arrays, sizes log-uniform in [2^8, 2^20], uniform keys",
            "cpu_oracle": cpu,
            "total_keys": total,
            "batched_ms": round(seg_ms, 3), "batched_gkeys_per_s": round(total / seg_ms / 1e6, 3),
            "plain_calls_ms": round(plain_ms, 3), "plain_calls_gkeys_per_s": round(total / plain_ms / 1e6, 3),
            "speedup": round(plain_ms / seg_ms, 3)}


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q))


def bench_serving(mms, torch, np, mmsgen, count: int = 2100, warm: int = 100, rho: float = 0.7,
                  arena_bytes: int = 64 << 30) -> dict:
    """Continuous batching through the serving loop vs a per-call FIFO loop
    on the same Poisson arrival trace."""
    import queue
    import threading
    POOL = 1 << 26
    pool_k = torch.from_numpy(mmsgen.uniform_u32(mmsgen.seed_for(5, 0), POOL).view(np.int32)).cuda()
    pool_v = torch.arange(POOL, dtype=torch.int32, device="cuda")
    sizes = mmsgen.loguniform_sizes(mmsgen.seed_for(5, 1), count, 10, 26).astype(np.int64)
    pairs = mmsgen.unit_doubles(mmsgen.seed_for(5, 2), count) < 0.5
    offs = (mmsgen.unit_doubles(mmsgen.seed_for(5, 3), count) * (POOL - sizes + 1)).astype(np.int64)
    unit_arrivals = mmsgen.poisson_arrivals(mmsgen.seed_for(5, 4), count, 1.0)
    torch.cuda.synchronize()

    def req(i):
        o, n = int(offs[i]), int(sizes[i])
        return pool_k[o:o + n], (pool_v[o:o + n] if pairs[i] else None)

    srv = mms.Server(budget_bytes=arena_bytes)
    try:
        # saturated throughput: a burst of requests submitted at once
        burst = list(range(min(256, count)))
        tk = [srv.submit(*req(i), stream=None) for i in burst]
        rs = [srv.wait(t) for t in tk]
        for t in tk:
            srv.release(t)
        x_sat = sum(int(sizes[i]) for i in burst) / (
            (max(r.t_done_us for r in rs) - min(r.t_submit_us for r in rs)) * 1e-6)
        mean_n = mmsgen.loguniform_mean(10, 26)
        rate = rho * x_sat / mean_n
        arrivals = unit_arrivals / rate

        # served: a submitting thread on the arrival schedule, a collector thread
        q = queue.Queue()
        results = [None] * count
        late = np.zeros(count)
        call = np.zeros(count)

        def collect():
            for _ in range(count):
                i, t = q.get()
                results[i] = srv.wait(t)
                srv.release(t)
        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for i in range(count):
            due = t0 + arrivals[i]
            while True:
                d = due - time.perf_counter()
                if d <= 0:
                    break
                time.sleep(d if d > 2e-3 else 0)
            t_call = time.perf_counter()
            q.put((i, srv.submit(*req(i), stream=None)))
            call[i] = time.perf_counter() - t_call
            late[i] = t_call - due
        th.join()
        st = srv.stats()
    finally:
        srv.close()
    meas = results[warm:]
    lat = [(r.t_done_us - r.t_submit_us) / 1e3 for r in meas]
    span_s = (max(r.t_done_us for r in meas) - min(r.t_submit_us for r in meas)) * 1e-6
    keys = int(sizes[warm:].sum())
    served = {"p50_ms": round(_pct(lat, 50), 3), "p99_ms": round(_pct(lat, 99), 3),
              "gkeys_per_s": round(keys / span_s / 1e9, 3),
              "mean_batch_requests": round(float(np.mean([r.batch_requests for r in meas])), 2),
              "batches": int(st["batches"]), "peak_arena_GB": round(st["peak_used_bytes"] / 1e9, 2),
              "submit_lateness_p99_ms": round(_pct(late[warm:] * 1e3, 99), 3),
              "submit_call_p99_ms": round(_pct(call[warm:] * 1e3, 99), 3)}

    # per-call FIFO: one plain sort per request on one stream, in arrival order
    nmax = int(sizes.max())
    outk = torch.empty(nmax, dtype=torch.int32, device="cuda")
    outv = torch.empty(nmax, dtype=torch.int32, device="cuda")
    ws = torch.empty(max(mms.workspace_bytes(nmax, pairs=True), 256), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    done = np.zeros(count)
    t0 = time.perf_counter()
    for i in range(count):
        due = t0 + arrivals[i]
        while True:
            d = due - time.perf_counter()
            if d <= 0:
                break
            time.sleep(d if d > 2e-3 else 0)
        k, v = req(i)
        n = k.numel()
        if v is None:
            mms.sort(k, out=outk[:n], i32=False, workspace=ws, stream=stream)
        else:
            mms.sort_pairs(k, v, out_keys=outk[:n], out_values=outv[:n], i32=False, workspace=ws,
                           stream=stream)
        stream.synchronize()
        done[i] = time.perf_counter() - t0
    lat_pc = (done - arrivals)[warm:] * 1e3
    pc_span = done[-1] - arrivals[warm]
    per_call = {"p50_ms": round(_pct(lat_pc, 50), 3), "p99_ms": round(_pct(lat_pc, 99), 3),
                "gkeys_per_s": round(keys / pc_span / 1e9, 3)}
    return {"workload": "Poisson arrivals, sizes log-uniform in [2^10, 2^26], half keys-only uint32, "
                        "half (uint32, uint32) pairs, 64 GB arena",
            "requests": count - warm, "warmup_requests": warm, "offered_load": rho,
            "saturated_gkeys_per_s": round(x_sat / 1e9, 3), "rate_per_s": round(rate, 1),
            "served": served, "per_call_fifo": per_call,
            "p99_per_call_over_served": round(per_call["p99_ms"] / served["p99_ms"], 3)}


def make_input(mmsgen, np, family: str, n: int, swaps: int, workload: int = 2):
    seed = mmsgen.seed_for(workload, 0)
    if family == "nearly":
        return mmsgen.nearly_sorted_u32(seed, n, swaps)
    return mmsgen.family(family, seed, n)


KIND_OF = {"tile_sort": "k_tile_sort", "partition": "k_corank_tiles", "merge": "k_merge"}


def measure(mms, torch, np, x_host, *, pairs: bool, i32: bool, steps: int, warmup: int,
            kind: str = "mms") -> dict:
    """Time `steps` sorts of x_host (already generated) after `warmup`
    untimed ones; per-kernel HIP-event timing of the same steps; checks that
    the last result is sorted (and stable for pairs) on the device.  kind:
    "mms" (32-bit keys), "mms64" (64-bit keys, x_host uint64) or "mergepath"
    (the merge-path baseline)."""
    n = int(x_host.size)
    wide = kind == "mms64"
    x = torch.from_numpy(x_host.view(np.int64 if wide else np.int32)).cuda()
    out = torch.empty_like(x)
    v = torch.arange(n, dtype=torch.int64 if wide else torch.int32, device="cuda") if pairs else None
    vout = torch.empty_like(v) if pairs else None
    if kind == "mergepath":
        need = mms.plan(n, mergepath=True).workspace_bytes
    else:
        need = mms.workspace_bytes(n, pairs=pairs, keys64=wide)
    ws = torch.empty(max(1, need), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        if kind == "mergepath":
            mms.sort_mergepath(x, out=out, i32=i32, workspace=ws)
        elif wide and pairs:
            mms.sort_pairs64(x, v, out_keys=out, out_values=vout, i64=i32, workspace=ws)
        elif wide:
            mms.sort64(x, out=out, i64=i32, workspace=ws)
        elif pairs:
            mms.sort_pairs(x, v, out_keys=out, out_values=vout, i32=i32, workspace=ws)
        else:
            mms.sort(x, out=out, i32=i32, workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # the timed steps: HIP events bracket the merge launches only (each timed
    # launch costs two event records on the stream), for the roofline figure
    mms.timing_reset()
    mms.timing_enable(True, kinds=["merge"])
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        step()
    stop.record(stream)
    torch.cuda.synchronize()
    mms.timing_enable(False)
    timed = mms.timing_read()
    ms_per_step = start.elapsed_time(stop) / steps
    # the per-phase breakdown from a few more steps with every launch timed
    b_steps = max(1, min(steps, 5))
    mms.timing_reset()
    mms.timing_enable(True)
    for _ in range(b_steps):
        step()
    torch.cuda.synchronize()
    mms.timing_enable(False)
    times = mms.timing_read()

    if wide:
        o = out if i32 else out ^ (-(2**63))      # unsigned order as signed order
        ok = bool((o[1:] >= o[:-1]).all())
    else:
        o = out.to(torch.int64)
        if not i32:
            o = o & 0xFFFFFFFF
        ok = bool((o[1:] >= o[:-1]).all())
    if pairs:
        tie = o[1:] == o[:-1]
        ok = ok and bool((vout[1:][tie] > vout[:-1][tie]).all())
    del o
    if not ok:
        raise RuntimeError("bench.py: output is not sorted")
    s_bytes = (8 if wide else 4) * (2 if pairs else 1)
    alg_bytes = 2 * s_bytes * n        # one read and one write of every element per launch
    phases = {k: {"launches_per_step": c // b_steps, "ms_per_step": round(t / b_steps, 4)}
              for k, (c, t) in times.items() if c}
    dom = max((k for k in ("tile_sort", "partition", "merge") if times[k][0]), key=lambda k: times[k][1])
    m_launches, m_ms = timed["merge"]                  # launches of the timed steps
    merge_avg_ms = m_ms / max(1, m_launches)
    d_launches, d_ms = timed[dom] if timed[dom][0] else times[dom]
    dom_avg = d_ms / max(1, d_launches)
    plan = mms.plan(n, pairs=pairs, i32=i32 and not wide, keys64=wide, mergepath=kind == "mergepath")
    del x, out, v, vout, ws
    return {"n": n, "ms_per_step": round(ms_per_step, 4), "gkeys_per_s": round(n / (ms_per_step * 1e-3) / 1e9, 4),
            "base_tile": plan.tile, "fanout": plan.fanout, "merge_tile": plan.merge_tile, "passes": plan.passes,
            "phases": phases,
            "dominant": {"kernel": KIND_OF[dom], "avg_launch_ms": round(dom_avg, 4),
                         "alg_bytes_per_launch": alg_bytes,
                         "frac": round(alg_bytes / (dom_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "merge_avg_launch_ms": round(merge_avg_ms, 4) if m_launches else None,
            "merge_frac": round(alg_bytes / (merge_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if m_launches else None,
            "all_passes_alg_GBps": round(plan.passes * alg_bytes / (ms_per_step * 1e-3) / 1e9, 1)}


def copy_probe(mms, torch, n: int) -> float:
    """Streaming copy of n uint32 (read + write), GB/s from HIP events."""
    a = torch.empty(n, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    mms.copy(a, b)
    torch.cuda.synchronize()
    mms.timing_reset()
    mms.timing_enable(True)
    for _ in range(10):
        mms.copy(a, b)
    mms.timing_enable(False)
    c_launch, c_ms = mms.timing_read()["copy"]
    return 2 * 4 * n / (c_ms / c_launch * 1e-3) / 1e9


def other_configs(mms, torch, np, mmsgen, steps: int, warmup: int) -> dict:
    """The other workloads, each timed the same way as the headline."""
    import oracle
    res = {}
    x = mmsgen.uniform_u32(mmsgen.seed_for(1, 0), 1 << 20)
    res["keys_2^20_uniform_u32"] = measure(mms, torch, np, x, pairs=False, i32=False, steps=steps * 5,
                                           warmup=warmup)
    x = mmsgen.uniform_u32(mmsgen.seed_for(2, 2), N_KEYS)
    res["keys_1e8_uniform_i32"] = measure(mms, torch, np, x, pairs=False, i32=True, steps=steps, warmup=warmup)
    for k, tag in ((0, "0"), (10**3, "1e3"), (10**6, "1e6"), (10**8, "1e8")):
        x = mmsgen.nearly_sorted_u32(mmsgen.seed_for(2, 1), N_KEYS, k)
        res[f"keys_1e8_nearly_sorted_i32_k{tag}"] = measure(mms, torch, np, x, pairs=False, i32=True,
                                                            steps=steps, warmup=warmup)
    for fam, name in (("uniform", "uniform"), ("sixteen", "16_distinct"), ("stride64", "stride64")):
        x = mmsgen.family(fam, mmsgen.seed_for(3, 0), N_PAIRS)
        r = measure(mms, torch, np, x, pairs=True, i32=False, steps=steps, warmup=warmup)
        if fam == "uniform":
            sample = 1 << 24
            xs = x[:sample].copy()
            vs = np.arange(sample, dtype=np.uint32)
            t0 = time.perf_counter()
            oracle.sort(xs, vs)
            dt = time.perf_counter() - t0
            r["cpu_oracle"] = {"value": round(sample / dt / 1e9, 6), "unit": "Gpairs/s", "cores": 1,
                               "sample": f"first {sample} pairs of the same input, {dt:.2f} s"}
        res[f"pairs_2^27_{name}"] = r
    # 8-byte keys (the paper's second workload)
    x = mmsgen.splitmix64(mmsgen.seed_for(15, 60), N_KEYS)
    res["keys64_1e8_uniform_u64"] = measure(mms, torch, np, x, pairs=False, i32=False, steps=steps,
                                            warmup=warmup, kind="mms64")
    x = mmsgen.splitmix64(mmsgen.seed_for(15, 61), N_PAIRS // 2)
    res["pairs64_2^26_uniform_u64"] = measure(mms, torch, np, x, pairs=True, i32=False, steps=steps,
                                              warmup=warmup, kind="mms64")
    del x
    res["mergepath_vs_mms"] = mergepath_comparison(mms, torch, np, mmsgen, steps=steps, warmup=warmup)
    return res


def mergepath_comparison(mms, torch, np, mmsgen, steps: int, warmup: int) -> dict:
    """The merge-path baseline (pairwise, per-thread serial merges) and the
    multiway mergesort on the same inputs: uniform, sorted, stride-64 and the
    conflict-heavy input built against the baseline's 15 outputs per thread,
    at 3840 * 2^14 keys (the adversary needs a power-of-two tile count)."""
    n = mmsgen.MERGEPATH_ITEMS * 256 * 2**14
    res = {"n": n}
    for fam in ("uniform", "sorted", "stride64", "mp_adversary"):
        x = mmsgen.family(fam, mmsgen.seed_for(16, 0), n)
        a = measure(mms, torch, np, x, pairs=False, i32=False, steps=steps, warmup=warmup, kind="mergepath")
        b = measure(mms, torch, np, x, pairs=False, i32=False, steps=steps, warmup=warmup)
        res[fam] = {"mergepath_ms": a["ms_per_step"], "mergepath_gkeys_per_s": a["gkeys_per_s"],
                    "mergepath_merge_avg_launch_ms": a["merge_avg_launch_ms"],
                    "mms_ms": b["ms_per_step"], "mms_gkeys_per_s": b["gkeys_per_s"],
                    "mms_merge_avg_launch_ms": b["merge_avg_launch_ms"]}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N_KEYS)
    ap.add_argument("--family", default="uniform",
                    choices=["uniform", "nearly", "sixteen", "stride64", "permutation", "sorted", "reverse",
                             "mp_adversary"])
    ap.add_argument("--swaps", type=int, default=0, help="random pair swaps of the nearly-sorted family")
    ap.add_argument("--i32", action="store_true", help="int32 keys (signed order)")
    ap.add_argument("--pairs", action="store_true", help="stable (key, index) pairs")
    ap.add_argument("--u64", action="store_true", help="64-bit keys (uniform family only; with --pairs, "
                    "(uint64, uint64) pairs)")
    ap.add_argument("--mergepath", action="store_true",
                    help="time the merge-path baseline instead of the multiway sort (keys only)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-sort comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop comparison")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sort runs on a single MI355X and this build "
              "has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import mmsgen
    import paper_1702_07961_amd as mms

    n = args.n
    if args.mergepath and args.pairs:
        print("bench.py: the merge-path baseline sorts keys only", file=sys.stderr)
        sys.exit(2)
    if args.u64 and (args.family != "uniform" or args.i32 or args.mergepath):
        print("bench.py: --u64 takes uniform unsigned keys and the multiway sort only", file=sys.stderr)
        sys.exit(2)
    headline = (args.family == "uniform" and not args.i32 and not args.pairs and not args.mergepath and
                not args.u64 and n == N_KEYS)
    if args.u64:
        x_host = mmsgen.splitmix64(mmsgen.seed_for(15, 61 if args.pairs else 60), n)
    else:
        x_host = make_input(mmsgen, np, args.family, n, args.swaps)
    m = measure(mms, torch, np, x_host, pairs=args.pairs, i32=args.i32, steps=args.steps, warmup=args.warmup,
                kind="mergepath" if args.mergepath else ("mms64" if args.u64 else "mms"))
    copy_gbs = copy_probe(mms, torch, n)

    fam = args.family + (f" ({args.swaps} swaps)" if args.family == "nearly" else "")
    workload = (f"plain {'stable pair' if args.pairs else 'keys-only'} sort of {n} {fam} "
                f"{'uint64' if args.u64 else 'int32' if args.i32 else 'uint32'} keys, ascending"
                + (", merge-path baseline" if args.mergepath else ""))
    if headline:
        workload = "plain sort of 1e8 uniform uint32 keys, keys only, ascending"
    alg_bytes = m["dominant"]["alg_bytes_per_launch"]
    merge_avg_ms = m["merge_avg_launch_ms"] or float("nan")
    achieved = alg_bytes / (merge_avg_ms * 1e-3) / 1e9
    unit = "Gpairs/s" if args.pairs else "Gkeys/s"
    rec = {
        # the headline run reports the headline metric; another workload names itself
        "metric": METRIC if headline else f"{unit} of a {workload}",
        "value": m["gkeys_per_s"],
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("u64" + ("+u64 pairs" if args.pairs else "")) if args.u64 else
                 (("i32" if args.i32 else "u32") + ("+u32 pairs" if args.pairs else "")),
        "data": "synthetic",
        "config": {"workload": workload,
                   "n": n, "input": f"{fam}, splitmix64 seed 0x4D4D5320",
                   "base_tile": m["base_tile"], "fanout": m["fanout"], "merge_tile": m["merge_tile"],
                   "passes": m["passes"]},
        "roofline": {"bound": "hbm", "kernel": "k_merge", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic() if headline else None,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": round(merge_avg_ms, 4)},
        "detail": {"phases": m["phases"], "all_passes_alg_GBps": m["all_passes_alg_GBps"],
                   "copy_probe_GBps": round(copy_gbs, 1)},
        "paper_context": PAPER_CONTEXT,
    }
    if not args.no_cpu and not args.pairs and not args.u64:
        rec["cpu_baseline"] = cpu_baseline(x_host, args.i32)
    del x_host
    if headline and not args.no_configs:
        rec["configs"] = other_configs(mms, torch, np, mmsgen, steps=10, warmup=2)
    if headline and not args.no_batched:
        rec["batched"] = bench_batched(mms, torch, np, mmsgen)
    if headline and not args.no_serving:
        rec["serving"] = bench_serving(mms, torch, np, mmsgen)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
