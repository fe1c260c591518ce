#!/usr/bin/env python3
"""Benchmark of the massive-PRNG hot path on one MI355X.

Headline (one JSON line on stdout): the plain generator writing 2^26 streams
x 256 iterations of uint64 (128 GiB of output per step) into HBM. A step is
one rngx_generate call over that whole grid (seeding is done once before the
warm-up). `value` is output GB/s over the timed steps; `roofline` reports the
generation kernel's own average duration from HIP events recorded on its
launch stream, against the 8 TB/s HBM3E peak; `cpu_baseline` times the CPU
oracle on a bounded sample of the same workload.

Run: python bench.py [--steps K] [--warmup W]. Only one GPU is measured.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RNG output GB/s (% HBM peak), batched vs plain; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0
GIB = 1 << 30
# The library's default plain launches (block, chunks, non-temporal,
# pace_gbs); u32 block 0 = chosen by size.
LIB_DEFAULT_U64 = (512, 2, 1, 7000)
LIB_DEFAULT_U32 = (0, 0, 0, 0)
# The request server's launch configuration for batches above 2^23 values
# (the grouped order), used by the in-pool batched comparator.
SERVER_LARGE_BATCH_CFG = dict(values_per_lane=16, waves_per_block=4, blocks=0, use_graph=False,
                              row_values=16, run_items=0, per_item=False, group=32,
                              group_steps=8, pace_gbs=6250)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def launch_key(launch):
    """What selects the kernel code of a plain launch: chunks, non-temporal
    stores, scheduled or not (block and the schedule's rate are launch
    parameters of the same code)."""
    return (int(launch["chunks"]), int(bool(launch["nontemporal"])),
            int(launch["pace_gbs"] > 0))


def counter_traffic(launch):
    """HBM bytes per launch of the headline kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (one `machine:` line per
    launch measured), or None if the kernel source changed since those
    counters were taken or none of them ran the kernel code `launch` selects."""
    import hashlib
    src = os.path.join(ROOT, "paper_1609_01257_amd", "csrc", "kernels.hip")
    summary = os.path.join(ROOT, "profiles", "gen_kernel_u64_2p26x256.md")
    try:
        lines = [l for l in open(summary) if l.startswith("machine:")]
    except OSError:
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in lines:
        kv = dict(tok.split("=", 1) for tok in line.split()[1:])
        try:
            b, c, nt, pace = (int(x) for x in kv.get("launch", "").split(","))
        except ValueError:
            continue
        taken = {"block": b, "chunks": c, "nontemporal": nt, "pace_gbs": pace}
        if kv.get("kernels_hip_sha256_16") == digest and launch_key(taken) == launch_key(launch):
            return int(kv["traffic_bytes_per_launch"])
    return None


def kernel_avg_s(stats, name):
    for agg_name, count, abs_s, _ in stats["agg"]:
        if agg_name == name:
            return abs_s / count, count
    raise RuntimeError("no %s events were profiled" % name)


def plain_run(torch, rngx, seed, n, iters, u32, warmup, steps, out=None):
    """Time `steps` generate calls of `iters` iterations over n streams
    (into `out` if given, else into a new buffer)."""
    rngx.init(seed, n)
    if out is None:
        out = torch.empty(n * iters, dtype=torch.int32 if u32 else torch.int64, device="cuda")
    gen = rngx.generate_u32 if u32 else rngx.generate
    for _ in range(warmup):
        gen(iters, out)
    torch.cuda.synchronize()
    rngx.profile_start()
    t0 = time.perf_counter()
    for _ in range(steps):
        gen(iters, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = rngx.profile_stats()
    avg, count = kernel_avg_s(st, "RNG_KERNEL")
    assert count == steps
    del out
    torch.cuda.empty_cache()
    esize = 4 if u32 else 8
    out_bytes = esize * n * iters
    return {
        "wall_s": t1 - t0,
        "out_gbs": out_bytes * steps / (t1 - t0) / 1e9,
        "kernel_avg_s": avg,
        "out_bytes_per_launch": out_bytes,
        "alg_bytes_per_launch": out_bytes + 16 * n,
        "kernel_gbs": (out_bytes + 16 * n) / avg / 1e9,
    }


def sweep(torch, rngx, reps):
    """HBM roofline sweep: n in 2^20..2^26 x 256 iterations x seeds 1..4 x
    u64 and u32 (32 runs), output kept in HBM; one output buffer per size
    and word type, shared by its four seeds. Each buffer is first timed at
    the library's default launch (seed 1, `default_gbs`), then the launch autotuner
    picks a configuration on it (`launch`, with row schedules among the
    candidates) and the four seeds run with that one."""
    from paper_1609_01257_amd import inputs
    rows = []
    iters = inputs.ROOFLINE_ITERS
    saved = (rngx.get_launch(False), rngx.get_launch(True))
    try:
        for n in inputs.ROOFLINE_N:
            for u32 in (False, True):
                out = torch.empty(n * iters, dtype=torch.int32 if u32 else torch.int64,
                                  device="cuda")
                rngx.set_launch(u32, *(LIB_DEFAULT_U32 if u32 else LIB_DEFAULT_U64))
                base = plain_run(torch, rngx, inputs.ROOFLINE_SEEDS[0], n, iters, u32, 1, reps,
                                 out=out)
                # At least about 8 GiB of timed output per candidate.
                tune_reps = max(2, (8 * GIB) // (n * iters * (4 if u32 else 8)))
                tune = rngx.autotune_plain(iters, out, reps=tune_reps, u32=u32)
                for seed in inputs.ROOFLINE_SEEDS:
                    r = plain_run(torch, rngx, seed, n, iters, u32, 1, reps, out=out)
                    rows.append({"n": n, "seed": seed, "dtype": "u32" if u32 else "u64",
                                 "kernel_gbs": round(r["kernel_gbs"], 1),
                                 "out_gbs": round(r["out_gbs"], 1),
                                 "frac_hbm": round(r["kernel_gbs"] / HBM_PEAK_GBS, 4),
                                 "launch": tune["best"],
                                 "default_gbs": round(base["kernel_gbs"], 1)})
                    log("sweep", rows[-1])
                del out
                torch.cuda.empty_cache()
    finally:
        rngx.set_launch(False, **saved[0])
        rngx.set_launch(True, **saved[1])
    return rows


def streaming(torch, rngx):
    """Paper-shaped streaming: 4,194,304 streams, seed 42, 2,000 iterations of
    32 MiB, generation and device-to-host copies overlapped on two streams
    through two device buffers and two pinned host slots (no host consumer,
    as in the paper's runs with output sent to the null device)."""
    from paper_1609_01257_amd import inputs
    cfg = inputs.STREAMING
    n, steps = cfg["n"], cfg["iters"]
    dev0 = torch.empty(n, dtype=torch.int64, device="cuda")
    dev1 = torch.empty(n, dtype=torch.int64, device="cuda")
    host = torch.empty(2 * n, dtype=torch.int64, pin_memory=True)
    rngx.init(cfg["seed"], n)
    rngx.stream_to_host(16, 1, dev0, dev1, host, 2)          # warm-up
    rngx.init(cfg["seed"], n)                                # restarts the profile window
    t0 = time.perf_counter()
    rngx.stream_to_host(steps, 1, dev0, dev1, host, 2)
    t1 = time.perf_counter()
    st = rngx.profile_stats()
    log(rngx.profile())
    agg = {name: (c, a) for name, c, a, _ in st["agg"]}
    step_bytes = 8 * n
    # The same run with event logging off: what the start and end events of
    # every kernel and copy cost the pipeline.
    rngx.init(cfg["seed"], n)
    rngx.profile_enable(False)
    try:
        t2 = time.perf_counter()
        rngx.stream_to_host(steps, 1, dev0, dev1, host, 2)
        t3 = time.perf_counter()
    finally:
        rngx.profile_enable(True)
    # Practical host-link ceiling: back-to-back pinned copies of one step.
    s = torch.cuda.Stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        for _ in range(5):
            host[:n].copy_(dev0, non_blocking=True)
        e0.record(s)
        reps = 100
        for _ in range(reps):
            host[:n].copy_(dev0, non_blocking=True)
        e1.record(s)
    s.synchronize()
    peak = step_bytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del dev0, dev1, host
    torch.cuda.empty_cache()
    reads = agg.get("READ_BUFFER", (0, 0.0))
    kern = agg.get("RNG_KERNEL", (0, 0.0))
    return {
        "workload": "4,194,304 streams, seed 42, 2,000 iterations x 32 MiB to pinned host",
        "wall_s": round(t1 - t0, 4),
        "host_link_gbs": round(step_bytes * steps / (t1 - t0) / 1e9, 2),
        "host_link_gbs_unprofiled": round(step_bytes * steps / (t3 - t2) / 1e9, 2),
        "read_gbs": round(step_bytes * reads[0] / reads[1] / 1e9, 2) if reads[1] else None,
        "pinned_copy_peak_gbs": round(peak, 2),
        "pcie5_x16_theoretical_gbs": 63.0,
        "rng_kernel_s": round(kern[1], 6), "rng_kernel_count": kern[0],
        "read_buffer_s": round(reads[1], 6), "read_buffer_count": reads[0],
        "overlap_s": round(st["overlap_s"], 6), "eff_s": round(st["eff_s"], 6),
        "elapsed_s": round(st["elapsed_s"], 6), "device_pct": round(st["device_pct"], 2),
    }


def batched(torch, rngx, steps):
    """Batched ragged streams: 4,096 streams with seeds from default_rng(1609),
    lengths log-uniform in [2^10, 2^24), one persistent launch per step,
    replayed from a HIP graph, launch configuration from the autotuner;
    compared with the plain kernel writing the same number of bytes, into
    another buffer and into the batched output buffer itself."""
    from paper_1609_01257_amd import inputs
    r = inputs.batched_requests()
    reqs = rngx.make_reqs(r.seeds, r.gids, r.offsets, r.lengths)
    out = torch.empty(r.total, dtype=torch.int64, device="cuda")
    rngx.set_batch_cfg(256, 4, 0, True)
    tune = rngx.autotune_batch(reqs, out, reps=2)
    log("autotune best:", tune["best"], "%.3f ms" % tune["best_ms"])
    rngx.generate_batch(reqs, out)
    torch.cuda.synchronize()
    rngx.profile_start()
    t0 = time.perf_counter()
    for _ in range(steps):
        rngx.generate_batch(reqs, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = rngx.profile_stats()
    avg, count = kernel_avg_s(st, "BATCH_KERNEL")
    # The persistent grid (S = 256, 8 waves per compute unit, runs of one
    # item) on the same table, whatever the autotuner picked.
    tuned = rngx.get_batch_cfg()
    rngx.set_batch_cfg(256, 4, 0, True, 16, 1, False)
    rngx.generate_batch(reqs, out)
    torch.cuda.synchronize()
    rngx.profile_start()
    for _ in range(steps):
        rngx.generate_batch(reqs, out)
    torch.cuda.synchronize()
    pavg, _ = kernel_avg_s(rngx.profile_stats(), "BATCH_KERNEL")
    rngx.set_batch_cfg(**tuned)
    # The plain generator writing the batched output buffer itself (2^24
    # streams x floor(total / 2^24) iterations): same memory, so the ratio
    # does not depend on where either buffer landed in HBM.
    it_in = r.total // (1 << 24)
    same = plain_run(torch, rngx, 1, 1 << 24, it_in, False, 1, steps,
                     out=out[: (1 << 24) * it_in])
    del out
    torch.cuda.empty_cache()
    nbytes = 8 * r.total
    # Plain generator at equal output bytes: 2^24 streams x ceil(total / 2^24) iterations.
    n_eq = 1 << 24
    it_eq = -(-r.total // n_eq)
    plain = plain_run(torch, rngx, 1, n_eq, it_eq, False, 1, steps)
    res = {
        "workload": "4,096 streams, seeds from default_rng(1609), lengths floor(2^U[10,24)), "
                    "%d values (%.2f GB) per launch" % (r.total, nbytes / 1e9),
        "out_gbs": round(nbytes * steps / (t1 - t0) / 1e9, 1),
        "kernel_avg_ms": round(avg * 1e3, 4),
        "kernel_gbs": round(nbytes / avg / 1e9, 1),
        "frac_hbm": round(nbytes / avg / 1e9 / HBM_PEAK_GBS, 4),
        "autotune_best": tune["best"],
        "autotune_candidates": len(tune["tried"]),
        "persistent_s256": {"kernel_avg_ms": round(pavg * 1e3, 4),
                            "kernel_gbs": round(nbytes / pavg / 1e9, 1),
                            "frac_hbm": round(nbytes / pavg / 1e9 / HBM_PEAK_GBS, 4)},
        "plain_equal_bytes": {"n_states": n_eq, "iters": it_eq,
                              "kernel_gbs": round(plain["kernel_gbs"], 1),
                              "out_gbs": round(plain["out_gbs"], 1)},
    }
    res["batched_vs_plain"] = round(res["kernel_gbs"] / plain["kernel_gbs"], 4)
    res["plain_same_buffer"] = {"n_states": 1 << 24, "iters": it_in,
                                "kernel_gbs": round(same["kernel_gbs"], 1)}
    res["batched_vs_plain_same_buffer"] = round(res["kernel_gbs"] / same["kernel_gbs"], 4)
    return res


def serving(torch, rngx, seconds, plain_gbs):
    """Serving: 2^20 resident streams, a 16 GB pool with memory-based
    admission, 4 streams, batches of up to 2,048 requests with at most 2 in
    flight, Poisson arrivals at 2k / 10k / 50k req/s (stream id uniform,
    length log-uniform in [2^12, 2^22)), results released on completion;
    latency from each request's scheduled arrival to its completion. Then a
    saturation run (a pre-filled backlog) for throughput, compared with the
    batched kernel writing the same requests into the same pool without the
    server (batches of the server's mean size, back to back)."""
    from paper_1609_01257_amd import inputs
    pool = torch.empty(16 * 10**9, dtype=torch.uint8, device="cuda")
    rngx.serve_start(1609, 1 << 20, pool, 4, 2048)
    res = {"workload": "2^20 resident streams, 16 GB pool, lengths floor(2^U[12,22)), "
                       "Poisson arrivals, %.0f s per rate" % seconds, "rates": []}
    try:
        # seconds = 0: the saturation run alone (for profiling it).
        for rate in (2000.0, 10000.0, 50000.0) if seconds > 0 else ():
            t, g, L = inputs.serving_arrivals(rate, seconds)
            st = rngx.serve_run_trace(t, g, L, timeout_s=seconds + 120)
            row = {"rate_req_s": rate, "requests": st["completed"],
                   "offered_gbs": round(8 * float(L.sum()) / seconds / 1e9, 2),
                   "gbs": round(st["gbs"], 2),
                   "p50_us": round(st["lat_p50_us"], 1), "p99_us": round(st["lat_p99_us"], 1),
                   "max_us": round(st["lat_max_us"], 1),
                   "wait_p99_us": round(st["wait_p99_us"], 1),
                   "submit_lag_p50_us": round(st["lag_p50_us"], 1),
                   "submit_lag_p99_us": round(st["lag_p99_us"], 1),
                   "launch_p50_us": round(st["launch_p50_us"], 1),
                   "exec_p50_us": round(st["exec_p50_us"], 1),
                   "mean_batch": round(st["mean_batch_requests"], 2),
                   "admission_stalls": st["admission_stalls"]}
            res["rates"].append(row)
            log("serving:", row)
        # Saturation: a backlog of requests all arriving at once, served three
        # times (one run lasts ~50 ms and varies by a few per cent); the
        # median run is reported.
        _, g, L = inputs.serving_arrivals(50000.0, 1.0, seed=4242)
        t = np.zeros(len(g))
        runs = sorted((rngx.serve_run_trace(t, g, L, timeout_s=600) for _ in range(3)),
                      key=lambda r: r["gbs"])
        st = runs[1]
        res["saturation"] = {"requests": st["completed"], "gb": round(st["bytes"] / 1e9, 2),
                             "gbs": round(st["gbs"], 1),
                             "gbs_runs": [round(r["gbs"], 1) for r in runs],
                             "mean_batch": round(st["mean_batch_requests"], 1),
                             "admission_stalls": st["admission_stalls"],
                             "p99_us": round(st["lat_p99_us"], 1)}
        res["saturation"]["served_vs_plain"] = round(st["gbs"] / plain_gbs, 4)
        rngx.serve_stop()
        # The same requests, in consecutive batches of the server's mean
        # batch size, each written by the batched kernel into the pool in the
        # schedule the server uses for large batches (the grouped order,
        # SERVER_LARGE_BATCH_CFG). Its rate over the kernels' own durations (HIP events on
        # their stream) is what the server would reach with no overhead of
        # its own: the ratio isolates the server from kernel speed and from
        # where the pool lies in HBM.
        per = max(1, int(round(st["mean_batch_requests"])))
        chunks = []
        for a in range(0, len(L), per):
            b = min(len(L), a + per)
            while 8 * int(L[a:b].sum()) > pool.numel():
                b -= 1
            chunks.append(rngx.make_reqs(np.full(b - a, 1609, dtype=np.uint64), g[a:b],
                                         np.zeros(b - a), L[a:b]))
        words = pool.view(torch.int64)
        # Each batch lands after the previous one, wrapping at the end of
        # the pool, as the server's ring places them.
        places, off = [], 0
        for c in chunks:
            size = int(c["length"].sum())
            if off + size > words.numel():
                off = 0
            places.append(words[off:off + size])
            off += (size + 31) & ~31     # 256-byte aligned, as the server's pool ring places them
        tuned = rngx.get_batch_cfg()
        rngx.set_batch_cfg(**SERVER_LARGE_BATCH_CFG)
        try:
            rngx.generate_batch(chunks[0], places[0])      # warm-up
            torch.cuda.synchronize()
            rngx.profile_start()
            t0 = time.perf_counter()
            for c, dst in zip(chunks, places):
                rngx.generate_batch(c, dst)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            kavg, kcount = kernel_avg_s(rngx.profile_stats(), "BATCH_KERNEL")
            assert kcount == len(chunks)
        finally:
            rngx.set_batch_cfg(**tuned)
        bip = 8 * float(L.sum()) / (kavg * kcount) / 1e9
        res["saturation"]["batched_in_pool_gbs"] = round(bip, 1)
        res["saturation"]["batched_in_pool_wall_gbs"] = round(8 * float(L.sum()) / dt / 1e9, 1)
        res["saturation"]["batched_in_pool_batches"] = len(chunks)
        res["saturation"]["served_vs_batched_in_pool"] = round(st["gbs"] / bip, 4)
        # The plain kernel writing the pool itself (2^22 states x 476
        # iterations = 15.97 GB per launch): the same memory the served
        # batches wrote, so the ratio does not depend on where either
        # buffer landed in HBM.
        n_pool, it_pool = 1 << 22, 476
        pp = plain_run(torch, rngx, 1, n_pool, it_pool, False, 1, 5,
                       out=pool.view(torch.int64)[: n_pool * it_pool])
        res["saturation"]["plain_in_pool_gbs"] = round(pp["kernel_gbs"], 1)
        res["saturation"]["served_vs_plain_in_pool"] = round(st["gbs"] / pp["kernel_gbs"], 4)
        log("serving saturation:", res["saturation"])
    finally:
        rngx.serve_stop()
        del pool
        torch.cuda.empty_cache()
    return res


def host_description():
    """CPU model, the oracle's compiler and flags (for the CPU baseline)."""
    import subprocess
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cc = subprocess.run(["gcc", "--version"], capture_output=True, text=True).stdout
        cc = cc.splitlines()[0].strip()
    except (OSError, IndexError):
        cc = "gcc"
    return {"cpu_model": model, "host_cpus": os.cpu_count(), "compiler": cc,
            "flags": "-std=c99 -O2"}


def cpu_baseline(n_total, iters, min_seconds=10.0, single_seconds=5.0):
    """The CPU oracle (plain C, sequential definition) on a bounded sample of
    the headline workload: T threads (the box's share of 16 cores, at most),
    each computing a contiguous slice of 2^17 work-items for all iterations
    with the oracle's gid-range entry, repeated until at least `min_seconds`
    have passed; plus the same oracle on one thread."""
    import concurrent.futures as cf
    import oracle
    lib = oracle.lib()
    threads = max(1, min(16, os.cpu_count() or 1))
    per = 1 << 17
    bufs = [np.empty(per * iters, dtype=np.uint64) for _ in range(threads)]

    def one(t):
        z = lib.oracle_generate_range(1, t * per, (t + 1) * per, 0, iters, bufs[t].ctypes.data)
        if z:
            raise AssertionError("oracle produced zero values")
        return bufs[t].nbytes

    nbytes, passes = 0, 0
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < min_seconds:
            nbytes += sum(ex.map(one, range(threads)))
            passes += 1
        dt = time.perf_counter() - t0
    mt = nbytes / dt / 1e9
    n1, d1, b1 = 0, 0.0, 0
    while d1 < single_seconds:
        t1 = time.perf_counter()
        b1 += one(0)
        d1 += time.perf_counter() - t1
        n1 += 1
    del bufs
    res = {"value": round(mt, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": "first %d of %d work-items x %d iterations (u64, %.1f GiB), one "
                     "contiguous slice of %d work-items per thread, computed %d times in "
                     "%.1f s" % (threads * per, n_total, iters, threads * per * iters * 8 / GIB,
                                 per, passes, dt),
           "single_thread_gbs": round(b1 / d1 / 1e9, 3)}
    res.update(host_description())
    return res


def trace_summary(path, match, split_ms, queues=None):
    """Device occupancy of the kernels whose names contain `match`, from a
    rocprofv3 kernel trace (the SQLite results database): the dispatches are
    cut into runs wherever the device stays idle longer than `split_ms`; per
    run, the span from the first start to the last end, the busy time (union
    of the kernels' intervals), the idle gaps between busy periods, and the
    mean number of kernels in flight. `queues`: only dispatches on these
    hardware queue ids (all if None)."""
    import sqlite3
    db = sqlite3.connect(path)
    cols = [r[1] for r in db.execute("pragma table_info(kernels)")]
    end = "end" if "end" in cols else "start + duration"
    rows = db.execute('select name, start, %s, queue_id from kernels order by start' % end).fetchall()
    ks = [(int(a), int(b), q) for nm, a, b, q in rows
          if match in nm and (queues is None or q in queues)]
    runs, cur, reach = [], [], 0
    for a, b, q in ks:
        if cur and a - reach > split_ms * 1e6:
            runs.append(cur)
            cur = []
        reach = max(reach, b) if cur else b
        cur.append((a, b, q))
    if cur:
        runs.append(cur)
    out = []
    for r in runs:
        span = max(b for _, b, _ in r) - r[0][0]
        busy, gaps, s0, e0 = 0, [], r[0][0], r[0][1]
        for a, b, _ in r[1:]:
            if a > e0:
                busy += e0 - s0
                gaps.append(a - e0)
                s0, e0 = a, b
            else:
                e0 = max(e0, b)
        busy += e0 - s0
        gaps.sort()
        pct = lambda p: gaps[min(len(gaps) - 1, int(p * len(gaps)))] / 1e3 if gaps else 0.0
        out.append({"kernels": len(r), "queues": sorted({q for _, _, q in r}),
                    "span_ms": round(span / 1e6, 3), "busy_ms": round(busy / 1e6, 3),
                    "busy_frac": round(busy / span, 4) if span else 1.0,
                    "gaps": len(gaps), "gap_total_ms": round(sum(gaps) / 1e6, 3),
                    "gap_p50_us": round(pct(0.5), 2), "gap_p99_us": round(pct(0.99), 2),
                    "gap_max_us": round(gaps[-1] / 1e3, 2) if gaps else 0.0,
                    "kernel_sum_ms": round(sum(b - a for a, b, _ in r) / 1e6, 3),
                    "mean_in_flight": round(sum(b - a for a, b, _ in r) / busy, 3) if busy else 0})
    return out


def trace_overlap(path, name_a, name_b):
    """From a rocprofv3 kernel trace: for kernels whose names contain
    `name_a` and `name_b`, their counts per hardware queue, total durations,
    and the time kernels of the first kind ran while a kernel of the second
    kind was running (overlap with the union of the second kind's
    intervals)."""
    import bisect
    import sqlite3
    db = sqlite3.connect(path)
    cols = [r[1] for r in db.execute("pragma table_info(kernels)")]
    end = "end" if "end" in cols else "start + duration"
    rows = db.execute("select name, start, %s, queue_id from kernels order by start" % end).fetchall()
    A = [(int(a), int(b), q) for nm, a, b, q in rows if name_a in nm]
    B = [(int(a), int(b), q) for nm, a, b, q in rows if name_b in nm]
    merged = []
    for a, b, _ in B:
        if merged and a <= merged[-1][1]:
            merged[-1][1] = max(merged[-1][1], b)
        else:
            merged.append([a, b])
    starts = [m[0] for m in merged]
    overlap = 0
    for a, b, _ in A:
        i = max(0, bisect.bisect_right(starts, a) - 1)
        while i < len(merged) and merged[i][0] < b:
            overlap += max(0, min(b, merged[i][1]) - max(a, merged[i][0]))
            i += 1

    def per_queue(K):
        out = {}
        for _, _, q in K:
            out[str(q)] = out.get(str(q), 0) + 1
        return out
    return {"a": name_a, "a_kernels": len(A), "a_queues": per_queue(A),
            "a_total_ms": round(sum(b - a for a, b, _ in A) / 1e6, 3),
            "b": name_b, "b_kernels": len(B), "b_queues": per_queue(B),
            "b_total_ms": round(sum(b - a for a, b, _ in B) / 1e6, 3),
            "overlap_ms": round(overlap / 1e6, 3)}


def trace_stats(path):
    """Per (kernel name, hardware queue) of a rocprofv3 kernel trace: the
    number of dispatches and their total, mean, p50, p99 and largest
    durations in microseconds."""
    import sqlite3
    db = sqlite3.connect(path)
    cols = [r[1] for r in db.execute("pragma table_info(kernels)")]
    end = "end" if "end" in cols else "start + duration"
    groups = {}
    for nm, a, b, q in db.execute("select name, start, %s, queue_id from kernels" % end):
        groups.setdefault((nm, q), []).append(int(b) - int(a))
    out = []
    for (nm, q), d in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        d.sort()
        pick = lambda p: d[min(len(d) - 1, int(p * len(d)))] / 1e3
        short = nm.replace("(anonymous namespace)::", "").split("(")[0]
        out.append({"kernel": short, "queue": q, "calls": len(d),
                    "total_us": round(sum(d) / 1e3, 1), "mean_us": round(sum(d) / len(d) / 1e3, 2),
                    "p50_us": round(pick(0.5), 2), "p99_us": round(pick(0.99), 2),
                    "max_us": round(d[-1] / 1e3, 2)})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-sweep", action="store_true", help="skip the size/dtype sweep")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="duration of each Poisson serving run (0: only the saturation run)")
    ap.add_argument("--headline-only", action="store_true",
                    help="run only the headline kernel (for profiling)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched ragged-stream step (for profiling)")
    ap.add_argument("--launch", metavar="B,C,NT,PACE",
                    type=lambda v: tuple(int(x) for x in v.split(",")),
                    help="plain launch configuration (block, chunks, non-temporal, pace_gbs) "
                         "of the headline instead of the autotuner's choice, or of "
                         "--plain-shape")
    ap.add_argument("--sweep-only", action="store_true",
                    help="run only the roofline sweep with its per-buffer autotuning")
    ap.add_argument("--streaming-only", action="store_true",
                    help="run only the paper-shaped streaming pipeline (for profiling)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving runs (for profiling)")
    ap.add_argument("--plain-shape", type=int, nargs=2, metavar=("N_STATES", "ITERS"),
                    help="run only the plain generator at this shape (for profiling)")
    ap.add_argument("--u32", action="store_true", help="with --plain-shape: 32-bit output")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 16 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--placement-probe", action="store_true",
                    help="only time one launch shape into three separately allocated buffers")
    ap.add_argument("--trace-summary", metavar="RESULTS_DB",
                    help="only summarise device occupancy in a rocprofv3 kernel trace")
    ap.add_argument("--trace-kernels", default="batch",
                    help="with --trace-summary: kernels whose names contain this text")
    ap.add_argument("--trace-split-ms", type=float, default=5.0,
                    help="with --trace-summary: idle time that separates two runs")
    ap.add_argument("--trace-queues", type=lambda v: {int(x) for x in v.split(",")},
                    help="with --trace-summary: comma-separated hardware queue ids")
    ap.add_argument("--trace-overlap", nargs=3, metavar=("RESULTS_DB", "NAME_A", "NAME_B"),
                    help="only report how long kernels named NAME_A ran while NAME_B kernels ran")
    ap.add_argument("--trace-stats", metavar="RESULTS_DB",
                    help="only list dispatch counts and durations per kernel and queue")
    args = ap.parse_args()
    if args.trace_stats:
        for row in trace_stats(args.trace_stats):
            print(json.dumps(row), flush=True)
        return
    if args.trace_overlap:
        print(json.dumps(trace_overlap(*args.trace_overlap)), flush=True)
        return
    if args.trace_summary:
        for i, run in enumerate(trace_summary(args.trace_summary, args.trace_kernels,
                                              args.trace_split_ms, args.trace_queues)):
            print(json.dumps(dict(run=i, **run)), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        log("bench.py measures a single GPU: the generator shards across GPUs with no "
            "communication, so only --gpus 1 is supported.")
        sys.exit(2)

    import torch
    from paper_1609_01257_amd import rngx

    torch.cuda.set_device(0)
    if args.copy_probe:
        # A plain copy of known size: reads and writes exactly 16 GiB each, so
        # HBM byte counters read on it give their scale factor.
        src = torch.ones(2 << 30, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d bytes written" % (src.numel() * 8, dst.numel() * 8))
        return
    if args.placement_probe:
        # One launch shape (u32, 2^26 states x 256 iterations, 64 GiB of
        # output) into three buffers from separate allocations: the write
        # rate of the row-ordered store stream depends on where a buffer
        # landed in HBM, reproducibly per buffer.
        # Each buffer is timed with the unscheduled launch (block 512, 2
        # chunks, normal stores) and with the library's default (scheduled).
        n, iters = 1 << 26, 256
        rngx.init(1, n)
        bufs = [torch.empty(n * iters, dtype=torch.int32, device="cuda") for _ in range(3)]
        res = []
        st = torch.cuda.current_stream()
        launches = {"unscheduled 512,2,0,0": (512, 2, 0, 0), "default": LIB_DEFAULT_U32}
        for i, buf in enumerate(bufs):
            entry = {"buffer": i}
            for name, cfg in launches.items():
                rngx.set_launch(True, *cfg)
                rngx.generate_u32(iters, buf)
                torch.cuda.synchronize()
                rates = []
                for _ in range(3):
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record(st)
                    rngx.generate_u32(iters, buf)
                    b.record(st)
                    b.synchronize()
                    rates.append(round(n * iters * 4 / (a.elapsed_time(b) * 1e-3) / 1e9, 1))
                log("placement probe: buffer %d at 0x%x, %s: %s GB/s" % (i, buf.data_ptr(), name,
                                                                         rates))
                entry[name] = rates
            res.append(entry)
        rngx.set_launch(True, *LIB_DEFAULT_U32)
        rngx.shutdown()
        print(json.dumps({"placement_probe": res}), flush=True)
        return
    if args.plain_shape:
        n_s, it_s = args.plain_shape
        if args.launch:
            rngx.set_launch(args.u32, *args.launch)
        log("plain %s, n=%d, iters=%d, launch %s" % ("u32" if args.u32 else "u64", n_s, it_s,
                                                     rngx.get_launch(args.u32)))
        launch = rngx.get_launch(args.u32)
        r = plain_run(torch, rngx, 1, n_s, it_s, args.u32, args.warmup, args.steps)
        r["frac_hbm"] = r["kernel_gbs"] / HBM_PEAK_GBS
        log("plain:", r)
        rngx.shutdown()
        print(json.dumps({"plain": r, "n_states": n_s, "iters": it_s, "u32": args.u32,
                          "launch": launch}), flush=True)
        return
    if args.batched_only:
        rngx.init(1, 64)          # opens the profiling window the step is timed in
        res = batched(torch, rngx, args.steps)
        log("batched:", res)
        rngx.shutdown()
        print(json.dumps({"batched": res}), flush=True)
        return
    if args.sweep_only:
        res = sweep(torch, rngx, 3)
        rngx.shutdown()
        print(json.dumps({"sweep": res}), flush=True)
        return
    if args.streaming_only:
        res = streaming(torch, rngx)
        log("streaming:", res)
        rngx.shutdown()
        print(json.dumps({"streaming": res}), flush=True)
        return
    if args.serving_only:
        # The plain kernel at the batched table's size, as in the full run.
        plain = plain_run(torch, rngx, 1, 1 << 24, 438, False, 1, 5)
        res = serving(torch, rngx, args.serve_seconds, plain["kernel_gbs"])
        rngx.shutdown()
        print(json.dumps({"serving": res}), flush=True)
        return
    n, iters, seed = 1 << 26, 256, 1
    out = torch.empty(n * iters, dtype=torch.int64, device="cuda")
    default_launch = rngx.get_launch(False)
    base = tune = None
    if args.launch:
        rngx.set_launch(False, *args.launch)
    else:
        # The library's default launch, then its launch autotuner on the
        # headline buffer (before the timed steps; the timed steps then run
        # the chosen configuration).
        log("headline: default launch", default_launch)
        base = plain_run(torch, rngx, seed, n, iters, False, 1, 3, out=out)
        log("headline, default launch:", base)
        rngx.init(seed, n)
        tune = rngx.autotune_plain(iters, out, reps=2)
        log("autotune best:", tune["best"], "%.3f ms" % tune["best_ms"])
    launch = rngx.get_launch(False)
    log("headline: plain u64, n=2^26, iters=256, warmup=%d steps=%d, launch %s"
        % (args.warmup, args.steps, launch))
    head = plain_run(torch, rngx, seed, n, iters, False, args.warmup, args.steps, out=out)
    del out
    torch.cuda.empty_cache()
    log("headline:", head)
    result = {
        "metric": METRIC,
        "value": round(head["out_gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["wall_s"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain generator, 2^26 streams x 256 iterations of uint64 "
                               "(128 GiB per step), seed 1, output kept in HBM",
                   "n_states": n, "iters": iters, "seed": seed,
                   "launch": launch,
                   "launch_source": "--launch" if args.launch else
                   "rngx_autotune_plain on the headline buffer before the timed steps "
                   "(%d candidates)" % len(tune["tried"])},
        "roofline": {"bound": "hbm",
                     "achieved": round(head["kernel_gbs"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(head["kernel_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": counter_traffic(launch),
                     "kernel": "gen_paced_kernel<u64>" if launch["pace_gbs"] else "gen_kernel<u64>",
                     "kernel_avg_ms": round(head["kernel_avg_s"] * 1e3, 4),
                     "alg_bytes_per_launch": head["alg_bytes_per_launch"]},
    }
    if base is not None:
        result["default_launch"] = {"launch": default_launch,
                                    "kernel_gbs": round(base["kernel_gbs"], 1),
                                    "frac_hbm": round(base["kernel_gbs"] / HBM_PEAK_GBS, 4)}
    if not args.headline_only:
        log("u32 headline shape")
        out32 = torch.empty(n * iters, dtype=torch.int32, device="cuda")
        if not args.launch:
            rngx.init(seed, n)
            rngx.autotune_plain(iters, out32, reps=2, u32=True)
        h32 = plain_run(torch, rngx, seed, n, iters, True, 1, max(3, args.steps // 4), out=out32)
        del out32
        torch.cuda.empty_cache()
        result["u32"] = {"out_gbs": round(h32["out_gbs"], 1),
                         "kernel_gbs": round(h32["kernel_gbs"], 1),
                         "frac_hbm": round(h32["kernel_gbs"] / HBM_PEAK_GBS, 4),
                         "launch": rngx.get_launch(True)}
        log("scrambled variant, headline shape")
        rngx.set_scrambler(rngx.SCRAMBLE_STAR)
        try:
            hs = plain_run(torch, rngx, seed, n, iters, False, 1, max(3, args.steps // 4))
        finally:
            rngx.set_scrambler(rngx.SCRAMBLE_NONE)
        result["scrambled"] = {"out_gbs": round(hs["out_gbs"], 1),
                               "kernel_gbs": round(hs["kernel_gbs"], 1),
                               "frac_hbm": round(hs["kernel_gbs"] / HBM_PEAK_GBS, 4),
                               "vs_plain": round(hs["kernel_gbs"] / head["kernel_gbs"], 4)}
        if not args.no_sweep:
            result["sweep"] = sweep(torch, rngx, 3)
        log("batched ragged streams")
        result["batched"] = batched(torch, rngx, max(3, args.steps // 4))
        log("batched:", result["batched"])
        log("serving")
        result["serving"] = serving(torch, rngx, args.serve_seconds,
                                    result["batched"]["plain_equal_bytes"]["kernel_gbs"])
        log("streaming (two-stream device-to-host pipeline)")
        result["streaming"] = streaming(torch, rngx)
        log("streaming:", result["streaming"])
    rngx.shutdown()
    if not args.no_cpu_baseline and not args.headline_only:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(n, iters)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
