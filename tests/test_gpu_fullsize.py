"""Full-size GPU parity: every value of the benchmark's workloads, at their
real sizes and in the launch configurations the benchmark times, compared
element by element with the CPU oracle.

- Plain roofline grid: 2^20, 2^22, 2^24 and 2^26 work-items x 256 iterations
  x seeds 1-4 x u64 and u32 (up to 128 GiB per run), plus the scrambled
  variant at the headline shape.
- Batched: the 4,096-stream table (58.7 GB) in the default, autotuned,
  persistent and one-wave-per-item launch schedules, request by request.
- Streaming: all 2,000 steps of 32 MiB of the paper-shaped pipeline, in
  both copy modes, are compared in tests/test_gpu_stream.py.
- Serving: two seconds of the 50k req/s Poisson trace; every request's
  device checksum served in the mix equals the one served alone, and the
  first 2,000 requests are compared in full with the oracle.

The device outputs are copied to host memory in blocks and checked by
tests/helpers/parity.c on host threads (see tests/parity.py). The oracle
produces its values sequentially; nothing here takes an expected value from
the library.
"""
import threading
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1609_01257_amd import inputs, rngx
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def checker(oracle):
    parity.build(force=False)
    yield
    parity._pinned.clear()


def _free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _say(msg):
    print(msg, flush=True)


ROOFLINE = [(n, seed, u32) for n in inputs.ROOFLINE_N for seed in inputs.ROOFLINE_SEEDS
            for u32 in (False, True)]


@pytest.mark.parametrize("n,seed,u32", ROOFLINE,
                         ids=["n%d-s%d-%s" % (n, s, "u32" if u else "u64") for n, s, u in ROOFLINE])
def test_roofline_grid_full(n, seed, u32):
    iters = inputs.ROOFLINE_ITERS
    _say("roofline grid n=%d seed=%d %s" % (n, seed, "u32" if u32 else "u64"))
    rngx.init(seed, n)
    out = torch.empty(iters * n, dtype=torch.int32 if u32 else torch.int64, device="cuda")
    (rngx.generate_u32 if u32 else rngx.generate)(iters, out)
    res = parity.compare_plain_device(out, n, iters, seed,
                                      word=parity.WORD_U32 if u32 else parity.WORD_U64)
    del out
    rngx.shutdown()
    _free()
    assert res["mismatches"] == 0, res
    assert res["values"] == n * iters


def test_scrambled_headline_full():
    n, iters, seed = 1 << 26, 256, 1
    rngx.init(seed, n)
    out = torch.empty(iters * n, dtype=torch.int64, device="cuda")
    rngx.set_scrambler(rngx.SCRAMBLE_STAR)
    try:
        rngx.generate(iters, out)
    finally:
        rngx.set_scrambler(rngx.SCRAMBLE_NONE)
    res = parity.compare_plain_device(out, n, iters, seed, word=parity.WORD_STAR)
    del out
    rngx.shutdown()
    _free()
    assert res["mismatches"] == 0, res


def test_plain_continues_across_calls_full():
    # The headline's steps: the same 2^26 streams generated again continue
    # where the previous call stopped (value numbers 256..511).
    n, iters, seed = 1 << 26, 256, 1
    rngx.init(seed, n)
    out = torch.empty(iters * n, dtype=torch.int64, device="cuda")
    rngx.generate(iters, out)
    rngx.generate(iters, out)
    res = parity.compare_plain_device(out, n, iters, seed, cursor=iters)
    del out
    rngx.shutdown()
    _free()
    assert res["mismatches"] == 0, res


@pytest.fixture(scope="module")
def batched_table(oracle):
    r = inputs.batched_requests()
    oreqs = oracle.make_reqs(r.seeds, r.gids, r.offsets, r.lengths)
    bases = np.concatenate([[0], np.cumsum(r.lengths)[:-1]]).astype(np.uint64)
    return r, rngx.make_reqs(r.seeds, r.gids, r.offsets, r.lengths), oreqs, bases


@pytest.mark.parametrize("schedule", ["bench-default", "autotuned", "persistent-S256",
                                      "per-item-S128", "grouped-S16", "grouped-S8-unscheduled"])
def test_batched_table_full(batched_table, schedule):
    r, reqs, oreqs, bases = batched_table
    _say("batched 4096-stream table, %s" % schedule)
    old = rngx.get_batch_cfg()
    out = torch.empty(r.total, dtype=torch.int64, device="cuda")
    try:
        rngx.set_batch_cfg(256, 4, 0, True)          # the benchmark's starting point
        if schedule == "autotuned":
            tune = rngx.autotune_batch(reqs, out, reps=1)
            _say("autotuner picked %s" % tune["best"])
        elif schedule == "persistent-S256":
            rngx.set_batch_cfg(256, 4, 0, True, 16, 1, False)
        elif schedule == "per-item-S128":
            rngx.set_batch_cfg(128, 4, 0, True, 16, 1, True)
        elif schedule == "grouped-S16":               # the library's default
            rngx.set_batch_cfg(16, 4, 0, True, 16, 0, False, 32, 8, 6250)
        elif schedule == "grouped-S8-unscheduled":
            rngx.set_batch_cfg(8, 2, 0, False, 8, 0, False, 128, 3, 0)
        out.fill_(0)
        rngx.generate_batch(reqs, out)
        res = parity.compare_requests_device(out, oreqs, bases)
    finally:
        rngx.set_batch_cfg(**old)
        del out
        _free()
    assert res["mismatches"] == 0, res
    assert res["values"] == r.total


def test_serving_trace_alone_vs_mix_and_oracle(oracle):
    """Two seconds of the 50k req/s trace (Poisson arrivals, stream ids
    uniform over 2^20, lengths floor(2^U[12, 22))) served by the benchmark's
    server (16 GB pool, 4 streams, batches of up to 2,048): requests are
    submitted at their arrival times and a consumer takes each result as it
    completes. Every request's device checksum in that mix equals the one
    of the same request served alone (one stream, batches of one), and the
    first 2,000 requests are compared in full with the oracle."""
    seed, n_states = 1609, 1 << 20
    t, g, L = inputs.serving_arrivals(50000.0, 2.0)
    k = len(t)
    offs = np.array(oracle.serve_offsets(zip(g.tolist(), L.tolist())), dtype=np.uint64)
    n_full = 2000
    oreqs = oracle.make_reqs([seed] * n_full, g[:n_full], offs[:n_full], L[:n_full])
    pool = torch.empty(16 * 10**9 // 256 * 256, dtype=torch.uint8, device="cuda")
    words = pool.view(torch.int64)
    base = pool.data_ptr()
    host = torch.empty(int(L.max()), dtype=torch.int64, pin_memory=True)

    def values(ptr, length):
        off = ptr - base
        assert off % 8 == 0 and 0 <= off and off + 8 * length <= pool.numel()
        return words[off // 8:off // 8 + length]

    mixed = np.zeros(k, dtype=np.uint64)
    tickets = np.zeros(k, dtype=np.uint64)
    published = [0]
    errors, full_bad = [], []
    stop = []
    cv = threading.Condition()

    def consumer():
        try:
            for i in range(k):
                with cv:
                    while published[0] <= i and not errors and not stop:
                        cv.wait(0.5)
                if errors or stop:
                    return
                tk = int(tickets[i])
                ptr = rngx.serve_wait(tk, 120.0)
                v = values(ptr, int(L[i]))
                mixed[i] = rngx.checksum(v, int(L[i]))
                if i < n_full:
                    host[:int(L[i])].copy_(v)
                    res = parity.check_requests(oreqs[i:i + 1], host.data_ptr(),
                                                np.zeros(1, dtype=np.uint64))
                    if res["mismatches"]:
                        full_bad.append((i, res))
                rngx.serve_release(tk)
        except Exception as e:       # reported by the main thread
            errors.append(repr(e))

    _say("serving: %d requests of the 50k req/s trace, mixed" % k)
    rngx.serve_start(seed, n_states, pool, 4, 2048)
    th = threading.Thread(target=consumer, daemon=True)
    th.start()
    try:
        t0 = time.perf_counter()
        i = 0
        while i < k and not errors:
            j = int(np.searchsorted(t, time.perf_counter() - t0, side="right"))
            if j <= i:
                time.sleep(1e-4)     # lets the consumer thread run
                continue
            tickets[i:j] = rngx.serve_submit_many(g[i:j], L[i:j])
            with cv:
                published[0] = j
                cv.notify()
            i = j
        th.join(600)
        assert not th.is_alive(), "consumer did not finish"
        st = rngx.serve_stats()
    finally:
        with cv:
            stop.append(True)
            cv.notify()
        rngx.serve_stop()
        th.join(60)
        if th.is_alive():
            errors.append("consumer still running")
    assert not errors, errors
    assert not full_bad, full_bad[:3]
    assert st["completed"] == k and st["batches"] < k, st

    _say("serving: the same %d requests, alone" % k)
    rngx.serve_start(seed, n_states, pool, 1, 1)
    diff = []
    try:
        for i in range(k):
            tk = rngx.serve_submit(int(g[i]), int(L[i]))
            ptr = rngx.serve_wait(tk, 60.0)
            if rngx.checksum(values(ptr, int(L[i])), int(L[i])) != int(mixed[i]):
                diff.append(i)
            rngx.serve_release(tk)
        st = rngx.serve_stats()
    finally:
        rngx.serve_stop()
        del pool, words, host
        _free()
    assert not diff, diff[:10]
    assert st["batches"] == k
