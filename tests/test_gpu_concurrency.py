"""GPU tests of the library's locking and lifetimes: batched calls from
several threads on their own streams while a server runs, and server
start/stop cycles that must give back their device memory."""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1609_01257_amd import inputs, rngx

pytestmark = pytest.mark.gpu


def test_threads_batching_while_a_server_serves(oracle):
    # Four threads call rngx_generate_batch on their own streams (ctypes
    # releases the interpreter lock during each call) while a fifth submits
    # to the server; every result is compared with the oracle afterwards.
    tables = [inputs.ragged_requests(m=9 + t, seed=300 + t, max_len=60000, max_offset=50000)
              for t in range(4)]
    expected = [oracle.generate_batch(oracle.make_reqs(r.seeds, r.gids, r.offsets, r.lengths))
                for r in tables]
    seed, n_states = 4711, 128
    pool = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")
    rngx.serve_start(seed, n_states, pool, 2, 16)
    hist = [(int(g), int(L)) for g, L in zip(np.arange(60) % n_states, 1000 + np.arange(60) * 37)]
    served, errors = {}, []

    def batcher(t):
        try:
            r = tables[t]
            reqs = rngx.make_reqs(r.seeds, r.gids, r.offsets, r.lengths)
            s = torch.cuda.Stream()
            outs = []
            for _ in range(5):
                out = torch.zeros(r.total, dtype=torch.int64, device="cuda")
                rngx.generate_batch(reqs, out, stream=s)
                outs.append(out)
            s.synchronize()
            for out in outs:
                if not np.array_equal(out.cpu().numpy().view(np.uint64), expected[t]):
                    errors.append("batch thread %d" % t)
        except Exception as e:          # reported below, with the thread's name
            errors.append("batch thread %d: %r" % (t, e))

    def submitter():
        try:
            for k, (g, L) in enumerate(hist):
                tk = rngx.serve_submit(g, L)
                ptr = rngx.serve_wait(tk, 30.0)
                off = ptr - pool.data_ptr()
                served[k] = pool[off:off + 8 * L].view(torch.int64).cpu().numpy().view(np.uint64)
                rngx.serve_release(tk)
        except Exception as e:
            errors.append("submitter: %r" % (e,))

    threads = [threading.Thread(target=batcher, args=(t,)) for t in range(4)]
    threads.append(threading.Thread(target=submitter))
    try:
        for th in threads:
            th.start()
        for th in threads:
            th.join(120)
        assert not any(th.is_alive() for th in threads), "a thread did not finish"
    finally:
        rngx.serve_stop()
    assert not errors, errors
    exp = oracle.serve_expected(seed, hist)
    for k, e in enumerate(exp):
        assert np.array_equal(served[k], e), k


def test_threads_submitting_to_shared_streams(oracle):
    # Four threads submit to the same few streams at once. Each request's
    # values are fixed when it is submitted (the stream's cursor moves under
    # the server's lock), and tickets are issued in submission order, so
    # ordering the submissions by ticket gives the history the oracle needs.
    seed, n_states = 777, 8
    pool = torch.zeros(256 << 20, dtype=torch.uint8, device="cuda")
    rngx.serve_start(seed, n_states, pool, 4, 64)
    subs, errors = [], []
    lock = threading.Lock()

    def submitter(t):
        try:
            rng = np.random.default_rng(900 + t)
            for _ in range(60):
                g, L = int(rng.integers(0, n_states)), int(rng.integers(1, 20000))
                tk = rngx.serve_submit(g, L)
                with lock:
                    subs.append((tk, g, L))
        except Exception as e:
            errors.append("submitter %d: %r" % (t, e))

    threads = [threading.Thread(target=submitter, args=(t,)) for t in range(4)]
    try:
        for th in threads:
            th.start()
        for th in threads:
            th.join(120)
        assert not any(th.is_alive() for th in threads), "a thread did not finish"
        assert not errors, errors
        subs.sort()
        exp = oracle.serve_expected(seed, [(g, L) for _, g, L in subs])
        for (tk, g, L), e in zip(subs, exp):
            ptr = rngx.serve_wait(tk, 30.0)
            off = ptr - pool.data_ptr()
            got = pool[off:off + 8 * L].view(torch.int64).cpu().numpy().view(np.uint64)
            assert np.array_equal(got, e), (tk, g, L)
            rngx.serve_release(tk)
    finally:
        rngx.serve_stop()


def test_server_cycles_release_device_memory():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    pool = torch.zeros(32 << 20, dtype=torch.uint8, device="cuda")
    rngx.serve_start(1, 1 << 20, pool, 4, 64)       # creates the batch tables once
    rngx.serve_stop()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for i in range(5):
        rngx.serve_start(i, 1 << 22, pool, 4, 1024)  # 32 MiB of resident states
        t = rngx.serve_submit(7, 100000)
        rngx.serve_wait(t, 30.0)
        rngx.serve_release(t)
        rngx.serve_stop()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert abs(free1 - free0) < (64 << 20)
