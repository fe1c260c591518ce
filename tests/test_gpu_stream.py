"""GPU parity of the two-stream device-to-host pipeline against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1609_01257_amd import inputs, rngx
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(params=["kernel", "runtime"])
def copy_mode(request):
    mode = rngx.COPY_KERNEL if request.param == "kernel" else rngx.COPY_RUNTIME
    old = rngx.get_copy_mode()
    rngx.set_copy_mode(mode, 512)
    yield request.param
    rngx.set_copy_mode(*old)


def _buffers(n, R, slots, u32=False):
    dt = torch.int32 if u32 else torch.int64
    dev0 = torch.empty(R * n, dtype=dt, device="cuda")
    dev1 = torch.empty(R * n, dtype=dt, device="cuda")
    host = torch.zeros(slots * R * n, dtype=dt, pin_memory=True)
    return dev0, dev1, host


@pytest.mark.parametrize("u32", [False, True])
@pytest.mark.parametrize("n,R,steps", [(1, 1, 5), (4099, 1, 9), (65537, 3, 4), (1 << 16, 2, 7)])
def test_every_step_to_its_own_slot(oracle, n, R, steps, u32, copy_mode):
    seed = 0 if n == 4099 else 17
    rngx.init(seed, n)
    dev0, dev1, host = _buffers(n, R, steps, u32)
    rngx.stream_to_host(steps, R, dev0, dev1, host, steps, u32=u32)
    got = host.numpy().view(np.uint32 if u32 else np.uint64).reshape(steps * R, n)
    exp = (oracle.generate_u32 if u32 else oracle.generate)(seed, n, steps * R)
    assert np.array_equal(got, exp)
    assert rngx.info()[2] == steps * R


def test_consumer_sees_steps_in_order_with_two_slots(oracle, copy_mode):
    seed, n, R, steps = 42, 10007, 2, 11
    rngx.init(seed, n)
    dev0, dev1, host = _buffers(n, R, 2)
    seen = []

    def consume(step, arr):
        seen.append((step, arr.copy()))
        return False
    rngx.stream_to_host(steps, R, dev0, dev1, host, 2, consume=consume)
    exp = oracle.generate(seed, n, steps * R)
    assert [s for s, _ in seen] == list(range(steps))
    for s, arr in seen:
        assert np.array_equal(arr.reshape(R, n), exp[s * R:(s + 1) * R])


def test_stream_continues_cursor_of_plain_calls(oracle):
    seed, n = 5, 3001
    rngx.init(seed, n)
    pre = torch.empty(4 * n, dtype=torch.int64, device="cuda")
    rngx.generate(4, pre)
    dev0, dev1, host = _buffers(n, 1, 6)
    rngx.stream_to_host(6, 1, dev0, dev1, host, 6)
    exp = oracle.generate(seed, n, 10)
    assert np.array_equal(host.numpy().view(np.uint64).reshape(6, n), exp[4:])


def test_consumer_abort_stops_and_reports(oracle):
    seed, n = 3, 2048
    rngx.init(seed, n)
    dev0, dev1, host = _buffers(n, 1, 2)
    seen = []

    def consume(step, arr):
        seen.append(step)
        return step == 3
    with pytest.raises(rngx.RngxError) as ei:
        rngx.stream_to_host(20, 1, dev0, dev1, host, 2, consume=consume)
    assert ei.value.code == rngx.RNGX_E_ABORTED
    assert seen == [0, 1, 2, 3]
    # Steps generated before the stop advanced the cursor; the generator
    # continues from there.
    c = rngx.info()[2]
    assert 4 <= c <= 6
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    rngx.generate(1, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64), oracle.generate(seed, n, 1, cursor=c)[0])


def test_consumer_exception_stops_and_propagates(oracle):
    seed, n = 4, 2048
    rngx.init(seed, n)
    dev0, dev1, host = _buffers(n, 1, 2)
    seen = []

    def consume(step, arr):
        seen.append(step)
        if step == 2:
            raise KeyError("consumer failed at step 2")
    with pytest.raises(KeyError):
        rngx.stream_to_host(20, 1, dev0, dev1, host, 2, consume=consume)
    assert seen == [0, 1, 2]
    # The library is usable afterwards and continues the cursor.
    c = rngx.info()[2]
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    rngx.generate(1, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64), oracle.generate(seed, n, 1, cursor=c)[0])


def test_forced_copy_failure_stops_and_reports(oracle, copy_mode):
    # The copy of step 5 fails (forced on the host, before it is enqueued):
    # the call drains both streams, hands no further step to the consumer,
    # and reports the failure; the library stays usable and the cursor has
    # advanced past every generated step.
    seed, n, ips = 6, 4096, 2
    try:
        rngx.init(seed, n)
        dev0, dev1, host = _buffers(n, ips, 2)
        exp = oracle.generate(seed, n, 40 * ips)
        seen = []

        def consume(step, arr):
            seen.append(step)
            assert np.array_equal(arr.reshape(ips, n), exp[step * ips:(step + 1) * ips])
        rngx.inject_copy_failure(5)
        with pytest.raises(rngx.RngxError) as ei:
            rngx.stream_to_host(20, ips, dev0, dev1, host, 2, consume=consume)
        assert ei.value.code == rngx.RNGX_E_HIP
        assert "step 5" in str(ei.value) and "forced" in str(ei.value)
        assert seen == [0, 1, 2, 3]
        assert rngx.info()[2] == 6 * ips
        # The hook fired once: the next run streams in full from the cursor.
        seen.clear()
        rngx.stream_to_host(4, ips, dev0, dev1, host, 2, consume=lambda k, a: seen.append(
            (k, np.array_equal(a.reshape(ips, n), exp[(6 + k) * ips:(7 + k) * ips]))))
        assert seen == [(k, True) for k in range(4)]
        # Armed for a step beyond the run: it does not fire, and it is
        # disarmed when the run ends.
        rngx.inject_copy_failure(100)
        rngx.stream_to_host(2, ips, dev0, dev1, host, 2)
        assert rngx.info()[2] == 12 * ips
    finally:
        rngx.inject_copy_failure(2**64 - 1)


def test_pageable_host_memory_uses_runtime_copy(oracle):
    # Ordinary (not page-locked) host memory cannot be written by the copy
    # kernel; the pipeline must still deliver every value.
    seed, n, steps = 12, 5003, 6
    rngx.init(seed, n)
    dev0 = torch.empty(n, dtype=torch.int64, device="cuda")
    dev1 = torch.empty(n, dtype=torch.int64, device="cuda")
    host = torch.zeros(steps * n, dtype=torch.int64)
    rngx.stream_to_host(steps, 1, dev0, dev1, host, steps)
    assert np.array_equal(host.numpy().view(np.uint64).reshape(steps, n),
                          oracle.generate(seed, n, steps))


def test_copy_mode_validation():
    old = rngx.get_copy_mode()
    L = rngx.lib()
    assert L.rngx_set_copy_mode(7, 512) == rngx.RNGX_E_INVAL
    assert L.rngx_set_copy_mode(0, 0) == rngx.RNGX_E_INVAL
    assert L.rngx_set_copy_mode(0, 65537) == rngx.RNGX_E_INVAL
    assert rngx.get_copy_mode() == old


def test_stream_argument_errors():
    rngx.init(0, 1024)
    dev0, dev1, host = _buffers(1024, 1, 2)
    L = rngx.lib()
    cb = rngx.CONSUME_FN()
    ok = (4, 1, 0, dev0.data_ptr(), dev1.data_ptr(), 8 * 1024, host.data_ptr(), 2, cb, None, 0, 0)
    assert L.rngx_stream_to_host(*ok) == rngx.RNGX_OK
    bad = [
        (4, 0) + ok[2:],                                         # iters_per_step 0
        ok[:3] + (0,) + ok[4:],                                   # NULL dev0
        ok[:4] + (dev0.data_ptr(),) + ok[5:],                     # same buffers
        ok[:5] + (8 * 1023,) + ok[6:],                            # step too large
        ok[:6] + (None,) + ok[7:],                                # NULL host
        ok[:7] + (0,) + ok[8:],                                   # zero slots
        ok[:3] + (dev0.data_ptr() + 4,) + ok[4:],                 # misaligned
    ]
    for args in bad:
        assert L.rngx_stream_to_host(*args) == rngx.RNGX_E_INVAL, args
    s = torch.cuda.Stream()
    same = ok[:10] + (s.cuda_stream, s.cuda_stream)
    assert L.rngx_stream_to_host(*same) == rngx.RNGX_E_INVAL
    assert L.rngx_stream_to_host(0, 1, 0, None, None, 0, None, 0, cb, None, 0, 0) == rngx.RNGX_OK


def test_profile_of_a_stream_has_fig3_rows():
    n, steps = 1 << 20, 16
    rngx.init(0, n)
    dev0, dev1, host = _buffers(n, 1, 2)
    rngx.stream_to_host(steps, 1, dev0, dev1, host, 2)
    st = rngx.profile_stats()
    counts = {name: c for name, c, _, _ in st["agg"]}
    assert counts == {"INIT_KERNEL": 1, "RNG_KERNEL": steps, "READ_BUFFER": steps}
    assert st["eff_s"] <= st["total_s"] and st["eff_s"] > 0
    assert 0 < st["device_pct"] <= 100.0 + 1e-6
    for a, b, ov in st["overlaps"]:
        assert {a, b} <= {"INIT_KERNEL", "RNG_KERNEL", "READ_BUFFER"} and ov > 0
    ev = rngx.profile_events()
    queues = {name: {q for nm, q, _, _ in ev if nm == name} for name in counts}
    assert len(queues["READ_BUFFER"]) == 1 and queues["READ_BUFFER"] != queues["RNG_KERNEL"]
    # Copies on one stream are in order and never overlap each other.
    reads = sorted((s, e) for nm, _, s, e in ev if nm == "READ_BUFFER")
    assert all(reads[i][1] <= reads[i + 1][0] for i in range(len(reads) - 1))
    text = rngx.profile()
    assert "READ_BUFFER" in text and "Time spent in device" in text


def test_paper_shaped_streaming_full_and_overlapped(oracle, copy_mode):
    """4,194,304 work-items, seed 42, 2,000 iterations (32 MiB each) through
    two device buffers and two pinned host slots: every value of every step
    is compared with the oracle as the consumer receives it, and generation
    overlaps the device-to-host reads (Fig. 2: kernels on one queue, reads
    on another, each kernel running while the previous buffer is read)."""
    cfg = inputs.STREAMING
    seed, n, steps = cfg["seed"], cfg["n"], cfg["iters"]
    # Streams created before the pipeline's own, as in a process that did
    # other work first: the pipeline must still get queues of its own.
    others = [torch.cuda.Stream() for _ in range(6)]
    st = parity.seed_states(seed, n)
    rngx.init(seed, n)
    dev0, dev1, host = _buffers(n, 1, 2)
    seen, bad = [], []

    def consume(step, arr):
        res = parity.check_rows_ptr(arr.ctypes.data, n, n, 1, st, parity.WORD_U64)
        seen.append(step)
        if res["mismatches"]:
            bad.append((step, res))
            return True
        return False
    rngx.stream_to_host(steps, 1, dev0, dev1, host, 2, consume=consume)
    assert not bad, bad[:3]
    assert seen == list(range(steps))
    prof = rngx.profile_stats()
    counts = {name: c for name, c, _, _ in prof["agg"]}
    assert counts["READ_BUFFER"] == steps and counts["RNG_KERNEL"] == steps
    pairs = {frozenset((a, b)): ov for a, b, ov in prof["overlaps"]}
    overlap = pairs.get(frozenset(("RNG_KERNEL", "READ_BUFFER")), 0.0)
    assert overlap > 0, prof["overlaps"]
    del others


def test_profile_export_of_a_streamed_run(tmp_path):
    # The exported table holds every logged event of the window: one init
    # kernel, one generation kernel and one read per step, the reads on
    # their own queue.
    import json
    n, steps = 1 << 16, 6
    rngx.init(9, n)
    dev0, dev1, host = _buffers(n, 1, 2)
    rngx.stream_to_host(steps, 1, dev0, dev1, host, 2)
    table = tmp_path / "t.tsv"
    rngx.profile_export(str(table), rngx.EXPORT_TABLE)
    rows = [l.split("\t") for l in table.read_text().splitlines()[1:]]
    names = [r[3] for r in rows]
    assert names.count("INIT_KERNEL") == 1 and names[0] == "INIT_KERNEL"
    assert names.count("RNG_KERNEL") == steps and names.count("READ_BUFFER") == steps
    assert {r[0] for r in rows if r[3] == "READ_BUFFER"}.isdisjoint(
        {r[0] for r in rows if r[3] == "RNG_KERNEL"})
    assert all(int(r[1]) <= int(r[2]) for r in rows)
    starts = [int(r[1]) for r in rows]
    assert starts == sorted(starts)
    trace = tmp_path / "t.json"
    rngx.profile_export(str(trace), rngx.EXPORT_TRACE)
    spans = [x for x in json.loads(trace.read_text())["traceEvents"] if x["ph"] == "X"]
    assert len(spans) == len(rows)


def test_scrambled_stream_matches_oracle(oracle):
    seed, n, R, steps = 12, 4099, 2, 5
    rngx.init(seed, n)
    dev0, dev1, host = _buffers(n, R, steps)
    rngx.set_scrambler(rngx.SCRAMBLE_STAR)
    try:
        rngx.stream_to_host(steps, R, dev0, dev1, host, steps)
    finally:
        rngx.set_scrambler(rngx.SCRAMBLE_NONE)
    got = host.numpy().view(np.uint64).reshape(steps * R, n)
    assert np.array_equal(got, oracle.generate_star(seed, n, steps * R))
