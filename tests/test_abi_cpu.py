"""CPU-side checks of the C ABI: the library loads, exports every function
include/rngx.h declares, reports errors without a GPU, and its host-side
profile analysis matches the oracle's (oracle/profile.py)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1609_01257_amd import rngx
from oracle import profile as oprof
from tests.test_profile_oracle import fig3_events

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rngx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rngx_\w+)\s*\(", text)))


def test_header_symbols_exported():
    names = declared_functions()
    assert len(names) >= 15
    L = ctypes.CDLL(rngx.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    assert set(declared_functions()) <= set(rngx._SIGS)


def test_strerror_and_codes():
    for code in (0, -1, -2, -3, -4, -5):
        assert rngx.strerror(code).startswith("RNGX_")
    assert "unknown" in rngx.strerror(-99)


def test_generate_before_init_is_noinit():
    rngx.shutdown()
    assert rngx.generate_ptr(4, 0) == rngx.RNGX_E_NOINIT
    assert "before rngx_init" in rngx.last_error()
    with pytest.raises(rngx.RngxError):
        rngx.info()


def test_host_seeding_applies_the_zero_fixup():
    # The library's host-side seeding, on the (seed, gid) pair whose hashed
    # state is zero, against the oracle.
    import oracle
    from tests.test_oracle_pins import inverse_hash_high, inverse_hash_low
    g_star = inverse_hash_low(0)
    seed = inverse_hash_high(inverse_hash_high(0) ^ oracle.hash_high(0)) << 32
    assert rngx.initial_state(seed, g_star) == oracle.init_state(seed, g_star)
    assert rngx.initial_state(seed, g_star) == oracle.hash_high(0) << 32
    assert rngx.initial_state(seed, g_star ^ 1) == oracle.init_state(seed, g_star ^ 1)


def test_profile_window_before_init_is_noinit():
    rngx.shutdown()
    L = rngx.lib()
    assert L.rngx_profile_start() == rngx.RNGX_E_NOINIT
    assert L.rngx_profile_reset() == rngx.RNGX_E_NOINIT
    assert "before rngx_init" in rngx.last_error()


def test_init_zero_states_is_inval():
    assert rngx.lib().rngx_init(0, 0) == rngx.RNGX_E_INVAL


def test_checkpoint_argument_errors_without_gpu():
    import numpy as np
    L = rngx.lib()
    rngx.shutdown()
    buf = np.zeros(4, dtype=np.uint64)
    assert L.rngx_get_state(buf.ctypes.data, 4, None, None) == rngx.RNGX_E_NOINIT
    assert L.rngx_set_state(1, None, 4, 0) == rngx.RNGX_E_INVAL
    ok = np.array([5, 6, 7, 8], dtype=np.uint64)
    assert L.rngx_set_state(1, ok.ctypes.data, 0, 0) == rngx.RNGX_E_INVAL
    bad = np.array([5, 6, 0, 8], dtype=np.uint64)          # xorshift fixes 0
    assert L.rngx_set_state(1, bad.ctypes.data, 4, 0) == rngx.RNGX_E_INVAL
    assert "state 2 is 0" in rngx.last_error()


def test_scrambler_validation_without_gpu():
    L = rngx.lib()
    assert L.rngx_set_scrambler(2) == rngx.RNGX_E_INVAL
    assert L.rngx_set_scrambler(-1) == rngx.RNGX_E_INVAL
    assert L.rngx_get_scrambler(None) == rngx.RNGX_E_INVAL
    rngx.set_scrambler(rngx.SCRAMBLE_STAR)
    assert rngx.get_scrambler() == rngx.SCRAMBLE_STAR
    rngx.set_scrambler(rngx.SCRAMBLE_NONE)
    assert rngx.get_scrambler() == rngx.SCRAMBLE_NONE


def test_set_launch_validation():
    for bad in [(32, 1, 0), (1088, 1, 0), (100, 1, 0), (256, 3, 0), (256, 0, 0), (256, 1, 2),
                (256, 1, 0, 999), (256, 1, 0, 20001)]:
        cfg = rngx.Launch(*bad)
        assert rngx.lib().rngx_set_launch(0, ctypes.byref(cfg)) == rngx.RNGX_E_INVAL
    assert "pace_gbs" in rngx.last_error()
    # The library's defaults: the scheduled launch for u64, its own choice
    # (block 0) for u32.
    default = rngx.get_launch(False)
    assert default == {"block": 512, "chunks": 2, "nontemporal": True, "pace_gbs": 7000}
    rngx.set_launch(False, 512, 4, True)
    assert rngx.get_launch(False) == {"block": 512, "chunks": 4, "nontemporal": True,
                                      "pace_gbs": 0}
    rngx.set_launch(False, 256, 2, False, 6500)
    assert rngx.get_launch(False) == {"block": 256, "chunks": 2, "nontemporal": False,
                                      "pace_gbs": 6500}
    rngx.set_launch(False, **default)
    # u32 defaults to the library's choice (block 0); it can be set
    # explicitly and back.
    assert rngx.get_launch(True)["block"] == 0
    rngx.set_launch(True, 256, 1, False)
    assert rngx.get_launch(True) == {"block": 256, "chunks": 1, "nontemporal": False,
                                     "pace_gbs": 0}
    rngx.set_launch(True, 0, 0, False)
    assert rngx.get_launch(True)["block"] == 0


def _cmp(lib_stats, orc):
    assert lib_stats["n_events"] >= 0
    assert [(a, c) for a, c, _, _ in lib_stats["agg"]] == [(a, c) for a, c, _, _ in orc.agg]
    for (_, _, s1, r1), (_, _, s2, r2) in zip(lib_stats["agg"], orc.agg):
        assert s1 == pytest.approx(s2, rel=1e-12, abs=1e-18)
        assert r1 == pytest.approx(r2, rel=1e-12, abs=1e-12)
    assert [(a, b) for a, b, _ in lib_stats["overlaps"]] == [(a, b) for a, b, _ in orc.overlaps]
    for (_, _, o1), (_, _, o2) in zip(lib_stats["overlaps"], orc.overlaps):
        assert o1 == pytest.approx(o2, rel=1e-12, abs=1e-18)
    for k in ("total_s", "overlap_s", "eff_s", "elapsed_s", "device_pct", "host_pct"):
        assert lib_stats[k] == pytest.approx(getattr(orc, k), rel=1e-12, abs=1e-15), k


def test_profile_analyze_fig3_matches_oracle():
    ev = fig3_events()
    rows = [(e.name, e.queue, e.start_ns, e.end_ns) for e in ev]
    _cmp(rngx.profile_analyze(rows, 9.054619), oprof.analyze(ev, 9.054619))


@pytest.mark.parametrize("seed", range(30))
def test_profile_analyze_random_matches_oracle(seed):
    rng = np.random.default_rng(100 + seed)
    nq = int(rng.integers(1, 5))
    rows = []
    for q in range(nq):
        t = int(rng.integers(0, 50))
        for _ in range(int(rng.integers(0, 40))):
            d = int(rng.integers(0, 30))
            rows.append((str(rng.choice(["INIT_KERNEL", "RNG_KERNEL", "READ_BUFFER", "X"])),
                         q, t, t + d))
            t += d + int(rng.integers(0, 10))
    # Sprinkle some events that overlap within one queue as well.
    if rows and seed % 3 == 0:
        n0, q0, s0, e0 = rows[0]
        rows.append((n0, q0, s0 + 1, e0 + 5))
    ev = [oprof.Event(n, str(q), s, e) for n, q, s, e in rows]
    _cmp(rngx.profile_analyze(rows, 1e-6 * (1 + seed)), oprof.analyze(ev, 1e-6 * (1 + seed)))


def test_profile_analyze_overlaps_beyond_total():
    # Four events of 10 ns in flight together on four queues: the six
    # pairwise overlaps (60 ns) exceed the total (40 ns), and the printed
    # formula gives a negative effective time.
    rows = [("K", q, 0, 10) for q in range(4)]
    ev = [oprof.Event(n, str(q), s, e) for n, q, s, e in rows]
    orc = oprof.analyze(ev, 1e-6)
    assert round(orc.eff_s * 1e9) == -20
    _cmp(rngx.profile_analyze(rows, 1e-6), orc)


def test_profile_analyze_rejects_backwards_event():
    with pytest.raises(rngx.RngxError):
        rngx.profile_analyze([("K", 0, 10, 5)], 1.0)


# --- host-side jump-ahead and seeding (no GPU) ---------------------------------

def test_initial_state_matches_oracle(oracle):
    rng = np.random.default_rng(9)
    for seed in [0, 1, 42, 2**64 - 1] + [int(v) for v in rng.integers(0, 2**64, 20, dtype=np.uint64)]:
        for gid in [0, 1, 2**32 - 1] + [int(v) for v in rng.integers(0, 2**32, 20)]:
            assert rngx.initial_state(seed, gid) == oracle.init_state(seed, gid)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 63, 64, 65, 1000, 4095, 65536, 123457, 1 << 20])
def test_jump_ahead_matches_sequential_oracle(oracle, k):
    for seed, gid in [(0, 0), (42, 7), (2**63, 12345)]:
        x0 = oracle.init_state(seed, gid)
        assert rngx.jump_ahead(x0, k) == oracle.value(seed, gid, k)


def test_jump_ahead_group_laws(oracle):
    # T^(2^64 - 1) = I (full period), T^a T^b = T^(a+b), including huge jumps.
    rng = np.random.default_rng(4)
    for _ in range(50):
        x = int(rng.integers(1, 2**64, dtype=np.uint64))
        assert rngx.jump_ahead(x, 2**64 - 1) == x
        a = int(rng.integers(0, 2**62, dtype=np.uint64))
        b = int(rng.integers(0, 2**62, dtype=np.uint64))
        assert rngx.jump_ahead(rngx.jump_ahead(x, a), b) == rngx.jump_ahead(x, a + b)
        # One step past a jump equals a jump one further.
        assert oracle.rng_step(rngx.jump_ahead(x, a)) == rngx.jump_ahead(x, a + 1)
    assert rngx.jump_ahead(0, 12345) == 0


def test_batch_argument_errors_without_gpu():
    L = rngx.lib()
    reqs = rngx.make_reqs([1], [0], [0], [4])
    # NULL request table with m > 0 is rejected before any device work.
    assert L.rngx_generate_batch(None, 3, None, 0, None) == rngx.RNGX_E_INVAL
    bad = reqs.copy()
    bad["reserved"] = 1
    assert L.rngx_generate_batch(bad.ctypes.data, 1, None, 4, None) == rngx.RNGX_E_INVAL
    assert "reserved" in rngx.last_error()
    # Total above the capacity, and a NULL output, are rejected up front.
    assert L.rngx_generate_batch(reqs.ctypes.data, 1, None, 3, None) == rngx.RNGX_E_INVAL
    assert L.rngx_generate_batch(reqs.ctypes.data, 1, None, 4, None) == rngx.RNGX_E_INVAL
    assert L.rngx_generate_batch(reqs.ctypes.data, 1, 8, 4, None) == rngx.RNGX_E_INVAL  # misaligned
    # Value numbers end at 2^64 - 1: offset + length may be 2^64, not more.
    late = rngx.make_reqs([1], [0], [2**64 - 5], [6])
    assert L.rngx_generate_batch(late.ctypes.data, 1, 16, 6, None) == rngx.RNGX_E_INVAL
    assert "2^64 - 1" in rngx.last_error()
    # The library's default: the grouped order.
    assert rngx.get_batch_cfg() == {"values_per_lane": 16, "waves_per_block": 4, "blocks": 0,
                                    "use_graph": True, "row_values": 16, "run_items": 0,
                                    "per_item": False, "group": 32, "group_steps": 8,
                                    "pace_gbs": 6250}
    default_batch = rngx.get_batch_cfg()
    for bad in [(100, 4, 0, 1, 16, 1, 0), (256, 5, 0, 1, 16, 1, 0), (256, 4, 70000, 1, 16, 1, 0),
                (256, 4, 0, 2, 16, 1, 0), (256, 4, 0, 1, 12, 1, 0), (256, 4, 0, 1, 16, 65, 0),
                (256, 4, 0, 1, 16, 1, 2),
                (8, 4, 0, 1, 16, 0, 0),                   # rows wider than S
                (256, 4, 0, 1, 16, 1, 0, 0, 16, 0),       # steps without a group
                (256, 4, 0, 1, 16, 1, 0, 0, 0, 7000),     # a schedule without a group
                (256, 4, 0, 1, 16, 1, 0, 48, 16, 0),      # not a group size
                (256, 3, 0, 1, 16, 1, 0, 64, 16, 0),      # group not whole blocks
                (256, 4, 0, 1, 16, 1, 0, 64, 0, 0),       # no steps
                (256, 4, 0, 1, 16, 1, 0, 64, 257, 0),
                (256, 4, 0, 1, 16, 1, 1, 64, 16, 0),      # one wave per item
                (256, 4, 0, 1, 16, 1, 0, 64, 16, 999),
                (256, 4, 0, 1, 16, 1, 0, 64, 16, 20001)]:
        assert L.rngx_set_batch_cfg(ctypes.byref(rngx.BatchCfg(*bad))) == rngx.RNGX_E_INVAL, bad
    assert "group_steps" in rngx.last_error()
    rngx.set_batch_cfg(512, 2, 100, False, 8, 3)
    assert rngx.get_batch_cfg() == {"values_per_lane": 512, "waves_per_block": 2, "blocks": 100,
                                    "use_graph": False, "row_values": 8, "run_items": 3,
                                    "per_item": False, "group": 0, "group_steps": 0,
                                    "pace_gbs": 0}
    rngx.set_batch_cfg(8, 2, 0, True, 8, 0, False, 128, 256, 20000)
    assert rngx.get_batch_cfg() == {"values_per_lane": 8, "waves_per_block": 2, "blocks": 0,
                                    "use_graph": True, "row_values": 8, "run_items": 0,
                                    "per_item": False, "group": 128, "group_steps": 256,
                                    "pace_gbs": 20000}
    rngx.set_batch_cfg(64, 4, 0, True, 16, 1, True)
    assert rngx.get_batch_cfg()["per_item"] is True
    rngx.set_batch_cfg(**default_batch)


def test_noalloc_batch_argument_errors_without_gpu():
    L = rngx.lib()
    big = rngx.make_reqs([1] * (rngx.NOALLOC_MAX_REQS + 1), range(rngx.NOALLOC_MAX_REQS + 1),
                         [0] * (rngx.NOALLOC_MAX_REQS + 1), [1] * (rngx.NOALLOC_MAX_REQS + 1))
    # More requests than the static table holds: rejected before any device work.
    assert L.rngx_generate_batch_noalloc(big.ctypes.data, len(big), 16, len(big),
                                         None) == rngx.RNGX_E_INVAL
    assert "exceed the limit of %d" % rngx.NOALLOC_MAX_REQS in rngx.last_error()
    # The allocating call's argument checks apply unchanged.
    reqs = rngx.make_reqs([1], [0], [0], [4])
    assert L.rngx_generate_batch_noalloc(None, 3, None, 0, None) == rngx.RNGX_E_INVAL
    assert L.rngx_generate_batch_noalloc(reqs.ctypes.data, 1, None, 3, None) == rngx.RNGX_E_INVAL
    assert L.rngx_generate_batch_noalloc(reqs.ctypes.data, 1, 8, 4, None) == rngx.RNGX_E_INVAL
    # Nothing requested: a successful no-op that touches no device.
    assert L.rngx_generate_batch_noalloc(None, 0, None, 0, None) == rngx.RNGX_OK


def test_tune_cache_errors_without_gpu(tmp_path):
    L = rngx.lib()
    assert L.rngx_tune_cache_load(None, None) == rngx.RNGX_E_INVAL
    assert L.rngx_tune_cache_save(None) == rngx.RNGX_E_INVAL
    assert L.rngx_tune_cache_load(str(tmp_path / "missing.jsonl").encode(), None) == rngx.RNGX_E_INVAL
    assert "cannot open" in rngx.last_error()
    # Lines are checked before the device is asked for: a truncated entry,
    # an unknown kind and a non-integer field are each rejected by line.
    good = ('{"device": "gfx950 256cu", "kind": "plain_u64", "block": 512, "chunks": 4, '
            '"nontemporal": 0, "ms": 1.000000, "tuned_on": "n=1 iters=1"}')
    for bad in ['{"device": "x", "kind": "plain_u64", "block": 512}',
                good.replace("plain_u64", "plain_u16"),
                good.replace('"chunks": 4', '"chunks": 4.5'),
                good.replace('"block": 512', '"block": -1'),
                good.replace('"nontemporal": 0', '"nontemporal": 0, "pace_gbs": -5')]:
        f = tmp_path / "c.jsonl"
        f.write_text(good + "\n" + bad + "\n")
        assert L.rngx_tune_cache_load(str(f).encode(), None) == rngx.RNGX_E_INVAL, bad
        assert "line 2" in rngx.last_error()
    # Batch lines written before the grouped order (no group keys) still
    # parse; a negative group does not.
    old_batch = ('{"device": "gfx950 256cu", "kind": "batch", "values_per_lane": 256, '
                 '"waves_per_block": 4, "blocks": 0, "use_graph": 1, "row_values": 16, '
                 '"run_items": 1, "per_item": 0, "ms": 1.000000, "tuned_on": "m=1 values=1"}')
    f = tmp_path / "b.jsonl"
    f.write_text(old_batch + "\n" + old_batch.replace('"per_item": 0', '"per_item": 0, "group": -1')
                 + "\n")
    assert L.rngx_tune_cache_load(str(f).encode(), None) == rngx.RNGX_E_INVAL
    assert "line 2" in rngx.last_error()
    # The plain autotuner needs an initialised generator.
    res = rngx.PlainTuneResult()
    assert L.rngx_autotune_plain(4, 0, 16, 1, None, ctypes.byref(res)) == rngx.RNGX_E_NOINIT
    assert L.rngx_autotune_plain(4, 0, 16, 0, None, ctypes.byref(res)) == rngx.RNGX_E_INVAL
    assert L.rngx_autotune_plain(4, 0, 16, 1, None, None) == rngx.RNGX_E_INVAL


def test_serve_calls_before_start_are_noinit():
    L = rngx.lib()
    t = rngx._u64()
    assert L.rngx_serve_submit(0, 1, 0, ctypes.byref(t)) == rngx.RNGX_E_NOINIT
    assert L.rngx_serve_try_submit(0, 1, 0, ctypes.byref(t)) == rngx.RNGX_E_NOINIT
    assert L.rngx_serve_release(1) == rngx.RNGX_E_NOINIT
    assert L.rngx_serve_stats(ctypes.byref(rngx.ServeReport())) == rngx.RNGX_E_NOINIT
    assert L.rngx_serve_stop() == rngx.RNGX_OK
    # Start-argument checks happen before any device work.
    assert L.rngx_serve_start(1, 0, 4096, 1 << 16, 4, 16) == rngx.RNGX_E_INVAL
    assert L.rngx_serve_start(1, 10, 4096 + 8, 1 << 16, 4, 16) == rngx.RNGX_E_INVAL
    assert L.rngx_serve_set_max_pending(0) == rngx.RNGX_E_INVAL


def test_serve_max_inflight_validation():
    L = rngx.lib()
    assert L.rngx_serve_set_max_inflight(0) == rngx.RNGX_E_INVAL
    assert L.rngx_serve_set_max_inflight(33) == rngx.RNGX_E_INVAL
    assert L.rngx_serve_set_max_inflight(32) == rngx.RNGX_OK
    assert L.rngx_serve_set_max_inflight(2) == rngx.RNGX_OK


def test_server_pool_ring_and_ticket_table_model(tmp_path):
    import subprocess
    src = os.path.join(ROOT, "tests", "helpers", "pool_model.cpp")
    exe = str(tmp_path / "pool_model")
    # Host-only code: built with g++ and the address/undefined-behaviour sanitizers.
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I",
                    os.path.join(ROOT, "paper_1609_01257_amd", "csrc"), src, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_profile_write_table_and_trace(tmp_path):
    import json
    ev = fig3_events()
    rows = [(e.name, e.queue, e.start_ns, e.end_ns) for e in ev]
    table = tmp_path / "events.tsv"
    rngx.profile_write(rows, str(table), rngx.EXPORT_TABLE)
    lines = table.read_text().splitlines()
    assert lines[0].split("\t") == ["queue", "t_start", "t_end", "event"]
    body = [l.split("\t") for l in lines[1:]]
    assert len(body) == len(ev)
    # Rows by start time; the first event's queue (Main) is q0, Comms is q1.
    want = sorted(ev, key=lambda e: e.start_ns)
    qname = {"Main": "q0", "Comms": "q1"}
    assert body == [[qname[e.queue], str(e.start_ns), str(e.end_ns), e.name] for e in want]
    trace = tmp_path / "events.json"
    rngx.profile_write(rows, str(trace), rngx.EXPORT_TRACE)
    doc = json.loads(trace.read_text())
    meta = [x for x in doc["traceEvents"] if x["ph"] == "M"]
    spans = [x for x in doc["traceEvents"] if x["ph"] == "X"]
    assert sorted(m["args"]["name"] for m in meta) == ["q0", "q1"]
    assert len(spans) == len(ev)
    for x, e in zip(spans, want):
        assert x["name"] == e.name and x["tid"] == int(qname[e.queue][1:])
        assert x["ts"] == pytest.approx(e.start_ns / 1e3, abs=1e-3)
        assert x["dur"] == pytest.approx((e.end_ns - e.start_ns) / 1e3, abs=1e-3)


def test_profile_write_errors(tmp_path):
    L = rngx.lib()
    ok = rngx._event_array([("A", 0, 5, 9)])
    assert L.rngx_profile_write(ok, 1, None, 0) == rngx.RNGX_E_INVAL
    assert L.rngx_profile_write(None, 1, str(tmp_path / "x").encode(), 0) == rngx.RNGX_E_INVAL
    assert L.rngx_profile_write(ok, 1, str(tmp_path / "x").encode(), 2) == rngx.RNGX_E_INVAL
    back = rngx._event_array([("A", 0, 9, 5)])
    assert L.rngx_profile_write(back, 1, str(tmp_path / "x").encode(), 0) == rngx.RNGX_E_INVAL
    assert L.rngx_profile_write(ok, 1, str(tmp_path / "no" / "dir").encode(), 0) == rngx.RNGX_E_INVAL
    assert "cannot open" in rngx.last_error()
    # Names with quotes, backslashes or control characters stay well-formed.
    import json
    odd = rngx._event_array([('a"b\\c\td', 0, 1, 2)])
    p = tmp_path / "odd.json"
    assert L.rngx_profile_write(odd, 1, str(p).encode(), 1) == rngx.RNGX_OK
    assert json.loads(p.read_text())["traceEvents"][-1]["name"] == 'a"b\\c_d'
    p = tmp_path / "odd.tsv"
    assert L.rngx_profile_write(odd, 1, str(p).encode(), 0) == rngx.RNGX_OK
    assert p.read_text().splitlines()[1].split("\t") == ["q0", "1", "2", 'a"b\\c_d']
