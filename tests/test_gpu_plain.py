"""GPU parity of the plain path (seeding + persistent generation) against the
CPU oracle, through the C ABI. Bit-exact: tolerance 0."""
import itertools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1609_01257_amd import inputs, rngx

pytestmark = pytest.mark.gpu


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def run(seed, n, iters, u32=False, offset=0, pre=0):
    """init, optionally skip `pre` iterations, then generate `iters` iterations
    into a buffer shifted by `offset` elements (to test unaligned rows)."""
    rngx.init(seed, n)
    if pre:
        scratch = torch.empty(pre * n, dtype=torch.int64, device="cuda")
        rngx.generate(pre, scratch)
    dt = torch.int32 if u32 else torch.int64
    buf = torch.zeros(iters * n + offset + 1, dtype=dt, device="cuda")
    view = buf[offset:offset + iters * n] if iters else buf[offset:offset + 1]
    (rngx.generate_u32 if u32 else rngx.generate)(iters, view)
    torch.cuda.synchronize()
    host = (_u32 if u32 else _u64)(buf)
    # Guard elements around the output must be untouched.
    assert (host[:offset] == 0).all() and host[offset + iters * n] == 0
    return host[offset:offset + iters * n].reshape(iters, n)


def test_small_config_full_parity(oracle):
    cfg = inputs.SMALL
    got = run(cfg["seed"], cfg["n"], cfg["iters"])
    exp = oracle.generate(cfg["seed"], cfg["n"], cfg["iters"])
    assert np.array_equal(got, exp)
    # The paper's first batch is the init output (seed 0 is the paper).
    assert int(got[0, 0]) == 0x103FE9A06B4ED927
    assert int(got[1, 0]) == 0x671A87CFF9A01BA8


ODD_N = [1, 2, 3, 63, 64, 65, 127, 129, 255, 257, 1023, 1025, 4097, 65537, 100003]


@pytest.mark.parametrize("u32", [False, True])
@pytest.mark.parametrize("n", ODD_N)
def test_ragged_sizes(oracle, n, u32):
    for iters, offset, seed in [(1, 0, 5), (2, 1, 0), (7, 0, 2**64 - 1), (3, 3, 42)]:
        got = run(seed, n, iters, u32=u32, offset=offset)
        exp = (oracle.generate_u32 if u32 else oracle.generate)(seed, n, iters)
        assert np.array_equal(got, exp), (n, iters, offset, seed)


def test_zero_iterations_is_noop(oracle):
    rngx.init(9, 100)
    rngx.generate(0, None)
    assert rngx.info()[2] == 0
    got = run(9, 100, 3)
    assert np.array_equal(got, oracle.generate(9, 100, 3))


@pytest.mark.parametrize("u32", [False, True])
@pytest.mark.parametrize("n", [1000, (1 << 20) + 3, (1 << 22) + 6])
def test_automatic_launch_choice(oracle, u32, n):
    # block 0: the library's choice (the scheduled launch on aligned rows,
    # the unscheduled kernel on shifted ones); same output.
    default = rngx.get_launch(u32)
    try:
        rngx.set_launch(u32, 0, 0, False)
        exp = (oracle.generate_u32 if u32 else oracle.generate)(8, n, 2)
        for offset in (0, 1):
            assert np.array_equal(run(8, n, 2, u32=u32, offset=offset), exp), offset
    finally:
        rngx.set_launch(u32, **default)


def test_library_defaults():
    rngx.init(1, 64)
    assert rngx.get_launch(False) == {"block": 512, "chunks": 2, "nontemporal": True,
                                      "pace_gbs": 7000}
    assert rngx.get_launch(True)["block"] == 0


@pytest.mark.parametrize("u32", [False, True])
def test_every_launch_config_gives_identical_output(oracle, u32):
    n, iters, seed = 100003, 5, 77
    exp = (oracle.generate_u32 if u32 else oracle.generate)(seed, n, iters)
    default = rngx.get_launch(u32)
    try:
        for block, chunks, nt in itertools.product([64, 128, 256, 512, 1024], [1, 2, 4], [0, 1]):
            rngx.set_launch(u32, block, chunks, nt)
            for offset in (0, 1):
                got = run(seed, n, iters, u32=u32, offset=offset)
                assert np.array_equal(got, exp), (block, chunks, nt, offset)
    finally:
        rngx.set_launch(u32, **default)


# Row-scheduled (paced) launches: a persistent grid walking strips of
# columns, every wavefront keeping to one row schedule. Shapes with 16-byte
# aligned rows and a partial last wavefront; 1-wavefront blocks of one chunk
# give several strips at these sizes; 1000 GB/s makes the waits long.
PACED = [(False, 64, 1, 0, 1000, (1 << 21) + 6), (False, 512, 4, 0, 6500, (1 << 22) + 2050),
         (False, 256, 2, 1, 3000, (1 << 21) + 1024), (True, 64, 1, 0, 2000, (1 << 21) + 4),
         (True, 512, 4, 0, 6000, (1 << 22) + 8196)]


@pytest.mark.parametrize("u32,block,chunks,nt,pace,n", PACED)
def test_paced_launches_give_identical_output(oracle, u32, block, chunks, nt, pace, n):
    iters, seed = 5, 4242
    exp = (oracle.generate_u32 if u32 else oracle.generate)(seed, n, iters)
    default = rngx.get_launch(u32)
    try:
        rngx.set_launch(u32, block, chunks, nt, pace)
        assert np.array_equal(run(seed, n, iters, u32=u32), exp)
        # Rows not 16-byte aligned, and single iterations, run unscheduled.
        assert np.array_equal(run(seed, n, iters, u32=u32, offset=1), exp)
        rngx.init(seed, n)
        one = torch.empty(n, dtype=torch.int32 if u32 else torch.int64, device="cuda")
        for k in range(2):
            (rngx.generate_u32 if u32 else rngx.generate)(1, one)
            torch.cuda.synchronize()
            got = _u32(one) if u32 else _u64(one)
            assert np.array_equal(got, exp[k]), k
    finally:
        rngx.set_launch(u32, **default)


def test_paced_scrambled_and_continued_calls(oracle):
    seed, n = 99, (1 << 21) + 2
    default = rngx.get_launch(False)
    try:
        rngx.set_launch(False, 128, 2, False, 4000)
        rngx.set_scrambler(rngx.SCRAMBLE_STAR)
        rngx.init(seed, n)
        a = torch.empty(3 * n, dtype=torch.int64, device="cuda")
        b = torch.empty(4 * n, dtype=torch.int64, device="cuda")
        rngx.generate(3, a)
        rngx.generate(4, b)
        torch.cuda.synchronize()
        exp = oracle.generate_star(seed, n, 7)
        assert np.array_equal(_u64(a).reshape(3, n), exp[:3])
        assert np.array_equal(_u64(b).reshape(4, n), exp[3:])
    finally:
        rngx.set_scrambler(rngx.SCRAMBLE_NONE)
        rngx.set_launch(False, **default)


def test_cursor_continues_across_calls_and_widths(oracle):
    seed, n = 31337, 4099
    rngx.init(seed, n)
    a = torch.empty(3 * n, dtype=torch.int64, device="cuda")
    b = torch.empty(4 * n, dtype=torch.int32, device="cuda")
    c = torch.empty(5 * n, dtype=torch.int64, device="cuda")
    rngx.generate(3, a)
    rngx.generate_u32(4, b)
    rngx.generate(5, c)
    torch.cuda.synchronize()
    assert rngx.info() == (seed, n, 12)
    exp = oracle.generate(seed, n, 12)
    assert np.array_equal(_u64(a).reshape(3, n), exp[:3])
    assert np.array_equal(_u32(b).reshape(4, n), (exp[3:7] & np.uint64(0xFFFFFFFF)).astype(np.uint32))
    assert np.array_equal(_u64(c).reshape(5, n), exp[7:])


def test_state_ordered_across_streams(oracle):
    seed, n = 8, 200000
    rngx.init(seed, n)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for k in range(6):
        o = torch.empty(2 * n, dtype=torch.int64, device="cuda")
        s = s1 if k % 2 == 0 else s2
        o.record_stream(s)
        rngx.generate(2, o, stream=s)
        outs.append(o)
    torch.cuda.synchronize()
    exp = oracle.generate(seed, n, 12)
    for k, o in enumerate(outs):
        assert np.array_equal(_u64(o).reshape(2, n), exp[2 * k:2 * k + 2]), k


def test_reinit_resets_cursor_and_profile(oracle):
    rngx.init(1, 1000)
    out = torch.empty(10 * 1000, dtype=torch.int64, device="cuda")
    rngx.generate(10, out)
    rngx.init(1, 1000)
    assert rngx.info()[2] == 0
    rngx.generate(2, out)
    torch.cuda.synchronize()
    st = rngx.profile_stats()
    counts = {name: c for name, c, _, _ in st["agg"]}
    assert counts == {"INIT_KERNEL": 1, "RNG_KERNEL": 1}
    assert np.array_equal(_u64(out)[:2000].reshape(2, 1000), oracle.generate(1, 1000, 2))


def test_profile_records_every_call():
    rngx.init(0, 1 << 16)
    out = torch.empty(4 << 16, dtype=torch.int64, device="cuda")
    for _ in range(5):
        rngx.generate(4, out)
    st = rngx.profile_stats()
    counts = {name: c for name, c, _, _ in st["agg"]}
    assert counts == {"INIT_KERNEL": 1, "RNG_KERNEL": 5}
    assert all(a > 0 for _, _, a, _ in st["agg"])
    assert st["elapsed_s"] > 0 and 0 < st["device_pct"] <= 100
    assert sum(r for _, _, _, r in st["agg"]) == pytest.approx(100.0)
    ev = rngx.profile_events()
    assert len(ev) == 6 and all(e[3] >= e[2] for e in ev)
    text = rngx.profile()
    assert "RNG_KERNEL" in text and "INIT_KERNEL" in text and "Time spent in device" in text
    # A reset starts an empty window that logs what follows.
    rngx.profile_reset()
    rngx.generate(4, out)
    st = rngx.profile_stats()
    assert {name: c for name, c, _, _ in st["agg"]} == {"RNG_KERNEL": 1}


def test_abi_errors_on_device():
    rngx.init(0, 1 << 20)
    out = torch.empty(16, dtype=torch.int64, device="cuda")
    assert rngx.generate_ptr(1, 0) == rngx.RNGX_E_INVAL                       # NULL
    assert rngx.generate_ptr(1, out.data_ptr() + 4) == rngx.RNGX_E_INVAL      # misaligned
    assert rngx.generate_ptr(1, out.data_ptr() + 2, u32=True) == rngx.RNGX_E_INVAL
    assert rngx.info()[2] == 0          # failed calls do not advance the cursor
    rngx.shutdown()
    assert rngx.generate_ptr(1, out.data_ptr()) == rngx.RNGX_E_NOINIT


def test_size_overflow_rejected():
    rngx.init(0, 2**32 - 1)                # 32 GiB of state
    out = torch.empty(16, dtype=torch.int64, device="cuda")
    # (2^32 - 1)^2 * 8 bytes overflows size_t.
    assert rngx.generate_ptr(2**32 - 1, out.data_ptr()) == rngx.RNGX_E_INVAL
    assert "overflow" in rngx.last_error()
    assert rngx.info()[2] == 0
    rngx.shutdown()
    torch.cuda.empty_cache()


def test_largest_state_count_sampled(oracle):
    # n = 2^32 - 1 work-items (the most a 32-bit count allows), 2 iterations:
    # the last, partial wave (511 work-items) and a second row that starts
    # 8 bytes off a 16-byte boundary; sampled values against the oracle.
    n, seed = 2**32 - 1, 7
    rngx.init(seed, n)
    out = torch.empty(2 * n, dtype=torch.int64, device="cuda")
    rngx.generate(2, out)
    gids = [0, 1, 2, 511, 512, 1 << 31, 123456789, n - 513, n - 512, n - 511, n - 2, n - 1]
    pos = [(k, g) for k in (0, 1) for g in gids]
    idx = torch.tensor([k * n + g for k, g in pos], device="cuda")
    got = out.index_select(0, idx).cpu().numpy().view(np.uint64)
    del out
    rngx.shutdown()
    torch.cuda.empty_cache()
    for (k, g), v in zip(pos, got):
        assert int(v) == oracle.value(seed, g, k), (k, g)


def test_shutdown_releases_device_memory():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    rngx.shutdown()
    free0, _ = torch.cuda.mem_get_info()
    rngx.init(3, 1 << 27)                  # 1 GiB of state
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    # The device's free-memory figure moves in allocation granules.
    assert free0 - free1 >= (1 << 30) - (64 << 20)
    rngx.shutdown()
    free2, _ = torch.cuda.mem_get_info()
    assert abs(free2 - free0) < (64 << 20)


def test_roofline_small_full(oracle):
    n, iters = 1 << 20, 16
    got = run(1, n, iters)
    assert np.array_equal(got, oracle.generate(1, n, iters))
    got32 = run(1, n, iters, u32=True)
    assert np.array_equal(got32, oracle.generate_u32(1, n, iters))


@pytest.mark.parametrize("n,i1,i2", [(1, 3, 5), (4099, 7, 11), (65536, 64, 1)])
def test_checkpoint_resume_continues_the_streams(oracle, n, i1, i2):
    seed = 0xfeedface12345678
    rngx.init(seed, n)
    first = torch.empty(n * i1, dtype=torch.int64, device="cuda")
    rngx.generate(i1, first)
    states, s, c = rngx.get_state()
    assert (s, c) == (seed, i1)
    # The checkpoint is the next value of every stream.
    assert np.array_equal(states, oracle.generate(seed, n, 1, cursor=i1).ravel())
    rngx.shutdown()
    rngx.set_state(s, states, c)
    assert rngx.info() == (seed, n, i1)
    rest = torch.empty(n * i2, dtype=torch.int64, device="cuda")
    rngx.generate(i2, rest)
    torch.cuda.synchronize()
    got = np.concatenate([_u64(first), _u64(rest)])
    assert np.array_equal(got, oracle.generate(seed, n, i1 + i2).ravel())


def test_set_state_from_oracle_states(oracle):
    # States computed on the CPU (value number 1000 of each stream) resume the
    # streams at that point, in u32 form too.
    seed, n = 3, 333
    rngx.set_state(seed, oracle.generate(seed, n, 1, cursor=1000).ravel(), 1000)
    out = torch.empty(n * 4, dtype=torch.int32, device="cuda")
    rngx.generate_u32(4, out)
    torch.cuda.synchronize()
    assert np.array_equal(_u32(out), oracle.generate_u32(seed, n, 4, cursor=1000).ravel())
    st, _, c = rngx.get_state()
    assert c == 1004 and np.array_equal(st, oracle.generate(seed, n, 1, cursor=1004).ravel())
    big = np.empty(n + 1, dtype=np.uint64)
    assert rngx.lib().rngx_get_state(big.ctypes.data, n + 1, None, None) == rngx.RNGX_E_INVAL


@pytest.fixture
def star():
    rngx.set_scrambler(rngx.SCRAMBLE_STAR)
    yield
    rngx.set_scrambler(rngx.SCRAMBLE_NONE)


@pytest.mark.parametrize("u32", [False, True])
@pytest.mark.parametrize("n", [1, 3, 64, 65, 1025, 100003])
def test_scrambled_output_matches_oracle(oracle, star, n, u32):
    for iters, offset, seed in [(1, 0, 5), (4, 1, 0), (3, 0, 2**64 - 1)]:
        got = run(seed, n, iters, u32=u32, offset=offset)
        exp = (oracle.generate_star_u32 if u32 else oracle.generate_star)(seed, n, iters)
        assert np.array_equal(got, exp), (n, iters, offset, seed)


@pytest.mark.parametrize("u32", [False, True])
def test_scrambled_every_launch_config(oracle, star, u32):
    n, iters, seed = 20011, 3, 9
    exp = (oracle.generate_star_u32 if u32 else oracle.generate_star)(seed, n, iters)
    default = rngx.get_launch(u32)
    try:
        for block, chunks, nt in itertools.product([64, 256, 1024], [1, 2, 4], [0, 1]):
            rngx.set_launch(u32, block, chunks, nt)
            assert np.array_equal(run(seed, n, iters, u32=u32), exp), (block, chunks, nt)
    finally:
        rngx.set_launch(u32, **default)


def test_scrambler_switch_keeps_the_state_sequence(oracle):
    # The scrambler changes only the emitted words: switching it between
    # calls continues the same streams.
    seed, n = 31, 777
    rngx.init(seed, n)
    a = torch.empty(2 * n, dtype=torch.int64, device="cuda")
    b = torch.empty(3 * n, dtype=torch.int64, device="cuda")
    rngx.generate(2, a)
    rngx.set_scrambler(rngx.SCRAMBLE_STAR)
    try:
        rngx.generate(3, b)
    finally:
        rngx.set_scrambler(rngx.SCRAMBLE_NONE)
    torch.cuda.synchronize()
    assert np.array_equal(_u64(a).reshape(2, n), oracle.generate(seed, n, 2))
    assert np.array_equal(_u64(b).reshape(3, n), oracle.generate_star(seed, n, 3, cursor=2))
    st, _, c = rngx.get_state()
    assert c == 5 and np.array_equal(st, oracle.generate(seed, n, 1, cursor=5).ravel())


def test_cursor_may_not_pass_the_last_value_number(oracle):
    # The cursor (the next value number) stays at most 2^64 - 1.
    st = oracle.generate(1, 4, 1).ravel()
    rngx.set_state(1, st, 2**64 - 4)
    out = torch.empty(4 * 4, dtype=torch.int64, device="cuda")
    assert rngx.lib().rngx_generate(4, out.data_ptr(), None) == rngx.RNGX_E_INVAL
    rngx.generate(3, out)
    assert rngx.info()[2] == 2**64 - 1
    assert rngx.lib().rngx_generate(1, out.data_ptr(), None) == rngx.RNGX_E_INVAL


@pytest.mark.parametrize("n", [12345, 65540])
@pytest.mark.parametrize("u32", [False, True])
def test_plain_autotuner_keeps_state_and_output(oracle, u32, n):
    # Every candidate starts from the same snapshot: the tuner's output is
    # the next n_iters iterations, the cursor does not move, and the fastest
    # configuration becomes the launch configuration of that output type.
    # 18 unscheduled bases, each base at 3 row schedules, then 8 more
    # schedules on the two bases fastest with one (run scheduled at
    # n = 65540, whose rows are 16-byte aligned).
    seed, iters = 9, 6
    old = rngx.get_launch(u32)
    try:
        rngx.init(seed, n)
        pre = torch.empty(3 * n, dtype=torch.int64, device="cuda")
        rngx.generate(3, pre)
        out = torch.zeros(iters * n + 1, dtype=torch.int32 if u32 else torch.int64, device="cuda")
        res = rngx.autotune_plain(iters, out, reps=1, u32=u32)
        tried = res["tried"]
        assert len(tried) == 88 and res["best_ms"] > 0
        bases = [c for c, _ in tried[:18]]
        assert all(c["pace_gbs"] == 0 for c in bases)
        assert len({tuple(c.values()) for c in bases}) == 18
        coarse = tried[18:72]
        assert [c["pace_gbs"] for c, _ in coarse] == [6000, 6750, 7500] * 18
        assert [{**c, "pace_gbs": 0} for c, _ in coarse[::3]] == bases
        best_sched = [min(t for _, t in coarse[3 * i:3 * i + 3]) for i in range(18)]
        top = sorted(range(18), key=lambda i: (best_sched[i], i))[:2]
        fine = tried[72:]
        fine_paces = [5500, 5750, 6250, 6500, 7000, 7250, 7750, 8000]
        assert [c["pace_gbs"] for c, _ in fine] == fine_paces * 2
        assert [{**c, "pace_gbs": 0} for c, _ in fine[::8]] == [bases[i] for i in top]
        # Confirmation: the four fastest again; the fastest of those wins.
        top4 = sorted(tried, key=lambda t: t[1])[:4]
        assert [c for c, _ in res["confirm"]] == [c for c, _ in top4]
        assert all(ms > 0 for _, ms in res["confirm"])
        assert res["best"] == min(res["confirm"], key=lambda t: t[1])[0]
        assert res["best_ms"] == min(ms for _, ms in res["confirm"])
        assert rngx.get_launch(u32) == res["best"]
        assert rngx.info()[2] == 3
        exp = oracle.generate(seed, n, 3 + 2 * iters)
        got = (_u32 if u32 else _u64)(out)
        assert got[-1] == 0
        want = exp[3:3 + iters]
        if u32:
            want = (want & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        assert np.array_equal(got[:-1].reshape(iters, n), want)
        # The generator continues from where it was before tuning.
        nxt = torch.empty(iters * n, dtype=torch.int64, device="cuda")
        rngx.generate(iters, nxt)
        torch.cuda.synchronize()
        assert np.array_equal(_u64(nxt).reshape(iters, n), exp[3:3 + iters])
    finally:
        rngx.set_launch(u32, **old)


def test_tune_cache_roundtrip(tmp_path):
    rngx.init(1, 4096)
    old64, old32, oldb = rngx.get_launch(False), rngx.get_launch(True), rngx.get_batch_cfg()
    path = tmp_path / "tune.jsonl"
    try:
        rngx.set_launch(False, 1024, 2, True, 6250)
        rngx.set_launch(True, 256, 1, False)
        rngx.set_batch_cfg(16, 4, 0, False, 16, 0, False, 64, 16, 7000)
        rngx.tune_cache_save(path)
        # An entry of another device is kept on save and ignored on load.
        other = ('{"device": "gfx000 1cu", "kind": "plain_u64", "block": 64, "chunks": 1, '
                 '"nontemporal": 0, "tuned_on": "x", "ms": 0.000000}')
        path.write_text(other + "\n" + path.read_text())
        rngx.set_launch(False, 512, 4, False)
        rngx.set_launch(True, 512, 4, False)
        rngx.set_batch_cfg()
        assert rngx.tune_cache_load(path) == 3
        assert rngx.get_launch(False) == {"block": 1024, "chunks": 2, "nontemporal": True,
                                          "pace_gbs": 6250}
        assert rngx.get_launch(True) == {"block": 256, "chunks": 1, "nontemporal": False,
                                         "pace_gbs": 0}
        assert rngx.get_batch_cfg() == {"values_per_lane": 16, "waves_per_block": 4,
                                        "blocks": 0, "use_graph": False, "row_values": 16,
                                        "run_items": 0, "per_item": False, "group": 64,
                                        "group_steps": 16, "pace_gbs": 7000}
        rngx.tune_cache_save(path)
        lines = path.read_text().splitlines()
        # Kept, in the current form (a line without pace_gbs has no schedule).
        assert lines[0] == other.replace('"nontemporal": 0,', '"nontemporal": 0, "pace_gbs": 0,')
        assert len(lines) == 4
    finally:
        rngx.set_launch(False, **old64)
        rngx.set_launch(True, **old32)
        rngx.set_batch_cfg(**oldb)
