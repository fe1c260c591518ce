"""GPU parity of the batched ragged-stream path against the oracle."""
import itertools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1609_01257_amd import inputs, rngx
from tests import gf2, parity

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _default_batch_cfg():
    old = rngx.get_batch_cfg()
    yield
    rngx.set_batch_cfg(**old)


def _reqs(r: inputs.Requests):
    return rngx.make_reqs(r.seeds, r.gids, r.offsets, r.lengths)


def _oracle_reqs(oracle, r: inputs.Requests):
    return oracle.make_reqs(r.seeds, r.gids, r.offsets, r.lengths)


def _run(reqs, total, pad=7):
    out = torch.zeros(total + pad, dtype=torch.int64, device="cuda")
    rngx.generate_batch(reqs, out)
    torch.cuda.synchronize()
    host = out.cpu().numpy().view(np.uint64)
    assert (host[total:] == 0).all(), "write past the packed output"
    return host[:total]


@pytest.mark.parametrize("seed", range(6))
def test_small_ragged_tables(oracle, seed):
    r = inputs.ragged_requests(m=37, seed=seed, max_len=70000, max_offset=200000)
    exp = oracle.generate_batch(_oracle_reqs(oracle, r))
    got = _run(_reqs(r), r.total)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("S,wpb,graph,row,run", list(itertools.product(
    [16, 32, 64, 128, 256, 512, 1024], [1, 2, 4], [False, True], [8, 16], [1, 3, 8, 64])))
def test_every_launch_config(oracle, S, wpb, graph, row, run):
    r = inputs.ragged_requests(m=23, seed=99, max_len=400000, max_offset=5000)
    exp = oracle.generate_batch(_oracle_reqs(oracle, r))
    rngx.set_batch_cfg(S, wpb, 37, graph, row, run)
    assert np.array_equal(_run(_reqs(r), r.total), exp)


@pytest.mark.parametrize("S,wpb,graph,row", list(itertools.product(
    [16, 32, 64, 128, 256, 512, 1024], [1, 2, 4], [False, True], [8, 16])))
def test_every_per_item_config(oracle, S, wpb, graph, row):
    # One wave per work item: the grid follows the item count.
    r = inputs.ragged_requests(m=23, seed=98, max_len=400000, max_offset=5000)
    exp = oracle.generate_batch(_oracle_reqs(oracle, r))
    rngx.set_batch_cfg(S, wpb, 0, graph, row, 1, True)
    assert np.array_equal(_run(_reqs(r), r.total), exp)


# The grouped order: groups of wavefronts moving through regions of
# consecutive tiles together, carrying state `group` tiles on within a
# request; 1 and 5 steps per region put most items at region edges, 16
# steps carry most of them; the 5-step cases also run a slow schedule.
@pytest.mark.parametrize("S,wpb,graph,group,steps", list(itertools.product(
    [8, 16, 64], [1, 4], [False, True], [16, 64, 128], [1, 5, 16])))
def test_every_group_config(oracle, S, wpb, graph, group, steps):
    r = inputs.ragged_requests(m=23, seed=97, max_len=400000, max_offset=5000)
    exp = oracle.generate_batch(_oracle_reqs(oracle, r))
    rngx.set_batch_cfg(S, wpb, 0, graph, 8 if S == 8 else 16, 0, False, group, steps,
                       2000 if steps == 5 else 0)
    assert np.array_equal(_run(_reqs(r), r.total), exp)


@pytest.mark.parametrize("entry", ["generate_batch", "generate_batch_noalloc"])
@pytest.mark.parametrize("star", [False, True])
def test_group_order_long_streams_and_scrambler(oracle, entry, star):
    # Requests of up to 2^21 values (many carried steps per wavefront), the
    # scheduled grouped order the autotuner tries, both entry points.
    r = inputs.ragged_requests(m=40, seed=5, max_len=1 << 21, max_offset=10**9)
    exp = oracle.generate_batch(_oracle_reqs(oracle, r))
    if star:
        exp = oracle.scramble_array(exp)
    rngx.set_batch_cfg(8, 4, 0, entry == "generate_batch", 8, 0, False, 32, 16, 7000)
    rngx.set_scrambler(rngx.SCRAMBLE_STAR if star else rngx.SCRAMBLE_NONE)
    try:
        out = torch.zeros(r.total + 9, dtype=torch.int64, device="cuda")
        getattr(rngx, entry)(_reqs(r), out[2:2 + r.total])
        torch.cuda.synchronize()
    finally:
        rngx.set_scrambler(rngx.SCRAMBLE_NONE)
    host = out.cpu().numpy().view(np.uint64)
    assert not host[:2].any() and not host[2 + r.total:].any()
    assert np.array_equal(host[2:2 + r.total], exp)


@pytest.mark.parametrize("m", [1, 2, 7, 15, 16, 17])
@pytest.mark.parametrize("S", [16, 64, 256])
def test_small_tables_in_kernel_arguments(oracle, m, S):
    # Up to 16 requests, one wave per item and no graph: the request table
    # travels in the kernel's arguments (17 takes the uploaded-table path).
    r = inputs.ragged_requests(m=m, seed=500 + m, max_len=90000, max_offset=10**6)
    exp = oracle.generate_batch(_oracle_reqs(oracle, r))
    for row in (8, 16):
        rngx.set_batch_cfg(S, 4, 0, False, row, 1, True)
        assert np.array_equal(_run(_reqs(r), r.total), exp), row


@pytest.mark.parametrize("entry", ["generate_batch", "generate_batch_noalloc"])
@pytest.mark.parametrize("cfg", [dict(values_per_lane=256, waves_per_block=4, blocks=0,
                                      use_graph=True, row_values=16, run_items=1),
                                 dict(values_per_lane=64, waves_per_block=2, blocks=0,
                                      use_graph=False, row_values=16, run_items=1,
                                      per_item=True),
                                 dict(values_per_lane=128, waves_per_block=4, blocks=50,
                                      use_graph=False, row_values=8, run_items=8)],
                         ids=["persistent", "per-item", "runs-rows8"])
def test_output_at_every_16_byte_offset_of_a_line(oracle, entry, cfg):
    # The packed output may start anywhere 16-byte aligned; its tiles are
    # laid on its 128-byte lines, whatever its offset in the line.
    r = inputs.ragged_requests(m=29, seed=77, max_len=90000, max_offset=3000)
    exp = oracle.generate_batch(_oracle_reqs(oracle, r))
    rngx.set_batch_cfg(**cfg)
    buf = torch.zeros(r.total + 32, dtype=torch.int64, device="cuda")
    assert buf.data_ptr() % 128 == 0
    for skew in range(0, 16, 2):
        buf.zero_()
        getattr(rngx, entry)(_reqs(r), buf[skew:skew + r.total])
        torch.cuda.synchronize()
        host = buf.cpu().numpy().view(np.uint64)
        assert not host[:skew].any() and not host[skew + r.total:].any(), skew
        assert np.array_equal(host[skew:skew + r.total], exp), skew


def test_per_item_graph_follows_item_count(oracle):
    # The captured graph is re-captured when the item count changes and
    # reused when it does not; every replay checked against the oracle.
    rngx.set_batch_cfg(64, 4, 0, True, 16, 1, True)
    for k, (m, seed) in enumerate([(40, 1), (41, 2), (41, 2), (7, 3), (40, 1)]):
        r = inputs.ragged_requests(m=m, seed=2000 + seed, max_len=50000, max_offset=10**6)
        exp = oracle.generate_batch(_oracle_reqs(oracle, r))
        assert np.array_equal(_run(_reqs(r), r.total), exp), k


def test_tiny_and_zero_length_requests(oracle):
    lengths = [1, 0, 2, 3, 0, 0, 1, 17, 1, 0, 64, 65, 127, 0]
    m = len(lengths)
    r = inputs.Requests(np.arange(m, dtype=np.uint64) * np.uint64(2**61 + 3),
                        np.arange(m, dtype=np.uint32) * 1000,
                        np.arange(m, dtype=np.uint64) * 7, np.array(lengths, dtype=np.uint64))
    exp = oracle.generate_batch(_oracle_reqs(oracle, r))
    for graph, row, run, per_item in ((False, 16, 1, False), (True, 8, 4, False),
                                      (False, 16, 1, True), (True, 8, 1, True)):
        rngx.set_batch_cfg(64, 1, 5, graph, row, run, per_item)
        assert np.array_equal(_run(_reqs(r), r.total), exp)


@pytest.fixture(scope="module")
def jumper(oracle):
    # k oracle steps for any k: powers of the step's GF(2) matrix, probed
    # from the oracle's own step function (independent of the library's
    # jump tables).
    return gf2.Jumper(oracle.rng_step)


def test_huge_offsets_use_jump_ahead(oracle, jumper):
    # Offsets far beyond what stepping could reach; checked through the
    # group law value(s, g, k) = M^k x0 with M the matrix of the oracle's
    # step: the first value of each request is M^k applied to the oracle's
    # initial state, and the checker continues from it with sequential
    # oracle steps.
    rng = np.random.default_rng(17)
    m = 12
    offs = rng.integers(2**40, 2**63, m, dtype=np.uint64)
    r = inputs.Requests(rng.integers(0, 2**64, m, dtype=np.uint64),
                        rng.integers(0, 2**32, m, dtype=np.uint64).astype(np.uint32),
                        offs, rng.integers(1, 3000, m).astype(np.uint64))
    got = _run(_reqs(r), r.total)
    starts = np.array([jumper.jump(oracle.init_state(int(r.seeds[j]), int(r.gids[j])),
                                   int(offs[j])) for j in range(m)], dtype=np.uint64)
    bases = np.concatenate([[0], np.cumsum(r.lengths)[:-1]]).astype(np.uint64)
    res = parity.check_requests(_oracle_reqs(oracle, r), got.ctypes.data, bases, starts=starts)
    assert res["mismatches"] == 0, res


def test_transpose_of_plain_output(oracle):
    # All seeds s, gid_j = j, length i, offset 0: the transpose of the plain grid.
    seed, n, iters = 77, 1000, 300
    r = rngx.make_reqs([seed] * n, np.arange(n), np.zeros(n), np.full(n, iters))
    got = _run(r, n * iters).reshape(n, iters)
    assert np.array_equal(got.T, oracle.generate(seed, n, iters))


def test_graph_replays_with_changing_tables(oracle):
    # One captured graph, replayed for different tables, with eager work and
    # synchronisations in between; every replay checked against the oracle.
    rngx.set_batch_cfg(256, 4, 64, True)
    big = torch.zeros(1 << 22, dtype=torch.int64, device="cuda")
    for k in range(5):
        r = inputs.ragged_requests(m=40 + k, seed=1000 + k, max_len=50000, max_offset=10**6)
        exp = oracle.generate_batch(_oracle_reqs(oracle, r))
        big.add_(1)                          # unrelated eager work on the device
        out = torch.zeros(r.total, dtype=torch.int64, device="cuda")
        rngx.generate_batch(_reqs(r), out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint64), exp), k
    assert int(big[0]) == 5


def test_checksum_matches_numpy(oracle):
    r = inputs.ragged_requests(m=10, seed=3, max_len=100000)
    exp = oracle.generate_batch(_oracle_reqs(oracle, r))
    out = torch.zeros(r.total, dtype=torch.int64, device="cuda")
    rngx.generate_batch(_reqs(r), out)
    idx = np.arange(r.total, dtype=np.uint64)
    with np.errstate(over="ignore"):
        want = int(np.sum(exp * (np.uint64(2) * idx + np.uint64(1)), dtype=np.uint64))
    assert rngx.checksum(out) == want


def test_autotune_agrees_across_candidates(oracle):
    r = inputs.ragged_requests(m=64, seed=8, max_len=300000)
    out = torch.zeros(r.total, dtype=torch.int64, device="cuda")
    res = rngx.autotune_batch(_reqs(r), out, reps=1)
    assert len(res["tried"]) == 60 and res["best_ms"] > 0
    assert {c["run_items"] for c, _ in res["tried"][:32]} == {1, 8}
    grouped = [c for c, _ in res["tried"][32:]]
    assert {(c["values_per_lane"], c["group"], c["group_steps"]) for c in grouped} == {
        (16, g, k) for g in (16, 32) for k in (8, 16)}
    assert {c["pace_gbs"] for c in grouped} == {5750, 6000, 6125, 6250, 6375, 6500, 6750}
    # Confirmation: the four fastest again; the fastest of those wins.
    top4 = sorted(res["tried"], key=lambda t: t[1])[:4]
    assert [c for c, _ in res["confirm"]] == [c for c, _ in top4]
    assert res["best"] == min(res["confirm"], key=lambda t: t[1])[0]
    assert res["best_ms"] == min(ms for _, ms in res["confirm"])
    assert {c["per_item"] for c, _ in res["tried"]} == {False}
    assert rngx.get_batch_cfg() == res["best"]
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64),
                          oracle.generate_batch(_oracle_reqs(oracle, r)))


def test_zero_state_fixup_on_the_device(oracle):
    # The one gid whose hashed state is zero under a seed with lo32 = 0 and
    # a chosen hi32 (built from the hashes' inverses, as in the oracle pin)
    # must start from the replacement state W(0) << 32 on the device too.
    from tests.test_oracle_pins import inverse_hash_high, inverse_hash_low
    g_star = inverse_hash_low(0)
    h_needed = inverse_hash_high(0)
    seed = inverse_hash_high(h_needed ^ oracle.hash_high(0)) << 32
    assert oracle.init_state(seed, g_star) == oracle.hash_high(0) << 32
    gids = [g_star, g_star ^ 1, g_star, g_star]
    offsets = [0, 0, 12345, 1000003]
    lengths = [100, 100, 50, 70]
    exp = oracle.generate_batch(oracle.make_reqs([seed] * 4, gids, offsets, lengths))
    assert exp[0] == oracle.hash_high(0) << 32
    for S, per_item in ((64, True), (256, False)):
        rngx.set_batch_cfg(S, 4, 0, False, 16, 1, per_item)
        got = _run(rngx.make_reqs([seed] * 4, gids, offsets, lengths), sum(lengths))
        assert np.array_equal(got, exp), (S, per_item)


def test_batch_errors_on_device():
    r = rngx.make_reqs([1, 2], [0, 1], [0, 0], [10, 20])
    out = torch.zeros(64, dtype=torch.int64, device="cuda")
    L = rngx.lib()
    assert L.rngx_generate_batch(r.ctypes.data, 2, out.data_ptr(), 29, None) == rngx.RNGX_E_INVAL
    assert L.rngx_generate_batch(r.ctypes.data, 2, out.data_ptr() + 8, 60, None) == rngx.RNGX_E_INVAL
    assert L.rngx_generate_batch(r.ctypes.data, 2, out.data_ptr(), 30, None) == rngx.RNGX_OK
    assert L.rngx_generate_batch(r.ctypes.data, 0, out.data_ptr(), 0, None) == rngx.RNGX_OK


def test_last_value_numbers_of_a_stream(oracle, jumper):
    # A request may end exactly at value number 2^64 - 1; checked through the
    # group law (value k+1 = one step from value k) from M^k x0, M the
    # matrix of the oracle's step. M^(2^64 - 1) is the identity (full
    # period), so value number 2^64 - 1 is the initial state itself.
    r = rngx.make_reqs([5, 5], [3, 4], [2**64 - 6, 2**64 - 1], [6, 1])
    got = _run(r, 7)
    assert int(got[6]) == oracle.init_state(5, 4)
    for j, (off, n, base) in enumerate([(2**64 - 6, 6, 0), (2**64 - 1, 1, 6)]):
        x = jumper.jump(oracle.init_state(5, 3 + j), off)
        for t in range(n):
            assert int(got[base + t]) == x, (j, t)
            x = oracle.rng_step(x)
    L = rngx.lib()
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    late = rngx.make_reqs([5], [3], [2**64 - 5], [6])
    assert L.rngx_generate_batch(late.ctypes.data, 1, out.data_ptr(), 8, None) == rngx.RNGX_E_INVAL


@pytest.mark.parametrize("S,per_item,graph,m", [(256, False, True, 23), (64, True, False, 23),
                                                (64, True, False, 9), (128, True, True, 23),
                                                (32, False, False, 23)])
def test_scrambled_batches_match_oracle(oracle, S, per_item, graph, m):
    # The scrambler applies to batched output: each value's scrambled word.
    r = inputs.ragged_requests(m=m, seed=77 + m, max_len=200000, max_offset=10**6)
    exp = oracle.scramble_array(oracle.generate_batch(_oracle_reqs(oracle, r)))
    rngx.set_batch_cfg(S, 4, 0 if per_item else 37, graph, 16, 1 if per_item else 3, per_item)
    rngx.set_scrambler(rngx.SCRAMBLE_STAR)
    try:
        got = _run(_reqs(r), r.total)
        # Switching back gives the plain words again (a captured graph too).
        rngx.set_scrambler(rngx.SCRAMBLE_NONE)
        plain = _run(_reqs(r), r.total)
    finally:
        rngx.set_scrambler(rngx.SCRAMBLE_NONE)
    assert np.array_equal(got, exp)
    assert np.array_equal(plain, oracle.generate_batch(_oracle_reqs(oracle, r)))
