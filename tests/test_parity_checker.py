"""CPU tests of the full-size parity checker (tests/helpers/parity.c): it
finds every planted difference, at the right place, whatever the thread
count, tile boundaries and word type, and reports none on the oracle's own
output."""
import numpy as np
import pytest

from tests import parity


@pytest.fixture(scope="module", autouse=True)
def built(oracle):
    parity.build(force=True)


@pytest.mark.parametrize("word", [parity.WORD_U64, parity.WORD_U32, parity.WORD_STAR,
                                  parity.WORD_STAR_U32])
def test_rows_equal_and_planted_differences(oracle, word):
    seed, n, rows = 11, 70001, 5
    gen = {parity.WORD_U64: oracle.generate, parity.WORD_U32: oracle.generate_u32,
           parity.WORD_STAR: oracle.generate_star,
           parity.WORD_STAR_U32: oracle.generate_star_u32}[word]
    got = gen(seed, n, rows, cursor=2)
    st = parity.seed_states(seed, n, cursor=2)
    assert parity.check_rows(got, st, word)["mismatches"] == 0
    # The state array has moved on by the rows checked.
    assert np.array_equal(st, oracle.generate(seed, n, 1, cursor=7)[0])
    bad = got.copy()
    bad[3, 40000] ^= 1
    bad[4, 0] ^= 1 << 7
    bad[3, 69999] ^= 1 << 31
    res = parity.check_rows(bad, parity.seed_states(seed, n, cursor=2), word)
    assert res["mismatches"] == 3 and res["first"] == (3, 40000)


def test_rows_in_pieces_and_threads(oracle, monkeypatch):
    seed, n, rows = 3, 4099, 9
    got = oracle.generate(seed, n, rows)
    for threads in (1, 3, 16):
        monkeypatch.setattr(parity, "THREADS", threads)
        st = parity.seed_states(seed, n)
        # Rows 0-3, then 4-8, with the same state array; and a column slice.
        assert parity.check_rows(got[:4], st, parity.WORD_U64)["mismatches"] == 0
        assert parity.check_rows(got[4:], st, parity.WORD_U64)["mismatches"] == 0
        st = parity.seed_states(seed, n)
        sub = st[1000:2000]
        bad = np.ascontiguousarray(got[:, 1000:2000])
        bad[8, 999] += np.uint64(1)
        res = parity.check_rows(bad, sub, parity.WORD_U64)
        assert res["mismatches"] == 1 and res["first"] == (8, 999)
        assert np.array_equal(st[1000:2000], oracle.generate(seed, n, 1, cursor=rows)[0, 1000:2000])
        assert np.array_equal(st[:1000], parity.seed_states(seed, 1000))  # untouched


def test_strided_rows(oracle):
    # Rows read with a stride larger than the row (a column window of a
    # wider output).
    seed, n, rows = 8, 5000, 4
    full = oracle.generate(seed, n, rows)
    st = parity.seed_states(seed, 300, g0=1200)
    ptr = full.ctypes.data + 1200 * 8
    assert parity.check_rows_ptr(ptr, n, 300, rows, st, parity.WORD_U64)["mismatches"] == 0


def test_requests_equal_and_planted_differences(oracle):
    seeds, gids = [1, 2**63 + 5, 7, 0], [0, 99, 2**32 - 1, 12]
    offs, lens = [0, 12345, 3, 70000], [5000, 70001, 1, 40000]
    reqs = oracle.make_reqs(seeds, gids, offs, lens)
    flat = oracle.generate_batch(reqs)
    bases = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
    assert parity.check_requests(reqs, flat.ctypes.data, bases)["mismatches"] == 0
    bad = flat.copy()
    bad[5000 + 32768] ^= np.uint64(1 << 63)     # request 1, second tile
    bad[-1] ^= np.uint64(2)                      # request 3, last value
    res = parity.check_requests(reqs, bad.ctypes.data, bases)
    assert res["mismatches"] == 2 and res["first"] == (1, 32768)
    # Requests spread over a buffer with gaps, in another order.
    order = [3, 0, 2]
    gap_bases = np.array([10, 50000, 90001], dtype=np.uint64)
    buf = np.zeros(200000, dtype=np.uint64)
    for b, r in zip(gap_bases, order):
        start = int(bases[r])
        buf[int(b):int(b) + lens[r]] = flat[start:start + lens[r]]
    assert parity.check_requests(reqs[order], buf.ctypes.data, gap_bases)["mismatches"] == 0
    # Scrambled words.
    star = oracle.scramble_array(flat)
    assert parity.check_requests(reqs, star.ctypes.data, bases,
                                 parity.WORD_STAR)["mismatches"] == 0


def test_requests_with_given_starts(oracle):
    # With starts given, the checker continues from them instead of stepping
    # to the offset; a wrong start is caught.
    reqs = oracle.make_reqs([5, 6], [1, 2], [2**40, 10], [100, 100])
    starts = np.array([oracle.value(5, 1, 0), oracle.value(6, 2, 10)], dtype=np.uint64)
    # Request 0 "at offset 2^40" with the offset-0 state as its start: the
    # expected values are those of offset 0.
    got = np.concatenate([oracle.generate_batch(oracle.make_reqs([5], [1], [0], [100])),
                          oracle.generate_batch(reqs[1:])])
    bases = np.array([0, 100], dtype=np.uint64)
    assert parity.check_requests(reqs, got.ctypes.data, bases, starts=starts)["mismatches"] == 0
    starts[1] = oracle.rng_step(int(starts[1]))
    res = parity.check_requests(reqs, got.ctypes.data, bases, starts=starts)
    assert res["mismatches"] == 100 and res["first"] == (1, 0)
