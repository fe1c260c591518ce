"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

The paper prints no output values for its generator, so the oracle is pinned
by: hand-traced values of its listings (tests/golden), the full-period
property of the (21,35,4) xorshift over GF(2) (Marsaglia's triple), the
GF(2) machinery itself checked by brute-force orbit enumeration at reduced
word widths, exhaustive bijectivity of both 32-bit hashes, the never-zero
invariant (including the one constructed seed/gid that triggers the zero
fix-up of the seeded reading), identities between its functions, and
bit-frequency sanity.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

from tests import gf2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


def _read_trace():
    blocks, cur, consts = {}, None, {}
    with open(os.path.join(GOLDEN, "init_rng_trace.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = line.split()
            if k == "gid":
                cur = int(v)
                blocks[cur] = {}
            elif k in ("J0", "W0"):
                consts[k] = int(v, 16)
            else:
                blocks[cur][k] = int(v, 16)
    return blocks, consts


# --- hand-traced values (Listings S4, S5) ------------------------------------

def test_hand_trace_seed0(oracle):
    blocks, consts = _read_trace()
    assert sorted(blocks) == [0, 1, 2, 3]
    assert oracle.hash_low(0) == consts["J0"]
    assert oracle.hash_high(0) == consts["W0"]
    for g, b in blocks.items():
        lo = oracle.hash_low(g)
        assert lo == b["J.r6"], g
        hi = oracle.hash_high(lo)
        assert hi == b["W.r5"], g
        x0 = oracle.init_state(0, g)
        assert x0 == b["x0"] == (hi << 32) | lo
        x1 = oracle.rng_step(x0)
        assert x1 == b["x1"]
        assert oracle.rng_step(x1) == b["x2"]
        assert oracle.value(0, g, 2) == b["x2"]
    # gid 0 carries the per-round trace; its last shift-xor is x1.
    assert blocks[0]["xs.r3"] == blocks[0]["x1"]


def test_seeded_extension_values(oracle):
    rows = 0
    with open(os.path.join(GOLDEN, "seeded_extension.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            s, g0, g1, x1 = line.split()
            seed = int(s, 16)
            assert oracle.init_state(seed, 0) == int(g0, 16), s
            assert oracle.init_state(seed, 1) == int(g1, 16), s
            assert oracle.value(seed, 0, 1) == int(x1, 16), s
            rows += 1
    assert rows == 4


def test_seed_zero_is_the_paper(oracle):
    # With seed 0 the seeded reading must reduce to Listing S4 exactly:
    # low = J(gid), high = W(low).
    rng = np.random.default_rng(7)
    for g in [0, 1, 2, 65535, 65536, 2**31, 2**32 - 1] + list(rng.integers(0, 2**32, 200)):
        g = int(g)
        lo = oracle.hash_low(g)
        assert oracle.init_state(0, g) == (oracle.hash_high(lo) << 32) | lo


# --- the xorshift over GF(2) ---------------------------------------------------

PRIMES_2_64_MINUS_1 = [3, 5, 17, 257, 641, 65537, 6700417]


def test_factorisation_of_2_64_minus_1():
    assert math.prod(PRIMES_2_64_MINUS_1) == M64
    assert all(gf2.is_prime(p) for p in PRIMES_2_64_MINUS_1)


def test_xorshift_is_linear_and_invertible(oracle):
    rng = np.random.default_rng(11)
    for _ in range(500):
        a, b = (int(v) for v in rng.integers(0, 2**64, 2, dtype=np.uint64))
        assert oracle.rng_step(a ^ b) == oracle.rng_step(a) ^ oracle.rng_step(b)
    assert oracle.rng_step(0) == 0

    # Inverse of one step, undoing the three shift-xors in reverse order.
    def undo_left(y, k):
        x = y
        for _ in range(64 // k + 1):
            x = (y ^ (x << k)) & M64
        return x

    def undo_right(y, k):
        x = y
        for _ in range(64 // k + 1):
            x = y ^ (x >> k)
        return x

    def back(x):
        return undo_left(undo_right(undo_left(x, 4), 35), 21)

    x0 = oracle.init_state(0, 12345)
    x = oracle.value(0, 12345, 1000)
    for _ in range(1000):
        x = back(x)
    assert x == x0


def test_xorshift_21_35_4_has_full_period(oracle):
    # The matrix is probed from the oracle itself (column j = step(e_j)); its
    # multiplicative order must be exactly 2^64 - 1, so every nonzero state
    # lies on one cycle through all 2^64 - 1 nonzero words.
    T = gf2.from_linear_map(oracle.rng_step, 64)
    assert gf2.has_full_period(T, PRIMES_2_64_MINUS_1)
    # Structure: T = (I + L^4)(I + R^35)(I + L^21), shifts applied in that order.
    def L(k):
        return gf2.from_linear_map(lambda x: (x << k) & M64, 64)

    def R(k):
        return gf2.from_linear_map(lambda x: x >> k, 64)

    def ip(m):
        return [row ^ (1 << r) for r, row in enumerate(m)]
    assert T == gf2.mul(ip(L(4)), gf2.mul(ip(R(35)), ip(L(21))))


def test_period_test_rejects_a_planted_wrong_triple():
    # Plant a mistake (last shift 5 instead of 4) in a copy of the step and
    # check that the period test notices it.
    def wrong(x):
        x ^= (x << 21) & M64
        x ^= x >> 35
        x ^= (x << 5) & M64
        return x
    assert not gf2.has_full_period(gf2.from_linear_map(wrong, 64), PRIMES_2_64_MINUS_1)


@pytest.mark.parametrize("w", [8, 12])
def test_gf2_period_machinery_by_orbit_enumeration(w):
    # Reduced word widths: the matrix-order test must agree with brute-force
    # orbit enumeration for every shift triple.
    primes = gf2.prime_factors((1 << w) - 1)
    full = 0
    for a in range(1, w):
        for b in range(1, w):
            for c in range(1, w):
                f = gf2.shift_xor_map(w, a, b, c)
                x, steps = f(1), 1
                while x != 1 and steps <= (1 << w):
                    x, steps = f(x), steps + 1
                by_orbit = steps == (1 << w) - 1
                by_matrix = gf2.has_full_period(gf2.from_linear_map(f, w), primes)
                assert by_orbit == by_matrix, (w, a, b, c)
                full += by_orbit
    assert full > 0


# --- the hashes: exhaustive bijectivity, never-zero ----------------------------

@pytest.fixture(scope="module")
def scanner(tmp_path_factory):
    src = os.path.join(os.path.dirname(__file__), "helpers", "bijection.c")
    so = str(tmp_path_factory.mktemp("scan") / "libscan.so")
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", so, src],
                   check=True)
    lib = ctypes.CDLL(so)
    lib.count_collisions.argtypes = [ctypes.c_void_p]
    lib.count_collisions.restype = ctypes.c_int64
    return lib


@pytest.mark.slow
@pytest.mark.parametrize("name", ["oracle_hash_low_range", "oracle_hash_high_range"])
def test_hashes_are_bijections_on_32_bits(oracle, scanner, name):
    fn = ctypes.cast(getattr(oracle.lib(), name), ctypes.c_void_p)
    assert scanner.count_collisions(fn) == 0


# Algebraic inverses of the two hashes, round by round (each round of
# Listing S4 is invertible). Used only to construct preimages; every
# preimage is then checked by evaluating the oracle forwards.
M32 = 0xFFFFFFFF


def _undo_xor_right(y, k):
    x = y
    for _ in range(32 // k + 1):
        x = y ^ (x >> k)
    return x


def _inv_mul(m):
    return pow(m, -1, 1 << 32)


def inverse_hash_low(y):
    a = _undo_xor_right(y ^ 0xB55A4F09, 16)
    a = ((a - 0xFD7046C5) * _inv_mul(9)) & M32
    x = 0
    for _ in range(5):                    # y = (x + c) ^ (x << 9)
        x = ((a ^ (x << 9)) - 0xD3A2646C) & M32
    a = x
    a = ((a - 0x165667B1) * _inv_mul(33)) & M32
    a = _undo_xor_right(a ^ 0xC761C23C, 19)
    a = ((a - 0x7ED55D16) * _inv_mul(4097)) & M32
    return a


def inverse_hash_high(y):
    a = _undo_xor_right(y, 15)
    a = (a * _inv_mul(0x27D4EB2D)) & M32
    a = _undo_xor_right(a, 4)
    a = (a * _inv_mul(9)) & M32
    a = _undo_xor_right(a, 16) ^ 61
    return a


def test_inverses_round_trip(oracle):
    rng = np.random.default_rng(3)
    for y in [0, 1, M32] + [int(v) for v in rng.integers(0, 2**32, 300)]:
        assert oracle.hash_low(inverse_hash_low(y)) == y
        assert oracle.hash_high(inverse_hash_high(y)) == y


def test_zero_fixup_is_reached_exactly_where_predicted(oracle):
    # At seed 0 the state is never zero: high = W(low) and W(0) != 0.
    assert oracle.hash_high(0) != 0
    # Seeded reading: the pre-fix-up state is zero iff J(gid ^ l) = 0 and
    # W(0 ^ h) = 0. With lo32(seed) = 0 (so l = 0) this needs
    # gid = J^-1(0) and W(hi32 seed) = W^-1(0) ^ W(0).
    g_star = inverse_hash_low(0)
    assert oracle.hash_low(g_star) == 0
    h_needed = inverse_hash_high(0)
    assert oracle.hash_high(h_needed) == 0
    hi_seed = inverse_hash_high(h_needed ^ oracle.hash_high(0))
    assert oracle.hash_high(hi_seed) ^ oracle.hash_high(0) == h_needed
    seed = hi_seed << 32
    assert oracle.init_state(seed, g_star) == oracle.hash_high(0) << 32
    # Its neighbours are ordinary, nonzero states.
    for g in (g_star ^ 1, (g_star + 7) & M32):
        assert oracle.init_state(seed, g) != 0
    # Any other gid under that seed is not the fixed-up state.
    assert oracle.init_state(seed, g_star ^ 1) != oracle.hash_high(0) << 32


def test_states_never_zero_small(oracle):
    for seed in (0, 1, 42, 2**63 + 5):
        out = oracle.generate(seed, 4096, 64)   # raises if any value is 0
        assert (out != 0).all()


# --- identities between the oracle's functions -------------------------------

def test_concatenation(oracle):
    for seed, n, a, b in [(0, 1000, 5, 7), (9, 33, 1, 16), (2**40, 7, 0, 3)]:
        whole = oracle.generate(seed, n, a + b)
        first = oracle.generate(seed, n, a)
        second = oracle.generate(seed, n, b, cursor=a)
        assert np.array_equal(whole, np.concatenate([first, second]))


def test_plain_matches_value_one_by_one(oracle):
    seed, n, i, c = 0xdeadbeef, 37, 11, 5
    out = oracle.generate(seed, n, i, cursor=c)
    for k in range(i):
        for g in range(n):
            assert int(out[k, g]) == oracle.value(seed, g, c + k)


def test_u32_is_low_half(oracle):
    a = oracle.generate(3, 513, 9, cursor=2)
    b = oracle.generate_u32(3, 513, 9, cursor=2)
    assert np.array_equal(b, (a & np.uint64(0xFFFFFFFF)).astype(np.uint32))


def test_batch_transpose_identity(oracle):
    seed, m, i = 42, 300, 17
    reqs = oracle.make_reqs([seed] * m, np.arange(m), np.zeros(m), np.full(m, i))
    batch = oracle.generate_batch(reqs).reshape(m, i)
    assert np.array_equal(batch, oracle.generate(seed, m, i).T)


def test_batch_offsets_and_packing(oracle):
    rng = np.random.default_rng(5)
    m = 40
    seeds = rng.integers(0, 2**64, m, dtype=np.uint64)
    gids = rng.integers(0, 2**32, m, dtype=np.uint64)
    offs = rng.integers(0, 300, m)
    lens = rng.integers(1, 50, m)
    out = oracle.generate_batch(oracle.make_reqs(seeds, gids, offs, lens))
    base = 0
    for j in range(m):
        for t in range(int(lens[j])):
            assert int(out[base + t]) == oracle.value(int(seeds[j]), int(gids[j]), int(offs[j]) + t)
        base += int(lens[j])
    assert base == len(out)


def test_serve_expected_cursor_rule(oracle):
    subs = [(5, 3), (7, 2), (5, 4), (5, 1), (9, 6), (7, 3)]
    res = oracle.serve_expected(11, subs)
    cursors = {5: 0, 7: 0, 9: 0}
    for (g, length), got in zip(subs, res):
        exp = [oracle.value(11, g, cursors[g] + t) for t in range(length)]
        assert [int(v) for v in got] == exp
        cursors[g] += length


# --- bit-frequency sanity (NIST SP 800-22, 2.1 frequency/monobit test) -------

def test_bit_frequency(oracle):
    out = oracle.generate(0, 65536, 256)       # 2^24 values
    N = out.size
    bits = np.unpackbits(out.view(np.uint8)).reshape(N, 64)
    ones = bits.sum(axis=0, dtype=np.int64)
    sigma = math.sqrt(0.25 / N)
    frac = ones / N
    assert np.all(np.abs(frac - 0.5) < 5 * sigma), frac
    total = int(ones.sum())
    nbits = 64 * N
    s_obs = abs(2 * total - nbits) / math.sqrt(nbits)
    p = math.erfc(s_obs / math.sqrt(2))
    assert p >= 0.01, p


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    # Every oracle function, edge sizes included, in a sanitized build: no
    # out-of-bounds access, leak-free allocation paths, no undefined shifts
    # or overflows of signed types.
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "oracle_sanity")
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-Wall", "-Wextra",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(root, "oracle", "oracle.c"),
                    os.path.join(root, "tests", "helpers", "oracle_sanity.c"), "-o", exe],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


# --- slice-at-a-time entries (gid ranges, continuation from a state array) ---

@pytest.mark.parametrize("seed,cursor", [(0, 0), (42, 3), (2**64 - 1, 17)])
def test_range_output_is_the_matching_columns(oracle, seed, cursor):
    # generate_range(g0, g1) equals columns g0..g1 of generate, and the seeded
    # states are value() one by one (value is pinned by the hand trace).
    n, iters = 3000, 6
    full = oracle.generate(seed, n, iters, cursor=cursor)
    for g0, g1 in [(0, n), (0, 1), (1234, 2999), (2999, 3000), (700, 700)]:
        assert np.array_equal(oracle.generate_range(seed, g0, g1, iters, cursor=cursor),
                              full[:, g0:g1]), (g0, g1)
    st = oracle.seed_range(seed, 5, 20, cursor)
    assert [int(v) for v in st] == [oracle.value(seed, g, cursor) for g in range(5, 25)]


def test_range_reaches_the_last_work_item(oracle):
    # The top of the 32-bit gid space, where the range ends at 2^32.
    top = 2**32
    got = oracle.generate_range(9, top - 4, top, 3)
    for j, g in enumerate(range(top - 4, top)):
        assert [int(v) for v in got[:, j]] == [oracle.value(9, g, k) for k in range(3)]


def test_continuation_concatenates(oracle):
    # Rows emitted from a state array continue where the last call stopped:
    # emit(a) then emit(b) equals emit(a + b), and the state array ends at the
    # next value of every stream.
    seed, n = 77, 513
    st = oracle.seed_range(seed, 0, n, 0)
    parts = [oracle.emit_rows(st, a) for a in (1, 4, 2)]
    assert np.array_equal(np.vstack(parts), oracle.generate(seed, n, 7))
    assert np.array_equal(st, oracle.generate(seed, n, 1, cursor=7)[0])


def test_continuation_words(oracle):
    # u32 rows are the low halves, scrambled rows the scrambled words of the
    # same states, scrambled u32 rows their high halves.
    seed, n, rows = 5, 301, 3
    plain = oracle.generate(seed, n, rows)
    for word, exp in [(oracle.WORD_U32, (plain & np.uint64(0xFFFFFFFF)).astype(np.uint32)),
                      (oracle.WORD_STAR, oracle.generate_star(seed, n, rows)),
                      (oracle.WORD_STAR_U32, oracle.generate_star_u32(seed, n, rows))]:
        st = oracle.seed_range(seed, 0, n, 0)
        assert np.array_equal(oracle.emit_rows(st, rows, word), exp), word


def test_gf2_jumper_follows_the_oracle_step(oracle):
    # The GPU tests' expected values for offsets no stepping could reach come
    # from powers of the oracle step's GF(2) matrix. Pinned here against the
    # oracle's sequential stepping for small k, the group law, and the full
    # period (M^(2^64 - 1) = I).
    J = gf2.Jumper(oracle.rng_step)
    rng = np.random.default_rng(64)
    for _ in range(6):
        seed, g = int(rng.integers(0, 2**63)), int(rng.integers(0, 2**32))
        k = int(rng.integers(0, 3000))
        x0 = oracle.init_state(seed, g)
        assert J.jump(x0, k) == oracle.value(seed, g, k)
        a, b = int(rng.integers(0, 2**63)), int(rng.integers(0, 2**63))
        assert J.jump(J.jump(x0, a), b) == J.jump(x0, a + b)
        assert J.jump(x0, 2**64 - 1) == x0
