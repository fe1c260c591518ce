"""Pins of the oracle's scrambled variant (the xorshift* reading of the
paper's remark that a more complex generator would cost nothing).

What fixes it besides its own definition:
  * Linear complexity (Berlekamp-Massey over GF(2)): every output bit of the
    plain generator is a GF(2)-linear recurrence of order at most 64 (the
    state is 64 bits and the step is linear), while a multiplicative
    scrambler makes the high bits nonlinear, so their linear complexity over
    a few hundred values is far above 64. Dropping the multiplication, or
    replacing it with anything GF(2)-linear (a shift, an XOR mask), fails.
  * Odd multiplier: bit 0 of x * M equals bit 0 of x, and multiplying by the
    inverse of M modulo 2^64 (found here by Newton iteration, not taken from
    the oracle) recovers the plain stream exactly.
  * The state sequence is the plain one, so concatenation over the cursor
    holds exactly as for the plain output.
"""
import numpy as np
import pytest

M = 2685821657736338717   # the xorshift* multiplier of Vigna (2016)
MASK = (1 << 64) - 1


def berlekamp_massey(bits):
    """Length of the shortest GF(2) LFSR that generates `bits`."""
    n = len(bits)
    c = [0] * (n + 1); b = [0] * (n + 1)
    c[0] = b[0] = 1
    L, m = 0, -1
    for i in range(n):
        d = bits[i]
        for j in range(1, L + 1):
            d ^= c[j] & bits[i - j]
        if d:
            t = c[:]
            shift = i - m
            for j in range(n + 1 - shift):
                c[j + shift] ^= b[j]
            if 2 * L <= i:
                L, m, b = i + 1 - L, i, t
    return L


def inverse_mod_2_64(a):
    x = a  # correct to 3 bits for odd a; each step doubles the correct bits
    for _ in range(6):
        x = (x * (2 - a * x)) & MASK
    return x


def test_berlekamp_massey_on_known_sequences():
    # An LFSR of order 5 (x^5 + x^2 + 1) has linear complexity 5; a single
    # 1 after zeros has complexity equal to its position + 1.
    s = [1, 0, 0, 1, 0]
    for i in range(5, 60):
        s.append(s[i - 5] ^ s[i - 3])
    assert berlekamp_massey(s) == 5
    assert berlekamp_massey([0] * 9 + [1]) == 10


def test_plain_bits_are_linear_star_bits_are_not(oracle):
    N = 400
    plain = oracle.generate(7, 3, N)            # 3 streams, N values each
    star = oracle.generate_star(7, 3, N)
    for g in range(3):
        for bit in (0, 31, 63):
            pb = [int(v >> np.uint64(bit)) & 1 for v in plain[:, g]]
            assert berlekamp_massey(pb) <= 64, (g, bit)
        for bit in (40, 63):
            sb = [int(v >> np.uint64(bit)) & 1 for v in star[:, g]]
            assert berlekamp_massey(sb) > 150, (g, bit)
    # The 32-bit form is the high half, also nonlinear.
    s32 = oracle.generate_star_u32(7, 1, N)[:, 0]
    assert berlekamp_massey([int(v >> np.uint32(31)) & 1 for v in s32]) > 150


def test_odd_multiplier_is_a_bijection_back_to_the_plain_stream(oracle):
    inv = inverse_mod_2_64(M)
    assert (M * inv) & MASK == 1
    plain = oracle.generate(0xdeadbeef, 257, 9, cursor=123)
    star = oracle.generate_star(0xdeadbeef, 257, 9, cursor=123)
    back = np.array([(int(v) * inv) & MASK for v in star.ravel()], dtype=np.uint64)
    assert np.array_equal(back, plain.ravel())
    assert np.array_equal(star & np.uint64(1), plain & np.uint64(1))


def test_u32_is_the_high_half(oracle):
    star = oracle.generate_star(3, 100, 5, cursor=11)
    assert np.array_equal(oracle.generate_star_u32(3, 100, 5, cursor=11),
                          (star >> np.uint64(32)).astype(np.uint32))


def test_star_concatenation_over_the_cursor(oracle):
    whole = oracle.generate_star(99, 50, 12)
    assert np.array_equal(whole, np.concatenate([oracle.generate_star(99, 50, 5),
                                                 oracle.generate_star(99, 50, 7, cursor=5)]))


def test_seed_zero_first_value_is_the_scrambled_paper_state(oracle):
    # The paper's first state of work-item 0 is pinned by the hand trace.
    x0 = 0x103fe9a06b4ed927
    assert int(oracle.generate(0, 1, 1)[0, 0]) == x0
    assert int(oracle.generate_star(0, 1, 1)[0, 0]) == (x0 * M) & MASK
    assert oracle.scramble(1) == M
