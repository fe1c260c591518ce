"""Linear algebra over GF(2) for w-bit words (test helper).

A w x w matrix is a list of w Python ints; row r holds, as bit j, whether
output bit r depends on input bit j, so (M x)_r = parity(row_r & x).
"""
from __future__ import annotations


def identity(w):
    return [1 << r for r in range(w)]


def from_linear_map(f, w):
    """Matrix of a GF(2)-linear map f on w-bit words, probed on unit vectors."""
    cols = [f(1 << j) for j in range(w)]
    rows = []
    for r in range(w):
        v = 0
        for j in range(w):
            if (cols[j] >> r) & 1:
                v |= 1 << j
        rows.append(v)
    return rows


def apply(m, x):
    y = 0
    for r, row in enumerate(m):
        if bin(row & x).count("1") & 1:
            y |= 1 << r
    return y


def mul(a, b):
    """(a b) x = a (b x)."""
    out = []
    for row in a:
        acc = 0
        j = 0
        while row:
            if row & 1:
                acc ^= b[j]
            row >>= 1
            j += 1
        out.append(acc)
    return out


def power(m, e):
    w = len(m)
    result = identity(w)
    base = m
    while e:
        if e & 1:
            result = mul(result, base)
        base = mul(base, base)
        e >>= 1
    return result


def prime_factors(n):
    fs, p = [], 2
    while p * p <= n:
        while n % p == 0:
            if p not in fs:
                fs.append(p)
            n //= p
        p += 1
    if n > 1:
        fs.append(n)
    return fs


def is_prime(n):
    return n > 1 and prime_factors(n) == [n]


def has_full_period(m, primes):
    """True iff the matrix has multiplicative order exactly 2^w - 1, i.e. the
    linear recurrence x -> m x visits every nonzero w-bit word."""
    w = len(m)
    order = (1 << w) - 1
    ident = identity(w)
    if power(m, order) != ident:
        return False
    return all(power(m, order // p) != ident for p in primes)


def shift_xor_map(w, a, b, c):
    """Reduced-width xorshift x ^= x<<a; x ^= x>>b; x ^= x<<c on w bits."""
    mask = (1 << w) - 1

    def f(x):
        x ^= (x << a) & mask
        x ^= x >> b
        x ^= (x << c) & mask
        return x
    return f


class Jumper:
    """k steps of a GF(2)-linear step map on w-bit words, for any k < 2^w:
    the matrices M^(2^b) are built once by repeated squaring of the step's
    matrix (probed from the step function on unit vectors), and M^k x is
    the product of those with b a set bit of k, applied one after another."""

    def __init__(self, step, w=64):
        self.pow2 = [from_linear_map(step, w)]
        for _ in range(w - 1):
            self.pow2.append(mul(self.pow2[-1], self.pow2[-1]))

    def jump(self, x, k):
        b = 0
        while k:
            if k & 1:
                x = apply(self.pow2[b], x)
            k >>= 1
            b += 1
        return x
