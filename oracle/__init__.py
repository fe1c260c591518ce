"""CPU oracle for the cf4ocl paper's massive PRNG example (Section 5,
Listings S4 and S5) -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package. The GPU library never imports it, and the two
share no code: this module loads ``liboracle.so`` (built from ``oracle.c``
with plain gcc) and exposes it with numpy arrays.

The definitions themselves live in ``oracle.c`` (generator and seeding) and
``profile.py`` (the event-profile arithmetic). This file adds only argument
marshalling and one plain bookkeeping rule for served requests
(:func:`serve_expected`).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# The oracle's request record, laid out as in oracle.c.
REQ_DTYPE = np.dtype([("seed", "<u8"), ("offset", "<u8"), ("length", "<u8"),
                      ("gid", "<u4"), ("reserved", "<u4")])


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc -O2 (plain C99)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-fPIC",
                        "-shared", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u32, u64, p = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
        L.oracle_hash_low.argtypes = [u32]
        L.oracle_hash_low.restype = u32
        L.oracle_hash_high.argtypes = [u32]
        L.oracle_hash_high.restype = u32
        L.oracle_init_state.argtypes = [u64, u32]
        L.oracle_init_state.restype = u64
        L.oracle_rng_step.argtypes = [u64]
        L.oracle_rng_step.restype = u64
        L.oracle_value.argtypes = [u64, u32, u64]
        L.oracle_value.restype = u64
        L.oracle_generate.argtypes = [u64, u32, u64, u32, p]
        L.oracle_generate.restype = u64
        L.oracle_generate_u32.argtypes = [u64, u32, u64, u32, p]
        L.oracle_generate_u32.restype = u64
        L.oracle_scramble.argtypes = [u64]
        L.oracle_scramble.restype = u64
        L.oracle_scramble_n.argtypes = [p, u64, p]
        L.oracle_scramble_n.restype = None
        L.oracle_generate_star.argtypes = [u64, u32, u64, u32, p]
        L.oracle_generate_star.restype = u64
        L.oracle_generate_star_u32.argtypes = [u64, u32, u64, u32, p]
        L.oracle_generate_star_u32.restype = u64
        L.oracle_generate_batch.argtypes = [p, u32, p]
        L.oracle_generate_batch.restype = u64
        L.oracle_seed_range.argtypes = [u64, u32, u64, u64, p]
        L.oracle_seed_range.restype = None
        L.oracle_emit_rows.argtypes = [p, u64, u32, ctypes.c_int, p, u64]
        L.oracle_emit_rows.restype = u64
        L.oracle_generate_range.argtypes = [u64, u64, u64, u64, u32, p]
        L.oracle_generate_range.restype = u64
        L.oracle_hash_low_range.argtypes = [u32, u64, p]
        L.oracle_hash_low_range.restype = None
        L.oracle_hash_high_range.argtypes = [u32, u64, p]
        L.oracle_hash_high_range.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# --- scalar definitions -----------------------------------------------------

def hash_low(a: int) -> int:
    """Listing S4 low-word hash J."""
    return int(lib().oracle_hash_low(a & 0xFFFFFFFF))


def hash_high(a: int) -> int:
    """Listing S4 high-word hash W."""
    return int(lib().oracle_hash_high(a & 0xFFFFFFFF))


def init_state(seed: int, gid: int) -> int:
    """Initial state of work-item ``gid`` under ``seed`` (seed 0 = paper)."""
    return int(lib().oracle_init_state(seed, gid))


def rng_step(x: int) -> int:
    """Listing S5: one (21,35,4) xorshift step."""
    return int(lib().oracle_rng_step(x))


def value(seed: int, gid: int, k: int) -> int:
    """k-th value of work-item ``gid``'s stream (k sequential steps)."""
    return int(lib().oracle_value(seed, gid, k))


# --- array definitions ------------------------------------------------------

def generate(seed: int, n: int, n_iters: int, cursor: int = 0) -> np.ndarray:
    """Plain output, iteration-major: out[k, g] = value(seed, g, cursor + k)."""
    out = np.empty((n_iters, n), dtype=np.uint64)
    zeros = lib().oracle_generate(seed, n, cursor, n_iters, _ptr(out))
    if zeros:
        raise AssertionError("oracle produced %d zero values" % zeros)
    return out


def generate_u32(seed: int, n: int, n_iters: int, cursor: int = 0) -> np.ndarray:
    """Low 32-bit halves of :func:`generate`."""
    out = np.empty((n_iters, n), dtype=np.uint32)
    zeros = lib().oracle_generate_u32(seed, n, cursor, n_iters, _ptr(out))
    if zeros:
        raise AssertionError("oracle produced %d zero values" % zeros)
    return out


def scramble(x: int) -> int:
    """The scrambled variant's output word for state x (xorshift* reading)."""
    return lib().oracle_scramble(x)


def scramble_array(values: np.ndarray) -> np.ndarray:
    """The scrambled words of an array of uint64 values."""
    a = np.ascontiguousarray(values, dtype=np.uint64)
    out = np.empty_like(a)
    lib().oracle_scramble_n(_ptr(a), a.size, _ptr(out))
    return out


def generate_star(seed: int, n: int, n_iters: int, cursor: int = 0) -> np.ndarray:
    """Scrambled plain output: out[k, g] = scramble(value(seed, g, cursor + k))."""
    out = np.empty((n_iters, n), dtype=np.uint64)
    zeros = lib().oracle_generate_star(seed, n, cursor, n_iters, _ptr(out))
    if zeros:
        raise AssertionError("oracle produced %d zero values" % zeros)
    return out


def generate_star_u32(seed: int, n: int, n_iters: int, cursor: int = 0) -> np.ndarray:
    """High 32-bit halves of :func:`generate_star`."""
    out = np.empty((n_iters, n), dtype=np.uint32)
    zeros = lib().oracle_generate_star_u32(seed, n, cursor, n_iters, _ptr(out))
    if zeros:
        raise AssertionError("oracle produced %d zero states" % zeros)
    return out


# Words oracle_emit_rows can emit: the state, its low half, the scrambled
# word, the high half of the scrambled word.
WORD_U64, WORD_U32, WORD_STAR, WORD_STAR_U32 = 0, 1, 2, 3


def seed_range(seed: int, g0: int, count: int, cursor: int = 0) -> np.ndarray:
    """States of work-items g0 .. g0+count-1 at value number ``cursor``
    (sequential steps from each initial state)."""
    if g0 < 0 or count < 0 or g0 + count > 1 << 32:
        raise ValueError("work-items must lie in [0, 2^32)")
    st = np.empty(count, dtype=np.uint64)
    lib().oracle_seed_range(seed, g0, count, cursor, _ptr(st))
    return st


def emit_rows(states: np.ndarray, n_rows: int, word: int = WORD_U64) -> np.ndarray:
    """Continue the plain loop from ``states`` (advanced in place): n_rows
    rows, each emitting every state and then stepping it."""
    if states.dtype != np.uint64 or not states.flags["C_CONTIGUOUS"]:
        raise ValueError("states must be a contiguous uint64 array")
    dt = np.uint32 if word in (WORD_U32, WORD_STAR_U32) else np.uint64
    out = np.empty((n_rows, states.size), dtype=dt)
    zeros = lib().oracle_emit_rows(_ptr(states), states.size, n_rows, word, _ptr(out),
                                   states.size)
    if zeros:
        raise AssertionError("oracle met %d zero states" % zeros)
    return out


def generate_range(seed: int, g0: int, g1: int, n_iters: int, cursor: int = 0) -> np.ndarray:
    """Columns g0 <= g < g1 of :func:`generate` (iteration-major)."""
    if not 0 <= g0 <= g1 <= 1 << 32:
        raise ValueError("need 0 <= g0 <= g1 <= 2^32")
    out = np.empty((n_iters, g1 - g0), dtype=np.uint64)
    zeros = lib().oracle_generate_range(seed, g0, g1, cursor, n_iters, _ptr(out))
    if zeros:
        raise AssertionError("oracle produced %d zero values" % zeros)
    return out


def make_reqs(seeds, gids, offsets, lengths) -> np.ndarray:
    m = len(lengths)
    r = np.zeros(m, dtype=REQ_DTYPE)
    r["seed"] = np.asarray(seeds, dtype=np.uint64)
    r["gid"] = np.asarray(gids, dtype=np.uint32)
    r["offset"] = np.asarray(offsets, dtype=np.uint64)
    r["length"] = np.asarray(lengths, dtype=np.uint64)
    return r


def generate_batch(reqs: np.ndarray) -> np.ndarray:
    """Requests packed in order: out[base_j + t] = value(seed_j, gid_j, offset_j + t)."""
    reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    total = int(reqs["length"].sum()) if len(reqs) else 0
    out = np.empty(total, dtype=np.uint64)
    zeros = lib().oracle_generate_batch(_ptr(reqs), len(reqs), _ptr(out))
    if zeros:
        raise AssertionError("oracle produced %d zero values" % zeros)
    return out


def serve_offsets(submissions) -> list:
    """First value number of each served request (the bookkeeping rule of
    :func:`serve_expected`): the sum of the lengths of the requests submitted
    to the same stream before it."""
    cursor = {}
    offs = []
    for g, length in submissions:
        c = cursor.get(g, 0)
        offs.append(c)
        cursor[g] = c + int(length)
    return offs


def serve_expected(seed: int, submissions) -> list:
    """Outputs of served requests, given the submission history.

    ``submissions`` is a sequence of (stream_id, length) in submission order.
    Request r on stream g continues g's stream where the requests submitted
    to g before r stopped: its first value is value number
    (sum of the lengths of g's earlier requests). Returns one uint64 array per
    request, in submission order.
    """
    offs = serve_offsets(submissions)
    reqs = make_reqs([seed] * len(offs), [g for g, _ in submissions], offs,
                     [int(length) for _, length in submissions])
    flat = generate_batch(reqs)
    res, base = [], 0
    for _, length in submissions:
        res.append(flat[base:base + int(length)])
        base += int(length)
    return res


def hash_low_range(start: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint32)
    lib().oracle_hash_low_range(start & 0xFFFFFFFF, count, _ptr(out))
    return out


def hash_high_range(start: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint32)
    lib().oracle_hash_high_range(start & 0xFFFFFFFF, count, _ptr(out))
    return out
