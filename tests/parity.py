"""Full-size element-wise comparison of device outputs with the oracle (test
helper).

``helpers/parity.c`` (built here into ``helpers/libparity.so``, linked to the
oracle's ``liboracle.so``) compares host copies of device outputs with values
the oracle produces on the fly, over host threads. The functions below copy
a device output to page-locked host memory in blocks (the next block's copy
overlaps the check of the current one) and feed the blocks to it, so outputs
of many gigabytes are compared value by value without holding a host copy of
the whole output or of the oracle's values.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

import oracle

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "helpers", "parity.c")
_LIB = os.path.join(_HERE, "helpers", "libparity.so")

# Host threads for the comparison (a GPU machine's share of cores is 16).
THREADS = max(1, min(16, os.cpu_count() or 1))

WORD_U64, WORD_U32, WORD_STAR, WORD_STAR_U32 = (oracle.WORD_U64, oracle.WORD_U32,
                                                oracle.WORD_STAR, oracle.WORD_STAR_U32)


class Result(ctypes.Structure):
    _fields_ = [("mismatches", ctypes.c_uint64), ("first_a", ctypes.c_uint64),
                ("first_b", ctypes.c_uint64), ("zeros", ctypes.c_uint64),
                ("failed", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def build(force: bool = True) -> str:
    olib = oracle.build(force=False)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-fPIC", "-shared",
                        "-pthread", "-o", tmp, _SRC, "-L", os.path.dirname(olib),
                        "-l:liboracle.so", "-Wl,-rpath,$ORIGIN/../../oracle"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        p, u32, u64, i = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.pc_check_plain_rows.argtypes = [p, u64, u64, u32, p, i, i, ctypes.POINTER(Result)]
        L.pc_check_plain_rows.restype = None
        L.pc_seed_states.argtypes = [u64, u64, u64, u64, p, i]
        L.pc_seed_states.restype = None
        L.pc_check_requests.argtypes = [p, u32, p, p, p, i, i, ctypes.POINTER(Result)]
        L.pc_check_requests.restype = None
        _lib = L
    return _lib


def _word_size(word: int) -> int:
    return 4 if word in (WORD_U32, WORD_STAR_U32) else 8


def _done(r: Result) -> dict:
    if r.failed:
        raise MemoryError("parity checker could not allocate its buffers")
    if r.zeros:
        raise AssertionError("oracle met %d zero states" % r.zeros)
    return {"mismatches": int(r.mismatches), "first": (int(r.first_a), int(r.first_b))}


def seed_states(seed: int, n: int, cursor: int = 0, g0: int = 0) -> np.ndarray:
    """value(seed, g0 + t, cursor) for t < n (the oracle, over host threads)."""
    st = np.empty(n, dtype=np.uint64)
    lib().pc_seed_states(seed, g0, n, cursor, st.ctypes.data, THREADS)
    return st


def check_rows_ptr(ptr: int, ld: int, n: int, n_rows: int, st: np.ndarray, word: int) -> dict:
    """Compare n_rows rows of n words at host address ``ptr`` (row stride ld
    words) with the oracle continuing from ``st`` (advanced in place)."""
    assert st.dtype == np.uint64 and st.flags["C_CONTIGUOUS"] and st.size >= n
    r = Result()
    lib().pc_check_plain_rows(ptr, ld, n, n_rows, st.ctypes.data, word, THREADS, ctypes.byref(r))
    return _done(r)


def check_rows(got: np.ndarray, st: np.ndarray, word: int) -> dict:
    """Compare a host array of shape (rows, n) with the oracle continuing from st."""
    got = np.ascontiguousarray(got)
    assert got.ndim == 2 and got.dtype.itemsize == _word_size(word)
    return check_rows_ptr(got.ctypes.data, got.shape[1], got.shape[1], got.shape[0], st, word)


def check_requests(reqs: np.ndarray, got_ptr: int, bases: np.ndarray, word: int = WORD_U64,
                   starts: np.ndarray = None) -> dict:
    """Compare requests (oracle.REQ_DTYPE) with the oracle: request r's values
    are at host address got_ptr + 8 * (bases[r] + t). ``starts`` (optional)
    gives each request's state at its offset."""
    reqs = np.ascontiguousarray(reqs, dtype=oracle.REQ_DTYPE)
    bases = np.ascontiguousarray(bases, dtype=np.uint64)
    assert bases.size == reqs.size
    sp = None
    if starts is not None:
        starts = np.ascontiguousarray(starts, dtype=np.uint64)
        assert starts.size == reqs.size
        sp = starts.ctypes.data
    r = Result()
    lib().pc_check_requests(reqs.ctypes.data, reqs.size, got_ptr, bases.ctypes.data, sp, word,
                            THREADS, ctypes.byref(r))
    return _done(r)


# --- device outputs ----------------------------------------------------------

_pinned = []   # page-locked buffers kept for reuse (pinning gigabytes is slow)


class _Blocks:
    """Two page-locked host buffers and a copy stream: block b + 1 is copied
    while block b is checked."""

    def __init__(self, torch, nbytes: int):
        self.torch = torch
        if len(_pinned) < 2 or _pinned[0].numel() < nbytes:
            _pinned.clear()
            _pinned.extend(torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
                           for _ in range(2))
        self.buf = list(_pinned)
        self.ev = [torch.cuda.Event() for _ in range(2)]
        self.stream = torch.cuda.Stream()

    def start(self, i: int, src_bytes):
        """Queue the copy of a flat uint8 device view into buffer i % 2."""
        b = i % 2
        with self.torch.cuda.stream(self.stream):
            self.buf[b][:src_bytes.numel()].copy_(src_bytes, non_blocking=True)
            self.ev[b].record(self.stream)

    def wait(self, i: int) -> int:
        b = i % 2
        self.ev[b].synchronize()
        return self.buf[b].data_ptr()


def compare_plain_device(out, n: int, iters: int, seed: int, cursor: int = 0,
                         word: int = WORD_U64, block_bytes: int = 1 << 30,
                         states: np.ndarray = None) -> dict:
    """Compare every value of a device plain output (iteration-major, ``iters``
    rows of ``n`` words, any integer dtype of the word's size) with the
    oracle. Rows are copied in blocks of about ``block_bytes``; a row longer
    than a block is split by columns. Returns the mismatch count and the
    first mismatch (row, column)."""
    import torch
    es = _word_size(word)
    flat = out.view(-1).view(torch.uint8)
    assert flat.numel() >= iters * n * es
    st = seed_states(seed, n, cursor) if states is None else states
    row_bytes = n * es
    if row_bytes <= block_bytes:
        rows = max(1, min(iters, block_bytes // row_bytes))
        pieces = [(k, min(rows, iters - k), 0, n) for k in range(0, iters, rows)]
    else:
        cols = max(1, block_bytes // es)
        pieces = [(k, 1, c, min(n, c + cols)) for k in range(iters) for c in range(0, n, cols)]
    blocks = _Blocks(torch, max(r * (c1 - c0) for _, r, c0, c1 in pieces) * es)
    torch.cuda.current_stream().synchronize()   # the output is complete

    def src(p):
        k, r, c0, c1 = p
        if c0 == 0 and c1 == n:
            return flat[k * row_bytes:(k + r) * row_bytes]
        return flat[k * row_bytes + c0 * es:k * row_bytes + c1 * es]

    total, first = 0, None
    blocks.start(0, src(pieces[0]))
    for i, p in enumerate(pieces):
        if i + 1 < len(pieces):
            blocks.start(i + 1, src(pieces[i + 1]))
        ptr = blocks.wait(i)
        k, r, c0, c1 = p
        # Columns c0..c1 of rows k..k+r: the states of those columns.
        sub = st[c0:c1]
        res = check_rows_ptr(ptr, c1 - c0, c1 - c0, r, sub, word)
        if res["mismatches"]:
            total += res["mismatches"]
            if first is None:
                first = (k + res["first"][0], c0 + res["first"][1])
    blocks.stream.synchronize()
    return {"mismatches": total, "first": first, "values": iters * n}


def compare_requests_device(out, reqs: np.ndarray, bases: np.ndarray, word: int = WORD_U64,
                            starts: np.ndarray = None, block_bytes: int = 1 << 30) -> dict:
    """Compare requests whose values lie in a device buffer (``bases[r]`` is the
    index, in 8-byte words of ``out``, of request r's first value) with the
    oracle. Requests are copied in groups of about ``block_bytes``, each group
    one contiguous span of ``out``; requests must be listed in increasing
    order of ``bases`` with non-overlapping spans."""
    import torch
    flat = out.view(-1).view(torch.int64)
    reqs = np.ascontiguousarray(reqs, dtype=oracle.REQ_DTYPE)
    bases = np.asarray(bases, dtype=np.uint64)
    lengths = reqs["length"].astype(np.uint64)
    ends = bases + lengths
    assert np.all(bases[1:] >= ends[:-1]), "requests must be ordered and disjoint"
    groups, j = [], 0
    words = max(1, block_bytes // 8)
    while j < len(reqs):
        k = j + 1
        while k < len(reqs) and int(ends[k] - bases[j]) <= words:
            k += 1
        groups.append((j, k))
        j = k
    span = max(int(ends[k - 1] - bases[j]) for j, k in groups)
    blocks = _Blocks(torch, span * 8)
    torch.cuda.current_stream().synchronize()

    def src(g):
        j, k = g
        return flat[int(bases[j]):int(ends[k - 1])].view(torch.uint8)

    total, first = 0, None
    blocks.start(0, src(groups[0]))
    for i, (j, k) in enumerate(groups):
        if i + 1 < len(groups):
            blocks.start(i + 1, src(groups[i + 1]))
        ptr = blocks.wait(i)
        res = check_requests(reqs[j:k], ptr, bases[j:k] - bases[j], word,
                             None if starts is None else starts[j:k])
        if res["mismatches"]:
            total += res["mismatches"]
            if first is None:
                first = (j + res["first"][0], res["first"][1])
    blocks.stream.synchronize()
    return {"mismatches": total, "first": first, "values": int(lengths.sum())}
