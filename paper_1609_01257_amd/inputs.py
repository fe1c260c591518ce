"""Seeded synthetic workloads shared by the tests and the benchmark.

This module draws inputs only; it holds none of the generator's arithmetic.
The paper's own workload is synthetic (n = 2^12 ... 2^24 values per
iteration, i = 10^2 ... 10^4 iterations, Section 6.2); these are workloads
of that shape plus the batched and served forms.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Plain method, small: 65,536 work-items, seed 0, 64 iterations.
SMALL = dict(seed=0, n=65536, iters=64)
# Streaming: 4,194,304 work-items (32 MiB per iteration), seed 42, 2,000 iterations.
STREAMING = dict(seed=42, n=4194304, iters=2000)
# HBM roofline sweep: 2^20 ... 2^26 work-items, 256 iterations, seeds 1..4.
ROOFLINE_N = (1 << 20, 1 << 22, 1 << 24, 1 << 26)
ROOFLINE_ITERS = 256
ROOFLINE_SEEDS = (1, 2, 3, 4)


@dataclass
class Requests:
    seeds: np.ndarray    # uint64
    gids: np.ndarray     # uint32
    offsets: np.ndarray  # uint64
    lengths: np.ndarray  # uint64

    def __len__(self):
        return len(self.lengths)

    @property
    def total(self) -> int:
        return int(self.lengths.sum())


def batched_requests(m: int = 4096, seed: int = 1609, lo_log2: float = 10.0,
                     hi_log2: float = 24.0) -> Requests:
    """Independent streams: seeds drawn from a seeded uint64 generator, lengths
    log-uniform in [2^lo_log2, 2^hi_log2), gid_j = j, offset 0."""
    rng = np.random.default_rng(seed)
    seeds = rng.integers(0, 2**64, size=m, dtype=np.uint64)
    lengths = np.floor(2.0 ** rng.uniform(lo_log2, hi_log2, size=m)).astype(np.uint64)
    return Requests(seeds, np.arange(m, dtype=np.uint32), np.zeros(m, dtype=np.uint64), lengths)


def ragged_requests(m: int, seed: int, max_len: int, max_offset: int = 0,
                    max_gid: int = 2**32) -> Requests:
    """Small ragged request tables for parity tests (uniform lengths 1..max_len)."""
    rng = np.random.default_rng(seed)
    seeds = rng.integers(0, 2**64, size=m, dtype=np.uint64)
    gids = rng.integers(0, max_gid, size=m, dtype=np.uint64).astype(np.uint32)
    offsets = (rng.integers(0, max_offset + 1, size=m, dtype=np.uint64)
               if max_offset else np.zeros(m, dtype=np.uint64))
    lengths = rng.integers(1, max_len + 1, size=m, dtype=np.uint64)
    return Requests(seeds, gids, offsets, lengths)


def serving_arrivals(rate_hz: float, duration_s: float, seed: int = None,
                     n_streams: int = 1 << 20, lo_log2: float = 12.0, hi_log2: float = 22.0):
    """Poisson arrivals: exponential gaps at `rate_hz` over `duration_s`; each
    request names a stream uniform over n_streams and a length log-uniform in
    [2^lo_log2, 2^hi_log2). Returns (arrival_s, stream_id, length) arrays."""
    rng = np.random.default_rng(1609 + int(rate_hz) if seed is None else seed)
    expected = int(rate_hz * duration_s * 1.2) + 16
    gaps = rng.exponential(1.0 / rate_hz, size=expected)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = np.cumsum(rng.exponential(1.0 / rate_hz, size=expected)) + t[-1]
        t = np.concatenate([t, more])
    t = t[t < duration_s]
    k = len(t)
    streams = rng.integers(0, n_streams, size=k, dtype=np.uint64).astype(np.uint32)
    lengths = np.floor(2.0 ** rng.uniform(lo_log2, hi_log2, size=k)).astype(np.uint64)
    return t, streams, lengths


def sample_positions(n: int, iters: int, count: int, seed: int = 0):
    """Uniform sample of (iteration, work-item) positions of a plain output,
    always including its four corners."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, iters, size=count, dtype=np.int64)
    g = rng.integers(0, n, size=count, dtype=np.int64)
    corners_k = np.array([0, 0, iters - 1, iters - 1], dtype=np.int64)
    corners_g = np.array([0, n - 1, 0, n - 1], dtype=np.int64)
    return np.concatenate([corners_k, k]), np.concatenate([corners_g, g])
