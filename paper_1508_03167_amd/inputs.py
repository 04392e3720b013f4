"""Seeded synthetic inputs for the benchmark configurations (numpy only).

This module draws workloads -- it holds none of MergeShuffle's arithmetic and
shares nothing with either the kernels or the CPU oracle.  Its streams are
numpy's Philox bit generator (the 4x64 variant), independent of the 4x32
generator the shuffle itself draws its bits from.

  * identity arrays (the plain-permutation configurations);
  * 16-byte records: uint64 key uniform from a seeded Philox stream, uint64
    payload = original index;
  * batched sizes: floor(2^(lo + (hi-lo) u)), u uniform, per-array seed =
    base seed + array id;
  * served requests: log-uniform sizes, element type uniformly uint32 or
    uint64 with random values, Poisson arrivals at a given rate.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def identity_u32(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.uint32)


def records16(n: int, seed: int) -> np.ndarray:
    """[n, 2] uint64: column 0 = random key, column 1 = index."""
    out = np.empty((n, 2), dtype=np.uint64)
    out[:, 0] = rng(seed).integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    out[:, 1] = np.arange(n, dtype=np.uint64)
    return out


def log_uniform_sizes(count: int, seed: int, lo_log2: float, hi_log2: float) -> np.ndarray:
    u = rng(seed).random(count)
    return np.floor(np.exp2(lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def batched_sizes(count: int = 4096, seed: int = 3) -> np.ndarray:
    """Array sizes of the batched configuration: log-uniform in [2^8, 2^20]."""
    return log_uniform_sizes(count, seed, 8.0, 20.0)


def served_requests(count: int, seed: int, rate_per_s: float, lo_log2: float = 10.0, hi_log2: float = 26.0):
    """List of dicts (arrival_s, n, elem_bytes, seed) for the served configuration."""
    g = rng(seed)
    sizes = np.floor(np.exp2(lo_log2 + (hi_log2 - lo_log2) * g.random(count))).astype(np.int64)
    wide = g.random(count) < 0.5
    gaps = g.exponential(1.0 / rate_per_s, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    seeds = g.integers(0, 2**63, size=count, dtype=np.int64)
    return [dict(arrival_s=float(arrivals[i]), n=int(sizes[i]), elem_bytes=8 if wide[i] else 4,
                 seed=int(seeds[i])) for i in range(count)]


def request_values(n: int, elem_bytes: int, seed: int) -> np.ndarray:
    dt = np.uint64 if elem_bytes == 8 else np.uint32
    return rng(seed ^ 0x5EED).integers(0, np.iinfo(dt).max, size=n, dtype=dt, endpoint=True)


def sample_positions(n: int, count: int, seed: int) -> np.ndarray:
    """Sorted distinct positions in [0, n) incl. both ends, for sampled checks."""
    if n <= count:
        return np.arange(n, dtype=np.int64)
    p = rng(seed).choice(n, size=count - 2, replace=False)
    return np.unique(np.concatenate([[0, n - 1], p])).astype(np.int64)
