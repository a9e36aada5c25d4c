"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws keys and query streams only; it holds none of the method's arithmetic (no hashing,
bucketing or search). Both the GPU library and the CPU oracle receive exactly the arrays made here.

Recipes (stand-ins for the paper's inputs: random keys, each queried in random order):

* ``u64_keys(n, seed)``: ``n`` distinct uint64 keys, uniform over [0, 2^64), from numpy's PCG64
  stream ``default_rng(seed)``. Duplicates are removed (later occurrences dropped, fresh draws
  appended) until ``n`` distinct keys remain; at 10^8 keys a duplicate is expected once in ~3700
  seeds, so in practice the first draw is returned unchanged. Order is the draw order.
* ``query_indices(n_keys, n_queries, seed)``: indices uniform with replacement.
* ``ascii_strings(n, seed)``: random strings over [a-z0-9], length uniform in [10, 50]; returned as
  one uint8 byte array plus uint64 offsets[n+1]. Strings of at most 12 characters are made distinct
  (packed base-36 into a uint64 and deduplicated); longer ones collide with probability < 1e-7 over
  10^8 strings, which the build would report as a duplicate.
* ``lognormal_sizes(count, median, sigma, lo, hi, seed)``: clipped lognormal integer sizes.
"""

from __future__ import annotations

import numpy as np

CHARSET = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz0123456789", dtype=np.uint8)


def u64_keys(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    keys = rng.bit_generator.random_raw(n).astype(np.uint64, copy=False)
    if n < 2:
        return keys
    while True:
        order = np.argsort(keys, kind="stable")
        srt = keys[order]
        dup_sorted = np.nonzero(srt[1:] == srt[:-1])[0] + 1
        if dup_sorted.size == 0:
            return keys
        drop = np.zeros(n, dtype=bool)
        drop[order[dup_sorted]] = True
        kept = keys[~drop]
        extra = rng.bit_generator.random_raw(int(drop.sum())).astype(np.uint64, copy=False)
        keys = np.concatenate([kept, extra])


def u64_key_sets(sizes, base_seed: int) -> list:
    """One key set per size, set t drawn from PCG64 default_rng(base_seed + t) (uniform uint64).
    Not deduplicated: the chance that any set of the 4096-set batched workload holds a repeated key
    is below 1e-5, and a repeat would surface as a DUPLICATE status of that build."""
    return [np.random.default_rng(base_seed + t).bit_generator.random_raw(int(n)).astype(np.uint64, copy=False)
            for t, n in enumerate(sizes)]


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    return np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, count))


def log_uniform_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)


def query_indices(n_keys: int, n_queries: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_keys, size=n_queries, dtype=np.int64)


def permutation(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).permutation(n)


def _pack_short(buf: np.ndarray, offs: np.ndarray, idx: np.ndarray) -> np.ndarray:
    # base-36 value of each string (plus its length, so "a" and "aa" differ) for strings <= 12 chars
    lut = np.zeros(256, dtype=np.uint64)
    lut[CHARSET] = np.arange(36, dtype=np.uint64)
    out = np.zeros(idx.size, dtype=np.uint64)
    lens = (offs[idx + 1] - offs[idx]).astype(np.int64)
    for t in range(12):
        has = lens > t
        pos = offs[idx[has]] + t
        out[has] = out[has] * np.uint64(36) + lut[buf[pos]]
    return out * np.uint64(16) + lens.astype(np.uint64)


def ascii_strings(n: int, seed: int, min_len: int = 10, max_len: int = 50):
    rng = np.random.default_rng(seed)
    lens = rng.integers(min_len, max_len + 1, size=n, dtype=np.int64)
    offs = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    buf = CHARSET[rng.integers(0, CHARSET.size, size=int(offs[-1]), dtype=np.uint8)]
    short = np.nonzero(lens <= 12)[0]
    while short.size > 1:
        packed = _pack_short(buf, offs, short)
        order = np.argsort(packed, kind="stable")
        srt = packed[order]
        dups = short[order[np.nonzero(srt[1:] == srt[:-1])[0] + 1]]
        if dups.size == 0:
            break
        for i in dups:  # redraw the later copy in place (same length)
            a, b = int(offs[i]), int(offs[i + 1])
            buf[a:b] = CHARSET[rng.integers(0, CHARSET.size, size=b - a, dtype=np.uint8)]
    return buf, offs


def lognormal_sizes(count: int, median: float, sigma: float, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = rng.lognormal(mean=np.log(median), sigma=sigma, size=count)
    return np.clip(np.rint(x), lo, hi).astype(np.int64)
