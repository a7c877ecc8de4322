"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws random numbers; it holds none of the sort's
arithmetic.  The paper measures on its own stored random three-digit data
(Section 4.2), which is not available; these generators stand in for it with
the workloads the hot path is measured on:

* ``uniform_i32``   keys uniform in [0, 2^31-1)                (plain method)
* ``loguniform_i32`` keys floor(10^(9u)) clipped to [1, 10^9)   (Benford-like,
  skewed most-significant-digit bucket sizes)
* ``dup_pairs_i32`` keys uniform in [0, 1000) (heavy duplicates) with
  payload = original index                                     (stable pairs)
* ``segments_i32``  16384 arrays, sizes log-uniform in [1, 2^16]  (batched)
* ``request_stream`` Poisson arrivals of int64 arrays, sizes log-uniform in
  [2^10, 2^24], keys uniform over the full int64 range          (serving)
* ``typed_keys``    keys of the other supported types (uint32/uint64, float32/
  float64 with NaNs, infinities, signed zeros and subnormals mixed in, and
  int32/int64 with their extremes), with duplicates

All use numpy's PCG64 ``default_rng(seed)``.
"""
from __future__ import annotations

import math

import numpy as np

INT32_HI = 2**31 - 1


def uniform_i32(n: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, INT32_HI, n, dtype=np.int32)


def loguniform_i32(n: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = np.floor(10.0 ** (9.0 * rng.random(n)))
    return np.clip(x, 1, 10**9 - 1).astype(np.int32)


def dup_pairs_i32(n: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 1000, n, dtype=np.int32)
    vals = np.arange(n, dtype=np.uint32)
    return keys, vals


def uniform_i64(n: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, n, dtype=np.int64, endpoint=True)


def segment_sizes(nseg: int = 16384, max_len: int = 2**16, seed: int = 0) -> np.ndarray:
    """Sizes log-uniform in [1, max_len]: floor(exp(u * ln(max_len + 1)))."""
    rng = np.random.default_rng(seed)
    u = rng.random(nseg)
    s = np.floor(np.exp(u * math.log(max_len + 1))).astype(np.int64)
    return np.clip(s, 1, max_len)


def segments_i32(nseg: int = 16384, max_len: int = 2**16, seed: int = 0):
    """(keys int32[total], offsets int64[nseg+1]) with log-uniform sizes."""
    sizes = segment_sizes(nseg, max_len, seed)
    off = np.zeros(nseg + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    rng = np.random.default_rng(seed + 1_000_003)
    keys = rng.integers(0, INT32_HI, int(off[-1]), dtype=np.int32)
    return keys, off


def request_sizes(count: int, lo: int = 2**10, hi: int = 2**24, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    u = rng.random(count)
    s = np.floor(np.exp(math.log(lo) + u * (math.log(hi + 1) - math.log(lo)))).astype(np.int64)
    return np.clip(s, lo, hi)


def request_stream(count: int, rate_per_s: float, lo: int = 2**10, hi: int = 2**24, seed: int = 0):
    """List of (arrival_time_s, int64 keys) with Poisson arrivals at rate_per_s."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, count)
    t = np.cumsum(gaps) - gaps[0]
    sizes = request_sizes(count, lo, hi, seed + 17)
    out = []
    for i in range(count):
        r = np.random.default_rng((seed, i))
        k = r.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, int(sizes[i]), dtype=np.int64, endpoint=True)
        out.append((float(t[i]), k))
    return out


def adversarial_i32(T: int = 8192):
    """Named edge-case arrays for int32 parity sweeps (no arithmetic of the sort)."""
    rng = np.random.default_rng(7)
    mn, mx = np.iinfo(np.int32).min, np.iinfo(np.int32).max
    cases = {}
    for n in [0, 1, 2, 3, 63, 64, 65, 255, 256, 257, T - 1, T, T + 1, 2 * T + 3, 4096 * 3 + 17, 2**16 + 1, 100_003]:
        cases[f"uniform_n{n}"] = rng.integers(0, INT32_HI, n, dtype=np.int32)
    n = 50_000
    cases["all_equal"] = np.full(n, 12345, np.int32)
    cases["all_zero"] = np.zeros(n, np.int32)
    cases["sorted"] = np.sort(rng.integers(0, INT32_HI, n, dtype=np.int32))
    cases["reverse"] = np.sort(rng.integers(0, INT32_HI, n, dtype=np.int32))[::-1].copy()
    cases["extremes"] = rng.choice(np.array([mn, mn + 1, -1, 0, 1, mx - 1, mx], np.int32), n)
    cases["full_range"] = rng.integers(mn, mx, n, dtype=np.int32, endpoint=True)
    cases["negative_only"] = rng.integers(mn, 0, n, dtype=np.int32)
    cases["one_bucket"] = rng.integers(0, 10**6, n, dtype=np.int32) + np.int32(7 * 10**6)
    cases["three_digit"] = rng.integers(0, 1000, n, dtype=np.int32)
    cases["two_values"] = rng.choice(np.array([5, 900], np.int32), n)
    cases["loguniform"] = loguniform_i32(n, 3)
    cases["sawtooth"] = (np.arange(n, dtype=np.int64) % 1000).astype(np.int32)
    return cases


def typed_keys(dtype, n: int, seed: int = 0) -> np.ndarray:
    """Keys of `dtype` (any of int32/uint32/float32/int64/uint64/float64): a
    fifth special values (extremes; for floats also NaN of both signs, the
    infinities, both zeros and the smallest subnormals), a third small
    values (duplicates), the rest over the type's whole range (floats:
    normal values of every magnitude)."""
    dt = np.dtype(dtype)
    rng = np.random.default_rng(seed)
    if dt.kind == "f":
        fi = np.finfo(dt)
        special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, -np.nan, 1.0, -1.0, fi.tiny, -fi.tiny, fi.max,
                            -fi.max, fi.smallest_subnormal, -fi.smallest_subnormal], dt)
        body = (rng.standard_normal(n) * 10.0 ** rng.integers(fi.minexp // 4, fi.maxexp // 4, n)).astype(dt)
        small = rng.integers(-20, 20, n).astype(dt)
    else:
        ii = np.iinfo(dt)
        special = np.array([ii.min, ii.max, 0, 1, ii.max - 1, ii.min + 1], dt)
        body = rng.integers(ii.min, ii.max, n, dtype=dt, endpoint=True)
        small = rng.integers(0, 40, n).astype(dt)
    pick = rng.random(n)
    return np.where(pick < 0.2, rng.choice(special, n), np.where(pick < 0.55, small, body)).astype(dt)
