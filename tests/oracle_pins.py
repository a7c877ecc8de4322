"""Checks that pin the CPU oracle to something other than itself.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises AssertionError
when the oracle disagrees with a brute-force route, a library routine, a
hand-worked example or an invariant.  ``test_oracle.py`` runs them on the
real oracle; ``test_oracle_mutants.py`` runs them on copies of the oracle
with a planted mistake and requires that some pin fails for every copy.

Independent routes used here (none re-types the oracle's own arithmetic):
* sorting: pure-Python stable insertion sort, numpy's stable sort/argsort;
* the decimal digit: the decimal *string* of u = k - beta (its length is D,
  its first character, after left-padding to D characters, is the digit),
  instead of the oracle's power table and integer division;
* bounds: counting by string digits, and lower_bound of the sorted output;
* hand-worked examples in ``golden/worked_examples.json``.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "worked_examples.json")
I32 = np.iinfo(np.int32)
I64 = np.iinfo(np.int64)


# ----------------------------------------------------------- brute force
def insertion_sort(seq):
    """Stable insertion sort of a list of comparable items (brute force)."""
    out = list(seq)
    for i in range(1, len(out)):
        x = out[i]
        j = i - 1
        while j >= 0 and x < out[j]:
            out[j + 1] = out[j]
            j -= 1
        out[j + 1] = x
    return out


def stable_pairs_brute(keys, vals):
    """Stable sort by key alone, by insertion on keys only (never on vals)."""
    items = list(zip([int(k) for k in keys], [int(v) for v in vals]))
    for i in range(1, len(items)):
        x = items[i]
        j = i - 1
        while j >= 0 and x[0] < items[j][0]:
            items[j + 1] = items[j]
            j -= 1
        items[j + 1] = x
    return [k for k, _ in items], [v for _, v in items]


def string_plan(keys):
    """(beta, D, p, digits) via decimal strings of u = k - beta."""
    ks = [int(k) for k in keys]
    if not ks:
        return 0, 1, 1, []
    beta = min(min(ks), 0)
    us = [k - beta for k in ks]
    D = len(str(max(us)))
    p = int("1" + "0" * (D - 1))
    digits = [int(str(u).rjust(D, "0")[0]) for u in us]
    return beta, D, p, digits


def string_plan2(keys):
    """Two-digit buckets via decimal strings: the first two characters of u
    written with D digits (a one-digit u gets a trailing zero)."""
    beta, D, p, _ = string_plan(keys)
    digits = [int((str(int(k) - beta).rjust(D, "0") + "0")[:2]) for k in keys]
    return beta, D, p, digits


def string_bounds2(keys):
    cnt = [0] * 100
    for d in string_plan2(keys)[3]:
        cnt[d] += 1
    b = [0]
    for c in cnt:
        b.append(b[-1] + c)
    return b


def string_bounds(keys):
    _, _, _, digits = string_plan(keys)
    cnt = [0] * 10
    for d in digits:
        cnt[d] += 1
    b = [0]
    for c in cnt:
        b.append(b[-1] + c)
    return b


# ----------------------------------------------------------------- pins
def pin_worked_examples(orc):
    with open(GOLDEN) as f:
        g = json.load(f)
    for dt, name in ((np.int32, "int32"), (np.int64, "int64")):
        for ex in g[name]:
            k = np.array(ex["keys"], dt)
            beta, D, p = orc.plan(k)
            assert (beta, D, p) == (ex["beta"], ex["D"], ex["p"]), ("plan", ex, (beta, D, p))
            assert orc.bounds(k).tolist() == ex["bounds"], ("bounds", ex)
            assert orc.sort_keys(k).tolist() == ex["sorted"], ("sorted", ex)
            assert string_plan(ex["keys"])[3] == ex["digits"], ("fixture digits", ex)
    for ex in g["pairs"]:
        k, v = orc.sort_pairs(np.array(ex["keys"], np.int32), np.array(ex["vals"], np.uint32))
        assert k.tolist() == ex["sorted_keys"] and v.tolist() == ex["sorted_vals"], ex


def pin_exhaustive_small(orc, max_n=5):
    """Every array of length 0..max_n over seven values, including the extremes."""
    for dt, info, top in ((np.int32, I32, max_n), (np.int64, I64, max_n - 1)):
        vals = [info.min, -2, -1, 0, 1, 2, info.max]
        for n in range(top + 1):
            for combo in itertools.product(vals, repeat=n):
                k = np.array(combo, dt)
                got = orc.sort_keys(k).tolist()
                assert got == insertion_sort(combo), (dt, combo, got)
                assert orc.bounds(k).tolist() == string_bounds(combo), (dt, combo)


def pin_pairs_brute(orc, cases=400, seed=11):
    rng = np.random.default_rng(seed)
    for _ in range(cases):
        n = int(rng.integers(0, 65))
        k = rng.integers(0, int(rng.integers(1, 6)), n).astype(np.int32)
        v = rng.permutation(n).astype(np.uint32)
        gk, gv = orc.sort_pairs(k, v)
        bk, bv = stable_pairs_brute(k, v)
        assert gk.tolist() == bk and gv.tolist() == bv, (k, v)


def pin_random_brute(orc, cases=300, seed=12):
    rng = np.random.default_rng(seed)
    for _ in range(cases):
        n = int(rng.integers(0, 65))
        dt = np.int32 if rng.random() < 0.5 else np.int64
        info = np.iinfo(dt)
        k = rng.integers(info.min, info.max, n, dtype=dt, endpoint=True)
        if rng.random() < 0.5:
            k = (k % 50).astype(dt)
        assert orc.sort_keys(k).tolist() == insertion_sort(k.tolist()), k


def pin_library(orc, seed=13):
    """Against numpy's stable sort / argsort at sizes that span many chunks."""
    rng = np.random.default_rng(seed)
    for n in [17, 1000, 4099, 65537, 200_003]:
        for dt in (np.int32, np.int64):
            info = np.iinfo(dt)
            k = rng.integers(info.min, info.max, n, dtype=dt, endpoint=True)
            assert np.array_equal(orc.sort_keys(k), np.sort(k, kind="stable")), (n, dt)
        k = rng.integers(0, 1000, n, dtype=np.int32)
        v = rng.integers(0, 2**32, n, dtype=np.uint32)
        gk, gv = orc.sort_pairs(k, v)
        order = np.argsort(k, kind="stable")
        assert np.array_equal(gk, k[order]) and np.array_equal(gv, v[order]), n


def pin_bounds_string_route(orc, seed=14):
    rng = np.random.default_rng(seed)
    cases = []
    for D in range(1, 11):  # int32: every digit count the type can produce
        hi = 10**D - 1 if D < 10 else I32.max
        lo = 10 ** (D - 1)
        k = rng.integers(0, lo, 50, dtype=np.int64)
        k[rng.integers(0, 50)] = rng.integers(lo, hi, endpoint=True)
        cases.append(k.astype(np.int32))
    for D in range(1, 21):  # int64, D = 20 needs a negative minimum
        if D < 20:
            lo, hi = 10 ** (D - 1), min(10**D - 1, I64.max)
            k = [int(x) for x in rng.integers(0, lo, 40, dtype=np.int64)]
            k.append(int(rng.integers(lo, hi, endpoint=True, dtype=np.int64)))
        else:
            k = [I64.min, I64.max] + [int(x) for x in rng.integers(I64.min, I64.max, 30, dtype=np.int64)]
        cases.append(np.array(k, np.int64))
    for D in range(1, 20):  # maxima exactly at 10^(D-1) and 10^D - 1 (digit-count edges)
        for top in (10 ** (D - 1), 10**D - 1, 10**D):
            for dt, info in ((np.int32, I32), (np.int64, I64)):
                if top <= info.max:
                    cases.append(np.array([0, top // 3, top], dt))
                    cases.append(np.array([-1, top - 1], dt))
    for _ in range(60):
        dt = np.int32 if rng.random() < 0.5 else np.int64
        info = np.iinfo(dt)
        lo = int(rng.integers(info.min, info.max, dtype=dt)) if rng.random() < 0.5 else 0
        hi = int(rng.integers(max(lo, 0), info.max, dtype=dt, endpoint=True))
        cases.append(rng.integers(lo, hi, int(rng.integers(1, 300)), dtype=dt, endpoint=True))
    for k in cases:
        beta, D, p, _ = string_plan(k.tolist())
        assert orc.plan(k) == (beta, D, p), (k.dtype, orc.plan(k), (beta, D, p))
        assert orc.bounds(k).tolist() == string_bounds(k.tolist()), k
        # second route: lower_bound of the sorted output at the bucket thresholds
        s = [int(x) for x in np.sort(k)]
        lb = [0] + [int(np.searchsorted(np.array(s, dtype=object), beta + b * p, side="left")) for b in range(1, 10)]
        lb.append(len(s))
        assert orc.bounds(k).tolist() == lb, k


def pin_radix_mode(orc, seed=15):
    """Section 3.4 pipeline run sequentially equals the plain sort."""
    rng = np.random.default_rng(seed)
    for n in [0, 1, 9, 1000, 30_011]:
        for dt in (np.int32, np.int64):
            info = np.iinfo(dt)
            for k in (rng.integers(info.min, info.max, n, dtype=dt, endpoint=True),
                      rng.integers(0, 1000, n).astype(dt)):
                rk, rb = orc.radix_sort_keys(k)
                assert np.array_equal(rk, orc.sort_keys(k)), (n, dt)
                assert np.array_equal(rb, orc.bounds(k)), (n, dt)
        k = rng.integers(0, 1000, n, dtype=np.int32)
        v = np.arange(n, dtype=np.uint32)
        rk, rv, _ = orc.radix_sort_pairs(k, v)
        pk, pv = orc.sort_pairs(k, v)
        assert np.array_equal(rk, pk) and np.array_equal(rv, pv), n


def pin_scatter(orc, seed=16):
    """Stable one-step scatter: buckets in digit order, input order inside each."""
    rng = np.random.default_rng(seed)
    for n in [0, 1, 7, 500, 4000]:
        for dt in (np.int32, np.int64):
            info = np.iinfo(dt)
            k = rng.integers(info.min, info.max, n, dtype=dt, endpoint=True)
            if dt == np.int32:
                sk, sv, b = orc.scatter(k, np.arange(n, dtype=np.uint32))
            else:
                sk, sv, b = orc.scatter(k)
            assert b.tolist() == string_bounds(k.tolist())
            _, _, _, digits_in = string_plan(k.tolist())
            _, _, _, digits_out = string_plan(sk.tolist())
            assert digits_out == sorted(digits_in), "buckets out of digit order"
            assert np.array_equal(np.sort(sk), np.sort(k)), "not a permutation"
            if sv is not None:
                assert np.array_equal(k[sv], sk), "payload does not follow its key"
                for bk in range(10):
                    seg = sv[b[bk]:b[bk + 1]]
                    assert np.all(np.diff(seg.astype(np.int64)) > 0), "scatter not stable"


def pin_bucket_tiles(orc, seed=17):
    rng = np.random.default_rng(seed)
    for n, T in [(0, 4), (1, 4), (100, 7), (5000, 64), (20_000, 1000)]:
        k = rng.integers(0, 3000, n, dtype=np.int32)
        v = np.arange(n, dtype=np.uint32)
        sk, sv, b = orc.scatter(k, v)
        tk, tv, tb = orc.bucket_tiles(k, T, v)
        assert np.array_equal(b, tb)
        for bk in range(10):
            for s0 in range(int(b[bk]), int(b[bk + 1]), T):
                e = min(s0 + T, int(b[bk + 1]))
                order = np.lexsort((sv[s0:e], sk[s0:e]))
                assert np.array_equal(tk[s0:e], sk[s0:e][order]), (n, T, bk, s0)
                assert np.array_equal(tv[s0:e], sv[s0:e][order]), (n, T, bk, s0)
        k64 = rng.integers(I64.min, I64.max, n, dtype=np.int64, endpoint=True)
        sk, _, b = orc.scatter(k64)
        tk, _, _ = orc.bucket_tiles(k64, T)
        for bk in range(10):
            for s0 in range(int(b[bk]), int(b[bk + 1]), T):
                e = min(s0 + T, int(b[bk + 1]))
                assert np.array_equal(tk[s0:e], np.sort(sk[s0:e])), (n, T, bk, s0)


def pin_segmented(orc, seed=18):
    rng = np.random.default_rng(seed)
    for dt in (np.int32, np.int64):
        info = np.iinfo(dt)
        sizes = rng.integers(0, 300, 40)
        sizes[[0, 5, 6]] = 0
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        k = rng.integers(info.min, info.max, int(off[-1]), dtype=dt, endpoint=True)
        out, bnd = orc.sort_segmented(k, off)
        for s in range(len(sizes)):
            a, e = off[s], off[s + 1]
            assert np.array_equal(out[a:e], np.sort(k[a:e])), s
            assert bnd[s].tolist() == string_bounds(k[a:e].tolist()), s


def pin_count(orc, seed=19):
    rng = np.random.default_rng(seed)
    for dt in (np.int32, np.int64):
        k = rng.integers(-20, 20, 500).astype(dt)
        for x in range(-22, 23):
            lt = sum(1 for y in k.tolist() if y < x)
            le = sum(1 for y in k.tolist() if y <= x)
            assert orc.count_lt_le(k, x) == (lt, le), (dt, x)


def pin_two_digit_worked_examples(orc):
    with open(GOLDEN) as f:
        g = json.load(f)["two_digit"]
    for ex in g["cases"]:
        k = np.array(ex["keys"], np.int32 if ex["dtype"] == "int32" else np.int64)
        assert string_plan2(ex["keys"])[3] == ex["digits"], ("fixture digits", ex)
        full = []
        steps = dict((b, v) for b, v in ex["bounds_steps"])
        cur = 0
        for b in range(101):
            cur = steps.get(b, cur)
            full.append(cur)
        full[100] = len(ex["keys"])
        assert orc.bounds(k, 2).tolist() == full, ("bounds100", ex)
        assert orc.radix_sort_keys(k, 2)[1].tolist() == full, ("radix bounds100", ex)


def pin_two_digit_string_route(orc, seed=24):
    """Hundred-bucket bounds by decimal strings, by lower_bound of the sorted
    output at beta + b*10^(D-2), and folded onto the ten-bucket bounds."""
    rng = np.random.default_rng(seed)
    cases = []
    for D in range(1, 11):
        hi = 10**D - 1 if D < 10 else I32.max
        k = rng.integers(0, 10 ** (D - 1), 60, dtype=np.int64)
        k[rng.integers(0, 60)] = rng.integers(10 ** (D - 1), hi, endpoint=True)
        cases.append(k.astype(np.int32))
    for D in range(1, 21):
        if D < 20:
            k = [int(x) for x in rng.integers(0, 10 ** (D - 1), 50, dtype=np.int64)]
            k.append(int(rng.integers(10 ** (D - 1), min(10**D - 1, I64.max), endpoint=True, dtype=np.int64)))
        else:
            k = [I64.min, I64.max] + [int(x) for x in rng.integers(I64.min, I64.max, 40, dtype=np.int64)]
        cases.append(np.array(k, np.int64))
    for D in range(1, 20):
        for top in (10 ** (D - 1), 10**D - 1, 10**D):
            for dt, info in ((np.int32, I32), (np.int64, I64)):
                if top <= info.max:
                    cases.append(np.array([0, top // 7, top // 3, top], dt))
    for _ in range(60):
        dt = np.int32 if rng.random() < 0.5 else np.int64
        info = np.iinfo(dt)
        lo = int(rng.integers(info.min, info.max, dtype=dt)) if rng.random() < 0.5 else 0
        hi = int(rng.integers(max(lo, 0), info.max, dtype=dt, endpoint=True))
        cases.append(rng.integers(lo, hi, int(rng.integers(1, 400)), dtype=dt, endpoint=True))
    for k in cases:
        b2 = orc.bounds(k, 2).tolist()
        assert b2 == string_bounds2(k.tolist()), k
        assert b2[::10] == orc.bounds(k).tolist(), k  # bucket b = buckets 10b .. 10b+9
        beta, D, p, _ = string_plan(k.tolist())
        if D >= 2:
            s = np.array(sorted(int(x) for x in k), dtype=object)
            lb = [0] + [int(np.searchsorted(s, beta + b * (p // 10), side="left")) for b in range(1, 100)] + [len(s)]
            assert b2 == lb, k


def pin_two_digit_radix_and_stages(orc, seed=25):
    """The hundred-bucket pipeline run sequentially equals the plain sort; its
    scatter is stable and in bucket order; its local sorts sort each
    partition of each bucket."""
    rng = np.random.default_rng(seed)
    for n in [0, 1, 9, 1000, 30_011]:
        for dt in (np.int32, np.int64):
            info = np.iinfo(dt)
            for k in (rng.integers(info.min, info.max, n, dtype=dt, endpoint=True),
                      rng.integers(0, 1000, n).astype(dt), rng.integers(0, 7, n).astype(dt)):
                rk, rb = orc.radix_sort_keys(k, 2)
                assert np.array_equal(rk, orc.sort_keys(k)), (n, dt)
                assert rb.tolist() == string_bounds2(k.tolist()), (n, dt)
        k = rng.integers(0, 1000, n, dtype=np.int32)
        v = np.arange(n, dtype=np.uint32)
        rk, rv, _ = orc.radix_sort_pairs(k, v, 2)
        pk, pv = orc.sort_pairs(k, v)
        assert np.array_equal(rk, pk) and np.array_equal(rv, pv), n
    for n, T in [(0, 4), (1, 4), (500, 7), (20_000, 64), (50_000, 1000)]:
        k = rng.integers(0, 3000, n, dtype=np.int32)
        v = np.arange(n, dtype=np.uint32)
        sk, sv, b = orc.scatter(k, v, 2)
        assert b.tolist() == string_bounds2(k.tolist())
        d_in, d_out = string_plan2(k.tolist())[3], string_plan2(sk.tolist())[3] if n else []
        assert d_out == sorted(d_in), "buckets out of order"
        assert np.array_equal(k[sv], sk), "payload does not follow its key"
        for bk in range(100):
            assert np.all(np.diff(sv[b[bk]:b[bk + 1]].astype(np.int64)) > 0), "scatter not stable"
        tk, tv, tb = orc.bucket_tiles(k, T, v, 2)
        assert np.array_equal(tb, b)
        for bk in range(100):
            for s0 in range(int(b[bk]), int(b[bk + 1]), T):
                e = min(s0 + T, int(b[bk + 1]))
                order = np.lexsort((sv[s0:e], sk[s0:e]))
                assert np.array_equal(tk[s0:e], sk[s0:e][order]) and np.array_equal(tv[s0:e], sv[s0:e][order])
        k64 = rng.integers(I64.min, I64.max, n, dtype=np.int64, endpoint=True)
        sk, _, b = orc.scatter(k64, digits=2)
        tk, _, _ = orc.bucket_tiles(k64, T, digits=2)
        for bk in range(100):
            for s0 in range(int(b[bk]), int(b[bk + 1]), T):
                e = min(s0 + T, int(b[bk + 1]))
                assert np.array_equal(tk[s0:e], np.sort(sk[s0:e])), (n, T, bk, s0)


ALL_PINS = [
    pin_worked_examples,
    pin_exhaustive_small,
    pin_pairs_brute,
    pin_random_brute,
    pin_library,
    pin_bounds_string_route,
    pin_radix_mode,
    pin_scatter,
    pin_bucket_tiles,
    pin_segmented,
    pin_count,
    pin_two_digit_worked_examples,
    pin_two_digit_string_route,
    pin_two_digit_radix_and_stages,
]
