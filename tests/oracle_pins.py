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
import math
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


def string_plan3(keys):
    """Three-digit buckets via decimal strings: the first three characters of
    u written with D digits (a u of one or two digits gets trailing zeros)."""
    beta, D, p, _ = string_plan(keys)
    digits = [int((str(int(k) - beta).rjust(D, "0") + "00")[:3]) for k in keys]
    return beta, D, p, digits


def string_bounds3(keys):
    cnt = [0] * 1000
    for d in string_plan3(keys)[3]:
        cnt[d] += 1
    b = [0]
    for c in cnt:
        b.append(b[-1] + c)
    return b


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


def pin_three_digit_worked_examples(orc):
    with open(GOLDEN) as f:
        g = json.load(f)["three_digit"]
    for ex in g["cases"]:
        k = np.array(ex["keys"], np.int32 if ex["dtype"] == "int32" else np.int64)
        assert string_plan3(ex["keys"])[3] == ex["digits"], ("fixture digits", ex)
        steps = dict((b, v) for b, v in ex["bounds_steps"])
        full, cur = [], 0
        for b in range(1001):
            cur = steps.get(b, cur)
            full.append(cur)
        full[1000] = len(ex["keys"])
        assert orc.bounds(k, 3).tolist() == full, ("bounds1000", ex)
        assert orc.radix_sort_keys(k, 3)[1].tolist() == full, ("radix bounds1000", ex)


def pin_three_digit_string_route(orc, seed=26):
    """Thousand-bucket bounds by decimal strings, by lower_bound of the sorted
    output at beta + b*10^(D-3), and folded onto the hundred-bucket bounds."""
    rng = np.random.default_rng(seed)
    cases = []
    for D in range(1, 11):
        hi = 10**D - 1 if D < 10 else I32.max
        k = rng.integers(0, 10 ** (D - 1), 80, dtype=np.int64)
        k[rng.integers(0, 80)] = rng.integers(10 ** (D - 1), hi, endpoint=True)
        cases.append(k.astype(np.int32))
    for D in range(1, 21):
        if D < 20:
            k = [int(x) for x in rng.integers(0, 10 ** (D - 1), 60, dtype=np.int64)]
            k.append(int(rng.integers(10 ** (D - 1), min(10**D - 1, I64.max), endpoint=True, dtype=np.int64)))
        else:
            k = [I64.min, I64.max] + [int(x) for x in rng.integers(I64.min, I64.max, 40, dtype=np.int64)]
        cases.append(np.array(k, np.int64))
    for D in range(1, 20):
        for top in (10 ** (D - 1), 10**D - 1, 10**D):
            for dt, info in ((np.int32, I32), (np.int64, I64)):
                if top <= info.max:
                    cases.append(np.array([0, top // 7, top // 3, top // 101, top], dt))
    for _ in range(40):
        dt = np.int32 if rng.random() < 0.5 else np.int64
        info = np.iinfo(dt)
        lo = int(rng.integers(info.min, info.max, dtype=dt)) if rng.random() < 0.5 else 0
        hi = int(rng.integers(max(lo, 0), info.max, dtype=dt, endpoint=True))
        cases.append(rng.integers(lo, hi, int(rng.integers(1, 2000)), dtype=dt, endpoint=True))
    for k in cases:
        b3 = orc.bounds(k, 3).tolist()
        assert b3 == string_bounds3(k.tolist()), k
        assert b3[::10] == orc.bounds(k, 2).tolist(), k  # bucket c of 100 = buckets 10c .. 10c+9
        beta, D, p, _ = string_plan(k.tolist())
        if D >= 3:
            s = np.array(sorted(int(x) for x in k), dtype=object)
            lb = [0] + [int(np.searchsorted(s, beta + b * (p // 100), side="left")) for b in range(1, 1000)] + [len(s)]
            assert b3 == lb, k


def pin_three_digit_radix_and_stages(orc, seed=27):
    """The thousand-bucket pipeline run sequentially equals the plain sort; its
    scatter is stable and in bucket order; its local sorts sort each
    partition of each bucket."""
    rng = np.random.default_rng(seed)
    for n in [0, 1, 9, 1000, 30_011]:
        for dt in (np.int32, np.int64):
            info = np.iinfo(dt)
            for k in (rng.integers(info.min, info.max, n, dtype=dt, endpoint=True),
                      rng.integers(0, 100_000, n).astype(dt), rng.integers(0, 7, n).astype(dt)):
                rk, rb = orc.radix_sort_keys(k, 3)
                assert np.array_equal(rk, orc.sort_keys(k)), (n, dt)
                assert rb.tolist() == string_bounds3(k.tolist()), (n, dt)
    for n, T in [(0, 4), (1, 4), (700, 7), (40_000, 64)]:
        k = rng.integers(0, 30_000, n, dtype=np.int32)
        v = np.arange(n, dtype=np.uint32)
        sk, sv, b = orc.scatter(k, v, 3)
        assert b.tolist() == string_bounds3(k.tolist())
        d_in, d_out = string_plan3(k.tolist())[3], string_plan3(sk.tolist())[3] if n else []
        assert d_out == sorted(d_in), "buckets out of order"
        assert np.array_equal(k[sv], sk), "payload does not follow its key"
        for bk in range(1000):
            assert np.all(np.diff(sv[b[bk]:b[bk + 1]].astype(np.int64)) > 0), "scatter not stable"
        tk, tv, tb = orc.bucket_tiles(k, T, v, 3)
        assert np.array_equal(tb, b)
        for bk in range(1000):
            for s0 in range(int(b[bk]), int(b[bk + 1]), T):
                e = min(s0 + T, int(b[bk + 1]))
                order = np.lexsort((sv[s0:e], sk[s0:e]))
                assert np.array_equal(tk[s0:e], sk[s0:e][order]) and np.array_equal(tv[s0:e], sv[s0:e][order])


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


# ------------------------------------------------------- other key types
TYPED = [np.int32, np.uint32, np.float32, np.int64, np.uint64, np.float64]


def total_order_key(x):
    """IEEE-754 total order as a Python sort key, from the values alone (no
    bit patterns): negative NaNs first, then the numbers by value with -0
    before +0, then positive NaNs (NaN payloads are not mixed here)."""
    x = float(x)
    neg = math.copysign(1.0, x) < 0
    if math.isnan(x):
        return (0,) if neg else (2,)
    return (1, x, 0 if neg else 1)


def typed_order_key(dt):
    if np.dtype(dt).kind == "f":
        return total_order_key
    return int


def brute_typed(keys, desc):
    """Stable order of the positions by Python's sort (stable also with
    reverse=True: equal keys keep their input order)."""
    kf = typed_order_key(keys.dtype)
    return sorted(range(len(keys)), key=lambda i: kf(keys[i]), reverse=desc)


def typed_samples(dt, n, rng):
    info = np.finfo(dt) if np.dtype(dt).kind == "f" else np.iinfo(dt)
    if np.dtype(dt).kind == "f":
        special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, -np.nan, 1.5, -1.5, info.tiny, -info.tiny,
                            info.max, -info.max, info.smallest_subnormal, -info.smallest_subnormal], dt)
        body = (rng.standard_normal(n) * 10.0 ** rng.integers(-5, 6, n)).astype(dt)
        body[rng.random(n) < 0.1] = 0.0
        return np.where(rng.random(n) < 0.2, rng.choice(special, n), body).astype(dt)
    special = np.array([info.min, info.max, 0, 1, info.max - 1], dt)
    body = rng.integers(info.min, info.max, n, dtype=dt, endpoint=True)
    small = rng.integers(0, 50, n).astype(dt)
    pick = rng.random(n)
    return np.where(pick < 0.15, rng.choice(special, n), np.where(pick < 0.5, small, body)).astype(dt)


def order_image_py(k, desc):
    """The order image of the oracle's reading for other key types, and
    whether its bucket rule is unsigned (u = image) or signed (u = image -
    min(min image, 0)).  Floats: m = the magnitude bits, image m or -1 - m."""
    dt = k.dtype
    if dt.kind == "u":
        top = int(np.iinfo(dt).max)
        return [top - int(x) if desc else int(x) for x in k], True
    if dt.kind == "f":
        ib = np.uint32 if dt.itemsize == 4 else np.uint64
        bits = k.view(ib)
        w = 8 * dt.itemsize
        img = []
        for b in bits:
            b = int(b)
            m = b & ((1 << (w - 1)) - 1)
            img.append(-1 - m if b >> (w - 1) else m)
    else:
        img = [int(x) for x in k]
    return ([-1 - v for v in img] if desc else img), False


def string_buckets_typed(k, desc, digits):
    """Each key's bucket: the first one, two or three characters of the
    decimal string of u, written with D digits (a shorter u gets trailing
    zeros)."""
    img, unsigned = order_image_py(k, desc)
    if not img:
        return []
    beta = 0 if unsigned else min(min(img), 0)
    us = [v - beta for v in img]
    D = len(str(max(us)))
    return [int((str(u).rjust(D, "0") + "00")[:digits]) for u in us]


def string_bounds_typed(k, desc, digits):
    ds = string_buckets_typed(k, desc, digits)
    cnt = [0] * 10**digits
    for d in ds:
        cnt[d] += 1
    b = [0]
    for c in cnt:
        b.append(b[-1] + c)
    return b


def pin_typed_brute(orc, seed=31):
    """Every key type, both directions, against Python's stable sort with
    comparison keys taken from the values (never from bit patterns); the
    payload (input positions) must come out in the same stable order."""
    rng = np.random.default_rng(seed)
    for dt in TYPED:
        for n in [0, 1, 2, 5, 40, 300]:
            k = typed_samples(dt, n, rng)
            for desc in (False, True):
                want = brute_typed(k, desc)
                gk, gv = orc.sort_typed(k, np.arange(n, dtype=np.uint32), descending=desc)
                assert gv.tolist() == want, (np.dtype(dt).name, n, desc)
                assert np.array_equal(gk.view(np.uint8), k[want].view(np.uint8)), (np.dtype(dt).name, n, desc)


def pin_typed_zero_and_nan_order(orc):
    """Hand-worked: -NaN < -inf < -1.5 < -0 < +0 < 1.5 < +inf < +NaN, and the
    reverse for descending order, whatever the input order."""
    for dt in (np.float32, np.float64):
        k = np.array([0.0, np.nan, -0.0, 1.5, -np.inf, -1.5, np.inf, -np.nan], dt)
        asc = [7, 4, 5, 2, 0, 3, 6, 1]
        gk, gv = orc.sort_typed(k, np.arange(8, dtype=np.uint32))
        assert gv.tolist() == asc, np.dtype(dt).name
        gk, gv = orc.sort_typed(k, np.arange(8, dtype=np.uint32), descending=True)
        assert gv.tolist() == asc[::-1], np.dtype(dt).name
        gk, gv = orc.sort_typed(np.array([0.0, -0.0, 0.0, -0.0], dt), np.arange(4, dtype=np.uint32))
        assert gv.tolist() == [1, 3, 0, 2], np.dtype(dt).name


def pin_typed_library(orc, seed=32):
    """numpy's stable sort on larger inputs: unsigned keys directly, floats
    without NaN or -0 (where numpy's order is the total order), descending as
    the stable ascending order of the negated floats / complemented
    unsigned values."""
    rng = np.random.default_rng(seed)
    for n in [1000, 40_001]:
        for dt in (np.uint32, np.uint64):
            k = typed_samples(dt, n, rng)
            idx = np.arange(n, dtype=np.uint32)
            gk, gv = orc.sort_typed(k, idx)
            assert np.array_equal(gv, np.argsort(k, kind="stable")), np.dtype(dt).name
            comp = np.iinfo(dt).max - k
            gk, gv = orc.sort_typed(k, idx, descending=True)
            assert np.array_equal(gv, np.argsort(comp, kind="stable")), np.dtype(dt).name
        for dt in (np.float32, np.float64):
            k = (rng.standard_normal(n) * 1e3).astype(dt)
            k[k == 0] = 1.0
            k[: n // 10] = k[n // 10: 2 * (n // 10)]  # duplicates
            idx = np.arange(n, dtype=np.uint32)
            assert np.array_equal(orc.sort_typed(k, idx)[1], np.argsort(k, kind="stable")), np.dtype(dt).name
            assert np.array_equal(orc.sort_typed(k, idx, descending=True)[1], np.argsort(-k, kind="stable"))
        for dt in (np.int32, np.int64):
            k = typed_samples(dt, n, rng)
            assert np.array_equal(orc.sort_typed(k)[0], orc.sort_keys(k)), np.dtype(dt).name


def pin_typed_bounds(orc, seed=33):
    """Bucket bounds of every type and direction by decimal strings of the
    order image's u, with ten, one hundred and one thousand buckets."""
    rng = np.random.default_rng(seed)
    for dt in TYPED:
        for n in [0, 1, 7, 200]:
            for _ in range(4):
                k = typed_samples(dt, n, rng)
                for desc in (False, True):
                    for digits in (1, 2, 3):
                        assert orc.bounds_typed(k, desc, digits).tolist() == string_bounds_typed(k, desc, digits), \
                            (np.dtype(dt).name, n, desc, digits, k)


def pin_typed_worked_examples(orc):
    with open(GOLDEN) as f:
        g = json.load(f)["typed"]
    for ex in g["cases"]:
        k = np.array(ex["keys"], dtype=ex["dtype"]) if "keys" in ex else np.array(ex["bits"], dtype=ex["bits_dtype"]).view(ex["dtype"])
        assert orc.bounds_typed(k, ex["descending"]).tolist() == ex["bounds"], ex["why"]
        assert orc.sort_typed(k, np.arange(k.size, dtype=np.uint32), ex["descending"])[1].tolist() == ex["order"], ex["why"]


def pin_typed_radix_and_stages(orc, seed=34):
    """Section 3.4 run sequentially on the order image equals the plain
    typed sort (ten, one hundred and one thousand buckets); the scatter keeps input order
    inside a bucket; the local sorts sort every partition of every bucket."""
    rng = np.random.default_rng(seed)
    for dt in TYPED:
        for n, T in [(0, 4), (9, 4), (3000, 64), (20_000, 1000)]:
            k = typed_samples(dt, n, rng)
            v = np.arange(n, dtype=np.uint32)
            for desc in (False, True):
                pk, pv = orc.sort_typed(k, v, desc)
                for digits in (1, 2, 3):
                    rk, rv, rb = orc.radix_sort_typed(k, v, desc, digits)
                    assert np.array_equal(rv, pv), (np.dtype(dt).name, n, desc, digits)
                    assert rb.tolist() == string_bounds_typed(k, desc, digits)
                    sk, sv, sb = orc.stage_typed(k, v, desc, 0, digits)
                    assert np.array_equal(sb, rb)
                    assert np.array_equal(sk.view(np.uint8), k[sv].view(np.uint8)), "key does not follow its position"
                    bk = string_buckets_typed(k, desc, digits)
                    out_b = [bk[i] for i in sv.tolist()]
                    assert out_b == sorted(out_b), "scatter not in bucket order"
                    for b in range(10**digits):
                        assert np.all(np.diff(sv[sb[b]:sb[b + 1]].astype(np.int64)) > 0), "scatter not stable"
                    tk, tv, _ = orc.stage_typed(k, v, desc, T, digits)
                    for b in range(10**digits):
                        for s0 in range(int(sb[b]), int(sb[b + 1]), T):
                            e = min(s0 + T, int(sb[b + 1]))
                            # the partition's positions, sorted stably by the typed order
                            want = [int(sv[s0 + i]) for i in brute_typed(sk[s0:e], desc)]
                            assert tv[s0:e].tolist() == want, (np.dtype(dt).name, n, desc, digits, b)


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
    pin_three_digit_worked_examples,
    pin_three_digit_string_route,
    pin_three_digit_radix_and_stages,
    pin_typed_brute,
    pin_typed_zero_and_nan_order,
    pin_typed_library,
    pin_typed_bounds,
    pin_typed_worked_examples,
    pin_typed_radix_and_stages,
]
