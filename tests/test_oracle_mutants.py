"""Plant plausible mistakes in copies of the oracle (on the CPU) and require
that at least one pin catches each of them.  Every mutant is compiled to a
temporary library and checked in a subprocess, so a mutant that crashes
counts as caught without taking the test runner down."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("compare_keys_only", "if (a->key != b->key) return a->key < b->key;\n    return a->idx < b->idx;",
     "return a->key < b->key;"),
    ("descending", "if (a->key != b->key) return a->key < b->key;", "if (a->key != b->key) return a->key > b->key;"),
    ("merge_right_on_equal_keys", "if (item_lt(&b[j], &a[i]))", "if (b[j].key <= a[i].key)"),
    ("drop_odd_list", "if (r < nruns) { /* odd list carried to the next round */",
     "if (0) { /* odd list carried to the next round */"),
    ("drop_merge_tail", "while (j < nb) out[k++] = b[j++];", ""),
    ("beta_always_zero", "pl.beta = mn < 0 ? mn : 0;", "pl.beta = 0;"),
    ("beta_always_min", "pl.beta = mn < 0 ? mn : 0;", "pl.beta = mn;"),
    ("digits_off_by_one", "while (d < 20 && x >= POW10[d]) d++;", "while (d < 20 && x > POW10[d]) d++;"),
    ("pow10_typo", "10000000000000ULL,", "1000000000000ULL,"),
    ("bounds_shifted", "bounds[b + 1] = bounds[b] + cnt[b];", "bounds[b + 1] = bounds[b] + cnt[b ? b - 1 : 0];"),
    ("scatter_reversed", "for (int64_t i = 0; i < n; i++) out[next[bucket_n(pl, s[i].key, digits)]++] = s[i];",
     "for (int64_t i = n - 1; i >= 0; i--) out[next[bucket_n(pl, s[i].key, digits)]++] = s[i];"),
    ("two_digit_drops_second_digit", "return (int)(u / POW10[pl->D - 2]);", "return (int)(u / POW10[pl->D - 1] * 10);"),
    ("one_digit_without_trailing_zero", "if (pl->D == 1) return (int)(10 * u);", "if (pl->D == 1) return (int)u;"),
    ("three_digit_reads_two", "return (int)(u / POW10[pl->D - 3]);", "return (int)(u / POW10[pl->D - 2] * 10);"),
    ("three_digit_short_u_unpadded", "if (pl->D < 3) return (int)(u * POW10[3 - pl->D]);", "if (pl->D < 3) return (int)(u * 10);"),
    ("three_digit_uses_two_digit_rule", "if (digits == 3) return bucket3_of(pl, k);", "if (digits == 3) return 10 * bucket2_of(pl, k);"),
    ("scatter_ignores_digit_count", "out[next[bucket_n(pl, s[i].key, digits)]++] = s[i];",
     "out[next[bucket_of(pl, s[i].key)]++] = s[i];"),
    ("tiles_skip_upper_buckets", "    for (int b = 0; b < nb; b++) {\n        for (int64_t t = bounds[b]; t < bounds[b + 1]; t += tile) {",
     "    for (int b = 0; b < 10; b++) {\n        for (int64_t t = bounds[b]; t < bounds[b + 1]; t += tile) {"),
    ("tile_not_bucket_aligned", "for (int64_t t = bounds[b]; t < bounds[b + 1]; t += tile) {\n            int64_t e = t + tile < bounds[b + 1] ? t + tile : bounds[b + 1];\n            quicksort(s, t, e - 1);\n        }\n    }\n    for (int64_t i = 0; i < n; i++) {",
     "for (int64_t t = bounds[b] - bounds[b] % tile; t < bounds[b + 1]; t += tile) {\n            int64_t e = t + tile < bounds[b + 1] ? t + tile : bounds[b + 1];\n            quicksort(s, t, e - 1);\n        }\n    }\n    for (int64_t i = 0; i < n; i++) {"),
    ("partition_skips_last", "for (int64_t j = low; j < high; j++) {", "for (int64_t j = low; j < high - 1; j++) {"),
    ("segment_bounds_unshifted", "if (bounds && oracle_bounds_i32(k + a, m, bounds + 11 * g)) return -1;",
     "if (bounds && oracle_bounds_i32(k, m, bounds + 11 * g)) return -1;"),
    ("float_negative_image_without_offset", "img = (b >> 31) ? -1 - m : m;", "img = (b >> 31) ? -m : m;"),
    ("float64_sign_ignored", "img = (b >> 63) ? -1 - m : m;", "img = m;"),
    ("descending_not_reversed", "return desc ? -1 - img : img;", "return img;"),
    ("unsigned_descending_not_reversed", "return desc ? (int64_t)(UINT32_MAX - x) : (int64_t)x;", "return (int64_t)x;"),
    ("u64_shift_wraps", "if (y >= h) return (int64_t)(y - h);", "if (y >= h) return (int64_t)y;"),
    ("u64_bias_not_fixed", "bounds_items_mode(load_items_typed(k, t, desc, n), n, digits, t == T_U64, bounds);",
     "bounds_items_mode(load_items_typed(k, t, desc, n), n, digits, 0, bounds);"),
    ("typed_gather_keeps_input_order", "memcpy((char*)k + w * (size_t)i, k0 + w * (size_t)s[i].idx, w);",
     "memcpy((char*)k + w * (size_t)i, k0 + w * (size_t)i, w);"),
    ("count_le_strict", "b += k[i] <= x;\n    }\n    *lt = a;\n    *le = b;\n}\n\nvoid oracle_count_lt_le_i64",
     "b += k[i] < x;\n    }\n    *lt = a;\n    *le = b;\n}\n\nvoid oracle_count_lt_le_i64"),
]

RUNNER = r"""
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle, oracle_pins as P
orc = oracle.load_variant({lib!r})
failed = []
for pin in P.ALL_PINS:
    try:
        pin(orc)
    except AssertionError:
        failed.append(pin.__name__)
    except Exception as e:
        failed.append(pin.__name__ + ':' + type(e).__name__)
print('FAILED_PINS', failed)
sys.exit(3 if failed else 0)
"""


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    with open(SRC) as f:
        src = f.read()
    assert src.count(old) >= 1, f"mutation site for {name} not found in oracle.c"
    mutated = src.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "m.c")
        lib = os.path.join(d, "m.so")
        with open(c, "w") as f:
            f.write(mutated)
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", lib, c])
        code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    # rc 3: a pin failed; negative rc: the mutant crashed (also caught)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout}\n{r.stderr}"
