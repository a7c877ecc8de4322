"""The CPU oracle against brute force, library routines, hand-worked examples
and invariants (see oracle_pins.py for what each pin uses)."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(orc, pin):
    pin(orc)


def test_brute_force_helpers_are_stable():
    # the brute-force route itself: insertion sort keeps equal keys in order
    keys, vals = P.stable_pairs_brute([2, 1, 2, 1, 0], [0, 1, 2, 3, 4])
    assert keys == [0, 1, 1, 2, 2] and vals == [4, 1, 3, 0, 2]
    assert P.string_plan([5, 50, 10, 9]) == (0, 2, 10, [0, 5, 1, 0])


def test_openmp_hybrid_baseline_equals_oracle(orc):
    """The benchmark's multi-core CPU comparison point (the paper's method with
    OpenMP) sorts exactly like the oracle, on any thread count."""
    import numpy as np

    import oracle

    r = np.random.default_rng(21)
    info = np.iinfo(np.int32)
    cases = [np.zeros(0, np.int32), np.array([5], np.int32), np.array([3, -1], np.int32),
             r.integers(0, 2**31 - 1, 100_003, dtype=np.int32),
             r.integers(info.min, info.max, 70_001, dtype=np.int32, endpoint=True),
             r.integers(0, 1000, 90_000).astype(np.int32), np.full(5000, 7, np.int32),
             np.array([info.min, info.max, 0, -1] * 50, np.int32)]
    for k in cases:
        for threads in (1, 3, 8):
            got, used = oracle.omp_hybrid_sort(k, threads)
            assert used == threads
            assert np.array_equal(got, orc.sort_keys(k)), (k.size, threads)
