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
