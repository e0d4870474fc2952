"""The binomial checkpoint schedule (host logic, no GPU): every step is reversed once, in
order, from an available state; no more than s slots are ever in use; and the number of
recomputed steps equals the closed-form minimum of Griewank & Walther, which a brute-force
dynamic programme over all split points confirms on small cases."""
from functools import lru_cache

import pytest

from paper_1511_06959_amd import revolve as R


@lru_cache(None)
def _dp(l, s):
    if l <= 1:
        return 0
    if s == 1:
        return l * (l - 1) // 2
    return min(m + _dp(l - m, s - 1) + _dp(m, s) for m in range(1, l))


def test_closed_form_matches_brute_force():
    for s in range(1, 7):
        for l in range(1, 45):
            assert R.min_advances(l, s) == _dp(l, s), (l, s)


@pytest.mark.parametrize("l", [1, 2, 3, 7, 20, 64, 137, 400])
@pytest.mark.parametrize("s", [1, 2, 3, 5, 10])
def test_schedule_valid_and_optimal(l, s):
    acts = R.schedule(l, s)
    assert R.simulate(acts, l, s) == R.min_advances(l, s)


def test_store_all_needs_one_pass():
    # with a slot for every state the schedule advances each step exactly once
    assert R.simulate(R.schedule(50, 51), 50, 51) == 49


def test_large_window_budget():
    # 5000 steps with 440 slots: two repetitions, about 1.9 forward steps per step
    assert R.repetitions(5000, 440) == 2
    assert R.min_advances(5000, 440) < 2 * 5000
    assert R.slots_for_budget(10, 105, 5000) == 10


def test_schedule_rejects_no_slot():
    with pytest.raises(ValueError):
        R.schedule(5, 0)
