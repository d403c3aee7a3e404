"""Pins of the pause-model oracle (Sec. 5.1 benchmark; eq. active_ratio):
the duration law, the counter layout of its draw, and the schedule against
hand-computed cases and an independent event-driven formulation."""
import math

import numpy as np
import pytest

from oracle import pause, rng


def test_zero_spread_is_the_mean_exactly():
    d = pause.durations_us(7, 2, 50, 125.0, 0.0)
    assert np.all(d == 125.0)


def test_duration_law_moments():
    # U(mu - sqrt(3) sigma, mu + sqrt(3) sigma) has mean mu and variance sigma^2
    mu, sigma, n = 100.0, 20.0, 20000
    d = pause.durations_us(3, 0, n, mu, sigma)
    a, w = pause.law(mu, sigma)
    assert np.all((d >= a) & (d <= a + w))
    assert abs(d.mean() - mu) < 5 * sigma / math.sqrt(n)
    # relative standard error of the sample variance of a uniform: sqrt(0.8 / n)
    assert abs(d.var() / sigma**2 - 1.0) < 5 * math.sqrt(0.8 / n)


def test_draw_uses_counter_word_three_and_numpy_philox():
    # numpy's Philox (independent implementation) with counter (i, l, 0, 1) - 1
    seed, level, i = 11, 3, 5
    v = (i + (level << 64) + (1 << 192) - 1) % 2**256
    prev = np.array([(v >> (64 * q)) & (2**64 - 1) for q in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=prev, key=np.array([seed, 0], dtype=np.uint64))
    word = int(bg.random_raw(1)[0])
    u = ((word >> 12) + 0.5) * 2.0 ** -52
    a, w = pause.law(40.0, 5.0)
    d = pause.durations_us(seed, level, i + 1, 40.0, 5.0)
    assert d[i] == a + w * u
    # not the xi stream (word 3 = 0)
    assert rng.philox4x64((i, level, 0, 0), (seed, 0))[0] != word


def test_ticks_round_half_up():
    t = pause.to_ticks(np.array([0.0, 0.004, 0.005, 1.0, 2.25]), 100.0)
    assert list(t) == [0, 0, 1, 100, 225]


def test_one_task_at_a_time():
    # width = capacity: tasks run one after the other, no idle slot
    ticks = np.array([5, 3, 7, 2])
    s = pause.schedule([4], [8], ticks, 8, 1)
    assert s["steps"] == 4 and s["step_lengths"] == [5, 3, 7, 2]
    assert list(s["done_step"]) == [0, 1, 2, 3]
    assert s["ideal_ratio"] == 1.0


def test_all_at_once_completes_in_duration_order():
    ticks = np.array([40, 10, 30, 10, 20])
    s = pause.schedule([5], [1], ticks, 8, 1)
    # boundaries at the distinct finish times 10, 20, 30, 40
    assert s["step_lengths"] == [10, 10, 10, 10]
    assert list(s["done_step"]) == [3, 0, 2, 0, 1]
    assert s["ideal_ratio"] == sum(ticks) / (8 * 40)


def test_finest_first_with_backfill_by_hand():
    # counts (4, 2), widths (1, 3), capacity 4, equal durations:
    # step 0: one level-1 task (3 slots) + one level-0 task; step 1 likewise;
    # step 2: the last two level-0 tasks (2 slots idle)
    ticks = np.full(6, 9)
    s = pause.schedule([4, 2], [1, 3], ticks, 4, 1)
    assert s["steps"] == 3
    assert list(s["done_step"]) == [0, 1, 2, 2, 0, 1]
    assert s["ideal_ratio"] == (2 * 3 + 4 * 1) / (4 * 3)


def test_batch_sums_durations():
    ticks = np.array([1, 2, 3, 4, 5])
    s = pause.schedule([5], [2], ticks, 2, 2)
    assert s["tasks"] == 3 and s["step_lengths"] == [3, 7, 5]
    assert list(s["done_step"]) == [0, 0, 1, 1, 2]


def test_min_step_wastes_the_rest_of_a_step():
    ticks = np.array([2, 10])
    s = pause.schedule([2], [1], ticks, 2, 1, min_step_ticks=6)
    assert s["step_lengths"] == [6, 6]
    assert list(s["done_step"]) == [0, 1]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_step_schedule_equals_event_simulation(seed):
    r = np.random.default_rng(seed)
    counts = [int(c) for c in r.integers(0, 12, size=3)]
    widths = [1, 3, 7]
    ticks = r.integers(0, 50, size=sum(counts))
    for batch in (1, 2, 3):
        s = pause.schedule(counts, widths, ticks, 9, batch)
        fin, idx = pause.event_schedule(counts, widths, ticks, 9, batch)
        assert list(s["done_step"]) == list(idx)
        ends = np.cumsum(s["step_lengths"]) if s["steps"] else np.array([])
        assert all(ends[s["done_step"][k]] == fin[k] for k in range(len(fin)))
