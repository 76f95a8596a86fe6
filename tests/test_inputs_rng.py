"""The random-draw specification (SplitMix64 + Lemire + partial Fisher-Yates)."""
import numpy as np

import kkm_inputs as ki
from kkm_inputs import rng


def test_splitmix64_reference_output():
    # published first output of SplitMix64 started from state 0
    assert rng.SplitMix64(0).next_u64() == 0xE220A8397B1DCDAF


def test_bounded_is_in_range_and_roughly_uniform():
    g = rng.SplitMix64(123)
    xs = np.array([g.bounded(7) for _ in range(70000)])
    assert xs.min() == 0 and xs.max() == 6
    cnt = np.bincount(xs, minlength=7)
    assert np.all(np.abs(cnt - 10000) < 500)


def test_uniform_in_unit_interval():
    g = rng.SplitMix64(5)
    u = np.array([g.uniform() for _ in range(10000)])
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.02


def test_landmarks_sorted_distinct_and_counted():
    for n, s in [(10000, 0.1), (20000, 0.02), (7, 0.5), (5, 0.01), (100, 1.0)]:
        L = ki.draw_landmarks(2001, 3, n, s)
        assert len(L) == ki.landmark_count(n, s)
        assert np.all(np.diff(L) > 0) and L.min() >= 0 and L.max() < n


def test_streams_differ_by_purpose_and_batch():
    a = ki.draw_landmarks(1, 0, 1000, 0.1)
    b = ki.draw_landmarks(1, 1, 1000, 0.1)
    assert not np.array_equal(a, b)
    assert ki.stream(1, 0, 0).next_u64() != ki.stream(1, 1, 0).next_u64()
