"""Pins of the baseline-removal oracle (section 2.3, first paragraph)."""
import numpy as np

import oracle


def test_constant_and_linear_series_are_flat():
    # a constant's window mean is itself; a straight line's symmetric window
    # mean is its centre value exactly (sum = (2R+1) * centre)
    for s in (np.full(100, 7), 3 + 2 * np.arange(100)):
        out = oracle.baseline_remove(s, 5, 40)
        assert out.shape == (90,) and (out == 40).all()


def test_spike_by_hand():
    # one spike of 22 at t = 10 in zeros, R = 2 (window 5): positions 6..10
    # of the output (windows covering sample 10) see floor(22/5) = 4; the
    # output at the spike itself (t = 8, input 10) is 22 - 4 + 0 = 18
    s = np.zeros(21, np.int64)
    s[10] = 22
    out = oracle.baseline_remove(s, 2, 0)
    want = np.zeros(17, np.int64)
    want[6:11] = -4
    want[8] = 18
    assert out.tolist() == want.tolist()


def test_brute_force_small():
    rng = np.random.default_rng(5)
    s = rng.integers(0, 3000, size=(3, 257))
    for r in (0, 1, 7, 100):
        out = oracle.baseline_remove(s, r, 1000)
        for d in range(3):
            for t in range(257 - 2 * r):
                win = sum(int(v) for v in s[d, t:t + 2 * r + 1])
                assert out[d, t] == int(s[d, t + r]) - win // (2 * r + 1) + 1000


def test_floor_of_negative_free_sums_and_radius_zero():
    s = np.array([5, 9, 1])
    assert oracle.baseline_remove(s, 0, 3).tolist() == [3, 3, 3]
