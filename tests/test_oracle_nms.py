"""Pins of the oracle's candidate selection (per-width non-maximum
suppression): a hand-worked list whose boundary cases sit exactly on the
strict window limits and whose ties need the stated order, and invariants
that hold for any list (kept events never suppress each other, every dropped
event has a kept neighbour of higher priority, widths are independent)."""
import numpy as np

from oracle import nms
from oracle.peaks import EVENT_FIELDS

WIDTHS = [1, 4]


def _ev(rows):
    """rows: (width_idx, dm_idx, t_peak, snr) -> event tuples."""
    return [(w, d, t - 1, t + 1, t, 100, np.float32(s)) for w, d, t, s in rows]


def test_hand_worked_list():
    ev = _ev([
        (0, 10, 1000, 7.0),   # 0: within 10 trials and 50 samples of 1 -> dropped
        (0, 20, 1050, 9.0),   # 1: highest S/N of width 0 (ties broken by DM) -> kept
        (0, 52, 1050, 8.0),   # 2: exactly 32 trials from 1 (not < 32) -> kept
        (0, 21, 1178, 6.5),   # 3: exactly 128 samples from 1 and 2 -> kept
        (1, 20, 1050, 6.2),   # 4: width 4: never suppressed by width 0 -> kept
        (1, 25, 1500, 6.2),   # 5: ties 4 on S/N, higher DM -> visited after 4; 450 < 512 -> dropped
        (0, 30, 900, 9.0),    # 6: ties 1 on S/N, higher DM; 150 samples from 1 -> kept
        (0, 40, 1000, 9.0),   # 7: ties 1 and 6, highest DM; 20 trials, 50 samples from 1 -> dropped
    ])
    assert nms(ev, WIDTHS) == [1, 2, 3, 4, 6]


def test_ties_fall_to_earlier_time_then_index():
    ev = _ev([(0, 5, 300, 7.0), (0, 5, 200, 7.0), (0, 5, 200, 7.0)])
    assert nms(ev, WIDTHS) == [1]


def _random_list(seed, n):
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n):
        w = int(rng.integers(0, 2))
        rows.append((w, int(rng.integers(0, 200)), int(rng.integers(0, 4000)),
                     float(np.round(rng.uniform(6, 9), 1))))   # rounding makes ties common
    return _ev(rows)


def _close(a, b):
    return a[0] == b[0] and abs(a[1] - b[1]) < 32 and abs(a[4] - b[4]) < 128 * WIDTHS[a[0]]


def _prio(e, i):
    return (-float(e[6]), e[1], e[4], i)


def test_invariants_on_random_lists():
    for seed in range(6):
        ev = _random_list(seed, 300)
        keep = nms(ev, WIDTHS)
        assert keep == sorted(set(keep))
        ks = set(keep)
        for a in keep:
            for b in keep:
                if a < b:
                    assert not _close(ev[a], ev[b]), (seed, a, b)
        for i in range(len(ev)):
            if i in ks:
                continue
            assert any(_close(ev[i], ev[j]) and _prio(ev[j], j) < _prio(ev[i], i) for j in keep), \
                (seed, i)
        # widths are independent
        per_w = []
        for w in range(2):
            idx = [i for i, e in enumerate(ev) if e[0] == w]
            per_w += [idx[k] for k in nms([ev[i] for i in idx], WIDTHS)]
        assert sorted(per_w) == keep


def test_structured_input_same_as_tuples():
    ev = _random_list(9, 120)
    arr = np.array([tuple(e) for e in ev],
                   dtype=[(f, t) for f, t in zip(EVENT_FIELDS, ["<i4", "<i4", "<i8", "<i8", "<i8",
                                                                "<i4", "<f4"])])
    assert nms(arr, WIDTHS) == nms(ev, WIDTHS)
