"""Pins of the event-clustering oracle (merging the per-series events of
section 2.3 across DM trials and boxcar widths)."""
import numpy as np
import pytest

import oracle
from oracle.cluster import cluster_events
import synth

# (width_idx, dm_idx, t_start, t_end, t_peak, b_peak, snr), widths [1, 2, 4]:
# spans are [t_start, t_end + w - 1]
HAND = [
    (0, 5, 100, 102, 101, 50, 7.0),    # 0: span 100..102
    (0, 6, 103, 104, 103, 60, 8.0),    # 1: span 103..104, touches 0 only at tol >= 1
    (0, 9, 102, 102, 102, 10, 6.5),    # 2: span 102..102, joins 3 through 3's width
    (1, 7, 101, 101, 101, 70, 9.0),    # 3: w = 2, span 101..102
    (1, 8, 200, 201, 200, 20, 6.0),    # 4: far in time
    (2, 5, 103, 103, 103, 80, 9.0),    # 5: w = 4, span 103..106, ties 3's snr
    (2, 20, 500, 501, 500, 5, 9.0),    # 6: far in DM and time
]
HAND_WIDTHS = [1, 2, 4]


def test_hand_built_tolerance_zero():
    labels, cl = cluster_events(HAND, HAND_WIDTHS, 2, 1, 0)
    assert labels.tolist() == [0, 1, 0, 0, 2, 3, 4]
    c = cl[0]
    assert (c["first"], c["rep"], c["n_members"]) == (0, 3, 3)
    assert (c["dm_lo"], c["dm_hi"], c["w_lo"], c["w_hi"], c["t_lo"], c["t_hi"]) == (5, 9, 0, 1, 100, 102)
    assert (c["t_peak"], c["dm_idx"], c["width_idx"], c["snr"]) == (101, 7, 1, 9.0)
    assert [x["rep"] for x in cl] == [3, 1, 4, 5, 6]


def test_hand_built_tolerance_one_and_tie():
    labels, cl = cluster_events(HAND, HAND_WIDTHS, 2, 1, 1)
    assert labels.tolist() == [0, 0, 0, 0, 1, 0, 2]
    c = cl[0]
    # 3 and 5 tie at snr 9: the lower index represents the cluster
    assert (c["rep"], c["n_members"], c["t_hi"], c["w_hi"]) == (3, 5, 106, 2)


def test_hand_built_wider_width_radius():
    labels, cl = cluster_events(HAND, HAND_WIDTHS, 2, 2, 0)
    # 1 (w = 1, span 103..104) and 5 (w = 4, span 103..106) become friends
    assert labels.tolist() == [0, 1, 0, 0, 2, 1, 3]
    assert cl[1]["rep"] == 5 and cl[1]["n_members"] == 2


def test_singletons_when_nothing_can_link():
    # width 1 everywhere, zero radii and tolerance: maximal runs of one
    # series are at least one sample apart, so no two events are friends
    ev = synth.make_event_list(3, 50, 1, 5000)
    labels, cl = cluster_events(ev, [1], 0, 0, 0)
    assert labels.tolist() == list(range(len(ev)))
    assert all(c["rep"] == c["first"] == i and c["n_members"] == 1 for i, c in enumerate(cl))


def test_one_series_is_interval_merging():
    # a single (width, DM) series reduces to merging sorted intervals whose
    # gap is at most the tolerance (textbook sweep)
    rng = np.random.default_rng(11)
    for w, tol in ((1, 0), (1, 3), (3, 0), (8, 2)):
        t = 0
        rows = []
        for _ in range(300):
            t += int(rng.integers(2, 12))
            e = t + int(rng.integers(0, 4))
            rows.append((0, 0, t, e, t, 1, 7.0))
            t = e
        labels, _ = cluster_events(rows, [w], 0, 0, tol)
        want, g, end = [], -1, None
        for (_, _, s, e, *_rest) in rows:
            if end is None or s > end + tol:
                g += 1
                end = e + w - 1
            else:
                end = max(end, e + w - 1)
            want.append(g)
        assert labels.tolist() == want, (w, tol)


def test_everything_links_when_bounds_are_huge():
    ev = synth.make_event_list(4, 200, 6, 20000)
    labels, cl = cluster_events(ev, [1, 2, 4, 8, 16, 32], 10 ** 6, 10 ** 6, 10 ** 9)
    assert (labels == 0).all() and len(cl) == 1
    c = cl[0]
    assert c["rep"] == int(np.argmax(ev["snr"]))          # argmax takes the first maximum
    assert (c["dm_lo"], c["dm_hi"]) == (int(ev["dm_idx"].min()), int(ev["dm_idx"].max()))
    assert c["t_lo"] == int(ev["t_start"].min())


def test_partition_invariants_and_coarsening():
    ev = synth.make_event_list(5, 400, 8, 60000, nclumps=30, nnoise=300)
    widths = [1 << i for i in range(8)]
    prev = None
    for params in ((0, 0, 0), (1, 0, 0), (2, 1, 0), (2, 1, 4), (6, 2, 16)):
        labels, cl = cluster_events(ev, widths, *params)
        # numbered by the first member, in order
        firsts = [int(np.nonzero(labels == c)[0][0]) for c in range(len(cl))]
        assert firsts == sorted(firsts) == [c["first"] for c in cl]
        for c, rec in enumerate(cl):
            m = np.nonzero(labels == c)[0]
            assert rec["n_members"] == len(m)
            assert ev["snr"][rec["rep"]] == ev["snr"][m].max()
            assert rec["rep"] == m[np.argmax(ev["snr"][m])]
        if prev is not None:
            # larger bounds only merge clusters
            for c in range(labels.max() + 1):
                assert len(np.unique(labels[prev == prev[labels == c][0]])) == 1
        prev = labels
    assert len(np.unique(prev)) < len(ev)


@pytest.fixture(scope="module")
def small_search():
    fb = synth.make_small(1)
    _, _, ev = oracle.search(fb.packed, fb.nsamps, fb.nchans, fb.f_top, fb.df, fb.tsamp,
                             fb.dm_list, fb.widths, fb.snr_thresh)
    return fb, ev


def test_each_injected_pulse_becomes_one_candidate(small_search):
    """The events of one dispersed pulse (many trials and widths) merge into
    one cluster represented near the pulse's trial and arrival time, and
    different pulses stay apart."""
    fb, ev = small_search
    labels, cl = cluster_events(ev, fb.widths, 2, 1, 0)
    assert len(cl) < len(ev) // 5
    seen = set()
    for p in fb.pulses:
        near = [i for i, e in enumerate(ev)
                if abs(e[1] - p.dm_idx) <= 2 and abs(e[4] - p.t0) <= p.width + 2]
        assert near
        cs = {int(labels[i]) for i in near}
        assert len(cs) == 1
        c = cl[cs.pop()]
        assert c["n_members"] >= len(near) and c["first"] not in seen
        seen.add(c["first"])
        assert abs(c["dm_idx"] - p.dm_idx) <= 2 and abs(c["t_peak"] - p.t0) <= p.width + 2
