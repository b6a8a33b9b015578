"""Pins of the oracle's boxcar, sigma-cut and peak finding (section 2.3)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle.peaks import series_events, thresholds
import synth
from conftest import GOLDEN


def test_boxcar_width1_and_direct_window_sum():
    rng = np.random.default_rng(3)
    s = rng.integers(0, 3073, size=(3, 300))
    widths = [1, 2, 4, 8, 32]
    bw = oracle.boxcar(s, widths)
    nbx = 300 - 32 + 1
    assert bw.shape == (5, 3, nbx)
    assert (bw[0] == s[:, :nbx]).all()
    for wi, w in enumerate(widths):
        for d in range(3):
            direct = np.array([s[d, t:t + w].sum() for t in range(nbx)])
            conv = np.convolve(s[d], np.ones(w, dtype=np.int64), mode="valid")[:nbx]
            assert (bw[wi, d] == direct).all() and (bw[wi, d] == conv).all()


def test_boxcar_large_values_exact():
    # running sums far beyond 2^32; the windows stay exact
    s = np.full((1, 5000), (1 << 31) - 1, dtype=np.int64)
    bw = oracle.boxcar(s, [1, 3])
    assert (bw[1] == 3 * ((1 << 31) - 1)).all()


def test_stats_match_numpy_float64():
    rng = np.random.default_rng(4)
    b = rng.integers(0, 200000, size=10007)
    n, s1, s2 = oracle.series_stats(b)
    mu = s1 / n
    sigma = math.sqrt((n * s2 - s1 * s1)) / n
    assert mu == pytest.approx(b.mean(), rel=1e-12)
    assert sigma == pytest.approx(b.std(ddof=0), rel=1e-12)


def test_threshold_equals_direct_definition():
    rng = np.random.default_rng(5)
    for trial in range(40):
        b = rng.integers(0, 50, size=int(rng.integers(2, 60)))
        n, s1, s2 = oracle.series_stats(b)
        k = float(np.float32(rng.uniform(0.1, 4.0)))
        thr = oracle.threshold_level(n, s1, s2, k)
        for v in range(0, 200):
            direct = oracle.is_event(v, n, s1, s2, k)
            assert direct == (thr is not None and v >= thr), (trial, v)


def test_integer_decision_equals_float_away_from_ties():
    rng = np.random.default_rng(6)
    checked = 0
    for _ in range(200):
        b = rng.integers(0, 1000, size=200)
        n, s1, s2 = oracle.series_stats(b)
        thr = oracle.threshold_level(n, s1, s2, 2.0)
        d = n * s2 - s1 * s1
        for v in b.tolist():
            snr = (n * v - s1) / math.sqrt(d)
            if abs(snr - 2.0) > 1e-9:
                assert (snr > 2.0) == (v >= thr)
                checked += 1
    assert checked > 10000


def test_exact_k_rejects_bad():
    for k in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(ValueError):
            oracle.exact_k(k)


def test_golden_runs():
    g = json.load(open(os.path.join(GOLDEN, "runs_handbuilt.json")))
    for case in g["run_cases"]:
        s = np.array(case["series"])
        runs = oracle.find_runs(s >= case["thr"])
        got = [[a, b, a + int(np.argmax(s[a:b + 1])), int(s[a + int(np.argmax(s[a:b + 1]))])]
               for a, b in runs]
        assert got == case["runs"]


def test_golden_sigma_cut():
    g = json.load(open(os.path.join(GOLDEN, "runs_handbuilt.json")))
    for case in g["sigma_cases"]:
        s = np.array(case["series"])
        n, s1, s2 = oracle.series_stats(s)
        assert oracle.threshold_level(n, s1, s2, case["k"]) == case["thr"]
        ev = series_events(s, case["k"], 0, 0)
        got = [[e[2], e[3], e[4], e[5], float(e[6])] for e in ev]
        assert got == case["events"]


def test_event_order_and_fields():
    rng = np.random.default_rng(8)
    bw = rng.integers(0, 10, size=(2, 3, 400))
    bw[1, 2, 50:55] = 40
    bw[0, 0, 399] = 40
    ev = oracle.find_events(bw, 3.0)
    keys = [(e[0], e[1], e[2]) for e in ev]
    assert keys == sorted(keys)
    assert (0, 0, 399) in keys and (1, 2, 50) in keys
    thr = thresholds(bw, 3.0)
    for e in ev:
        w, d, ts, te, tp, bp, snr = e
        seg = bw[w, d, ts:te + 1]
        assert (seg >= thr[w, d]).all() and bp == seg.max() and tp == ts + int(np.argmax(seg))
        assert ts == 0 or bw[w, d, ts - 1] < thr[w, d]
        assert te == 399 or bw[w, d, te + 1] < thr[w, d]


def test_small_config_pulses_recovered_at_their_trial():
    """Each injected pulse peaks at its own trial DM and arrival sample."""
    fb = synth.make_small(1)
    dly = oracle.delay_table(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    x = oracle.unpack_2bit(fb.packed, fb.nsamps, fb.nchans)
    out = oracle.dedisperse(x, dly)
    assert out.shape == (100, 28691)
    bw = oracle.boxcar(out, fb.widths)
    for p in fb.pulses:
        wi = max(i for i, w in enumerate(fb.widths) if w <= p.width)
        w = fb.widths[wi]
        win = bw[wi, :, p.t0 - 8:p.t0 + 8]
        d_best, t_best = np.unravel_index(int(np.argmax(win)), win.shape)
        assert abs(d_best - p.dm_idx) <= 1
        assert p.t0 - 8 + t_best in range(p.t0, p.t0 + p.width - w + 1)
    ev = oracle.find_events(bw, fb.snr_thresh)
    for p in fb.pulses:
        assert any(abs(e[1] - p.dm_idx) <= 2 and abs(e[4] - p.t0) <= p.width + 2 for e in ev)
