"""Peak finding: sigma-cut mask -> contiguous runs -> events (oracle).

Section 2.3 of the paper: after the sigma-cut, contiguous regions above the
threshold are gathered into individual events (a reduce-by-key over the
mask).  Readings:
  * a run is a maximal set of consecutive t of one (width, DM) series with
    B[t] >= B_thr; runs never merge across DMs or widths;
  * an event records (width_idx, dm_idx, t_start, t_end inclusive,
    t_peak = the first t of the run where B is largest, B at t_peak, S/N at
    t_peak);
  * events are listed in (width_idx, dm_idx, t_start) order.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .sigma_cut import series_stats, threshold_level, snr_value

EVENT_FIELDS = ("width_idx", "dm_idx", "t_start", "t_end", "t_peak", "b_peak", "snr")


def find_runs(mask: np.ndarray) -> List[Tuple[int, int]]:
    """Maximal runs of True as (start, end_inclusive), in order."""
    m = np.asarray(mask, dtype=np.int8)
    if m.size == 0:
        return []
    edges = np.diff(np.concatenate(([0], m, [0])))
    starts = np.nonzero(edges == 1)[0]
    ends = np.nonzero(edges == -1)[0] - 1
    return list(zip(starts.tolist(), ends.tolist()))


def series_events(b: np.ndarray, k: float, w_idx: int, d_idx: int):
    """Events of one boxcar series."""
    n, s1, s2 = series_stats(b)
    thr = threshold_level(n, s1, s2, k)
    if thr is None:
        return []
    out = []
    for ts, te in find_runs(np.asarray(b) >= thr):
        seg = np.asarray(b[ts:te + 1])
        tp = ts + int(np.argmax(seg))        # argmax returns the first maximum
        bp = int(b[tp])
        out.append((w_idx, d_idx, ts, te, tp, bp, snr_value(bp, n, s1, s2)))
    return out


def find_events(bw: np.ndarray, k: float):
    """bw: [nwidths][ndm][n_bx] boxcar series.  Returns the event list in
    (width_idx, dm_idx, t_start) order."""
    ev = []
    for wi in range(bw.shape[0]):
        for d in range(bw.shape[1]):
            ev.extend(series_events(bw[wi, d], k, wi, d))
    return ev


def thresholds(bw: np.ndarray, k: float) -> np.ndarray:
    """B_thr per (width, DM) as int64, with -1 for 'no events' (D == 0)."""
    out = np.empty(bw.shape[:2], dtype=np.int64)
    for wi in range(bw.shape[0]):
        for d in range(bw.shape[1]):
            n, s1, s2 = series_stats(bw[wi, d])
            t = threshold_level(n, s1, s2, k)
            out[wi, d] = -1 if t is None else t
    return out
