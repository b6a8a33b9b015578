"""Baseline (red-noise) removal by a running mean (oracle; test infrastructure).

Section 2.3, first paragraph: recorded series carry slow baseline wiggles;
the usual time-domain remedy is to subtract a running mean over a window (a
wide boxcar), computed from a running sum by differencing the points one
window radius either side.  Readings (the paper gives no window or rounding):
the window is the 2R + 1 samples centred on the sample; only positions whose
window lies wholly inside the series are produced; the mean is taken as the
floor of the exact window sum divided by 2R + 1, so the result is an integer,
and a caller-chosen constant offset keeps it non-negative:

    out[t] = s[t + R] - floor(sum_{j=t}^{t+2R} s[j] / (2R + 1)) + offset,
    0 <= t < n - 2R.
"""
from __future__ import annotations

import numpy as np


def baseline_remove(series: np.ndarray, radius: int, offset: int) -> np.ndarray:
    """Rows of `series` ([..., n]) with the running mean removed (int64)."""
    s = np.asarray(series, dtype=np.int64)
    w = 2 * radius + 1
    n = s.shape[-1]
    if n - 2 * radius < 1:
        raise ValueError("series shorter than the window")
    p = np.zeros(s.shape[:-1] + (n + 1,), dtype=np.int64)
    np.cumsum(s, axis=-1, out=p[..., 1:])
    sums = p[..., w:] - p[..., :n + 1 - w]          # window [t, t + 2R], t < n - 2R
    centre = s[..., radius:n - radius]
    return centre - np.floor_divide(sums, w) + offset
