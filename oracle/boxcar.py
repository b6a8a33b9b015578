"""Boxcar matched filter via a running sum (oracle; test infrastructure).

Section 2.3 of the paper: the time series is convolved with boxcars of
increasing width (2, 4, 8, ... samples), computed from a running (prefix) sum
as the difference of two of its points.  Readings:
  * leading window: B_w[t] = sum_{j<w} s[t+j] = P[t+w] - P[t], with
    P[0] = 0, P[t+1] = P[t] + s[t];
  * every width shares one valid length n_bx = nout - w_max + 1, so that all
    widths cover the same start samples;
  * width 1 is allowed (B_1 = s).
"""
from __future__ import annotations

import numpy as np


def n_boxcar(nout: int, widths) -> int:
    return int(nout) - int(max(widths)) + 1


def prefix_sum(s: np.ndarray) -> np.ndarray:
    """P with P[0] = 0 and P[t+1] = P[t] + s[t], in int64 along the last axis."""
    s = np.asarray(s, dtype=np.int64)
    p = np.zeros(s.shape[:-1] + (s.shape[-1] + 1,), dtype=np.int64)
    np.cumsum(s, axis=-1, out=p[..., 1:])
    return p


def boxcar(s: np.ndarray, widths) -> np.ndarray:
    """int64 [nwidths][...][n_bx]: B_w[t] = P[t+w] - P[t] for t < n_bx."""
    s = np.asarray(s)
    nout = s.shape[-1]
    nbx = n_boxcar(nout, widths)
    if nbx <= 0:
        raise ValueError("widest boxcar exceeds the series")
    p = prefix_sum(s)
    return np.stack([p[..., w:w + nbx] - p[..., :nbx] for w in widths])
