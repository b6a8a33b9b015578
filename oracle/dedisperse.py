"""Brute-force ("direct") incoherent dedispersion (oracle; test infrastructure).

Section 2.2 of the paper: every trial DM is a complete integration over the
frequency channels of the channel time series, each shifted by its delay.
Written out:

    out[d][t] = sum_{c < nchans} x[c][t + delay[d][c]],   0 <= t < nout,
    nout = nsamps - max_delay

(only samples where every channel's shifted window lies inside the data are
produced; no padding).  Inputs are 2-bit levels, so the sum is an exact
integer; accumulation is int32.
"""
from __future__ import annotations

import numpy as np


def dedisperse(x: np.ndarray, delays: np.ndarray, nout: int | None = None) -> np.ndarray:
    """x: uint8 [nchans][nsamps]; delays: int [ndm][nchans].
    Returns int32 [ndm][nout]: one slice-add per (trial, channel)."""
    nchans, nsamps = x.shape
    delays = np.asarray(delays, dtype=np.int64)
    if nout is None:
        nout = nsamps - int(delays.max())
    if nout <= 0:
        raise ValueError("too few samples for the largest delay")
    ndm = delays.shape[0]
    out = np.zeros((ndm, nout), dtype=np.int32)
    for d in range(ndm):
        acc = out[d]
        for c in range(nchans):
            s = int(delays[d, c])
            np.add(acc, x[c, s:s + nout], out=acc, casting="unsafe")
    return out


def brute_dedisperse(x, delays, nout):
    """The same sum as three plain Python loops, for tiny inputs only."""
    nchans = len(x)
    out = []
    for d in range(len(delays)):
        row = []
        for t in range(nout):
            s = 0
            for c in range(nchans):
                s += int(x[c][t + int(delays[d][c])])
            row.append(s)
        out.append(row)
    return np.array(out, dtype=np.int64).reshape(len(delays), nout)
