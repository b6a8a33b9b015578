"""2-bit filterbank unpacking (oracle; test infrastructure only).

Section 1 of the paper: the backend writes filterbank data -- one time series
per frequency channel -- with 2 bits per sample, about 4 MB/s per beam for
1024 channels every 64 us (1024 * 2 / 8 / 64e-6 = 4.000e6 B/s).  The bit
layout is not given; the reading taken is the recorder's time-major order:
nchans/4 bytes per time sample, channel c in bits [2(c%4), 2(c%4)+1] of byte
t*nchans/4 + c/4, an unsigned level 0..3.
"""
from __future__ import annotations

import numpy as np


def unpack_2bit(packed: np.ndarray, nsamps: int, nchans: int) -> np.ndarray:
    """Return x[c][t] (uint8, 0..3), channel-major."""
    if nchans % 4:
        raise ValueError("nchans must be a multiple of 4")
    b = np.asarray(packed, dtype=np.uint8).reshape(nsamps, nchans // 4)
    x = np.empty((nchans, nsamps), dtype=np.uint8)
    for c in range(nchans):
        x[c] = (b[:, c // 4] >> (2 * (c % 4))) & 3
    return x


def bytes_per_second(nchans: int, tsamp: float, bits: int = 2) -> float:
    """Data rate of one beam: nchans * bits / 8 per sample interval."""
    return nchans * bits / 8.0 / tsamp
