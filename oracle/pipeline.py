"""The search chain end to end (oracle; test infrastructure).

Section 2 of the paper lists the detection stages; the ones restated here are
dedispersion (section 2.2), boxcar matched filtering and peak finding
(section 2.3), run in that order on one beam of packed 2-bit data.
"""
from __future__ import annotations

import numpy as np

from .delays import delay_table
from .unpack import unpack_2bit
from .dedisperse import dedisperse
from .boxcar import boxcar
from .peaks import find_events


def search(packed: np.ndarray, nsamps: int, nchans: int, f_top: float, df: float,
           tsamp: float, dm_list, widths, k: float):
    """Returns (delays, out, events)."""
    delays = delay_table(nchans, f_top, df, tsamp, dm_list)
    x = unpack_2bit(packed, nsamps, nchans)
    out = dedisperse(x, delays)
    bw = boxcar(out, widths)
    return delays, out, find_events(bw, k)
