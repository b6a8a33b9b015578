"""Candidate selection for triage: per-width non-maximum suppression
(oracle; test infrastructure).

The paper's search ends with events (section 2.3) and names interference as
what swamps them with false positives (section 2.1); the triage network that
scores candidates is an addition to the method, and so is the rule that
picks the candidates it scores.  Reading taken:

  * events of different boxcar widths never suppress each other;
  * within a width w, events are visited from the highest S/N down (ties:
    lower DM index first, then earlier t_peak, then lower list index);
  * an event is kept unless an already kept event of the same width lies
    within 32 trials and 128 w samples of it, both strictly:
    |dm_a - dm_b| < 32 and |t_peak_a - t_peak_b| < 128 w (the 64-trial by
    256 w-sample tile of a candidate, centred);
  * the kept events are returned as their indices into the list, ascending.

Written out as the greedy definition with every kept event tested: O(n k).
"""
from __future__ import annotations

import numpy as np

DM_HALF = 32
T_HALF_PER_WIDTH = 128


def nms(events, widths, dm_half: int = DM_HALF, t_half_per_width: int = T_HALF_PER_WIDTH):
    """events: structured array (EVENT_FIELDS layout) or list of tuples
    (width_idx, dm_idx, t_start, t_end, t_peak, b_peak, snr).  Returns the
    ascending indices of the kept events."""
    if isinstance(events, np.ndarray) and events.dtype.names:
        rows = [(int(e["width_idx"]), int(e["dm_idx"]), int(e["t_peak"]), float(e["snr"]))
                for e in events]
    else:
        rows = [(int(e[0]), int(e[1]), int(e[4]), float(np.float32(e[6]))) for e in events]
    keep = []
    for wi in sorted({r[0] for r in rows}):
        w = int(widths[wi])
        idx = [i for i, r in enumerate(rows) if r[0] == wi]
        idx.sort(key=lambda i: (-rows[i][3], rows[i][1], rows[i][2], i))
        kept = []
        for i in idx:
            d, t = rows[i][1], rows[i][2]
            if any(abs(d - rows[j][1]) < dm_half and abs(t - rows[j][2]) < t_half_per_width * w
                   for j in kept):
                continue
            kept.append(i)
        keep.extend(kept)
    return sorted(keep)
