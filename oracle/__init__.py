"""CPU oracle for the transient-search hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct restatement of what the path computes, used
to prove the HIP library right.  Only the test suite, the package smoke check
and the CPU-baseline leg of the benchmark may import it; the product path
never does, and this package shares no code with the HIP library.

Every function cites the passage of the paper it follows.  Where the paper is
silent (it prints no delay formula, bit layout, rounding, S/N estimator or
event definition) the oracle takes one stated reading, recorded in each
module's docstring.  All integer results are exact; floating point is IEEE
double unless noted.

Parity pins: every function here is pinned by the CPU tests against closed
forms, invariants, brute force or hand-built fixtures; none is pinned only by
re-running itself.
"""
from .delays import (K_DM, channel_freqs, delay_table, max_delay,
                     nearest_tie_distance)
from .unpack import unpack_2bit
from .dedisperse import dedisperse, brute_dedisperse
from .boxcar import prefix_sum, boxcar, n_boxcar
from .sigma_cut import (series_stats, threshold_level, snr_value, exact_k,
                        is_event)
from .peaks import find_runs, find_events, EVENT_FIELDS
from .pipeline import search
from .coincidence import zero_dm_series, rfi_mask, binomial_tail, replace_masked
from .baseline import baseline_remove
from .cluster import cluster_events, CLUSTER_FIELDS
from .subband import subband_dedisperse, subband_plan, effective_delays
from .nms import nms

__all__ = [
    "baseline_remove", "cluster_events", "CLUSTER_FIELDS", "nms",
    "subband_dedisperse", "subband_plan", "effective_delays",
    "zero_dm_series", "rfi_mask", "binomial_tail", "replace_masked",
    "K_DM", "channel_freqs", "delay_table", "max_delay", "nearest_tie_distance",
    "unpack_2bit", "dedisperse", "brute_dedisperse", "prefix_sum", "boxcar",
    "n_boxcar", "series_stats", "threshold_level", "snr_value", "exact_k",
    "is_event", "find_runs", "find_events", "EVENT_FIELDS", "search",
]
