"""Multibeam coincidence RFI mask (oracle; test infrastructure only).

Section 2.1 of the paper: interference is not localised on the sky, so the 13
beams of the multibeam receiver serve as reference antennas for one another.
The method is a transform of the multibeam time series: each sample of the 13
beams is tested against a signal-to-noise threshold, and the sample is
flagged as interference (a boolean mask) when enough beams exceed it.  The
paper's example threshold is 3 sigma in 4 or more beams, for which it bounds
the chance of flagging a noise sample by C(13, 4) * 0.01^4.

Readings (the paper leaves them open):
  * the series of a beam is its zero-DM series z_b[t] = sum_c x_b[c][t] over
    the samples all beams cover;
  * mean and sigma are the population statistics of z_b over those samples;
  * exceeding k sigma means the strict S/N > k of the sigma-cut, decided
    exactly with the same integer threshold (sigma_cut.threshold_level); a
    constant series never exceeds.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

from .sigma_cut import series_stats, threshold_level
from .unpack import unpack_2bit


def zero_dm_series(packed: np.ndarray, nsamps: int, nchans: int) -> np.ndarray:
    """z[t] = sum over channels of the 2-bit levels of sample t (int64)."""
    return unpack_2bit(packed, nsamps, nchans).sum(axis=0, dtype=np.int64)


def beam_threshold(z: np.ndarray, k: float):
    """Smallest z that exceeds k sigma in this beam, or None (constant beam)."""
    n, s1, s2 = series_stats(z)
    return threshold_level(n, s1, s2, k)


def rfi_mask(series: Sequence[np.ndarray], k: float, min_beams: int):
    """(mask bool[n], votes int[n], thresholds) for equal-length beam series."""
    thr = [beam_threshold(z, k) for z in series]
    votes = np.zeros(len(series[0]), dtype=np.int64)
    for z, t in zip(series, thr):
        if t is not None:
            votes += (np.asarray(z) >= t)
    return votes >= min_beams, votes, thr


def binomial_tail(nbeams: int, p: float, m: int) -> float:
    """P(at least m of nbeams independent beams exceed), each with chance p."""
    return sum(math.comb(nbeams, j) * p ** j * (1.0 - p) ** (nbeams - j)
               for j in range(m, nbeams + 1))


def replace_masked(x: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Apply the mask to one beam's levels x[c][t] (reading: a flagged sample
    is replaced by the mean level in every channel).  The 2-bit quantiser is
    symmetric, so its mean level is 1.5; even channels get level 1 and odd
    channels level 2, which keeps every sample's channel sum at exactly
    1.5 * nchans.  Returns a new array."""
    y = np.array(x, dtype=np.uint8, copy=True)
    m = np.asarray(mask, dtype=bool)
    fill = np.where(np.arange(y.shape[0]) % 2 == 0, 1, 2).astype(np.uint8)
    y[:, m] = fill[:, None]
    return y
