"""Subband (two-stage) dedispersion (oracle; test infrastructure).

Section 2.2 calls its brute-force method the "direct" algorithm, implying
cheaper ones.  The common one is subband dedispersion: split the band into
subbands, dedisperse each subband on a coarse DM grid (the delays inside a
subband change slowly with DM), then dedisperse the subband series on the
fine grid using each subband's own arrival delay.  The result approximates
the direct sum with an effective delay per (trial, channel).  Readings (the
paper gives no parameters):

  * nsub subbands of S = nchans / nsub consecutive channels; subband s starts
    at channel c0 = s * S, its reference channel;
  * fine trials are grouped G at a time in list order (the last group may be
    shorter); group q's coarse DM is the DM of its middle trial,
    index q * G + (size_q - 1) // 2;
  * stage 1: each subband is a filterbank of its own, top frequency
    f_top + c0 * df, with the delay law and rounding of the direct plan:
        sub[s][q][t] = sum_{c' < S} x[c0 + c'][t + dsub[s][q][c']];
  * stage 2: out[d][t] = sum_s sub[s][q(d)][t + delay[d][c0(s)]], with
    delay the direct plan's table;
  * both stages keep exact integers; the output covers
        nout = nsamps - max_{d,s} (delay[d][c0(s)] + max dsub[s]),
    every position whose reads stay inside the data.
The effective delay of channel c = c0 + c' at trial d is
delay[d][c0] + dsub[s][q(d)][c'].
"""
from __future__ import annotations

import numpy as np

from .delays import delay_table
from .dedisperse import dedisperse


def groups(ndm: int, group: int):
    """(q [ndm]: coarse index of each trial, mid [ncoarse]: its middle trial)."""
    q = np.arange(ndm) // group
    ncoarse = int(q[-1]) + 1
    mid = np.array([g * group + (min(group, ndm - g * group) - 1) // 2 for g in range(ncoarse)],
                   dtype=np.int64)
    return q, mid


def subband_plan(nchans: int, f_top: float, df: float, tsamp: float, dm_list, nsub: int,
                 group: int):
    """Returns (q, coarse_dms, dsub [nsub][ncoarse][S], inter [ndm][nsub], nout_loss)
    where nout_loss = nsamps - nout."""
    if nchans % nsub:
        raise ValueError("nsub must divide nchans")
    S = nchans // nsub
    dm = np.asarray(dm_list, dtype=np.float64)
    full = delay_table(nchans, f_top, df, tsamp, dm)
    q, mid = groups(len(dm), group)
    coarse = dm[mid]
    dsub = np.stack([delay_table(S, f_top + (s * S) * df, df, tsamp, coarse) for s in range(nsub)])
    inter = full[:, ::S].astype(np.int64)                      # delay[d][c0(s)]
    loss = int((inter + dsub.reshape(nsub, -1).max(axis=1)[None, :]).max())
    return q, coarse, dsub.astype(np.int64), inter, loss


def effective_delays(nchans, f_top, df, tsamp, dm_list, nsub, group) -> np.ndarray:
    """[ndm][nchans] delay that the two stages apply to each channel."""
    q, _, dsub, inter, _ = subband_plan(nchans, f_top, df, tsamp, dm_list, nsub, group)
    S = nchans // nsub
    eff = np.empty((len(q), nchans), dtype=np.int64)
    for s in range(nsub):
        eff[:, s * S:(s + 1) * S] = inter[:, s:s + 1] + dsub[s][q]
    return eff


def subband_dedisperse(x: np.ndarray, f_top: float, df: float, tsamp: float, dm_list, nsub: int,
                       group: int) -> np.ndarray:
    """x: [nchans][nsamps] levels.  Returns out [ndm][nout] (int64)."""
    nchans, nsamps = x.shape
    q, _, dsub, inter, loss = subband_plan(nchans, f_top, df, tsamp, dm_list, nsub, group)
    S = nchans // nsub
    nout = nsamps - loss
    if nout < 1:
        raise ValueError("too few samples for the plan")
    out = np.zeros((len(q), nout), dtype=np.int64)
    for s in range(nsub):
        sub = dedisperse(x[s * S:(s + 1) * S], dsub[s])        # stage 1: [ncoarse][nsamps - max]
        for d in range(len(q)):                                  # stage 2
            a = int(inter[d, s])
            out[d] += sub[q[d], a:a + nout]
    return out
