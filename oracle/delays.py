"""Dispersion delay table (oracle; test infrastructure only).

Section 2.2 of the paper: the interstellar medium delays a signal by an
amount that grows with the column of free electrons (the dispersion measure,
DM) and that depends on frequency; each DM trial therefore integrates every
channel's time series shifted by that channel's delay.  The paper prints no
formula, so the oracle takes the cold-plasma law with the standard constant

    delay[d][c] = round( K * DM_d * (f_c^-2 - f_top^-2) / tsamp ),
    K = 4.148808e3 s MHz^2 pc^-1 cm^3,  f in MHz, tsamp in s,

with these readings of what the paper leaves open:
  * channel frequencies f_c = f_top + c*df, channel 0 = f_top (highest), df<0;
  * "round" is round-half-away-from-zero on the IEEE double value;
  * evaluation order, one rounding per operation, no fused multiply-add:
        fc = f_top + c*df
        a  = 1/(fc*fc) - 1/(f_top*f_top)
        x  = ((K*DM)*a)/tsamp
  * max_delay is the single maximum over the whole table.
"""
from __future__ import annotations

import math

import numpy as np

K_DM = 4.148808e3  # s MHz^2 pc^-1 cm^3


def channel_freqs(nchans: int, f_top: float, df: float) -> np.ndarray:
    """f_c = f_top + c*df (section 1: the filterbank's channels across the band)."""
    c = np.arange(nchans, dtype=np.float64)
    return f_top + c * df


def _delay_real(nchans, f_top, df, tsamp, dm_list) -> np.ndarray:
    fc = channel_freqs(nchans, f_top, df)
    a = 1.0 / (fc * fc) - 1.0 / (f_top * f_top)
    kdm = K_DM * np.asarray(dm_list, dtype=np.float64)
    return ((kdm[:, None] * a[None, :]) / tsamp)


def delay_table(nchans: int, f_top: float, df: float, tsamp: float,
                dm_list) -> np.ndarray:
    """int64 [ndm][nchans]: the per-channel shift, in samples, that DM trial d
    applies before integrating over channels (section 2.2)."""
    x = _delay_real(nchans, f_top, df, tsamp, dm_list)
    fl = np.floor(x)
    return (fl + (x - fl >= 0.5)).astype(np.int64)


def max_delay(delays: np.ndarray) -> int:
    return int(delays.max()) if delays.size else 0


def nearest_tie_distance(nchans, f_top, df, tsamp, dm_list) -> float:
    """min over (d, c) of |frac(x) - 1/2|: how close any entry came to a
    rounding tie (a result under ~1e-9 would make the table fragile)."""
    x = _delay_real(nchans, f_top, df, tsamp, dm_list)
    return float(np.min(np.abs((x - np.floor(x)) - 0.5)))


def delay_scalar(f_top: float, df: float, tsamp: float, dm: float, c: int) -> int:
    """One entry, with plain Python floats (same operation order)."""
    fc = f_top + c * df
    a = 1.0 / (fc * fc) - 1.0 / (f_top * f_top)
    x = ((K_DM * dm) * a) / tsamp
    fl = math.floor(x)
    return int(fl + (1 if x - fl >= 0.5 else 0))
