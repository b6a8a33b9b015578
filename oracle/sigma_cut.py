"""Sigma-cut on boxcar series, decided exactly (oracle; test infrastructure).

Section 2.3 of the paper: peak finding first applies a sigma-cut to each
reduced time series.  The paper does not say how the mean and sigma are
estimated; the reading taken is the population mean and standard deviation
of the series itself (over its n = n_bx samples), from exact integer sums

    S1 = sum B,   S2 = sum B^2,   D = n*S2 - S1^2   (so sigma = sqrt(D)/n),

and for a sample B the statistic L = n*B - S1, giving S/N = L / sqrt(D).
"S/N > k" is strict and is decided without rounding: with k a binary
fraction (any float), L > k*sqrt(D) <=> L >= isqrt(floor(k^2 * D)) + 1, i.e.

    B >= B_thr = ceil( (S1 + isqrt(floor(k^2 D)) + 1) / n ).

A series with D = 0 (constant) has no events.  The reported S/N is
float32( double(L) / sqrt(double(D)) ).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def series_stats(b: np.ndarray):
    """(n, S1, S2) of one series as Python ints (exact)."""
    b = np.asarray(b, dtype=np.int64)
    n = int(b.size)
    s1 = int(b.sum(dtype=np.int64))
    m = int(np.abs(b).max()) if n else 0
    if n * m * m < (1 << 62):          # the int64 sum cannot overflow
        s2 = int((b * b).sum(dtype=np.int64))
    else:
        s2 = sum(int(v) * int(v) for v in b.tolist())
    return n, s1, s2


def exact_k(k: float) -> Fraction:
    """The threshold as the exact binary fraction of its float32 value."""
    k32 = float(np.float32(k))
    if not math.isfinite(k32) or k32 <= 0.0:
        raise ValueError("S/N threshold must be a positive finite number")
    return Fraction(k32)


def threshold_level(n: int, s1: int, s2: int, k: float):
    """Smallest integer B with S/N(B) > k, or None when D == 0."""
    d = n * s2 - s1 * s1
    if d < 0:
        raise AssertionError("negative variance: sums are inconsistent")
    if d == 0:
        return None
    kk = exact_k(k)
    q = kk * kk * d                      # exact rational k^2 * D
    lmin = math.isqrt(q.numerator // q.denominator) + 1
    num = s1 + lmin
    return -((-num) // n)               # ceil(num / n)


def is_event(b: int, n: int, s1: int, s2: int, k: float) -> bool:
    """The event test written directly: L > 0 and L^2 > k^2 D (exact)."""
    d = n * s2 - s1 * s1
    if d == 0:
        return False
    lval = n * int(b) - s1
    kk = exact_k(k)
    return lval > 0 and Fraction(lval * lval) > kk * kk * d


def snr_value(b: int, n: int, s1: int, s2: int) -> np.float32:
    d = n * s2 - s1 * s1
    lval = n * int(b) - s1
    return np.float32(float(lval) / math.sqrt(float(d)))
