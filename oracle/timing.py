"""Multi-core timing harness for the oracle (test infrastructure only).

Runs the oracle's own functions unchanged, splitting independent DM trials
over worker processes (fork; the unpacked input is shared copy-on-write).
Used only to report a CPU baseline beside the GPU measurement.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np

from .boxcar import boxcar
from .dedisperse import dedisperse
from .peaks import find_events
from .unpack import unpack_2bit

_G = {}


def _work(rows):
    x, dly, nout, widths, k = _G["x"], _G["dly"], _G["nout"], _G["widths"], _G["k"]
    out = dedisperse(x, dly[rows], nout=nout)
    ev = find_events(boxcar(out, widths), k)
    return len(rows), len(ev)


def cpu_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def time_chain(packed, nsamps, nchans, delays, rows, widths, k, procs=None):
    """Wall time of unpack (whole beam) and of dedisperse + boxcar + peaks for
    the DM trials `rows`, on `procs` processes.  Returns a dict."""
    procs = procs or cpu_cores()
    nout = nsamps - int(delays.max())
    t0 = time.perf_counter()
    x = unpack_2bit(packed, nsamps, nchans)
    t1 = time.perf_counter()
    _G.update(x=x, dly=np.asarray(delays), nout=nout, widths=list(widths), k=k)
    chunks = [list(c) for c in np.array_split(np.asarray(rows), max(1, len(rows) // 4))
              if len(c)]
    ctx = mp.get_context("fork")
    t2 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_work, chunks)
    t3 = time.perf_counter()
    _G.clear()
    return dict(unpack_s=t1 - t0, rows_s=t3 - t2, nrows=sum(r[0] for r in res),
                nevents=sum(r[1] for r in res), nout=nout, procs=procs)
