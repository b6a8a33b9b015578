"""Shared helpers of the GPU parity tests (inputs, oracle results, devices)."""
import functools
import sys

import numpy as np

import oracle
import synth


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def to_dev(arr: np.ndarray):
    torch = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(arr)).to("cuda")


@functools.lru_cache(maxsize=None)
def small_case():
    fb = synth.make_small(1)
    dly = oracle.delay_table(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    x = oracle.unpack_2bit(fb.packed, fb.nsamps, fb.nchans)
    out = oracle.dedisperse(x, dly)
    return fb, dly, x, out


@functools.lru_cache(maxsize=None)
def small_search():
    fb, dly, x, out = small_case()
    bw = oracle.boxcar(out, fb.widths)
    ev = oracle.find_events(bw, fb.snr_thresh)
    return bw, ev


@functools.lru_cache(maxsize=None)
def survey_case():
    return synth.make_survey_beam(2)


def events_equal(gpu_ev, ref_ev, rel=1e-5):
    """Integer fields bit-exact, S/N within `rel`."""
    assert len(gpu_ev) == len(ref_ev), (len(gpu_ev), len(ref_ev))
    for g, r in zip(gpu_ev, ref_ev):
        gi = (int(g["width_idx"]), int(g["dm_idx"]), int(g["t_start"]), int(g["t_end"]),
              int(g["t_peak"]), int(g["b_peak"]))
        assert gi == tuple(int(v) for v in r[:6]), (gi, r)
        assert abs(float(g["snr"]) - float(r[6])) <= rel * abs(float(r[6])) + 1e-12, (g, r)


# ---------------------------------------------------------------------------
# The oracle over every DM row of a large block, in forked worker processes
# (the unpacked input and the GPU's results, copied to the host beforehand,
# are shared copy-on-write).  Used for whole-output parity at full size.
# ---------------------------------------------------------------------------

_PAR = {}


def _par_rows(rows):
    from oracle.peaks import series_events
    x, dly, nout = _PAR["x"], _PAR["dly"], _PAR["nout"]
    ref = oracle.dedisperse(x, dly[rows], nout=nout)
    bad = []
    for got in _PAR["got"]:
        bad.append(int((got[rows].astype(np.int64) != ref).sum()))
    ev = {}
    widths = _PAR["widths"]
    if widths:
        bw = oracle.boxcar(ref, widths)
        for wi in range(len(widths)):
            for j, d in enumerate(rows):
                ev[(wi, d)] = series_events(bw[wi, j], _PAR["k"], wi, d)
    return bad, ev


def oracle_all_rows(x, dly, nout, got_arrays, widths=None, k=None, rows_per_task=2):
    """Dedisperse every row of `dly` with the oracle (forked workers, one per
    core up to 16) and compare it with each host array in `got_arrays`
    ([ndm][nout], any integer type).  Returns (mismatching elements per
    array, the oracle's events of all rows in (width, DM, t_start) order, or
    None without widths)."""
    import multiprocessing as mp
    import os
    ndm = dly.shape[0]
    try:
        procs = len(os.sched_getaffinity(0))
    except AttributeError:
        procs = os.cpu_count() or 1
    procs = max(1, min(procs, 16))
    _PAR.update(x=x, dly=np.asarray(dly), nout=int(nout), got=list(got_arrays),
                widths=list(widths) if widths else None, k=k)
    tasks = [list(range(r, min(r + rows_per_task, ndm))) for r in range(0, ndm, rows_per_task)]
    try:
        with mp.get_context("fork").Pool(procs) as pool:
            res = pool.map(_par_rows, tasks, chunksize=1)
    finally:
        _PAR.clear()
    bad = [sum(r[0][i] for r in res) for i in range(len(got_arrays))]
    if not widths:
        return bad, None
    allev = {}
    for _, ev in res:
        allev.update(ev)
    events = [e for wi in range(len(widths)) for d in range(ndm) for e in allev[(wi, d)]]
    return bad, events
