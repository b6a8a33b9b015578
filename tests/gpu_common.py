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
