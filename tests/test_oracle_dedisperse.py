"""Pins of the oracle's unpacking and dedispersion (sections 1 and 2.2)."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.unpack import bytes_per_second
import synth
from conftest import GOLDEN


def test_unpack_golden_layout():
    g = json.load(open(os.path.join(GOLDEN, "layout_2bit.json")))
    packed = np.array([int(b, 2) for b in g["bytes_binary"]], dtype=np.uint8)
    x = oracle.unpack_2bit(packed, g["nsamps"], g["nchans"])
    assert x.tolist() == g["levels_c_by_t"]


def test_paper_data_rate():
    # Section 1 puts the 2-bit data rate of one beam at about 4 MB/s (1024 ch, 64 us).
    assert bytes_per_second(1024, 64e-6) == pytest.approx(4.0e6, rel=1e-12)


def test_unpack_roundtrip_generator():
    rng = np.random.default_rng(0)
    q = rng.integers(0, 4, size=(37, 16), dtype=np.uint8)
    x = oracle.unpack_2bit(synth.pack_2bit(q), 37, 16)
    assert (x == q.T).all()


def _rand(nchans, nsamps, seed, hi=4):
    return np.random.default_rng(seed).integers(0, hi, size=(nchans, nsamps), dtype=np.uint8)


@pytest.mark.parametrize("nchans,nsamps,ndm,seed", [(4, 40, 3, 1), (8, 120, 6, 2),
                                                    (12, 160, 5, 3), (4, 9, 1, 4)])
def test_brute_force_tiny(nchans, nsamps, ndm, seed):
    rng = np.random.default_rng(seed)
    x = _rand(nchans, nsamps, seed)
    dly = np.sort(rng.integers(0, nsamps // 3, size=(ndm, nchans)), axis=1)
    nout = nsamps - int(dly.max())
    ref = oracle.brute_dedisperse(x.tolist(), dly.tolist(), nout)
    got = oracle.dedisperse(x, dly)
    assert got.shape == (ndm, nout)
    assert (got == ref).all()


def test_dm_zero_is_channel_sum():
    x = _rand(64, 2500, 7)
    dly = oracle.delay_table(64, 1581.8, -6.25, 64e-6, [0.0, 50.0])
    out = oracle.dedisperse(x, dly)
    nout = out.shape[1]
    assert (out[0] == x[:, :nout].astype(np.int64).sum(axis=0)).all()


def test_dispersed_delta_full_sum():
    nchans, nsamps = 64, 9000
    dms = np.linspace(0, 300, 13)
    dly = oracle.delay_table(nchans, 1581.8, -6.25, 64e-6, dms)
    nout = nsamps - int(dly.max())
    d_star, t0 = 7, 123
    x = np.zeros((nchans, nsamps), dtype=np.uint8)
    x[np.arange(nchans), t0 + dly[d_star]] = 1
    out = oracle.dedisperse(x, dly)
    assert out[d_star, t0] == nchans
    assert out.max() == nchans
    assert (out[d_star] == nchans).sum() == 1
    # neighbouring trials collect strictly less of the sweep
    assert out[d_star - 1].max() < nchans and out[d_star + 1].max() < nchans


def test_linearity_shift_conservation():
    nchans, nsamps = 32, 2000
    dms = np.linspace(0, 100, 9)
    dly = oracle.delay_table(nchans, 1500.0, -10.0, 64e-6, dms)
    a = _rand(nchans, nsamps, 11, hi=2)
    b = _rand(nchans, nsamps, 12, hi=2)
    oa, ob, oab = (oracle.dedisperse(v, dly) for v in (a, b, a + b))
    assert (oab == oa + ob).all()
    # time-shift equivariance: dropping s leading samples shifts the output
    s = 17
    osh = oracle.dedisperse(a[:, s:], dly)
    assert (osh == oa[:, s:]).all()
    # conservation: each trial's total equals the sum of the windows it reads
    nout = oa.shape[1]
    for d in range(len(dms)):
        tot = sum(int(a[c, dly[d, c]:dly[d, c] + nout].sum()) for c in range(nchans))
        assert int(oa[d].sum()) == tot


def test_noise_statistics_small_config():
    fb = synth.make_small(1)
    x = oracle.unpack_2bit(fb.packed, fb.nsamps, fb.nchans)
    # 2-bit quantiser of N(0,1) at +-0.98, 0: mean 1.5, variance 0.904172
    assert x.mean() == pytest.approx(1.5, abs=2e-3)
    assert x.var() == pytest.approx(0.904172, abs=5e-3)
    dly = oracle.delay_table(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list[:3])
    out = oracle.dedisperse(x, dly, nout=fb.nsamps - 4077)
    # channel sums of 256 levels: 384 +- 15.21 (pulses add a little)
    assert out.mean() == pytest.approx(384.0, abs=0.5)
    assert out.std() == pytest.approx(15.21, rel=0.05)


def test_too_few_samples():
    x = _rand(4, 10, 1)
    with pytest.raises(ValueError):
        oracle.dedisperse(x, np.array([[0, 3, 6, 10]]))
