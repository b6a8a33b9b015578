"""Pins of the subband (two-stage) dedispersion oracle: its exact reductions
to direct dedispersion, a brute-force check of the two-stage sum, the closed
form of its delay error, and recovery of injected pulses."""
import numpy as np
import pytest

import oracle
from oracle.subband import effective_delays, subband_dedisperse, subband_plan
import synth


def _tiny(seed, nchans, nsamps):
    return np.random.default_rng(seed).integers(0, 4, size=(nchans, nsamps), dtype=np.uint8)


DMS = np.linspace(0.0, 100.0, 23)
NCH, FTOP, DF, TS = 32, 1581.8, -12.5, 64e-6


def test_one_channel_subbands_are_direct():
    x = _tiny(1, NCH, 3000)
    full = oracle.delay_table(NCH, FTOP, DF, TS, DMS)
    for g in (1, 4, 23):
        out = subband_dedisperse(x, FTOP, DF, TS, DMS, NCH, g)
        assert out.shape == (23, 3000 - int(full.max()))
        assert (out == oracle.dedisperse(x, full)).all(), g


def test_one_subband_one_trial_per_group_is_direct():
    x = _tiny(2, NCH, 3000)
    full = oracle.delay_table(NCH, FTOP, DF, TS, DMS)
    out = subband_dedisperse(x, FTOP, DF, TS, DMS, 1, 1)
    assert (out == oracle.dedisperse(x, full)).all()


def test_two_stages_equal_the_effective_delay_sum_brute_force():
    x = _tiny(3, 16, 700)
    dms = np.linspace(0.0, 60.0, 9)
    for nsub, g in ((4, 2), (2, 3), (8, 9), (16, 4)):
        out = subband_dedisperse(x, FTOP, DF, TS, dms, nsub, g)
        eff = effective_delays(16, FTOP, DF, TS, dms, nsub, g)
        assert out.shape[1] <= 700 - int(eff.max())
        ref = oracle.brute_dedisperse(x.tolist(), eff.tolist(), out.shape[1])
        assert (out == ref).all(), (nsub, g)


def test_delay_error_closed_form():
    """eff - delay comes only from using the group's DM inside a subband:
    |eff - delay| <= K |DM_q - DM_d| |f_c^-2 - f_c0^-2| / tsamp + 1.5 (three
    roundings), and at most 1 where the trial is its group's middle one."""
    dms = synth.dm_list_expm1(1200, 1000.0)
    nch, ftop, df, ts = 1024, synth.F_TOP, synth.DF_SURVEY, synth.TSAMP
    full = oracle.delay_table(nch, ftop, df, ts, dms)
    for nsub, g in ((32, 8), (16, 5)):
        q, coarse, _, _, _ = subband_plan(nch, ftop, df, ts, dms, nsub, g)
        eff = effective_delays(nch, ftop, df, ts, dms, nsub, g)
        S = nch // nsub
        f = ftop + np.arange(nch) * df
        f0 = f[(np.arange(nch) // S) * S]
        bound = oracle.K_DM * np.abs(coarse[q][:, None] - dms[:, None]) * \
            np.abs(f[None, :] ** -2 - f0[None, :] ** -2) / ts + 1.5 + 1e-6
        err = np.abs(eff - full)
        assert (err <= bound).all(), (nsub, g)
        on_grid = coarse[q] == dms
        assert on_grid.sum() >= 1200 // g and (err[on_grid] <= 1).all()
        assert err.max() > 1        # the approximation is real


def test_plan_shapes_and_bad_arguments():
    q, coarse, dsub, inter, loss = subband_plan(NCH, FTOP, DF, TS, DMS, 4, 5)
    assert q.tolist() == [i // 5 for i in range(23)] and len(coarse) == 5
    assert coarse.tolist() == DMS[[2, 7, 12, 17, 21]].tolist()   # last group of 3: middle index 21
    assert dsub.shape == (4, 5, 8) and inter.shape == (23, 4)
    assert (dsub[:, :, 0] == 0).all() and (inter[:, 0] == 0).all()
    with pytest.raises(ValueError):
        subband_plan(NCH, FTOP, DF, TS, DMS, 5, 2)


def test_small_config_pulses_keep_their_peak():
    """32 subbands of 8 channels, groups of 2 trials (delay error at most 3
    samples): every injected pulse of the small beam still peaks within a
    trial of its own, at >= 85% of the direct peak (the narrowest, width 4,
    keeps 88%; coarser plans smear it more, 16 x 4 keeps 68%)."""
    fb = synth.make_small(1)
    dly = oracle.delay_table(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    x = oracle.unpack_2bit(fb.packed, fb.nsamps, fb.nchans)
    direct = oracle.dedisperse(x, dly)
    sb = subband_dedisperse(x, fb.f_top, fb.df, fb.tsamp, fb.dm_list, 32, 2)
    n = min(direct.shape[1], sb.shape[1])
    bw_d = oracle.boxcar(direct[:, :n], fb.widths)
    bw_s = oracle.boxcar(sb[:, :n], fb.widths)
    mean_d, mean_s = bw_d.mean(axis=2, keepdims=True), bw_s.mean(axis=2, keepdims=True)
    for p in fb.pulses:
        wi = max(i for i, w in enumerate(fb.widths) if w <= p.width)
        lo, hi = p.t0 - 8, p.t0 + p.width + 8
        pk_d = (bw_d[wi, :, lo:hi] - mean_d[wi]).max()
        win = bw_s[wi, :, lo:hi] - mean_s[wi]
        d_best = int(np.unravel_index(int(np.argmax(win)), win.shape)[0])
        assert abs(d_best - p.dm_idx) <= 1
        assert win.max() >= 0.85 * pk_d, (p, win.max(), pk_d)
