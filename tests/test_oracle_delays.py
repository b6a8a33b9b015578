"""Pins of the oracle's delay table (section 2.2 and its stated readings)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.delays import delay_scalar
import synth


SMALL = dict(nchans=256, f_top=1581.8, df=-1.5625, tsamp=64e-6)
SURVEY = dict(nchans=1024, f_top=1581.8, df=-400.0 / 1024, tsamp=64e-6)


def exact_delay(f_top, df, tsamp, dm, c):
    """The same law in exact rational arithmetic on the double inputs,
    rounded half away from zero: an independent evaluation."""
    ft = Fraction(f_top)
    fc = ft + c * Fraction(df)
    x = Fraction(oracle.K_DM) * Fraction(dm) * (1 / (fc * fc) - 1 / (ft * ft)) / Fraction(tsamp)
    fl = x.numerator // x.denominator
    return fl + (1 if x - fl >= Fraction(1, 2) else 0), float(x - fl)


def test_max_delay_closed_form_small():
    dms = synth.dm_list_linear(100, 200.0)
    t = oracle.delay_table(dm_list=dms, **SMALL)
    # lowest channel 1581.8 - 255*1.5625 = 1183.3625 MHz at DM 200: x = 4076.763
    assert oracle.max_delay(t) == 4077
    ref, frac = exact_delay(1581.8, -1.5625, 64e-6, 200.0, 255)
    assert ref == 4077 and abs(frac - 0.763) < 1e-3


def test_max_delay_closed_form_survey():
    dms = synth.dm_list_expm1(1200, 1000.0)
    t = oracle.delay_table(dm_list=dms, **SURVEY)
    # lowest channel 1182.190625 MHz at DM 1000: x = 20475.638
    assert t.shape == (1200, 1024)
    assert oracle.max_delay(t) == 20476
    assert dms[-1] == 1000.0 and dms[0] == 0.0


def test_zero_row_and_column_and_monotone():
    dms = synth.dm_list_expm1(200, 1000.0)
    t = oracle.delay_table(dm_list=dms, **SURVEY)
    assert (t[:, 0] == 0).all()          # f_c = f_top: no delay
    assert (t[0, :] == 0).all()          # DM = 0: no delay
    assert (np.diff(t, axis=1) >= 0).all()   # lower frequency, later arrival
    assert (np.diff(t, axis=0) >= 0).all()   # larger DM, longer delay


@pytest.mark.parametrize("cfg,dms", [
    (SMALL, synth.dm_list_linear(100, 200.0)),
    (SURVEY, synth.dm_list_expm1(1200, 1000.0)[::37]),
])
def test_table_matches_exact_rational(cfg, dms):
    t = oracle.delay_table(dm_list=dms, **cfg)
    rng = np.random.default_rng(5)
    for _ in range(400):
        d = int(rng.integers(0, len(dms)))
        c = int(rng.integers(0, cfg["nchans"]))
        ref, frac = exact_delay(cfg["f_top"], cfg["df"], cfg["tsamp"], dms[d], c)
        if abs(frac - 0.5) > 1e-6:
            assert t[d, c] == ref, (d, c)


def test_table_matches_independent_sky_model():
    """The generator's sweep (other units, other operation order) lands every
    channel in the same sample except within 1e-6 of a rounding tie."""
    dms = synth.dm_list_expm1(1200, 1000.0)[::10]
    t = oracle.delay_table(dm_list=dms, **SURVEY)
    x = oracle.delays._delay_real(SURVEY["nchans"], SURVEY["f_top"], SURVEY["df"],
                                  SURVEY["tsamp"], dms)
    safe = np.abs(x - np.floor(x) - 0.5) > 1e-6
    for d, dm in enumerate(dms):
        sky = synth.sky_arrival_offsets(SURVEY["nchans"], SURVEY["f_top"], SURVEY["df"],
                                        SURVEY["tsamp"], dm)
        assert (sky[safe[d]] == t[d][safe[d]]).all()


def test_scalar_and_vector_agree():
    dms = synth.dm_list_linear(100, 200.0)
    t = oracle.delay_table(dm_list=dms, **SMALL)
    for d in (0, 1, 50, 99):
        for c in (0, 1, 128, 255):
            assert t[d, c] == delay_scalar(1581.8, -1.5625, 64e-6, dms[d], c)


def test_round_half_away_from_zero():
    """An exact .5 rounds up (C round), not to even."""
    # f_top = 1, channel 1 at 0.5 MHz: a = 1/0.25 - 1 = 3 exactly.
    for dm in np.linspace(1.0, 3.0, 2001):
        y = (oracle.K_DM * dm) * 3.0
        ts = y / 2.5
        x = y / ts
        if x == 2.5:
            t = oracle.delay_table(2, 1.0, -0.5, ts, [dm])
            assert t[0, 1] == 3
            break
    else:
        pytest.skip("no exact tie constructed")


def test_no_near_ties_in_configs():
    assert oracle.nearest_tie_distance(dm_list=synth.dm_list_linear(100, 200.0),
                                       **SMALL) > 1e-9
    assert oracle.nearest_tie_distance(dm_list=synth.dm_list_expm1(1200, 1000.0),
                                       **SURVEY) > 1e-9
