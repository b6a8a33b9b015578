"""Pins of the multibeam coincidence mask oracle (section 2.1)."""
import itertools
import json
import math
import os

import numpy as np

import oracle
import synth
from conftest import GOLDEN


def test_false_flag_probability_matches_the_papers_bound():
    """Brute force over all 2^13 beam subsets equals the binomial tail, which
    stays under the paper's bound C(13,4) * 0.01^4 = 7.15e-6."""
    p, n, m = 0.01, 13, 4
    brute = 0.0
    for bits in itertools.product((0, 1), repeat=n):
        k = sum(bits)
        if k >= m:
            brute += p ** k * (1 - p) ** (n - k)
    assert math.isclose(oracle.binomial_tail(n, p, m), brute, rel_tol=1e-12)
    assert math.comb(13, 4) == 715 and math.isclose(715 * 0.01 ** 4, 7.15e-6)
    assert brute <= 7.15e-6 and math.isclose(brute, 6.652e-6, rel_tol=1e-3)


def test_hand_built_thresholds_and_votes():
    # z = [0]*7 + [8]: S1 = 8, S2 = 64, D = 8*64 - 64 = 448.  The spike's S/N
    # is (8*8 - 8)/sqrt(448) = 2.6458: it exceeds k = 1, 2, 2.5, 2.6 and not
    # 2.65; worked by hand: k = 1 -> isqrt(448) = 21, ceil(30/8) = 4;
    # k = 2 -> isqrt(1792) = 42, ceil(51/8) = 7; k = 2.65 -> isqrt(3146) = 56,
    # ceil(65/8) = 9.
    z = np.array([0] * 7 + [8])
    assert oracle.coincidence.beam_threshold(z, 1.0) == 4
    assert oracle.coincidence.beam_threshold(z, 2.0) == 7
    for k, exceeds in [(1.0, True), (2.0, True), (2.5, True), (2.6, True), (2.65, False)]:
        assert (8 >= oracle.coincidence.beam_threshold(z, k)) == exceeds, k
    other = np.array([3, 1, 4, 1, 5, 9, 2, 6])
    flat = np.full(8, 5)                      # D = 0: never exceeds
    beams = [z, z, z, z, other, flat]
    mask, votes, thr = oracle.rfi_mask(beams, 1.0, 4)
    assert thr[5] is None
    # beam 4 (values 3 1 4 1 5 9 2 6: S1 = 31, S2 = 173, D = 423, k = 1:
    # isqrt(423) = 20, ceil(52/8) = 7) votes at t = 5 only
    assert thr[4] == 7
    assert votes.tolist() == [0, 0, 0, 0, 0, 1, 0, 4]
    assert mask[7] and not mask[:7].any()
    assert not oracle.rfi_mask(beams, 1.0, 6)[0].any()


def test_zero_dm_series_is_the_channel_sum():
    rng = np.random.default_rng(4)
    q = rng.integers(0, 4, size=(300, 32), dtype=np.uint8)     # [t][c]
    packed = synth.pack_2bit(q)
    z = oracle.zero_dm_series(packed, 300, 32)
    assert (z == q.sum(axis=1)).all()
    # and equals dedispersion at zero delay
    out = oracle.dedisperse(oracle.unpack_2bit(packed, 300, 32), np.zeros((1, 32), np.int64))
    assert (out[0] == z).all()
    with open(os.path.join(GOLDEN, "layout_2bit.json")) as f:
        fx = json.load(f)
    packed_fx = np.array([int(b, 2) for b in fx["bytes_binary"]], np.uint8)
    zz = oracle.zero_dm_series(packed_fx, fx["nsamps"], fx["nchans"])
    assert (zz == np.array(fx["levels_c_by_t"]).sum(axis=0)).all()


def test_mask_rate_of_independent_beams_is_the_binomial_tail():
    """13 independent integer Gaussian beams, k = 1, at least 4 beams: the
    masked fraction matches the Poisson-binomial tail of the beams' own
    exceed rates within 5 standard errors."""
    rng = np.random.default_rng(9)
    n = 100_000
    beams = [np.rint(1000 * rng.standard_normal(n)).astype(np.int64) + 5000 for _ in range(13)]
    mask, votes, thr = oracle.rfi_mask(beams, 1.0, 4)
    ps = [float((b >= t).mean()) for b, t in zip(beams, thr)]
    # Poisson-binomial distribution of the vote count by convolution
    dist = np.array([1.0])
    for p in ps:
        dist = np.convolve(dist, [1 - p, p])
    tail = dist[4:].sum()
    se = math.sqrt(tail * (1 - tail) / n)
    assert abs(mask.mean() - tail) < 5 * se, (mask.mean(), tail)
    assert all(abs(p - 0.1587) < 0.01 for p in ps)


def test_common_impulses_are_masked_and_nothing_else():
    packed, imps, amps, _ = synth.make_coincidence_beams(5, nbeams=13, nsamps=1 << 14, nchans=64)
    zs = [oracle.zero_dm_series(p, 1 << 14, 64) for p in packed]
    mask, votes, thr = oracle.rfi_mask(zs, 3.0, 4)
    inside = np.zeros(1 << 14, bool)
    for im in imps:
        inside[im.t:im.t + im.width] = True
    assert mask.any() and not (mask & ~inside).any()
    # single-beam signals (the dispersed pulses) never reach 4 beams
    assert (votes[~inside] < 4).all()


def test_replacement_keeps_the_mean_level_exactly():
    rng = np.random.default_rng(21)
    x = rng.integers(0, 4, size=(12, 50), dtype=np.uint8)
    mask = np.zeros(50, bool)
    mask[[0, 7, 8, 49]] = True
    y = oracle.replace_masked(x, mask)
    assert (y[:, ~mask] == x[:, ~mask]).all()
    assert (y[:, mask] == np.array([1, 2] * 6, np.uint8)[:, None]).all()
    assert (y[:, mask].sum(axis=0) == 18).all()          # 1.5 * 12 channels
    # 1.5 is the quantiser's mean level: its edges are symmetric about 0
    q = synth.quantise(np.random.default_rng(3).standard_normal(400000))
    assert abs(q.mean() - 1.5) < 0.005
    lo, mid, hi = synth.QUANT_EDGES
    assert lo == -hi and mid == 0.0


def test_applied_mask_removes_common_impulses_and_keeps_pulses():
    """64 channels, 13 beams with common zero-DM impulses: after the mask is
    applied no sample is flagged again, the low-DM events of the impulses
    are gone, and the dispersed pulse of beam 0 keeps >= 90% of its S/N at
    its trial (masked impulse samples inside its sweep cost a little)."""
    nsamps, nchans = 1 << 14, 64
    beams, imps, amps, pulses = synth.make_coincidence_beams(5, nsamps=nsamps, nchans=nchans,
                                                             npulses=1, impulse_rate=30.0,
                                                             dm_max=60.0)
    assert len(imps) >= 10
    z = [oracle.zero_dm_series(b, nsamps, nchans) for b in beams]
    mask, votes, thr = oracle.rfi_mask(z, 3.0, 4)
    assert mask.sum() > 0
    x0 = oracle.unpack_2bit(beams[0], nsamps, nchans)
    y0 = oracle.replace_masked(x0, mask)
    ys = [oracle.replace_masked(oracle.unpack_2bit(b, nsamps, nchans), mask) for b in beams]
    z2 = [y.sum(axis=0, dtype=np.int64) for y in ys]
    mask2, _, _ = oracle.rfi_mask(z2, 3.0, 4)
    assert not (mask2 & mask).any()
    dms = np.linspace(0.0, 60.0, 31)
    dly = oracle.delay_table(nchans, synth.F_TOP, -400.0 / nchans, synth.TSAMP, dms)
    widths = [1, 2, 4, 8]
    ev_before = oracle.find_events(oracle.boxcar(oracle.dedisperse(x0, dly), widths), 6.0)
    ev_after = oracle.find_events(oracle.boxcar(oracle.dedisperse(y0, dly), widths), 6.0)
    near_imp = lambda ev: sum(1 for e in ev if e[1] <= 1 and
                              any(abs(e[4] - im.t) <= 8 for im in imps))
    assert near_imp(ev_before) > 0 and near_imp(ev_after) == 0
    p = pulses[0][0]
    d = int(np.argmin(np.abs(dms - p.dm)))
    wi = max(i for i, w in enumerate(widths) if w <= p.width)

    def snr(x):
        b = oracle.boxcar(oracle.dedisperse(x, dly[d:d + 1]), widths)[wi, 0]
        return (b[p.t0 - 16:p.t0 + p.width + 16].max() - b.mean()) / b.std()
    before, after = snr(x0), snr(y0)
    assert before > 5.0 and after >= 0.9 * before, (before, after)
