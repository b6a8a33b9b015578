"""GPU parity of the plan, the 2-bit ingest and the dedispersion kernel
(section 2.2) against the oracle, through the C ABI.  Bit-exact."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import log, small_case, survey_case, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def _plan(fb_or_args):
    from paper_1112_0065_amd import _lib as L
    return L.dedisp_plan_create(*fb_or_args)


def test_delay_tables_equal_oracle():
    from paper_1112_0065_amd import _lib as L
    for nchans, ft, df, dms in [
        (256, 1581.8, -1.5625, synth.dm_list_linear(100, 200.0)),
        (1024, 1581.8, -400.0 / 1024, synth.dm_list_expm1(1200, 1000.0)),
        (64, 1400.0, -3.0, [0.0, 0.0, 10.0, 10.0, 55.5]),
    ]:
        p = L.dedisp_plan_create(nchans, ft, df, 64e-6, dms)
        ref = oracle.delay_table(nchans, ft, df, 64e-6, dms)
        got = L.dedisp_plan_copy_delays(p)
        assert (got == ref).all()
        assert p.max_delay == oracle.max_delay(ref)
    log("delay tables ok")


def _run(p, packed, nsamps, dtype, tile=None):
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    inp = to_dev(packed)
    out = torch.full((p.ndm, nsamps - p.max_delay), 0x5A5A, dtype=dtype, device="cuda")
    ws = torch.empty(L.dedisp_workspace_bytes(p, nsamps), dtype=torch.uint8, device="cuda")
    if tile is None:
        L.dedisp_execute(p, inp, nsamps, out, ws)
    else:
        L.dedisp_execute_tile(p, inp, nsamps, out, ws, tile)
    torch.cuda.synchronize()
    return as_i64(out)


def as_i64(out):
    """Host int64 copy; 16-bit series are stored in int16 tensors and read as uint16."""
    torch = torch_dev()
    a = out.cpu().numpy()
    if out.dtype == torch.int16:
        a = a.view(np.uint16)
    return a.astype(np.int64)


def test_small_config_every_tile_both_dtypes():
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    fb, dly, x, ref = small_case()
    p = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    for tile in L.dedisp_tile_candidates():
        for dtype in (torch.int16, torch.int32):
            log("small config tile", tile, dtype)
            got = _run(p, fb.packed, fb.nsamps, dtype, tile)
            assert got.shape == ref.shape
            bad = np.argwhere(got != ref)
            assert bad.size == 0, (tile, dtype, bad[:5])


def test_default_tile_and_determinism():
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    fb, dly, x, ref = small_case()
    p = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    a = _run(p, fb.packed, fb.nsamps, torch.int16)
    b = _run(p, fb.packed, fb.nsamps, torch.int16)
    assert (a == ref).all() and (a == b).all()


@pytest.mark.parametrize("nchans,nsamps,dms,seed", [
    (4, 100, [0.0], 1),                         # DM 0 only: plain channel sum
    (8, 300, [0.0, 40.0, 80.0], 2),
    (12, 2500, list(np.linspace(0, 300, 7)), 3),
    (64, 6000, list(np.linspace(0, 120, 37)), 4),  # ragged DM blocks
    (1364, 3000, [0.0, 1.0, 2.0, 5.0, 9.0], 5),    # largest 12-level counter
    (1368, 3000, [0.0, 1.0, 2.0, 5.0, 9.0], 6),    # 16-level counter
])
def test_tiny_and_edge_shapes(nchans, nsamps, dms, seed):
    torch = torch_dev()
    from paper_1112_0065_amd import _lib as L
    df = -400.0 / max(nchans, 64)
    fb = synth.make_tiny(seed, nchans, nsamps, dms, df=df)
    p = L.dedisp_plan_create(nchans, fb.f_top, df, fb.tsamp, dms)
    dly = oracle.delay_table(nchans, fb.f_top, df, fb.tsamp, dms)
    ref = oracle.dedisperse(oracle.unpack_2bit(fb.packed, nsamps, nchans), dly)
    for dtype in (torch.int16, torch.int32):
        for tile in [None, (4, 1, 16), (32, 1, 32), (16, 2, 32)]:
            log("edge", nchans, nsamps, len(dms), dtype, tile)
            got = _run(p, fb.packed, nsamps, dtype, tile)
            assert (got == ref).all(), (nchans, dtype, tile)


def test_grouped_item_order_whole_output():
    """4096 channels x 200 trials: the work items go in several groups of DM
    blocks with a shorter last group (16 trials per block: groups of 4, 4, 4
    and 1 blocks; 32: 2, 2, 2, 1; 8: 8, 8, 8, 1) over three time tiles, the
    last one ragged.  The whole output equals the oracle's."""
    torch = torch_dev()
    from paper_1112_0065_amd import _lib as L
    nchans = 4096
    dms = list(np.linspace(0.0, 30.0, 200))
    df = -400.0 / nchans
    dly = oracle.delay_table(nchans, synth.F_TOP, df, synth.TSAMP, dms)
    nsamps = int(dly.max()) + 5000
    fb = synth.make_tiny(9, nchans, nsamps, dms, df=df)
    p = L.dedisp_plan_create(nchans, fb.f_top, df, fb.tsamp, dms)
    ref = oracle.dedisperse(oracle.unpack_2bit(fb.packed, nsamps, nchans), dly)
    for tile in [None, (32, 1, 16), (8, 1, 16)]:
        log("grouped items 4096 ch x 200 trials, tile", tile)
        got = _run(p, fb.packed, nsamps, torch.int32, tile)
        assert got.shape == ref.shape and (got == ref).all(), tile


@pytest.mark.parametrize("extra", [1, 2, 31, 32, 33, 2047, 2048, 2049, 4095, 4097])
def test_ragged_output_lengths(extra):
    """nout just around multiples of the 32-sample group and the time tile."""
    torch = torch_dev()
    from paper_1112_0065_amd import _lib as L
    nchans, dms = 32, [0.0, 25.0, 50.0]
    df = -10.0
    dly = oracle.delay_table(nchans, synth.F_TOP, df, synth.TSAMP, dms)
    nsamps = int(dly.max()) + extra
    fb = synth.make_tiny(extra, nchans, nsamps, dms, df=df)
    p = L.dedisp_plan_create(nchans, fb.f_top, df, fb.tsamp, dms)
    ref = oracle.dedisperse(oracle.unpack_2bit(fb.packed, nsamps, nchans), dly)
    for dtype in (torch.int16, torch.int32):
        got = _run(p, fb.packed, nsamps, dtype, (4, 2, 16))
        assert got.shape == (3, extra) and (got == ref).all()


def test_all_threes_maximum_sums():
    """Every sample at level 3: each output equals 3*nchans (the range limit
    of the 12- and 16-level counters and of uint16 at 21844 channels)."""
    torch = torch_dev()
    from paper_1112_0065_amd import _lib as L
    # 1364 / 21844: the largest sums of the two counters (4-channel last
    # chunk); 1360 / 21840: the same near the limit through 8-channel stages
    # (an odd number of them: 170 is even, 2730 is even; 1352 gives 169)
    for nchans, nsamps, tiles in [(1364, 700, [(4, 1, 16)]), (21844, 300, [(4, 1, 16)]),
                                  (1352, 700, [(16, 1, 8), (4, 1, 8)]),
                                  (1360, 700, [(16, 1, 8)]), (21840, 300, [(16, 1, 8)])]:
        dms = [0.0, 0.5]
        df = -0.01
        lv = np.full((nsamps, nchans), 3, np.uint8)
        fb = synth.make_tiny(0, nchans, nsamps, dms, df=df, levels=lv)
        p = L.dedisp_plan_create(nchans, fb.f_top, df, fb.tsamp, dms)
        for dtype in (torch.int16, torch.int32):
            for tile in tiles:
                log("all threes", nchans, dtype, tile)
                got = _run(p, fb.packed, nsamps, dtype, tile)
                assert (got == 3 * nchans).all(), (nchans, dtype, tile)


def test_too_few_samples_and_bad_args():
    torch = torch_dev()
    from paper_1112_0065_amd import _lib as L
    p = L.dedisp_plan_create(16, 1500.0, -5.0, 64e-6, [0.0, 100.0])
    buf = torch.zeros(16 * 4096 // 4, dtype=torch.uint8, device="cuda")
    out = torch.zeros((2, 10), dtype=torch.int32, device="cuda")
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.DedispError) as e:
        L.dedisp_execute(p, buf, p.max_delay, out, ws)
    assert e.value.status == L.ERR_TOO_FEW_SAMPLES
    with pytest.raises(L.DedispError) as e:
        L.dedisp_execute_tile(p, buf, 4096, out, ws, (5, 1, 16))
    assert e.value.status == L.ERR_INVALID_ARG
    for bad in [(6, 1500.0, -5.0, 64e-6, [0.0]), (16, 1500.0, 5.0, 64e-6, [0.0]),
                (16, 1500.0, -5.0, 0.0, [0.0]), (16, 1500.0, -5.0, 64e-6, [3.0, 1.0]),
                (16, 1500.0, -5.0, 64e-6, [-1.0]), (16, 1500.0, -100.0, 64e-6, [0.0])]:
        with pytest.raises(L.DedispError) as e:
            L.dedisp_plan_create(*bad)
        assert e.value.status == L.ERR_INVALID_ARG


def test_survey_config_whole_output_and_events():
    """Survey-shaped beam at full size (2^19 samples, 1024 channels, 1200
    trials), default tile, both output types: every element of the output
    equals the oracle's, and the whole event list of find_peaks on it (widths
    1..512, S/N > 6) equals the oracle's events of every (width, DM) series.
    The oracle runs on all host cores (forked workers)."""
    import time
    torch = torch_dev()
    from paper_1112_0065_amd import _lib as L
    from gpu_common import events_equal, oracle_all_rows
    fb = survey_case()
    p = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    dly = oracle.delay_table(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    assert p.max_delay == 20476
    nout = fb.nsamps - 20476
    inp = to_dev(fb.packed)
    ws = torch.empty(L.dedisp_workspace_bytes(p, fb.nsamps), dtype=torch.uint8, device="cuda")
    host = []
    for dtype in (torch.int16, torch.int32):
        out = torch.empty((1200, nout), dtype=dtype, device="cuda")
        log("survey full size", dtype)
        L.dedisp_execute(p, inp, fb.nsamps, out, ws)
        torch.cuda.synchronize()
        if dtype == torch.int16:
            pws = torch.empty(L.find_peaks_workspace_bytes(1200, nout, fb.widths),
                              dtype=torch.uint8, device="cuda")
            evb = torch.empty((1 << 20) * 40, dtype=torch.uint8, device="cuda")
            n = L.find_peaks(out, 1200, nout, fb.widths, fb.snr_thresh, evb, 1 << 20, pws)
            ev = L.events_from_buffer(evb, n)
            host.append(out.cpu().numpy().view(np.uint16))
            del pws, evb
        else:
            host.append(out.cpu().numpy())
        del out
    x = oracle.unpack_2bit(fb.packed, fb.nsamps, fb.nchans)
    t0 = time.time()
    bad, ref_ev = oracle_all_rows(x, dly, nout, host, fb.widths, fb.snr_thresh)
    log("oracle over all 1200 rows", round(time.time() - t0, 1), "s; mismatches", bad,
        "events gpu", len(ev), "oracle", len(ref_ev))
    assert bad == [0, 0]
    events_equal(ev, ref_ev)


def _planes_reference(x, nwords):
    """The channel-major bit-plane copy by its definition: for channel c,
    word j is a pair of 32-bit planes whose bit b is bit 0 (first) or bit 1
    (second) of the level of sample 32j + b; samples past the input, the
    two trailing words included, are zero."""
    nchans, nsamps = x.shape
    lv = np.zeros((nchans, 32 * nwords), dtype=np.uint8)
    lv[:, :nsamps] = x
    lo = np.packbits((lv & 1).astype(np.uint8), axis=1, bitorder="little").view("<u4")
    hi = np.packbits((lv >> 1).astype(np.uint8), axis=1, bitorder="little").view("<u4")
    return np.stack([lo, hi], axis=-1)   # [nchans][nwords][2]


@pytest.mark.parametrize("nchans,nsamps", [(1024, 4096), (1024, 4096 + 64), (256, (1 << 15) + 37),
                                           (1360, 1000), (4, 33), (2048, 512 * 3 + 511)])
def test_repack_layout_every_word(nchans, nsamps):
    """dedisp_repack writes every word of the bit-plane copy, and each equals
    its definition from the oracle's unpacked levels.  The workspace is filled
    with 0xAB first, so a word left unwritten fails.  The shapes cover whole
    and partial 512-sample tiles (a row length of 2 ceil(nsamps / 64) + 2
    words, whose two trailing words the last data tile writes when the data
    words end on a tile boundary), partial channel tiles and a tiny beam."""
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    rng = np.random.default_rng(nchans * 7 + nsamps)
    packed = rng.integers(0, 256, size=nsamps * nchans // 4, dtype=np.uint8)
    p = L.dedisp_plan_create(nchans, 1581.8, -400.0 / nchans, 64e-6, [0.0, 1.0])
    nwords = 2 * ((nsamps + 63) // 64) + 2
    nbytes = L.dedisp_workspace_bytes(p, nsamps)
    assert nbytes >= nchans * nwords * 8
    ws = torch.full((nbytes,), 0xAB, dtype=torch.uint8, device="cuda")
    log("repack layout", nchans, nsamps)
    L.dedisp_repack(p, to_dev(packed), nsamps, ws)
    torch.cuda.synchronize()
    got = ws[: nchans * nwords * 8].cpu().numpy().view("<u4").reshape(nchans, nwords, 2)
    ref = _planes_reference(oracle.unpack_2bit(packed, nsamps, nchans), nwords)
    bad = np.argwhere(got != ref)
    assert len(bad) == 0, (len(bad), bad[:5].tolist())
