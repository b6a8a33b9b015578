"""GPU tests of the multibeam batch (one persistent launch + graph replay)
and of the tile autotuner: results identical to the single-beam path and to
the oracle."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_common import events_equal, log, small_case, to_dev, torch_dev

pytestmark = pytest.mark.gpu

WIDTHS = [1, 2, 4, 8, 16]


def _beams(n, nchans=256, ndm=64):
    """Uneven beams: lengths and DM ranges differ per beam (as in a
    multibeam receiver whose beams are processed with their own plans)."""
    out = []
    for b in range(n):
        nsamps = 24000 + 5000 * b
        dm_max = 60.0 + 25.0 * ((5 * b) % 7)
        fb = synth.make_beam(500 + b, nsamps, dm_max, 3, nchans=nchans, df=-400.0 / nchans,
                             ndm=ndm, widths=WIDTHS, snr_thresh=5.0, name=f"b{b}")
        out.append(fb)
    return out


def _single(plan, fb, inp, out_dtype, torch, L):
    nout = fb.nsamps - plan.max_delay
    out = torch.empty((plan.ndm, nout), dtype=out_dtype, device="cuda")
    ws = torch.empty(L.dedisp_workspace_bytes(plan, fb.nsamps), dtype=torch.uint8, device="cuda")
    L.dedisp_execute(plan, inp, fb.nsamps, out, ws)
    pws = torch.empty(L.find_peaks_workspace_bytes(plan.ndm, nout, WIDTHS), dtype=torch.uint8,
                      device="cuda")
    evb = torch.empty(4096 * 40, dtype=torch.uint8, device="cuda")
    n = L.find_peaks(out, plan.ndm, nout, WIDTHS, 5.0, evb, 4096, pws)
    return out, L.events_from_buffer(evb, n)


@pytest.mark.parametrize("u16", [True, False])
def test_batch_equals_single_beam_and_oracle(u16):
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    fbs = _beams(6)
    plans = [L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list) for fb in fbs]
    dt = torch.int16 if u16 else torch.int32
    ins = [to_dev(fb.packed) for fb in fbs]
    outs = [torch.empty((p.ndm, fb.nsamps - p.max_delay), dtype=dt, device="cuda")
            for p, fb in zip(plans, fbs)]
    evs = [torch.empty(4096 * 40, dtype=torch.uint8, device="cuda") for _ in fbs]
    batch = L.dedisp_batch_create(plans, WIDTHS, 5.0, out_u16=u16)
    tile, grid, caps = L.dedisp_batch_info(batch)
    log("batch tile", tile, "grid", grid)
    counts = L.dedisp_batch_execute(batch, ins, [fb.nsamps for fb in fbs], outs, evs, [4096] * 6)
    assert L.dedisp_batch_info(batch)[2] == 1
    for b, (p, fb) in enumerate(zip(plans, fbs)):
        s_out, s_ev = _single(p, fb, ins[b], dt, torch, L)
        assert torch.equal(outs[b], s_out), b
        b_ev = L.events_from_buffer(evs[b], counts[b])
        assert b_ev.tobytes() == s_ev.tobytes(), b
    # two beams against the oracle
    for b in (0, 5):
        fb = fbs[b]
        dly = oracle.delay_table(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
        ref = oracle.dedisperse(oracle.unpack_2bit(fb.packed, fb.nsamps, fb.nchans), dly)
        got = outs[b].cpu().numpy()
        got = (got.view(np.uint16) if u16 else got).astype(np.int64)
        assert (got == ref).all()
        events_equal(L.events_from_buffer(evs[b], counts[b]),
                     oracle.find_events(oracle.boxcar(ref, WIDTHS), 5.0))


def test_batch_replays_and_recapture():
    """Graph replays with eager work in between give identical results; a
    changed length re-captures and stays exact."""
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    fbs = _beams(3)
    plans = [L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list) for fb in fbs]
    ins = [to_dev(fb.packed) for fb in fbs]
    outs = [torch.empty((p.ndm, fb.nsamps - p.max_delay), dtype=torch.int16, device="cuda")
            for p, fb in zip(plans, fbs)]
    evs = [torch.empty(4096 * 40, dtype=torch.uint8, device="cuda") for _ in fbs]
    batch = L.dedisp_batch_create(plans, WIDTHS, 5.0)
    ns = [fb.nsamps for fb in fbs]
    first = None
    for rep in range(4):
        cnt = L.dedisp_batch_execute(batch, ins, ns, outs, evs, [4096] * 3)
        snap = [o.clone() for o in outs] + [e.clone() for e in evs]
        # eager work and a sync between replays
        junk = torch.randn(1 << 20, device="cuda").sum().item()
        assert np.isfinite(junk)
        for o in outs:
            o.fill_(0)
        if first is None:
            first = (cnt, snap)
        else:
            assert cnt == first[0]
            assert all(torch.equal(a, b) for a, b in zip(snap, first[1]))
    assert L.dedisp_batch_info(batch)[2] == 1
    # shorter second beam: new capture, exact against the single-beam path
    ns2 = list(ns)
    ns2[1] = ns[1] - 3001
    outs2 = list(outs)
    outs2[1] = torch.empty((plans[1].ndm, ns2[1] - plans[1].max_delay), dtype=torch.int16,
                           device="cuda")
    L.dedisp_batch_execute(batch, ins, ns2, outs2, evs, [4096] * 3)
    assert L.dedisp_batch_info(batch)[2] == 2
    fb1 = fbs[1]
    short = synth.Filterbank(fb1.name, fb1.seed, fb1.nchans, ns2[1], fb1.f_top, fb1.df, fb1.tsamp,
                             fb1.dm_list, fb1.widths, fb1.snr_thresh,
                             fb1.packed[: ns2[1] * fb1.nchans // 4], [])
    s_out, _ = _single(plans[1], short, ins[1], torch.int16, torch, L)
    assert torch.equal(outs2[1], s_out)


def test_autotune_small_config(tmp_path):
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    fb, dly, x, ref = small_case()
    p = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    cache = str(tmp_path / "tune.json")
    best, rejected = L.dedisp_autotune(p, fb.nsamps, True, cache)
    log("autotune best", best, "rejected", rejected)
    assert rejected == 0
    assert best in L.dedisp_tile_candidates()
    assert L.dedisp_default_tile(p) == best
    entries = json.load(open(cache))
    key = [k for k in entries if ":nchans=256:ndm=128:u16" in k]
    assert key and entries[key[0]][:3] == list(best)
    # a plan created with the cache in the environment starts from it
    os.environ["DEDISP_TUNE_CACHE"] = cache
    try:
        p2 = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    finally:
        del os.environ["DEDISP_TUNE_CACHE"]
    assert L.dedisp_default_tile(p2) == best
    out = torch.empty((p2.ndm, fb.nsamps - p2.max_delay), dtype=torch.int16, device="cuda")
    ws = torch.empty(L.dedisp_workspace_bytes(p2, fb.nsamps), dtype=torch.uint8, device="cuda")
    L.dedisp_execute(p2, to_dev(fb.packed), fb.nsamps, out, ws)
    assert (out.cpu().numpy().view(np.uint16).astype(np.int64) == ref).all()
    # batch reading the same cache uses the tuned shape
    b = L.dedisp_batch_create([p2], WIDTHS, 5.0, tune_cache_path=cache)
    assert L.dedisp_batch_info(b)[0] == best


def test_batch_at_multibeam_survey_shape():
    """The shape the benchmark times: 13 beams of 1024 channels and 1200
    trials, lengths 2^17 + 2^15 b and DM ranges to 500 + 125 ((5b) mod 13)
    (beam b reads a prefix of one seeded pool), widths 1..512, S/N > 6.  The
    batch's outputs and events are byte-equal to the single-beam path for
    every beam; sampled rows of every beam, and their events, equal the
    oracle's."""
    from paper_1112_0065_amd import _lib as L
    from oracle.peaks import series_events
    torch = torch_dev()
    shapes = synth.multibeam_shapes()
    nmax = max(n for n, _ in shapes)
    pool = synth.fast_chunk(300, nmax, npulses=20)
    widths = [1 << i for i in range(10)]
    plans, ins, outs, evs, ns = [], [], [], [], []
    for b, (n, dm_max) in enumerate(shapes):
        p = L.dedisp_plan_create(1024, synth.F_TOP, synth.DF_SURVEY, synth.TSAMP,
                                 synth.dm_list_expm1(1200, dm_max))
        plans.append(p)
        ins.append(to_dev(pool[: n * 256]))
        outs.append(torch.empty((1200, n - p.max_delay), dtype=torch.int16, device="cuda"))
        evs.append(torch.empty((1 << 20) * 40, dtype=torch.uint8, device="cuda"))
        ns.append(n)
    batch = L.dedisp_batch_create(plans, widths, 6.0, out_u16=True)
    log("multibeam batch", L.dedisp_batch_info(batch)[:2])
    counts = L.dedisp_batch_execute(batch, ins, ns, outs, evs, [1 << 20] * 13)
    torch.cuda.synchronize()
    log("multibeam events per beam", counts)
    x_all = oracle.unpack_2bit(pool, nmax, 1024)
    rng = np.random.default_rng(13)
    for b, (p, n) in enumerate(zip(plans, ns)):
        nout = n - p.max_delay
        ws = torch.empty(L.dedisp_workspace_bytes(p, n), dtype=torch.uint8, device="cuda")
        single = torch.empty((1200, nout), dtype=torch.int16, device="cuda")
        L.dedisp_execute(p, ins[b], n, single, ws)
        pws = torch.empty(L.find_peaks_workspace_bytes(1200, nout, widths), dtype=torch.uint8,
                          device="cuda")
        evb = torch.empty((1 << 20) * 40, dtype=torch.uint8, device="cuda")
        ns_ev = L.find_peaks(single, 1200, nout, widths, 6.0, evb, 1 << 20, pws)
        assert torch.equal(outs[b], single), b
        b_ev = L.events_from_buffer(evs[b], counts[b])
        assert ns_ev == counts[b] and b_ev.tobytes() == L.events_from_buffer(evb, ns_ev).tobytes(), b
        del single, pws, evb, ws
        # sampled rows against the oracle
        rows = sorted({0, 1199, int(rng.integers(1, 1199))})
        dly = oracle.delay_table(1024, synth.F_TOP, synth.DF_SURVEY, synth.TSAMP,
                                 synth.dm_list_expm1(1200, shapes[b][1]))
        ref = oracle.dedisperse(x_all[:, :n], dly[rows], nout=nout)
        got = outs[b][rows].cpu().numpy().view(np.uint16).astype(np.int64)
        assert (got == ref).all(), b
        bw = oracle.boxcar(ref, widths)
        for j, d in enumerate(rows):
            for wi in range(len(widths)):
                want = series_events(bw[wi, j], 6.0, wi, d)
                mine = [e for e in b_ev if int(e["width_idx"]) == wi and int(e["dm_idx"]) == d]
                events_equal(mine, want)
        log("beam", b, "n", n, "events", counts[b], "rows", rows, "ok")


def test_batch_stages_equal_standalone_and_oracle_chain():
    """The batch with its optional stages -- coincidence mask before
    dedispersion, baseline removal after -- gives every beam the events of
    the standalone chain (dedisp_rfi_mask + dedisp_rfi_apply on copies of the
    inputs over the samples all beams share, dedisp_execute, baseline_remove,
    find_peaks) bit for bit, and two beams the events of the oracle chain;
    the graph is captured again when the stages change, and switching them
    off restores the plain results."""
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    nb, nch, n0, R, K, MB = 6, 256, 30000, 48, 3.0, 3
    packed, imps, _, _ = synth.make_coincidence_beams(31, nbeams=nb, nsamps=n0, nchans=nch,
                                                      npulses=2, impulse_rate=40.0, dm_max=150.0)
    bpc = nch // 4
    ns = [n0 - 1500 * b for b in range(nb)]                 # uneven lengths
    n_common = min(ns)
    dms = [synth.dm_list_linear(48, 60.0 + 20.0 * b) for b in range(nb)]
    plans = [L.dedisp_plan_create(nch, synth.F_TOP, -400.0 / nch, synth.TSAMP, dms[b])
             for b in range(nb)]
    ins = [to_dev(packed[b][:ns[b] * bpc].copy()) for b in range(nb)]
    outs = [torch.empty((48, ns[b] - plans[b].max_delay), dtype=torch.int16, device="cuda")
            for b in range(nb)]
    evs = [torch.empty(4096 * 40, dtype=torch.uint8, device="cuda") for _ in range(nb)]
    caps = [4096] * nb
    batch = L.dedisp_batch_create(plans, WIDTHS, 5.0, out_u16=True)
    plain = L.dedisp_batch_execute(batch, ins, ns, outs, evs, caps)
    plain_ev = [L.events_from_buffer(evs[b], plain[b]).tobytes() for b in range(nb)]
    L.dedisp_batch_set_stages(batch, K, MB, R)
    counts = L.dedisp_batch_execute(batch, ins, ns, outs, evs, caps)
    got = [L.events_from_buffer(evs[b], counts[b]) for b in range(nb)]
    # the inputs are untouched
    for b in range(nb):
        assert (ins[b].cpu().numpy() == packed[b][:ns[b] * bpc]).all()

    # standalone chain
    ws = torch.empty(L.dedisp_rfi_mask_workspace_bytes(nb, n_common), dtype=torch.uint8,
                     device="cuda")
    mask = torch.empty(n_common, dtype=torch.uint8, device="cuda")
    nmask = L.dedisp_rfi_mask(ins, nch, n_common, K, MB, mask, ws)
    log("batch stages: flagged samples", nmask, "impulses", len(imps))
    assert nmask > 0
    copies = [t.clone() for t in ins]
    L.dedisp_rfi_apply(copies, nch, n_common, mask)
    for b in range(nb):
        p = plans[b]
        nout = ns[b] - p.max_delay
        out = torch.empty((48, nout), dtype=torch.int16, device="cuda")
        dws = torch.empty(L.dedisp_workspace_bytes(p, ns[b]), dtype=torch.uint8, device="cuda")
        L.dedisp_execute(p, copies[b], ns[b], out, dws)
        flat = torch.empty((48, nout - 2 * R), dtype=torch.int16, device="cuda")
        L.baseline_remove(out, 48, nout, R, 3 * nch, flat)
        pws = torch.empty(L.find_peaks_workspace_bytes(48, nout - 2 * R, WIDTHS),
                          dtype=torch.uint8, device="cuda")
        evb = torch.empty(4096 * 40, dtype=torch.uint8, device="cuda")
        n = L.find_peaks(flat, 48, nout - 2 * R, WIDTHS, 5.0, evb, 4096, pws)
        ref = L.events_from_buffer(evb, n)
        assert n == counts[b] and ref.tobytes() == got[b].tobytes(), b
        assert (out.cpu().numpy() == outs[b].cpu().numpy()).all()

    # oracle chain on two beams
    zs = [oracle.zero_dm_series(packed[b][:n_common * bpc], n_common, nch) for b in range(nb)]
    omask, _, _ = oracle.rfi_mask(zs, K, MB)
    assert (omask == mask.cpu().numpy().astype(bool)).all()
    for b in (0, nb - 1):
        p = plans[b]
        x = oracle.unpack_2bit(packed[b][:ns[b] * bpc], ns[b], nch)
        full_mask = np.zeros(ns[b], bool)
        full_mask[:n_common] = omask
        x = oracle.replace_masked(x, full_mask)
        dly = oracle.delay_table(nch, synth.F_TOP, -400.0 / nch, synth.TSAMP, dms[b])
        ded = oracle.dedisperse(x, dly)
        flat = oracle.baseline_remove(ded, R, 3 * nch)
        events_equal(got[b], oracle.find_events(oracle.boxcar(flat, WIDTHS), 5.0))

    # stages off: the plain results again, from a fresh capture
    L.dedisp_batch_set_stages(batch, 0.0, 0, 0)
    again = L.dedisp_batch_execute(batch, ins, ns, outs, evs, caps)
    assert again == plain
    assert [L.events_from_buffer(evs[b], again[b]).tobytes() for b in range(nb)] == plain_ev
    _, _, captures = L.dedisp_batch_info(batch)
    assert captures == 3
