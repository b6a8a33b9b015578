"""GPU tests of the streaming server: streamed results equal the oracle on
each chunk's window (which itself equals the one-shot result restricted to
that window), each chunk's result is the same alone and in the 13-beam mix,
gaps, ordering errors and HBM-budget back-pressure."""
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_common import events_equal, log, to_dev, torch_dev

pytestmark = pytest.mark.gpu

WIDTHS = [1, 2, 4, 8, 16]
K = 5.0
C = 8192
NCH = 256


def _stream(seed, nchunks, dm_max):
    """One beam of nchunks*C samples (generator: survey recipe at 256 ch)."""
    fb = synth.make_beam(seed, nchunks * C, dm_max, 4, nchans=NCH, df=-400.0 / NCH, ndm=64,
                         widths=WIDTHS, snr_thresh=K, name=f"s{seed}")
    return fb


def _chunk(fb, k):
    bpc = fb.nchans // 4
    return fb.packed[k * C * bpc:(k + 1) * C * bpc]


def _drain(srv, want, timeout_s=120):
    from paper_1112_0065_amd import _lib as L
    got = []
    t0 = time.time()
    while len(got) < want and time.time() - t0 < timeout_s:
        got += L.dedisp_serve_poll(srv, 64, 200)
    assert len(got) == want, (len(got), want)
    return got


def _oracle_window(fb, dly, t_abs0, nsamps):
    x = oracle.unpack_2bit(fb.packed, fb.nsamps, fb.nchans)[:, t_abs0:t_abs0 + nsamps]
    out = oracle.dedisperse(x, dly)
    return out, oracle.find_events(oracle.boxcar(out, WIDTHS), K)


def test_stream_matches_oracle_windows():
    from paper_1112_0065_amd import _lib as L
    torch_dev()
    nch = 4
    fbs = [_stream(700 + b, nch, 80.0 + 30 * b) for b in range(3)]
    plans = [L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list) for fb in fbs]
    budget = 40 * L.dedisp_serve_slot_bytes(plans, C, WIDTHS)
    srv = L.dedisp_serve_create(plans, C, WIDTHS, K, budget)
    for k in range(nch):
        for b, fb in enumerate(fbs):
            while not L.dedisp_serve_submit(srv, b, k, _chunk(fb, k), L.dedisp_now_ns()):
                time.sleep(0.01)
    res = _drain(srv, 3 * nch)
    st = L.dedisp_serve_stats(srv)
    log("serve stats", st)
    assert st["chunks_done"] == 3 * nch and st["p50_ns"] <= st["p99_ns"] <= st["max_ns"]
    for b, fb in enumerate(fbs):
        dly = oracle.delay_table(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
        md = int(dly.max())
        H = md + WIDTHS[-1] - 1
        one_shot = oracle.dedisperse(oracle.unpack_2bit(fb.packed, fb.nsamps, fb.nchans), dly)
        mine = sorted([r for r in res if r["beam"] == b], key=lambda r: r["seq"])
        assert [r["seq"] for r in mine] == list(range(nch))
        covered = 0
        for r in mine:
            k = r["seq"]
            start = 0 if k == 0 else k * C - H
            nsamps = C if k == 0 else C + H
            assert r["t_abs0"] == start and r["flags"] & L.CHUNK_GAP == 0
            assert r["n_bx"] == (C - H if k == 0 else C)
            out_w, ev_w = _oracle_window(fb, dly, start, nsamps)
            # the window's series is the one-shot series over the same samples
            assert (out_w == one_shot[:, start:start + out_w.shape[1]]).all()
            events_equal(r["events"], ev_w)
            covered += r["n_bx"]
        # positions covered by the chunks are contiguous and complete
        assert covered == nch * C - H


def test_alone_equals_in_mix():
    """Every beam's chunks give identical events alone and among 13 beams,
    and the mix really ran as continuous batches (several beams' chunks in
    one launch)."""
    from paper_1112_0065_amd import _lib as L
    torch_dev()
    fbs = [_stream(800 + b, 2, 60.0 + 10 * b) for b in range(13)]
    plans = [L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list) for fb in fbs]
    budget = 30 * L.dedisp_serve_slot_bytes(plans, C, WIDTHS)
    mix = L.dedisp_serve_create(plans, C, WIDTHS, K, budget)
    for k in range(2):
        for b in range(13):
            while not L.dedisp_serve_submit(mix, b, k, _chunk(fbs[b], k), L.dedisp_now_ns()):
                time.sleep(0.01)
    res_mix = _drain(mix, 26)
    st = L.dedisp_serve_stats(mix)
    log("mix stats", st)
    mix.close()
    assert st["max_batch"] >= 2, st
    assert st["batches"] < 26, st
    for b in range(13):
        alone = L.dedisp_serve_create([plans[b]], C, WIDTHS, K, budget)
        for k in range(2):
            assert L.dedisp_serve_submit(alone, 0, k, _chunk(fbs[b], k), L.dedisp_now_ns())
        res_alone = _drain(alone, 2)
        alone.close()
        for k in range(2):
            a = [r for r in res_alone if r["seq"] == k][0]
            m = [r for r in res_mix if r["beam"] == b and r["seq"] == k][0]
            assert a["t_abs0"] == m["t_abs0"] and a["n_events"] == m["n_events"]
            assert a["events"].tobytes() == m["events"].tobytes()


def test_gap_order_budget_and_backpressure():
    from paper_1112_0065_amd import _lib as L
    torch_dev()
    fb = _stream(900, 6, 100.0)
    plan = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    slot = L.dedisp_serve_slot_bytes([plan], C, WIDTHS)
    with pytest.raises(L.DedispError) as e:
        L.dedisp_serve_create([plan], C, WIDTHS, K, slot // 2)
    assert e.value.status == L.ERR_OUT_OF_MEMORY
    # one slot only: chunks queue behind each other; staging holds 2*slots+beams
    srv = L.dedisp_serve_create([plan], C, WIDTHS, K, slot + (1 << 22))
    assert L.dedisp_serve_stats(srv)["slots"] == 1
    admitted = 0
    busy = 0
    for k in (0, 1, 3, 4, 5):           # chunk 2 never arrives: a gap
        while not L.dedisp_serve_submit(srv, 0, k, _chunk(fb, k), L.dedisp_now_ns()):
            busy += 1
            time.sleep(0.005)
        admitted += 1
    with pytest.raises(L.DedispError) as e:
        L.dedisp_serve_submit(srv, 0, 4, _chunk(fb, 4), L.dedisp_now_ns())
    assert e.value.status == L.ERR_INVALID_ARG
    res = sorted(_drain(srv, admitted), key=lambda r: r["seq"])
    flags = {r["seq"]: r["flags"] for r in res}
    assert flags[3] & L.CHUNK_GAP and not flags[1] & L.CHUNK_GAP and not flags[4] & L.CHUNK_GAP
    r3 = [r for r in res if r["seq"] == 3][0]
    dly = oracle.delay_table(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    H = int(dly.max()) + WIDTHS[-1] - 1
    assert r3["t_abs0"] == 3 * C and r3["n_bx"] == C - H
    _, ev = _oracle_window(fb, dly, 3 * C, C)
    events_equal(r3["events"], ev)
    st = L.dedisp_serve_stats(srv)
    assert st["max_batch"] == 1 and st["chunks_done"] == admitted
    log("one-slot stats", st, "busy retries", busy)
    srv.close()


def test_serve_scores_with_trained_model():
    """With the trained network attached, the candidates of a chunk (the
    events per-width non-maximum suppression keeps, as the oracle selects
    them) get the score the standalone path (dedisperse -> find_peaks ->
    tiles -> forward) gives the same window, bit for bit, every other event
    gets -1, and the FALLBACK flag stays clear; without a network the flag is
    set and the events are unchanged."""
    from paper_1112_0065_amd import _lib as L
    from paper_1112_0065_amd import triage_train as T
    torch = torch_dev()
    model, _, _ = T.load_default()
    fb = _stream(905, 3, 120.0)
    plan = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    budget = 12 * L.dedisp_serve_slot_bytes([plan], C, WIDTHS)
    res = {}
    for mdl in (model, None):
        srv = L.dedisp_serve_create([plan], C, WIDTHS, K, budget, model=mdl)
        for k in range(3):
            assert L.dedisp_serve_submit(srv, 0, k, _chunk(fb, k), L.dedisp_now_ns())
        res[mdl is None] = sorted(_drain(srv, 3), key=lambda r: r["seq"])
        srv.close()
    bpc = fb.nchans // 4
    H = plan.max_delay + WIDTHS[-1] - 1
    dropped = 0
    for r, r0 in zip(res[False], res[True]):
        assert r["flags"] & L.CHUNK_FALLBACK == 0 and r0["flags"] & L.CHUNK_FALLBACK
        assert r["events"].tobytes() == r0["events"].tobytes() and r0["scores"] is None
        k = r["seq"]
        start = 0 if k == 0 else k * C - H
        nsamps = C if k == 0 else C + H
        inp = torch.from_numpy(fb.packed[start * bpc:(start + nsamps) * bpc].copy()).cuda()
        nout = nsamps - plan.max_delay
        ws = torch.empty(L.dedisp_workspace_bytes(plan, nsamps), dtype=torch.uint8, device="cuda")
        out = torch.empty((plan.ndm, nout), dtype=torch.int16, device="cuda")
        L.dedisp_execute(plan, inp, nsamps, out, ws)
        pws = torch.empty(L.find_peaks_workspace_bytes(plan.ndm, nout, WIDTHS), dtype=torch.uint8,
                          device="cuda")
        evb = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
        n = L.find_peaks(out, plan.ndm, nout, WIDTHS, K, evb, (1 << 20) // 40, pws)
        ev = L.events_from_buffer(evb, n)
        # the chunk's events are the window's (times relative to t_abs0)
        assert n == r["n_events"] and n > 0
        assert ev.tobytes() == r["events"].tobytes()
        keep = oracle.nms(ev, WIDTHS)
        assert list(L.dedisp_candidates_nms(ev, WIDTHS)) == keep
        nk = len(keep)
        # a chunk with a single event keeps it; suppression must drop some
        # events over the three chunks
        assert r["n_candidates"] == nk and 0 < nk <= n
        dropped += n - nk
        cand = ev[keep]
        evd = torch.from_numpy(np.frombuffer(cand.tobytes(), np.uint8).copy()).cuda()
        tiles = torch.empty((nk, 64, 256), dtype=torch.int16, device="cuda")
        L.triage_tiles(out, plan.ndm, nout, WIDTHS, pws, evd, nk, tiles)
        sc = torch.empty(nk, dtype=torch.float32, device="cuda")
        L.triage_score(model, tiles, nk, sc)
        torch.cuda.synchronize()
        log("chunk", k, "events", n, "candidates", nk, "scores", r["scores"][keep][:4])
        assert r["scores"] is not None and len(r["scores"]) == n
        assert (sc.cpu().numpy() == r["scores"][keep]).all()
        rest = np.ones(n, bool)
        rest[keep] = False
        assert (r["scores"][rest] == -1.0).all()
    assert dropped > 0


def test_serve_clusters_each_chunk():
    """With clustering on, every result carries the clusters of its own
    events, equal to the oracle's clustering of those events; set after the
    first submit it is refused."""
    from paper_1112_0065_amd import _lib as L
    torch_dev()
    nch = 3
    fbs = [_stream(760 + b, nch, 90.0 + 20 * b) for b in range(2)]
    plans = [L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list) for fb in fbs]
    budget = 40 * L.dedisp_serve_slot_bytes(plans, C, WIDTHS)
    srv = L.dedisp_serve_create(plans, C, WIDTHS, K, budget)
    L.dedisp_serve_set_clustering(srv, 2, 1, 0)
    for k in range(nch):
        for b, fb in enumerate(fbs):
            while not L.dedisp_serve_submit(srv, b, k, _chunk(fb, k), L.dedisp_now_ns()):
                time.sleep(0.01)
    with pytest.raises(L.DedispError) as ei:
        L.dedisp_serve_set_clustering(srv, 1, 1, 0)
    assert ei.value.status == L.ERR_BUSY
    res = _drain(srv, 2 * nch)
    total_ev = total_cl = 0
    for r in res:
        assert r["flags"] & L.CHUNK_CLUSTERED and r["clusters"] is not None
        _, ref = oracle.cluster_events(r["events"], WIDTHS, 2, 1, 0)
        got = r["clusters"]
        assert len(got) == len(ref)
        for g, c in zip(got, ref):
            assert tuple(int(g[k]) for k in oracle.CLUSTER_FIELDS[:-1]) == \
                tuple(c[k] for k in oracle.CLUSTER_FIELDS[:-1]) and float(g["snr"]) == c["snr"]
        total_ev += len(r["events"])
        total_cl += len(got)
    log(f"served {total_ev} events in {total_cl} clusters")
    assert total_ev > total_cl > 0
    srv.close()


def test_serve_stages_equal_standalone_chain():
    """With the coincidence mask (per round of chunks) and baseline removal
    on, every served chunk equals the standalone chain on its window: the
    round's mask (dedisp_rfi_mask over the round's raw chunks) applied to
    each chunk, the window of the masked stream (overlap grown by 2R),
    dedisp_execute, baseline_remove, find_peaks; one window also equals the
    oracle chain.  A round runs as one batch."""
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    nb, nch, nk, R, KR, MB = 4, NCH, 3, 32, 3.0, 2
    packed, imps, _, _ = synth.make_coincidence_beams(41, nbeams=nb, nsamps=nk * C, nchans=nch,
                                                      npulses=3, impulse_rate=30.0, dm_max=100.0)
    bpc = nch // 4
    dms = [synth.dm_list_linear(64, 60.0 + 10.0 * b) for b in range(nb)]
    plans = [L.dedisp_plan_create(nch, synth.F_TOP, -400.0 / nch, synth.TSAMP, dms[b])
             for b in range(nb)]
    budget = 30 * L.dedisp_serve_slot_bytes(plans, C, WIDTHS)
    srv = L.dedisp_serve_create(plans, C, WIDTHS, K, budget)
    L.dedisp_serve_set_stages(srv, KR, MB, R)
    for k in range(nk):
        for b in range(nb):
            while not L.dedisp_serve_submit(srv, b, k, packed[b][k * C * bpc:(k + 1) * C * bpc],
                                            L.dedisp_now_ns()):
                time.sleep(0.01)
    res = _drain(srv, nb * nk)
    st = L.dedisp_serve_stats(srv)
    with pytest.raises(L.DedispError) as ei:
        L.dedisp_serve_set_stages(srv, 0.0, 0, 0)
    assert ei.value.status == L.ERR_BUSY
    srv.close()
    log("serve stages stats", st)
    assert st["max_batch"] >= nb

    # the masked streams, round by round
    masked = [np.empty(nk * C * bpc, np.uint8) for _ in range(nb)]
    ws = torch.empty(L.dedisp_rfi_mask_workspace_bytes(nb, C), dtype=torch.uint8, device="cuda")
    mask = torch.empty(C, dtype=torch.uint8, device="cuda")
    flagged = 0
    for k in range(nk):
        chunks = [to_dev(packed[b][k * C * bpc:(k + 1) * C * bpc].copy()) for b in range(nb)]
        flagged += L.dedisp_rfi_mask(chunks, nch, C, KR, MB, mask, ws)
        L.dedisp_rfi_apply(chunks, nch, C, mask)
        for b in range(nb):
            masked[b][k * C * bpc:(k + 1) * C * bpc] = chunks[b].cpu().numpy()
    log("flagged samples", flagged, "impulses", len(imps))
    assert flagged > 0
    checked_oracle = False
    for r in res:
        b, k = r["beam"], r["seq"]
        p = plans[b]
        Hb = p.max_delay + WIDTHS[-1] - 1 + 2 * R
        start = 0 if k == 0 else k * C - Hb
        nsamps = (k + 1) * C - start
        assert r["t_abs0"] == start + R
        win = masked[b][start * bpc:(k + 1) * C * bpc]
        nout = nsamps - p.max_delay
        out = torch.empty((64, nout), dtype=torch.int16, device="cuda")
        dws = torch.empty(L.dedisp_workspace_bytes(p, nsamps), dtype=torch.uint8, device="cuda")
        L.dedisp_execute(p, to_dev(win.copy()), nsamps, out, dws)
        flat = torch.empty((64, nout - 2 * R), dtype=torch.int16, device="cuda")
        L.baseline_remove(out, 64, nout, R, 3 * nch, flat)
        pws = torch.empty(L.find_peaks_workspace_bytes(64, nout - 2 * R, WIDTHS), dtype=torch.uint8,
                          device="cuda")
        evb = torch.empty(4096 * 40, dtype=torch.uint8, device="cuda")
        n = L.find_peaks(flat, 64, nout - 2 * R, WIDTHS, K, evb, 4096, pws)
        assert n == r["n_events"] and r["n_bx"] == nout - 2 * R - WIDTHS[-1] + 1
        assert L.events_from_buffer(evb, n).tobytes() == r["events"].tobytes(), (b, k)
        if k == 1 and not checked_oracle:
            x = oracle.unpack_2bit(win, nsamps, nch)
            dly = oracle.delay_table(nch, synth.F_TOP, -400.0 / nch, synth.TSAMP, dms[b])
            fl = oracle.baseline_remove(oracle.dedisperse(x, dly), R, 3 * nch)
            events_equal(r["events"], oracle.find_events(oracle.boxcar(fl, WIDTHS), K))
            checked_oracle = True
    assert checked_oracle
