"""GPU parity of event clustering across DM and width against the oracle,
through the C ABI: cluster labels and records bit-exact (the snr of a record
is copied from its representative event, so it matches exactly too)."""
import numpy as np
import pytest

import oracle
from oracle.cluster import CLUSTER_FIELDS
import synth
from gpu_common import log, small_search, small_case, survey_case, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def _run(ev, ndm, widths, dr, wr, tol, capacity=None):
    """Cluster the structured event array on the GPU: (n, labels, records)."""
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    n = len(ev)
    cap = n if capacity is None else capacity
    evd = to_dev(np.frombuffer(np.ascontiguousarray(ev).tobytes(), np.uint8).copy()) if n else None
    ws = torch.empty(max(L.dedisp_cluster_workspace_bytes(n, ndm, len(widths)), 1), dtype=torch.uint8,
                     device="cuda")
    cb = torch.empty(max(cap, 1) * 72, dtype=torch.uint8, device="cuda")
    lab = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    nc = L.dedisp_cluster_events(evd, n, ndm, widths, dr, wr, tol, cb, cap, ws, labels=lab)
    torch.cuda.synchronize()
    return nc, lab.cpu().numpy()[:n].astype(np.int64), L.clusters_from_buffer(cb, min(nc, cap))


def _same(got_labels, got, ref_labels, ref):
    assert got_labels.tolist() == ref_labels.tolist()
    assert len(got) == len(ref)
    for g, r in zip(got, ref):
        gi = tuple(float(g[k]) if k == "snr" else int(g[k]) for k in CLUSTER_FIELDS)
        ri = tuple(float(r[k]) if k == "snr" else int(r[k]) for k in CLUSTER_FIELDS)
        assert gi == ri, (gi, ri)


@pytest.mark.parametrize("seed,ndm,nwidths,nout,nclumps,nnoise,params", [
    (1, 300, 8, 100000, 20, 200, (2, 1, 0)),
    (2, 1200, 10, 1 << 20, 120, 3000, (2, 1, 0)),
    (3, 1200, 10, 1 << 20, 120, 3000, (0, 0, 0)),
    (4, 1200, 10, 1 << 20, 120, 3000, (5, 2, 8)),
    (5, 64, 3, 4000, 60, 900, (3, 2, 20)),        # dense: large clusters, many ties
    (6, 1200, 10, 1 << 20, 250, 6000, (1, 0, 2)),
])
def test_matches_oracle_synthetic(seed, ndm, nwidths, nout, nclumps, nnoise, params):
    ev = synth.make_event_list(seed, ndm, nwidths, nout, nclumps=nclumps, nnoise=nnoise)
    widths = [1 << i for i in range(nwidths)]
    ref_l, ref = oracle.cluster_events(ev, widths, *params)
    nc, gl, got = _run(ev, ndm, widths, *params)
    log(f"seed {seed}: {len(ev)} events -> {nc} clusters")
    assert nc == len(ref)
    _same(gl, got, ref_l, [dict(r) for r in ref])


def test_small_config_pipeline_events():
    """Cluster the events the GPU search finds in the small beam."""
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    fb, dly, x, out = small_case()
    s = to_dev(out.astype(np.int32))
    nout = out.shape[1]
    pws = torch.empty(L.find_peaks_workspace_bytes(100, nout, fb.widths), dtype=torch.uint8,
                      device="cuda")
    cap = 1 << 14
    evb = torch.empty(cap * 40, dtype=torch.uint8, device="cuda")
    n = L.find_peaks(s, 100, nout, fb.widths, fb.snr_thresh, evb, cap, pws)
    ev = L.events_from_buffer(evb, n)
    for params in ((2, 1, 0), (1, 0, 0), (3, 2, 5)):
        ref_l, ref = oracle.cluster_events(ev, fb.widths, *params)
        nc, gl, got = _run(ev, 100, fb.widths, *params)
        log(f"small beam {params}: {n} events -> {nc} clusters")
        _same(gl, got, ref_l, ref)


def test_survey_beam_events():
    """The survey beam at full size: its events clustered on the GPU match
    the oracle's clustering of the same events."""
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    fb = survey_case()
    p = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    nout = fb.nsamps - p.max_delay
    ws = torch.empty(L.dedisp_workspace_bytes(p, fb.nsamps), dtype=torch.uint8, device="cuda")
    out = torch.empty((1200, nout), dtype=torch.int16, device="cuda")
    L.dedisp_execute(p, to_dev(fb.packed), fb.nsamps, out, ws)
    pws = torch.empty(L.find_peaks_workspace_bytes(1200, nout, fb.widths), dtype=torch.uint8,
                      device="cuda")
    evb = torch.empty((1 << 20) * 40, dtype=torch.uint8, device="cuda")
    n = L.find_peaks(out, 1200, nout, fb.widths, fb.snr_thresh, evb, 1 << 20, pws)
    ev = L.events_from_buffer(evb, n)
    ref_l, ref = oracle.cluster_events(ev, fb.widths, 2, 1, 0)
    nc, gl, got = _run(ev, 1200, fb.widths, 2, 1, 0)
    log(f"survey beam: {n} events -> {nc} clusters")
    _same(gl, got, ref_l, ref)
    # pulses that the search detected (events near their trial and arrival)
    # each map to a cluster of their own: one candidate per pulse, and the
    # clusters are far fewer than the events
    rep_of = []
    dmi, tpk = ev["dm_idx"].astype(np.int64), ev["t_peak"].astype(np.int64)
    for pu in fb.pulses:
        d = int(np.argmin(np.abs(fb.dm_list - pu.dm)))
        near = np.nonzero((np.abs(dmi - d) <= 2) & (np.abs(tpk - pu.t0) <= pu.width + 2))[0]
        if len(near):
            best = int(near[np.argmax(ev["snr"][near])])
            rep_of.append(int(ref_l[best]))
    log(f"{len(rep_of)} of {len(fb.pulses)} pulses detected, in {len(set(rep_of))} clusters")
    assert len(rep_of) >= len(fb.pulses) // 2
    assert len(set(rep_of)) == len(rep_of)
    assert nc < n // 50


def test_one_long_chain():
    """Every event a friend of the next: one cluster of 60000 events reached
    through long union-find chains."""
    ndm = 60000
    rows = [(w, d, 1000 + d, 1001 + d, 1000 + d, 5, np.float32(6 + (d * 7919 + w) % 97 / 8))
            for w in range(2) for d in range(ndm)]
    ev = np.array(rows, dtype=synth.EVENT_DTYPE)
    ref_l, ref = oracle.cluster_events(ev[:3000], [1, 2], 1, 0, 0)   # oracle on a prefix
    assert len(ref) == 1 and ref[0]["n_members"] == 3000
    nc, gl, got = _run(ev, ndm, [1, 2], 1, 1, 0)
    assert nc == 1 and (gl == 0).all()
    c = got[0]
    best = int(np.argmax(ev["snr"]))
    assert (int(c["rep"]), int(c["n_members"]), int(c["dm_lo"]), int(c["dm_hi"])) == \
        (best, 2 * ndm, 0, ndm - 1)
    assert (int(c["t_lo"]), int(c["t_hi"])) == (1000, 1001 + ndm - 1 + 1)


def test_empty_single_and_deterministic():
    nc, gl, got = _run(np.zeros(0, synth.EVENT_DTYPE), 10, [1], 1, 1, 0)
    assert nc == 0 and len(got) == 0
    one = np.array([(0, 3, 5, 9, 7, 11, np.float32(7.5))], synth.EVENT_DTYPE)
    nc, gl, got = _run(one, 10, [1, 2], 1, 1, 0)
    assert nc == 1 and gl.tolist() == [0]
    assert (int(got[0]["rep"]), int(got[0]["t_hi"]), float(got[0]["snr"])) == (0, 9, 7.5)
    ev = synth.make_event_list(9, 1200, 10, 1 << 20, nclumps=300, nnoise=5000)
    a = _run(ev, 1200, [1 << i for i in range(10)], 3, 1, 4)
    b = _run(ev, 1200, [1 << i for i in range(10)], 3, 1, 4)
    assert a[0] == b[0] and (a[1] == b[1]).all() and a[2].tobytes() == b[2].tobytes()


def test_capacity_keeps_the_first_clusters():
    from paper_1112_0065_amd import _lib as L
    ev = synth.make_event_list(12, 300, 6, 100000)
    widths = [1 << i for i in range(6)]
    ref_l, ref = oracle.cluster_events(ev, widths, 2, 1, 0)
    cap = len(ref) // 3
    with pytest.raises(L.DedispError) as ei:
        _run(ev, 300, widths, 2, 1, 0, capacity=cap)
    assert ei.value.status == L.ERR_CAPACITY and f"n_clusters={len(ref)}" in str(ei.value)
    # the same call with the buffer kept: records in order up to capacity
    torch = torch_dev()
    evd = to_dev(np.frombuffer(ev.tobytes(), np.uint8).copy())
    ws = torch.empty(L.dedisp_cluster_workspace_bytes(len(ev), 300, 6), dtype=torch.uint8, device="cuda")
    cb = torch.empty(cap * 72, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.DedispError):
        L.dedisp_cluster_events(evd, len(ev), 300, widths, 2, 1, 0, cb, cap, ws)
    got = L.clusters_from_buffer(cb, cap)
    assert [int(g["first"]) for g in got] == [c["first"] for c in ref[:cap]]


def test_bad_input_is_rejected():
    from paper_1112_0065_amd import _lib as L
    ev = synth.make_event_list(13, 100, 4, 50000)
    widths = [1, 2, 4, 8]
    cases = []
    e = ev.copy(); e[[3, 4]] = e[[4, 3]]; cases.append(("unsorted", e, 100))
    e = ev.copy(); e["dm_idx"][-1] = 100; cases.append(("dm out of range", e, 100))
    e = ev.copy(); e["snr"][5] = np.nan; cases.append(("nan snr", e, 100))
    e = ev.copy(); e["t_end"][7] = e["t_start"][7] - 1; cases.append(("t_end < t_start", e, 100))
    for name, e, ndm in cases:
        with pytest.raises(L.DedispError) as ei:
            _run(e, ndm, widths, 1, 1, 0)
        assert ei.value.status == L.ERR_INVALID_ARG, name
    # argument ranges are checked on the host
    with pytest.raises(L.DedispError):
        _run(ev, 100, widths, -1, 0, 0)
    with pytest.raises(L.DedispError):
        _run(ev, 100, widths, 1, 32, 0)
    with pytest.raises(L.DedispError):
        _run(ev, 100, [1, 0, 4, 8], 1, 1, 0)
    # the library still works afterwards
    nc, _, _ = _run(ev, 100, widths, 1, 1, 0)
    assert nc == len(oracle.cluster_events(ev, widths, 1, 1, 0)[1])
