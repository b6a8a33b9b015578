"""Host-side candidate export and baseband-dump trigger windows (no GPU:
pure host code behind the C ABI)."""
import numpy as np
import pytest

from paper_1112_0065_amd import _lib as L


def _clusters(rows):
    c = np.zeros(len(rows), L.CLUSTER_DTYPE)
    for k, r in enumerate(rows):
        for name, v in r.items():
            c[k][name] = v
    return c


def test_candidate_list_round_trip(tmp_path):
    rows = [dict(first=0, rep=3, t_lo=100, t_hi=140, t_peak=120, n_members=12, dm_lo=4, dm_hi=9,
                 w_lo=0, w_hi=2, dm_idx=6, width_idx=1, snr=np.float32(11.3)),
            dict(first=5, rep=5, t_lo=9000, t_hi=9001, t_peak=9000, n_members=1, dm_lo=0, dm_hi=0,
                 w_lo=0, w_hi=0, dm_idx=0, width_idx=0, snr=np.float32(6.0000005))]
    c = _clusters(rows)
    dm_list = np.array([0.0, 0.1, 0.2, 0.30000000000000004, 1.5, 2.25, 3.1, 4.0, 5.0, 6.0])
    path = tmp_path / "cands.txt"
    L.dedisp_write_candidates(path, c, dm_list, [1, 2, 4], 64e-6, t_offset=1 << 20, beam=7)
    lines = path.read_text().splitlines()
    assert lines[0].startswith("# snr t_peak time_s dm")
    assert len(lines) == 3
    for line, r in zip(lines[1:], rows):
        f = line.split()
        assert np.float32(float(f[0])) == r["snr"]
        assert int(f[1]) == r["t_peak"] + (1 << 20)
        assert float(f[2]) == (r["t_peak"] + (1 << 20)) * 64e-6
        assert float(f[3]) == dm_list[r["dm_idx"]]
        assert [int(x) for x in f[4:]] == [r["dm_idx"], [1, 2, 4][r["width_idx"]], r["width_idx"],
                                            r["n_members"], r["t_lo"] + (1 << 20),
                                            r["t_hi"] + (1 << 20), r["dm_lo"], r["dm_hi"], 7]
    with pytest.raises(L.DedispError):
        bad = c.copy()
        bad["dm_idx"][0] = 10
        L.dedisp_write_candidates(path, bad, dm_list, [1, 2, 4], 64e-6)


def test_trigger_windows_by_hand():
    # 3 trials x 4 channels
    delays = np.array([[0, 1, 2, 3], [0, 2, 4, 6], [0, 3, 6, 9]], np.int32)
    rows = [dict(t_lo=10, t_hi=12, dm_lo=0, dm_hi=1, n_members=5, snr=np.float32(9.0)),   # 10..18
            dict(t_lo=19, t_hi=19, dm_lo=2, dm_hi=2, n_members=2, snr=np.float32(12.0)),  # 19..28
            dict(t_lo=40, t_hi=41, dm_lo=0, dm_hi=0, n_members=1, snr=np.float32(20.0)),  # members < 2
            dict(t_lo=50, t_hi=50, dm_lo=1, dm_hi=2, n_members=3, snr=np.float32(5.0)),   # snr < 6
            dict(t_lo=95, t_hi=99, dm_lo=2, dm_hi=2, n_members=9, snr=np.float32(7.0))]   # clipped
    c = _clusters(rows)
    w = L.dedisp_trigger_windows(c, delays, 6.0, 2, 0, 100)
    # windows 10..18 and 19..28 touch and merge; the last ends at the data's end
    assert [(int(x["start"]), int(x["end"]), float(x["snr"]), int(x["cluster"]), int(x["n_clusters"]))
            for x in w] == [(10, 29, 12.0, 1, 2), (95, 100, 7.0, 4, 1)]
    w = L.dedisp_trigger_windows(c, delays, 6.0, 1, 3, 100)
    assert [(int(x["start"]), int(x["end"])) for x in w] == [(7, 32), (37, 48), (92, 100)]
    with pytest.raises(L.DedispError) as ei:
        L.dedisp_trigger_windows(c, delays, 6.0, 1, 3, 100, capacity=2)
    assert ei.value.status == L.ERR_CAPACITY and "n_windows=3" in str(ei.value)
    assert len(L.dedisp_trigger_windows(c[:0], delays, 6.0, 1, 0, 100)) == 0


def test_trigger_windows_cover_exactly_the_selected_samples():
    rng = np.random.default_rng(3)
    ndm, nchans, nsamps = 40, 16, 5000
    delays = np.sort(rng.integers(0, 300, size=(ndm, nchans)), axis=1).astype(np.int32)
    delays[:, 0] = 0
    n = 300
    t_lo = rng.integers(0, nsamps, n)
    dlo = rng.integers(0, ndm, n)
    rows = [dict(t_lo=int(t_lo[k]), t_hi=int(t_lo[k] + rng.integers(0, 30)), dm_lo=int(dlo[k]),
                 dm_hi=int(min(ndm - 1, dlo[k] + rng.integers(0, 5))), n_members=int(rng.integers(1, 9)),
                 snr=np.float32(rng.choice([6.0, 7.5, 9.0, 11.0]))) for k in range(n)]
    c = _clusters(rows)
    pad = 7
    w = L.dedisp_trigger_windows(c, delays, 7.0, 3, pad, nsamps)
    want = np.zeros(nsamps + 1, bool)
    best = {}
    for k, r in enumerate(rows):
        if r["snr"] < 7.0 or r["n_members"] < 3:
            continue
        sl = delays[r["dm_lo"]:r["dm_hi"] + 1]
        s = max(0, r["t_lo"] + int(sl.min()) - pad)
        e = min(nsamps, r["t_hi"] + int(sl.max()) + pad + 1)
        want[s:e] = True
        best[k] = (s, e)
    got = np.zeros(nsamps + 1, bool)
    for x in w:
        got[x["start"]:x["end"]] = True
    assert (got == want).all()
    # sorted, disjoint and not touching; each window's snr is its strongest cluster's
    assert all(w["end"][:-1] < w["start"][1:])
    for x in w:
        inside = [k for k, (s, e) in best.items() if s >= x["start"] and e <= x["end"]]
        assert x["n_clusters"] == len(inside)
        top = max(rows[k]["snr"] for k in inside)
        assert x["snr"] == top and x["cluster"] == min(k for k in inside if rows[k]["snr"] == top)


def test_candidate_nms_equals_oracle():
    """The library's per-width non-maximum suppression keeps exactly the
    oracle's candidates, on seeded event lists with many S/N ties, events on
    the window boundaries, and several widths (host code, no GPU)."""
    import oracle
    from paper_1112_0065_amd import _lib as L
    widths = [1, 2, 4, 8, 16]
    for seed in range(8):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(0, 2500))
        ev = np.zeros(n, dtype=L.EVENT_DTYPE)
        ev["width_idx"] = rng.integers(0, len(widths), n)
        ev["dm_idx"] = rng.integers(0, 400, n)
        ev["t_peak"] = rng.integers(0, 200000, n)
        # boundary cases: pairs exactly 32 trials or 128 w samples apart
        k = n // 10
        if k:
            ev["dm_idx"][:k] = 100 + 32 * rng.integers(0, 3, k)
            ev["t_peak"][:k] = 5000 + 128 * np.array(widths)[ev["width_idx"][:k]] * rng.integers(0, 3, k)
        ev["t_start"] = ev["t_peak"] - 1
        ev["t_end"] = ev["t_peak"] + 1
        ev["snr"] = np.round(rng.uniform(6, 12, n), 1).astype(np.float32)
        got = L.dedisp_candidates_nms(ev, widths)
        want = oracle.nms(ev, widths)
        assert list(got) == want, seed
    with pytest.raises(L.DedispError):
        bad = np.zeros(1, dtype=L.EVENT_DTYPE)
        bad["width_idx"] = 7
        L.dedisp_candidates_nms(bad, widths)
