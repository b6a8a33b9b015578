"""GPU test of the allocation-free peak finder (find_peaks_noalloc): its
events and counts equal find_peaks' on the same series, over two calls in a
row -- the second on a smaller input, so that the static scratch still holds
the first call's contents -- and inputs whose workspace exceeds the scratch
are refused before any launch."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import events_equal, log, torch_dev

pytestmark = pytest.mark.gpu

WIDTHS = [1, 2, 4, 8, 16, 32, 64]


def _case(seed, ndm, nsamps, dm_max):
    """A dedispersed seeded beam (the small-config recipe at 256 channels)."""
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    fb = synth.make_beam(seed, nsamps, dm_max, 6, nchans=256, df=-400.0 / 256, ndm=ndm,
                         widths=WIDTHS, snr_thresh=5.0, name=f"na{seed}")
    p = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    nout = fb.nsamps - p.max_delay
    inp = torch.from_numpy(fb.packed).cuda()
    ws = torch.empty(L.dedisp_workspace_bytes(p, fb.nsamps), dtype=torch.uint8, device="cuda")
    out = torch.empty((ndm, nout), dtype=torch.int16, device="cuda")
    L.dedisp_execute(p, inp, fb.nsamps, out, ws)
    torch.cuda.synchronize()
    return fb, out, ndm, nout


def _both(out, ndm, nout, k):
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    cap = 1 << 16
    pws = torch.empty(L.find_peaks_workspace_bytes(ndm, nout, WIDTHS), dtype=torch.uint8,
                      device="cuda")
    ev_a = torch.empty(cap * 40, dtype=torch.uint8, device="cuda")
    ev_b = torch.empty(cap * 40, dtype=torch.uint8, device="cuda")
    na = L.find_peaks(out, ndm, nout, WIDTHS, k, ev_a, cap, pws)
    nb = L.find_peaks_noalloc(out, ndm, nout, WIDTHS, k, ev_b, cap)
    return na, nb, L.events_from_buffer(ev_a, na), L.events_from_buffer(ev_b, nb)


def test_noalloc_equals_find_peaks_twice_then_smaller():
    torch_dev()
    big = _case(61, 96, 60000, 150.0)
    small = _case(62, 24, 12000, 60.0)
    for fb, out, ndm, nout in (big, small):
        log("no-alloc find_peaks", fb.name, ndm, nout)
        na, nb, ea, eb = _both(out, ndm, nout, fb.snr_thresh)
        log("  events", na, nb)
        assert na == nb and na > 0
        assert ea.tobytes() == eb.tobytes()
        # and the oracle agrees on the smaller case's series
        if ndm == 24:
            ser = out.cpu().numpy().view(np.uint16).astype(np.int64)
            events_equal(eb, oracle.find_events(oracle.boxcar(ser, WIDTHS), fb.snr_thresh))


def test_noalloc_refuses_inputs_beyond_the_scratch():
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    ndm, nout = 1200, 1 << 20
    assert L.find_peaks_workspace_bytes(ndm, nout, WIDTHS) > (32 << 20)
    series = torch.zeros((ndm, nout), dtype=torch.int16, device="cuda")
    ev = torch.empty(40 * 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.DedispError) as e:
        L.find_peaks_noalloc(series, ndm, nout, WIDTHS, 6.0, ev, 16)
    assert e.value.status == L.ERR_UNSUPPORTED
    del series
