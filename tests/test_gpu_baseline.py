"""GPU parity of baseline (red-noise) removal (section 2.3) against the
oracle through the C ABI, and what it buys the search: a slow baseline
wiggle inflates every series' sigma so that the sigma-cut misses the
injected pulses; with the running mean removed they are all found."""
import numpy as np
import pytest

import oracle
from gpu_common import events_equal, log, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def _dev(a, u16):
    return to_dev(a.astype(np.uint16).view(np.int16) if u16 else a.astype(np.int32))


def _run(series, radius, offset, in_u16, out_u16):
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    ndm, nout = series.shape
    out = torch.empty((ndm, nout - 2 * radius), dtype=torch.int16 if out_u16 else torch.int32,
                      device="cuda")
    L.baseline_remove(_dev(series, in_u16), ndm, nout, radius, offset, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return o.view(np.uint16).astype(np.int64) if out_u16 else o.astype(np.int64)


@pytest.mark.parametrize("radius", [0, 1, 7, 2048, 8192])
def test_matches_oracle(radius):
    rng = np.random.default_rng(radius)
    nout = 30001 + 2 * radius
    s = rng.integers(0, 3073, size=(5, nout))
    ref = oracle.baseline_remove(s, radius, 3072)
    for in_u16, out_u16 in [(True, True), (True, False), (False, True), (False, False)]:
        got = _run(s, radius, 3072, in_u16, out_u16)
        assert (got == ref).all(), (radius, in_u16, out_u16)


def test_red_noise_removed_pulses_kept():
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    rng = np.random.default_rng(3)
    ndm, nout = 8, 200_000
    t = np.arange(nout)
    noise = np.rint(30 * rng.standard_normal((ndm, nout))).astype(np.int64)
    wiggle = np.rint(40 * np.sin(2 * np.pi * t / 20000.0)).astype(np.int64)
    s = 1536 + noise + wiggle
    pulses = [(20000, 16), (77000, 64), (150000, 4)]
    for t0, w in pulses:
        s[:, t0:t0 + w] += int(round(12 * 30 / np.sqrt(w)))      # S/N ~12 at width w
    widths = [1, 4, 16, 64, 256]

    def search(series):
        n = series.shape[1]
        ws = torch.empty(L.find_peaks_workspace_bytes(ndm, n, widths), dtype=torch.uint8,
                         device="cuda")
        evb = torch.empty((1 << 18) * 40, dtype=torch.uint8, device="cuda")
        k = L.find_peaks(_dev(series, True), ndm, n, widths, 6.0, evb, 1 << 18, ws)
        return L.events_from_buffer(evb, k)

    R = 1024
    flat = _run(s, R, 3072, True, True)
    assert (flat == oracle.baseline_remove(s, R, 3072)).all()
    before, after = search(s), search(flat)

    def near(ev, shift):
        return np.array([any(abs(int(e["t_peak"]) + shift - t0) <= w + 300 for t0, w in pulses)
                         for e in ev], bool)

    nb, na = near(before, 0), near(after, R)

    def found(ev, shift):
        return sum(any(abs(int(e["t_peak"]) + shift - t0) <= w + 300 for e in ev)
                   for t0, w in pulses)

    log("events before", len(before), "false", int((~nb).sum()), "pulses found", found(before, 0),
        "| after", len(after), "false", int((~na).sum()), "pulses found", found(after, R))
    # the wiggle inflates every series' sigma and hides the pulses; with the
    # running mean removed every pulse is found, with no false events
    assert found(before, 0) < len(pulses) and found(after, R) == len(pulses)
    assert (~na).sum() <= 2 and na.sum() > 10 * max(1, nb.sum())
    # the events of the flattened series are those of the oracle chain
    events_equal(after, oracle.find_events(oracle.boxcar(oracle.baseline_remove(s, R, 3072),
                                                         widths), 6.0))


def test_bad_arguments():
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    s = _dev(np.zeros((2, 100), np.int64), True)
    out = torch.empty((2, 100), dtype=torch.int16, device="cuda")
    for r, st in [(-1, L.ERR_INVALID_ARG), (8193, L.ERR_INVALID_ARG), (50, L.ERR_TOO_FEW_SAMPLES)]:
        with pytest.raises(L.DedispError) as e:
            L.baseline_remove(s, 2, 100, r, 0, out)
        assert e.value.status == st
