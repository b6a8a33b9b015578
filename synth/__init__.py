"""Seeded synthetic 2-bit filterbank generator.

This module only *makes inputs*: Gaussian noise, a 2-bit quantiser, a forward
model of dispersed pulses arriving from the sky, simple RFI, and the packing
of samples into the time-major 2-bit byte stream that the library ingests.
It holds none of the search method's arithmetic (no delay table, no
dedispersion, no boxcar, no statistics) and serves both the oracle and the
HIP path with identical bytes.

Shapes follow the survey backend of the paper's introduction: 1024 channels
over 400 MHz centred at 1381.8 MHz, 64 us sampling, 2 bits per sample,
13 beams, ~1200 DM trials (section 2.2).

Random streams (NumPy PCG64):
  * noise: ``default_rng(SeedSequence(seed).spawn(2)[0])``, standard normals
    drawn time-major in blocks of ``block`` samples x nchans channels;
  * pulse parameters: ``default_rng(SeedSequence(seed).spawn(2)[1])``, drawn
    in a fixed order before any noise is generated.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# Survey-backend constants (paper, section 1).
# ---------------------------------------------------------------------------
TSAMP = 64e-6            # s
F_TOP = 1581.8           # MHz: 1381.8 + 400/2, highest channel
DF_SURVEY = -400.0 / 1024.0   # MHz per channel, 1024 channels
NBEAMS = 13

# Quantiser edges of the 2-bit digitiser model: levels 0..3.
QUANT_EDGES = (-0.98, 0.0, 0.98)

# Sky model: the dispersion sweep of a pulse as seen by the receiver, in
# milliseconds, for frequencies in GHz (4.148808 ms GHz^2 per unit DM).
_SKY_SWEEP_MS_GHZ2 = 4.148808


def quantise(x: np.ndarray) -> np.ndarray:
    """Map float samples to 2-bit levels: <-0.98 -> 0, [-0.98,0) -> 1,
    [0,0.98) -> 2, >=0.98 -> 3."""
    q = (x >= QUANT_EDGES[0]).astype(np.uint8)
    q += (x >= QUANT_EDGES[1])
    q += (x >= QUANT_EDGES[2])
    return q


def pack_2bit(q: np.ndarray) -> np.ndarray:
    """Pack levels ``q[t][c]`` (uint8 0..3, time-major) into the byte stream:
    byte ``t*nchans/4 + c/4`` holds channel c in bits ``2*(c%4)``
    (least-significant pair first)."""
    nsamps, nchans = q.shape
    assert nchans % 4 == 0
    q4 = q.reshape(nsamps, nchans // 4, 4).astype(np.uint8)
    b = q4[..., 0] | (q4[..., 1] << 2) | (q4[..., 2] << 4) | (q4[..., 3] << 6)
    return np.ascontiguousarray(b.reshape(-1))


def sky_arrival_offsets(nchans: int, f_top: float, df: float, tsamp: float,
                        dm: float) -> np.ndarray:
    """Forward model of a dispersed pulse: the sample, relative to its arrival
    at ``f_top``, in which the pulse reaches each channel's frequency.

    Arrival lag t(f) = 4.148808 ms * DM * (f_GHz^-2 - ftop_GHz^-2); the pulse
    lands in sample floor(t/tsamp + 1/2).  This is a model of the sky, written
    in its own units; it is not the search's delay table.
    """
    f_ghz = (f_top + df * np.arange(nchans, dtype=np.float64)) * 1e-3
    ft_ghz = f_top * 1e-3
    lag_ms = _SKY_SWEEP_MS_GHZ2 * dm * (f_ghz ** -2 - ft_ghz ** -2)
    return np.floor(lag_ms / (tsamp * 1e3) + 0.5).astype(np.int64)


def dm_list_linear(ndm: int, dm_max: float) -> np.ndarray:
    """DM_k = dm_max * k / (ndm - 1), endpoints included."""
    return np.array([dm_max * k / (ndm - 1) for k in range(ndm)], dtype=np.float64)


def dm_list_expm1(ndm: int, dm_max: float, scale: float = 500.0) -> np.ndarray:
    """DM_k = dm_max * expm1(k/scale) / expm1((ndm-1)/scale): spacing grows
    with DM (0.2 at DM 0 to ~2.2 at DM 1000 for 1200 trials to 1000); the
    last entry is exactly dm_max."""
    den = math.expm1((ndm - 1) / scale)
    return np.array([dm_max * (math.expm1(k / scale) / den) for k in range(ndm)],
                    dtype=np.float64)


@dataclasses.dataclass
class Pulse:
    dm: float
    width: int          # samples
    t0: int             # arrival sample at f_top
    amp: float          # float-domain amplitude (0 for level-step pulses)
    snr: float = 0.0    # nominal S/N (float-domain pulses)
    dm_idx: int = -1    # trial index when injected on the trial grid


@dataclasses.dataclass
class Filterbank:
    """One beam of packed 2-bit data plus the truth of every injection."""
    name: str
    seed: int
    nchans: int
    nsamps: int
    f_top: float
    df: float
    tsamp: float
    dm_list: np.ndarray
    widths: List[int]
    snr_thresh: float
    packed: np.ndarray              # uint8 [nsamps * nchans / 4]
    pulses: List[Pulse]
    rfi: dict = dataclasses.field(default_factory=dict)

    @property
    def sha256(self) -> str:
        return hashlib.sha256(self.packed.tobytes()).hexdigest()

    def params(self) -> dict:
        return dict(name=self.name, seed=self.seed, nchans=self.nchans,
                    nsamps=self.nsamps, f_top=self.f_top, df=self.df,
                    tsamp=self.tsamp, ndm=len(self.dm_list),
                    dm_max=float(self.dm_list[-1]), widths=list(self.widths),
                    snr_thresh=self.snr_thresh, npulses=len(self.pulses),
                    numpy=np.__version__)


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    s_noise, s_par = ss.spawn(2)
    return np.random.default_rng(s_noise), np.random.default_rng(s_par)


def _noise_levels(rng: np.random.Generator, nsamps: int, nchans: int,
                  inject, block: int = 1 << 15) -> np.ndarray:
    """Draw N(0,1) noise block by block (time-major), let ``inject(x, t_lo)``
    add float-domain signals to the block, quantise and pack it."""
    out = np.empty(nsamps * nchans // 4, dtype=np.uint8)
    for t_lo in range(0, nsamps, block):
        n = min(block, nsamps - t_lo)
        x = rng.standard_normal((n, nchans), dtype=np.float32)
        if inject is not None:
            inject(x, t_lo)
        out[t_lo * nchans // 4:(t_lo + n) * nchans // 4] = pack_2bit(quantise(x))
    return out


def _add_window(x: np.ndarray, t_lo: int, c: int, a: int, b: int, val: float):
    """x[t - t_lo, c] += val for t in [a, b) clipped to the block."""
    lo = max(a, t_lo)
    hi = min(b, t_lo + x.shape[0])
    if lo < hi:
        x[lo - t_lo:hi - t_lo, c] += val


def _float_pulse_injector(pulses: Sequence[Pulse], offsets: Sequence[np.ndarray]):
    def inject(x, t_lo):
        n = x.shape[0]
        for p, off in zip(pulses, offsets):
            starts = p.t0 + off
            hit = np.nonzero((starts < t_lo + n) & (starts + p.width > t_lo))[0]
            for c in hit:
                _add_window(x, t_lo, int(c), int(starts[c]), int(starts[c]) + p.width,
                            p.amp)
    return inject


# ---------------------------------------------------------------------------
# Configurations.
# ---------------------------------------------------------------------------

def make_small(seed: int = 1) -> Filterbank:
    """CPU-scale case: 256 channels from 1581.8 MHz down in steps of
    1.5625 MHz, 64 us, 2^15 samples, 100 trials linear over DM 0..200,
    widths 1..64 (powers of two), S/N > 6.  Five dispersed boxcar pulses on
    the trial grid (width 1..16) that raise the 2-bit level by one (capped
    at 3) along their sweep."""
    nchans, nsamps, f_top, df = 256, 1 << 15, F_TOP, -1.5625
    dm_list = dm_list_linear(100, 200.0)
    rng_n, rng_p = _streams(seed)
    sweep_max = int(sky_arrival_offsets(nchans, f_top, df, TSAMP, dm_list[-1]).max())
    span_hi = nsamps - sweep_max - 128
    slot = (span_hi - 64) // 5
    pulses = []
    for i in range(5):
        di = int(rng_p.integers(0, 100))
        w = int(rng_p.integers(1, 17))
        t0 = 64 + i * slot + int(rng_p.integers(0, slot - 16))
        pulses.append(Pulse(dm=float(dm_list[di]), width=w, t0=t0, amp=0.0,
                            dm_idx=di))
    packed = _noise_levels(rng_n, nsamps, nchans, None)
    q = _unpack_levels(packed, nsamps, nchans)
    for p in pulses:
        off = sky_arrival_offsets(nchans, f_top, df, TSAMP, p.dm)
        for c in range(nchans):
            s = p.t0 + int(off[c])
            seg = q[s:s + p.width, c]
            np.minimum(seg + 1, 3, out=seg)
    packed = pack_2bit(q)
    return Filterbank("small_256ch_2^15", seed, nchans, nsamps, f_top, df, TSAMP,
                      dm_list, [1, 2, 4, 8, 16, 32, 64], 6.0, packed, pulses)


def _unpack_levels(packed: np.ndarray, nsamps: int, nchans: int) -> np.ndarray:
    """Inverse of :func:`pack_2bit` (generator-side, used to apply level-step
    injections after quantisation)."""
    b = packed.reshape(nsamps, nchans // 4)
    q = np.empty((nsamps, nchans // 4, 4), dtype=np.uint8)
    for k in range(4):
        q[..., k] = (b >> (2 * k)) & 3
    return q.reshape(nsamps, nchans)


def _snr_pulses(rng_p: np.random.Generator, npulses: int, nchans: int,
                nsamps: int, dm_lo: float, dm_hi: float, f_top: float, df: float,
                tsamp: float, snr_lo: float = 6.0, snr_hi: float = 30.0,
                w_max: int = 500) -> List[Pulse]:
    """Pulses with DM ~ U(dm_lo, dm_hi), width round(exp(U(0, ln w_max)))
    samples, nominal S/N ~ U(snr_lo, snr_hi); t0 stratified into ``npulses``
    equal slots of the range where the whole sweep fits, with a margin of
    one width.  Float amplitude A = S/N / sqrt(nchans * W)."""
    dms = rng_p.uniform(dm_lo, dm_hi, npulses)
    ws = np.rint(np.exp(rng_p.uniform(0.0, math.log(w_max), npulses))).astype(int)
    ws = np.maximum(ws, 1)
    snrs = rng_p.uniform(snr_lo, snr_hi, npulses)
    u = rng_p.uniform(0.0, 1.0, npulses)
    sweep_max = int(sky_arrival_offsets(nchans, f_top, df, tsamp, dm_hi).max())
    usable = nsamps - sweep_max - 2 * w_max - 2
    slot = usable / npulses
    pulses = []
    for i in range(npulses):
        w = int(ws[i])
        lo = w_max + i * slot
        t0 = int(lo + u[i] * max(slot - w, 1.0))
        amp = float(snrs[i] / math.sqrt(nchans * w))
        pulses.append(Pulse(dm=float(dms[i]), width=w, t0=t0, amp=amp,
                            snr=float(snrs[i])))
    return pulses


def make_beam(seed: int, nsamps: int, dm_max: float, npulses: int,
              nchans: int = 1024, f_top: float = F_TOP,
              df: float = DF_SURVEY, ndm: int = 1200,
              widths: Optional[List[int]] = None, snr_thresh: float = 6.0,
              name: str = "beam") -> Filterbank:
    """Survey-shaped beam: noise + float-domain dispersed boxcar pulses."""
    rng_n, rng_p = _streams(seed)
    dm_list = dm_list_expm1(ndm, dm_max)
    pulses = _snr_pulses(rng_p, npulses, nchans, nsamps, 0.0, dm_max, f_top, df,
                         TSAMP)
    offs = [sky_arrival_offsets(nchans, f_top, df, TSAMP, p.dm) for p in pulses]
    packed = _noise_levels(rng_n, nsamps, nchans, _float_pulse_injector(pulses, offs))
    if widths is None:
        widths = [1 << i for i in range(10)]
    return Filterbank(name, seed, nchans, nsamps, f_top, df, TSAMP, dm_list,
                      list(widths), snr_thresh, packed, pulses)


def make_survey_beam(seed: int = 2) -> Filterbank:
    """Survey-shaped single beam: 1024 channels, 2^19 samples (33.55 s),
    1200 trials to DM 1000 with growing spacing, 50 pulses, widths 1..512."""
    return make_beam(seed, 1 << 19, 1000.0, 50, name="survey_1024ch_2^19")


def multibeam_shapes(nbeams: int = NBEAMS):
    """Per-beam (nsamps, dm_max) of the uneven 13-beam batch:
    nsamps_b = 2^17 + 2^15 * b, dm_max_b = 500 + 125 * ((5b) mod 13)."""
    return [((1 << 17) + (1 << 15) * b, 500.0 + 125.0 * ((5 * b) % 13))
            for b in range(nbeams)]


def make_multibeam_beam(b: int) -> Filterbank:
    nsamps, dm_max = multibeam_shapes()[b]
    return make_beam(300 + b, nsamps, dm_max, 10, name=f"multibeam_b{b}")


@dataclasses.dataclass
class Impulse:
    t: int          # first sample
    width: int      # samples
    amp: float      # added to every channel (float domain, units of sigma)


def make_rfi_beam(seed: int, nsamps: int = 1 << 17, dm_max: float = 1000.0,
                  npulses: int = 8, nchans: int = 1024, ndm: int = 1200,
                  impulse_rate: float = 0.5, name: str = "rfi_beam") -> Filterbank:
    """Survey-shaped beam with dispersed pulses and three kinds of
    interference (the paper's section 2.1 names interference as the main
    source of false events; its forms here are a model):
      * zero-DM broadband impulses: Poisson, `impulse_rate` per second,
        width U{1..8} samples, amplitude U(2, 6) sigma in every channel;
      * persistent narrowband channels: 5% of channels with +1 sigma offset
        and twice the noise sigma;
      * 50 Hz periodic interference: 16-sample pulses every 312.5 samples
        (start rounded half away from zero) on a contiguous 10% band at
        1 sigma, active inside one random 2 s window.
    Pulses follow the survey recipe (DM U(0, dm_max), width log-uniform
    1..500 samples, nominal S/N U(6, 30))."""
    rng_n, rng_p = _streams(seed)
    dm_list = dm_list_expm1(ndm, dm_max)
    df = -400.0 / nchans
    pulses = _snr_pulses(rng_p, npulses, nchans, nsamps, 0.0, dm_max, F_TOP, df, TSAMP)
    offs = [sky_arrival_offsets(nchans, F_TOP, df, TSAMP, p.dm) for p in pulses]
    dur = nsamps * TSAMP
    nimp = int(rng_p.poisson(impulse_rate * dur))
    imps = [Impulse(int(rng_p.integers(0, nsamps - 8)), int(rng_p.integers(1, 9)),
                    float(rng_p.uniform(2.0, 6.0))) for _ in range(nimp)]
    nb = rng_p.choice(nchans, size=max(1, nchans // 20), replace=False)
    band0 = int(rng_p.integers(0, nchans - nchans // 10))
    band = np.arange(band0, band0 + nchans // 10)
    win0 = int(rng_p.integers(0, max(1, nsamps - int(2.0 / TSAMP))))
    win1 = min(nsamps, win0 + int(2.0 / TSAMP))
    starts = []
    k = 0
    while True:
        s = math.floor(312.5 * k + 0.5)
        if s >= nsamps:
            break
        if win0 <= s < win1:
            starts.append(s)
        k += 1
    pulse_inj = _float_pulse_injector(pulses, offs)

    def inject(x, t_lo):
        n = x.shape[0]
        x[:, nb] = x[:, nb] * 2.0 + 1.0
        pulse_inj(x, t_lo)
        for im in imps:
            lo, hi = max(im.t, t_lo), min(im.t + im.width, t_lo + n)
            if lo < hi:
                x[lo - t_lo:hi - t_lo, :] += im.amp
        for s in starts:
            lo, hi = max(s, t_lo), min(s + 16, t_lo + n)
            if lo < hi:
                x[lo - t_lo:hi - t_lo, band] += 1.0

    packed = _noise_levels(rng_n, nsamps, nchans, inject)
    return Filterbank(name, seed, nchans, nsamps, F_TOP, df, TSAMP, dm_list,
                      [1 << i for i in range(10)], 6.0, packed, pulses,
                      rfi=dict(impulses=imps, narrowband=nb.tolist(), band=[band0, band0 + nchans // 10],
                               periodic_window=[win0, win1]))


def make_coincidence_beams(seed: int, nbeams: int = NBEAMS, nsamps: int = 1 << 17,
                           nchans: int = 1024, npulses: int = 2, impulse_rate: float = 2.0,
                           dm_max: float = 1000.0):
    """Beams of one receiver over the same samples, for the coincidence mask:
    independent noise and dispersed pulses per beam (survey recipe), plus
    broadband zero-DM impulses common to all beams -- Poisson, `impulse_rate`
    per second, width U{1..8} samples -- whose amplitude differs per beam,
    U(0.5, 3) sigma per channel.  Returns (list of packed arrays, impulses,
    amplitudes [impulse][beam], pulses per beam)."""
    root = np.random.default_rng(np.random.SeedSequence([seed, 77]))
    df = -400.0 / nchans
    nimp = int(root.poisson(impulse_rate * nsamps * TSAMP))
    imps = [Impulse(int(root.integers(0, nsamps - 8)), int(root.integers(1, 9)), 0.0)
            for _ in range(nimp)]
    amps = root.uniform(0.5, 3.0, (nimp, nbeams))
    packed, pulses_all = [], []
    for b in range(nbeams):
        rng_n, rng_p = _streams(seed * 1000 + b)
        pulses = _snr_pulses(rng_p, npulses, nchans, nsamps, 0.0, dm_max, F_TOP, df, TSAMP)
        offs = [sky_arrival_offsets(nchans, F_TOP, df, TSAMP, p.dm) for p in pulses]
        pulse_inj = _float_pulse_injector(pulses, offs)

        def inject(x, t_lo, b=b, pulse_inj=pulse_inj):
            n = x.shape[0]
            pulse_inj(x, t_lo)
            for i, im in enumerate(imps):
                lo, hi = max(im.t, t_lo), min(im.t + im.width, t_lo + n)
                if lo < hi:
                    x[lo - t_lo:hi - t_lo, :] += amps[i, b]

        packed.append(_noise_levels(rng_n, nsamps, nchans, inject))
        pulses_all.append(pulses)
    return packed, imps, amps, pulses_all


def fast_levels(rng: np.random.Generator, nsamps: int, nchans: int) -> np.ndarray:
    """2-bit levels with the quantiser's level probabilities (0.163543,
    0.336457, 0.336457, 0.163543) drawn directly from 16-bit uniforms -- a
    faster stand-in for quantised Gaussian noise, time-major [nsamps][nchans]."""
    u = np.frombuffer(rng.bytes(2 * nsamps * nchans), dtype=np.uint16).reshape(nsamps, nchans)
    q = (u >= 10718).astype(np.uint8)
    q += (u >= 32768)
    q += (u >= 54818)
    return q


def fast_chunk(seed: int, nsamps: int, nchans: int = 1024, f_top: float = F_TOP,
               df: float = DF_SURVEY, npulses: int = 5, dm_max: float = 1000.0) -> np.ndarray:
    """Packed chunk of fast-level noise with `npulses` dispersed boxcar pulses
    (throughput inputs).  A pulse of width W and nominal S/N s raises the
    level by one (capped at 3) along its sweep in a random fraction
    f = s * 0.95 / (0.84 * sqrt(nchans * W)) of the channels (a +1 step adds
    ~0.84 on average; one level's sigma is 0.95)."""
    rng = np.random.default_rng(seed)
    q = fast_levels(rng, nsamps, nchans)
    for _ in range(npulses):
        dm = float(rng.uniform(0, dm_max))
        w = int(rng.integers(1, 65))
        snr = float(rng.uniform(8.0, 30.0))
        frac = min(1.0, snr * 0.95 / (0.84 * math.sqrt(nchans * w)))
        chans = np.nonzero(rng.uniform(size=nchans) < frac)[0]
        off = sky_arrival_offsets(nchans, f_top, df, TSAMP, dm)
        if off.max() + w + 1 >= nsamps:
            continue
        t0 = int(rng.integers(0, nsamps - off.max() - w))
        for c in chans:
            seg = q[t0 + off[c]:t0 + off[c] + w, c]
            np.minimum(seg + 1, 3, out=seg)
    return pack_2bit(q)


def make_tiny(seed: int, nchans: int, nsamps: int, dm_list: Sequence[float],
              f_top: float = F_TOP, df: float = -12.5, tsamp: float = TSAMP,
              widths: Sequence[int] = (1, 2, 4), snr_thresh: float = 3.0,
              levels: Optional[np.ndarray] = None) -> Filterbank:
    """Uniform random 2-bit levels (or the given ``levels[t][c]``) for small
    parity and edge cases."""
    rng = np.random.default_rng(seed)
    if levels is None:
        levels = rng.integers(0, 4, size=(nsamps, nchans), dtype=np.uint8)
    packed = pack_2bit(np.asarray(levels, dtype=np.uint8))
    return Filterbank(f"tiny_{nchans}x{nsamps}", seed, nchans, nsamps, f_top, df,
                      tsamp, np.asarray(dm_list, dtype=np.float64), list(widths),
                      snr_thresh, packed, [])


# ---------------------------------------------------------------------------
# Event lists for the clustering stage.
# ---------------------------------------------------------------------------

EVENT_DTYPE = np.dtype([("width_idx", "<i4"), ("dm_idx", "<i4"), ("t_start", "<i8"),
                        ("t_end", "<i8"), ("t_peak", "<i8"), ("b_peak", "<i4"),
                        ("snr", "<f4")])


def make_event_list(seed: int, ndm: int, nwidths: int, nout: int, nclumps: int = 20,
                    nnoise: int = 200, dm_extent: int = 40, max_run: int = 6,
                    snr_levels: int = 16) -> np.ndarray:
    """A valid find_peaks-style event list (structured, EVENT_DTYPE): events in
    (width_idx, dm_idx, t_start) order, runs of one series maximal (a gap of
    at least one sample) and inside [0, nout).

    Clumps imitate a dispersed pulse: a range of up to ``dm_extent`` trials
    and a range of widths, with a run in each (trial, width) whose start
    drifts by a sample or two per trial; noise events are isolated runs at
    random places.  snr takes one of ``snr_levels`` values so that ties
    occur."""
    rng = np.random.default_rng(seed)
    runs = {}

    def add(w, d, s, e):
        if 0 <= d < ndm and 0 <= w < nwidths:
            s, e = max(0, s), min(nout - 1, e)
            if s <= e:
                runs.setdefault((w, d), []).append((s, e))

    for _ in range(nclumps):
        d0 = int(rng.integers(0, ndm))
        nd = int(rng.integers(1, dm_extent + 1))
        w0 = int(rng.integers(0, nwidths))
        nw = int(rng.integers(1, min(4, nwidths) + 1))
        t0 = int(rng.integers(0, nout))
        drift = int(rng.integers(-2, 3))
        for d in range(d0, d0 + nd):
            if rng.random() < 0.1:
                continue                               # a trial where the cut missed
            for w in range(w0, w0 + nw):
                s = t0 + drift * (d - d0) + int(rng.integers(-1, 2))
                add(w, d, s, s + int(rng.integers(0, max_run)))
    for _ in range(nnoise):
        s = int(rng.integers(0, nout))
        add(int(rng.integers(0, nwidths)), int(rng.integers(0, ndm)), s, s + int(rng.integers(0, 3)))
    rows = []
    for (w, d) in sorted(runs):
        merged = []
        for s, e in sorted(runs[(w, d)]):
            if merged and s <= merged[-1][1] + 1:        # touching runs are one run
                merged[-1][1] = max(merged[-1][1], e)
            else:
                merged.append([s, e])
        for s, e in merged:
            rows.append((w, d, s, e, int(rng.integers(s, e + 1)), int(rng.integers(1, 1 << 20)),
                         np.float32(6.0 + rng.integers(0, snr_levels) * 0.5)))
    return np.array(rows, dtype=EVENT_DTYPE)
