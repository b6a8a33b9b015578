#!/usr/bin/env python3
"""Benchmark of the transient-search hot path on one MI355X.

Workload (the headline line): the survey-shaped single beam -- 1024 channels
over 400 MHz centred at 1381.8 MHz, 64 us sampling, 2^19 samples of 2-bit
data, 1200 DM trials to DM 1000 with growing spacing, 50 injected pulses,
widths 1..512, S/N > 6 -- synthetic and seeded (the survey data itself is not
available).

One step = the whole single-beam path on data already resident in HBM:
2-bit repack -> dedispersion to uint16 -> boxcar + exact sigma-cut + peak
finding -> the event records copied to the host.  Metric: DM-trial samples
per second (ndm * nout / mean step time); the median and 95th-percentile
step times are reported beside it.  The tile shape is autotuned first.

Also reported: the dedispersion kernel against its ALU roofline (HIP events
around that kernel only, on the stream it runs on) at the published clock
and at the shader clock measured under full vector load; HBM traffic from
committed rocprofv3 counters when they match the current kernel source; the
CPU oracle timed on a bounded sample on this host; the small 256-channel
case; the 13-beam batch (autotuned, real-time factor
sum_b nsamps_b tsamp / (13 T_wall)); 13-beam streaming at the real-time rate
with interference and the triage network attached, a run whose HBM budget
holds only 3 chunk slots, and an unpaced run; one leg per next row.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Derived ALU peak of the bit-sliced dedispersion.  The chip issues
# 256 CUs x 64 32-bit lane operations per clock at 2.4 GHz (3.93e13/s).  In
# the bit-sliced form one lane operation handles 32 samples of one bit-plane;
# adding one channel's 32 two-bit samples to a trial's counters takes at
# least 6 of them: two funnel shifts (align the lo and hi planes to the
# delay) and two full adders of two 3-input bit operations each (the carry-
# save reduction absorbs the two new bits).  Peak = 3.93e13 * 32 / 6 adds/s.
CUS, CLOCK_HZ = 256, 2.4e9
LANE_OPS = CUS * 64 * CLOCK_HZ
PEAK_BITSLICE_ADDS = LANE_OPS * 32 / 6
# LDS: each (trial, channel, 32 samples) reads 16 bytes per lane; at 128
# bytes per clock per CU that bounds the adds at 256 * 2.4e9 * 128 / 16 * 32.
PEAK_LDS_ADDS = CUS * CLOCK_HZ * 128 / 16 * 32
# The conventional integer-add peak (one 16-bit add per lane and half, with
# packed adds): what a kernel adding unpacked samples could reach at most.
PEAK_PK16_ADDS = CUS * 64 * 2 * CLOCK_HZ
HBM_PEAK = 8e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dedisperse_survey_traffic.json")
KERNEL_SOURCES = ["dedisperse.hip", "bitslice.hpp", "csa_tree.inc", "dedisp_internal.hpp"]
CHUNK = 1 << 17            # streaming chunk: 8.388608 s at 64 us
RFI_K, RFI_MIN_BEAMS = 3.0, 4   # coincidence mask: 3 sigma in >= 4 of the 13 beams
BASELINE_R = 2048               # baseline removal radius (samples)
T_START = time.perf_counter()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1112_0065_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record():
    """The committed counter summary of the dedispersion kernel, or None when
    it is missing or was taken on other kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t


def host_info():
    import numpy as np
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count()
    from oracle import timing
    return {"cpu_model": model, "cpus_affine": aff, "oracle_processes": timing.cpu_cores(),
            "numpy": np.__version__, "python": platform.python_version()}


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


def cpu_baseline(fb, delays, nrows):
    import numpy as np
    from oracle import timing
    rows = np.linspace(0, len(fb.dm_list) - 1, nrows).round().astype(int)
    r = timing.time_chain(fb.packed, fb.nsamps, fb.nchans, delays, rows, fb.widths,
                          fb.snr_thresh)
    # whole-beam time estimate: one unpack plus every trial at the sampled rate
    est = r["unpack_s"] + r["rows_s"] * len(fb.dm_list) / r["nrows"]
    value = len(fb.dm_list) * r["nout"] / est
    adds_per_s = r["nrows"] * r["nout"] * fb.nchans / r["rows_s"]
    return {"value": value, "unit": "DM-trial samples/s", "cores": r["procs"], "kind": "oracle",
            "sample": (f"oracle unpack of the whole beam ({r['unpack_s']:.2f} s) + dedisperse/"
                       f"boxcar/peaks of {r['nrows']} of {len(fb.dm_list)} evenly spaced DM "
                       f"trials over the full {r['nout']} samples ({r['rows_s']:.2f} s on "
                       f"{r['procs']} processes), scaled to all trials"),
            "est_beam_s": est, "channel_adds_per_s": adds_per_s}


def run_single_beam(fb, steps, warmup, out_i32=False, tune=True, kernel_events=True):
    """Time `steps` whole single-beam steps (after `warmup`) on data resident
    in HBM.  Returns a dict with per-step times, stage times and the tile."""
    import numpy as np
    import torch

    from paper_1112_0065_amd import _lib as L

    ndm = len(fb.dm_list)
    plan = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    tuned = None
    if tune:
        t0 = time.perf_counter()
        best, rej = L.dedisp_autotune(plan, fb.nsamps, out_u16=not out_i32)
        tuned = {"tile": list(best), "rejected": rej, "seconds": time.perf_counter() - t0}
    nout = fb.nsamps - plan.max_delay
    out_dtype = torch.int32 if out_i32 else torch.int16
    inp = torch.from_numpy(fb.packed).to("cuda")
    ws = torch.empty(L.dedisp_workspace_bytes(plan, fb.nsamps), dtype=torch.uint8, device="cuda")
    out = torch.empty((ndm, nout), dtype=out_dtype, device="cuda")
    pws = torch.empty(L.find_peaks_workspace_bytes(ndm, nout, fb.widths), dtype=torch.uint8,
                      device="cuda")
    cap = 1 << 20
    evb = torch.empty(cap * 40, dtype=torch.uint8, device="cuda")
    host_ev = torch.empty(cap * 40, dtype=torch.uint8, pin_memory=True)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t_rep, t_ded, t_pk = [], [], []
    state = {"n": 0}

    def step(record):
        if record:
            ev[0].record(stream)
        L.dedisp_repack(plan, inp, fb.nsamps, ws, stream)
        if record:
            ev[1].record(stream)
        L.dedisp_execute_repacked(plan, ws, fb.nsamps, out, None, stream)
        if record:
            ev[2].record(stream)
        n = L.find_peaks(out, ndm, nout, fb.widths, fb.snr_thresh, evb, cap, pws, stream)
        if record:
            ev[3].record(stream)
        # the event records to the host (find_peaks has synchronised the stream)
        host_ev[:n * 40].copy_(evb[:n * 40])
        state["n"] = n
        if record:
            torch.cuda.synchronize()
            t_rep.append(ev[0].elapsed_time(ev[1]))
            t_ded.append(ev[1].elapsed_time(ev[2]))
            t_pk.append(ev[2].elapsed_time(ev[3]))

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    # timed region: K whole steps, bracketed by synchronisation; every step
    # ends synchronised (find_peaks reads its event count, then the records
    # are copied), so each step's wall time is taken too
    per = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        step(False)
        per.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if kernel_events:
        # per-kernel durations (events), on separate passes so the
        # synchronisation they need stays out of the timed region above
        for _ in range(steps):
            step(True)
    res = {"plan": plan, "ndm": ndm, "nout": nout, "elapsed": elapsed, "per_step_s": per,
           "n_events": state["n"], "tuned": tuned, "t_rep": t_rep, "t_ded": t_ded, "t_pk": t_pk,
           "tile": list(L.dedisp_default_tile(plan)),
           "buffers": (inp, ws, out, pws, evb)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=128)
    ap.add_argument("--out-i32", action="store_true", help="int32 series instead of uint16")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shapes")
    ap.add_argument("--no-small", action="store_true", help="skip the 256-channel small case")
    ap.add_argument("--no-multibeam", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-triage", action="store_true", help="skip the triage network leg")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the baseline-removal, clustering, subband and coincidence-mask legs")
    ap.add_argument("--serve-chunks", type=int, default=32,
                    help="chunks per beam when streaming at the real-time rate")
    ap.add_argument("--serve-unpaced-chunks", type=int, default=16,
                    help="chunks per beam in the unpaced streaming run")
    ap.add_argument("--serve-speed", type=float, default=1.0,
                    help="arrival rate as a multiple of real time")
    ap.add_argument("--serve-rfi", type=int, default=1,
                    help="1: the paced streaming run applies the coincidence mask per round")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--time-budget", type=float, default=540.0,
                    help="wall seconds (from the start of the process) the extra legs may use: a "
                         "leg that would not end within it is skipped and recorded as skipped; "
                         "0 = no limit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: every beam and DM trial of this workload fits one "
              "MI355X, and the library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1112_0065_amd import _lib as L

    torch.cuda.set_device(0)
    dev = L.dedisp_device_info()
    clock_ghz = L.dedisp_clock_probe(50000)
    log(f"device {dev['name']} {dev['arch']}: {dev['compute_units']} CUs, max clock "
        f"{dev['max_clock_khz'] / 1e6:.2f} GHz, shader clock under load {clock_ghz:.3f} GHz")
    log("generating survey-shaped beam (seed 2) ...")
    fb = synth.make_survey_beam(2)

    if args.calib_copy_mib:
        # a plain copy of known size: what the HBM counters read for it
        # calibrates the traffic of the kernels below
        src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log("survey beam: autotune + timed steps ...")
    r = run_single_beam(fb, args.steps, args.warmup, args.out_i32, tune=not args.no_tune)
    plan, ndm, nout = r["plan"], r["ndm"], r["nout"]
    n_events = r["n_events"]
    log(f"events per step: {n_events}")
    ms_step = r["elapsed"] / args.steps * 1e3
    value = ndm * nout * args.steps / r["elapsed"]
    ded_ms = float(np.mean(r["t_ded"]))
    adds = ndm * nout * fb.nchans
    achieved = adds / (ded_ms * 1e-3)
    tr = traffic_record()
    eff_peak = PEAK_BITSLICE_ADDS * clock_ghz * 1e9 / CLOCK_HZ
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_BITSLICE_ADDS / 1e12,
                "unit": "Tadd/s", "frac": achieved / PEAK_BITSLICE_ADDS,
                "traffic": tr.get("hbm_bytes_per_launch") if tr else None,
                "kernel": "dedisperse_kernel", "kernel_ms": ded_ms,
                "kernel_ms_median": float(np.median(r["t_ded"])),
                "algorithmic_adds_per_launch": adds,
                "peak_basis": f"{CUS} CUs x 64 lanes x {CLOCK_HZ / 1e9} GHz x 32 samples / 6 lane-ops",
                "shader_clock_ghz_under_load": clock_ghz,
                "frac_at_shader_clock": achieved / eff_peak,
                "lds_peak": PEAK_LDS_ADDS / 1e12, "lds_frac": achieved / PEAK_LDS_ADDS,
                "pk16_peak": PEAK_PK16_ADDS / 1e12, "frac_of_pk16": achieved / PEAK_PK16_ADDS}
    if tr and tr.get("effective_clock_ghz"):
        roofline["counter_clock_ghz"] = tr["effective_clock_ghz"]

    cpu = None
    delays = None
    if not args.no_cpu_baseline:
        import oracle
        log("timing the CPU oracle on a bounded sample ...")
        delays = oracle.delay_table(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
        cpu = cpu_baseline(fb, delays, args.cpu_rows)

    rec = {
        "metric": "DM-trial samples/sec (dedisp) + real-time factor for 13 beams; p99 chunk latency",
        "value": value,
        "unit": "DM-trial samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": pct(r["per_step_s"], 50) * 1e3,
        "ms_per_step_p95": pct(r["per_step_s"], 95) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32" if args.out_i32 else "u16",
        "data": "synthetic (seeded 2-bit noise + injected dispersed pulses)",
        "config": {"workload": "survey beam: 1024 ch, 2^19 samples, 1200 DM trials to 1000, "
                               "widths 1..512, S/N>6",
                   "nchans": fb.nchans, "nsamps": fb.nsamps, "ndm": ndm, "nout": nout,
                   "max_delay": plan.max_delay, "widths": fb.widths, "parallelism": "1 GPU",
                   "input_sha256": fb.sha256, "tile": r["tile"]},
        "autotune": r["tuned"],
        "events_per_step": n_events,
        "stages_ms": {"repack": float(np.mean(r["t_rep"])), "dedisperse": ded_ms,
                      "boxcar_peaks_events": float(np.mean(r["t_pk"]))},
        "real_time_factor_1beam": fb.nsamps * fb.tsamp / (ms_step * 1e-3),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "device": {**dev, "shader_clock_ghz_under_load": clock_ghz},
        "host": host_info(),
    }
    legs = {}
    rec["legs_s"] = legs

    def leg(name, need_s, fn):
        """Run one extra leg, timing it, unless it would overrun the budget."""
        el = time.perf_counter() - T_START
        if args.time_budget and el + need_s > args.time_budget:
            log(f"skipping {name}: {el:.0f} s elapsed, about {need_s:.0f} s more needed, "
                f"budget {args.time_budget:.0f} s")
            legs[name] = {"skipped": True, "elapsed_s": round(el, 1), "needed_s": need_s}
            return None
        log(f"{name} ...")
        t0 = time.perf_counter()
        res = fn()
        legs[name] = round(time.perf_counter() - t0, 1)
        return res

    legs["survey_beam"] = round(time.perf_counter() - T_START, 1)
    # extra legs in order of priority: the 13-beam batch and streaming first
    # (the metric's other two parts), then the small case and the next rows
    inp, ws, out, pws, evb = r["buffers"]
    keep_ev = L.events_from_buffer(evb, n_events)
    direct_ms = rec["stages_ms"]["repack"] + ded_ms
    del r, out, ws, pws, evb, inp
    torch.cuda.empty_cache()
    if not args.no_multibeam:
        rec["multibeam"] = leg("13-beam batch", 40, lambda: bench_multibeam(args, cpu))
        if rec["multibeam"]:
            rec["rtf_13beam"] = rec["multibeam"]["rtf_batch"]
    if not args.no_serve:
        payloads = leg("streaming payloads", 30, serve_payloads)
        if payloads:
            paced_s = (args.serve_chunks + 2) * CHUNK * synth.TSAMP / args.serve_speed + 15
            rec["serve"] = leg(f"13-beam streaming at the real-time rate ({args.serve_chunks} "
                               "chunks per beam)", paced_s, lambda: bench_serve(args, payloads))
            rec["serve_queueing"] = leg("13-beam streaming with 3 chunk slots (forced queueing)",
                                        15, lambda: bench_serve_queueing(args, payloads))
            rec["serve_unpaced"] = leg("13-beam streaming, unpaced", 20,
                                       lambda: bench_serve_unpaced(args, payloads))
            rec["serve_unpaced_stages"] = leg(
                "13-beam streaming, unpaced, coincidence mask and baseline removal", 20,
                lambda: bench_serve_unpaced(args, payloads, (RFI_K, RFI_MIN_BEAMS, BASELINE_R)))
            if rec["serve"]:
                rec["p99_chunk_latency_s"] = rec["serve"]["p99_s"]
                if not args.no_cpu_baseline:
                    cc = leg("CPU oracle per streaming chunk", 25,
                             lambda: cpu_chunk_time(payloads[0]))
                    if cc:
                        rec["serve"]["cpu_oracle_per_chunk"] = cc
            del payloads
    if not args.no_small:
        rec["small_case"] = leg("small 256-channel case", 20, lambda: bench_small(args))
    if not args.no_next:
        nx = leg("survey next rows", 40, lambda: bench_next_single(args, fb, keep_ev, direct_ms))
        if nx:
            rec.update(nx)
        rec["rfi_mask"] = leg("13-beam coincidence mask", 15, lambda: bench_rfi_mask(args))
    if not args.no_triage:
        rec["triage"] = leg("triage network, 256 tiles", 20, lambda: bench_triage(args))
    legs["total"] = round(time.perf_counter() - T_START, 1)
    print(json.dumps(rec), flush=True)


def bench_next_single(args, fb, ev, direct_ms):
    """Next-row legs on the survey beam: baseline removal, clustering,
    subband dedispersion.  `ev`: the beam's events (host records) from the
    timed steps; the series is dedispersed again here."""
    import numpy as np
    import torch

    from paper_1112_0065_amd import _lib as L

    ndm = len(fb.dm_list)
    plan = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    nout = fb.nsamps - plan.max_delay
    inp = torch.from_numpy(fb.packed).to("cuda")
    ws = torch.empty(L.dedisp_workspace_bytes(plan, fb.nsamps), dtype=torch.uint8, device="cuda")
    out = torch.empty((ndm, nout), dtype=torch.int16, device="cuda")
    L.dedisp_execute(plan, inp, fb.nsamps, out, ws)
    del ws
    n_events = len(ev)
    evb = torch.from_numpy(np.frombuffer(ev.tobytes(), np.uint8).copy()).to("cuda")
    res = {}
    # baseline removal (running mean, radius 2048) of the survey series: one
    # read and one write of the uint16 rows
    R = 2048
    flat = torch.empty((ndm, nout - 2 * R), dtype=torch.int16, device="cuda")
    L.baseline_remove(out, ndm, nout, R, 3 * fb.nchans, flat)
    torch.cuda.synchronize()
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b0.record()
    for _ in range(10):
        L.baseline_remove(out, ndm, nout, R, 3 * fb.nchans, flat)
    b1.record()
    b1.synchronize()
    bl_ms = b0.elapsed_time(b1) / 10
    bl_bytes = ndm * nout * 2 + ndm * (nout - 2 * R) * 2
    res["baseline"] = {"radius": R, "ms": bl_ms, "algorithmic_bytes": bl_bytes,
                       "achieved_GBps": bl_bytes / (bl_ms * 1e-3) / 1e9,
                       "hbm_frac": bl_bytes / (bl_ms * 1e-3) / HBM_PEAK,
                       "output_samples_per_s": ndm * (nout - 2 * R) / (bl_ms * 1e-3)}
    if not args.no_cpu_baseline:
        import oracle
        rows = out[:16].cpu().numpy().view(np.uint16).astype(np.int64)
        t_c = time.perf_counter()
        oracle.baseline_remove(rows, R, 3 * fb.nchans)
        t_c = time.perf_counter() - t_c
        res["baseline"]["cpu_oracle"] = {
            "value": 16 * (nout - 2 * R) / t_c, "unit": "output samples/s", "cores": 1,
            "kind": "oracle", "sample": f"16 of {ndm} survey series ({t_c:.2f} s)"}
    del flat, out
    res["cluster"] = bench_cluster(evb, n_events, ndm, fb.widths, not args.no_cpu_baseline)
    res["subband"] = bench_subband(fb, plan, inp, ev, direct_ms, not args.no_cpu_baseline)
    return res


def bench_small(args):
    """The small case: 256 channels (1581.8 MHz down, 1.5625 MHz steps), 2^15
    samples, 100 trials to DM 200, 5 pulses, widths 1..64, S/N > 6.  Launch-
    bound on the GPU; the oracle runs it in full on the host cores."""
    import numpy as np

    import synth
    fb = synth.make_small(1)
    r = run_single_beam(fb, max(args.steps, 50), args.warmup, tune=not args.no_tune,
                        kernel_events=False)
    value = r["ndm"] * r["nout"] * len(r["per_step_s"]) / r["elapsed"]
    res = {"workload": "256 ch, 2^15 samples, 100 DM trials to 200, widths 1..64, S/N>6",
           "value": value, "unit": "DM-trial samples/s",
           "ms_per_step": r["elapsed"] / len(r["per_step_s"]) * 1e3,
           "ms_per_step_median": pct(r["per_step_s"], 50) * 1e3,
           "ms_per_step_p95": pct(r["per_step_s"], 95) * 1e3,
           "events_per_step": r["n_events"], "tile": r["tile"], "autotune": r["tuned"],
           "input_sha256": fb.sha256}
    if not args.no_cpu_baseline:
        import oracle
        from oracle import timing
        dly = oracle.delay_table(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
        t = timing.time_chain(fb.packed, fb.nsamps, fb.nchans, dly, np.arange(len(fb.dm_list)),
                              fb.widths, fb.snr_thresh)
        tot = t["unpack_s"] + t["rows_s"]
        res["cpu_oracle"] = {"value": r["ndm"] * r["nout"] / tot, "unit": "DM-trial samples/s",
                             "cores": t["procs"], "kind": "oracle",
                             "sample": f"the whole case ({tot:.2f} s, {t['nevents']} events)"}
    del r
    return res


def serve_payloads(n=8):
    """Chunk payloads of the streaming runs: survey-shaped 2^17-sample beams
    with 8 dispersed pulses and the three kinds of interference (zero-DM
    impulses, 5% narrowband channels, 50 Hz periodic), seeds 400..; beams and
    sequence numbers cycle through them."""
    import multiprocessing as mp
    from oracle import timing
    with mp.get_context("fork").Pool(min(n, timing.cpu_cores())) as pool:
        fbs = pool.map(_rfi_payload, [400 + k for k in range(n)])
    return fbs


def _rfi_payload(seed):
    import synth
    return synth.make_rfi_beam(seed, CHUNK)


def cpu_chunk_time(fb, nrows=128):
    """The oracle's time for one streaming chunk of one beam: the window of
    C + H samples, all 1200 trials (scaled from `nrows` evenly spaced ones),
    boxcars and peaks, against the chunk's 8.39 s duration."""
    import numpy as np

    import oracle
    from oracle import timing
    dly = oracle.delay_table(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    H = int(dly.max()) + fb.widths[-1] - 1
    # the window: the chunk's H predecessors (here the tail of the same
    # payload: the same sizes and work as in the stream)
    bpc = fb.nchans // 4
    win = np.concatenate([fb.packed[-H * bpc:], fb.packed])
    ns = CHUNK + H
    rows = np.linspace(0, len(fb.dm_list) - 1, nrows).round().astype(int)
    t = timing.time_chain(win, ns, fb.nchans, dly, rows, fb.widths, fb.snr_thresh)
    est = t["unpack_s"] + t["rows_s"] * len(fb.dm_list) / t["nrows"]
    dur = CHUNK * fb.tsamp
    return {"seconds_per_beam_chunk": est, "chunk_seconds": dur,
            "seconds_per_13_beam_round": 13 * est, "cpu_rtf_13beam": dur / (13 * est),
            "cores": t["procs"], "kind": "oracle",
            "sample": f"{t['nrows']} of 1200 trials of one chunk window ({ns} samples), scaled"}


def bench_multibeam(args, cpu=None):
    """13 beams of uneven length (2^17 + 2^15 b samples) and DM range (max
    500 + 125 ((5b) mod 13)), 1200 trials each: one persistent launch in a HIP
    graph (dedisp_batch_execute), its tile shape autotuned on the beam with the
    largest delays, against 13 sequential single-beam calls.  Real-time
    factor = sum_b nsamps_b tsamp / (13 T_wall)."""
    import tempfile

    import numpy as np
    import torch

    import synth
    from paper_1112_0065_amd import _lib as L

    shapes = synth.multibeam_shapes()
    nmax = max(n for n, _ in shapes)
    pool = synth.fast_chunk(300, nmax, npulses=20)      # beam b reads a prefix of it
    plans, ins, outs, evs, ns = [], [], [], [], []
    widths = [1 << i for i in range(10)]
    for b, (n, dm_max) in enumerate(shapes):
        p = L.dedisp_plan_create(1024, synth.F_TOP, synth.DF_SURVEY, synth.TSAMP,
                                 synth.dm_list_expm1(1200, dm_max))
        plans.append(p)
        ins.append(torch.from_numpy(pool[: n * 256]).to("cuda"))
        outs.append(torch.empty((1200, n - p.max_delay), dtype=torch.int16, device="cuda"))
        evs.append(torch.empty((1 << 20) * 40, dtype=torch.uint8, device="cuda"))
        ns.append(n)
    cap = [1 << 20] * len(plans)
    tuned = None
    cache = None
    if not args.no_tune:
        heavy = max(range(len(plans)), key=lambda b: plans[b].max_delay)
        cache = os.path.join(tempfile.mkdtemp(prefix="dedisp_tune_"), "tune.json")
        t0 = time.perf_counter()
        best, rej = L.dedisp_autotune(plans[heavy], ns[heavy], out_u16=True, cache_path=cache)
        tuned = {"on_beam": heavy, "tile": list(best), "rejected": rej,
                 "seconds": time.perf_counter() - t0}
    batch = L.dedisp_batch_create(plans, widths, 6.0, out_u16=True, tune_cache_path=cache)
    tile, grid, _ = L.dedisp_batch_info(batch)
    reps = max(3, args.steps // 4)
    L.dedisp_batch_execute(batch, ins, ns, outs, evs, cap)      # capture + warm-up
    torch.cuda.synchronize()
    per = []
    for _ in range(reps):
        t0 = time.perf_counter()
        counts = L.dedisp_batch_execute(batch, ins, ns, outs, evs, cap)
        torch.cuda.synchronize()
        per.append(time.perf_counter() - t0)
    t_batch = float(np.mean(per))
    # the same batch with the pipeline's optional stages: coincidence mask
    # before dedispersion (over the 2^17 samples all beams share), baseline
    # removal after
    L.dedisp_batch_set_stages(batch, RFI_K, RFI_MIN_BEAMS, BASELINE_R)
    L.dedisp_batch_execute(batch, ins, ns, outs, evs, cap)      # capture + warm-up
    torch.cuda.synchronize()
    per_st = []
    for _ in range(reps):
        t0 = time.perf_counter()
        counts_st = L.dedisp_batch_execute(batch, ins, ns, outs, evs, cap)
        torch.cuda.synchronize()
        per_st.append(time.perf_counter() - t0)
    L.dedisp_batch_set_stages(batch, 0.0, 0, 0)
    # the same work as 13 sequential single-beam calls (the same tile)
    wss = [torch.empty(L.dedisp_workspace_bytes(p, n), dtype=torch.uint8, device="cuda")
           for p, n in zip(plans, ns)]
    pwss = [torch.empty(L.find_peaks_workspace_bytes(1200, n - p.max_delay, widths),
                        dtype=torch.uint8, device="cuda") for p, n in zip(plans, ns)]

    def sequential():
        for b in range(len(plans)):
            L.dedisp_execute_tile(plans[b], ins[b], ns[b], outs[b], wss[b], tile)
            L.find_peaks(outs[b], 1200, ns[b] - plans[b].max_delay, widths, 6.0, evs[b], cap[b],
                         pwss[b])

    sequential()
    torch.cuda.synchronize()
    seq = []
    for _ in range(reps):
        t0 = time.perf_counter()
        sequential()
        torch.cuda.synchronize()
        seq.append(time.perf_counter() - t0)
    t_seq = float(np.mean(seq))
    beam_s = sum(ns) * synth.TSAMP
    dm_samples = sum(1200 * (n - p.max_delay) for p, n in zip(plans, ns))
    adds = dm_samples * 1024
    res = {"beams": len(plans), "beam_seconds": beam_s, "tile": list(tile), "grid": grid,
           "autotune": tuned,
           "ms_batch": t_batch * 1e3, "ms_batch_median": pct(per, 50) * 1e3,
           "ms_batch_p95": pct(per, 95) * 1e3, "ms_sequential": t_seq * 1e3,
           "rtf_batch": beam_s / (len(plans) * t_batch),
           "rtf_sequential": beam_s / (len(plans) * t_seq),
           "beam_seconds_per_s_batch": beam_s / t_batch,
           "dm_trial_samples_per_s_batch": dm_samples / t_batch,
           "channel_adds_per_launch": adds,
           "events": int(sum(counts)),
           "with_stages": {"ms_batch": float(np.mean(per_st)) * 1e3,
                           "ms_batch_median": pct(per_st, 50) * 1e3,
                           "rtf": beam_s / (len(plans) * float(np.mean(per_st))),
                           "events": int(sum(counts_st)),
                           "rfi_mask": {"k_sigma": RFI_K, "min_beams": RFI_MIN_BEAMS},
                           "baseline_radius": BASELINE_R},
           "rtf_definition": "sum_b nsamps_b * tsamp / (13 * T_wall)",
           "data": "one seeded fast-noise pool of 2^19 samples with 20 pulses; beam b reads "
                   "its first nsamps_b samples"}
    if cpu:
        est = adds / cpu["channel_adds_per_s"]
        res["cpu_oracle_extrapolated"] = {
            "seconds": est, "rtf": beam_s / (len(plans) * est), "cores": cpu["cores"],
            "kind": "oracle", "extrapolated": True,
            "sample": "the survey beam's measured oracle channel-add rate applied to the "
                      "13-beam work (dedispersion only)"}
    del batch
    return res


def _served_recall(results, payloads, plan, tau):
    """Recall over the injected pulses a chunk window fully contains, and
    false candidates, for the plain detector (every candidate) and for
    triage (score >= tau), from the served results."""
    import numpy as np

    import synth
    from paper_1112_0065_amd import triage_train as T
    sweep = None
    found_p = found_t = total = fp_p = fp_t = 0
    H = plan.max_delay + 511
    for r in results:
        if r["scores"] is None:
            continue
        fb = payloads[(r["beam"] + r["seq"]) % len(payloads)]
        if sweep is None:
            sweep = np.array([int(synth.sky_arrival_offsets(fb.nchans, fb.f_top, fb.df, fb.tsamp,
                                                            float(d))[-1]) for d in fb.dm_list])
        off = r["seq"] * CHUNK - r["t_abs0"]     # payload sample 0 in the searched series
        ok = [j for j, p in enumerate(fb.pulses)
              if p.t0 < CHUNK - H and
              p.t0 + p.width + int(synth.sky_arrival_offsets(fb.nchans, fb.f_top, fb.df, fb.tsamp,
                                                             p.dm)[-1]) <= CHUNK]
        total += len(ok)
        sel = r["scores"] >= 0
        cand = r["events"][sel].copy()
        sc = r["scores"][sel]
        cand["t_peak"] -= off
        _, match = T.label(cand, fb, sweep)
        good = set(ok)
        hit = [(m, s) for m, s in zip(match.tolist(), sc.tolist()) if m in good]
        found_p += len({m for m, _ in hit})
        found_t += len({m for m, s in hit if s >= tau})
        fp_p += int((match < 0).sum())
        fp_t += int(((match < 0) & (sc >= tau)).sum())
    return {"pulses": total, "recall_plain": found_p / max(total, 1),
            "recall_triage": found_t / max(total, 1), "false_plain": fp_p, "false_triage": fp_t,
            "tau": tau, "note": "plain = every candidate (per-width NMS of the events) kept; "
                                "triage = candidates scoring >= tau"}


def _serve_run(plans, payloads, model, budget, sched, pace=True, progress_every=0, stages=None):
    """Feed the server on the schedule [(due_ns, beam, seq)] (real-time
    arrivals when pace, else as fast as it admits); `stages` = (rfi k_sigma,
    rfi min beams, baseline radius) or None; returns (results, stats, wall
    seconds, busy retries)."""
    from paper_1112_0065_amd import _lib as L
    widths = [1 << i for i in range(10)]
    srv = L.dedisp_serve_create(plans, CHUNK, widths, 6.0, budget, model=model)
    if stages:
        L.dedisp_serve_set_stages(srv, *stages)
    t_start = L.dedisp_now_ns()
    done = []
    busy = 0
    for i, (due, b, k) in enumerate(sched):
        if pace:
            while L.dedisp_now_ns() - t_start < due:
                done += L.dedisp_serve_poll(srv, 64, 0)
                time.sleep(0.0005)
        arrival = t_start + int(due) if pace else None
        while not L.dedisp_serve_submit(srv, b, k, payloads[(b + k) % len(payloads)].packed,
                                        arrival if pace else L.dedisp_now_ns()):
            busy += 1
            done += L.dedisp_serve_poll(srv, 64, 1)
        if progress_every and (i + 1) % progress_every == 0:
            log(f"  submitted {i + 1}/{len(sched)} chunks, {len(done)} results")
    while len(done) < len(sched):
        done += L.dedisp_serve_poll(srv, 64, 100)
    wall = (L.dedisp_now_ns() - t_start) * 1e-9
    st = L.dedisp_serve_stats(srv)
    srv.close()
    return done, st, wall, busy


def _serve_plans():
    import synth
    from paper_1112_0065_amd import _lib as L
    dms = synth.dm_list_expm1(1200, 1000.0)
    return [L.dedisp_plan_create(1024, synth.F_TOP, synth.DF_SURVEY, synth.TSAMP, dms)
            for _ in range(13)]


def bench_serve(args, payloads):
    """13 beams streaming chunks of 2^17 samples (8.39 s) at the real-time
    rate, beam b starting b/13 of a chunk late; 1200 trials to DM 1000;
    interference in every chunk; the trained triage network attached (it
    scores each chunk's candidates before the result is returned); HBM budget
    32 GiB.  Latency = completion minus arrival of the chunk's last sample."""
    import numpy as np

    import synth
    from paper_1112_0065_amd import _lib as L
    from paper_1112_0065_amd import triage_train as T

    model, tau, _ = T.load_default()
    plans = _serve_plans()
    nchunks, speed = args.serve_chunks, args.serve_speed
    period_ns = CHUNK * synth.TSAMP * 1e9 / speed
    sched = sorted((b * period_ns / 13 + (k + 1) * period_ns, b, k)
                   for b in range(13) for k in range(nchunks))
    stages = (RFI_K, RFI_MIN_BEAMS, 0) if args.serve_rfi else None
    done, st, wall, busy = _serve_run(plans, payloads, model, 32 << 30, sched, pace=True,
                                      progress_every=13, stages=stages)
    late = sum(1 for r in done if r["flags"] & L.CHUNK_LATE)
    fallback = sum(1 for r in done if r["flags"] & L.CHUNK_FALLBACK)
    lat = np.array([r["done_ns"] - r["arrival_ns"] for r in done], np.float64) * 1e-9
    beam_s = 13 * nchunks * CHUNK * synth.TSAMP
    return {"beams": 13, "chunks": len(done), "chunks_per_beam": nchunks, "chunk_samples": CHUNK,
            "speed_vs_real_time": speed, "deadline_s": st["deadline_ns"] * 1e-9 / speed,
            "p50_s": st["p50_ns"] * 1e-9, "p99_s": st["p99_ns"] * 1e-9, "max_s": st["max_ns"] * 1e-9,
            "mean_s": float(lat.mean()),
            "deadline_misses": late if speed == 1.0 else None, "fallback_chunks": fallback,
            "batches": st["batches"], "mean_batch": st["mean_batch"], "max_batch": st["max_batch"],
            "slots": st["slots"], "busy_retries": busy, "wall_s": wall,
            "rtf": beam_s / (13 * wall),
            "events": int(sum(r["n_events"] for r in done)),
            "candidates_scored": int(sum(r["n_candidates"] for r in done)),
            "triage": _served_recall(done, payloads, plans[0], tau),
            "stages": ({"rfi_mask": {"k_sigma": RFI_K, "min_beams": RFI_MIN_BEAMS},
                        "note": "each round of 13 chunks (one sequence number) is masked and "
                                "batched together, so a chunk waits for the round's last "
                                "(staggered) beam: latency includes up to 12/13 of a chunk"}
                       if stages else None),
            "data": f"{len(payloads)} interference chunk payloads (make_rfi_beam seeds 400..) "
                    "cycled over beams and sequence numbers"}


def _serve_burst(plans, payloads, model, budget, nchunks, threads, stages=None):
    """Every beam submits its chunks as fast as the server admits them, from
    `threads` submitting threads (beam b on thread b % threads, each beam in
    sequence order; BUSY is retried): the arrival rate exceeds what the
    slots drain, so admission queues.  Returns (results, stats, wall
    seconds, busy retries)."""
    import threading

    from paper_1112_0065_amd import _lib as L
    widths = [1 << i for i in range(10)]
    srv = L.dedisp_serve_create(plans, CHUNK, widths, 6.0, budget, model=model)
    if stages:
        L.dedisp_serve_set_stages(srv, *stages)
    busy = [0] * threads

    def feed(t):
        for k in range(nchunks):
            for b in range(t, len(plans), threads):
                while not L.dedisp_serve_submit(srv, b, k, payloads[(b + k) % len(payloads)].packed,
                                                L.dedisp_now_ns()):
                    busy[t] += 1
                    time.sleep(0.0002)

    t_start = L.dedisp_now_ns()
    ths = [threading.Thread(target=feed, args=(t,)) for t in range(threads)]
    for th in ths:
        th.start()
    done = []
    want = nchunks * len(plans)
    while len(done) < want:
        done += L.dedisp_serve_poll(srv, 64, 100)
    for th in ths:
        th.join()
    wall = (L.dedisp_now_ns() - t_start) * 1e-9
    st = L.dedisp_serve_stats(srv)
    srv.close()
    return done, st, wall, sum(busy)


def bench_serve_queueing(args, payloads):
    """The same 13 beams with an HBM budget of the resident overlaps plus 3
    chunk slots, 4 chunks per beam submitted from 4 threads as fast as the
    server admits them: admission holds the rest back (BUSY) and every batch
    takes the slots that have drained (at most 3 chunks)."""
    import synth
    from paper_1112_0065_amd import _lib as L
    from paper_1112_0065_amd import triage_train as T

    model, _, _ = T.load_default()
    plans = _serve_plans()
    widths = [1 << i for i in range(10)]
    slot = L.dedisp_serve_slot_bytes(plans, CHUNK, widths)
    resident = sum((p.max_delay + 511) * 256 for p in plans)
    budget = resident + 3 * slot + slot // 2
    done, st, wall, busy = _serve_burst(plans, payloads, model, budget, 4, 4)
    beam_s = 13 * 4 * CHUNK * synth.TSAMP
    return {"beams": 13, "chunks": len(done), "slots": st["slots"],
            "budget_bytes": budget, "slot_bytes": slot, "busy_retries": busy,
            "batches": st["batches"], "mean_batch": st["mean_batch"], "max_batch": st["max_batch"],
            "p50_s": st["p50_ns"] * 1e-9, "p99_s": st["p99_ns"] * 1e-9, "max_s": st["max_ns"] * 1e-9,
            "wall_s": wall, "rtf": beam_s / (13 * wall)}


def bench_serve_unpaced(args, payloads, stages=None):
    """The same 13-beam server (no triage) fed as fast as it accepts chunks
    (4 submitting threads, BUSY = back-pressure, retried): the sustained
    real-time factor of streaming, sum of beam-seconds / (13 T_wall), with
    continuous batching of whatever is queued; `stages` as for _serve_run."""
    import synth

    plans = _serve_plans()
    nchunks = args.serve_unpaced_chunks
    done, st, wall, busy = _serve_burst(plans, payloads, None, 32 << 30, nchunks, 4, stages)
    beam_s = 13 * nchunks * CHUNK * synth.TSAMP
    res = {"beams": 13, "chunks": len(done), "beam_seconds": beam_s, "wall_s": wall,
           "rtf": beam_s / (13 * wall), "beam_seconds_per_s": beam_s / wall,
           "batches": st["batches"], "mean_batch": st["mean_batch"],
           "max_batch": st["max_batch"], "slots": st["slots"], "busy_retries": busy,
           "p50_s": st["p50_ns"] * 1e-9, "p99_s": st["p99_ns"] * 1e-9}
    if stages:
        res["stages"] = {"rfi_mask": {"k_sigma": stages[0], "min_beams": stages[1]},
                         "baseline_radius": stages[2]}
    return res


def bench_subband(fb, plan, inp, ev_direct, direct_ms, cpu=False):
    """Subband dedispersion of the survey beam in place of the direct sum:
    time per beam (repack + both stages, HIP events on the stream; direct_ms
    is repack + direct dedispersion of the same beam), and what
    the approximation costs: for each injected pulse, the best S/N of the
    events near its trial and arrival, against the direct path's."""
    import numpy as np
    import torch

    from paper_1112_0065_amd import _lib as L

    ndm = len(fb.dm_list)

    def best_snr(ev):
        out = []
        dmi, tpk = ev["dm_idx"].astype(np.int64), ev["t_peak"].astype(np.int64)
        for pu in fb.pulses:
            d = int(np.argmin(np.abs(fb.dm_list - pu.dm)))
            near = (np.abs(dmi - d) <= 2) & (np.abs(tpk - pu.t0) <= pu.width + 2)
            out.append(float(ev["snr"][near].max()) if near.any() else 0.0)
        return np.array(out)

    ref = best_snr(ev_direct)
    res = {}
    for nsub, group in ((32, 8), (16, 8), (64, 4)):
        sb = L.dedisp_subband_create(plan, nsub, group)
        nout = fb.nsamps - sb.max_delay
        ws = torch.empty(L.dedisp_subband_workspace_bytes(sb, fb.nsamps), dtype=torch.uint8,
                         device="cuda")
        out = torch.empty((ndm, nout), dtype=torch.int16, device="cuda")
        stream = torch.cuda.current_stream()
        L.dedisp_subband_execute(sb, inp, fb.nsamps, out, ws, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record(stream)
        for _ in range(reps):
            L.dedisp_subband_execute(sb, inp, fb.nsamps, out, ws, stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        pws = torch.empty(L.find_peaks_workspace_bytes(ndm, nout, fb.widths), dtype=torch.uint8,
                          device="cuda")
        eb = torch.empty((1 << 20) * 40, dtype=torch.uint8, device="cuda")
        n = L.find_peaks(out, ndm, nout, fb.widths, fb.snr_thresh, eb, 1 << 20, pws)
        got = best_snr(L.events_from_buffer(eb, n))
        found = ref > 0
        ratio = got[found] / ref[found]
        res[f"{nsub}x{group}"] = {
            "nsub": nsub, "group": group, "ncoarse": sb.ncoarse, "stage1_tile": list(sb.tile),
            "ms": ms,
            "dm_trial_samples_per_s": ndm * nout / (ms * 1e-3),
            "speedup_vs_direct": direct_ms / ms, "events": n,
            "pulses_found_direct": int(found.sum()), "pulses_found": int((got[found] > 0).sum()),
            "snr_ratio_median": float(np.median(ratio)), "snr_ratio_min": float(ratio.min())}
        if cpu and (nsub, group) == (16, 8):
            import oracle
            ns = sb.max_delay + 8192                     # 8192 output samples
            x = oracle.unpack_2bit(fb.packed[:ns * fb.nchans // 4], ns, fb.nchans)
            t_c = time.perf_counter()
            oracle.subband_dedisperse(x, fb.f_top, fb.df, fb.tsamp, fb.dm_list, nsub, group)
            t_c = time.perf_counter() - t_c
            res[f"{nsub}x{group}"]["cpu_oracle"] = {
                "value": ndm * 8192 / t_c, "unit": "DM-trial samples/s", "cores": 1,
                "kind": "oracle", "sample": f"the first {ns} samples of the beam, 8192 outputs "
                                            f"per trial ({t_c:.2f} s)"}
        del ws, out, pws, eb
        sb.close()
        torch.cuda.empty_cache()
    return res


# Multiply-adds of the triage network per 64 x 256 tile (3x3 convolutions at
# 64x256, 32x128, 16x64 and 8x32 with 1->32->32->32->32 channels; pooling,
# bias and the final layer are negligible), counted as 2 FLOP each.
TRIAGE_FWD_FLOP = 2 * 9 * 32 * (1 * 64 * 256 + 32 * 32 * 128 + 32 * 16 * 64 + 32 * 8 * 32)


def bench_triage(args, reps=20, n=256):
    """The triage network on one batch of 256 seeded candidate tiles: scoring
    (forward) and a training step (forward, input- and weight-gradients,
    Adam), each timed with HIP events on the stream it runs on; achieved
    TFLOP/s with the training step counted as three forward passes.  The CPU
    leg times the oracle's forward and backward on 16 of the tiles."""
    import numpy as np
    import torch

    from paper_1112_0065_amd import _lib as L

    rng = np.random.default_rng(7)
    x = rng.standard_normal((n, 64, 256)).astype(np.float32)
    x[::2, 28:36, 100:160] += 3.0
    tiles = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).cuda()
    labels = torch.tensor([1.0, 0.0] * (n // 2), dtype=torch.float32, device="cuda")
    scores = torch.empty(n, dtype=torch.float32, device="cuda")
    m = L.triage_create(None, 0)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    fwd_ms = timed(lambda: L.triage_score(m, tiles, n, scores, stream))
    train_ms = timed(lambda: L.triage_train_step(m, tiles, labels, n, 1e-4, stream))
    fwd_flop = TRIAGE_FWD_FLOP * n
    res = {"tiles": n, "forward_ms": fwd_ms, "train_step_ms": train_ms,
           "forward_flop_per_tile": TRIAGE_FWD_FLOP,
           "forward_tflops": fwd_flop / (fwd_ms * 1e-3) / 1e12,
           "train_tflops": 3 * fwd_flop / (train_ms * 1e-3) / 1e12,
           "peak_bf16_tflops": 2500.0,
           "tiles_per_s_scoring": n / (fwd_ms * 1e-3)}
    res["forward_frac_of_bf16_peak"] = res["forward_tflops"] / 2500.0
    if not args.no_cpu_baseline:
        from oracle import cnn
        p = cnn.init_params(0)
        k = 16
        t_c = time.perf_counter()
        logits, cache = cnn.forward(p, cnn.round_bf16(x[:k].astype(np.float64)))
        cnn.backward(p, cache, logits, np.array([1.0, 0.0] * (k // 2)))
        t_c = time.perf_counter() - t_c
        res["cpu_oracle"] = {"value": k / t_c, "unit": "tiles/s (forward + backward)", "cores": 1,
                             "kind": "oracle", "sample": f"{k} of the {n} tiles ({t_c:.2f} s)"}
    del m
    return res


def bench_cluster(evb, n_events, ndm, widths, cpu=False):
    """Clustering of events across DM and width (friends of friends, DM
    radius 2, width radius 1, no time slack): the survey beam's own events,
    and a dense synthetic list of about a million events.  Each call includes
    its host synchronisation (the cluster count is read back)."""
    import numpy as np
    import torch

    import synth
    from paper_1112_0065_amd import _lib as L

    def run(buf, n, nd, ws_w):
        ws = torch.empty(max(L.dedisp_cluster_workspace_bytes(n, nd, len(ws_w)), 1),
                         dtype=torch.uint8, device="cuda")
        cb = torch.empty(max(n, 1) * 72, dtype=torch.uint8, device="cuda")
        nc = L.dedisp_cluster_events(buf, n, nd, ws_w, 2, 1, 0, cb, n, ws)
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            L.dedisp_cluster_events(buf, n, nd, ws_w, 2, 1, 0, cb, n, ws)
        dt = (time.perf_counter() - t0) / reps
        return {"events": n, "clusters": nc, "ms": dt * 1e3, "events_per_s": n / dt}

    res = {"survey_beam": run(evb, n_events, ndm, widths)}
    if cpu:
        import oracle
        m = min(3000, n_events)
        ev = L.events_from_buffer(evb, m)
        t_c = time.perf_counter()
        oracle.cluster_events(ev, widths, 2, 1, 0)
        t_c = time.perf_counter() - t_c
        res["cpu_oracle"] = {"value": m / t_c, "unit": "events/s", "cores": 1, "kind": "oracle",
                             "sample": f"first {m} survey events ({t_c:.2f} s; all pairs tested, "
                                       "so the rate falls as the list grows)"}
    ev = synth.make_event_list(77, 1200, 10, 1 << 22, nclumps=20000, nnoise=300000)
    buf = torch.from_numpy(np.frombuffer(ev.tobytes(), np.uint8).copy()).to("cuda")
    res["dense_synthetic"] = run(buf, len(ev), 1200, [1 << i for i in range(10)])
    return res


def bench_rfi_mask(args):
    """Multibeam coincidence mask over 13 beams x 2^19 samples x 1024
    channels (3 sigma in >= 4 beams).  HBM roofline: the packed inputs are
    read once (13 x 128 MiB); the zero-DM series is written, read by the
    statistics pass and read again by the vote (4 B x 3 per beam-sample); the
    mask is written (1 B per sample)."""
    import numpy as np
    import torch

    import synth
    from paper_1112_0065_amd import _lib as L

    nsamps, nb = 1 << 19, 13
    pool = synth.fast_chunk(500, nsamps, npulses=4)
    ins = [torch.from_numpy(pool).to("cuda") for _ in range(nb)]
    ws = torch.empty(L.dedisp_rfi_mask_workspace_bytes(nb, nsamps), dtype=torch.uint8,
                     device="cuda")
    mask = torch.empty(nsamps, dtype=torch.uint8, device="cuda")
    L.dedisp_rfi_mask(ins, 1024, nsamps, 3.0, 4, mask, ws)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        n = L.dedisp_rfi_mask(ins, 1024, nsamps, 3.0, 4, mask, ws)
    dt = (time.perf_counter() - t0) / reps
    alg = nb * nsamps * (256 + 12) + nsamps
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ns = 1 << 14
        t_c = time.perf_counter()
        zs = [oracle.zero_dm_series(pool[:ns * 256], ns, 1024) for _ in range(nb)]
        oracle.rfi_mask(zs, 3.0, 4)
        t_c = time.perf_counter() - t_c
        cpu = {"value": ns / t_c, "unit": "13-beam samples/s", "cores": 1, "kind": "oracle",
               "sample": f"13 beams x {ns} samples ({t_c:.2f} s)"}
    return {"beams": nb, "nsamps": nsamps, "ms": dt * 1e3, "masked": n, "cpu_oracle": cpu,
            "samples_per_s": nsamps / dt,
            "algorithmic_bytes": alg, "achieved_GBps": alg / dt / 1e9,
            "hbm_frac": alg / dt / 8e12,
            "note": "includes the host synchronisation of the call; the same payload in every beam"}


if __name__ == "__main__":
    main()
