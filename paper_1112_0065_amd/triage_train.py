"""Training data, training and evaluation of the triage network.

Candidates come from the pipeline itself: seeded synthetic beams with
injected dispersed pulses and interference (zero-DM impulses, narrowband
channels, 50 Hz periodic) are dedispersed and searched on the GPU, the
events are thinned by per-width non-maximum suppression, labelled against
the injections, and turned into 64-DM x 256-step tiles by the library's
tile kernel.  The network is trained with the library's own forward,
backward and Adam kernels.  The plain S/N detector (every candidate kept)
is both the fallback and the yardstick: triage keeps a candidate when its score
reaches a threshold chosen on the validation beams so that recall stays
within half a percent of the plain detector's.

Run on a GPU:  python -m paper_1112_0065_amd.triage_train --out DIR
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import _lib as L

WIDTHS = [1 << i for i in range(10)]
SNR = 6.0
NSAMPS = 1 << 17
# beam seeds: training from TRAIN_SEED on; validation 600.., test 700..;
# 800.. is left for independent evaluations
TRAIN_SEED = 10000


def nms(events: np.ndarray, ndm: int) -> np.ndarray:
    """Candidates: per-width non-maximum suppression (the library's
    dedisp_candidates_nms, which the streaming server runs too): keep the
    highest-S/N event of every 64-DM x 256*w-sample window (ties to the lower
    (dm, t)).  Returns indices."""
    return L.dedisp_candidates_nms(events, WIDTHS, 32, 128)


def label(events: np.ndarray, fb, sweep_trial: np.ndarray):
    """An event matches injected pulse p when its peak time and band-crossing
    delay are both within max(w, W_p) (+2 samples in time) of the pulse's.
    sweep_trial[d]: delay of the lowest channel at trial d (samples).
    Returns (labels 0/1, matched pulse index or -1)."""
    import synth
    lab = np.zeros(len(events), np.float32)
    match = np.full(len(events), -1, np.int64)
    psweep = [int(synth.sky_arrival_offsets(fb.nchans, fb.f_top, fb.df, fb.tsamp, p.dm)[-1])
              for p in fb.pulses]
    for i, e in enumerate(events):
        w = WIDTHS[int(e["width_idx"])]
        for j, p in enumerate(fb.pulses):
            tol = max(w, p.width)
            if abs(int(e["t_peak"]) - p.t0) <= tol + 2 and \
                    abs(int(sweep_trial[int(e["dm_idx"])]) - psweep[j]) <= tol:
                lab[i] = 1.0
                match[i] = j
                break
    return lab, match


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "triage_weights.bin")


def load_default():
    """The committed trained network and its score cut: (model, tau, report)."""
    with open(os.path.splitext(WEIGHTS)[0] + ".json") as f:
        report = json.load(f)
    return L.triage_create(WEIGHTS), float(report["tau"]), report


def _gen(seed):
    import synth
    return synth.make_rfi_beam(seed, NSAMPS)


def beams(seeds, procs=None):
    procs = procs or max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(procs) as pool:
        for fb in pool.imap(_gen, seeds):
            yield fb


def build(seeds, procs=None, log=print):
    """Run the search on every beam and return (tiles uint16 [n][64][256],
    labels [n], per-beam records)."""
    import torch
    tiles, labels, recs = [], [], []
    plan = None
    for fb in beams(seeds, procs):
        if plan is None:
            plan = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
            sweep = L.dedisp_plan_copy_delays(plan)[:, -1]
            nout = fb.nsamps - plan.max_delay
            ws = torch.empty(L.dedisp_workspace_bytes(plan, fb.nsamps), dtype=torch.uint8, device="cuda")
            out = torch.empty((plan.ndm, nout), dtype=torch.int16, device="cuda")
            pws = torch.empty(L.find_peaks_workspace_bytes(plan.ndm, nout, WIDTHS), dtype=torch.uint8,
                              device="cuda")
            evb = torch.empty((1 << 20) * 40, dtype=torch.uint8, device="cuda")
        L.dedisp_execute(plan, torch.from_numpy(fb.packed).to("cuda"), fb.nsamps, out, ws)
        n = L.find_peaks(out, plan.ndm, nout, WIDTHS, SNR, evb, 1 << 20, pws)
        ev = L.events_from_buffer(evb, n)
        keep = nms(ev, plan.ndm)
        cand = ev[keep]
        lab, match = label(cand, fb, sweep)
        if len(cand):
            evd = torch.from_numpy(np.frombuffer(cand.tobytes(), np.uint8).copy()).to("cuda")
            t = torch.empty((len(cand), 64, 256), dtype=torch.int16, device="cuda")
            L.triage_tiles(out, plan.ndm, nout, WIDTHS, pws, evd, len(cand), t)
            tiles.append(t.cpu().numpy().view(np.uint16))
            labels.append(lab)
        recs.append(dict(seed=fb.seed, npulses=len(fb.pulses), events=int(n), candidates=len(cand),
                         positives=int(lab.sum()), match=match.tolist()))
        log(f"beam {fb.seed}: {n} events, {len(cand)} candidates, {int(lab.sum())} positive")
    return (np.concatenate(tiles) if tiles else np.zeros((0, 64, 256), np.uint16),
            np.concatenate(labels) if labels else np.zeros(0, np.float32), recs)


def scores(model, tiles: np.ndarray, batch: int = 1024) -> np.ndarray:
    import torch
    out = []
    for i in range(0, len(tiles), batch):
        t = torch.from_numpy(tiles[i:i + batch].view(np.int16)).to("cuda")
        s = torch.empty(len(t), dtype=torch.float32, device="cuda")
        L.triage_forward(model, t, len(t), scores=s)
        out.append(s.cpu().numpy())
    return np.concatenate(out) if out else np.zeros(0, np.float32)


def evaluate(sc: np.ndarray, recs, tau: float) -> dict:
    """Recall over injected pulses and false-candidate rate, plain detector
    (every candidate kept) against triage (score >= tau)."""
    off = 0
    found_plain = found_tri = total = 0
    fp_plain = fp_tri = 0
    for r in recs:
        m = np.array(r["match"], np.int64)
        s = sc[off:off + len(m)]
        off += len(m)
        total += r["npulses"]
        found_plain += len(set(m[m >= 0].tolist()))
        found_tri += len(set(m[(m >= 0) & (s >= tau)].tolist()))
        fp_plain += int((m < 0).sum())
        fp_tri += int(((m < 0) & (s >= tau)).sum())
    return dict(pulses=total, recall_plain=found_plain / max(total, 1),
                recall_triage=found_tri / max(total, 1), false_plain=fp_plain, false_triage=fp_tri,
                fpr_triage_vs_plain=fp_tri / max(fp_plain, 1), tau=tau)


def choose_tau(sc, recs, slack=0.005):
    best = 0.0
    for tau in np.linspace(0.01, 0.99, 99):
        r = evaluate(sc, recs, float(tau))
        if r["recall_triage"] >= r["recall_plain"] - slack:
            best = float(tau)
    return best


def train(model, tiles, labels, epochs, batch=256, lr=1e-3, seed=0, log=print):
    import torch
    rng = np.random.default_rng(seed)
    n = len(tiles)
    dt = torch.from_numpy(tiles.view(np.int16)).to("cuda")
    dl = torch.from_numpy(labels.astype(np.float32)).to("cuda")
    losses = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to("cuda")
        tot, k = 0.0, 0
        for i in range(0, n - batch + 1, batch):
            sel = perm[i:i + batch]
            tot += L.triage_train_step(model, dt[sel].contiguous(), dl[sel].contiguous(), batch, lr)
            k += 1
        losses.append(tot / max(k, 1))
        log(f"epoch {ep}: loss {losses[-1]:.4f}")
    return losses


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--train", type=int, default=640)
    ap.add_argument("--val", type=int, default=80)
    ap.add_argument("--test", type=int, default=80)
    ap.add_argument("--epochs", type=int, default=15)
    ap.add_argument("--lr", type=float, default=1e-3)
    args = ap.parse_args()

    def log(*a):
        print(*a, flush=True)

    os.makedirs(args.out, exist_ok=True)
    t0 = time.time()
    tr = build(range(TRAIN_SEED, TRAIN_SEED + args.train), log=log)
    va = build(range(600, 600 + args.val), log=log)
    te = build(range(700, 700 + args.test), log=log)
    log(f"datasets built in {time.time() - t0:.1f} s: train {len(tr[1])} ({int(tr[1].sum())} pos), "
        f"val {len(va[1])}, test {len(te[1])}")
    model = L.triage_create(None, 1)
    t1 = time.time()
    losses = train(model, tr[0], tr[1], args.epochs, lr=args.lr, log=log)
    t_train = time.time() - t1
    tau = choose_tau(scores(model, va[0]), va[2])
    res_val = evaluate(scores(model, va[0]), va[2], tau)
    res_test = evaluate(scores(model, te[0]), te[2], tau)
    path = os.path.join(args.out, "triage.bin")
    L.triage_save(model, path)
    report = dict(train_candidates=len(tr[1]), train_positives=int(tr[1].sum()), epochs=args.epochs,
                  lr=args.lr, batch=256, losses=losses, train_seconds=t_train, tau=tau,
                  val=res_val, test=res_test, nsamps=NSAMPS, widths=WIDTHS, snr_thresh=SNR,
                  seeds=dict(train=[TRAIN_SEED, TRAIN_SEED + args.train], val=[600, 600 + args.val],
                             test=[700, 700 + args.test]))
    with open(os.path.join(args.out, "triage.json"), "w") as f:
        json.dump(report, f, indent=1)
    log(json.dumps(report))


if __name__ == "__main__":
    sys.exit(main())
