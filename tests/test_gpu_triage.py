"""GPU tests of the triage network: tiles, forward, backward and Adam
against the oracle (same bfloat16 rounding points; float32 vs float64 sums),
reproducible training, save / load, fallback on a bad model."""
import os

import numpy as np
import pytest

import oracle
from oracle import cnn
from gpu_common import log, small_case, to_dev, torch_dev

pytestmark = pytest.mark.gpu

ORDER = [n for n, _ in cnn.param_shapes()]


def flat(params):
    return np.concatenate([np.asarray(params[k], np.float32).reshape(-1) for k in ORDER])


def unflat(v):
    out, o = {}, 0
    for name, shape in cnn.param_shapes():
        k = int(np.prod(shape))
        out[name] = np.asarray(v[o:o + k], np.float64).reshape(shape)
        o += k
    return out


def _params(seed):
    p = cnn.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for k in p:
        if k.startswith("b"):
            p[k] = cnn.to_f32(rng.standard_normal(p[k].shape) * 0.05)
    return p


def _tiles(seed, n):
    rng = np.random.default_rng(seed)
    t = rng.standard_normal((n, 64, 256))
    t[::2, 28:36, 100:160] += 3.0        # a bright patch on half of them
    return cnn.bf16_bits(t), cnn.round_bf16(t)


def _dev_tiles(bits):
    return to_dev(bits.view(np.int16))


def test_forward_backward_match_oracle():
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    p = _params(1)
    bits, vals = _tiles(2, 8)
    labels = np.array([1, 0] * 4, np.float64)
    m = L.triage_create(None, 0)
    L.triage_set_params(m, flat(p))
    t = _dev_tiles(bits)
    lab = torch.tensor(labels, dtype=torch.float32, device="cuda")
    logits = torch.empty(8, dtype=torch.float32, device="cuda")
    L.triage_forward(m, t, 8, logits=logits)
    torch.cuda.synchronize()
    ref_logits, cache = cnn.forward({k: v for k, v in p.items()}, vals, bf16=True)
    got = logits.cpu().numpy()
    log("logits gpu", got[:4], "ref", ref_logits[:4])
    assert np.all(np.abs(got - ref_logits) <= 1e-2 * (1 + np.abs(ref_logits)))
    loss = L.triage_forward_backward(m, t, lab, 8)
    assert loss == pytest.approx(cnn.bce_loss(ref_logits, labels), rel=1e-2, abs=1e-3)
    _, g = L.triage_get_params(m)
    ref = cnn.backward(p, cache, ref_logits, labels, bf16=True)
    gg = unflat(g)
    for k in ORDER:
        num = np.linalg.norm(gg[k] - ref[k])
        den = np.linalg.norm(ref[k]) + 1e-12
        log("grad", k, "rel L2", num / den)
        assert num / den <= 2e-2, k


def test_score_is_sigmoid_of_forward_logit():
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    p = _params(2)
    bits, vals = _tiles(9, 5)
    m = L.triage_create(None, 0)
    L.triage_set_params(m, flat(p))
    t = _dev_tiles(bits)
    logits = torch.empty(5, dtype=torch.float32, device="cuda")
    scores = torch.empty(5, dtype=torch.float32, device="cuda")
    L.triage_forward(m, t, 5, logits=logits)
    L.triage_score(m, t, 5, scores)
    torch.cuda.synchronize()
    ref_logits, _ = cnn.forward(p, vals, bf16=True)
    lg = logits.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(lg - ref_logits) <= 1e-2 * (1 + np.abs(ref_logits)))
    assert np.allclose(scores.cpu().numpy(), 1.0 / (1.0 + np.exp(-lg)), rtol=1e-6, atol=1e-7)


def test_adam_step_matches_oracle():
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    p = _params(3)
    bits, vals = _tiles(4, 6)
    labels = np.array([1, 0, 1, 1, 0, 0], np.float64)
    m = L.triage_create(None, 0)
    L.triage_set_params(m, flat(p))
    lab = torch.tensor(labels, dtype=torch.float32, device="cuda")
    L.triage_train_step(m, _dev_tiles(bits), lab, 6, lr=1e-3)
    new, g = L.triage_get_params(m)
    # oracle step from the GPU's own gradient isolates the optimiser
    mm = {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in p.items()}
    vv = {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in p.items()}
    want = cnn.adam_step(p, unflat(g), mm, vv, 1, lr=1e-3)
    assert np.allclose(new, flat(want), rtol=1e-5, atol=1e-7)


def test_adam_chain_of_steps_matches_oracle():
    """Six consecutive training steps on batches whose labels flip and whose
    tiles change, so the gradients change sign and size from step to step:
    after every step the GPU's parameters equal a chain of oracle Adam steps
    (t = 1..6, the moments carried over) fed the GPU's own gradients.  Step
    counts, both decay rates and the bias corrections all enter from the
    second step on."""
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    p = _params(4)
    m = L.triage_create(None, 0)
    L.triage_set_params(m, flat(p))
    mm = {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in p.items()}
    vv = {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in p.items()}
    ref = {k: np.asarray(v, np.float32) for k, v in p.items()}
    lr = 2e-3
    prev_g = None
    for t in range(1, 7):
        bits, _ = _tiles(40 + t, 8)
        labels = np.array([1, 0] * 4 if t % 2 else [0, 1] * 4, np.float64)
        lab = torch.tensor(labels, dtype=torch.float32, device="cuda")
        L.triage_train_step(m, _dev_tiles(bits), lab, 8, lr=lr)
        new, g = L.triage_get_params(m)
        ref = cnn.adam_step(ref, unflat(g), mm, vv, t, lr=lr)
        want = flat(ref)
        err = np.abs(new - want).max()
        log("adam step", t, "max |gpu - oracle|", err)
        assert np.allclose(new, want, rtol=1e-5, atol=1e-7), t
        if prev_g is not None:
            assert (np.sign(g) != np.sign(prev_g)).mean() > 0.1   # the gradients really change
        prev_g = g
        ref = {k: np.asarray(v, np.float32) for k, v in unflat(new).items()}


def test_training_reproducible_and_resumable(tmp_path):
    """N+M steps equal N steps, save, load, M steps -- bit for bit; loss
    decreases on a separable toy set."""
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    bits, _ = _tiles(5, 64)
    labels = torch.tensor([1.0, 0.0] * 32, device="cuda")
    t = _dev_tiles(bits)
    a = L.triage_create(None, 11)
    losses = [L.triage_train_step(a, t, labels, 64, lr=3e-3) for _ in range(12)]
    log("toy losses", losses)
    assert losses[-1] < 0.95 * losses[0] and min(losses[6:]) < min(losses[:3])
    b = L.triage_create(None, 11)
    for _ in range(7):
        L.triage_train_step(b, t, labels, 64, lr=3e-3)
    path = str(tmp_path / "m.bin")
    L.triage_save(b, path)
    c = L.triage_create(path)
    for _ in range(5):
        L.triage_train_step(c, t, labels, 64, lr=3e-3)
    pa, _ = L.triage_get_params(a)
    pc, _ = L.triage_get_params(c)
    assert pa.tobytes() == pc.tobytes()


def test_bad_models_are_rejected(tmp_path):
    from paper_1112_0065_amd import _lib as L
    torch_dev()
    with pytest.raises(L.DedispError) as e:
        L.triage_create(str(tmp_path / "missing.bin"))
    assert e.value.status == L.ERR_INVALID_ARG
    m = L.triage_create(None, 1)
    p, _ = L.triage_get_params(m)
    path = str(tmp_path / "nan.bin")
    p[5] = np.nan
    L.triage_set_params(m, np.nan_to_num(p))
    L.triage_save(m, path)
    raw = bytearray(open(path, "rb").read())
    raw[16 + 4 * 5:16 + 4 * 6] = np.array([np.nan], np.float32).tobytes()
    open(path, "wb").write(bytes(raw))
    with pytest.raises(L.DedispError):
        L.triage_create(path)


def test_tiles_match_oracle():
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    fb, dly, x, out = small_case()
    ndm, nout = out.shape
    series = to_dev(out.astype(np.uint16).view(np.int16))
    pws = torch.empty(L.find_peaks_workspace_bytes(ndm, nout, fb.widths), dtype=torch.uint8, device="cuda")
    evb = torch.empty(4096 * 40, dtype=torch.uint8, device="cuda")
    n = L.find_peaks(series, ndm, nout, fb.widths, fb.snr_thresh, evb, 4096, pws)
    ev = L.events_from_buffer(evb, n)
    pick = list(range(0, n, max(1, n // 6)))[:6]
    sub = np.concatenate([ev[i:i + 1] for i in pick])
    evd = to_dev(np.frombuffer(sub.tobytes(), np.uint8).copy())
    tiles = torch.empty((len(pick), 64, 256), dtype=torch.int16, device="cuda")
    L.triage_tiles(series, ndm, nout, fb.widths, pws, evd, len(pick), tiles)
    got = cnn.bf16_value(tiles.cpu().numpy().view(np.uint16))
    bw = oracle.boxcar(out, fb.widths)
    nbx = bw.shape[2]
    for k, e in enumerate(sub):
        wi = int(e["width_idx"])
        stats = [oracle.series_stats(bw[wi, d]) for d in range(ndm)]
        ref = cnn.candidate_tile(bw[wi], stats, int(e["dm_idx"]), int(e["t_peak"]),
                                 fb.widths[wi], ndm, nbx)
        assert (got[k] == ref).all(), k
