"""Pins of the triage-network oracle: parameter count, bfloat16 rounding,
finite differences of the float64 network, and a float64 cross-check with
torch's CPU convolution / pooling and autograd (library cross-check)."""
import math

import numpy as np
import pytest

from oracle import cnn


def test_parameter_count():
    # 32*9+32 + 3*(32*32*9+32) + 32+1
    assert cnn.n_params() == 28097


def test_bf16_round_to_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7 + 2 ** -8, -2.5,
                     0.0, 3.0e38, 1e-40])
    bits = cnn.bf16_bits(vals)
    assert bits[0] == 0x3F80
    assert bits[1] == 0x3F80          # tie -> even (down)
    assert bits[2] == 0x3F82          # tie -> even (up)
    assert bits[3] == 0x3F82          # tie between 0x3F81 and 0x3F82 -> even
    assert bits[4] == 0xC020
    assert bits[5] == 0
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([vals[:6], rng.standard_normal(10000) * 10.0 ** rng.integers(-8, 8, 10000)])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert (cnn.bf16_bits(x) == ref).all()


def _torch_net(params, tiles):
    import torch
    import torch.nn.functional as F
    x = torch.tensor(np.asarray(tiles, np.float64))[:, None]
    tp = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in params.items()}
    for l in range(1, 5):
        x = F.max_pool2d(F.relu(F.conv2d(x, tp[f"w{l}"], tp[f"b{l}"], padding=1)), 2)
    g = x.mean(dim=(2, 3))
    return g @ tp["wf"] + tp["bf"][0], tp


def _rand_params(seed):
    rng = np.random.default_rng(seed)
    p = cnn.init_params(seed)
    for k in p:
        if k.startswith("b"):
            p[k] = cnn.to_f32(rng.standard_normal(p[k].shape) * 0.05)
    return p


def test_forward_and_grads_match_torch_float64():
    import torch
    p = _rand_params(3)
    rng = np.random.default_rng(4)
    tiles = rng.standard_normal((3, 64, 256))
    labels = np.array([1.0, 0.0, 1.0])
    logits, cache = cnn.forward(p, tiles, bf16=False)
    tl, tp = _torch_net(p, tiles)
    assert np.allclose(logits, tl.detach().numpy(), rtol=1e-12, atol=1e-12)
    loss = torch.nn.functional.binary_cross_entropy_with_logits(tl, torch.tensor(labels))
    assert cnn.bce_loss(logits, labels) == pytest.approx(loss.item(), rel=1e-12)
    loss.backward()
    grads = cnn.backward(p, cache, logits, labels, bf16=False)
    for k, t in tp.items():
        assert np.allclose(grads[k], t.grad.numpy(), rtol=1e-9, atol=1e-12), k


def test_backward_finite_differences():
    """Central differences of the float64 network (no library involved)."""
    p = {k: np.asarray(v, np.float64) for k, v in _rand_params(5).items()}
    rng = np.random.default_rng(6)
    tiles = rng.standard_normal((2, 64, 256))
    labels = np.array([0.0, 1.0])
    logits, cache = cnn.forward(p, tiles, bf16=False)
    grads = cnn.backward(p, cache, logits, labels, bf16=False)
    eps = 1e-6
    for k in ["w1", "b1", "w2", "b3", "w4", "b4", "wf", "bf"]:
        flat = p[k].reshape(-1)
        for i in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[i]
            flat[i] = old + eps
            lp = cnn.bce_loss(cnn.forward(p, tiles, bf16=False)[0], labels)
            flat[i] = old - eps
            lm = cnn.bce_loss(cnn.forward(p, tiles, bf16=False)[0], labels)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            an = grads[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-8, (k, i, fd, an)


def test_bf16_network_close_to_float64():
    p = _rand_params(7)
    rng = np.random.default_rng(8)
    tiles = cnn.round_bf16(rng.standard_normal((4, 64, 256)))
    l16, _ = cnn.forward(p, tiles, bf16=True)
    l64, _ = cnn.forward(p, tiles, bf16=False)
    assert np.allclose(l16, l64, rtol=5e-2, atol=5e-2)


def test_adam_first_step_is_sign_step():
    p = {"a": np.array([1.0, -2.0, 3.0], np.float32)}
    g = {"a": np.array([0.5, -0.25, 1e-3])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    out = cnn.adam_step(p, g, m, v, 1, lr=1e-3)
    # t = 1: m_hat = g, v_hat = g^2 -> step = lr * g / (|g| + eps)
    want = p["a"] - 1e-3 * g["a"] / (np.abs(g["a"]) + 1e-8)
    assert np.allclose(out["a"], want, rtol=0, atol=1e-7)


def test_tile_origin_and_values():
    assert cnn.tile_origin(5, 1000, 2, 1200, 500000) == (0, 744)
    assert cnn.tile_origin(1190, 100, 4, 1200, 500000) == (1136, 0)
    assert cnn.tile_origin(600, 499990, 1, 1200, 500000) == (568, 500000 - 256)
    # short series: origin 0, columns beyond the series are zero
    rows = [np.arange(100)] * 64
    stats = [(100, int(np.arange(100).sum()), int((np.arange(100) ** 2).sum()))] * 64
    t = cnn.candidate_tile(rows, stats, 10, 50, 1, 64, 100)
    n, s1, s2 = stats[0]
    assert t[0, 0] == cnn.round_bf16(np.float32((0 * n - s1) / math.sqrt(n * s2 - s1 * s1)))
    assert (t[:, 100:] == 0).all()


def test_adam_three_steps_hand_computed():
    """Three Adam steps on two parameters whose gradients change sign and
    size at every step, so that the moment decays (beta1 = 0.9 on the mean,
    beta2 = 0.999 on the square), the bias corrections 1 - beta^t and the
    step count all change the result.  Expected values worked out by hand
    from the update
        m_t = b1 m_{t-1} + (1 - b1) g_t,   v_t = b2 v_{t-1} + (1 - b2) g_t^2,
        p_t = p_{t-1} - lr (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps)
    with lr = 0.1; e.g. for the first parameter at t = 2:
        m_2 = 0.9 * 0.05 + 0.1 * (-2) = -0.155,
        v_2 = 0.999 * 0.00025 + 0.001 * 4 = 0.00424975,
        m_2 / 0.19 = -0.815789..., v_2 / 0.001999 = 2.125938...,
        p_2 = 0.9 + 0.1 * 0.815789 / 1.458060 = 0.955950.
    (Swapping beta1 and beta2 gives 0.950337 there; running step 2 with
    t = 1 gives 0.997405.)"""
    p = {"a": np.array([1.0, -0.5], np.float32)}
    gs = [np.array([0.5, 1e-3]), np.array([-2.0, 3.0]), np.array([0.25, -0.5])]
    want = [np.array([0.9000000020, -0.5999990000]),
            np.array([0.9559503510, -0.6744350020]),
            np.array([0.9911908279, -0.7206834531])]
    want_m = [np.array([0.05, 1e-4]), np.array([-0.155, 0.30009]), np.array([-0.1145, 0.220081])]
    want_v = [np.array([2.5e-4, 1e-9]), np.array([0.00424975, 0.009000000999]),
              np.array([0.00430800025, 0.009241000998001])]
    m = {"a": np.zeros(2)}
    v = {"a": np.zeros(2)}
    for t in range(1, 4):
        p = cnn.adam_step(p, {"a": gs[t - 1]}, m, v, t, lr=0.1)
        assert p["a"].dtype == np.float32
        assert np.allclose(m["a"], want_m[t - 1], rtol=1e-12, atol=0)
        assert np.allclose(v["a"], want_v[t - 1], rtol=1e-12, atol=0)
        assert np.allclose(p["a"], want[t - 1], rtol=0, atol=2e-7), (t, p["a"], want[t - 1])
