"""Triage network and candidate tiles (oracle; test infrastructure only).

The paper's section 2.1 warns that radio-frequency interference can swamp a
detection system with false positives.  The learned triage stage scores
each candidate event with a small convolutional network; the paper gives no
network, so this oracle defines the one the GPU path implements:

  tile: 64 DM rows x 256 time steps of an event's boxcar width w,
        rows [d_peak-32, d_peak+32) shifted to fit inside [0, ndm),
        columns t0 + j*w with t0 = t_peak - 128*w clamped to
        [0, n_bx - 255*w - 1] (0 when the series is shorter), value
        (n*B - S1)/sqrt(D) of that row's series (0 where D == 0 or the
        column lies beyond the series), rounded to bfloat16;
  net : 4 x [3x3 conv, pad 1, + bias, ReLU, 2x2 max-pool]
        channels 1 -> 32 -> 32 -> 32 -> 32, 64x256 -> 4x16,
        global average -> fully connected 32 -> 1 -> logit;
  loss: binary cross-entropy with logits, mean over the batch;
  optimiser: Adam on float32 master weights.

Precision follows the GPU: convolution inputs, weights and ReLU outputs are
bfloat16 (round to nearest even), sums are exact here (float64) and float32
on the GPU; the gradients entering the convolution backward (dZ) are rounded
to bfloat16.  ``bf16=False`` gives the same network in plain float64 (for
finite-difference pins).  Max-pool ties go to the first element in raster
order of the 2x2 window.
"""
from __future__ import annotations

import math

import numpy as np

CH = 32
H0, W0 = 64, 256
NLAYERS = 4


# ---------------------------------------------------------------------------
# bfloat16 rounding (round to nearest even on the float32 bit pattern)
# ---------------------------------------------------------------------------

def to_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def bf16_bits(x) -> np.ndarray:
    """float -> bfloat16 bit pattern (uint16), RNE via float32."""
    u = to_f32(x).view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    return ((u + bias) >> 16).astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def round_bf16(x) -> np.ndarray:
    return bf16_value(bf16_bits(x))


# ---------------------------------------------------------------------------
# Parameters
# ---------------------------------------------------------------------------

def param_shapes():
    shapes = [("w1", (CH, 1, 3, 3)), ("b1", (CH,))]
    for l in (2, 3, 4):
        shapes += [(f"w{l}", (CH, CH, 3, 3)), (f"b{l}", (CH,))]
    shapes += [("wf", (CH,)), ("bf", (1,))]
    return shapes


def n_params() -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes())


def init_params(seed: int) -> dict:
    """He-normal conv weights, zero biases, small FC (float32 values)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in param_shapes():
        if name.startswith("w") and name != "wf":
            fan_in = shape[1] * 9
            p[name] = to_f32(rng.standard_normal(shape) * math.sqrt(2.0 / fan_in))
        elif name == "wf":
            p[name] = to_f32(rng.standard_normal(shape) * math.sqrt(1.0 / CH))
        else:
            p[name] = np.zeros(shape, dtype=np.float32)
    return p


# ---------------------------------------------------------------------------
# Layers (NCHW, float64)
# ---------------------------------------------------------------------------

def conv3x3(x, w):
    """z[n,co,y,x] = sum_{ci,ky,kx} xpad[n,ci,y+ky,x+kx] w[co,ci,ky,kx]."""
    n, ci, h, wd = x.shape
    xp = np.zeros((n, ci, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    z = np.zeros((n, w.shape[0], h, wd))
    for ky in range(3):
        for kx in range(3):
            z += np.einsum("nchw,oc->nohw", xp[:, :, ky:ky + h, kx:kx + wd], w[:, :, ky, kx])
    return z


def conv3x3_dgrad(dz, w):
    """dx[n,ci,y,x] = sum_{co,ky,kx} dz[n,co,y-ky+1,x-kx+1] w[co,ci,ky,kx]."""
    n, co, h, wd = dz.shape
    dzp = np.zeros((n, co, h + 2, wd + 2))
    dzp[:, :, 1:-1, 1:-1] = dz
    dx = np.zeros((n, w.shape[1], h, wd))
    for ky in range(3):
        for kx in range(3):
            sl = dzp[:, :, 2 - ky:2 - ky + h, 2 - kx:2 - kx + wd]
            dx += np.einsum("nohw,oc->nchw", sl, w[:, :, ky, kx])
    return dx


def conv3x3_wgrad(x, dz):
    """dw[co,ci,ky,kx] = sum_{n,y,x} dz[n,co,y,x] xpad[n,ci,y+ky,x+kx]."""
    n, ci, h, wd = x.shape
    xp = np.zeros((n, ci, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dw = np.zeros((dz.shape[1], ci, 3, 3))
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", dz, xp[:, :, ky:ky + h, kx:kx + wd])
    return dw


def maxpool2(a):
    """2x2 max-pool; returns (pooled, index of the first maximum 0..3)."""
    n, c, h, w = a.shape
    v = a.reshape(n, c, h // 2, 2, w // 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(n, c, h // 2, w // 2, 4)
    idx = np.argmax(v, axis=-1)          # first maximum in raster order
    return np.take_along_axis(v, idx[..., None], -1)[..., 0], idx


def maxpool2_bwd(dp, idx, shape):
    n, c, h, w = shape
    g = np.zeros((n, c, h // 2, w // 2, 4))
    np.put_along_axis(g, idx[..., None], dp[..., None], -1)
    return g.reshape(n, c, h // 2, w // 2, 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(shape)


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------

def forward(params: dict, tiles, bf16: bool = True):
    """tiles: [N][64][256] (already bf16 values when bf16=True).
    Returns (logits [N], cache)."""
    rb = round_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    x = np.asarray(tiles, dtype=np.float64)[:, None]
    cache = []
    for l in range(1, NLAYERS + 1):
        w = rb(params[f"w{l}"])
        z = conv3x3(x, w) + np.asarray(params[f"b{l}"], np.float64)[None, :, None, None]
        a = rb(np.maximum(z, 0.0))
        p, idx = maxpool2(a)
        cache.append((x, w, a, idx))
        x = p
    g = x.mean(axis=(2, 3))                               # [N][32]
    logits = g @ np.asarray(params["wf"], np.float64) + float(params["bf"][0])
    return logits, (cache, g)


def bce_loss(logits, labels):
    z = np.asarray(logits, np.float64)
    y = np.asarray(labels, np.float64)
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def backward(params: dict, cache, logits, labels, bf16: bool = True) -> dict:
    rb = round_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    layers, g = cache
    n = len(logits)
    y = np.asarray(labels, np.float64)
    dlogit = (1.0 / (1.0 + np.exp(-np.asarray(logits, np.float64))) - y) / n
    grads = {"wf": g.T @ dlogit, "bf": np.array([dlogit.sum()])}
    dg = dlogit[:, None] * np.asarray(params["wf"], np.float64)[None, :]
    x_last = layers[-1][2]
    hp, wp = x_last.shape[2] // 2, x_last.shape[3] // 2
    dp = np.broadcast_to(dg[:, :, None, None] / (hp * wp), (n, CH, hp, wp)).copy()
    for l in range(NLAYERS, 0, -1):
        x, w, a, idx = layers[l - 1]
        da = maxpool2_bwd(dp, idx, a.shape)
        dz = rb(da * (a > 0))
        grads[f"w{l}"] = conv3x3_wgrad(x, dz)
        grads[f"b{l}"] = dz.sum(axis=(0, 2, 3))
        if l > 1:
            dp = conv3x3_dgrad(dz, w)
    return grads


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on float32 master weights (t counts from 1)."""
    out = {}
    for k in params:
        g = np.asarray(grads[k], np.float64)
        m[k] = b1 * np.asarray(m[k], np.float64) + (1 - b1) * g
        v[k] = b2 * np.asarray(v[k], np.float64) + (1 - b2) * g * g
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        out[k] = to_f32(np.asarray(params[k], np.float64) - lr * mh / (np.sqrt(vh) + eps))
    return out


# ---------------------------------------------------------------------------
# Candidate tiles
# ---------------------------------------------------------------------------

def tile_origin(d_peak: int, t_peak: int, w: int, ndm: int, nbx: int):
    d0 = min(max(d_peak - 32, 0), max(ndm - 64, 0))
    t0 = t_peak - 128 * w
    t0 = min(max(t0, 0), max(nbx - 255 * w - 1, 0))
    return d0, t0


def candidate_tile(bw_rows, stats_rows, d_peak, t_peak, w, ndm, nbx):
    """bw_rows[d]: boxcar series of width w for DM d; stats_rows[d] = (n, S1, S2).
    Returns the 64x256 tile as bf16 values (float64 array)."""
    d0, t0 = tile_origin(d_peak, t_peak, w, ndm, nbx)
    tile = np.zeros((64, 256))
    for r in range(64):
        d = d0 + r
        if d >= ndm:
            continue
        n, s1, s2 = stats_rows[d]
        dd = n * s2 - s1 * s1
        if dd == 0:
            continue
        sq = math.sqrt(float(dd))
        for j in range(256):
            t = t0 + j * w
            if t < nbx:
                tile[r, j] = float(np.float32(float(n * int(bw_rows[d][t]) - s1) / sq))
    return round_bf16(tile)
