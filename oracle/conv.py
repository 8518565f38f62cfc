"""FP64 oracle: the 3x3 conv net that warm-starts the depth offsets.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper initialises offsets at zero (Sec. 3.2); the learned warm start is
this build's addition: delta0 = Net(R, G, B, h) with six 3x3 'same'
(zero-padded) convolutions 4 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, ReLU after the
first five, no output activation; the output is an offset in metres.

The depth channel h is the observed depth minus its local 3x3 mean (over
the neighbours inside the image), in units of 2 cm.  Depth itself (metres,
0.5-5 m) would be stored in BF16 with a spacing of 4-31 mm, as coarse as the
centimetre-level sensor noise the converged offsets undo; the high-passed
depth keeps that noise resolvable (BF16 spacing below 0.1 mm at |h| < 1).

Precision model of the GPU path, emulated here where it rounds: weights,
the network input and every stored activation are BF16 (round to nearest
even); products accumulate in FP32 on the GPU (FP64 here); biases are FP32;
the output delta0 is FP32.  In the backward the per-layer gradient of the
pre-activation is rounded to BF16 before it enters the next product.

Layouts: activations [H][W][C]; weights [3][3][C_out][C_in] (tap-major).
"""
from __future__ import annotations

import numpy as np

CHANNELS = [4, 32, 32, 32, 32, 32, 1]
DEPTH_HP_SCALE = 0.02   # metres per unit of the depth channel


def bf16(x):
    """Round float32-representable values to bfloat16, round-to-nearest-even
    (IEEE binary32 with the low 16 mantissa bits rounded away)."""
    a = np.asarray(x, np.float64).astype(np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(a)
    if nan.any():
        out[nan] = np.nan
    return out


def depth_channel(depth):
    """h = (D - mean of D over the 3x3 neighbourhood inside the image) / 2 cm."""
    D = np.asarray(depth, np.float64)
    H, W = D.shape
    s = np.zeros((H, W))
    n = np.zeros((H, W))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            ys = slice(max(0, dy), H + min(0, dy))
            yd = slice(max(0, -dy), H + min(0, -dy))
            xs = slice(max(0, dx), W + min(0, dx))
            xd = slice(max(0, -dx), W + min(0, -dx))
            s[yd, xd] += D[ys, xs]
            n[yd, xd] += 1.0
    return (D - s / n) / DEPTH_HP_SCALE


def net_input(rgb, depth):
    """[H][W][4] input: colour planes and the high-passed depth channel."""
    rgb = np.asarray(rgb, np.float64)
    return np.concatenate([rgb.transpose(1, 2, 0), depth_channel(depth)[..., None]], 2)


def conv3x3(x, w, b=None):
    """Direct definition: y[p][co] = b[co] + sum_{ky,kx,ci} w[ky][kx][co][ci] x[p + (ky-1, kx-1)][ci]."""
    H, W, C = x.shape
    pad = np.zeros((H + 2, W + 2, C))
    pad[1:-1, 1:-1] = x
    cout = w.shape[2]
    y = np.zeros((H, W, cout))
    for ky in range(3):
        for kx in range(3):
            y += pad[ky:ky + H, kx:kx + W] @ w[ky, kx].T
    if b is not None:
        y += b
    return y


def conv3x3_input_grad(dy, w):
    """Adjoint of conv3x3 with respect to its input."""
    H, W, cout = dy.shape
    cin = w.shape[3]
    dpad = np.zeros((H + 2, W + 2, cin))
    for ky in range(3):
        for kx in range(3):
            dpad[ky:ky + H, kx:kx + W] += dy @ w[ky, kx]
    return dpad[1:-1, 1:-1]


def conv3x3_weight_grad(dy, x):
    """Adjoint with respect to the weights: dW[ky][kx][co][ci]."""
    H, W, C = x.shape
    pad = np.zeros((H + 2, W + 2, C))
    pad[1:-1, 1:-1] = x
    cout = dy.shape[2]
    dw = np.zeros((3, 3, cout, C))
    d2 = dy.reshape(-1, cout)
    for ky in range(3):
        for kx in range(3):
            dw[ky, kx] = d2.T @ pad[ky:ky + H, kx:kx + W].reshape(-1, C)
    return dw


def init_params(seed):
    """He-uniform weights and zero biases (the last layer starts at zero
    output scale 0.1x so the untrained net predicts offsets near 0)."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(6):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        lim = np.sqrt(6.0 / (9 * cin))
        w = rng.uniform(-lim, lim, size=(3, 3, cout, cin))
        if l == 5:
            w *= 0.1
        params.append((w.astype(np.float32), np.zeros(cout, np.float32)))
    return params


def forward(params, x0, emulate_bf16=True):
    """Returns (delta0 [H][W], list of stored activations, list of pre-acts)."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, np.float64))
    acts = [r(x0)]
    pres = []
    for l, (w, b) in enumerate(params):
        pre = conv3x3(acts[-1], r(w), np.asarray(b, np.float64))
        pres.append(pre)
        if l < 5:
            acts.append(r(np.maximum(pre, 0.0)))
    return pres[-1][..., 0], acts, pres


def backward(params, acts, d_delta, emulate_bf16=True):
    """Gradients (dW, db) per layer for an upstream grad d_delta [H][W]."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, np.float64))
    grads = [None] * 6
    dpre = r(np.asarray(d_delta, np.float64)[..., None])
    for l in range(5, -1, -1):
        w, _ = params[l]
        grads[l] = (conv3x3_weight_grad(dpre, acts[l]), dpre.sum((0, 1)))
        if l > 0:
            dx = conv3x3_input_grad(dpre, r(w))
            dpre = r(dx * (acts[l] > 0))
    return grads


def l1(delta0, target):
    """Training loss: mean |delta0 - delta*| and its gradient."""
    e = np.asarray(delta0, np.float64) - np.asarray(target, np.float64)
    return float(np.abs(e).mean()), np.sign(e) / e.size
