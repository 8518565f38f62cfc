"""Pins for the conv-net oracle (CPU only): library convolutions, torch
autograd, finite differences and the BF16 rounding definition."""
import numpy as np
import pytest
import scipy.signal

from oracle import conv


def test_conv3x3_matches_scipy_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(9, 11, 3))
    w = rng.normal(size=(3, 3, 4, 3))
    b = rng.normal(size=4)
    y = conv.conv3x3(x, w, b)
    for co in range(4):
        ref = b[co] + sum(scipy.signal.correlate2d(x[:, :, ci], w[:, :, co, ci], mode="same")
                          for ci in range(3))
        np.testing.assert_allclose(y[:, :, co], ref, atol=1e-12)


def test_conv_adjoints_match_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = rng.normal(size=(7, 6, 5))
    w = rng.normal(size=(3, 3, 4, 5))
    dy = rng.normal(size=(7, 6, 4))
    xt = torch.tensor(x.transpose(2, 0, 1)[None], requires_grad=True)
    wt = torch.tensor(w.transpose(2, 3, 0, 1), requires_grad=True)   # [co][ci][ky][kx]
    yt = torch.nn.functional.conv2d(xt, wt, padding=1)
    np.testing.assert_allclose(yt[0].detach().numpy().transpose(1, 2, 0), conv.conv3x3(x, w), atol=1e-12)
    yt.backward(torch.tensor(dy.transpose(2, 0, 1)[None]))
    np.testing.assert_allclose(conv.conv3x3_input_grad(dy, w), xt.grad[0].numpy().transpose(1, 2, 0), atol=1e-11)
    np.testing.assert_allclose(conv.conv3x3_weight_grad(dy, x), wt.grad.numpy().transpose(2, 3, 0, 1), atol=1e-11)


def test_bf16_rounding_definition():
    one = 1.0
    assert conv.bf16(one) == 1.0
    assert conv.bf16(1.0 + 2.0 ** -8) == 1.0                       # tie -> even
    assert conv.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6       # tie -> even (up)
    assert conv.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert conv.bf16(-2.5) == -2.5
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    v = rng.normal(size=10000).astype(np.float32) * 10
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(conv.bf16(v), ref)


def test_network_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    params = conv.init_params(0)
    params = [(w.astype(np.float64), rng.normal(size=b.shape) * 0.1) for w, b in params]
    x0 = rng.uniform(size=(6, 5, 4))
    tgt = rng.normal(size=(6, 5)) * 0.01
    d0, acts, _ = conv.forward(params, x0, emulate_bf16=False)
    _, g = conv.l1(d0, tgt)
    grads = conv.backward(params, acts, g, emulate_bf16=False)
    h = 1e-6
    for l, (ci, co, ky, kx) in [(0, (1, 3, 0, 2)), (2, (5, 7, 1, 1)), (5, (9, 0, 2, 0))]:
        w = params[l][0]
        old = w[ky, kx, co, ci]
        w[ky, kx, co, ci] = old + h
        lp = conv.l1(conv.forward(params, x0, False)[0], tgt)[0]
        w[ky, kx, co, ci] = old - h
        lm = conv.l1(conv.forward(params, x0, False)[0], tgt)[0]
        w[ky, kx, co, ci] = old
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grads[l][0][ky, kx, co, ci]) < 1e-7 + 1e-5 * abs(fd)
    b = params[3][1]
    old = b[4]
    b[4] = old + h
    lp = conv.l1(conv.forward(params, x0, False)[0], tgt)[0]
    b[4] = old - h
    lm = conv.l1(conv.forward(params, x0, False)[0], tgt)[0]
    b[4] = old
    assert abs((lp - lm) / (2 * h) - grads[3][1][4]) < 1e-7
