"""Pins of the SSIM term of Eq. 1 in the oracle: the window, the zero-padded
filter against scipy's correlation, SSIM(x, x) = 1, closed forms on constant
images (interior and a corner, where the window mass inside the image sets
the statistics), finite differences and a torch float64 autograd
re-derivation of the gradient."""
import numpy as np
import pytest
import scipy.ndimage

from oracle import loss


def test_window_is_the_normalised_gaussian():
    g = loss.ssim_window()
    assert g.shape == (11,) and abs(g.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(g, g[::-1], rtol=0, atol=0)
    # neighbouring taps differ by exp(-(k^2 - (k-1)^2) / (2 sigma^2))
    for k in range(1, 6):
        assert abs(g[5 + k] / g[5 + k - 1] - np.exp(-(2 * k - 1) / (2 * 1.5 ** 2))) < 1e-14


def test_filter_equals_scipy_zero_padded_correlation():
    rng = np.random.default_rng(0)
    img = rng.normal(size=(23, 31))
    g = loss.ssim_window()
    ref = scipy.ndimage.correlate1d(scipy.ndimage.correlate1d(img, g, axis=1, mode="constant", cval=0.0),
                                    g, axis=0, mode="constant", cval=0.0)
    np.testing.assert_allclose(loss.ssim_filter(img), ref, rtol=1e-13, atol=1e-14)
    # a single impulse spreads into the window itself (correlation orientation)
    imp = np.zeros((15, 15))
    imp[7, 7] = 1.0
    np.testing.assert_allclose(loss.ssim_filter(imp)[2:13, 2:13], np.outer(g, g), rtol=1e-14, atol=1e-17)


def test_identical_images_have_unit_ssim_and_no_gradient():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(3, 20, 26))
    np.testing.assert_allclose(loss.ssim_map(x[0], x[0]), 1.0, atol=1e-12)
    L, g = loss.ssim_loss(x, x)
    assert abs(L) < 1e-12 and np.abs(g).max() < 1e-12


def test_constant_images_closed_form_interior_and_corner():
    """x = a, y = b: where the window mass inside the image is s, mu = a s,
    sigma_x^2 = a^2 s (1 - s), sigma_xy = a b s (1 - s); in the interior
    (s = 1) SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.7, 0.3
    H, W = 30, 40
    S = loss.ssim_map(np.full((H, W), a), np.full((H, W), b))
    C1, C2 = loss.SSIM_C1, loss.SSIM_C2
    # (the sigma terms vanish up to rounding of order 1e-16, divided by C2 ~ 1e-3)
    assert abs(S[15, 20] - (2 * a * b + C1) / (a * a + b * b + C1)) < 1e-12
    g = loss.ssim_window()
    for (y, x) in ((0, 0), (2, 37), (29, 3)):
        sy = g[max(0, 5 - y):min(11, H - y + 5)].sum()
        sx = g[max(0, 5 - x):min(11, W - x + 5)].sum()
        s = sy * sx
        v = s * (1 - s)
        ref = ((2 * a * b * s * s + C1) * (2 * a * b * v + C2)) / (((a * a + b * b) * s * s + C1) * ((a * a + b * b) * v + C2))
        assert abs(S[y, x] - ref) < 1e-12, (y, x)


def test_ssim_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    t = rng.uniform(size=(3, 13, 17))
    r = np.clip(t + rng.normal(size=t.shape) * 0.1, 0, 1)
    L, g = loss.ssim_loss(r, t)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 6, 8), (2, 12, 16), (0, 3, 15), (2, 11, 1)]:
        a = r.copy()
        b = r.copy()
        a[idx] += h
        b[idx] -= h
        fd = (loss.ssim_loss(a, t)[0] - loss.ssim_loss(b, t)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-8 + 1e-6 * abs(fd), (idx, fd, g[idx])


def test_ssim_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    t = rng.uniform(size=(3, 19, 24))
    r = np.clip(t + rng.normal(size=t.shape) * 0.2, 0, 1)
    L, g = loss.ssim_loss(r, t)
    w1 = torch.tensor(loss.ssim_window(), dtype=torch.float64)
    win = (w1[:, None] * w1[None, :])[None, None]
    y = torch.tensor(r, dtype=torch.float64, requires_grad=True)
    x = torch.tensor(t, dtype=torch.float64)
    f = lambda img: torch.nn.functional.conv2d(img[:, None], win, padding=5)[:, 0]
    mx, my = f(x), f(y)
    sxx, syy, sxy = f(x * x) - mx * mx, f(y * y) - my * my, f(x * y) - mx * my
    C1, C2 = loss.SSIM_C1, loss.SSIM_C2
    S = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
    Lt = 1 - S.mean()
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-14
    np.testing.assert_allclose(y.grad.numpy(), g, rtol=1e-10, atol=1e-15)


def test_mapping_loss_is_eq1_with_supplement_weights():
    rng = np.random.default_rng(4)
    t = rng.uniform(size=(3, 12, 14))
    r = rng.uniform(size=(3, 12, 14))
    d, td = rng.uniform(1, 3, size=(12, 14)), rng.uniform(1, 3, size=(12, 14))
    td[::4, ::3] = 0.0
    L, gr, gd = loss.mapping_loss(r, d, t, td)
    L1, g1, gd1 = loss.l1_loss(r, d, t, td)
    Ls, gs = loss.ssim_loss(r, t)
    assert abs(L - (L1 + 0.2 * Ls)) < 1e-15
    np.testing.assert_allclose(gr, g1 + 0.2 * gs, rtol=1e-15)
    np.testing.assert_array_equal(gd, gd1)
    # finite differences of the whole loss w.r.t. one rendered colour value
    # away from the L1 kink
    h = 1e-7
    idx = (1, 5, 6)
    a, b = r.copy(), r.copy()
    a[idx] += h
    b[idx] -= h
    fd = (loss.mapping_loss(a, d, t, td)[0] - loss.mapping_loss(b, d, t, td)[0]) / (2 * h)
    assert abs(fd - gr[idx]) < 1e-7
