"""FP64 oracle: L1 terms of the mapping loss (Eq. 1) and their upstream grads.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Eq. 1 sums, over the rendered views k, rho |V_k - V'_k|_1 + tau L_S +
sigma U_k |D_k - D'_k|_1 with rho, tau, sigma = 0.8, 0.2, 1.0 (supplement,
"Further Implementation Details").  Each L1 term is read as a mean over its
valid elements (the paper leaves the normalisation open); U_k = [D_k > 0].
The rendered depth D' is the unnormalised accumulated depth.  The
subgradient of |x| at 0 is 0.

L_S is the structural-similarity term of the SSIM reference the paper cites,
read as L_S = 1 - mean SSIM(V, V') over pixels and colour channels, with
that reference's constants: an 11 x 11 Gaussian window of standard
deviation 1.5 (normalised to sum 1), C1 = (0.01 L)^2, C2 = (0.03 L)^2 for a
dynamic range L = 1, and local statistics mu = G * x, sigma_x^2 =
G * x^2 - mu_x^2, sigma_xy = G * (x y) - mu_x mu_y.  The window is applied as
a 'same' correlation with zero padding (the paper does not say how borders
are handled; zero padding is the 3DGS-lineage convention).
"""
from __future__ import annotations

import numpy as np

RHO = 0.8
TAU = 0.2
SIGMA = 1.0


def l1_loss(rgb, depth, t_rgb, t_depth, w_rgb=RHO, w_depth=SIGMA):
    """Loss value and grads w.r.t. rendered rgb [3,H,W] and depth [H,W]."""
    rgb = np.asarray(rgb, np.float64)
    depth = np.asarray(depth, np.float64)
    t_rgb = np.asarray(t_rgb, np.float64)
    t_depth = np.asarray(t_depth, np.float64)
    U = t_depth > 0
    n_rgb = rgb.size
    n_d = max(int(U.sum()), 1)
    e_rgb = rgb - t_rgb
    e_d = np.where(U, depth - t_depth, 0.0)
    loss = w_rgb * np.abs(e_rgb).sum() / n_rgb + w_depth * np.abs(e_d).sum() / n_d
    g_rgb = w_rgb * np.sign(e_rgb) / n_rgb
    g_depth = w_depth * np.sign(e_d) / n_d
    return float(loss), g_rgb, g_depth


SSIM_WIN = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window():
    """The 1-D Gaussian window: SSIM_WIN taps, std SSIM_SIGMA, sum 1."""
    k = np.arange(SSIM_WIN, dtype=np.float64) - SSIM_WIN // 2
    g = np.exp(-k * k / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def ssim_filter(img):
    """'same' 2-D correlation of an [H, W] image with the separable window
    g g^T, zero outside the image: out[y, x] = sum_ij g_i g_j img[y+i-5, x+j-5]."""
    img = np.asarray(img, np.float64)
    H, W = img.shape
    g = ssim_window()
    r = SSIM_WIN // 2
    pad = np.zeros((H + 2 * r, W + 2 * r))
    pad[r:r + H, r:r + W] = img
    tmp = np.zeros((H + 2 * r, W))
    for j in range(SSIM_WIN):
        tmp += g[j] * pad[:, j:j + W]
    out = np.zeros((H, W))
    for i in range(SSIM_WIN):
        out += g[i] * tmp[i:i + H]
    return out


def ssim_map(x, y):
    """Per-pixel SSIM of two [H, W] images (SSIM reference, Gaussian window)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = ssim_filter(x), ssim_filter(y)
    sxx = ssim_filter(x * x) - mx * mx
    syy = ssim_filter(y * y) - my * my
    sxy = ssim_filter(x * y) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def ssim_loss(rgb, t_rgb, with_abs=False):
    """L_S = 1 - mean SSIM over the channels of the rendered colour ``rgb``
    [C, H, W] against the observed ``t_rgb``, and dL_S / d rgb.

    With S = A1 A2 / (B1 B2), A1 = 2 mu_x mu_y + C1, A2 = 2 s_xy + C2,
    B1 = mu_x^2 + mu_y^2 + C1, B2 = s_xx + s_yy + C2 (x observed, y rendered)
    and the statistics written through the filtered moments mu_y = G*y,
    e_yy = G*y^2, e_xy = G*(x y), the partials per pixel q are
      dS/dmu_y = S (2 mu_x / A1 - 2 mu_x / A2 - 2 mu_y / B1 + 2 mu_y / B2),
      dS/de_yy = -S / B2,   dS/de_xy = 2 S / A2,
    and the adjoint of the correlation is the correlation with the flipped
    (here identical) window, so
      dL/dy = -(1 / n) [G*(dS/dmu_y) + 2 y G*(dS/de_yy) + x G*(dS/de_xy)]
    with n = C H W.  with_abs: also the same sum with every term replaced by
    its absolute value (a bound on the magnitudes an evaluation combines, for
    tolerances)."""
    rgb = np.asarray(rgb, np.float64)
    t_rgb = np.asarray(t_rgb, np.float64)
    C, H, W = rgb.shape
    n = C * H * W
    total = 0.0
    grad = np.zeros_like(rgb)
    gabs = np.zeros_like(rgb)
    for c in range(C):
        x, y = t_rgb[c], rgb[c]
        mx, my = ssim_filter(x), ssim_filter(y)
        sxx = ssim_filter(x * x) - mx * mx
        syy = ssim_filter(y * y) - my * my
        sxy = ssim_filter(x * y) - mx * my
        A1 = 2 * mx * my + SSIM_C1
        A2 = 2 * sxy + SSIM_C2
        B1 = mx * mx + my * my + SSIM_C1
        B2 = sxx + syy + SSIM_C2
        S = A1 * A2 / (B1 * B2)
        total += S.sum()
        d_my = S * (2 * mx / A1 - 2 * mx / A2 - 2 * my / B1 + 2 * my / B2)
        d_eyy = -S / B2
        d_exy = 2 * S / A2
        grad[c] = -(ssim_filter(d_my) + 2 * y * ssim_filter(d_eyy) + x * ssim_filter(d_exy)) / n
        if with_abs:
            gabs[c] = (ssim_filter(np.abs(d_my)) + 2 * np.abs(y) * ssim_filter(np.abs(d_eyy))
                       + np.abs(x) * ssim_filter(np.abs(d_exy))) / n
    if with_abs:
        return 1.0 - total / n, grad, gabs
    return 1.0 - total / n, grad


def mapping_loss(rgb, depth, t_rgb, t_depth, w_rgb=RHO, w_ssim=TAU, w_depth=SIGMA):
    """Eq. 1 for one view: w_rgb L1(rgb) + w_ssim L_S + w_depth U L1(depth),
    with its gradients w.r.t. the rendered rgb and depth."""
    L, g_rgb, g_depth = l1_loss(rgb, depth, t_rgb, t_depth, w_rgb, w_depth)
    if w_ssim:
        Ls, gs = ssim_loss(rgb, t_rgb)
        L += w_ssim * Ls
        g_rgb = g_rgb + w_ssim * gs
    return float(L), g_rgb, g_depth
