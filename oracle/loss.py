"""FP64 oracle: L1 terms of the mapping loss (Eq. 1) and their upstream grads.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Eq. 1 sums, over the rendered views k, rho |V_k - V'_k|_1 + tau L_S +
sigma U_k |D_k - D'_k|_1 with rho, tau, sigma = 0.8, 0.2, 1.0 (supplement,
"Further Implementation Details").  Each L1 term is read as a mean over its
valid elements (the paper leaves the normalisation open); U_k = [D_k > 0].
The SSIM term L_S is not part of this path.  The rendered depth D' is the
unnormalised accumulated depth.  The subgradient of |x| at 0 is 0.
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
