"""FP64 oracle: Adam step for the per-pixel Gaussian parameters.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The supplement gives learning rates only (colour 0.0025, radius 0.005,
opacity 0.05, offset 0.01); the optimiser is read as Adam with
beta = (0.9, 0.999) and eps = 1e-8, stepping radius as log r and opacity as
logit o (the spaces those rates belong to in 3DGS).  Opacity is kept in
[0, 1] and radius at or above R_MIN after each step.
"""
from __future__ import annotations

import numpy as np

LR = dict(rgb=0.0025, radius=0.005, opacity=0.05, offset=0.01)
BETA1 = 0.9
BETA2 = 0.999
EPS = 1e-8
R_MIN = 1e-6


def adam_step(p, g, m, v, step, lr):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = BETA1 * np.asarray(m, np.float64) + (1.0 - BETA1) * g
    v = BETA2 * np.asarray(v, np.float64) + (1.0 - BETA2) * g * g
    mh = m / (1.0 - BETA1 ** step)
    vh = v / (1.0 - BETA2 ** step)
    return p - lr * mh / (np.sqrt(vh) + EPS), m, v


SPACE = dict(rgb="linear", offset="linear", radius="log", opacity="logit")


def adam_step_space(p, g, m, v, step, lr, space):
    """Adam in the parameter's optimisation space: theta = p ("linear"),
    log p ("log") or log(p / (1 - p)) ("logit"); g is dL/dp and is mapped to
    dL/dtheta; returns (p, m, v) with m, v the moments of dL/dtheta.  The
    supplement's rates are the 3DGS values for log-scale and logit-opacity,
    hence radius in log space and opacity in logit space."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    if space == "log":
        p = np.maximum(p, 1e-12)
        th, gth = np.log(p), g * p
    elif space == "logit":
        p = np.clip(p, 1e-6, 1.0 - 1e-6)
        th, gth = np.log(p / (1.0 - p)), g * p * (1.0 - p)
    else:
        th, gth = p, g
    th, m, v = adam_step(th, gth, m, v, step, lr)
    if space == "log":
        return np.exp(th), m, v
    if space == "logit":
        return 1.0 / (1.0 + np.exp(-th)), m, v
    return th, m, v


def clamp(name, p):
    if name == "opacity":
        return np.clip(p, 0.0, 1.0)
    if name == "radius":
        return np.maximum(p, R_MIN)
    return p
