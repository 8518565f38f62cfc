"""FP64 SE(3) exponential and logarithm for the left-twist pose update.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A twist xi = (rho, phi) (translation first) acts on a world->camera pose by
left multiplication, T <- Exp(xi) T.  Exp(xi) = [[R, V rho], [0, 1]] with
R = exp([phi]x) (Rodrigues) and V = I + (1 - cos th)/th^2 [phi]x
+ (th - sin th)/th^3 [phi]x^2, th = |phi|.  The paper does not fix a pose
parametrisation; this is the standard one for Gauss-Newton on SE(3).
"""
from __future__ import annotations

import numpy as np


def hat(w):
    w = np.asarray(w, np.float64)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def _coeffs(th):
    """A = sin th / th, B = (1 - cos th)/th^2, C = (th - sin th)/th^3 with
    Taylor series near 0."""
    if th < 1e-4:
        t2 = th * th
        return 1.0 - t2 / 6.0 + t2 * t2 / 120.0, 0.5 - t2 / 24.0 + t2 * t2 / 720.0, \
            1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0
    return np.sin(th) / th, (1.0 - np.cos(th)) / th ** 2, (th - np.sin(th)) / th ** 3


def exp(xi):
    """4x4 matrix Exp(xi) for xi = (rho, phi)."""
    xi = np.asarray(xi, np.float64)
    rho, phi = xi[:3], xi[3:]
    th = float(np.linalg.norm(phi))
    A, B, C = _coeffs(th)
    K = hat(phi)
    R = np.eye(3) + A * K + B * (K @ K)
    V = np.eye(3) + B * K + C * (K @ K)
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = V @ rho
    return T


def log(T):
    """Inverse of ``exp`` for rotation angles below pi."""
    T = np.asarray(T, np.float64)
    R, t = T[:3, :3], T[:3, 3]
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    th = float(np.arccos(c))
    if th < 1e-8:
        phi = 0.5 * np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    else:
        phi = th / (2.0 * np.sin(th)) * np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0],
                                                   R[1, 0] - R[0, 1]])
    th = float(np.linalg.norm(phi))
    A, B, C = _coeffs(th)
    K = hat(phi)
    V = np.eye(3) + B * K + C * (K @ K)
    rho = np.linalg.solve(V, t)
    return np.concatenate([rho, phi])


def left_update(R, t, xi):
    """(R, t) <- Exp(xi) (R, t) for a world->camera pose."""
    T = np.eye(4)
    T[:3, :3] = np.asarray(R, np.float64)
    T[:3, 3] = np.asarray(t, np.float64)
    T2 = exp(xi) @ T
    return T2[:3, :3], T2[:3, 3]
