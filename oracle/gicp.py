"""FP64 oracle: tracking a depth frame against a set of geometry Gaussians
with Generalized ICP (paper Sec. 3.3, "Matching a Frame to a Scene" and
"Generalized ICP for Matching", Eq. 2; the supplement gives the sampling
ratio R and the neighbour count K_c; Tab. 11 ablates the correspondence
metric and the scale normalisation).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain NumPy float64.

What is computed, with the readings taken where the paper is silent:

* Sampling: the pixels (u, v) with u and v multiples of R (a stride-R grid in
  both image axes) and a positive depth.  Each becomes the point
  a = D(u, v) ((u - cx) / fx, (v - cy) / fy, 1) in its camera's frame.
* Local geometry: the covariance of each point's K_c nearest points of the
  same sampled set (Euclidean, the point itself included, ties by index),
  normalised by K_c.  Its eigen-decomposition (the SVD of a symmetric
  matrix) gives the scales and the rotation; the eigenvector of the
  smallest eigenvalue is the point's normal.
* Scale normalisation ("ellipse", Tab. 11): the eigenvalues are divided by
  the largest and floored at EPS, C' = U diag(1, max(l2/l1, EPS),
  max(l3/l1, EPS)) U^T, which keeps the ellipse's in-plane shape; the
  flat-plane normalisation of GICP would be diag(1, 1, EPS).
* Correspondence (point to surface): a source point moved into the target
  frame, X = R a + t, is matched among its K_c nearest target points within
  D_MAX (by Euclidean distance, ties by index) to the surface element
  closest to it, min_b (n_b . (X - b))^2 + EPS |X - b|^2 (ties by Euclidean
  rank): the distance to b's tangent plane, with EPS |X - b|^2 added so that
  on a plane, where every candidate has zero plane distance, the nearest
  point is taken (the plane distance alone does not identify a point
  there).  A point with no target within D_MAX has no pair.
* Eq. 2 as GICP defines it: sum over pairs of e^T (C_b + R C_a R^T)^-1 e,
  e = b - X (the printed equation omits the inverse and writes the pose for
  its rotation).  Gauss-Newton in the left twist xi = (rho, phi) of the
  camera-to-target pose P = (R, t), P <- Exp(xi) P: with M = (C_b + R C_a
  R^T)^-1 held fixed in a step, J = de/dxi = -[I | -[X]x], H = sum J^T M J,
  g = sum J^T M e, dxi = -H^-1 g by Cholesky (damped like ``track.solve``).
"""
from __future__ import annotations

import numpy as np

from . import se3

EPS = 1e-3          # floor of the normalised eigenvalues
D_MAX = 0.1         # metres: pairs farther apart are not used
DAMP = 1e-9


def sample_points(depth, cam, R_s):
    """Stride-R grid points of a depth map in camera coordinates.
    Returns (points [n, 3], pixel indices [n]) in row-major pixel order."""
    D = np.asarray(depth, np.float32).astype(np.float64)
    H, W = D.shape
    fx, fy = float(np.float32(cam["fx"])), float(np.float32(cam["fy"]))
    cx, cy = float(np.float32(cam["cx"])), float(np.float32(cam["cy"]))
    vs, us = np.mgrid[0:H:R_s, 0:W:R_s]
    us, vs = us.ravel(), vs.ravel()
    d = D[vs, us]
    keep = d > 0
    us, vs, d = us[keep], vs[keep], d[keep]
    x = d * ((us - cx) / fx)
    y = d * ((vs - cy) / fy)
    return np.stack([x, y, d], 1), vs * W + us


def knn(queries, points, k):
    """Indices [nq, k] of the k nearest points (squared Euclidean distance
    ((dx^2 + dy^2) + dz^2), ties by index), nearest first."""
    q = np.asarray(queries, np.float64)
    p = np.asarray(points, np.float64)
    out = np.empty((len(q), k), np.int64)
    idx = np.arange(len(p))
    for i0 in range(0, len(q), 256):
        qq = q[i0:i0 + 256]
        d = (qq[:, None, 0] - p[None, :, 0]) ** 2 + (qq[:, None, 1] - p[None, :, 1]) ** 2
        d = d + (qq[:, None, 2] - p[None, :, 2]) ** 2
        for r in range(len(qq)):
            order = np.lexsort((idx, d[r]))
            out[i0 + r] = order[:k]
    return out


def local_gaussians(points, k):
    """Per point: the normalised covariance C' [n, 3, 3], the normal [n, 3]
    and the raw eigenvalues [n, 3] (ascending) of its K_c-neighbour
    covariance."""
    p = np.asarray(points, np.float64)
    nb = knn(p, p, k)
    Q = p[nb]                                    # [n, k, 3]
    mu = Q.mean(1)
    Dv = Q - mu[:, None, :]
    C = np.einsum("nki,nkj->nij", Dv, Dv) / k
    lam, U = np.linalg.eigh(C)                   # ascending
    l1 = lam[:, 2]
    safe = np.where(l1 > 0, l1, 1.0)
    s = np.stack([np.maximum(lam[:, 0] / safe, EPS), np.maximum(lam[:, 1] / safe, EPS),
                  np.ones(len(p))], 1)
    s = np.where((l1 > 0)[:, None], s, np.array([EPS, EPS, 1.0]))
    Cn = np.einsum("nij,nj,nkj->nik", U, s, U)
    return dict(points=p, cov=Cn, normal=U[:, :, 0], eig=lam, nb=nb)


def transform(points, R, t):
    """X = R a + t with each row summed in the fixed order ((r0 a0 + r1 a1) +
    r2 a2) + t (the order is part of the correspondence decision)."""
    a = np.asarray(points, np.float64)
    R = np.asarray(R, np.float64)
    t = np.asarray(t, np.float64)
    return np.stack([((R[i, 0] * a[:, 0] + R[i, 1] * a[:, 1]) + R[i, 2] * a[:, 2]) + t[i] for i in range(3)], 1)


def surface_distance(E, Nrm):
    """(n . e)^2 + EPS |e|^2 with both dot products summed in the order
    (x + y) + z."""
    dn = (Nrm[..., 0] * E[..., 0] + Nrm[..., 1] * E[..., 1]) + Nrm[..., 2] * E[..., 2]
    ee = (E[..., 0] * E[..., 0] + E[..., 1] * E[..., 1]) + E[..., 2] * E[..., 2]
    return dn * dn + EPS * ee


def correspond(src, tgt, R, t, k, with_margins=False):
    """Point-to-surface correspondences of the source points moved by (R, t):
    target index per source point (-1: none within D_MAX) and X = R a + t.
    with_margins: also, per source point, the relative gaps of the three
    decisions (K-th vs (K+1)-th Euclidean distance, best vs second surface
    distance, squared distance vs D_MAX^2), for flagging near-ties."""
    X = transform(src["points"], R, t)
    P = tgt["points"]
    kk = min(k + 1 if with_margins else k, len(P))
    nb = knn(X, P, kk)
    nbk = nb[:, :min(k, len(P))]

    def sq(i):
        f = X - P[nb[:, i]]
        return (f[:, 0] * f[:, 0] + f[:, 1] * f[:, 1]) + f[:, 2] * f[:, 2]

    d2k = np.stack([sq(i) for i in range(nbk.shape[1])], 1)          # [n, k]
    within = d2k <= D_MAX * D_MAX
    E = X[:, None, :] - P[nbk]
    dist = np.where(within, surface_distance(E, tgt["normal"][nbk]), np.inf)
    best = np.argmin(dist, 1)                    # first minimum = lowest Euclidean rank
    has = within.any(1)
    j = np.where(has, nbk[np.arange(len(X)), best], -1)
    if not with_margins:
        return j, X
    gap_knn = (np.abs(sq(k) - sq(k - 1)) / np.maximum(sq(k), 1e-300)) if nb.shape[1] > k else np.full(len(X), np.inf)
    srt = np.sort(dist, 1)
    gap_best = np.where(np.isfinite(srt[:, 1]), np.abs(srt[:, 1] - srt[:, 0]) / np.maximum(srt[:, 1], 1e-300),
                        np.inf) if k > 1 else np.full(len(X), np.inf)
    gap_dmax = (np.abs(d2k - D_MAX * D_MAX) / (D_MAX * D_MAX)).min(1)
    return j, X, dict(knn=gap_knn, best=gap_best, dmax=gap_dmax)


def linearise(src, tgt, R, t, k):
    """Eq. 2 cost, normal equations and correspondences at the pose (R, t)."""
    R = np.asarray(R, np.float64)
    j, X = correspond(src, tgt, R, t, k)
    ok = j >= 0
    Xa = X[ok]
    e = tgt["points"][j[ok]] - Xa
    Cs = np.einsum("ij,njk,lk->nil", R, src["cov"][ok], R)
    M = np.linalg.inv(tgt["cov"][j[ok]] + Cs)
    n = len(Xa)
    J = np.zeros((n, 3, 6))
    J[:, :, :3] = -np.eye(3)
    J[:, :, 3:] = np.stack([se3.hat(x) for x in Xa]) if n else np.zeros((0, 3, 3))
    MJ = np.einsum("nij,njk->nik", M, J)
    Hm = np.einsum("nji,njk->ik", J, MJ)
    gv = np.einsum("nji,nj->i", J, np.einsum("nij,nj->ni", M, e))
    cost = float(np.einsum("ni,ni->", e, np.einsum("nij,nj->ni", M, e)))
    return dict(H=Hm, g=gv, cost=cost, n=int(n), corr=j, X=X, e=e, M=M, J=J)


def solve(Hm, gv):
    """dxi = -H^-1 g by Cholesky; damping DAMP tr(H) (x10 per retry) if needed."""
    lam = 0.0
    for _ in range(12):
        try:
            L = np.linalg.cholesky(Hm + lam * np.eye(6))
            y = np.linalg.solve(L, -gv)
            return np.linalg.solve(L.T, y), lam
        except np.linalg.LinAlgError:
            lam = DAMP * np.trace(Hm) if lam == 0.0 else lam * 10.0
    return np.zeros(6), lam


def track(src, tgt, R0, t0, k, iters=30):
    """Fixed-iteration Gauss-Newton from the camera-to-target pose (R0, t0)."""
    R = np.asarray(R0, np.float64)
    t = np.asarray(t0, np.float64)
    trace = []
    for _ in range(iters):
        lin = linearise(src, tgt, R, t, k)
        dxi, lam = solve(lin["H"], lin["g"])
        trace.append(dict(R=R.copy(), t=t.copy(), H=lin["H"], g=lin["g"], cost=lin["cost"], n=lin["n"],
                          dxi=dxi, lam=lam))
        R, t = se3.left_update(R, t, dxi)
    return dict(R=R, t=t, trace=trace)
