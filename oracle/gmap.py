"""FP64 oracle: the global set T of geometry Gaussians the tracker matches
against (paper Sec. 3.3, "Matching a Frame to a Scene" and "Update Gaussian
Set T") and render-based filling of missing depth (Sec. 3.2, initialising
Gaussians where the depth map has no value).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain NumPy float64.

Readings, where the paper is silent:

* T holds geometry Gaussians in world coordinates: point, ellipse-normalised
  covariance and normal, as ``gicp.local_gaussians`` builds them for a frame.
* After frame i is tracked, with camera-to-world pose P_i = (R, t), its set
  T_i is moved into the world (p_w = R p + t summed in ``gicp.transform``'s
  order, C_w = R C R^T, n_w = R n) and each of its Gaussians is added unless
  it overlaps T: T keeps at most one Gaussian per cubic voxel of side VOXEL,
  the voxel of p being floor(p / VOXEL) per axis, and a new Gaussian whose
  voxel is taken -- by T, or by a new one of the same frame with a lower
  index -- is not added.  New Gaussians are appended in index order.
* Tracking a frame against T is GICP with T as the target set: the oracle's
  ``gicp.correspond`` / ``linearise`` / ``track`` take any target set.
* Missing depth: a pixel with depth <= 0 takes D'/A, the depth a previous
  keyframe's Gaussians render at the new pose divided by their alpha, where
  A >= FILL_ALPHA; elsewhere it keeps no depth.  Valid depths are kept.
"""
from __future__ import annotations

import numpy as np

from . import gicp

VOXEL = 0.02          # metres
FILL_ALPHA = 0.5


def voxel_key(points, voxel=VOXEL):
    """Integer voxel coordinates floor(p / voxel) per axis, [n, 3]."""
    return np.floor(np.asarray(points, np.float64) / voxel).astype(np.int64)


def to_world(frame_set, R, t):
    """A frame's set moved by the camera-to-world pose (R, t)."""
    R = np.asarray(R, np.float64)
    return dict(points=gicp.transform(frame_set["points"], R, t),
                cov=np.einsum("ij,njk,lk->nil", R, frame_set["cov"], R),
                normal=frame_set["normal"] @ R.T)


def insert(gmap, frame_set, R, t, voxel=VOXEL):
    """T after adding the non-overlapping Gaussians of a frame set tracked at
    (R, t); gmap None is the empty set.  Returns (T, indices of the frame's
    Gaussians that were added)."""
    w = to_world(frame_set, R, t)
    taken = set()
    if gmap is not None:
        taken = set(map(tuple, voxel_key(gmap["points"], voxel)))
    add = []
    for i, k in enumerate(map(tuple, voxel_key(w["points"], voxel))):
        if k not in taken:
            taken.add(k)
            add.append(i)
    add = np.array(add, np.int64)
    new = {key: w[key][add] for key in ("points", "cov", "normal")}
    if gmap is not None:
        new = {key: np.concatenate([gmap[key], new[key]], 0) for key in ("points", "cov", "normal")}
    return new, add


def fill_depth(depth, rendered_depth, rendered_alpha):
    """Depth with its holes (<= 0) filled by D'/A where A >= FILL_ALPHA."""
    d = np.asarray(depth, np.float64).copy()
    A = np.asarray(rendered_alpha, np.float64)
    Dp = np.asarray(rendered_depth, np.float64)
    hole = d <= 0
    ok = hole & (A >= FILL_ALPHA)
    d[hole] = 0.0
    d[ok] = Dp[ok] / A[ok]
    return d
