"""Seeded synthetic RGBD inputs for the splatting path.

This module only *generates inputs*: camera intrinsics, world->camera poses,
depth/colour frames of an analytic box-shaped room and per-pixel Gaussian
parameters in their documented initial state.  It holds none of the
splatting, compositing or tracking arithmetic; the FP64 oracle and the HIP
path both consume what it produces and nothing else is shared between them.

Conventions
-----------
* A camera is ``dict(H, W, fx, fy, cx, cy)``; pixel (u, v) is centred at the
  integer point (u, v).
* A pose is world->camera: ``X_cam = R @ X_world + t`` (``R`` row-major 3x3).
* Planes are float32, row-major ``[H, W]``; colour is planar ``[3, H, W]``.
* Randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).

The initial radius is the paper's initialisation rule r = D / F (supplement,
"Further Implementation Details"), with F = fx; initial offsets are zero
unless a workload asks for random ones.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation

__all__ = [
    "intrinsics", "perturb_pose", "pose_from_c2w", "Room", "make_room",
    "keyframe_from_frame", "plane_scene", "room_frame_scene", "room_window", "tracking_scene",
    "small_scene", "crop_camera",
]


# ----------------------------------------------------------------------------
# cameras and poses
# ----------------------------------------------------------------------------
def intrinsics(W: int, H: int) -> dict:
    """Pinhole camera with fx = fy = 0.9375 W and the principal point at the
    image centre (64x48 -> 60, 32, 24; 640x480 -> 600, 320, 240;
    1200x680 -> 1125, 600, 340)."""
    f = 0.9375 * W
    return dict(H=int(H), W=int(W), fx=float(f), fy=float(f), cx=W / 2.0, cy=H / 2.0)


def crop_camera(cam: dict, W: int, H: int) -> dict:
    """Same focal length, smaller sensor centred on the same principal point."""
    return dict(H=int(H), W=int(W), fx=cam["fx"], fy=cam["fy"], cx=W / 2.0, cy=H / 2.0)


def _rot(axis_angle) -> np.ndarray:
    return Rotation.from_rotvec(np.asarray(axis_angle, dtype=np.float64)).as_matrix()


def _unit(rng) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def perturb_pose(R, t, rng, max_trans, max_rot_deg, exact=False):
    """Left-multiply a world->camera pose by a random rigid motion.

    Translation magnitude ~ U[0, max_trans] (metres) and rotation angle ~
    U[0, max_rot_deg] (degrees) about isotropic random axes; with
    ``exact=True`` the magnitudes are exactly the maxima.
    """
    tr = max_trans if exact else rng.uniform(0.0, max_trans)
    an = np.deg2rad(max_rot_deg if exact else rng.uniform(0.0, max_rot_deg))
    dR = _rot(_unit(rng) * an)
    dt = _unit(rng) * tr
    R = np.asarray(R, np.float64)
    t = np.asarray(t, np.float64)
    return (dR @ R).astype(np.float32), (dR @ t + dt).astype(np.float32)


def pose_from_c2w(R_wc, C):
    """World->camera pose of a camera at centre C with orientation R_wc."""
    R_wc = np.asarray(R_wc, np.float64)
    C = np.asarray(C, np.float64)
    return R_wc.T.astype(np.float32), (-R_wc.T @ C).astype(np.float32)


def corner_pose(room, C=(0.0, 0.0, 0.0)):
    """World->camera pose of a camera at C looking at the room's (+x, +y, +z)
    corner (image y down): three walls in view, so a frame's geometry pins
    all six degrees of freedom."""
    C = np.asarray(C, np.float64)
    z = np.asarray(room.hi, np.float64) - C
    z /= np.linalg.norm(z)
    x = np.cross(np.array([0.0, 1.0, 0.0]), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    return pose_from_c2w(np.stack([x, y, z], 1), C)


# ----------------------------------------------------------------------------
# analytic room: an axis-aligned box around the origin, value-noise colour
# ----------------------------------------------------------------------------
class Room:
    """Axis-aligned box [lo, hi] with 3-octave value-noise colour on its walls."""

    LATTICE = 64

    def __init__(self, lo, hi, lattices):
        self.lo = np.asarray(lo, np.float64)
        self.hi = np.asarray(hi, np.float64)
        self.lattices = lattices  # [octave][channel] -> (L, L, L) table in [0, 1]

    def colour(self, P: np.ndarray) -> np.ndarray:
        """Value noise at world points P (..., 3): base cell 0.5 m, frequency
        x2 and amplitude x1/2 per octave, smoothstep trilinear interpolation,
        independent lattice per channel; normalised to [0, 1]."""
        L = self.LATTICE
        out = np.zeros((3,) + P.shape[:-1])
        amp_sum = 0.0
        for o in range(3):
            cell = 0.5 / (2 ** o)
            amp = 0.5 ** o
            amp_sum += amp
            g = P / cell + 1000.0  # shift keeps lattice coordinates positive
            i0 = np.floor(g).astype(np.int64)
            f = g - i0
            s = f * f * (3.0 - 2.0 * f)
            for c in range(3):
                lat = self.lattices[o][c]
                acc = 0.0
                for dx in (0, 1):
                    wx = s[..., 0] if dx else 1.0 - s[..., 0]
                    for dy in (0, 1):
                        wy = s[..., 1] if dy else 1.0 - s[..., 1]
                        for dz in (0, 1):
                            wz = s[..., 2] if dz else 1.0 - s[..., 2]
                            val = lat[(i0[..., 0] + dx) % L, (i0[..., 1] + dy) % L,
                                      (i0[..., 2] + dz) % L]
                            acc = acc + wx * wy * wz * val
                out[c] += amp * acc
        return out / amp_sum

    def raycast(self, cam: dict, R, t):
        """Analytic z-depth and colour of the box seen from a world->camera pose."""
        H, W = cam["H"], cam["W"]
        R = np.asarray(R, np.float64)
        t = np.asarray(t, np.float64)
        u = np.arange(W, dtype=np.float64)[None, :].repeat(H, 0)
        v = np.arange(H, dtype=np.float64)[:, None].repeat(W, 1)
        dc = np.stack([(u - cam["cx"]) / cam["fx"], (v - cam["cy"]) / cam["fy"],
                       np.ones_like(u)], -1)          # camera-frame ray, z = 1
        R_wc = R.T
        C = -R.T @ t
        dw = dc @ R_wc.T                                # world-frame direction
        tmax = np.full((H, W), np.inf)
        for i in range(3):
            di = dw[..., i]
            with np.errstate(divide="ignore", invalid="ignore"):
                tp = np.where(di > 0, (self.hi[i] - C[i]) / di, np.inf)
                tn = np.where(di < 0, (self.lo[i] - C[i]) / di, np.inf)
            tmax = np.minimum(tmax, np.minimum(tp, tn))
        P = C + tmax[..., None] * dw
        depth = tmax  # camera ray has unit z, so the ray parameter is z-depth
        return depth.astype(np.float32), self.colour(P).astype(np.float32)


def make_room(rng) -> Room:
    """Walls at distances ~ U[0.5, 5] m along -x, +x, -y, +y, +z; the -z wall
    sits 5 m behind the origin."""
    d = rng.uniform(0.5, 5.0, size=5)
    lo = np.array([-d[0], -d[2], -5.0])
    hi = np.array([d[1], d[3], d[4]])
    L = Room.LATTICE
    lattices = [[rng.uniform(0.0, 1.0, size=(L, L, L)) for _ in range(3)] for _ in range(3)]
    return Room(lo, hi, lattices)


def keyframe_from_frame(cam, R, t, depth, rgb, opacity, offset=None, sigma=None):
    """Pixel-aligned Gaussian parameters in their initial state: radius = D/fx
    (paper's initialisation), offset zero unless given."""
    H, W = cam["H"], cam["W"]
    depth = np.ascontiguousarray(depth, np.float32)
    kf = dict(
        cam=dict(cam),
        R=np.asarray(R, np.float32).copy(),
        t=np.asarray(t, np.float32).copy(),
        depth=depth,
        offset=np.zeros((H, W), np.float32) if offset is None else np.ascontiguousarray(offset, np.float32),
        radius=(depth / np.float32(cam["fx"])).astype(np.float32),
        opacity=np.ascontiguousarray(opacity, np.float32),
        rgb=None if rgb is None else np.ascontiguousarray(rgb, np.float32),
    )
    if sigma is not None:
        kf["sigma"] = np.ascontiguousarray(sigma, np.float32)
    return kf


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def plane_scene(seed: int = 0) -> dict:
    """64x48 tilted plane, fx = fy = 60, cx = 32, cy = 24, keyframe at identity.

    Depth: 1/z affine in u from 1 m (u = 0) to 4 m (u = 63) plus N(0, 1 cm);
    offsets 0, radius D/fx, opacity 0.9, RGB ~ U[0, 1].  View 0 is the
    identity, view 1 a 1 cm / 0.5 degree perturbation.  Target (seed + 1): RGB
    ~ U[0, 1] and the noise-free plane.
    """
    rng = np.random.default_rng(seed)
    cam = dict(H=48, W=64, fx=60.0, fy=60.0, cx=32.0, cy=24.0)
    u = np.arange(64, dtype=np.float64)
    inv = 1.0 + (0.25 - 1.0) * u / 63.0
    plane = np.repeat((1.0 / inv)[None, :], 48, 0)
    depth = plane + rng.normal(0.0, 0.01, size=plane.shape)
    rgb = rng.uniform(0.0, 1.0, size=(3, 48, 64))
    R0, t0 = np.eye(3, dtype=np.float32), np.zeros(3, np.float32)
    kf = keyframe_from_frame(cam, R0, t0, depth, rgb, np.full((48, 64), 0.9, np.float32))
    R1, t1 = perturb_pose(R0, t0, rng, 0.01, 0.5, exact=True)
    views = [dict(cam=dict(cam), R=R0.copy(), t=t0.copy()), dict(cam=dict(cam), R=R1, t=t1)]
    trng = np.random.default_rng(seed + 1)
    target = dict(rgb=trng.uniform(0.0, 1.0, size=(3, 48, 64)).astype(np.float32),
                  depth=plane.astype(np.float32))
    return dict(kfs=[kf], views=views, target=target)


def room_frame_scene(seed: int = 10, W: int = 640, H: int = 480) -> dict:
    """One keyframe of a box room (walls 0.5-5 m), value-noise colour, opacity
    ~ U[0.5, 1], offsets 0, rendered into one view perturbed by up to 2 cm and
    1 degree.  The target is the analytic ray-cast frame at the view."""
    rng = np.random.default_rng(seed)
    room = make_room(rng)
    cam = intrinsics(W, H)
    R0, t0 = np.eye(3, dtype=np.float32), np.zeros(3, np.float32)
    depth, rgb = room.raycast(cam, R0, t0)
    kf = keyframe_from_frame(cam, R0, t0, depth, rgb,
                             rng.uniform(0.5, 1.0, size=(H, W)).astype(np.float32))
    Rv, tv = perturb_pose(R0, t0, rng, 0.02, 1.0)
    tdepth, trgb = room.raycast(cam, Rv, tv)
    return dict(kfs=[kf], views=[dict(cam=dict(cam), R=Rv, t=tv)],
                target=dict(rgb=trgb, depth=tdepth), room=room)


def room_window(seed: int = 20, W: int = 640, H: int = 480, n: int = 8) -> dict:
    """Mapping window: n keyframes of one room at centres (0.05k - 0.175, 0, 0)
    with yaw (k - 3.5) * 2 degrees; offsets ~ U[-0.05, 0.05]; n views are the
    keyframe poses perturbed by up to 5 cm / 3 degrees; targets are ray-cast."""
    rng = np.random.default_rng(seed)
    room = make_room(rng)
    cam = intrinsics(W, H)
    kfs, views, targets = [], [], []
    for k in range(n):
        yaw = np.deg2rad((k - 3.5) * 2.0)
        R, t = pose_from_c2w(_rot([0.0, yaw, 0.0]), [0.05 * k - 0.175, 0.0, 0.0])
        depth, rgb = room.raycast(cam, R, t)
        off = rng.uniform(-0.05, 0.05, size=(H, W)).astype(np.float32)
        kfs.append(keyframe_from_frame(cam, R, t, depth, rgb,
                                       rng.uniform(0.5, 1.0, size=(H, W)).astype(np.float32),
                                       offset=off))
    for k in range(n):
        Rv, tv = perturb_pose(kfs[k]["R"], kfs[k]["t"], rng, 0.05, 3.0)
        views.append(dict(cam=dict(cam), R=Rv, t=tv))
        d, c = room.raycast(cam, Rv, tv)
        targets.append(dict(rgb=c, depth=d))
    return dict(kfs=kfs, views=views, targets=targets, room=room)


def tracking_scene(seed: int = 30, W: int = 1200, H: int = 680) -> dict:
    """Tracking: geometry Gaussians of the previous frame (identity pose) with
    per-pixel depth std sigma ~ U[0.005, 0.05] m, opacity 0.9, offsets 0;
    the new frame's ground-truth pose is exactly 3 cm and 2 degrees away.
    ``obs_depth`` is the analytic ray-cast depth at the ground truth."""
    rng = np.random.default_rng(seed)
    room = make_room(rng)
    cam = intrinsics(W, H)
    R0, t0 = np.eye(3, dtype=np.float32), np.zeros(3, np.float32)
    depth, _ = room.raycast(cam, R0, t0)
    sigma = rng.uniform(0.005, 0.05, size=(H, W)).astype(np.float32)
    geo = keyframe_from_frame(cam, R0, t0, depth, None,
                              np.full((H, W), 0.9, np.float32), sigma=sigma)
    Rg, tg = perturb_pose(R0, t0, rng, 0.03, 2.0, exact=True)
    obs, _ = room.raycast(cam, Rg, tg)
    return dict(geo=geo, cam=cam, gt=dict(R=Rg, t=tg), init=dict(R=R0.copy(), t=t0.copy()),
                obs_depth=obs, room=room)


def small_scene(seed: int, W: int, H: int, n_kf: int = 1, n_views: int = 1,
                max_trans: float = 0.02, max_rot: float = 1.0, offset_amp: float = 0.0,
                opacity_range=(0.5, 1.0), fx_scale: float = 0.9375) -> dict:
    """A room scene at an arbitrary (small) size for parity tests: n_kf
    keyframes near the origin, n_views views perturbed from them."""
    rng = np.random.default_rng(seed)
    room = make_room(rng)
    f = fx_scale * W
    cam = dict(H=int(H), W=int(W), fx=float(f), fy=float(f), cx=W / 2.0, cy=H / 2.0)
    kfs, views, targets = [], [], []
    for k in range(n_kf):
        if k == 0:
            R, t = np.eye(3, dtype=np.float32), np.zeros(3, np.float32)
        else:
            R, t = perturb_pose(np.eye(3), np.zeros(3), rng, 0.05, 3.0)
        depth, rgb = room.raycast(cam, R, t)
        off = None
        if offset_amp > 0:
            off = rng.uniform(-offset_amp, offset_amp, size=(H, W)).astype(np.float32)
        kfs.append(keyframe_from_frame(cam, R, t, depth, rgb,
                                       rng.uniform(*opacity_range, size=(H, W)).astype(np.float32),
                                       offset=off))
    for k in range(n_views):
        base = kfs[k % n_kf]
        Rv, tv = perturb_pose(base["R"], base["t"], rng, max_trans, max_rot)
        views.append(dict(cam=dict(cam), R=Rv, t=tv))
        d, c = room.raycast(cam, Rv, tv)
        targets.append(dict(rgb=c, depth=d))
    return dict(kfs=kfs, views=views, targets=targets, room=room)
