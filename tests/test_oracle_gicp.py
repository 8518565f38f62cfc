"""Pins of the GICP tracking oracle (paper Sec. 3.3, Eq. 2): each checks it
against something other than its own formulas -- scipy's KD-tree, closed
forms on planes, invariances, finite differences and exact recovery of a
known rigid motion."""
import numpy as np
import pytest

from oracle import gicp, se3
from paper_2603_21055_amd import synth


def _rand_pose(rng, trans, deg):
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    w = rng.normal(size=3)
    w /= np.linalg.norm(w)
    xi = np.concatenate([v * trans, w * np.deg2rad(deg)])
    T = se3.exp(xi)
    return T[:3, :3], T[:3, 3]


def test_knn_equals_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(0)
    p = rng.normal(size=(700, 3))
    q = rng.normal(size=(300, 3))
    got = gicp.knn(q, p, 10)
    _, ref = cKDTree(p).query(q, k=10)
    assert (got == ref).all()


def test_knn_ties_by_index():
    p = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, 0, 2.0]])
    got = gicp.knn(np.zeros((1, 3)), p, 3)
    assert got.tolist() == [[0, 1, 2]]


def test_plane_normal_and_normalised_covariance():
    """Points of the plane z = 0.3 x - 0.2 y + 2: the normal is the plane's,
    and the normalised covariance has eigenvalue EPS along it."""
    ys, xs = np.mgrid[-10:10, -10:10] * 0.01
    x, y = xs.ravel(), ys.ravel()
    p = np.stack([x, y, 0.3 * x - 0.2 * y + 2.0], 1)
    g = gicp.local_gaussians(p, 10)
    n_true = np.array([-0.3, 0.2, 1.0]) / np.linalg.norm([-0.3, 0.2, 1.0])
    assert np.allclose(np.abs(g["normal"] @ n_true), 1.0, atol=1e-9)
    assert np.allclose(g["eig"][:, 0], 0.0, atol=1e-15)
    Cn = g["cov"]
    assert np.allclose(np.einsum("nij,j->ni", Cn, n_true), gicp.EPS * n_true[None, :], atol=1e-9)
    # the largest normalised eigenvalue is 1
    assert np.allclose(np.linalg.eigvalsh(Cn)[:, 2], 1.0, atol=1e-9)


def test_normalised_covariance_is_scale_invariant_and_rotates_with_points():
    rng = np.random.default_rng(1)
    p = rng.normal(size=(300, 3)) * np.array([1.0, 0.4, 0.05])
    g = gicp.local_gaussians(p, 12)
    g2 = gicp.local_gaussians(3.7 * p, 12)
    assert np.allclose(g2["cov"], g["cov"], atol=1e-9)
    R, _ = _rand_pose(rng, 0.0, 40.0)
    g3 = gicp.local_gaussians(p @ R.T, 12)
    assert (g3["nb"] == g["nb"]).all()
    assert np.allclose(g3["cov"], np.einsum("ij,njk,lk->nil", R, g["cov"], R), atol=1e-9)


def _frame(seed, W=160, H=120, R=None, t=None):
    rng = np.random.default_rng(seed)
    room = synth.make_room(rng)
    cam = synth.intrinsics(W, H)
    R0 = np.eye(3) if R is None else R
    t0 = np.zeros(3) if t is None else t
    depth, _ = room.raycast(cam, R0.astype(np.float32), t0.astype(np.float32))
    return room, cam, depth


def test_point_to_surface_correspondence_hand_case():
    """Three target points; the nearest one by distance is off the source's
    plane, the second lies in it: point to surface takes the second."""
    tgt = dict(points=np.array([[0.0, 0, 1.0], [0.05, 0, 1.02], [0.5, 0.5, 1.0]]),
               normal=np.array([[1.0, 0, 0], [0, 0, 1.0], [0, 0, 1.0]]))
    src = dict(points=np.array([[0.01, 0.0, 1.02]]))
    j, X = gicp.correspond(src, tgt, np.eye(3), np.zeros(3), 2)
    assert j.tolist() == [1]
    # beyond D_MAX nothing is matched
    src = dict(points=np.array([[0.0, 0.0, 1.5]]))
    j, _ = gicp.correspond(src, tgt, np.eye(3), np.zeros(3), 2)
    assert j.tolist() == [-1]


def test_distance_cut_applies_before_the_surface_match():
    """Of the two nearest targets the one on the source's surface lies
    0.105 m away (beyond D_MAX), the other 0.03 m away off it: the cut
    removes the first as a candidate, so the source pairs with the second
    instead of with nothing."""
    tgt = dict(points=np.array([[0.03, 0.0, 1.0], [0.0, 0.0, 1.105]]),
               normal=np.array([[1.0, 0, 0], [1.0, 0, 0]]))
    src = dict(points=np.array([[0.0, 0.0, 1.0]]))
    E = src["points"][:, None, :] - tgt["points"][None]
    ds = gicp.surface_distance(E, tgt["normal"][None])
    assert ds[0, 1] < ds[0, 0]                   # the far one is the better surface match
    j, _ = gicp.correspond(src, tgt, np.eye(3), np.zeros(3), 2)
    assert j.tolist() == [0]


def test_jacobian_matches_finite_differences():
    room, cam, depth = _frame(3)
    pts, _ = gicp.sample_points(depth, cam, 4)
    tgt = gicp.local_gaussians(pts, 10)
    rng = np.random.default_rng(4)
    R, t = _rand_pose(rng, 0.01, 0.5)
    lin = gicp.linearise(tgt, tgt, R, t, 10)
    ok = lin["corr"] >= 0
    a = tgt["points"][ok]
    b = tgt["points"][lin["corr"][ok]]
    h = 1e-7
    for k in range(6):
        d = np.zeros(6)
        d[k] = h
        Rp, tp = se3.left_update(R, t, d)
        Rm, tm = se3.left_update(R, t, -d)
        ep = b - (a @ Rp.T + tp)
        em = b - (a @ Rm.T + tm)
        fd = (ep - em) / (2 * h)
        assert np.allclose(fd, lin["J"][:, :, k], atol=1e-6), k


def test_normal_equations_symmetric_psd_and_step_from_fd_jacobian():
    room, cam, depth = _frame(5)
    pts, _ = gicp.sample_points(depth, cam, 4)
    tgt = gicp.local_gaussians(pts, 10)
    rng = np.random.default_rng(6)
    R, t = _rand_pose(rng, 0.01, 0.5)
    lin = gicp.linearise(tgt, tgt, R, t, 10)
    Hm = lin["H"]
    assert np.allclose(Hm, Hm.T, rtol=1e-12, atol=1e-9)
    assert np.linalg.eigvalsh(Hm).min() > 0
    # the same step from the FD Jacobian with M and the pairs held fixed
    ok = lin["corr"] >= 0
    a = tgt["points"][ok]
    b = tgt["points"][lin["corr"][ok]]
    Jfd = np.zeros_like(lin["J"])
    h = 1e-7
    for k in range(6):
        d = np.zeros(6)
        d[k] = h
        Rp, tp = se3.left_update(R, t, d)
        Rm, tm = se3.left_update(R, t, -d)
        Jfd[:, :, k] = ((b - (a @ Rp.T + tp)) - (b - (a @ Rm.T + tm))) / (2 * h)
    Hf = np.einsum("nji,njk,nkl->il", Jfd, lin["M"], Jfd)
    gf = np.einsum("nji,njk,nk->i", Jfd, lin["M"], lin["e"])
    s1 = gicp.solve(Hm, lin["g"])[0]
    s2 = np.linalg.solve(Hf, -gf)
    assert np.allclose(s1, s2, rtol=1e-5, atol=1e-9)


def test_exact_recovery_of_a_rigid_motion():
    """Source = the target's points moved by P^-1, on a curved surface (where
    a point's true counterpart is the only candidate with zero plane
    distance at the solution): GN from the identity recovers P exactly, with
    every pair matched and zero cost.  (On a flat wall every candidate lies
    in the plane, so point-to-surface matching is ambiguous in-plane; that
    case is covered by the ray-cast recovery below.)"""
    ys, xs = np.mgrid[-30:30, -40:40] * 0.01
    x, y = xs.ravel(), ys.ravel()
    pts = np.stack([x, y, 2.0 + 0.1 * np.sin(5 * x) * np.cos(4 * y) + 0.05 * x * y], 1)
    tgt = gicp.local_gaussians(pts, 10)
    rng = np.random.default_rng(8)
    R, t = _rand_pose(rng, 0.01, 1.0)
    src_pts = (pts - t) @ R                       # P^-1 applied: a = R^T (b - t)
    src = gicp.local_gaussians(src_pts, 10)
    out = gicp.track(src, tgt, np.eye(3), np.zeros(3), 10, iters=25)
    assert np.abs(out["R"] - R).max() < 1e-9
    assert np.abs(out["t"] - t).max() < 1e-9
    assert out["trace"][-1]["cost"] < 1e-20
    assert out["trace"][-1]["n"] == len(pts)


def test_recovers_a_new_frame_pose_in_the_room():
    """A frame looking into a corner of the room (three walls) and a new frame
    ray-cast 3 cm / 2 degrees away, each with its own samples: GN lands
    within 2 mm / 0.05 degree of the new frame's pose."""
    rng = np.random.default_rng(9)
    room = synth.make_room(rng)
    cam = synth.intrinsics(200, 150)
    R0, t0 = synth.corner_pose(room)
    d0, _ = room.raycast(cam, R0, t0)
    Rg, tg = synth.perturb_pose(R0, t0, rng, 0.03, 2.0, exact=True)
    d1, _ = room.raycast(cam, Rg, tg)
    tgt = gicp.local_gaussians(gicp.sample_points(d0, cam, 4)[0], 10)
    src = gicp.local_gaussians(gicp.sample_points(d1, cam, 4)[0], 10)
    # target points live in frame 0's camera coordinates; the new frame's
    # camera-to-frame-0 pose is T0 T1^-1
    R0d, t0d = np.asarray(R0, np.float64), np.asarray(t0, np.float64)
    Rgd, tgd = np.asarray(Rg, np.float64), np.asarray(tg, np.float64)
    Rc = R0d @ Rgd.T
    tc = t0d - Rc @ tgd
    out = gicp.track(src, tgt, np.eye(3), np.zeros(3), 10, iters=30)
    ang = np.degrees(np.arccos(np.clip((np.trace(out["R"].T @ Rc) - 1) / 2, -1, 1)))
    assert np.linalg.norm(out["t"] - tc) < 2e-3, np.linalg.norm(out["t"] - tc)
    assert ang < 0.05, ang
    # three distinct wall normals in view, and the start was 3 cm / 2 degrees off
    n = np.abs(tgt["normal"] @ R0d)
    assert all((n[:, k] > 0.99).sum() > 50 for k in range(3)), [(n[:, k] > 0.99).sum() for k in range(3)]
    assert np.linalg.norm(tc) > 0.02
