"""Pins of the global geometry set and hole-filling oracle (paper Sec. 3.3
"Update Gaussian Set T", Sec. 3.2 initialisation where depth is missing):
hand-worked voxel cases, idempotent re-insertion, consistency of tracking
against T with tracking against the frame it came from, and closed-form
hole filling."""
import numpy as np

from oracle import gicp, gmap, se3
from paper_2603_21055_amd import synth


def _set(points):
    n = len(points)
    return dict(points=np.asarray(points, np.float64), cov=np.tile(np.eye(3), (n, 1, 1)),
                normal=np.tile([0.0, 0.0, 1.0], (n, 1)))


def test_voxel_keys_hand_worked():
    k = gmap.voxel_key(np.array([[0.019, -0.001, 0.04], [0.02, 0.0, -0.02], [-0.0400001, 1.0, 0.0]]))
    assert k.tolist() == [[0, -1, 2], [1, 0, -1], [-3, 50, 0]]


def test_insert_keeps_one_per_voxel_lowest_index_first():
    pts = [[0.001, 0.001, 1.001], [0.015, 0.002, 1.019], [0.025, 0.0, 1.0], [0.005, 0.005, 1.005]]
    T, add = gmap.insert(None, _set(pts), np.eye(3), np.zeros(3))
    # points 0, 1 and 3 share voxel (0, 0, 50): only 0 is added
    assert add.tolist() == [0, 2]
    assert np.allclose(T["points"], np.array(pts)[[0, 2]])
    # a second frame: its point in a taken voxel is not added, the free one is appended
    T2, add2 = gmap.insert(T, _set([[0.03, 0.001, 1.0], [0.05, 0.0, 1.0]]), np.eye(3), np.zeros(3))
    assert add2.tolist() == [1]
    assert np.allclose(T2["points"][:2], T["points"]) and np.allclose(T2["points"][2], [0.05, 0.0, 1.0])


def test_insert_moves_into_the_world_and_is_idempotent():
    rng = np.random.default_rng(0)
    p = rng.uniform(-1, 1, size=(400, 3))
    s = gicp.local_gaussians(p, 8)
    T = se3.exp(np.array([0.1, -0.2, 0.3, 0.2, -0.1, 0.3]))
    R, t = T[:3, :3], T[:3, 3]
    M, add = gmap.insert(None, s, R, t)
    assert np.allclose(M["points"], (p @ R.T + t)[add])
    assert np.allclose(M["cov"], np.einsum("ij,njk,lk->nil", R, s["cov"], R)[add])
    assert np.allclose(M["normal"], (s["normal"] @ R.T)[add])
    M2, add2 = gmap.insert(M, s, R, t)
    assert len(add2) == 0 and len(M2["points"]) == len(M["points"])


def test_tracking_against_T_equals_tracking_against_its_frame():
    """T built from one frame at the identity, every sample in its own voxel,
    is that frame's set: GICP against T follows GICP against the frame."""
    rng = np.random.default_rng(9)
    room = synth.make_room(rng)
    cam = synth.intrinsics(200, 150)
    R0, t0 = synth.corner_pose(room)
    d0, _ = room.raycast(cam, R0, t0)
    Rg, tg = synth.perturb_pose(R0, t0, rng, 0.03, 2.0, exact=True)
    d1, _ = room.raycast(cam, Rg, tg)
    tgt = gicp.local_gaussians(gicp.sample_points(d0, cam, 4)[0], 10)
    src = gicp.local_gaussians(gicp.sample_points(d1, cam, 4)[0], 10)
    T, add = gmap.insert(None, tgt, np.eye(3), np.zeros(3))
    assert len(add) == len(tgt["points"])          # samples ~6 cm apart: one per voxel
    a = gicp.track(src, tgt, np.eye(3), np.zeros(3), 10, iters=8)
    b = gicp.track(src, T, np.eye(3), np.zeros(3), 10, iters=8)
    assert np.allclose(a["R"], b["R"], atol=1e-12) and np.allclose(a["t"], b["t"], atol=1e-12)


def test_fill_depth_closed_form():
    depth = np.array([[1.0, 0.0, -1.0, 2.0]])
    rd = np.array([[0.5, 0.9, 0.3, 0.7]])
    ra = np.array([[0.5, 0.9, 0.4, 0.7]])
    out = gmap.fill_depth(depth, rd, ra)
    assert out.tolist() == [[1.0, 1.0, 0.0, 2.0]]
