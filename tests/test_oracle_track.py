"""Pins for the tracking, SE(3), loss and optimiser oracles (CPU only)."""
import numpy as np
import pytest
import scipy.linalg
from scipy.spatial.transform import Rotation

from oracle import loss, optim, se3, splat, track
from paper_2603_21055_amd import synth


def _model_obs(sc, R, t):
    """Depth observation rendered by the oracle's own model at (R, t)."""
    lin = track.linearise(sc["geo"], sc["cam"], R, t, np.ones((sc["cam"]["H"], sc["cam"]["W"])))
    obs = np.where(lin["valid"], lin["mu"], 0.0)
    return obs.reshape(sc["cam"]["H"], sc["cam"]["W"])


# ---------------------------------------------------------------- SE(3)
def test_se3_exp_matches_library_routines():
    rng = np.random.default_rng(0)
    for _ in range(20):
        xi = rng.normal(size=6) * np.array([0.1, 0.1, 0.1, 0.5, 0.5, 0.5])
        T = se3.exp(xi)
        np.testing.assert_allclose(T[:3, :3], Rotation.from_rotvec(xi[3:]).as_matrix(), atol=1e-13)
        M = np.zeros((4, 4))
        M[:3, :3] = se3.hat(xi[3:])
        M[:3, 3] = xi[:3]
        np.testing.assert_allclose(T, scipy.linalg.expm(M), atol=1e-12)
        np.testing.assert_allclose(se3.log(T), xi, atol=1e-10)
    # tiny angles use the series branch
    xi = np.array([0.01, -0.02, 0.03, 1e-7, -2e-7, 3e-7])
    M = np.zeros((4, 4))
    M[:3, :3] = se3.hat(xi[3:])
    M[:3, 3] = xi[:3]
    np.testing.assert_allclose(se3.exp(xi), scipy.linalg.expm(M), atol=1e-15)


# ---------------------------------------------------------------- tracking
@pytest.fixture(scope="module")
def small_track():
    sc = synth.tracking_scene(31, W=96, H=54)
    sc["obs_model"] = _model_obs(sc, sc["gt"]["R"].astype(np.float64), sc["gt"]["t"].astype(np.float64))
    return sc


def test_residual_vanishes_at_ground_truth(small_track):
    sc = small_track
    lin = track.linearise(sc["geo"], sc["cam"], sc["gt"]["R"].astype(np.float64),
                          sc["gt"]["t"].astype(np.float64), sc["obs_model"])
    assert lin["n_valid"] > 0.8 * 96 * 54
    assert np.abs(lin["r"]).max() < 1e-9
    # H is symmetric positive semi-definite
    np.testing.assert_allclose(lin["H"], lin["H"].T, atol=1e-9 * np.abs(lin["H"]).max())
    assert np.linalg.eigvalsh(lin["H"]).min() > -1e-9 * np.abs(lin["H"]).max()


def test_gauss_newton_recovers_model_pose(small_track):
    sc = small_track
    out = track.track_gn(sc["geo"], sc["cam"], sc["init"]["R"], sc["init"]["t"], sc["obs_model"],
                         iters=30)
    dT = np.eye(4)
    dT[:3, :3] = out["R"] @ sc["gt"]["R"].astype(np.float64).T
    dT[:3, 3] = out["t"] - dT[:3, :3] @ sc["gt"]["t"].astype(np.float64)
    err = se3.log(dT)
    assert np.linalg.norm(err[:3]) < 1e-5
    assert np.degrees(np.linalg.norm(err[3:])) < 1e-4
    # log-likelihood increases from the start to the end
    lls = [t["loglik"] for t in out["trace"]]
    assert lls[-1] > lls[0]


def test_jacobian_matches_finite_differences(small_track):
    sc = small_track
    R = sc["init"]["R"].astype(np.float64)
    t = sc["init"]["t"].astype(np.float64)
    # linearise half-way to the ground truth so the Jacobian is generic
    R, t = se3.left_update(R, t, np.array([0.005, -0.004, 0.003, 0.004, -0.003, 0.002]))
    lin = track.linearise(sc["geo"], sc["cam"], R, t, sc["obs_model"])
    h = 1e-7
    n0 = lin["fwd"]["n"].ravel()
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        Rp, tp = se3.left_update(R, t, e)
        Rm, tm = se3.left_update(R, t, -e)
        lp = track.linearise(sc["geo"], sc["cam"], Rp, tp, sc["obs_model"])
        lm = track.linearise(sc["geo"], sc["cam"], Rm, tm, sc["obs_model"])
        same = (lp["fwd"]["n"].ravel() == n0) & (lm["fwd"]["n"].ravel() == n0) & lin["valid"] \
            & lp["valid"] & lm["valid"]
        fd = -(lp["mu"] - lm["mu"]) / (2 * h) / lin["s"]
        an = lin["J"][:, k]
        assert same.sum() > 0.8 * lin["n_valid"]
        np.testing.assert_allclose(fd[same], an[same], rtol=1e-4,
                                   atol=1e-5 * np.abs(an[same]).max())


def test_single_plane_leaves_three_unobservable_directions():
    cam = dict(H=30, W=40, fx=37.5, fy=37.5, cx=20.0, cy=15.0)
    depth = np.full((30, 40), 2.0, np.float32)
    geo = synth.keyframe_from_frame(cam, np.eye(3), np.zeros(3), depth, None,
                                    np.full((30, 40), 0.9, np.float32),
                                    sigma=np.full((30, 40), 0.01, np.float32))
    obs = np.full((30, 40), 2.01)
    lin = track.linearise(geo, cam, np.eye(3), np.zeros(3), obs)
    ev = np.linalg.eigvalsh(lin["H"])
    assert (ev < 1e-9 * ev.max()).sum() == 3
    dxi, lam = track.solve(lin["H"], lin["g"])
    assert np.isfinite(dxi).all()


# ---------------------------------------------------------------- loss / optimiser
def test_l1_grads_match_finite_differences():
    rng = np.random.default_rng(3)
    rgb, trgb = rng.uniform(size=(3, 6, 5)), rng.uniform(size=(3, 6, 5))
    dep, tdep = rng.uniform(1, 2, size=(6, 5)), rng.uniform(1, 2, size=(6, 5))
    tdep[0, 0] = 0.0       # invalid depth pixel is masked out
    L0, gr, gd = loss.l1_loss(rgb, dep, trgb, tdep)
    h = 1e-7
    for idx in [(0, 1, 2), (2, 5, 4), (1, 0, 0)]:
        a = rgb.copy()
        a[idx] += h
        b = rgb.copy()
        b[idx] -= h
        fd = (loss.l1_loss(a, dep, trgb, tdep)[0] - loss.l1_loss(b, dep, trgb, tdep)[0]) / (2 * h)
        assert abs(fd - gr[idx]) < 1e-7
    for idx in [(0, 0), (3, 2)]:
        a = dep.copy()
        a[idx] += h
        b = dep.copy()
        b[idx] -= h
        fd = (loss.l1_loss(rgb, a, trgb, tdep)[0] - loss.l1_loss(rgb, b, trgb, tdep)[0]) / (2 * h)
        assert abs(fd - gd[idx]) < 1e-7
    assert gd[0, 0] == 0.0


def test_adam_first_step_is_sign_step_and_scale_invariant():
    rng = np.random.default_rng(4)
    p, g = rng.normal(size=50), rng.normal(size=50)
    z = np.zeros(50)
    p1, m, v = optim.adam_step(p, g, z, z, 1, 0.01)
    np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), atol=1e-7)
    g2 = rng.normal(size=50)
    a, _, _ = optim.adam_step(p1, g2, m, v, 2, 0.01)
    _, m5, v5 = optim.adam_step(p, 5.0 * g, z, z, 1, 0.01)
    b, _, _ = optim.adam_step(p1, 5.0 * g2, m5, v5, 2, 0.01)
    np.testing.assert_allclose(a, b, atol=1e-8)


def test_linearise_tolerance_terms_bound_the_values(small_track):
    """The absolute-term sums dominate the values they bound (triangle
    inequality), and the per-pixel pieces reassemble H and g."""
    sc = small_track
    lin = track.linearise(sc["geo"], sc["cam"], sc["init"]["R"].astype(np.float64),
                          sc["init"]["t"].astype(np.float64), np.asarray(sc["obs_depth"], np.float64))
    assert (lin["aH"] >= np.abs(lin["H"])).all() and (lin["ag"] >= np.abs(lin["g"])).all()
    assert lin["aloglik"] >= abs(lin["loglik"])
    np.testing.assert_allclose(lin["J"].T @ lin["J"], lin["H"], rtol=1e-12)
    assert (lin["fH"] >= 0).all() and lin["floglik"] >= 0
