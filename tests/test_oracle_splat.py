"""Pins for the FP64 splatting oracle (CPU only).

Each test checks the oracle against something other than itself: a closed
form, an invariant, a brute-force evaluation, finite differences, a library
routine or an independent autograd re-derivation.
"""
import json
import os

import numpy as np
import pytest

from oracle import splat
from paper_2603_21055_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _tiny_kf(depths, opac, cols, H=1, W=1, fx=100.0):
    """A 1x1 keyframe per entry, all on the optical axis at identity pose."""
    kfs = []
    for d, o, c in zip(depths, opac, cols):
        cam = dict(H=H, W=W, fx=fx, fy=fx, cx=0.0, cy=0.0)
        kf = synth.keyframe_from_frame(cam, np.eye(3), np.zeros(3),
                                       np.full((H, W), d, np.float32),
                                       np.array(c, np.float32).reshape(3, 1, 1),
                                       np.full((H, W), o, np.float32))
        kfs.append(kf)
    return kfs


def _loss(fwd, gr, gd, ga):
    return float((fwd["rgb"] * gr).sum() + (fwd["depth"] * gd).sum() + (fwd["alpha"] * ga).sum())


# ---------------------------------------------------------------- footprint
def test_on_axis_footprint_is_1p3_identity():
    # r = z/fx on the optical axis gives sigma = 1 px; dilation 0.3 -> 1.3 I
    kfs = _tiny_kf([2.0], [0.9], [(1, 0, 0)])
    kfs[0]["radius"][:] = np.float32(2.0) / np.float32(100.0)
    g = splat.preprocess(kfs[0], kfs[0]["cam"], np.eye(3), np.zeros(3))
    r = float(np.float32(2.0) / np.float32(100.0))
    expect = (r * 100.0 / 2.0) ** 2 + 0.3
    assert abs(g["s00"][0] - expect) < 1e-12 and abs(g["s11"][0] - expect) < 1e-12
    assert g["s01"][0] == 0.0
    assert abs(g["ca"][0] - 1.0 / expect) < 1e-12 and g["rho"][0] == 4.0


def test_footprint_matches_fd_of_projected_mean():
    # the mean moves by J dX when the view translation moves by dX, so finite
    # differences of the oracle's own mean give J independently of the
    # analytic J used in Sigma2 = r^2 J J^T + 0.3 I
    sc = synth.small_scene(5, 20, 15, max_trans=0.05, max_rot=3.0)
    kf, view = sc["kfs"][0], sc["views"][0]
    R = view["R"].astype(np.float64)
    t = view["t"].astype(np.float64)
    g0 = splat.preprocess(kf, view["cam"], R, t)
    h = 1e-6
    J = np.zeros((kf["cam"]["H"] * kf["cam"]["W"], 2, 3))
    for k in range(3):
        tp, tm = t.copy(), t.copy()
        tp[k] += h
        tm[k] -= h
        gp = splat.preprocess(kf, view["cam"], R, tp)
        gm = splat.preprocess(kf, view["cam"], R, tm)
        J[:, 0, k] = (gp["mx"] - gm["mx"]) / (2 * h)
        J[:, 1, k] = (gp["my"] - gm["my"]) / (2 * h)
    S = g0["r"][:, None, None] ** 2 * np.einsum("nik,njk->nij", J, J)
    np.testing.assert_allclose(S[:, 0, 0] + 0.3, g0["s00"], rtol=1e-6)
    np.testing.assert_allclose(S[:, 0, 1], g0["s01"], rtol=1e-5, atol=1e-8)
    np.testing.assert_allclose(S[:, 1, 1] + 0.3, g0["s11"], rtol=1e-6)
    # conic is the inverse and rho bounds the 3-sigma ellipse
    for i in range(0, len(S), 37):
        Sig = np.array([[g0["s00"][i], g0["s01"][i]], [g0["s01"][i], g0["s11"][i]]])
        Q = np.linalg.inv(Sig)
        np.testing.assert_allclose([g0["ca"][i], g0["cb"][i], g0["cc"][i]],
                                   [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-12)
        assert g0["rho"][i] >= 3.0 * np.sqrt(np.linalg.eigvalsh(Sig).max())


def test_identity_pose_projects_to_own_pixel():
    sc = synth.plane_scene(0)
    g = splat.preprocess(sc["kfs"][0], sc["views"][0]["cam"], sc["views"][0]["R"], sc["views"][0]["t"])
    assert np.abs(g["mx"] - g["u"]).max() < 1e-12
    assert np.abs(g["my"] - g["v"]).max() < 1e-12


def test_identity_pose_offset_slides_along_own_ray():
    sc = synth.small_scene(6, 16, 12)
    kf = sc["kfs"][0]
    g0 = splat.preprocess(kf, kf["cam"], kf["R"], kf["t"])
    kf2 = dict(kf, offset=(kf["offset"] + np.float32(0.01)).astype(np.float32))
    g1 = splat.preprocess(kf2, kf["cam"], kf["R"], kf["t"])
    assert np.abs(g1["mx"] - g0["mx"]).max() < 1e-11
    assert np.abs(g1["z"] - g0["z"] - 0.01).max() < 1e-6


# ---------------------------------------------------------------- invariants
def test_similarity_invariance():
    sc = synth.small_scene(7, 24, 18, n_kf=2, n_views=1, offset_amp=0.02)
    base = splat.render_job(sc["kfs"], sc["views"][0], [0, 1])
    s = 2.0
    kfs = []
    for kf in sc["kfs"]:
        k2 = dict(kf)
        for key in ("depth", "offset", "radius"):
            k2[key] = (kf[key].astype(np.float64) * s)
        k2["t"] = kf["t"].astype(np.float64) * s
        kfs.append(k2)
    view = dict(sc["views"][0], t=sc["views"][0]["t"].astype(np.float64) * s)
    sc2 = splat.render_job(kfs, view, [0, 1])
    np.testing.assert_allclose(sc2["rgb"], base["rgb"], atol=1e-12)
    np.testing.assert_allclose(sc2["alpha"], base["alpha"], atol=1e-12)
    np.testing.assert_allclose(sc2["depth"], s * base["depth"], atol=1e-11)


def test_adjusted_depth_is_absolute_value():
    # |D + delta|: (D, delta) renders like (D + delta, 0) and like (-(D + delta), 0);
    # delta = 0 is the paper's "fixed at depth" mode
    sc = synth.small_scene(8, 20, 15, offset_amp=0.05)
    kf = sc["kfs"][0]
    a = splat.render_job([kf], sc["views"][0], [0])
    s = kf["depth"].astype(np.float64) + kf["offset"].astype(np.float64)
    b = splat.render_job([dict(kf, depth=s, offset=np.zeros_like(s))], sc["views"][0], [0])
    c = splat.render_job([dict(kf, depth=-s, offset=np.zeros_like(s))], sc["views"][0], [0])
    for k in ("rgb", "depth", "alpha"):
        np.testing.assert_allclose(a[k], b[k], atol=1e-13)
        np.testing.assert_allclose(a[k], c[k], atol=1e-13)


# ---------------------------------------------------------------- compositing
def test_stack_transmittance_closed_form():
    # Gaussians stacked on one pixel ray: q = 0, alpha = min(0.99, o)
    depths = [3.0, 1.0, 2.0, 4.0]
    opac = [0.95, 0.95, 0.95, 0.95]
    cols = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]
    kfs = _tiny_kf(depths, opac, cols)
    view = dict(cam=kfs[0]["cam"], R=np.eye(3), t=np.zeros(3))
    out = splat.render_job(kfs, view, [0, 1, 2, 3])
    a = float(np.float32(0.95))
    order = np.argsort(depths)
    T, rgb, dep, n = 1.0, np.zeros(3), 0.0, 0
    for i in order:                       # 1.0, 2.0, 3.0; the 4th would drop T below 1e-4
        if T * (1 - a) < 1e-4:
            break
        rgb += a * T * np.array(cols[i])
        dep += a * T * depths[i]
        T *= 1 - a
        n += 1
    assert n == 3 and out["n"][0, 0] == 3
    assert abs(out["alpha"][0, 0] - (1 - (1 - a) ** 3)) < 1e-15
    np.testing.assert_allclose(out["rgb"][:, 0, 0], rgb, atol=1e-15)
    assert abs(out["depth"][0, 0] - dep) < 1e-14


def test_two_gaussian_order_swap():
    kfs = _tiny_kf([1.0, 2.0], [0.6, 0.3], [(1, 0, 0), (0, 1, 0)])
    view = dict(cam=kfs[0]["cam"], R=np.eye(3), t=np.zeros(3))
    o1, o2 = float(np.float32(0.6)), float(np.float32(0.3))
    a = splat.render_job(kfs, view, [0, 1])["rgb"][:, 0, 0]
    np.testing.assert_allclose(a, [o1, (1 - o1) * o2, 0], atol=1e-15)
    kfs[0]["depth"][:] = 3.0
    kfs[0]["radius"][:] = np.float32(3.0 / 100.0)
    b = splat.render_job(kfs, view, [0, 1])["rgb"][:, 0, 0]
    np.testing.assert_allclose(b, [(1 - o2) * o1, o2, 0], atol=1e-15)


def test_alpha_clamp_and_min_alpha():
    kfs = _tiny_kf([1.0, 2.0], [1.0, 0.003], [(1, 0, 0), (0, 1, 0)])
    view = dict(cam=kfs[0]["cam"], R=np.eye(3), t=np.zeros(3))
    out = splat.render_job(kfs, view, [0, 1])
    # first clamps to 0.99, second is below 1/255 and skipped
    assert out["n"][0, 0] == 1
    np.testing.assert_allclose(out["rgb"][:, 0, 0], [0.99, 0, 0], atol=1e-15)


def test_bruteforce_equals_culled_c1_both_views():
    sc = synth.plane_scene(0)
    for view in sc["views"]:
        a = splat.render_job(sc["kfs"], view, [0])
        b = splat.render_bruteforce(sc["kfs"], view, [0])
        for k in ("rgb", "depth", "alpha"):
            assert np.abs(a[k] - b[k]).max() <= 1e-14
        assert (a["n"] == b["n"]).all()


def test_bruteforce_equals_culled_two_keyframes():
    sc = synth.small_scene(9, 16, 12, n_kf=2, n_views=2, offset_amp=0.03, max_trans=0.05, max_rot=3)
    for view in sc["views"]:
        a = splat.render_job(sc["kfs"], view, [0, 1])
        b = splat.render_bruteforce(sc["kfs"], view, [0, 1])
        for k in ("rgb", "depth", "alpha"):
            assert np.abs(a[k] - b[k]).max() <= 1e-14
        assert (a["n"] == b["n"]).all()


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8), (16, 8)])
def test_tiled_walk_equals_untiled(tile):
    sc = synth.small_scene(11, 37, 21, n_kf=2, n_views=1, offset_amp=0.03, max_trans=0.05, max_rot=3)
    a = splat.render_job(sc["kfs"], sc["views"][0], [0, 1])
    b = splat.render_tiled(sc["kfs"], sc["views"][0], [0, 1], *tile)
    for k in ("rgb", "depth", "alpha"):
        assert np.abs(a[k] - b[k]).max() <= 1e-14
    assert (a["n"] == b["n"]).all()


def test_binning_is_conservative_and_sorted():
    sc = synth.small_scene(12, 45, 29, n_kf=2, n_views=1, offset_amp=0.03, max_trans=0.05, max_rot=3)
    fwd = splat.render_job(sc["kfs"], sc["views"][0], [0, 1])
    g = fwd["g"]
    for TW, TH in ((16, 16), (8, 8)):
        b = splat.bin_and_sort(g, 45, 29, TW, TH)
        inst = set(zip(b["tile"].tolist(), b["gid"].tolist()))
        P = fwd["P"]
        px, py = P["pix"] % 45, P["pix"] // 45
        tiles = (py // TH) * b["ntx"] + px // TW
        gids = g["gid"][P["gi"]]
        assert all((int(t), int(q)) in inst for t, q in zip(tiles, gids))
        key = np.stack([b["tile"], b["zbits"].astype(np.int64), b["gid"]], 1)
        assert (np.diff(key[:, 0]) >= 0).all()
        same = key[1:, 0] == key[:-1, 0]
        z_up = key[1:, 1] > key[:-1, 1]
        tie = (key[1:, 1] == key[:-1, 1]) & (key[1:, 2] > key[:-1, 2])
        assert (~same | z_up | tie).all()
        r = b["ranges"]
        assert r[0, 0] == 0 and r[-1, 1] == len(b["tile"]) and (r[1:, 0] == r[:-1, 1]).all()


# ---------------------------------------------------------------- adjoint
def _fd_scene():
    sc = synth.small_scene(13, 14, 10, n_kf=2, n_views=1, offset_amp=0.03, max_trans=0.02, max_rot=1)
    kfs = []
    for kf in sc["kfs"]:
        k2 = dict(kf)
        for key in ("depth", "offset", "radius", "opacity", "rgb"):
            k2[key] = kf[key].astype(np.float64)
        kfs.append(k2)
    view = dict(sc["views"][0], R=sc["views"][0]["R"].astype(np.float64),
                t=sc["views"][0]["t"].astype(np.float64))
    rng = np.random.default_rng(0)
    gr, gd, ga = rng.normal(size=(3, 10, 14)), rng.normal(size=(10, 14)), rng.normal(size=(10, 14))
    return kfs, view, gr, gd, ga


def _same_sets(a, b):
    return (a["n"] == b["n"]).all() and len(a["P"]["gi"]) == len(b["P"]["gi"]) and \
        (a["P"]["gi"] == b["P"]["gi"]).all() and (a["comp"]["con"] == b["comp"]["con"]).all()


def test_adjoint_matches_finite_differences():
    kfs, view, gr, gd, ga = _fd_scene()
    ids = [0, 1]
    f0 = splat.render_job(kfs, view, ids)
    b = splat.render_backward(kfs, [view], [(0, ids)], [f0], [gr], [gd], [ga])
    rng = np.random.default_rng(1)
    checked = 0
    for name, gkey in (("offset", "d_offset"), ("radius", "d_radius"), ("opacity", "d_opacity"),
                       ("rgb", "d_rgb")):
        for _ in range(10):
            f = int(rng.integers(0, 2))
            arr = kfs[f][name]
            idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
            h = 1e-6 * max(1.0, abs(float(arr[idx])))
            old = arr[idx]
            arr[idx] = old + h
            fp = splat.render_job(kfs, view, ids)
            arr[idx] = old - h
            fm = splat.render_job(kfs, view, ids)
            arr[idx] = old
            if not (_same_sets(fp, f0) and _same_sets(fm, f0)):
                continue
            fd = (_loss(fp, gr, gd, ga) - _loss(fm, gr, gd, ga)) / (2 * h)
            an = b["kf"][f][gkey][idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, f, idx, fd, an)
            checked += 1
    assert checked >= 30


def test_depth_and_offset_gradients_coincide():
    kfs, view, gr, gd, ga = _fd_scene()
    f0 = splat.render_job(kfs, view, [0, 1])
    b = splat.render_backward(kfs, [view], [(0, [0, 1])], [f0], [gr], [gd], [ga])
    rng = np.random.default_rng(2)
    for _ in range(8):
        idx = (int(rng.integers(0, 10)), int(rng.integers(0, 14)))
        arr = kfs[0]["depth"]
        old = arr[idx]
        h = 1e-6
        arr[idx] = old + h
        fp = splat.render_job(kfs, view, [0, 1])
        arr[idx] = old - h
        fm = splat.render_job(kfs, view, [0, 1])
        arr[idx] = old
        fd = (_loss(fp, gr, gd, ga) - _loss(fm, gr, gd, ga)) / (2 * h)
        assert abs(fd - b["kf"][0]["d_offset"][idx]) <= 1e-6 * max(1.0, abs(fd))


def test_pose_gradient_matches_left_twist_fd():
    from oracle import se3
    kfs, view, gr, gd, ga = _fd_scene()
    f0 = splat.render_job(kfs, view, [0, 1])
    b = splat.render_backward(kfs, [view], [(0, [0, 1])], [f0], [gr], [gd], [ga])
    h = 1e-7
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        Rp, tp = se3.left_update(view["R"], view["t"], e)
        Rm, tm = se3.left_update(view["R"], view["t"], -e)
        fp = splat.render_job(kfs, dict(view, R=Rp, t=tp), [0, 1])
        fm = splat.render_job(kfs, dict(view, R=Rm, t=tm), [0, 1])
        assert _same_sets(fp, f0) and _same_sets(fm, f0)
        fd = (_loss(fp, gr, gd, ga) - _loss(fm, gr, gd, ga)) / (2 * h)
        assert abs(fd - b["d_pose"][0, k]) <= 2e-6 * max(1.0, abs(fd)), (k, fd, b["d_pose"][0, k])


def test_adjoint_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    from tests.torch_ref import render_torch
    kfs, view, gr, gd, ga = _fd_scene()
    f0 = splat.render_job(kfs, view, [0, 1])
    b = splat.render_backward(kfs, [view], [(0, [0, 1])], [f0], [gr], [gd], [ga])
    res = render_torch(kfs, view, [0, 1], gr, gd, ga)
    np.testing.assert_allclose(res["rgb"], f0["rgb"], atol=1e-12)
    for f in range(2):
        for name, key in (("offset", "d_offset"), ("radius", "d_radius"), ("opacity", "d_opacity"),
                          ("rgb", "d_rgb")):
            np.testing.assert_allclose(res["grad"][f][name], b["kf"][f][key], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(res["pose"], b["d_pose"][0], rtol=1e-9, atol=1e-11)


def test_non_learnable_keyframe_gets_no_grad():
    kfs, view, gr, gd, ga = _fd_scene()
    f0 = splat.render_job(kfs, view, [0, 1])
    b = splat.render_backward(kfs, [view], [(0, [0, 1])], [f0], [gr], [gd], [ga], learnable={1})
    assert np.abs(b["kf"][0]["d_offset"]).max() == 0.0
    assert np.abs(b["kf"][1]["d_offset"]).max() > 0.0


# ---------------------------------------------------------------- paper numbers
def test_paper_constants_fixture():
    from oracle import loss, optim
    c = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))
    assert (loss.RHO, loss.TAU, loss.SIGMA) == (c["loss_weights"]["rho"], c["loss_weights"]["tau"],
                                                c["loss_weights"]["sigma"])
    for k in ("rgb", "radius", "opacity", "offset"):
        assert optim.LR[k] == c["learning_rates"][k]
    # the per-Gaussian learnable planes: offset, radius, opacity, 3 colours
    kf = synth.plane_scene(0)["kfs"][0]
    n_attr = sum(kf[k].reshape(-1, kf["depth"].size).shape[0] for k in ("offset", "radius", "opacity", "rgb"))
    assert n_attr == c["attributes_per_gaussian"]["value"]
    W, H = c["learnable_gaussians_one_frame"]["frame"]
    assert W * H == c["learnable_gaussians_one_frame"]["value"]


def test_window_render_equals_full_render_inside_the_window():
    """render_window: pixel outputs inside the window and the gradients of the
    Gaussians it marks complete equal the whole-frame oracle's."""
    sc = synth.small_scene(13, 45, 29, n_kf=2, n_views=1, offset_amp=0.03, max_trans=0.05, max_rot=3)
    view = sc["views"][0]
    full = splat.render_job(sc["kfs"], view, [0, 1])
    win = (9, 4, 33, 22)
    wr = splat.render_window(sc["kfs"], view, [0, 1], win)
    sl = (slice(win[1], win[3]), slice(win[0], win[2]))
    for k in ("depth", "alpha", "n"):
        np.testing.assert_array_equal(wr[k][sl], full[k][sl])
    np.testing.assert_array_equal(wr["rgb"][:, sl[0], sl[1]], full["rgb"][:, sl[0], sl[1]])
    np.testing.assert_array_equal(wr["flags"][sl], full["flags"][sl])
    rng = np.random.default_rng(3)
    gr, gd, ga = rng.normal(size=(3, 29, 45)), rng.normal(size=(29, 45)), rng.normal(size=(29, 45))
    bf = splat.backward_job(sc["kfs"], view, full, gr, gd, ga)
    bw = splat.backward_job(sc["kfs"], view, wr, gr, gd, ga)
    comp = wr["complete"]
    assert comp.sum() > 50
    pos = {int(x): i for i, x in enumerate(full["g"]["gid"])}
    at = np.array([pos[int(x)] for x in wr["g"]["gid"][comp]])
    for k in ("d_rgb", "d_opacity", "d_radius", "d_offset", "a_offset"):
        np.testing.assert_allclose(bw[k][comp], bf[k][at], rtol=1e-12, atol=1e-15)
