"""Pins of the oracle parts that the first pin set left open: Adam in its
log / logit spaces, the parameter clamps, the binning rectangles (C8) and the
warm-start net's input.  Each checks the oracle against something other than
its own formula: finite differences, hand-worked cases, brute force over
tiles, or a closed form."""
import numpy as np
import pytest

from oracle import conv, optim, splat
from paper_2603_21055_amd import synth


# ---------------------------------------------------------------- Adam spaces
def _loss(p, c):
    """A smooth test loss of the parameter p with a known, varied gradient."""
    return float(np.sum(c * np.sin(3.0 * p) + 0.5 * c * c * p * p))


def _dloss(p, c):
    return c * 3.0 * np.cos(3.0 * p) + c * c * p


def _to_p(theta, space):
    if space == "log":
        return np.exp(theta)
    if space == "logit":
        return 1.0 / (1.0 + np.exp(-theta))
    return theta


def _to_theta(p, space):
    if space == "log":
        return np.log(p)
    if space == "logit":
        return np.log(p / (1.0 - p))
    return p


@pytest.mark.parametrize("space", ["linear", "log", "logit"])
def test_adam_space_gradient_is_fd_of_loss_in_theta(space):
    """After one step from zero moments, m / (1 - beta1) is the gradient the
    step used; it must be dL/dtheta of L(p(theta)) by central differences."""
    rng = np.random.default_rng(40)
    p = rng.uniform(0.05, 0.95, 64)
    c = rng.normal(size=64)
    z = np.zeros(64)
    _, m, v = optim.adam_step_space(p, _dloss(p, c), z, z, 1, 0.01, space)
    g_used = m / (1.0 - optim.BETA1)
    th = _to_theta(p, space)
    h = 1e-6
    fd = np.array([(_loss(_to_p(th[i] + h, space), c[i]) - _loss(_to_p(th[i] - h, space), c[i])) / (2 * h)
                   for i in range(64)])
    np.testing.assert_allclose(g_used, fd, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(v / (1.0 - optim.BETA2), fd * fd, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("space", ["log", "logit"])
def test_adam_space_step_is_adam_on_theta(space):
    """A third step with non-zero moments equals plain Adam applied by hand
    to theta = log p (logit p) with the finite-difference gradient, mapped
    back to p."""
    rng = np.random.default_rng(41)
    p = rng.uniform(0.1, 0.9, 32)
    c = rng.normal(size=32)
    m0 = rng.normal(size=32) * 0.1
    v0 = rng.uniform(0.01, 0.2, 32)
    p_new, m_new, v_new = optim.adam_step_space(p, _dloss(p, c), m0, v0, 3, 0.05, space)
    th = _to_theta(p, space)
    h = 1e-6
    fd = np.array([(_loss(_to_p(th[i] + h, space), c[i]) - _loss(_to_p(th[i] - h, space), c[i])) / (2 * h)
                   for i in range(32)])
    b1, b2, t = optim.BETA1, optim.BETA2, 3
    m = b1 * m0 + (1 - b1) * fd
    v = b2 * v0 + (1 - b2) * fd * fd
    th_new = th - 0.05 * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + optim.EPS)
    np.testing.assert_allclose(p_new, _to_p(th_new, space), rtol=1e-8)
    np.testing.assert_allclose(m_new, m, rtol=1e-6, atol=1e-12)


def test_adam_space_closed_forms_and_guards():
    """Closed forms of the two maps: d sigmoid/d theta = 1/4 at p = 1/2,
    d exp/d theta = p; the logit guard keeps theta finite at p = 0 and 1 and
    the log guard at p = 0."""
    z = np.zeros(3)
    g = np.array([0.8, -1.2, 2.0])
    _, m, _ = optim.adam_step_space(np.full(3, 0.5), g, z, z, 1, 0.05, "logit")
    np.testing.assert_allclose(m / (1 - optim.BETA1), g / 4.0, rtol=1e-12)
    _, m, _ = optim.adam_step_space(np.array([1.0, np.e, 0.25]), g, z, z, 1, 0.005, "log")
    np.testing.assert_allclose(m / (1 - optim.BETA1), g * np.array([1.0, np.e, 0.25]), rtol=1e-12)
    p, _, _ = optim.adam_step_space(np.array([0.0, 1.0, 0.5]), g, z, z, 1, 0.05, "logit")
    assert np.isfinite(p).all() and (p > 0).all() and (p < 1).all()
    # from p = 0 the guard's p = 1e-6 takes one logit step of
    # -lr g_theta / (|g_theta| + eps), g_theta = g p (1 - p) (eps matters here)
    p0 = 1e-6
    gth = 0.8 * p0 * (1 - p0)
    expect0 = 1.0 / (1.0 + np.exp(-(np.log(p0 / (1 - p0)) - 0.05 * gth / (gth + optim.EPS))))
    assert abs(p[0] - expect0) <= 1e-12
    p, _, _ = optim.adam_step_space(np.array([0.0, 0.3, 2.0]), g, z, z, 1, 0.005, "log")
    assert np.isfinite(p).all() and (p > 0).all()
    # a first step moves theta by -lr sign(g): p scales by exp(-lr sign(g))
    np.testing.assert_allclose(p[1:], np.array([0.3, 2.0]) * np.exp(-0.005 * np.sign(g[1:])), rtol=1e-9)


def test_clamp_keeps_parameters_in_their_domains():
    """Opacity is a probability, radius a positive standard deviation; the
    other parameters are unbounded."""
    np.testing.assert_array_equal(optim.clamp("opacity", np.array([-0.5, 0.0, 0.3, 1.0, 1.7])),
                                  [0.0, 0.0, 0.3, 1.0, 1.0])
    r = optim.clamp("radius", np.array([-1.0, 0.0, 1e-7, 1e-6, 0.5]))
    np.testing.assert_array_equal(r, [1e-6, 1e-6, 1e-6, 1e-6, 0.5])
    for name in ("rgb", "offset"):
        x = np.array([-3.0, 0.0, 0.7, 12.0])
        np.testing.assert_array_equal(optim.clamp(name, x), x)


# ---------------------------------------------------------------- binning (C8)
def _g(mx, my, rho, valid=None, z=None):
    n = len(mx)
    return dict(mx=np.asarray(mx, np.float64), my=np.asarray(my, np.float64), rho=np.asarray(rho, np.float64),
                valid=np.ones(n, bool) if valid is None else np.asarray(valid, bool),
                zkey=np.asarray(np.arange(1, n + 1) if z is None else z, np.float32),
                gid=np.arange(n, dtype=np.int64))


def test_tile_rects_hand_worked_cases():
    """C8 on cases worked by hand, 8x8 tiles over a 45x29 view (6 x 4 tiles)."""
    g = _g(mx=[15.5, -3.0, 46.0, 12.0, 7.5, 3.0],
           my=[7.2, 2.0, 30.0, 12.0, 20.0, 3.0],
           rho=[4, 4, 4, 4, 4, 4],
           valid=[1, 1, 1, 1, 1, 0])
    x0, x1, y0, y1, ntx, nty = splat.tile_rects(g, 45, 29, 8, 8)
    assert (ntx, nty) == (6, 4)
    # m = (15.5, 7.2), rho = 4: x in [11.5, 19.5] -> tiles 1..2, y in [3.2, 11.2] -> 0..1
    assert (x0[0], x1[0], y0[0], y1[0]) == (1, 3, 0, 2)
    # left of the image: [-7, 1] clamps to tile 0; y [-2, 6] -> tile 0
    assert (x0[1], x1[1], y0[1], y1[1]) == (0, 1, 0, 1)
    # right/bottom edge: x [42, 50] -> 5..5 (tile 6 does not exist), y [26, 34] -> tile 3 only
    assert (x0[2], x1[2], y0[2], y1[2]) == (5, 6, 3, 4)
    # bounds exactly on tile borders: x in [8, 16] -> tiles 1..2 (pixel 16 is at distance rho)
    assert (x0[3], x1[3], y0[3], y1[3]) == (1, 3, 1, 3)
    # x in [3.5, 11.5] -> tiles 0..1; y in [16, 24] -> 2..3
    assert (x0[4], x1[4], y0[4], y1[4]) == (0, 2, 2, 4)
    # a culled Gaussian covers nothing
    assert x1[5] == x0[5] and y1[5] == y0[5]


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (32, 8), (16, 8)])
def test_tile_rects_equal_brute_force_interval_overlap(tile):
    """The rectangle is exactly the set of tiles whose half-open pixel span
    [t T, (t + 1) T) meets the closed bounding interval [m - rho, m + rho]
    inside the view: checked tile by tile on random means, including means
    outside the view and bounds that land on tile borders."""
    TW, TH = tile
    W, H = 45, 29
    rng = np.random.default_rng(42)
    n = 600
    mx = rng.uniform(-12, W + 12, n)
    my = rng.uniform(-12, H + 12, n)
    rho = rng.integers(1, 12, n).astype(np.float64)
    # a quarter of the bounds exactly on a tile border
    k = n // 4
    mx[:k] = rng.integers(0, W // TW + 1, k) * TW + rho[:k]
    my[k:2 * k] = rng.integers(0, H // TH + 1, k) * TH - rho[k:2 * k]
    g = _g(mx, my, rho)
    x0, x1, y0, y1, ntx, nty = splat.tile_rects(g, W, H, TW, TH)
    for i in range(n):
        xs = [t for t in range(ntx) if t * TW <= mx[i] + rho[i] and mx[i] - rho[i] < (t + 1) * TW]
        ys = [t for t in range(nty) if t * TH <= my[i] + rho[i] and my[i] - rho[i] < (t + 1) * TH]
        got_x = list(range(x0[i], x1[i]))
        got_y = list(range(y0[i], y1[i]))
        if not xs or not ys:
            assert len(got_x) * len(got_y) == 0, i
        else:
            assert got_x == xs and got_y == ys, (i, mx[i], my[i], rho[i])


def test_bin_and_sort_equals_brute_force_instance_list():
    """The instance list is the multiset {(tile, z bits, gid)} over every
    (Gaussian, tile of its rectangle), in lexicographic order: built here by
    explicit loops and Python's sort, with depth ties broken by gid."""
    sc = synth.small_scene(43, 45, 29, n_kf=2, n_views=1, offset_amp=0.03, max_trans=0.05, max_rot=3)
    g = splat.gather_job(sc["kfs"], sc["views"][0], [0, 1])
    # force some equal depth keys so the gid tie-break is exercised
    g = dict(g)
    z = g["zkey"].copy()
    z[1::7] = z[0::7][:len(z[1::7])]
    g["zkey"] = z
    for TW, TH in ((8, 8), (16, 16)):
        x0, x1, y0, y1, ntx, nty = splat.tile_rects(g, 45, 29, TW, TH)
        inst = []
        for i in range(len(g["gid"])):
            for ty in range(y0[i], y1[i]):
                for tx in range(x0[i], x1[i]):
                    inst.append((ty * ntx + tx, int(g["zkey"][i].view(np.uint32)), int(g["gid"][i])))
        inst.sort()
        b = splat.bin_and_sort(g, 45, 29, TW, TH)
        got = list(zip(b["tile"].tolist(), b["zbits"].astype(np.int64).tolist(), b["gid"].tolist()))
        assert got == inst
        for t in range(ntx * nty):
            s, e = b["ranges"][t]
            assert all(x[0] == t for x in got[s:e])
            assert sum(1 for x in inst if x[0] == t) == e - s


# ---------------------------------------------------------------- net input
def test_net_input_layout_one_pixel_and_small_image():
    """Channel order (R, G, B, depth channel) per pixel in [H][W][4], worked
    by hand on single pixels of a 2 x 3 image."""
    rgb = np.zeros((3, 2, 3))
    rgb[0] = [[0.1, 0.2, 0.3], [0.4, 0.5, 0.6]]
    rgb[1] = 1.0 - rgb[0]
    rgb[2] = 0.25
    depth = np.array([[2.5, 1.0, 5.0], [0.5, 4.0, 3.0]])
    x = conv.net_input(rgb, depth)
    assert x.shape == (2, 3, 4)
    np.testing.assert_allclose(x[0, 0], [0.1, 0.9, 0.25, conv.depth_channel(depth)[0, 0]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(x[1, 2], [0.6, 0.4, 0.25, conv.depth_channel(depth)[1, 2]], rtol=0, atol=1e-15)


def test_depth_channel_closed_forms():
    """h = (D - local 3x3 mean) / 2 cm: zero on a constant depth and on a
    plane's interior (the mean of an affine function over a symmetric window
    is its centre value); an edge pixel of a ramp sees the one-sided mean; a
    spike of height s gives 8s/9 at its centre and -s/9 at its 8 neighbours
    (3s/4 and -s/4 in a corner, whose window holds 4 pixels)."""
    H, W = 7, 9
    s = conv.DEPTH_HP_SCALE
    np.testing.assert_allclose(conv.depth_channel(np.full((H, W), 2.7)), 0.0, atol=1e-12)
    yy, xx = np.mgrid[0:H, 0:W]
    ramp = 1.0 + 0.01 * xx + 0.03 * yy
    h = conv.depth_channel(ramp)
    np.testing.assert_allclose(h[1:-1, 1:-1], 0.0, atol=1e-12)
    # left column, interior rows: window columns {0, 1} -> mean x = 0.5
    np.testing.assert_allclose(h[1:-1, 0], -0.5 * 0.01 / s, rtol=1e-12)
    spike = np.full((H, W), 2.0)
    spike[3, 4] += 0.05
    h = conv.depth_channel(spike)
    assert abs(h[3, 4] - 8 * 0.05 / 9 / s) < 1e-12
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy or dx:
                assert abs(h[3 + dy, 4 + dx] + 0.05 / 9 / s) < 1e-12
    assert np.abs(h[:, :2]).max() == 0.0 and np.abs(h[:, 7:]).max() == 0.0
    corner = np.full((H, W), 2.0)
    corner[0, 0] += 0.04
    h = conv.depth_channel(corner)
    assert abs(h[0, 0] - 0.75 * 0.04 / s) < 1e-12
    assert abs(h[1, 1] + 0.04 / 9 / s) < 1e-12 and abs(h[0, 1] + 0.04 / 6 / s) < 1e-12


def test_depth_channel_equals_pixel_loop():
    rng = np.random.default_rng(44)
    D = rng.uniform(0.5, 5.0, (6, 11))
    h = conv.depth_channel(D)
    for y in range(6):
        for x in range(11):
            nb = [D[j, i] for j in range(max(0, y - 1), min(6, y + 2)) for i in range(max(0, x - 1), min(11, x + 2))]
            assert abs(h[y, x] - (D[y, x] - sum(nb) / len(nb)) / conv.DEPTH_HP_SCALE) < 1e-9


# ------------------------------------------------ tolerance model of the weights
def test_transmittance_conditioning_bounds_fp32_weights():
    """The gradient tolerances scale each term by 1 + kappa_j, kappa_j the
    sum of alpha_i / (1 - alpha_i) over the pixel's earlier contributors
    (``composite``'s Kb).  The claim behind it, on random chains with
    near-opaque layers and the T_MIN stop rule: weights w_j = alpha_j T_j
    evaluated in float32 from alphas with a relative error of up to 2^-17
    (what the float32 q of a pair displaced by up to 64 px carries: half its
    error, 2^-24 |dq/ddx| |Delta|) stay within 1e-5 (1 + kappa_j) |w_j| of the
    float64 value, while the unconditioned 1e-5 |w_j| does not hold for all
    of them."""
    rng = np.random.default_rng(5)
    f32 = np.float32
    worst_c, worst_plain = 0.0, 0.0
    for _ in range(2000):
        n = int(rng.integers(5, 60))
        a64 = np.where(rng.uniform(size=n) < 0.3, rng.uniform(0.95, 0.99, n), rng.uniform(1 / 255, 0.95, n))
        a32 = np.minimum(a64 * (1.0 + rng.uniform(-1, 1, n) * 2.0 ** -17), 0.99).astype(f32)
        T64, T32, kap = 1.0, f32(1.0), 0.0
        for j in range(n):
            if T64 * (1.0 - a64[j]) < splat.T_MIN:
                break
            w64 = a64[j] * T64
            w32 = float(f32(a32[j] * T32))
            rel = abs(w32 - w64) / w64
            worst_c = max(worst_c, rel / (1e-5 * (1.0 + kap)))
            worst_plain = max(worst_plain, rel / 1e-5)
            T64 *= 1.0 - a64[j]
            T32 = f32(T32 * f32(f32(1.0) - a32[j]))
            kap += a64[j] / (1.0 - a64[j])
    assert worst_c <= 1.0, worst_c
    assert worst_plain > 1.0, worst_plain


def test_composite_reports_the_conditioning():
    """Kb / K of ``composite`` on a hand-made stack at one pixel: three
    Gaussians with alphas 0.5, 0.99, 0.99."""
    g = dict(col=np.zeros((3, 3)), z=np.array([1.0, 2.0, 3.0]))
    P = dict(pix=np.zeros(3, np.int64), alpha=np.array([0.5, 0.99, 0.99]), gi=np.arange(3))
    out = splat.composite(g, P, 1)
    # the third would take T to 0.5 * 0.01 * 0.01 = 5e-5 < 1e-4: not composited
    assert out["con"].tolist() == [True, True, False]
    assert np.allclose(out["Kb"][:2], [0.0, 1.0])
    assert np.isclose(out["K"][0], 1.0 + 99.0)
