"""FP64 oracle: splatting pixel-aligned simplified Gaussians, forward and adjoint.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain NumPy float64.

What is computed (paper Sec. 3.1-3.2; the paper names the operation
``splat(G_i, p_k)`` without formulas, so the formulas below follow the 3DGS
conventions it builds on; every constant is named here):

* A Gaussian sits at pixel (u, v) of keyframe f at z-depth d = |D + delta|
  (Sec. 3.2, adjusted depth map), i.e. at X_f = d * ((u-cx)/fx, (v-cy)/fy, 1).
  Its covariance is isotropic r^2 I with r a world-space standard deviation
  (Sec. 3.1 keeps one variance term, "radius").
* It is moved into view k by T_rel = T_k T_f^-1 (world->camera poses), culled
  if z < Z_NEAR, projected to m = (fx x/z + cx, fy y/z + cy), and its screen
  covariance is Sigma2 = r^2 J J^T + LOWPASS I with the perspective Jacobian J.
* A pixel p takes Gaussian j iff q = (p-m)^T Sigma2^-1 (p-m) <= Q_CUT and
  alpha = min(ALPHA_MAX, o exp(-q/2)) >= ALPHA_MIN.
* Contributors are composited front to back by (depth key, gid), where the
  depth key is z rounded to float32 and gid = kf_index * H * W + v * W + u.
  Compositing stops before the first contributor that would bring the
  transmittance below T_MIN.  RGB = sum w c, D' = sum w z (unnormalised),
  A = 1 - T, with w = alpha * T.
* The adjoint is the exact derivative with the index sets (cuts, clamp,
  termination) held fixed.  The pose gradient is taken with respect to a
  left twist xi = (rho, phi) on the view's world->camera pose:
  T_k <- Exp(xi) T_k, so dX/dxi = [I | -[X]x].

Binning contract: tile rectangles are an integer function of FP64 values
computed with the exact operation order written in ``preprocess`` (no fused
multiply-add); see ``tile_rects`` / ``bin_and_sort``.
"""
from __future__ import annotations

import numpy as np

LOWPASS = 0.3           # screen-space dilation, px^2
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
Z_NEAR = 0.2            # metres
Q_CUT = 9.0             # 3-sigma ellipse

# near-threshold margins used to flag pixels whose contributor set is decided
# by a rounding-level difference between FP32 and FP64 evaluation
FLAG_Q = 1e-4
FLAG_ALPHA = 1e-7
FLAG_CLAMP = 1e-6
FLAG_T = 1e-9


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
def relative_pose(view_R, view_t, kf_R, kf_t):
    """T_rel = T_view * T_kf^-1 for world->camera poses, in FP64.

    R_rel[i][j] = (Rv[i][0] Rf[j][0] + Rv[i][1] Rf[j][1]) + Rv[i][2] Rf[j][2]
    t_rel[i]    = tv[i] - ((R_rel[i][0] tf[0] + R_rel[i][1] tf[1]) + R_rel[i][2] tf[2])
    (operation order fixed: it feeds the binning contract).
    """
    # float32 poses (what the library receives) promote exactly; float64 poses
    # are accepted so finite differences can perturb below float32 resolution
    Rv = [[float(x) for x in row] for row in np.asarray(view_R)]
    Rf = [[float(x) for x in row] for row in np.asarray(kf_R)]
    tv = [float(x) for x in np.asarray(view_t)]
    tf = [float(x) for x in np.asarray(kf_t)]
    Rr = [[(Rv[i][0] * Rf[j][0] + Rv[i][1] * Rf[j][1]) + Rv[i][2] * Rf[j][2]
           for j in range(3)] for i in range(3)]
    tr = [tv[i] - ((Rr[i][0] * tf[0] + Rr[i][1] * tf[1]) + Rr[i][2] * tf[2]) for i in range(3)]
    return np.array(Rr, np.float64), np.array(tr, np.float64)


def _f(x):
    """float32 camera constant promoted to float64 (what the kernel sees)."""
    return float(np.float32(x))


def preprocess(kf: dict, vcam: dict, vR, vt) -> dict:
    """Per-Gaussian view-space quantities of keyframe ``kf`` seen from view
    (vcam, vR, vt).  All FP64; operation order is part of the binning contract.
    """
    cam = kf["cam"]
    H, W = cam["H"], cam["W"]
    R, t = relative_pose(vR, vt, kf["R"], kf["t"])
    D = kf["depth"].astype(np.float64).ravel()
    dl = kf["offset"].astype(np.float64).ravel()
    r = kf["radius"].astype(np.float64).ravel()
    s = D + dl
    d = np.abs(s)
    sgn = np.where(s >= 0.0, 1.0, -1.0)              # sign(0) taken as +1
    u = np.tile(np.arange(W, dtype=np.float64), H)
    v = np.repeat(np.arange(H, dtype=np.float64), W)
    xn = (u - _f(cam["cx"])) / _f(cam["fx"])
    yn = (v - _f(cam["cy"])) / _f(cam["fy"])
    X0, X1, X2 = d * xn, d * yn, d
    x = ((R[0, 0] * X0 + R[0, 1] * X1) + R[0, 2] * X2) + t[0]
    y = ((R[1, 0] * X0 + R[1, 1] * X1) + R[1, 2] * X2) + t[1]
    z = ((R[2, 0] * X0 + R[2, 1] * X1) + R[2, 2] * X2) + t[2]
    valid = z >= Z_NEAR
    zs = np.where(valid, z, 1.0)                      # avoid 0-division on culled ones
    fx, fy, cx, cy = _f(vcam["fx"]), _f(vcam["fy"]), _f(vcam["cx"]), _f(vcam["cy"])
    tx = x / zs
    ty = y / zs
    mx = fx * tx + cx
    my = fy * ty + cy
    jx = fx / zs
    jy = fy / zs
    k00 = (jx * jx) * (1.0 + tx * tx)
    k01 = (jx * jy) * (tx * ty)
    k11 = (jy * jy) * (1.0 + ty * ty)
    r2 = r * r
    s00 = r2 * k00 + LOWPASS
    s01 = r2 * k01
    s11 = r2 * k11 + LOWPASS
    det = s00 * s11 - s01 * s01
    ca = s11 / det
    cb = -s01 / det
    cc = s00 / det
    hd = 0.5 * (s00 - s11)
    lam = 0.5 * (s00 + s11) + np.sqrt(hd * hd + s01 * s01)
    rho = np.ceil(3.0 * np.sqrt(lam))
    return dict(H=H, W=W, N=H * W, x=x, y=y, z=z, valid=valid, mx=mx, my=my,
                s00=s00, s01=s01, s11=s11, ca=ca, cb=cb, cc=cc, rho=rho,
                zkey=z.astype(np.float32), d=d, sgn=sgn, xn=xn, yn=yn, r=r,
                R=R, t=t, fx=fx, fy=fy, cx=cx, cy=cy, u=u, v=v)


# ----------------------------------------------------------------------------
# the job's Gaussian set
# ----------------------------------------------------------------------------
GAUSS_KEYS = ("x", "y", "z", "valid", "mx", "my", "s00", "s01", "s11", "ca", "cb", "cc",
              "rho", "zkey", "d", "sgn", "xn", "yn", "r", "gid", "kf", "part", "o", "u", "v")


def gather_job(kfs, view, kf_ids, channels="rgb") -> dict:
    """Concatenate the preprocessed Gaussians of keyframes ``kf_ids`` seen
    from ``view``; colour channels are RGB or, for tracking, sigma^2."""
    parts = []
    for f in kf_ids:
        kf = kfs[f]
        g = preprocess(kf, view["cam"], view["R"], view["t"])
        N = g["N"]
        g["gid"] = f * N + np.arange(N, dtype=np.int64)
        g["kf"] = np.full(N, f, np.int64)
        g["part"] = np.full(N, len(parts), np.int64)
        g["o"] = kf["opacity"].astype(np.float64).ravel()
        if channels == "rgb":
            g["col"] = kf["rgb"].astype(np.float64).reshape(3, -1).T
        else:
            sg = kf["sigma"].astype(np.float64).ravel()
            g["col"] = (sg * sg)[:, None]
        parts.append(g)
    out = {}
    for key in GAUSS_KEYS:
        out[key] = np.concatenate([p[key] for p in parts])
    out["col"] = np.concatenate([p["col"] for p in parts], 0)
    out["parts"] = parts
    out["kf_ids"] = list(kf_ids)
    return out


# ----------------------------------------------------------------------------
# contribution rule
# ----------------------------------------------------------------------------
def _pair_eval(g, gi, px, py):
    """q, G, raw and clamped alpha for (Gaussian gi, pixel (px, py)) pairs."""
    dx = px - g["mx"][gi]
    dy = py - g["my"][gi]
    a, b, c = g["ca"][gi], g["cb"][gi], g["cc"][gi]
    q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy
    G = np.exp(-0.5 * q)
    raw = g["o"][gi] * G
    alpha = np.minimum(ALPHA_MAX, raw)
    return dx, dy, q, G, raw, alpha


def candidate_pairs(g, W, H):
    """All (Gaussian, pixel) pairs with the pixel inside the Gaussian's integer
    bounding square |p - m|_inf <= rho.  Since rho >= 3 sqrt(lambda_max), every
    pixel with q <= 9 is inside it, so the square is a superset of the ellipse."""
    gis, pxs, pys = [], [], []
    valid = g["valid"]
    for R in np.unique(g["rho"][valid]):
        sel = np.nonzero(valid & (g["rho"] == R))[0]
        R = int(R)
        x0 = np.ceil(g["mx"][sel] - R).astype(np.int64)
        x1 = np.floor(g["mx"][sel] + R).astype(np.int64)
        y0 = np.ceil(g["my"][sel] - R).astype(np.int64)
        y1 = np.floor(g["my"][sel] + R).astype(np.int64)
        for oy in range(2 * R + 2):
            py = y0 + oy
            rowok = (py <= y1) & (py >= 0) & (py < H)
            if not rowok.any():
                continue
            for ox in range(2 * R + 2):
                px = x0 + ox
                keep = rowok & (px <= x1) & (px >= 0) & (px < W)
                if keep.any():
                    gis.append(sel[keep])
                    pxs.append(px[keep])
                    pys.append(py[keep])
    if not gis:
        e = np.zeros(0, np.int64)
        return e, e, e
    return np.concatenate(gis), np.concatenate(pxs), np.concatenate(pys)


def contributor_pairs(g, W, H):
    """Pairs passing the contribution rule, sorted by (pixel, depth key, gid),
    plus per-pixel near-threshold flags."""
    gi, px, py = candidate_pairs(g, W, H)
    dx, dy, q, G, raw, alpha = _pair_eval(g, gi, px.astype(np.float64), py.astype(np.float64))
    pix = py * W + px
    near = (np.abs(q - Q_CUT) < FLAG_Q)
    keep = (q <= Q_CUT) & (alpha >= ALPHA_MIN)
    near |= keep & ((np.abs(alpha - ALPHA_MIN) < FLAG_ALPHA) | (np.abs(raw - ALPHA_MAX) < FLAG_CLAMP))
    flags = np.zeros(W * H, bool)
    flags[pix[near]] = True
    sel = np.nonzero(keep)[0]
    zbits = g["zkey"][gi[sel]].view(np.uint32)
    order = np.lexsort((g["gid"][gi[sel]], zbits, pix[sel]))
    sel = sel[order]
    P = dict(gi=gi[sel], pix=pix[sel], dx=dx[sel], dy=dy[sel], q=q[sel], G=G[sel],
             raw=raw[sel], alpha=alpha[sel])
    # depth keys that are bit-equal for different Gaussians of one pixel are
    # ordered by gid on both sides; nothing to flag.
    return P, flags


# ----------------------------------------------------------------------------
# compositing (front to back)
# ----------------------------------------------------------------------------
def composite(g, P, n_pix, flags=None):
    """Front-to-back compositing of sorted contributor pairs, one rank at a
    time across all pixels.  Returns per-pixel colour, depth, alpha, count and
    per-pair transmittance-before and contribution mask."""
    n = len(P["pix"])
    C = g["col"].shape[1]
    pix = P["pix"]
    starts = np.searchsorted(pix, np.arange(n_pix))
    counts = np.bincount(pix, minlength=n_pix)
    T = np.ones(n_pix)
    done = np.zeros(n_pix, bool)
    col = np.zeros((n_pix, C))
    dep = np.zeros(n_pix)
    cnt = np.zeros(n_pix, np.int64)
    Tb = np.zeros(n)
    con = np.zeros(n, bool)
    # conditioning of the transmittance product: a relative perturbation e of
    # alpha_i moves T after it by e * alpha_i / (1 - alpha_i) relatively, so
    # kappa sums that factor over the contributors composited so far (Kb:
    # before each pair, K: the pixel's total)
    K = np.zeros(n_pix)
    Kb = np.zeros(n)
    kmax = int(counts.max()) if n else 0
    for k in range(kmax):
        p = np.nonzero((counts > k) & ~done)[0]
        if len(p) == 0:
            break
        idx = starts[p] + k
        a = P["alpha"][idx]
        test = T[p] * (1.0 - a)
        if flags is not None:
            flags[p[np.abs(test - T_MIN) < FLAG_T]] = True
        stop = test < T_MIN
        done[p[stop]] = True
        p, idx, a, test = p[~stop], idx[~stop], a[~stop], test[~stop]
        Tb[idx] = T[p]
        Kb[idx] = K[p]
        con[idx] = True
        w = a * T[p]
        gi = P["gi"][idx]
        col[p] += w[:, None] * g["col"][gi]
        dep[p] += w * g["z"][gi]
        T[p] = test
        K[p] += a / (1.0 - a)
        cnt[p] += 1
    return dict(col=col, depth=dep, alpha=1.0 - T, T=T, n=cnt, Tb=Tb, con=con, Kb=Kb, K=K)


def render_job(kfs, view, kf_ids, channels="rgb"):
    """Culled oracle forward for one job.  Returns dict with ``rgb`` [C,H,W],
    ``depth`` [H,W], ``alpha`` [H,W], ``n`` [H,W], ``flags`` [H,W] and the
    internals the adjoint needs."""
    cam = view["cam"]
    H, W = cam["H"], cam["W"]
    g = gather_job(kfs, view, kf_ids, channels)
    P, flags = contributor_pairs(g, W, H)
    out = composite(g, P, H * W, flags)
    C = g["col"].shape[1]
    return dict(rgb=out["col"].T.reshape(C, H, W), depth=out["depth"].reshape(H, W),
                alpha=out["alpha"].reshape(H, W), n=out["n"].reshape(H, W),
                flags=flags.reshape(H, W), g=g, P=P, comp=out, H=H, W=W)


def render_window(kfs, view, kf_ids, win, channels="rgb"):
    """``render_job`` evaluated on the pixels of the window win = (x0, y0, x1,
    y1) (half-open) only: the job's Gaussians whose integer bounding square
    meets the window are the only ones that can reach its pixels, and their
    pairs with pixels outside it are dropped.  Pixel outputs inside the window
    equal render_job's; per-Gaussian gradients of ``backward_job`` on the
    result are complete for the Gaussians whose in-image square lies inside
    the window (``complete`` mask, aligned with the returned Gaussian set)."""
    cam = view["cam"]
    H, W = cam["H"], cam["W"]
    x0, y0, x1, y1 = win
    g = gather_job(kfs, view, kf_ids, channels)
    lo_x = np.maximum(np.ceil(g["mx"] - g["rho"]), 0)
    hi_x = np.minimum(np.floor(g["mx"] + g["rho"]), W - 1)
    lo_y = np.maximum(np.ceil(g["my"] - g["rho"]), 0)
    hi_y = np.minimum(np.floor(g["my"] + g["rho"]), H - 1)
    meets = g["valid"] & (hi_x >= x0) & (lo_x <= x1 - 1) & (hi_y >= y0) & (lo_y <= y1 - 1)
    idx = np.nonzero(meets)[0]
    sub = {k: g[k][idx] for k in GAUSS_KEYS}
    sub["col"] = g["col"][idx]
    sub["parts"] = g["parts"]
    sub["kf_ids"] = g["kf_ids"]
    P, flags = contributor_pairs(sub, W, H)
    px, py = P["pix"] % W, P["pix"] // W
    inside = (px >= x0) & (px < x1) & (py >= y0) & (py < y1)
    P = {k: v[inside] for k, v in P.items()}
    flags = flags.reshape(H, W)
    wmask = np.zeros((H, W), bool)
    wmask[y0:y1, x0:x1] = True
    flags &= wmask
    out = composite(sub, P, H * W, flags.ravel())
    flags = out_flags = flags.ravel()
    complete = (lo_x[idx] >= x0) & (hi_x[idx] <= x1 - 1) & (lo_y[idx] >= y0) & (hi_y[idx] <= y1 - 1)
    C = sub["col"].shape[1]
    return dict(rgb=out["col"].T.reshape(C, H, W), depth=out["depth"].reshape(H, W),
                alpha=out["alpha"].reshape(H, W), n=out["n"].reshape(H, W),
                flags=out_flags.reshape(H, W), window=wmask, g=sub, P=P, comp=out, H=H, W=W,
                complete=complete)


def render_bruteforce(kfs, view, kf_ids):
    """O(P*N) forward: every pixel tests every Gaussian of the job, no
    bounding square, then composites its sorted contributors in a Python loop."""
    cam = view["cam"]
    H, W = cam["H"], cam["W"]
    g = gather_job(kfs, view, kf_ids)
    M = len(g["gid"])
    rgb = np.zeros((3, H, W))
    dep = np.zeros((H, W))
    alp = np.zeros((H, W))
    cnt = np.zeros((H, W), np.int64)
    allg = np.nonzero(g["valid"])[0]
    for py in range(H):
        for px in range(W):
            dx, dy, q, G, raw, alpha = _pair_eval(g, allg, float(px), float(py))
            ok = (q <= Q_CUT) & (alpha >= ALPHA_MIN)
            js = allg[ok]
            al = alpha[ok]
            order = sorted(range(len(js)), key=lambda i: (int(g["zkey"][js[i]].view(np.uint32)),
                                                          int(g["gid"][js[i]])))
            T = 1.0
            c = np.zeros(3)
            dd = 0.0
            n = 0
            for i in order:
                a = al[i]
                if T * (1.0 - a) < T_MIN:
                    break
                c += a * T * g["col"][js[i]]
                dd += a * T * g["z"][js[i]]
                T *= 1.0 - a
                n += 1
            rgb[:, py, px] = c
            dep[py, px] = dd
            alp[py, px] = 1.0 - T
            cnt[py, px] = n
    assert M == len(g["gid"])
    return dict(rgb=rgb, depth=dep, alpha=alp, n=cnt)


def render(kfs, views, jobs, channels="rgb"):
    """Forward for a list of jobs ``(view_index, [kf indices])``."""
    return [render_job(kfs, views[v], ids, channels) for v, ids in jobs]


# ----------------------------------------------------------------------------
# adjoint
# ----------------------------------------------------------------------------
def _suffix_sums(P, comp, vals, n_pix):
    """For each contributing pair i of a pixel, sum over the later contributors
    k > i of the pixel of vals_k (vals: [n, K])."""
    pix = P["pix"]
    con = comp["con"]
    starts = np.searchsorted(pix, np.arange(n_pix))
    counts = np.bincount(pix, minlength=n_pix)
    S = np.zeros(vals.shape)
    acc = np.zeros((n_pix, vals.shape[1]))
    kmax = int(counts.max()) if len(pix) else 0
    for k in range(kmax - 1, -1, -1):
        p = np.nonzero(counts > k)[0]
        idx = starts[p] + k
        m = con[idx]
        p, idx = p[m], idx[m]
        S[idx] = acc[p]
        acc[p] += vals[idx]
    return S


def pair_grads(g, P, comp, g_col, g_dep, g_alp):
    """Per contributing pair: d loss / d (alpha, colour, z) and the derived
    geometric grads (m, conic, opacity).  g_col [n_pix, C], g_dep/g_alp [n_pix]."""
    n_pix = len(comp["T"])
    con = comp["con"]
    pix = P["pix"]
    gi = P["gi"]
    a = P["alpha"]
    Ti = comp["Tb"]
    w = np.where(con, a * Ti, 0.0)
    col = g["col"][gi]
    z = g["z"][gi]
    vals = np.concatenate([w[:, None] * col, (w * z)[:, None]], 1)
    S = _suffix_sums(P, comp, vals, n_pix)
    C = col.shape[1]
    gc = g_col[pix]
    gd = g_dep[pix]
    ga = g_alp[pix]
    Tf = comp["T"][pix]
    inv = 1.0 / (1.0 - a)
    galpha = (gc * (col * Ti[:, None] - S[:, :C] * inv[:, None])).sum(1) \
        + gd * (z * Ti - S[:, C] * inv) + ga * Tf * inv
    unclamped = P["raw"] < ALPHA_MAX
    g_o = np.where(unclamped, galpha * P["G"], 0.0)
    g_q = np.where(unclamped, -0.5 * a * galpha, 0.0)
    dx, dy = P["dx"], P["dy"]
    A, B, Cc = g["ca"][gi], g["cb"][gi], g["cc"][gi]
    out = dict(
        g_mx=g_q * (-2.0 * (A * dx + B * dy)),
        g_my=g_q * (-2.0 * (B * dx + Cc * dy)),
        g_a=g_q * dx * dx, g_b=g_q * 2.0 * dx * dy, g_c=g_q * dy * dy,
        g_o=g_o, g_col=gc * w[:, None], g_z=gd * w, galpha=galpha,
    )
    # the same terms with every product expanded to absolute values: bounds
    # the rounding error of any evaluation order (tolerances, not the value).
    # Each term is also scaled by its conditioning: a term carrying T before
    # pair k by 1 + kappa_k (the prefix conditioning of the transmittance
    # product, see composite), so the suffix sums take every later
    # contributor with its own factor; a term divided by 1 - alpha_j by
    # 1 + alpha_j / (1 - alpha_j); the final T by the pixel's total 1 + kappa.
    kb = 1.0 + comp["Kb"]
    ka = 1.0 + a / (1.0 - a)
    kt = 1.0 + comp["K"][pix]
    avals = np.concatenate([np.abs(w * kb)[:, None] * np.abs(col), np.abs(w * kb * z)[:, None]], 1)
    aS = _suffix_sums(P, comp, avals, n_pix)
    aal = (np.abs(gc) * (np.abs(col) * (Ti * kb)[:, None] + aS[:, :C] * (inv * ka)[:, None])).sum(1) \
        + np.abs(gd) * (np.abs(z) * Ti * kb + aS[:, C] * inv * ka) + np.abs(ga) * Tf * inv * ka * kt
    aq = np.where(unclamped, 0.5 * a * aal, 0.0)
    out.update(
        a_mx=aq * 2.0 * (np.abs(A * dx) + np.abs(B * dy)),
        a_my=aq * 2.0 * (np.abs(B * dx) + np.abs(Cc * dy)),
        a_a=aq * dx * dx, a_b=aq * 2.0 * np.abs(dx * dy), a_c=aq * dy * dy,
        a_o=np.where(unclamped, aal * P["G"], 0.0), a_col=np.abs(gc) * (w * kb)[:, None],
        a_z=np.abs(gd) * w * kb,
    )
    for k in list(out):
        v = out[k]
        out[k] = np.where(con[:, None], v, 0.0) if v.ndim == 2 else np.where(con, v, 0.0)
    return out


def geom_to_X_abs(g, idx, fx, fy, a_mx, a_my, a_a, a_b, a_c, a_z):
    """``geom_to_X`` with every factor replaced by its absolute value and every
    difference by a sum: a bound on the magnitudes the chain rule combines."""
    x, y, z = np.abs(g["x"][idx]), np.abs(g["y"][idx]), g["z"][idx]
    r = np.abs(g["r"][idx])
    s00, s01, s11 = g["s00"][idx], g["s01"][idx], g["s11"][idx]
    n = len(idx)
    det = s00 * s11 - s01 * s01
    Q = np.empty((n, 2, 2))
    Q[:, 0, 0] = s11 / det
    Q[:, 0, 1] = Q[:, 1, 0] = np.abs(s01) / det
    Q[:, 1, 1] = s00 / det
    Gm = np.empty((n, 2, 2))
    Gm[:, 0, 0] = a_a
    Gm[:, 0, 1] = Gm[:, 1, 0] = 0.5 * a_b
    Gm[:, 1, 1] = a_c
    GS = np.einsum("nij,njk,nkl->nil", Q, Gm, Q)
    a00, a01, a11 = GS[:, 0, 0], 2.0 * GS[:, 0, 1], GS[:, 1, 1]
    iz = 1.0 / z
    K00 = fx * fx * (iz * iz + x * x * iz ** 4)
    K01 = fx * fy * x * y * iz ** 4
    K11 = fy * fy * (iz * iz + y * y * iz ** 4)
    a_r = 2.0 * r * (a00 * K00 + a01 * K01 + a11 * K11)
    r2 = r * r
    ax = r2 * (a00 * 2.0 * fx * fx * x * iz ** 4 + a01 * fx * fy * y * iz ** 4)
    ay = r2 * (a01 * fx * fy * x * iz ** 4 + a11 * 2.0 * fy * fy * y * iz ** 4)
    az = r2 * (a00 * fx * fx * (2.0 * iz ** 3 + 4.0 * x * x * iz ** 5)
               + a01 * 4.0 * fx * fy * x * y * iz ** 5
               + a11 * fy * fy * (2.0 * iz ** 3 + 4.0 * y * y * iz ** 5))
    ax = ax + a_mx * fx * iz
    ay = ay + a_my * fy * iz
    az = az + a_mx * fx * x * iz * iz + a_my * fy * y * iz * iz + a_z
    return np.stack([ax, ay, az], 1), a_r


def geom_to_X(g, idx, fx, fy, g_mx, g_my, g_a, g_b, g_c, g_z):
    """Chain rule from (m, conic, z) grads to the view-space centre X and the
    radius r for Gaussians ``idx`` seen by a view with focal lengths fx, fy
    (vectorised; grad arrays aligned with idx)."""
    x, y, z = g["x"][idx], g["y"][idx], g["z"][idx]
    r = g["r"][idx]
    s00, s01, s11 = g["s00"][idx], g["s01"][idx], g["s11"][idx]
    n = len(idx)
    # conic = Sigma2^-1: dL/dSigma = -Q G Q with G = [[g_a, g_b/2], [g_b/2, g_c]]
    det = s00 * s11 - s01 * s01
    Q = np.empty((n, 2, 2))
    Q[:, 0, 0] = s11 / det
    Q[:, 0, 1] = Q[:, 1, 0] = -s01 / det
    Q[:, 1, 1] = s00 / det
    Gm = np.empty((n, 2, 2))
    Gm[:, 0, 0] = g_a
    Gm[:, 0, 1] = Gm[:, 1, 0] = 0.5 * g_b
    Gm[:, 1, 1] = g_c
    GS = -np.einsum("nij,njk,nkl->nil", Q, Gm, Q)
    g_s00 = GS[:, 0, 0]
    g_s01 = GS[:, 0, 1] + GS[:, 1, 0]           # s01 fills both off-diagonal slots
    g_s11 = GS[:, 1, 1]
    # Sigma2 = r^2 K + LOWPASS I with K = J J^T
    iz = 1.0 / z
    K00 = fx * fx * (iz * iz + x * x * iz ** 4)
    K01 = fx * fy * x * y * iz ** 4
    K11 = fy * fy * (iz * iz + y * y * iz ** 4)
    g_r = 2.0 * r * (g_s00 * K00 + g_s01 * K01 + g_s11 * K11)
    r2 = r * r
    gx = r2 * (g_s00 * 2.0 * fx * fx * x * iz ** 4 + g_s01 * fx * fy * y * iz ** 4)
    gy = r2 * (g_s01 * fx * fy * x * iz ** 4 + g_s11 * 2.0 * fy * fy * y * iz ** 4)
    gz = r2 * (g_s00 * fx * fx * (-2.0 * iz ** 3 - 4.0 * x * x * iz ** 5)
               + g_s01 * (-4.0) * fx * fy * x * y * iz ** 5
               + g_s11 * fy * fy * (-2.0 * iz ** 3 - 4.0 * y * y * iz ** 5))
    # m = (fx x/z + cx, fy y/z + cy)
    gx = gx + g_mx * fx * iz
    gy = gy + g_my * fy * iz
    gz = gz - g_mx * fx * x * iz * iz - g_my * fy * y * iz * iz
    # depth channel accumulates z itself
    gz = gz + g_z
    return np.stack([gx, gy, gz], 1), g_r


def backward_job(kfs, view, fwd, g_rgb, g_depth, g_alpha):
    """Adjoint of one job.  Returns per-Gaussian grads (aligned with the job's
    gathered set) for colour, opacity, radius, offset, the 6-vector pose grad
    and absolute-term sums used for tolerances."""
    g, P, comp = fwd["g"], fwd["P"], fwd["comp"]
    fx, fy = _f(view["cam"]["fx"]), _f(view["cam"]["fy"])
    H, W = fwd["H"], fwd["W"]
    n_pix = H * W
    C = g["col"].shape[1]
    gc = np.asarray(g_rgb, np.float64).reshape(C, -1).T
    gd = np.asarray(g_depth, np.float64).ravel()
    ga = np.asarray(g_alpha, np.float64).ravel()
    pg = pair_grads(g, P, comp, gc, gd, ga)
    M = len(g["gid"])
    gi = P["gi"]

    def acc(v):
        return np.bincount(gi, weights=v, minlength=M)

    G = {k: acc(pg[k]) for k in ("g_mx", "g_my", "g_a", "g_b", "g_c", "g_o", "g_z")}
    G["g_col"] = np.stack([acc(pg["g_col"][:, c]) for c in range(C)], 1)
    A = {"g_" + k[2:]: acc(pg[k]) for k in ("a_mx", "a_my", "a_a", "a_b", "a_c", "a_o", "a_z")}
    A["g_col"] = np.stack([acc(pg["a_col"][:, c]) for c in range(C)], 1)

    idx = np.nonzero(g["valid"])[0]
    gX = np.zeros((M, 3))
    g_r = np.zeros(M)
    gX[idx], g_r[idx] = geom_to_X(g, idx, fx, fy, G["g_mx"][idx], G["g_my"][idx], G["g_a"][idx],
                                  G["g_b"][idx], G["g_c"][idx], G["g_z"][idx])
    # absolute bound: the absolute terms through the chain with |factors|
    aX = np.zeros((M, 3))
    a_r = np.zeros(M)
    if len(idx):
        aX[idx], a_r[idx] = geom_to_X_abs(g, idx, fx, fy, A["g_mx"][idx], A["g_my"][idx], A["g_a"][idx],
                                          A["g_b"][idx], A["g_c"][idx], A["g_z"][idx])
    # X = R_rel (d * ray) + t_rel: dL/dd = (R^T gX) . ray, then |D + delta|
    ray = np.stack([g["xn"], g["yn"], np.ones(M)], 1)
    Rall = np.stack([p["R"] for p in g["parts"]], 0)[g["part"]]
    gXf = np.einsum("nji,nj->ni", Rall, gX)            # R^T gX
    g_d = (gXf * ray).sum(1)
    g_off = g_d * g["sgn"]
    aXf = np.einsum("nji,nj->ni", np.abs(Rall), aX)
    a_off = (aXf * np.abs(ray)).sum(1)
    # pose: dL/dxi = (gX, X x gX) per Gaussian, summed
    X = np.stack([g["x"], g["y"], g["z"]], 1)
    per = np.concatenate([gX, np.cross(X, gX)], 1)
    per[~g["valid"]] = 0.0
    aper = np.concatenate([aX, np.abs(X[:, [1, 2, 0]]) * aX[:, [2, 0, 1]]
                           + np.abs(X[:, [2, 0, 1]]) * aX[:, [1, 2, 0]]], 1)
    aper[~g["valid"]] = 0.0
    return dict(d_rgb=G["g_col"], d_opacity=G["g_o"], d_radius=g_r, d_offset=g_off,
                d_pose=per.sum(0), a_rgb=A["g_col"], a_opacity=A["g_o"], a_radius=a_r,
                a_offset=a_off, a_pose=aper.sum(0), gX=gX, kf=g["kf"], gid=g["gid"],
                pairs=pg)


def render_backward(kfs, views, jobs, fwds, g_rgb, g_depth, g_alpha, learnable=None):
    """Adjoint over a list of jobs.  Gradients of keyframe parameters are summed
    over jobs (``+=`` semantics); the pose gradient is one 6-vector per job.
    ``learnable``: set of keyframe indices whose grads are produced (others 0).
    """
    out = []
    for f, kf in enumerate(kfs):
        H, W = kf["cam"]["H"], kf["cam"]["W"]
        out.append(dict(d_rgb=np.zeros((3, H, W)), d_opacity=np.zeros((H, W)),
                        d_radius=np.zeros((H, W)), d_offset=np.zeros((H, W)),
                        a_rgb=np.zeros((3, H, W)), a_opacity=np.zeros((H, W)),
                        a_radius=np.zeros((H, W)), a_offset=np.zeros((H, W))))
    d_pose, a_pose = [], []
    for j, (v, ids) in enumerate(jobs):
        b = backward_job(kfs, views[v], fwds[j], g_rgb[j], g_depth[j], g_alpha[j])
        g = fwds[j]["g"]
        for part_i, f in enumerate(ids):
            if learnable is not None and f not in learnable:
                continue
            sl = slice(part_i * g["parts"][part_i]["N"], (part_i + 1) * g["parts"][part_i]["N"])
            H, W = kfs[f]["cam"]["H"], kfs[f]["cam"]["W"]
            o = out[f]
            o["d_rgb"] += b["d_rgb"][sl].T.reshape(3, H, W)
            o["d_opacity"] += b["d_opacity"][sl].reshape(H, W)
            o["d_radius"] += b["d_radius"][sl].reshape(H, W)
            o["d_offset"] += b["d_offset"][sl].reshape(H, W)
            o["a_rgb"] += b["a_rgb"][sl].T.reshape(3, H, W)
            o["a_opacity"] += b["a_opacity"][sl].reshape(H, W)
            o["a_radius"] += b["a_radius"][sl].reshape(H, W)
            o["a_offset"] += b["a_offset"][sl].reshape(H, W)
        d_pose.append(b["d_pose"])
        a_pose.append(b["a_pose"])
    return dict(kf=out, d_pose=np.array(d_pose), a_pose=np.array(a_pose))


# ----------------------------------------------------------------------------
# binning contract
# ----------------------------------------------------------------------------
def tile_rects(g, W, H, TW, TH):
    """Tile rectangle [x0, x1) x [y0, y1) of every Gaussian (FP64 decision):
    x0 = max(0, floor((mx - rho) / TW)), x1 = min(ntx, floor((mx + rho) / TW) + 1),
    same for y; culled Gaussians cover nothing."""
    ntx = -(-W // TW)
    nty = -(-H // TH)
    mx, my, rho = g["mx"], g["my"], g["rho"]
    x0 = np.maximum(0, np.floor((mx - rho) / TW)).astype(np.int64)
    x1 = np.minimum(ntx, np.floor((mx + rho) / TW) + 1).astype(np.int64)
    y0 = np.maximum(0, np.floor((my - rho) / TH)).astype(np.int64)
    y1 = np.minimum(nty, np.floor((my + rho) / TH) + 1).astype(np.int64)
    x1 = np.maximum(x1, x0)
    y1 = np.maximum(y1, y0)
    cull = ~g["valid"]
    x1[cull] = x0[cull]
    y1[cull] = y0[cull]
    return x0, x1, y0, y1, ntx, nty


def bin_and_sort(g, W, H, TW, TH):
    """Instance list of one job: one (tile, depth-key bits, gid) per overlapped
    tile, sorted lexicographically; returns tile ids, keys, gids and per-tile
    [start, end) ranges."""
    x0, x1, y0, y1, ntx, nty = tile_rects(g, W, H, TW, TH)
    tiles, zb, gids = [], [], []
    zbits = g["zkey"].view(np.uint32).astype(np.uint64)
    cnt = (x1 - x0) * (y1 - y0)
    for R in np.unique(cnt):
        if R == 0:
            continue
        sel = np.nonzero(cnt == R)[0]
        w = (x1 - x0)[sel]
        for k in range(int(R)):
            tx = x0[sel] + k % w
            ty = y0[sel] + k // w
            tiles.append(ty * ntx + tx)
            zb.append(zbits[sel])
            gids.append(g["gid"][sel])
    if tiles:
        tiles = np.concatenate(tiles)
        zb = np.concatenate(zb)
        gids = np.concatenate(gids).astype(np.uint64)
    else:
        tiles = zb = gids = np.zeros(0, np.uint64)
    order = np.lexsort((gids, zb, tiles))
    tiles, zb, gids = tiles[order], zb[order], gids[order]
    nt = ntx * nty
    ranges = np.stack([np.searchsorted(tiles, np.arange(nt), "left"),
                       np.searchsorted(tiles, np.arange(nt), "right")], 1)
    return dict(tile=tiles.astype(np.int64), zbits=zb.astype(np.uint32),
                gid=gids.astype(np.int64), ranges=ranges, ntx=ntx, nty=nty)


def render_tiled(kfs, view, kf_ids, TW, TH):
    """Forward through the binning contract: each pixel walks its tile's sorted
    instance list, applies the contribution rule and composites.  Equal to
    ``render_job`` for every tile shape when the bounding squares are
    conservative, which is what makes tiling a pure acceleration."""
    cam = view["cam"]
    H, W = cam["H"], cam["W"]
    g = gather_job(kfs, view, kf_ids)
    b = bin_and_sort(g, W, H, TW, TH)
    pos = {int(x): i for i, x in enumerate(g["gid"])}
    rgb = np.zeros((3, H, W))
    dep = np.zeros((H, W))
    T = np.ones((H, W))
    cnt = np.zeros((H, W), np.int64)
    for tile in range(b["ntx"] * b["nty"]):
        ty, tx = divmod(tile, b["ntx"])
        ys = np.arange(ty * TH, min(H, ty * TH + TH))
        xs = np.arange(tx * TW, min(W, tx * TW + TW))
        py, px = np.meshgrid(ys, xs, indexing="ij")
        py, px = py.ravel(), px.ravel()
        done = np.zeros(len(px), bool)
        Tt = np.ones(len(px))
        s, e = b["ranges"][tile]
        for k in range(s, e):
            gi = np.full(len(px), pos[int(b["gid"][k])])
            _, _, q, _, _, alpha = _pair_eval(g, gi, px.astype(np.float64), py.astype(np.float64))
            ok = (q <= Q_CUT) & (alpha >= ALPHA_MIN) & ~done
            test = Tt * (1.0 - alpha)
            stop = ok & (test < T_MIN)
            done |= stop
            ok &= ~stop
            w = np.where(ok, alpha * Tt, 0.0)
            rgb[:, py, px] += w * g["col"][gi].T
            dep[py, px] += w * g["z"][gi]
            cnt[py, px] += ok
            Tt = np.where(ok, test, Tt)
        T[py, px] = Tt
    return dict(rgb=rgb, depth=dep, alpha=1.0 - T, n=cnt, bins=b)
