"""FP64 oracle: per-pixel depth-distribution tracking by Gauss-Newton.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The abstract models the depth around each pixel as a Gaussian distribution
and aligns every frame with those distributions; Sec. 3.3 attaches a Gaussian
to each back-projected point.  Specialised to one dimension along the ray:

* T1  The previous frame's geometry Gaussians are the pixel-aligned Gaussians
      of the splatting oracle (offset, radius D/fx, opacity 0.9) with a
      per-pixel depth standard deviation sigma_j.
* T2  They are rendered into the new view at pose T with sigma^2 as the only
      colour channel: per pixel A, D' and S = sum w sigma^2, so the predicted
      depth is mu = D'/A with variance s^2 = S/A.
* T3  A pixel is valid iff A >= A_VALID and D_obs > 0; r = (D_obs - mu)/s and
      the log-likelihood is sum_valid(-r^2/2 - ln s - ln(2 pi)/2).
* T4  J = dr/dxi = -(dD'/dxi - mu dA/dxi) / (A s), s held fixed.  The oracle
      forms dD'/dxi and dA/dxi per pixel as sums over its contributors of the
      exact per-pair partial derivatives (left twist on the view pose).
* T5  H = sum J^T J, g = sum J^T r, dxi = -H^-1 g by Cholesky (damped by
      DAMP * tr(H), growing x10, when H is not positive definite), then
      T <- Exp(dxi) T, for a fixed number of iterations.

``linearise`` also returns, per entry of H, g and the log-likelihood, the
sum of the absolute values of every term that forms it (aH, ag, aloglik)
and the absolute contribution of the pixels whose validity or contributor
set is decided within rounding of a threshold (fH, fg, floglik): the
elementwise parity bound of a lower-precision evaluation is built from them.
"""
from __future__ import annotations

import numpy as np

from . import se3, splat

A_VALID = 0.9
DAMP = 1e-9
FLAG_A = 1e-6   # |A - A_VALID| below which FP32 and FP64 may disagree on validity


def _pair_jacobians(g, P, fx, fy):
    """d alpha/d xi and d z/d xi for every contributor pair ([n, 6] each)."""
    gi = P["gi"]
    a = P["alpha"]
    dx, dy = P["dx"], P["dy"]
    A, B, C = g["ca"][gi], g["cb"][gi], g["cc"][gi]
    # dq/dX through the mean and the conic (g_q = 1)
    vX, _ = splat.geom_to_X(g, gi, fx, fy,
                            g_mx=-2.0 * (A * dx + B * dy), g_my=-2.0 * (B * dx + C * dy),
                            g_a=dx * dx, g_b=2.0 * dx * dy, g_c=dy * dy,
                            g_z=np.zeros(len(gi)))
    X = np.stack([g["x"][gi], g["y"][gi], g["z"][gi]], 1)
    dq = np.concatenate([vX, np.cross(X, vX)], 1)
    dadq = np.where(P["raw"] < splat.ALPHA_MAX, -0.5 * a, 0.0)
    dalpha = dadq[:, None] * dq
    ez = np.zeros_like(X)
    ez[:, 2] = 1.0
    dz = np.concatenate([ez, np.cross(X, ez)], 1)
    return dalpha, dz


def linearise(geo, cam, R, t, obs_depth):
    """Residuals, Jacobians and the normal equations at pose (R, t)."""
    view = dict(cam=cam, R=R, t=t)
    fwd = splat.render_job([geo], view, [0], channels="sigma2")
    g, P, comp = fwd["g"], fwd["P"], fwd["comp"]
    n_pix = cam["H"] * cam["W"]
    con = comp["con"]
    pix = P["pix"]
    a = P["alpha"]
    Ti = comp["Tb"]
    w = np.where(con, a * Ti, 0.0)
    z = g["z"][P["gi"]]
    S = splat._suffix_sums(P, comp, (w * z)[:, None], n_pix)[:, 0]
    fx, fy = splat._f(cam["fx"]), splat._f(cam["fy"])
    dalpha, dz = _pair_jacobians(g, P, fx, fy)
    inv = 1.0 / (1.0 - a)
    cD = np.where(con, z * Ti - S * inv, 0.0)
    cA = np.where(con, comp["T"][pix] * inv, 0.0)
    dD = np.zeros((n_pix, 6))
    dA = np.zeros((n_pix, 6))
    for k in range(6):
        dD[:, k] = np.bincount(pix, weights=cD * dalpha[:, k] + w * dz[:, k], minlength=n_pix)
        dA[:, k] = np.bincount(pix, weights=cA * dalpha[:, k], minlength=n_pix)
    Apix = comp["alpha"]
    Dp = comp["depth"]
    Ss = comp["col"][:, 0]
    obs = np.asarray(obs_depth, np.float64).ravel()
    valid = (Apix >= A_VALID) & (obs > 0)
    # every pixel with some coverage gets its residual and Jacobian, so the
    # pixels next to the validity threshold can be bounded below
    cov = (Apix > 0) & (Ss > 0) & (obs > 0)
    Av = np.where(cov, Apix, 1.0)
    mu = Dp / Av
    s = np.sqrt(np.where(cov, Ss / Av, 1.0))
    r_all = np.where(cov, (obs - mu) / s, 0.0)
    J_all = -(dD - mu[:, None] * dA) / (Av * s)[:, None]
    J_all[~cov] = 0.0
    r = np.where(valid, r_all, 0.0)
    J = np.where(valid[:, None], J_all, 0.0)
    Hm = J.T @ J
    gv = J.T @ r
    llp = -0.5 * r_all * r_all - np.log(s) - 0.5 * np.log(2 * np.pi)
    ll = float(np.sum(np.where(valid, llp, 0.0)))

    # Tolerance terms.  (1) Absolute-term sums: every product and difference
    # of the per-pair partials, the per-pixel sums and the normal-equation
    # sums taken with absolute values (a bound on the rounding error of any
    # evaluation order, in units of the working precision).
    aX, _ = splat.geom_to_X_abs(g, P["gi"], fx, fy,
                                a_mx=2.0 * (np.abs(g["ca"][P["gi"]] * P["dx"]) + np.abs(g["cb"][P["gi"]] * P["dy"])),
                                a_my=2.0 * (np.abs(g["cb"][P["gi"]] * P["dx"]) + np.abs(g["cc"][P["gi"]] * P["dy"])),
                                a_a=P["dx"] ** 2, a_b=2.0 * np.abs(P["dx"] * P["dy"]), a_c=P["dy"] ** 2,
                                a_z=np.zeros(len(P["gi"])))
    Xa = np.abs(np.stack([g["x"][P["gi"]], g["y"][P["gi"]], z], 1))
    adq = np.concatenate([aX, Xa[:, [1, 2, 0]] * aX[:, [2, 0, 1]] + Xa[:, [2, 0, 1]] * aX[:, [1, 2, 0]]], 1)
    adalpha = np.where(P["raw"] < splat.ALPHA_MAX, 0.5 * a, 0.0)[:, None] * adq
    adz = np.stack([np.zeros_like(z), np.zeros_like(z), np.ones_like(z), Xa[:, 1], Xa[:, 0],
                    np.zeros_like(z)], 1)
    acD = np.where(con, z * Ti + S * inv, 0.0)
    aD = np.zeros((n_pix, 6))
    aA = np.zeros((n_pix, 6))
    for k in range(6):
        aD[:, k] = np.bincount(pix, weights=acD * adalpha[:, k] + w * adz[:, k], minlength=n_pix)
        aA[:, k] = np.bincount(pix, weights=cA * adalpha[:, k], minlength=n_pix)
    aJ = np.where(cov[:, None], (aD + np.abs(mu)[:, None] * aA) / (Av * s)[:, None], 0.0)
    ar = np.where(cov, (np.abs(obs) + np.abs(mu)) / s, 0.0)
    Ja = np.abs(J_all)
    ra = np.abs(r_all)
    vm = valid[:, None].astype(np.float64)
    aH = (aJ * vm).T @ Ja + (Ja * vm).T @ aJ + (Ja * vm).T @ Ja
    ag = (aJ * vm).T @ ra + (Ja * vm).T @ ar + (Ja * vm).T @ ra
    all_ = float(np.sum(np.where(valid, 0.5 * r_all * r_all + np.abs(np.log(s)) + 0.5 * np.log(2 * np.pi)
                                 + ra * ar, 0.0)))
    # (2) Pixels whose validity or contributor set a rounding-level
    # difference can change (splat flags, or A within FLAG_A of A_VALID):
    # their whole absolute contribution.
    amb = (fwd["flags"].ravel() | (np.abs(Apix - A_VALID) < FLAG_A)) & cov
    am = amb[:, None].astype(np.float64)
    fH = (Ja * am).T @ Ja
    fg = (Ja * am).T @ ra
    fll = float(np.sum(np.where(amb, np.abs(llp), 0.0)))
    return dict(H=Hm, g=gv, loglik=ll, r=r, J=J, valid=valid, mu=mu, s=s, A=Apix,
                flags=fwd["flags"].ravel(), n_valid=int(valid.sum()), fwd=fwd,
                aH=aH, ag=ag, aloglik=all_, fH=fH, fg=fg, floglik=fll, n_ambiguous=int(amb.sum()))


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


def track_gn(geo, cam, R0, t0, obs_depth, iters=30):
    """Fixed-iteration Gauss-Newton from (R0, t0); returns the pose trace."""
    R = np.asarray(R0, np.float64)
    t = np.asarray(t0, np.float64)
    trace = []
    for _ in range(iters):
        lin = linearise(geo, cam, R, t, obs_depth)
        dxi, lam = solve(lin["H"], lin["g"])
        trace.append(dict(R=R.copy(), t=t.copy(), H=lin["H"], g=lin["g"], loglik=lin["loglik"],
                          dxi=dxi, lam=lam, n_valid=lin["n_valid"]))
        R, t = se3.left_update(R, t, dxi)
    return dict(R=R, t=t, trace=trace)
