"""Independent re-derivation of the splat forward in torch float64, differentiated
by autograd.  Used only to pin the oracle's hand-written adjoint on tiny scenes.

Written separately from ``oracle/splat.py``: the projection Jacobian is a
3x2 matrix product, the conic a matrix inverse, the pose a first-order left
twist X + rho + phi x X, and every pixel composites its contributors in a
Python loop.  Index sets (which pairs contribute) are decided without grad.
"""
import numpy as np
import torch


def render_torch(kfs, view, kf_ids, g_rgb, g_depth, g_alpha):
    dt = torch.float64
    cam = view["cam"]
    H, W = cam["H"], cam["W"]
    fx, fy = float(np.float32(cam["fx"])), float(np.float32(cam["fy"]))
    cx, cy = float(np.float32(cam["cx"])), float(np.float32(cam["cy"]))
    xi = torch.zeros(6, dtype=dt, requires_grad=True)
    Rv = torch.tensor(np.asarray(view["R"], np.float64), dtype=dt)
    tv = torch.tensor(np.asarray(view["t"], np.float64), dtype=dt)
    params, means, conics, zs, ops, cols, gids = [], [], [], [], [], [], []
    for f in kf_ids:
        kf = kfs[f]
        kc = kf["cam"]
        p = {k: torch.tensor(np.asarray(kf[k], np.float64), dtype=dt, requires_grad=True)
             for k in ("offset", "radius", "opacity", "rgb")}
        params.append(p)
        D = torch.tensor(np.asarray(kf["depth"], np.float64), dtype=dt)
        Rf = torch.tensor(np.asarray(kf["R"], np.float64), dtype=dt)
        tf = torch.tensor(np.asarray(kf["t"], np.float64), dtype=dt)
        Rr = Rv @ Rf.T
        tr = tv - Rr @ tf
        vv, uu = torch.meshgrid(torch.arange(kc["H"], dtype=dt), torch.arange(kc["W"], dtype=dt),
                                indexing="ij")
        ray = torch.stack([(uu - float(np.float32(kc["cx"]))) / float(np.float32(kc["fx"])),
                           (vv - float(np.float32(kc["cy"]))) / float(np.float32(kc["fy"])),
                           torch.ones_like(uu)], -1).reshape(-1, 3)
        d = torch.abs(D + p["offset"]).reshape(-1, 1)
        X = (d * ray) @ Rr.T + tr
        X = X + xi[:3] + torch.cross(xi[3:].expand_as(X), X, dim=1)
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        m = torch.stack([fx * x / z + cx, fy * y / z + cy], 1)
        J = torch.zeros(len(z), 2, 3, dtype=dt)
        J[:, 0, 0] = fx / z
        J[:, 0, 2] = -fx * x / z ** 2
        J[:, 1, 1] = fy / z
        J[:, 1, 2] = -fy * y / z ** 2
        r = p["radius"].reshape(-1)
        S = (r ** 2)[:, None, None] * (J @ J.transpose(1, 2)) + 0.3 * torch.eye(2, dtype=dt)
        means.append(m)
        conics.append(torch.linalg.inv(S))
        zs.append(z)
        ops.append(p["opacity"].reshape(-1))
        cols.append(p["rgb"].reshape(3, -1).T)
        N = kc["H"] * kc["W"]
        gids.append(np.arange(N) + f * N)
    m = torch.cat(means)
    Q = torch.cat(conics)
    z = torch.cat(zs)
    o = torch.cat(ops)
    c = torch.cat(cols)
    gid = np.concatenate(gids)
    zkey = z.detach().numpy().astype(np.float32).view(np.uint32)
    loss = torch.zeros((), dtype=dt)
    out_rgb = np.zeros((3, H, W))
    gr = torch.tensor(np.asarray(g_rgb, np.float64), dtype=dt)
    gd = torch.tensor(np.asarray(g_depth, np.float64), dtype=dt)
    ga = torch.tensor(np.asarray(g_alpha, np.float64), dtype=dt)
    for py in range(H):
        for px in range(W):
            pix = torch.tensor([px, py], dtype=dt)
            dd = pix - m
            q = torch.einsum("ni,nij,nj->n", dd, Q, dd)
            G = torch.exp(-0.5 * q)
            a = torch.clamp(o * G, max=0.99)
            with torch.no_grad():
                ok = ((q <= 9.0) & (a >= 1.0 / 255.0) & (z >= 0.2)).numpy()
            idx = [int(i) for i in np.nonzero(ok)[0]]
            idx.sort(key=lambda i: (int(zkey[i]), int(gid[i])))
            T = torch.ones((), dtype=dt)
            col = torch.zeros(3, dtype=dt)
            dep = torch.zeros((), dtype=dt)
            for i in idx:
                if float(T * (1 - a[i])) < 1e-4:
                    break
                col = col + a[i] * T * c[i]
                dep = dep + a[i] * T * z[i]
                T = T * (1 - a[i])
            out_rgb[:, py, px] = col.detach().numpy()
            loss = loss + (gr[:, py, px] * col).sum() + gd[py, px] * dep + ga[py, px] * (1 - T)
    loss.backward()
    grads = []
    for p in params:
        grads.append({k: (v.grad.numpy() if v.grad is not None else np.zeros(v.shape))
                      for k, v in p.items()})
    return dict(rgb=out_rgb, grad=grads, pose=xi.grad.numpy())
