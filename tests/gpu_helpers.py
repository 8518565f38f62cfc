"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
on a synthetic scene and compare with the FP64 oracle."""
import numpy as np

from oracle import splat


def device():
    import torch
    return torch.device("cuda", 0)


def upload(scene_kfs, dev):
    from paper_2603_21055_amd import sgad
    return [sgad.to_device(kf, dev) for kf in scene_kfs]


def gpu_render(ctx, kfs_d, views, jobs, with_count=True):
    import torch
    dev = ctx.device
    nj = len(jobs)
    H, W = views[0]["cam"]["H"], views[0]["cam"]["W"]
    rgb = torch.empty((nj, 3, H, W), device=dev)
    dep = torch.empty((nj, H, W), device=dev)
    alp = torch.empty((nj, H, W), device=dev)
    cnt = torch.empty((nj, H, W), device=dev, dtype=torch.int32) if with_count else None
    saved = ctx.render_fwd(kfs_d, views, jobs, rgb, dep, alp, cnt)
    return saved, dict(rgb=rgb, depth=dep, alpha=alp, count=cnt)


def gpu_backward(ctx, saved, kfs_d, g_rgb, g_depth, g_alpha, n_jobs, learnable):
    import torch
    dev = ctx.device
    grads = []
    for f, kf in enumerate(kfs_d):
        H, W = kf["depth"].shape
        grads.append(dict(d_rgb=torch.zeros((3, H, W), device=dev), d_opacity=torch.zeros((H, W), device=dev),
                          d_radius=torch.zeros((H, W), device=dev), d_offset=torch.zeros((H, W), device=dev)))
    d_pose = torch.zeros((n_jobs, 6), device=dev)
    ctx.render_bwd(saved, g_rgb, g_depth, g_alpha, grads, d_pose, learnable)
    return grads, d_pose


def rel_err(gpu, orc, mask=None):
    """max |gpu - orc| over the unmasked entries / max(|orc|_inf, 1e-6)."""
    gpu = np.asarray(gpu, np.float64)
    orc = np.asarray(orc, np.float64)
    if mask is not None:
        gpu, orc = gpu[mask], orc[mask]
    if orc.size == 0:
        return 0.0
    return float(np.abs(gpu - orc).max() / max(np.abs(orc).max(), 1e-6))


def assert_forward_parity(out, orc_jobs, tol=1e-5, max_flag_frac=2e-3):
    """Values within tol (per channel, relative to the channel max) on pixels
    the oracle does not flag as threshold-ambiguous; counts bit-exact there."""
    for j, o in enumerate(orc_jobs):
        ok = ~o["flags"]
        assert o["flags"].mean() <= max_flag_frac, o["flags"].mean()
        g_rgb = out["rgb"][j].cpu().numpy()
        for c in range(3):
            e = rel_err(g_rgb[c], o["rgb"][c], ok)
            assert e <= tol, ("rgb", j, c, e)
        e = rel_err(out["depth"][j].cpu().numpy(), o["depth"], ok)
        assert e <= tol, ("depth", j, e)
        e = rel_err(out["alpha"][j].cpu().numpy(), o["alpha"], ok)
        assert e <= tol, ("alpha", j, e)
        if out.get("count") is not None:
            cnt = out["count"][j].cpu().numpy()
            assert (cnt[ok] == o["n"][ok]).all(), ("count", j, int((cnt[ok] != o["n"][ok]).sum()))


def flagged_gaussians(orc_job):
    """Gaussians (as (kf, pixel) pairs) with a candidate pair at a flagged pixel."""
    g = orc_job["g"]
    W = orc_job["W"]
    gi, px, py = splat.candidate_pairs(g, W, orc_job["H"])
    bad = orc_job["flags"].ravel()[py * W + px]
    sel = np.unique(gi[bad])
    N = orc_job["g"]["parts"][0]["N"]
    return set(zip((g["gid"][sel] // N).tolist(), (g["gid"][sel] % N).tolist()))


def assert_grad_parity(gpu_grads, gpu_pose, orc_b, orc_jobs, learnable, rtol=1e-3, atol_rel=1e-5):
    """|g - o| <= rtol |o| + atol_rel * A elementwise, A the oracle's sum of
    absolute terms; Gaussians next to flagged pixels are excluded."""
    bad = set()
    for o in orc_jobs:
        bad |= flagged_gaussians(o)
    for f, gg in enumerate(gpu_grads):
        ob = orc_b["kf"][f]
        H, W = ob["d_offset"].shape
        mask = np.ones(H * W, bool)
        for (kf, pix) in bad:
            if kf == f:
                mask[pix] = False
        mask = mask.reshape(H, W)
        for name, gk, ak in (("offset", "d_offset", "a_offset"), ("radius", "d_radius", "a_radius"),
                             ("opacity", "d_opacity", "a_opacity")):
            g = gg[gk].cpu().numpy().astype(np.float64)
            o = ob[gk]
            a = ob[ak]
            if f not in learnable:
                assert np.abs(g).max() == 0.0
                continue
            err = np.abs(g - o) - (rtol * np.abs(o) + atol_rel * a)
            assert (err[mask] <= 0).all(), (name, f, float(err[mask].max()), int((err[mask] > 0).sum()))
        g = gg["d_rgb"].cpu().numpy().astype(np.float64)
        if f in learnable:
            err = np.abs(g - ob["d_rgb"]) - (rtol * np.abs(ob["d_rgb"]) + atol_rel * ob["a_rgb"])
            assert (err[:, mask] <= 0).all(), ("rgb", f, float(err[:, mask].max()))
    p = gpu_pose.cpu().numpy().astype(np.float64)
    err = np.abs(p - orc_b["d_pose"]) - (rtol * np.abs(orc_b["d_pose"]) + atol_rel * orc_b["a_pose"])
    assert (err <= 0).all(), ("pose", p, orc_b["d_pose"], orc_b["a_pose"])
