"""Mapping driver: autograd wrapper and the per-iteration optimiser loop.

``SplatFn`` is a torch.autograd.Function around the library's forward and
adjoint; ``Mapper`` runs the paper's mapping iteration (Sec. 3.2, Eq. 1 with
its L1 colour, SSIM and masked L1 depth terms; supplement weights and
learning rates) entirely in library kernels: forward splat -> Eq. 1 loss and
upstream grads -> adjoint -> multi-tensor Adam.
"""
from __future__ import annotations

import numpy as np

from . import sgad

# supplement learning rates; radius steps as log r and opacity as logit o (the
# spaces these rates belong to in 3DGS), colour and offset linearly
LR = dict(rgb=0.0025, radius=0.005, opacity=0.05, offset=0.01)
W_RGB, W_SSIM, W_DEPTH = 0.8, 0.2, 1.0                           # Eq. 1 weights (supplement)
R_MIN = 1e-6


class SplatFn:
    """torch.autograd.Function factory bound to one sgad.Context.

    ``SplatFn(ctx, kfs, views, jobs, learnable)(*params)`` with params the
    flat list [offset, radius, opacity, rgb] per learnable keyframe (order of
    ``learnable``) plus one pose tensor of shape [n_jobs, 6] (zeros; its grad
    is the left-twist pose gradient).  Returns (rgb, depth, alpha)."""

    def __new__(cls, ctx, kfs, views, jobs, learnable):
        import torch

        learn = list(learnable)

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(fctx, *params):
                dev = ctx.device
                H, W = views[0]["cam"]["H"], views[0]["cam"]["W"]
                nj = len(jobs)
                kk = [dict(k) for k in kfs]
                for i, f in enumerate(learn):
                    kk[f]["offset"], kk[f]["radius"], kk[f]["opacity"], kk[f]["rgb"] = params[4 * i:4 * i + 4]
                rgb = torch.empty((nj, 3, H, W), device=dev)
                dep = torch.empty((nj, H, W), device=dev)
                alp = torch.empty((nj, H, W), device=dev)
                saved = ctx.render_fwd(kk, views, jobs, rgb, dep, alp)
                fctx.saved_handle = saved
                fctx.kk = kk
                return rgb, dep, alp

            @staticmethod
            def backward(fctx, g_rgb, g_dep, g_alp):
                dev = ctx.device
                grads = []
                for f, kf in enumerate(fctx.kk):
                    if f in learn:
                        Hk, Wk = kf["depth"].shape
                        grads.append(dict(d_rgb=torch.zeros((3, Hk, Wk), device=dev),
                                          d_opacity=torch.zeros((Hk, Wk), device=dev),
                                          d_radius=torch.zeros((Hk, Wk), device=dev),
                                          d_offset=torch.zeros((Hk, Wk), device=dev)))
                    else:
                        grads.append(None)
                d_pose = torch.zeros((len(jobs), 6), device=dev)
                ctx.render_bwd(fctx.saved_handle, g_rgb.contiguous(),
                               None if g_dep is None else g_dep.contiguous(),
                               None if g_alp is None else g_alp.contiguous(), grads, d_pose, learn)
                ctx.release(fctx.saved_handle)
                out = []
                for f in learn:
                    g = grads[f]
                    out += [g["d_offset"], g["d_radius"], g["d_opacity"], g["d_rgb"]]
                return tuple(out) + (d_pose,)

        return _Fn.apply


class Mapper:
    """Optimises the learnable keyframes of a window against target views.

    kfs: device keyframe dicts (their tensors are updated in place);
    views / jobs: as for sgad.Context.render_fwd; targets: per-job device
    tensors t_rgb [n_jobs, 3, H, W], t_depth [n_jobs, H, W]."""

    def __init__(self, ctx, kfs, views, jobs, learnable, t_rgb, t_depth, with_count=False, lr=None,
                 w_ssim=W_SSIM):
        """lr: learning rates per parameter group (default the supplement's)."""
        import torch
        self.w_ssim = float(w_ssim)
        self.ctx, self.kfs, self.views, self.jobs = ctx, kfs, views, jobs
        self.learn = list(learnable)
        self.t_rgb, self.t_depth = t_rgb, t_depth
        dev = ctx.device
        nj = len(jobs)
        H, W = views[0]["cam"]["H"], views[0]["cam"]["W"]
        self.rgb = torch.empty((nj, 3, H, W), device=dev)
        self.dep = torch.empty((nj, H, W), device=dev)
        self.alp = torch.empty((nj, H, W), device=dev)
        self.cnt = torch.empty((nj, H, W), device=dev, dtype=torch.int32) if with_count else None
        self.g_rgb = torch.empty_like(self.rgb)
        self.g_dep = torch.empty_like(self.dep)
        self.loss = torch.zeros(nj, device=dev, dtype=torch.float64)
        self.grads, self.groups = [], []
        for f, kf in enumerate(kfs):
            if f not in self.learn:
                self.grads.append(None)
                continue
            g = dict(d_rgb=torch.zeros_like(kf["rgb"]), d_opacity=torch.zeros_like(kf["opacity"]),
                     d_radius=torch.zeros_like(kf["radius"]), d_offset=torch.zeros_like(kf["offset"]))
            self.grads.append(g)
            for name, gk, lo, hi, sp in (("rgb", "d_rgb", -np.inf, np.inf, sgad.SPACE_LINEAR),
                                         ("opacity", "d_opacity", 0.0, 1.0, sgad.SPACE_LOGIT),
                                         ("radius", "d_radius", R_MIN, np.inf, sgad.SPACE_LOG),
                                         ("offset", "d_offset", -np.inf, np.inf, sgad.SPACE_LINEAR)):
                p = kf[name]
                rate = (lr or LR)[name]
                self.groups.append((p, g[gk], torch.zeros_like(p), torch.zeros_like(p), rate, lo, hi, sp))
        self.t = 0
        self.graph = None

    def step(self):
        """One mapping iteration; returns nothing (loss stays on the device)."""
        c = self.ctx
        saved = c.render_fwd(self.kfs, self.views, self.jobs, self.rgb, self.dep, self.alp, self.cnt)
        c.eq1_loss(self.rgb, self.dep, self.t_rgb, self.t_depth, self.g_rgb, self.g_dep, self.loss,
                   W_RGB, self.w_ssim, W_DEPTH)
        c.render_bwd(saved, self.g_rgb, self.g_dep, None, self.grads, None, self.learn)
        c.release(saved)
        self.t += 1
        c.adam_step(self.groups, self.t)

    def capture(self):
        """Record one mapping iteration as a graph (after at least one eager
        step, which sizes the workspace); later iterations are replay()."""
        if self.graph is not None:
            return
        c = self.ctx
        c.graph_begin()
        try:
            self.step()          # recorded, not run
        finally:
            g = c.graph_end()
        self.t -= 1
        self.graph = g

    def replay(self):
        """One mapping iteration by replaying the captured graph."""
        self.ctx.graph_launch(self.graph)
        self.t += 1

    def release_graph(self):
        if self.graph is not None:
            self.ctx.graph_destroy(self.graph)
            self.graph = None

    def loss_value(self) -> float:
        return float(self.loss.sum().item())
