"""Offset warm-start network: delta0 = Net(R, G, B, h), h the high-passed depth.

Six 3x3 convolutions 4 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1 with ReLU after the
first five, BF16 MFMA with FP32 accumulation, all in the HIP library; this
module only holds the tensors and sequences the calls.  The paper starts the
offsets at zero (Sec. 3.2); the zero start stays the fallback.
"""
from __future__ import annotations

import numpy as np

from . import sgad

CHANNELS = [4, 32, 32, 32, 32, 32, 1]


def init_params(seed: int = 0):
    """He-uniform weights [3][3][cout][cin] and zero biases; the last layer is
    scaled by 0.1 so the untrained net predicts offsets near zero."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(6):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        lim = np.sqrt(6.0 / (9 * cin))
        w = rng.uniform(-lim, lim, size=(3, 3, cout, cin))
        if l == 5:
            w *= 0.1
        out.append((w.astype(np.float32), np.zeros(cout, np.float32)))
    return out


class OffsetNet:
    def __init__(self, ctx: "sgad.Context", params=None, seed: int = 0):
        import torch
        self.ctx = ctx
        dev = ctx.device
        params = params if params is not None else init_params(seed)
        self.w32, self.b32, self.w16, self.wt16 = [], [], [], []
        self.dw, self.db, self.state = [], [], []
        for l, (w, b) in enumerate(params):
            cin, cout = CHANNELS[l], CHANNELS[l + 1]
            w9 = torch.from_numpy(np.ascontiguousarray(np.asarray(w, np.float32).reshape(9, cout, cin))).to(dev)
            self.w32.append(w9)
            self.b32.append(torch.from_numpy(np.asarray(b, np.float32).copy()).to(dev))
            self.w16.append(torch.empty((9, cout, cin), dtype=torch.bfloat16, device=dev))
            self.wt16.append(torch.empty((9, cin, cout), dtype=torch.bfloat16, device=dev))
            self.dw.append(torch.zeros_like(w9))
            self.db.append(torch.zeros_like(self.b32[-1]))
            self.state.append([torch.zeros_like(w9), torch.zeros_like(w9),
                               torch.zeros_like(self.b32[-1]), torch.zeros_like(self.b32[-1])])
        self.t = 0
        self.refresh()

    def refresh(self):
        """Rebuild the bf16 (and transposed) weight copies from the FP32 masters."""
        for l in range(6):
            self.ctx.conv_weights(CHANNELS[l], CHANNELS[l + 1], self.w32[l], self.w16[l], self.wt16[l])

    def params_numpy(self):
        out = []
        for l in range(6):
            cin, cout = CHANNELS[l], CHANNELS[l + 1]
            out.append((self.w32[l].cpu().numpy().reshape(3, 3, cout, cin), self.b32[l].cpu().numpy()))
        return out

    def forward(self, rgb, depth):
        """rgb [3, H, W], depth [H, W] (float32 device) -> delta0 [H, W]."""
        import torch
        H, W = depth.shape
        dev = self.ctx.device
        x = torch.empty((H, W, 4), dtype=torch.bfloat16, device=dev)
        self.ctx.net_input(H, W, rgb, depth, x)
        self.acts = [x]
        for l in range(5):
            y = torch.empty((H, W, CHANNELS[l + 1]), dtype=torch.bfloat16, device=dev)
            self.ctx.conv_fwd(H, W, CHANNELS[l], CHANNELS[l + 1], 0, self.acts[-1], self.w16[l], self.b32[l], y)
            self.acts.append(y)
        delta = torch.empty((H, W), dtype=torch.float32, device=dev)
        self.ctx.conv_fwd(H, W, 32, 1, 1, self.acts[-1], self.w16[5], self.b32[5], delta)
        return delta

    def backward(self, dpre):
        """dpre: bf16 [H, W] gradient of the output; accumulates dw / db."""
        import torch
        H, W = dpre.shape[:2]
        dy = dpre
        for l in range(5, -1, -1):
            cin, cout = CHANNELS[l], CHANNELS[l + 1]
            self.ctx.conv_wgrad(H, W, cin, cout, self.acts[l], dy, self.dw[l], self.db[l])
            if l > 0:
                dx = torch.empty((H, W, cin), dtype=torch.bfloat16, device=self.ctx.device)
                self.ctx.conv_dgrad(H, W, cin, cout, dy, self.wt16[l], self.acts[l], dx)
                dy = dx

    def train_step(self, batch, lr=1e-3):
        """One Adam step on a batch of (rgb, depth, target) device tensors; the
        loss (mean over the batch) stays on the device and is returned."""
        import torch
        dev = self.ctx.device
        losses = torch.zeros(len(batch), dtype=torch.float64, device=dev)
        for i, (rgb, depth, target) in enumerate(batch):
            delta = self.forward(rgb, depth)
            g = torch.empty(delta.shape, dtype=torch.bfloat16, device=dev)
            self.ctx.offset_l1(delta, target, g, losses[i:i + 1])
            self.backward(g)
        self.t += 1
        groups = []
        for l in range(6):
            m, v, mb, vb = self.state[l]
            groups.append((self.w32[l], self.dw[l], m, v, lr, -1e30, 1e30))
            groups.append((self.b32[l], self.db[l], mb, vb, lr, -1e30, 1e30))
        self.ctx.adam_step(groups, self.t)
        self.refresh()
        return losses
