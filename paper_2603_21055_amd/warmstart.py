"""Learned offset warm start: data from the method's own converged offsets,
training of the BF16 conv net, and the warm-vs-plain mapping comparison.

Training frames are 160x120 crops at the 640x480 focal length (fx = 600, so
one pixel covers the same angle as in the evaluation frames) of random box
rooms seen from random orientations; the keyframe depth carries N(0, 1 cm)
noise.  The target offsets are what plain mapping converges to: a fixed
number of mapping iterations of the keyframe (offsets from zero) against
noise-free ray-cast renders at its own view and two neighbours perturbed by
up to 2 cm / 1 degree.  The network sees (R, G, B, h) with h the noisy depth minus its
local 3x3 mean, in units of 2 cm.

Evaluation: an 8-keyframe 640x480 window with the same depth noise, every
view rendering all keyframes; plain mapping starts from zero offsets at the
supplement's learning rates, warm mapping from the network's prediction;
reported are the plain loss after `plain_iters` iterations and the first
iteration at which the warm run's loss is at or below it.

Adam moves every parameter by about its learning rate in its first steps
whatever the gradient, so the supplement's 1 cm offset step undoes a
prediction that is already closer than that.  The warm start therefore comes
with its own offset step size, a hyperparameter of the warm start chosen on
a validation window (a different seed from the evaluation window): the
candidate with the lowest loss after the selection horizon.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

from . import sgad, synth
from .mapping import Mapper
from .offsetnet import OffsetNet

DEPTH_NOISE = 0.01


def _rand_rot(rng, max_deg):
    from scipy.spatial.transform import Rotation
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    return Rotation.from_rotvec(v * np.deg2rad(rng.uniform(0, max_deg))).as_matrix()


def training_frame(seed: int, W: int = 160, H: int = 120, f: float = 600.0) -> dict:
    """One training frame (CPU, numpy): noisy keyframe and three targets."""
    rng = np.random.default_rng(seed)
    room = synth.make_room(rng)
    cam = dict(H=H, W=W, fx=f, fy=f, cx=W / 2.0, cy=H / 2.0)
    R, t = synth.pose_from_c2w(_rand_rot(rng, 60.0), rng.uniform(-0.3, 0.3, size=3))
    depth, rgb = room.raycast(cam, R, t)
    noisy = (depth + rng.normal(0.0, DEPTH_NOISE, size=depth.shape)).astype(np.float32)
    kf = synth.keyframe_from_frame(cam, R, t, noisy, rgb,
                                   rng.uniform(0.5, 1.0, size=(H, W)).astype(np.float32))
    views, targets = [dict(cam=dict(cam), R=R, t=t)], [dict(rgb=rgb, depth=depth)]
    for _ in range(2):
        Rv, tv = synth.perturb_pose(R, t, rng, 0.02, 1.0)
        d, c = room.raycast(cam, Rv, tv)
        views.append(dict(cam=dict(cam), R=Rv, t=tv))
        targets.append(dict(rgb=c, depth=d))
    return dict(kf=kf, views=views, targets=targets)


def _gen(args):
    return training_frame(*args)


def make_frames(seeds, workers: int = 8, start: str = "fork"):
    """Training frames on `workers` CPU processes; start="spawn" starts fresh
    interpreters (for a caller that has already opened the GPU, which must
    not fork)."""
    if workers <= 1:
        return [training_frame(s) for s in seeds]
    import multiprocessing
    with multiprocessing.get_context(start).Pool(workers) as p:
        return p.map(_gen, [(s,) for s in seeds])


def converged_offsets(ctx, frame, iters: int = 200, avg: int = 50):
    """Run plain mapping on one frame and return (rgb, noisy depth, offsets);
    the offsets are the mean of the last `avg` iterates (Adam keeps moving
    each parameter by about its learning rate, so single iterates jitter)."""
    import torch
    dev = ctx.device
    kf = sgad.to_device(frame["kf"], dev)
    t_rgb = torch.from_numpy(np.stack([t["rgb"] for t in frame["targets"]])).to(dev)
    t_dep = torch.from_numpy(np.stack([t["depth"] for t in frame["targets"]])).to(dev)
    jobs = [(v, [0]) for v in range(len(frame["views"]))]
    m = Mapper(ctx, [kf], frame["views"], jobs, [0], t_rgb, t_dep)
    acc = torch.zeros_like(kf["offset"])
    for i in range(iters):
        m.step()
        if i >= iters - avg:
            acc += kf["offset"]
    return kf["rgb"], kf["depth"], acc / float(min(avg, iters))


def train(ctx, data, epochs: int = 20, batch: int = 8, lr: float = 1e-3, seed: int = 0, log=None):
    net = OffsetNet(ctx, seed=seed)
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(data))
        losses = []
        for b0 in range(0, len(data), batch):
            losses.append(net.train_step([data[i] for i in order[b0:b0 + batch]], lr=lr))
        ep_loss = float(np.mean([l.mean().item() for l in losses]))
        hist.append(ep_loss)
        if log:
            log(f"epoch {ep}: L1 {ep_loss * 1e3:.3f} mm")
    return net, hist


def eval_window(seed: int = 3000, W: int = 640, H: int = 480, n: int = 8) -> dict:
    """8-keyframe window with noisy keyframe depth (CPU, numpy)."""
    sc = synth.room_window(seed, W=W, H=H, n=n)
    rng = np.random.default_rng(seed + 1)
    for kf in sc["kfs"]:
        kf["depth"] = (kf["depth"] + rng.normal(0.0, DEPTH_NOISE, size=kf["depth"].shape)).astype(np.float32)
        kf["radius"] = (kf["depth"] / np.float32(kf["cam"]["fx"])).astype(np.float32)
        kf["offset"] = np.zeros_like(kf["depth"])
    return sc


def mapping_curve(ctx, sc, net, iters: int, lr=None):
    """Loss after each of `iters` mapping iterations of the whole window; the
    offsets start at zero (net None) or at the network's prediction; lr:
    learning rates per parameter group (default: the supplement's)."""
    import torch
    dev = ctx.device
    kfs = [sgad.to_device(k, dev) for k in sc["kfs"]]
    if net is not None:
        for k in kfs:
            k["offset"].copy_(net.forward(k["rgb"], k["depth"]))
    n = len(kfs)
    t_rgb = torch.from_numpy(np.stack([t["rgb"] for t in sc["targets"]])).to(dev)
    t_dep = torch.from_numpy(np.stack([t["depth"] for t in sc["targets"]])).to(dev)
    jobs = [(v, list(range(n))) for v in range(n)]
    m = Mapper(ctx, kfs, sc["views"], jobs, list(range(n)), t_rgb, t_dep, lr=lr)
    curve = torch.zeros(iters, dtype=torch.float64, device=dev)
    for i in range(iters):
        m.step()
        curve[i] = m.loss.sum()
    torch.cuda.synchronize()
    return curve.cpu().numpy()


OFFSET_STEPS = (0.01, 0.005, 0.003, 0.002)   # candidate warm-start offset learning rates (m)


def select_offset_lr(ctx, net, seed=2990, size=(640, 480), n=4, iters=30, candidates=OFFSET_STEPS):
    """Offset learning rate of warm-started mapping: the candidate whose run
    on a validation window (seed `seed`, never the evaluation window) ends
    with the lowest loss after `iters` iterations.  Returns (lr, losses)."""
    from .mapping import LR
    sc = eval_window(seed, W=size[0], H=size[1], n=n)
    losses = {}
    for lr in candidates:
        losses[lr] = float(mapping_curve(ctx, sc, net, iters, lr=dict(LR, offset=lr))[-1])
    best = min(candidates, key=lambda c: losses[c])
    return best, losses


def iters_to_level(plain, warm, k):
    """First iteration (1-based) at which the warm curve is at or below the
    plain curve's loss after k iterations, or None."""
    hit = np.nonzero(warm <= plain[k - 1])[0]
    return int(hit[0]) + 1 if len(hit) else None


def experiment(ctx, frames, epochs=20, batch=8, map_iters=200, plain_iters=50, log=print,
               eval_seed=3000, eval_size=(640, 480), eval_n=8, select=True, other_seeds=()):
    """frames: from make_frames (generated before the device is opened, so the
    worker processes never inherit a device context)."""
    t0 = time.time()
    n_frames = len(frames)
    log(f"converging offsets ({map_iters} mapping iterations per frame)")
    data = []
    for i, fr in enumerate(frames):
        rgb, dep, off = converged_offsets(ctx, fr, map_iters)
        data.append((rgb, dep, off))
        if i % 100 == 99:
            log(f"  {i + 1} frames ({time.time() - t0:.0f} s)")
    log("training")
    net, hist = train(ctx, data, epochs=epochs, batch=batch, log=log)
    from .mapping import LR
    warm_lr = LR["offset"]
    sel = {}
    if select:
        warm_lr, sel = select_offset_lr(ctx, net)
        log(f"warm-start offset learning rate {warm_lr} (validation losses {sel})")
    log("evaluating")
    sc = eval_window(eval_seed, W=eval_size[0], H=eval_size[1], n=eval_n)
    plain = mapping_curve(ctx, sc, None, plain_iters)
    warm = mapping_curve(ctx, sc, net, plain_iters, lr=dict(LR, offset=warm_lr))
    # iterations the warm start needs to reach the loss plain mapping has after
    # k iterations, for several k
    levels = {str(k): iters_to_level(plain, warm, k) for k in (2, 5, 10, 20, plain_iters)}
    target = plain[-1]
    warm_iters = iters_to_level(plain, warm, plain_iters)
    # the same comparison on further evaluation windows (other seeds)
    others = {}
    for sd in other_seeds:
        sc2 = eval_window(sd, W=eval_size[0], H=eval_size[1], n=eval_n)
        p2 = mapping_curve(ctx, sc2, None, plain_iters)
        w2 = mapping_curve(ctx, sc2, net, plain_iters, lr=dict(LR, offset=warm_lr))
        others[str(sd)] = {str(k): iters_to_level(p2, w2, k) for k in (5, 10, 20, plain_iters)}
    return dict(plain_iters=plain_iters, plain_final_loss=float(target), warm_iters_to_plain_loss=warm_iters,
                warm_iters_to_plain_level=levels, plain_first_loss=float(plain[0]), warm_first_loss=float(warm[0]),
                warm_final_loss=float(warm[-1]), plain_curve=plain.tolist(), warm_curve=warm.tolist(),
                warm_offset_lr=warm_lr, offset_lr_validation={str(k): v for k, v in sel.items()},
                eval_seed=eval_seed, other_seeds=others,
                train_loss=hist, n_frames=n_frames, epochs=epochs, seconds=time.time() - t0)


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--map-iters", type=int, default=200)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", type=str, default=None)
    a = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    log(f"generating {a.frames} training frames")
    frames = make_frames(range(1000, 1000 + a.frames), a.workers)
    ctx = sgad.Context(0)
    res = experiment(ctx, frames, a.epochs, map_iters=a.map_iters, log=log)
    s = json.dumps({k: v for k, v in res.items() if not k.endswith("curve")})
    print(s, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f)


if __name__ == "__main__":
    main()
