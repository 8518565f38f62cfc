"""Learned offset warm start end to end at a small scale: offsets the method
converges to on synthetic frames train the conv net, whose prediction must
start mapping of an unseen window at a lower loss than zero offsets."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_warm_start_lowers_the_first_mapping_loss():
    import torch
    from paper_2603_21055_amd import sgad, warmstart
    print("warm start: 48 frames", flush=True)
    frames = warmstart.make_frames(range(7000, 7048), workers=1)   # no fork of a process using the GPU
    ctx = sgad.Context(0)
    try:
        data = [warmstart.converged_offsets(ctx, fr, iters=120, avg=40) for fr in frames]
        net, hist = warmstart.train(ctx, data, epochs=12, batch=8)
        assert hist[-1] < hist[0]
        sc = warmstart.eval_window(3001, W=640, H=480, n=2)
        plain = warmstart.mapping_curve(ctx, sc, None, 3)
        warm = warmstart.mapping_curve(ctx, sc, net, 3)
        print("plain", plain, "warm", warm, flush=True)
        assert np.isfinite(plain).all() and np.isfinite(warm).all()
        assert warm[0] < plain[0]
        torch.cuda.synchronize()
    finally:
        ctx.close()
