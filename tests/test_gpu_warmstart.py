"""Learned offset warm start end to end at a reduced scale: offsets the
method converges to on synthetic frames train the conv net (1,000 frames,
half of the bench's); with its validation-selected offset step size,
warm-started mapping of an unseen 8-keyframe 640x480 window starts at a
lower loss and reaches the loss plain mapping (zero offsets, the
supplement's rates) has after 5 iterations in fewer iterations.  (Whether it
also reaches plain's 50-iteration loss sooner depends on the window: the
bench reports three seeds.)"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_warm_start_starts_lower_and_keeps_an_early_lead():
    import os

    import torch
    from paper_2603_21055_amd import sgad, warmstart
    print("warm start: 1000 frames", flush=True)
    # spawned workers: this process may already hold the GPU, so it must not fork
    frames = warmstart.make_frames(range(7000, 8000), workers=min(16, os.cpu_count() or 1), start="spawn")
    ctx = sgad.Context(0)
    try:
        res = warmstart.experiment(ctx, frames, epochs=20, map_iters=150, plain_iters=50,
                                   eval_seed=3001, eval_size=(640, 480), eval_n=8, log=print)
        plain, warm = np.array(res["plain_curve"]), np.array(res["warm_curve"])
        print("plain", plain[[0, 4, 9, 19, 49]], "warm", warm[[0, 4, 9, 19, 49]],
              "offset lr", res["warm_offset_lr"], "levels", res["warm_iters_to_plain_level"], flush=True)
        assert np.isfinite(plain).all() and np.isfinite(warm).all()
        assert res["train_loss"][-1] < res["train_loss"][0]
        assert warm[0] < 0.8 * plain[0]
        lvl = res["warm_iters_to_plain_level"]
        assert lvl["5"] is not None and lvl["5"] < 5
        torch.cuda.synchronize()
    finally:
        ctx.close()
