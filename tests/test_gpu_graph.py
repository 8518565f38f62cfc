"""Graph capture of a mapping iteration (sgad_graph_*): replays against the
eager path.  Each replay is checked after eager work and a synchronisation,
so a replay that drifted from the captured state would show."""
import numpy as np
import pytest

from paper_2603_21055_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2603_21055_amd import sgad
    assert torch.cuda.is_available()
    c = sgad.Context(0)
    yield c
    c.close()


def _mapper(ctx, seed=31, lr=None):
    import torch
    from paper_2603_21055_amd import sgad
    from paper_2603_21055_amd.mapping import Mapper
    sc = synth.small_scene(seed, 64, 48, n_kf=2, n_views=2, offset_amp=0.02, max_trans=0.03, max_rot=2)
    dev = ctx.device
    kfs = [sgad.to_device(k, dev) for k in sc["kfs"]]
    jobs = [(0, [0, 1]), (1, [0, 1])]
    t_rgb = torch.from_numpy(np.stack([t["rgb"] for t in sc["targets"]])).to(dev)
    t_dep = torch.from_numpy(np.stack([t["depth"] for t in sc["targets"]])).to(dev)
    return Mapper(ctx, kfs, sc["views"], jobs, [0, 1], t_rgb, t_dep, with_count=True, lr=lr), kfs


def test_replays_of_a_frozen_step_equal_the_eager_step(ctx):
    """Learning rates 0: every iteration renders the same parameters, so each
    replay's forward must equal the eager one bit for bit."""
    import torch
    print("graph: frozen step", flush=True)
    from paper_2603_21055_amd import sgad
    m, _ = _mapper(ctx, lr=dict(rgb=0.0, radius=0.0, opacity=0.0, offset=0.0))
    # linear parameter spaces: with a zero rate the update is the identity
    # (the log / logit round trips of radius and opacity are not)
    m.groups = [gr[:7] + (sgad.SPACE_LINEAR,) for gr in m.groups]
    m.step()
    torch.cuda.synchronize()
    rgb0, dep0, cnt0 = m.rgb.clone(), m.dep.clone(), m.cnt.clone()
    loss0 = m.loss.clone()
    m.capture()
    try:
        for i in range(4):
            m.replay()
            torch.cuda.synchronize()
            assert torch.equal(m.rgb, rgb0) and torch.equal(m.dep, dep0) and torch.equal(m.cnt, cnt0), i
            assert torch.allclose(m.loss, loss0, rtol=1e-12, atol=0.0), (i, m.loss, loss0)
            # eager work and a synchronisation between replays
            x = torch.arange(4096, device=ctx.device, dtype=torch.float32)
            assert float((x * 2).sum().item()) == 4095 * 4096
            ctx.sync()
    finally:
        m.release_graph()


def test_replayed_iterations_follow_the_eager_ones(ctx):
    """Adam's step count advances per replay: four replays after one eager
    step track five eager steps (same losses, same parameters up to the order
    of floating-point atomics)."""
    import torch
    print("graph: adam steps", flush=True)
    a, kfa = _mapper(ctx)
    b, kfb = _mapper(ctx)
    la, lb = [], []
    for _ in range(5):
        a.step()
        la.append(a.loss.sum().item())
    b.step()
    lb.append(b.loss.sum().item())
    b.capture()
    try:
        for _ in range(4):
            b.replay()
            lb.append(b.loss.sum().item())
            ctx.sync()
    finally:
        b.release_graph()
    print("eager", la, "graph", lb, flush=True)
    np.testing.assert_allclose(lb, la, rtol=1e-4)
    assert la[-1] < la[0]
    for f in range(2):
        for name in ("offset", "radius", "opacity", "rgb"):
            pa, pb = kfa[f][name], kfb[f][name]
            rel = float((pa - pb).norm() / pa.norm())
            assert rel < 1e-3, (f, name, rel)


def test_capture_needs_a_sized_workload_and_refuses_sync(ctx):
    import torch
    from paper_2603_21055_amd import sgad
    from paper_2603_21055_amd.mapping import Mapper
    print("graph: refusals", flush=True)
    sc = synth.small_scene(32, 40, 24)
    dev = ctx.device
    kfs = [sgad.to_device(k, dev) for k in sc["kfs"]]
    t_rgb = torch.from_numpy(sc["targets"][0]["rgb"][None].copy()).to(dev)
    t_dep = torch.from_numpy(sc["targets"][0]["depth"][None].copy()).to(dev)
    m = Mapper(ctx, kfs, sc["views"], [(0, [0])], [0], t_rgb, t_dep)
    ctx.graph_begin()
    with pytest.raises(sgad.SgadError):
        ctx.sync()
    with pytest.raises(sgad.SgadError):
        m.step()                  # this workload has never run eagerly
    try:
        g = ctx.graph_end()       # nothing was recorded
    except sgad.SgadError:
        g = None
    if g is not None:
        ctx.graph_destroy(g)
    m.step()                      # eager again after the capture closed
    torch.cuda.synchronize()
    ctx.sync()


def test_kernels_of_replays_are_timed(ctx):
    """Timing events captured as graph nodes get fresh events per launch."""
    import torch
    print("graph: timing", flush=True)
    m, _ = _mapper(ctx, seed=33)
    m.step()
    torch.cuda.synchronize()
    ctx.timing(True)
    m.capture()
    try:
        ctx.timing(True)          # reset the accumulators
        for _ in range(3):
            m.replay()
        torch.cuda.synchronize()
        rep = ctx.timing_report()
        ctx.timing(False)
    finally:
        m.release_graph()
    print(rep, flush=True)
    for k in ("preprocess", "sort", "composite_fwd", "l1_loss", "composite_bwd", "adam"):
        n, ms = rep[k]
        assert n == 3 and 0.0 < ms < 1e3, (k, n, ms)
