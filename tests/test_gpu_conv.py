"""GPU parity of the BF16-MFMA conv net against the FP64 oracle that emulates
its BF16 roundings (tolerances: one bf16 step elementwise where the output
is rounded to bf16; 1e-2 normwise for network outputs and gradients, whose
inputs went through several bf16 roundings that FP32 vs FP64 accumulation
can tip to the neighbouring bf16 value)."""
import numpy as np
import pytest

from oracle import conv as oconv

pytestmark = pytest.mark.gpu

BF16_STEP = 2.0 ** -7   # bf16 keeps 8 significant bits: neighbours are at most 2^-7 |x| apart


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2603_21055_amd import sgad
    assert torch.cuda.is_available()
    c = sgad.Context(0)
    yield c
    c.close()


def _bf(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev).to(torch.bfloat16)


def _np(t):
    import torch
    return t.to(torch.float32).cpu().numpy().astype(np.float64)


def _layer_weights(ctx, cin, cout, seed):
    import torch
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(3, 3, cout, cin)).astype(np.float32) * np.float32(np.sqrt(2.0 / (9 * cin)))
    b = rng.normal(size=cout).astype(np.float32) * np.float32(0.1)
    w9 = torch.from_numpy(np.ascontiguousarray(w.reshape(9, cout, cin))).to(ctx.device)
    w16 = torch.empty((9, cout, cin), dtype=torch.bfloat16, device=ctx.device)
    wt16 = torch.empty((9, cin, cout), dtype=torch.bfloat16, device=ctx.device)
    ctx.conv_weights(cin, cout, w9, w16, wt16)
    return w, b, w16, wt16


# 37x45: 9 ragged 16x16 tiles, fewer than the persistent workgroups (one tile
# each); 330x530: 714 tiles, more than the 512 persistent workgroups, so
# workgroups walk several tiles and prefetch the next tile's patch while the
# current one runs, with ragged last row and column
SIZES = [(37, 45), (330, 530)]


@pytest.mark.parametrize("H,W", SIZES)
@pytest.mark.parametrize("cin,cout", [(4, 32), (32, 32), (32, 1)])
def test_single_layer_forward(ctx, cin, cout, H, W):
    import torch
    print(f"conv fwd {cin}->{cout} {H}x{W}", flush=True)
    rng = np.random.default_rng(cin * 100 + cout)
    x = rng.normal(size=(H, W, cin)).astype(np.float32)
    w, b, w16, _ = _layer_weights(ctx, cin, cout, 1)
    xb = _bf(x, ctx.device)
    bt = torch.from_numpy(b).to(ctx.device)
    if cout == 1:
        y = torch.empty((H, W), dtype=torch.float32, device=ctx.device)
        ctx.conv_fwd(H, W, cin, cout, 1, xb, w16, bt, y)
        torch.cuda.synchronize()
        ref = oconv.conv3x3(oconv.bf16(x), oconv.bf16(w), b.astype(np.float64))[..., 0]
        got = y.cpu().numpy().astype(np.float64)
        # FP32 output: FP32 accumulation error of K = 9 cin products, elementwise
        absterms = oconv.conv3x3(np.abs(oconv.bf16(x)), np.abs(oconv.bf16(w)), np.abs(b.astype(np.float64)))
        viol = np.abs(got - ref)[..., None] - 9 * cin * 2.0 ** -24 * absterms
        assert viol.max() <= 0, (float(viol.max()), int((viol > 0).sum()))
    else:
        y = torch.empty((H, W, cout), dtype=torch.bfloat16, device=ctx.device)
        ctx.conv_fwd(H, W, cin, cout, 0, xb, w16, bt, y)
        torch.cuda.synchronize()
        pre = oconv.conv3x3(oconv.bf16(x), oconv.bf16(w), b.astype(np.float64))
        ref = oconv.bf16(np.maximum(pre, 0.0))
        # FP32 accumulation of K = 9 cin products moves a pre-activation by up
        # to K * 2^-24 of its absolute terms: across the ReLU kink or a bf16
        # rounding boundary
        absterms = oconv.conv3x3(np.abs(oconv.bf16(x)), np.abs(oconv.bf16(w)), np.abs(b.astype(np.float64)))
        got = _np(y)
        viol = np.abs(got - ref) - (BF16_STEP * np.abs(ref) + 9 * cin * 2.0 ** -24 * absterms)
        assert viol.max() <= 0, (float(viol.max()), int((viol > 0).sum()))
        assert (got == ref).mean() > 0.99


@pytest.mark.parametrize("H,W", [(33, 40), (330, 530)])
@pytest.mark.parametrize("cin,cout", [(32, 32), (32, 1)])
def test_single_layer_input_gradient(ctx, cin, cout, H, W):
    import torch
    print(f"conv dgrad {cin}->{cout} {H}x{W}", flush=True)
    rng = np.random.default_rng(7 + cout)
    dy = rng.normal(size=(H, W, cout)).astype(np.float32)
    mask = np.maximum(rng.normal(size=(H, W, cin)), 0.0).astype(np.float32)
    w, b, w16, wt16 = _layer_weights(ctx, cin, cout, 2)
    dx = torch.empty((H, W, cin), dtype=torch.bfloat16, device=ctx.device)
    ctx.conv_dgrad(H, W, cin, cout, _bf(dy, ctx.device), wt16, _bf(mask, ctx.device), dx)
    torch.cuda.synchronize()
    ref = oconv.bf16(oconv.conv3x3_input_grad(oconv.bf16(dy), oconv.bf16(w)) * (oconv.bf16(mask) > 0))
    absterms = oconv.conv3x3_input_grad(np.abs(oconv.bf16(dy)), np.abs(oconv.bf16(w)))
    got = _np(dx)
    viol = np.abs(got - ref) - (BF16_STEP * np.abs(ref) + 9 * cout * 2.0 ** -24 * absterms)
    assert viol.max() <= 0, (float(viol.max()), int((viol > 0).sum()))


@pytest.mark.parametrize("cin,cout,H,W", [(4, 32, 50, 70), (32, 32, 50, 70), (32, 1, 50, 70),
                                          (32, 32, 330, 530), (4, 32, 330, 530)])
def test_single_layer_weight_gradient(ctx, cin, cout, H, W):
    """50x70: 20 ragged tiles; 330x530: 714 tiles, more than the persistent
    workgroups, so workgroups accumulate several tiles."""
    import torch
    print(f"conv wgrad {cin}->{cout} {H}x{W}", flush=True)
    rng = np.random.default_rng(11 + cin + cout)
    x = rng.normal(size=(H, W, cin)).astype(np.float32)
    dy = rng.normal(size=(H, W, cout)).astype(np.float32)
    dw = torch.zeros((9, cout, cin), dtype=torch.float32, device=ctx.device)
    db = torch.zeros(cout, dtype=torch.float32, device=ctx.device)
    ctx.conv_wgrad(H, W, cin, cout, _bf(x, ctx.device), _bf(dy, ctx.device), dw, db)
    torch.cuda.synchronize()
    ref = oconv.conv3x3_weight_grad(oconv.bf16(dy), oconv.bf16(x))
    got = dw.cpu().numpy().reshape(3, 3, cout, cin)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    np.testing.assert_allclose(db.cpu().numpy(), oconv.bf16(dy).sum((0, 1)), rtol=1e-5, atol=1e-3)
    # the outputs accumulate: a second call on the same inputs adds the same sums
    first_w, first_b = dw.clone(), db.clone()
    ctx.conv_wgrad(H, W, cin, cout, _bf(x, ctx.device), _bf(dy, ctx.device), dw, db)
    torch.cuda.synchronize()
    torch.testing.assert_close(dw, 2 * first_w, rtol=1e-6, atol=1e-6 * float(first_w.abs().max()))
    torch.testing.assert_close(db, 2 * first_b, rtol=1e-6, atol=1e-6 * float(first_b.abs().max()))


def test_net_input_matches_oracle(ctx):
    """k_net_input: colour planes and the high-passed depth channel, each
    rounded to bf16 once (FP32 vs FP64 evaluation of the channel can tip the
    rounding to a neighbouring bf16 value)."""
    import torch
    from paper_2603_21055_amd import synth
    sc = synth.small_scene(51, 97, 61)
    kf = sc["kfs"][0]
    rng = np.random.default_rng(5)
    depth = (kf["depth"] + rng.normal(size=kf["depth"].shape) * 0.01).astype(np.float32)
    dev = ctx.device
    x0 = torch.empty((61, 97, 4), dtype=torch.bfloat16, device=dev)
    ctx.net_input(61, 97, torch.from_numpy(kf["rgb"]).to(dev), torch.from_numpy(depth).to(dev), x0)
    torch.cuda.synchronize()
    got = _np(x0)
    ref = oconv.net_input(kf["rgb"], depth)
    np.testing.assert_array_equal(got[..., :3], oconv.bf16(ref[..., :3]))
    # FP32 sum of 9 depths (|D| <= 5 m) then a difference: error <= 12 ulp(5 m) / 0.02 m
    err = np.abs(got[..., 3] - oconv.bf16(ref[..., 3]))
    assert (err <= BF16_STEP * np.abs(ref[..., 3]) + 12 * 2.0 ** -21 / 0.02).all(), float(err.max())
    assert (got[..., 3] == oconv.bf16(ref[..., 3])).mean() > 0.9


def test_network_forward_and_gradients(ctx):
    import torch
    from paper_2603_21055_amd.offsetnet import OffsetNet, init_params
    from paper_2603_21055_amd import synth
    print("offset net fwd/bwd 96x72", flush=True)
    sc = synth.small_scene(50, 96, 72)
    kf = sc["kfs"][0]
    params = init_params(3)
    rng = np.random.default_rng(4)
    params = [(w, (rng.normal(size=b.shape) * 0.05).astype(np.float32)) for w, b in params]
    net = OffsetNet(ctx, params)
    dev = ctx.device
    rgb = torch.from_numpy(kf["rgb"]).to(dev)
    dep = torch.from_numpy(kf["depth"]).to(dev)
    delta = net.forward(rgb, dep)
    target = torch.from_numpy(rng.normal(size=(72, 96)).astype(np.float32) * 0.01).to(dev)
    g = torch.empty((72, 96), dtype=torch.bfloat16, device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.offset_l1(delta, target, g, loss)
    net.backward(g)
    torch.cuda.synchronize()
    x0 = oconv.net_input(kf["rgb"], kf["depth"])
    d0, acts, _ = oconv.forward(params, x0)
    got = delta.cpu().numpy()
    assert np.linalg.norm(got - d0) <= 1e-2 * np.linalg.norm(d0)
    L, gd = oconv.l1(got, target.cpu().numpy())      # same sign pattern as the GPU's
    assert abs(loss.item() - L) <= 1e-6 * L
    grads = oconv.backward(params, acts, gd)
    for l in range(6):
        gw = net.dw[l].cpu().numpy().reshape(grads[l][0].shape)
        e = np.linalg.norm(gw - grads[l][0]) / np.linalg.norm(grads[l][0])
        print(f"layer {l}: weight-grad rel err {e:.2e}", flush=True)
        assert e <= 1e-2
        gb = net.db[l].cpu().numpy()
        assert np.linalg.norm(gb - grads[l][1]) <= 1e-2 * np.linalg.norm(grads[l][1]) + 1e-6


def test_training_reduces_loss(ctx):
    import torch
    from paper_2603_21055_amd.offsetnet import OffsetNet
    from paper_2603_21055_amd import synth
    print("offset net training", flush=True)
    dev = ctx.device
    batch = []
    for s in range(4):
        sc = synth.small_scene(60 + s, 64, 48)
        kf = sc["kfs"][0]
        rng = np.random.default_rng(s)
        noise = rng.normal(size=kf["depth"].shape).astype(np.float32) * 0.01
        # learnable target: the offset that undoes a known depth perturbation
        batch.append((torch.from_numpy(kf["rgb"]).to(dev), torch.from_numpy(kf["depth"] + noise).to(dev),
                      torch.from_numpy(-noise).to(dev)))
    net = OffsetNet(ctx, seed=0)
    first = net.train_step(batch).mean().item()
    for _ in range(60):
        last = net.train_step(batch)
    torch.cuda.synchronize()
    assert last.mean().item() < first


def test_misaligned_pointers_rejected(ctx):
    """The conv entry points refuse activation pointers that are not 16-byte
    aligned (checked on the host, before any launch)."""
    import torch
    from paper_2603_21055_amd import sgad
    H, W = 16, 16
    buf = torch.zeros(H * W * 32 + 8, dtype=torch.bfloat16, device=ctx.device)
    x_bad = buf[1:1 + H * W * 32]
    dy = torch.zeros((H, W, 32), dtype=torch.bfloat16, device=ctx.device)
    dw = torch.zeros((9, 32, 32), dtype=torch.float32, device=ctx.device)
    db = torch.zeros(32, dtype=torch.float32, device=ctx.device)
    with pytest.raises(sgad.SgadError, match="16-byte aligned"):
        ctx.conv_wgrad(H, W, 32, 32, x_bad, dy, dw, db)
    w16 = torch.zeros((9, 32, 32), dtype=torch.bfloat16, device=ctx.device)
    bias = torch.zeros(32, dtype=torch.float32, device=ctx.device)
    y = torch.empty((H, W, 32), dtype=torch.bfloat16, device=ctx.device)
    with pytest.raises(sgad.SgadError, match="16-byte aligned"):
        ctx.conv_fwd(H, W, 32, 32, 0, x_bad, w16, bias, y)
    torch.cuda.synchronize()
    assert float(dw.abs().sum()) == 0.0
