"""GPU parity of the splat forward/adjoint (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import splat
from paper_2603_21055_amd import synth
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu

TILES = [(16, 16), (8, 8), (16, 8), (32, 8)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2603_21055_amd import sgad
    assert torch.cuda.is_available()
    c = sgad.Context(0)
    yield c
    c.close()


def _upstream(seed, nj, Hh, W):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(nj, 3, Hh, W)) / (Hh * W), rng.normal(size=(nj, Hh, W)) / (Hh * W),
            rng.normal(size=(nj, Hh, W)) / (Hh * W))


def _run_case(ctx, sc, jobs, tile, learnable, seed=0, check_grads=True, max_flag_frac=H.MAX_FLAG_FRAC):
    import torch
    print(f"case tile={tile} jobs={jobs} size={sc['views'][0]['cam']['W']}x{sc['views'][0]['cam']['H']}",
          flush=True)
    ctx.set_tile(*tile)
    kfs_d = H.upload(sc["kfs"], ctx.device)
    saved, out = H.gpu_render(ctx, kfs_d, sc["views"], jobs)
    orc = [splat.render_job(sc["kfs"], sc["views"][v], ids) for v, ids in jobs]
    torch.cuda.synchronize()
    H.assert_forward_parity(out, orc, max_flag_frac=max_flag_frac)
    if check_grads:
        Hh, W = sc["views"][0]["cam"]["H"], sc["views"][0]["cam"]["W"]
        gr, gd, ga = (H.zero_flagged(u, orc) for u in _upstream(seed, len(jobs), Hh, W))
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(ctx.device)
        grads, d_pose = H.gpu_backward(ctx, saved, kfs_d, t(gr), t(gd), t(ga), len(jobs), learnable)
        torch.cuda.synchronize()
        b = splat.render_backward(sc["kfs"], sc["views"], jobs, orc,
                                  [g.astype(np.float32).astype(np.float64) for g in gr],
                                  [g.astype(np.float32).astype(np.float64) for g in gd],
                                  [g.astype(np.float32).astype(np.float64) for g in ga], learnable=set(learnable))
        H.assert_grad_parity(grads, d_pose, b, orc, set(learnable))
    ctx.release(saved)
    ctx.sync()
    return out


@pytest.mark.parametrize("tile", TILES)
def test_plane_forward_backward_parity(ctx, tile):
    sc = synth.plane_scene(0)
    _run_case(ctx, sc, [(1, [0])], tile, learnable=[0])


def test_plane_identity_view(ctx):
    sc = synth.plane_scene(0)
    _run_case(ctx, sc, [(0, [0])], (16, 16), learnable=[0])


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_two_keyframes_two_views_ragged(ctx, tile):
    # 37x21 spans several tiles with ragged edges in both directions
    sc = synth.small_scene(21, 37, 21, n_kf=2, n_views=2, offset_amp=0.03, max_trans=0.05, max_rot=3)
    jobs = [(0, [0, 1]), (1, [0, 1]), (1, [1])]
    _run_case(ctx, sc, jobs, tile, learnable=[0, 1])


def test_neighbour_keyframe_is_fixed(ctx):
    sc = synth.small_scene(22, 48, 32, n_kf=2, n_views=1, offset_amp=0.03)
    _run_case(ctx, sc, [(0, [0, 1])], (16, 16), learnable=[1])


def test_medium_frame_parity(ctx):
    sc = synth.small_scene(23, 160, 120, n_kf=1, n_views=1)
    _run_case(ctx, sc, [(0, [0])], (16, 16), learnable=[0])


def test_tile_shape_does_not_change_forward(ctx):
    import torch
    sc = synth.small_scene(24, 100, 75, n_kf=2, n_views=1, offset_amp=0.03, max_trans=0.05, max_rot=3)
    kfs_d = H.upload(sc["kfs"], ctx.device)
    outs = []
    for tile in TILES:
        ctx.set_tile(*tile)
        saved, out = H.gpu_render(ctx, kfs_d, sc["views"], [(0, [0, 1])])
        torch.cuda.synchronize()
        outs.append({k: v.cpu().numpy() for k, v in out.items()})
        ctx.release(saved)
    for o in outs[1:]:
        for k in ("rgb", "depth", "alpha", "count"):
            assert np.array_equal(o[k], outs[0][k]), k


VARIANTS = [(1, 16), (2, 16), (4, 16), (1, 32), (4, 32)]


@pytest.mark.parametrize("variant", VARIANTS)
def test_wave_tile_variants_parity(ctx, variant):
    """Every 8x8 kernel variant (chunks the forward publishes at once, adjoint
    sub-chunk) matches the oracle, forward and gradients."""
    ctx.set_tile_variant(*variant)
    try:
        sc = synth.small_scene(25, 100, 75, n_kf=2, n_views=1, offset_amp=0.03, max_trans=0.05, max_rot=3)
        _run_case(ctx, sc, [(0, [0, 1])], (8, 8), learnable=[0, 1])
    finally:
        ctx.set_tile_variant(4, 16)


def test_wave_tile_variants_do_not_change_forward(ctx):
    import torch
    sc = synth.small_scene(26, 100, 75, n_kf=2, n_views=1, offset_amp=0.03, max_trans=0.05, max_rot=3)
    kfs_d = H.upload(sc["kfs"], ctx.device)
    ctx.set_tile(8, 8)
    outs = []
    try:
        for v in VARIANTS:
            ctx.set_tile_variant(*v)
            saved, out = H.gpu_render(ctx, kfs_d, sc["views"], [(0, [0, 1])])
            torch.cuda.synchronize()
            assert ctx.get_tile_variant() == v
            outs.append({k: x.cpu().numpy() for k, x in out.items()})
            ctx.release(saved)
    finally:
        ctx.set_tile_variant(4, 16)
    for o in outs[1:]:
        for k in ("rgb", "depth", "alpha", "count"):
            assert np.array_equal(o[k], outs[0][k]), k


def test_workspace_bytes(ctx):
    """The slot sizes the forward allocates: records 92 B per Gaussian-view
    pair, tile tables, keys (8 B each) with their contributor masks,
    per-pixel state and the adjoint's 32 B gradient record per keyframe
    Gaussian; the key list grows with the instance count."""
    sc = synth.small_scene(27, 64, 48, n_kf=2, n_views=2)
    kfs_d = H.upload(sc["kfs"], ctx.device)
    jobs = [(0, [0, 1]), (1, [1])]
    b0 = ctx.workspace_bytes(kfs_d, sc["views"], jobs)
    b1 = ctx.workspace_bytes(kfs_d, sc["views"], jobs, instances=100_000)
    b2 = ctx.workspace_bytes(kfs_d, sc["views"], jobs, instances=200_000)
    npairs, N, P, M = 3, 64 * 48, 64 * 48, 2 * 8 * 6
    floor = npairs * N * 92 + 2 * P * 8 + (4 * M + 2) * 4 + M * 24 + 2 * N * 32
    assert b0 > floor and b1 > floor
    # 100,000 more instances: 1.25x as many keys, 8 B each, and their masks
    # (8 B per key, allocated in whole 64-key chunks)
    grown = (b2 - b1) / (100_000 * 1.25)
    assert abs(grown - 16.0) <= 512 / (100_000 * 1.25), grown


def test_forward_is_deterministic(ctx):
    import torch
    sc = synth.small_scene(25, 64, 48, n_kf=2, n_views=1, offset_amp=0.03)
    kfs_d = H.upload(sc["kfs"], ctx.device)
    ctx.set_tile(16, 16)
    res = []
    for _ in range(3):
        saved, out = H.gpu_render(ctx, kfs_d, sc["views"], [(0, [0, 1])])
        torch.cuda.synchronize()
        res.append({k: v.cpu().numpy() for k, v in out.items()})
        ctx.release(saved)
    for r in res[1:]:
        for k in r:
            assert np.array_equal(r[k], res[0][k])


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_binning_and_sort_bit_exact(ctx, tile):
    import torch
    sc = synth.small_scene(26, 45, 29, n_kf=2, n_views=2, offset_amp=0.03, max_trans=0.05, max_rot=3)
    kfs_d = H.upload(sc["kfs"], ctx.device)
    ctx.set_tile(*tile)
    jobs = [(0, [0, 1]), (1, [1])]
    saved, _ = H.gpu_render(ctx, kfs_d, sc["views"], jobs)
    torch.cuda.synchronize()
    for j, (v, ids) in enumerate(jobs):
        ranges, keys = ctx.instances(saved, j)
        g = splat.gather_job(sc["kfs"], sc["views"][v], ids)
        b = splat.bin_and_sort(g, 45, 29, *tile)
        assert np.array_equal(ranges.astype(np.int64), b["ranges"]), "tile ranges differ"
        assert np.array_equal((keys >> np.uint64(32)).astype(np.uint32), b["zbits"]), "depth keys differ"
        assert np.array_equal((keys & np.uint64(0xFFFFFFFF)).astype(np.int64), b["gid"]), "gids differ"
    ctx.release(saved)


def _wide_scene(fac, opacity_range=(0.5, 1.0)):
    """Three 48x32 keyframes whose radii are scaled by `fac`: every tile list
    is long (8x8 tiles: 372-768 entries at fac 1, 1242-3325 at fac 4; 16x16
    tiles: 4161-4608 at fac 8)."""
    sc = synth.small_scene(29, 48, 32, n_kf=3, n_views=1, max_trans=0.03, max_rot=2,
                           opacity_range=opacity_range)
    for kf in sc["kfs"]:
        kf["radius"] = (kf["radius"] * np.float32(fac)).astype(np.float32)
    return sc


@pytest.mark.parametrize("fac,tile,lo,hi", [(1, (8, 8), 257, 1024), (4, (8, 8), 1025, 4096),
                                            (8, (16, 16), 4097, 1 << 30)])
def test_long_lists_sort_bit_exact(ctx, fac, tile, lo, hi):
    """Lists sorted in registers (8 and 16 keys per lane), in LDS and in global
    memory keep the oracle's order bit for bit."""
    import torch
    print(f"long lists fac={fac} tile={tile}", flush=True)
    sc = _wide_scene(fac)
    kfs_d = H.upload(sc["kfs"], ctx.device)
    ctx.set_tile(*tile)
    saved, _ = H.gpu_render(ctx, kfs_d, sc["views"], [(0, [0, 1, 2])])
    torch.cuda.synchronize()
    ranges, keys = ctx.instances(saved, 0)
    g = splat.gather_job(sc["kfs"], sc["views"][0], [0, 1, 2])
    b = splat.bin_and_sort(g, 48, 32, *tile)
    lens = b["ranges"][:, 1] - b["ranges"][:, 0]
    assert ((lens >= lo) & (lens <= hi)).any()
    assert np.array_equal(ranges.astype(np.int64), b["ranges"])
    assert np.array_equal((keys >> np.uint64(32)).astype(np.uint32), b["zbits"])
    assert np.array_equal((keys & np.uint64(0xFFFFFFFF)).astype(np.int64), b["gid"])
    ctx.release(saved)


def test_long_lists_sorted_without_the_long_pass(ctx):
    """The long-segment pass runs only when the previous forward of the same
    workload had a segment over 1024 keys; a segment that grows past it in
    between is sorted by the register kernel's global-memory fallback."""
    import torch
    print("long lists: fallback sort", flush=True)
    ctx.set_tile(8, 8)
    short = _wide_scene(1)      # every list <= 768 keys
    saved, _ = H.gpu_render(ctx, H.upload(short["kfs"], ctx.device), short["views"], [(0, [0, 1, 2])])
    ctx.release(saved)
    ctx.sync()                  # the slot now knows its longest segment
    sc = _wide_scene(4)         # same sizes, lists of 1242-3325 keys
    saved, _ = H.gpu_render(ctx, H.upload(sc["kfs"], ctx.device), sc["views"], [(0, [0, 1, 2])])
    torch.cuda.synchronize()
    ranges, keys = ctx.instances(saved, 0)
    g = splat.gather_job(sc["kfs"], sc["views"][0], [0, 1, 2])
    b = splat.bin_and_sort(g, 48, 32, 8, 8)
    assert (b["ranges"][:, 1] - b["ranges"][:, 0]).max() > 1024
    assert np.array_equal(ranges.astype(np.int64), b["ranges"])
    assert np.array_equal((keys >> np.uint64(32)).astype(np.uint32), b["zbits"])
    assert np.array_equal((keys & np.uint64(0xFFFFFFFF)).astype(np.int64), b["gid"])
    ctx.release(saved)
    ctx.sync()


def test_long_lists_two_kilo_pass(ctx):
    """Once the workload's longest segment is known to be <= 2048 keys the
    long pass runs with half the LDS (1025..2048-key segments as four
    512-key runs merged in two levels); a segment that then grows past 2048
    is sorted in global memory by the same pass."""
    import torch
    print("long lists: 2048-key pass", flush=True)
    ctx.set_tile(8, 8)

    def check(sc):
        saved, _ = H.gpu_render(ctx, H.upload(sc["kfs"], ctx.device), sc["views"], [(0, [0, 1, 2])])
        torch.cuda.synchronize()
        ranges, keys = ctx.instances(saved, 0)
        g = splat.gather_job(sc["kfs"], sc["views"][0], [0, 1, 2])
        b = splat.bin_and_sort(g, 48, 32, 8, 8)
        assert np.array_equal(ranges.astype(np.int64), b["ranges"])
        assert np.array_equal((keys >> np.uint64(32)).astype(np.uint32), b["zbits"])
        assert np.array_equal((keys & np.uint64(0xFFFFFFFF)).astype(np.int64), b["gid"])
        ctx.release(saved)
        ctx.sync()              # the slot records the longest segment
        return (b["ranges"][:, 1] - b["ranges"][:, 0]).max()

    mid = _wide_scene(2.5)      # lists of 748-1898 keys
    assert 1024 < check(mid) <= 2048
    assert 1024 < check(mid) <= 2048     # now through the 2048-key pass
    assert check(_wide_scene(3.5)) > 2048   # past it: the global-memory network


@pytest.mark.parametrize("fac", [1, 4])
def test_long_lists_render_parity(ctx, fac):
    """Faint wide Gaussians: hundreds of contributors per pixel, so the walks
    cross many 64-entry chunks (forward and backward).  With ~1700 candidates
    per pixel, 2-3% of the pixels hold a pair within the q-flag band of 9."""
    sc = _wide_scene(fac, opacity_range=(0.02, 0.08))
    _run_case(ctx, sc, [(0, [0, 1, 2])], (8, 8), learnable=[0, 1, 2], max_flag_frac=0.05)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_full_frame_640x480_parity(ctx, tile):
    sc = synth.room_frame_scene(10)
    _run_case(ctx, sc, [(0, [0])], tile, learnable=[0])


def test_everything_culled_renders_empty(ctx):
    import torch
    sc = synth.small_scene(27, 32, 24)
    view = dict(sc["views"][0])
    view["t"] = np.array([0.0, 0.0, -50.0], np.float32)   # scene far behind the camera
    kfs_d = H.upload(sc["kfs"], ctx.device)
    saved, out = H.gpu_render(ctx, kfs_d, [view], [(0, [0])])
    torch.cuda.synchronize()
    assert float(out["alpha"].abs().max()) == 0.0 and int(out["count"].max()) == 0
    ctx.release(saved)


def test_invalid_arguments_are_rejected(ctx):
    import torch
    from paper_2603_21055_amd import sgad
    sc = synth.small_scene(28, 16, 12)
    kfs_d = H.upload(sc["kfs"], ctx.device)
    with pytest.raises(sgad.SgadError) as e:
        H.gpu_render(ctx, kfs_d, sc["views"], [(3, [0])])     # view index out of range
    assert e.value.status == sgad.EINVAL
    bad = dict(sc["views"][0])
    bad["t"] = np.array([np.nan, 0, 0], np.float32)
    with pytest.raises(sgad.SgadError) as e:
        H.gpu_render(ctx, kfs_d, [bad], [(0, [0])])
    assert e.value.status == sgad.EINVAL
    with pytest.raises(sgad.SgadError):
        ctx.set_tile(12, 12)


def test_nonfinite_depth_is_latched(ctx):
    import torch
    from paper_2603_21055_amd import sgad
    sc = synth.small_scene(29, 16, 12)
    kfs_d = H.upload(sc["kfs"], ctx.device)
    kfs_d[0]["depth"][3, 4] = float("nan")
    saved, _ = H.gpu_render(ctx, kfs_d, sc["views"], [(0, [0])])
    with pytest.raises(sgad.SgadError) as e:
        ctx.sync()
    assert e.value.status == sgad.EDATA
    ctx.release(saved)
    ctx.sync()   # cleared
    # the flag belongs to that call: the same slot, with the input repaired,
    # reports nothing (each forward clears the flags it handed back)
    kfs_d[0]["depth"][3, 4] = 2.0
    for tile in ((8, 8), (16, 16), (8, 8)):
        ctx.set_tile(*tile)
        saved, _ = H.gpu_render(ctx, kfs_d, sc["views"], [(0, [0])])
        ctx.release(saved)
        ctx.sync()
    ctx.set_tile(0, 0)


def test_autotuner_picks_a_config_and_results_do_not_change(ctx):
    import torch
    sc = synth.small_scene(30, 160, 120, n_kf=2, n_views=1, offset_amp=0.02)
    kfs_d = H.upload(sc["kfs"], ctx.device)
    jobs = [(0, [0, 1])]
    ctx.set_tile(16, 16)
    saved, ref = H.gpu_render(ctx, kfs_d, sc["views"], jobs)
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy() for k, v in ref.items()}
    ctx.release(saved)
    ctx.set_tile(0, 0)
    tile, ms = ctx.autotune(kfs_d, sc["views"], jobs, reps=2)
    print(f"autotune: tile {tile}, {ms:.3f} ms per forward + adjoint", flush=True)
    assert tile in [(8, 8), (16, 8), (16, 16), (32, 8)] and ms > 0
    saved, out = H.gpu_render(ctx, kfs_d, sc["views"], jobs)
    torch.cuda.synchronize()
    assert ctx.get_tile() == tile
    for k in ("rgb", "depth", "alpha", "count"):
        assert np.array_equal(out[k].cpu().numpy(), ref[k]), k
    ctx.release(saved)
    ctx.sync()
