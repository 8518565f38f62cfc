"""sgad_conv3x3_wgrad_noalloc (partial sums in the library's static device
array, no allocation) against sgad_conv3x3_wgrad (partial sums in the
context's workspace) through the C ABI: two calls in a row, the second on a
smaller input, each from fresh zero accumulators and then accumulating."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _bf(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev).to(torch.bfloat16).contiguous()


def _check(a, b):
    a = a.cpu().numpy().astype(np.float64)
    b = b.cpu().numpy().astype(np.float64)
    # the two paths differ only in where the rows live; the rows' sums are
    # added to the outputs by atomics whose order may differ
    np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * float(np.abs(b).max()))


@pytest.mark.parametrize("first,second", [((480, 640, 32, 32), (100, 150, 4, 32)),
                                          ((330, 530, 4, 32), (61, 97, 32, 1))])
def test_noalloc_wgrad_equals_workspace_wgrad(first, second):
    import torch
    from paper_2603_21055_amd import sgad
    ctx = sgad.Context(0)
    dev = ctx.device
    try:
        for k, (H, W, cin, cout) in enumerate((first, second)):
            print(f"noalloc wgrad call {k}: {cin}->{cout} {H}x{W}", flush=True)
            rng = np.random.default_rng(100 + k + cin + H)
            x = _bf(rng.normal(size=(H, W, cin)), dev)
            dy = _bf(rng.normal(size=(H, W, cout)), dev)
            outs = []
            for fn in (ctx.conv_wgrad, ctx.conv_wgrad_noalloc):
                dw = torch.zeros((9, cout, cin), dtype=torch.float32, device=dev)
                db = torch.zeros(cout, dtype=torch.float32, device=dev)
                fn(H, W, cin, cout, x, dy, dw, db)
                torch.cuda.synchronize()
                outs.append((dw.clone(), db.clone()))
                # accumulation: a second call adds the same sums
                fn(H, W, cin, cout, x, dy, dw, db)
                torch.cuda.synchronize()
                _check(dw, 2 * outs[-1][0])
                _check(db, 2 * outs[-1][1])
            _check(outs[1][0], outs[0][0])
            _check(outs[1][1], outs[0][1])
            assert float(outs[0][0].abs().max()) > 0
    finally:
        ctx.close()


def test_noalloc_wgrad_rejects_bad_arguments():
    import torch
    from paper_2603_21055_amd import sgad
    ctx = sgad.Context(0)
    dev = ctx.device
    try:
        x = torch.zeros((8, 8, 32), dtype=torch.bfloat16, device=dev)
        dy = torch.zeros((8, 8, 32), dtype=torch.bfloat16, device=dev)
        dw = torch.zeros((9, 32, 32), dtype=torch.float32, device=dev)
        db = torch.zeros(32, dtype=torch.float32, device=dev)
        with pytest.raises(sgad.SgadError):
            ctx.conv_wgrad_noalloc(8, 8, 16, 32, x, dy, dw, db)      # unsupported layer
        with pytest.raises(sgad.SgadError):
            ctx.conv_wgrad_noalloc(0, 8, 32, 32, x, dy, dw, db)      # empty image
    finally:
        ctx.close()
