"""What the trained warm start gains over the plain random start.

The committed network (trained on the library's own simulations of 256^2
images) is applied to fresh 1024^2 images; the chains with the learned start
must stop in fewer sweeps and reach the same prediction MAE (within 1% on
random masks, where the seed-to-seed spread is small).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_1811_01604_amd as mpr  # noqa: E402
from paper_1811_01604_amd import warmstart  # noqa: E402

pytestmark = pytest.mark.gpu


def test_warm_start_gain():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    params, info = warmstart.load()
    ctx = mpr.Context(0)
    model = warmstart.WarmStart(ctx, params)
    s = warmstart.evaluate(ctx, model, size=1024, seeds=2, workers=4)
    ctx.close()
    print(s)
    for kind in ("random", "cloud"):
        assert s[kind]["sweeps_warm"] < s[kind]["sweeps_plain"]
        assert s[kind]["time_to_fill_warm_s"] < s[kind]["time_to_fill_plain_s"] * 1.05
    assert abs(s["random"]["mae_warm_over_plain"] - 1.0) < 0.01
    assert abs(s["cloud"]["mae_warm_over_plain"] - 1.0) < 0.05


def test_warm_start_inference_at_full_size_sampled_pixels():
    """The committed network on a 2048 x 2048 evaluation image (50% random
    gaps), checked at sampled pixels: 18 stacked 3x3 convolutions make an
    output pixel depend on the input within 18 pixels, so the oracle computes
    it from that crop of the same bfloat16 input (zero padding at the image
    edges, as on the GPU).  Bar as for the whole network on small inputs:
    max error 6e-2 of the largest output magnitude, cosine >= 0.998."""
    import math
    import sys

    import oracle
    from oracle import cnn

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    size, r = 2048, cnn.N_LAYERS
    params, _ = warmstart.load()
    z, m = warmstart._eval_field(("random", size, 0))
    po, _ = oracle.map_to_angles(z.astype(np.float64), m)
    phi32 = po.astype(np.float32)
    ctx = mpr.Context(0)
    model = warmstart.WarmStart(ctx, params)
    x = torch.empty((1, size, size, 32), dtype=torch.bfloat16, device="cuda")
    y = torch.empty_like(x)
    ctx.cnn_encode(torch.from_numpy(phi32).cuda().view(1, size, size), torch.from_numpy(m).cuda().view(1, size, size), x)
    ws = torch.empty(ctx.cnn_workspace_size(1, size, size, False), dtype=torch.uint8, device="cuda")
    ctx.cnn_forward(model.p, model.packed, x, ws, y, training=False)
    yg = y.float().cpu().numpy()[0, ..., :2].astype(np.float64)
    ctx.close()
    wsz = 9 * 32 * 32
    flat = params.astype(np.float64)
    rp = [(cnn.bf16_round(flat[k * (wsz + 32):k * (wsz + 32) + wsz].reshape(9, 32, 32)),
           np.float32(flat[k * (wsz + 32) + wsz:(k + 1) * (wsz + 32)]).astype(np.float64))
          for k in range(cnn.N_LAYERS)]
    rng = np.random.default_rng(2)
    pix = [(0, 0), (0, size - 1), (size - 1, 0), (size - 1, size - 1), (0, 1000), (size - 1, 77), (513, 0),
           (1500, size - 1), (5, 9), (17, 30)] + [tuple(v) for v in rng.integers(0, size, size=(14, 2))]
    got, want = [], []
    for py, px in pix:
        y0, y1 = max(py - r, 0), min(py + r + 1, size)
        x0, x1 = max(px - r, 0), min(px + r + 1, size)
        xo = cnn.bf16_round(cnn.encode(phi32[y0:y1, x0:x1].astype(np.float64)[None], m[y0:y1, x0:x1][None]))
        yo, _ = cnn.forward(rp, xo)
        want.append(yo[0, py - y0, px - x0, :2])
        got.append(yg[py, px])
    got, want = np.array(got), np.array(want)
    scale = np.max(np.abs(want))
    err = float(np.max(np.abs(got - want)) / scale)
    c = float(got.ravel() @ want.ravel() / (np.linalg.norm(got) * np.linalg.norm(want)))
    print(f"  2048^2 inference at {len(pix)} pixels: max rel err {err:.2e}, cosine {c:.6f}", file=sys.stderr)
    assert err <= 6e-2 and c >= 0.998
    assert math.isfinite(err)
