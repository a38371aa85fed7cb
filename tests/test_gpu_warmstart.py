"""What the trained warm start gains over the plain random start.

The committed network (trained on the library's own simulations of 256^2
images) is applied to fresh 1024^2 images in the paper's layout (one chain of
M = 100 states): the chains with the learned start must stop in fewer sweeps,
fill faster and reach the same prediction MAE, within 1% of the plain
start's on both mask kinds.  With M as 100 chains of one state each, every
chain would start from the same network output and its single state would
stay correlated with it; the library refuses that warm start.
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
    fields = warmstart.make_eval_fields(size=1024, seeds=8, workers=0)
    ctx = mpr.Context(0)
    model = warmstart.WarmStart(ctx, params)
    s = warmstart.evaluate(ctx, model, fields, layouts=((1, 100), (100, 1)))
    ctx.close()
    print(s)
    for kind in ("random", "cloud"):
        r = s["1x100"][kind]
        assert r["sweeps_warm"] < r["sweeps_plain"]
        assert r["time_to_fill_warm_s"] < r["time_to_fill_plain_s"]
        assert abs(r["mae_warm_over_plain"] - 1.0) <= 0.01, (kind, r["mae_warm_over_plain"], r["mae_ratio_ci95"])
        assert "refused" in s["100x1"][kind]["warm"]


def test_warm_start_with_one_state_per_chain_is_refused():
    """(R, K) = (100, 1): mpr_simulate returns MPR_ERR_ARG for phi_init, as
    for any K below warm_min_states (100); with the check off it runs."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    z, m = warmstart._eval_field(("random", 64, 0))
    ctx = mpr.Context(0)
    try:
        imgs = mpr.images([(64, 64)])
        zd, md = torch.from_numpy(z).cuda(), torch.from_numpy(m).cuda()
        phi = torch.empty_like(zd)
        ctx.map_to_angles(imgs, zd, md, phi)
        init = torch.full_like(phi, 1.0)
        for R, K in ((100, 1), (4, 25), (2, 50), (1, 99)):
            prm = mpr.default_params(R=R, K=K)
            ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
            with pytest.raises(mpr.MprError) as e:
                ctx.simulate(imgs, phi, md, np.array([0.05]), prm, ws, torch.empty_like(phi), phi_init=init)
            assert e.value.code == mpr.MPR_ERR_ARG and "warm_min_states" in str(e.value)
        prm = mpr.default_params(R=1, K=100)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        ctx.simulate(imgs, phi, md, np.array([0.05]), prm, ws, torch.empty_like(phi), phi_init=init)
        prm = mpr.default_params(R=100, K=1, warm_min_states=0)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        ctx.simulate(imgs, phi, md, np.array([0.05]), prm, ws, torch.empty_like(phi), phi_init=init)
    finally:
        ctx.close()


def test_warm_start_inference_at_full_size_sampled_pixels():
    """The committed network on a 2048 x 2048 evaluation image (50% random
    gaps), checked at sampled pixels: 18 stacked 3x3 convolutions make an
    output pixel depend on the input within 18 pixels, so the oracle computes
    it from that crop of the same bfloat16 input (zero padding at the image
    edges, as on the GPU), with bfloat16 storage between layers as on the GPU
    (inside the crop's valid cone every value is the full image's).  Bar:
    max error 2e-2 of the largest output magnitude, cosine >= 0.999."""
    import math
    import sys

    import oracle
    from cnn_bf16 import forward_bf16
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
        yo, _ = forward_bf16(rp, xo)
        want.append(yo[0, py - y0, px - x0, :2])
        got.append(yg[py, px])
    got, want = np.array(got), np.array(want)
    scale = np.max(np.abs(want))
    err = float(np.max(np.abs(got - want)) / scale)
    c = float(got.ravel() @ want.ravel() / (np.linalg.norm(got) * np.linalg.norm(want)))
    print(f"  2048^2 inference at {len(pix)} pixels: max rel err {err:.2e}, cosine {c:.6f}", file=sys.stderr)
    assert err <= 2e-2 and c >= 0.999
    assert math.isfinite(err)
