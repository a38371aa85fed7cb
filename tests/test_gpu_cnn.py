"""GPU parity of the warm-start network kernels against the FP64 oracle.

The oracle runs on the same bfloat16-rounded inputs and weights the kernels
see.  Every comparison: max error <= 2e-2 of the output's largest magnitude
and cosine similarity >= 0.999.  For the whole network the test composes the
oracle's layer functions with the same bfloat16 storage between layers as the
kernels (activations, the loss gradient and the backpropagated gradients are
rounded to bfloat16 where the kernels store them), so that both sides see
the same inputs at every layer.
"""
import math
import sys

import numpy as np
import pytest

from cnn_bf16 import backward_bf16, forward_bf16, network_case, rounded
from oracle import cnn

torch = pytest.importorskip("torch")
import paper_1811_01604_amd as mpr  # noqa: E402

pytestmark = pytest.mark.gpu
WSZ = 9 * 32 * 32


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mpr.Context(0)
    yield c
    c.close()


def to_bf16(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda").to(torch.bfloat16)


def from_dev(t):
    return t.float().cpu().numpy().astype(np.float64)


def flat_params(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)


def close(got, want, rel=2e-2, cos=0.999):
    g, w = got.ravel(), want.ravel()
    scale = max(np.max(np.abs(w)), 1e-30)
    err = np.max(np.abs(g - w)) / scale
    c = float(g @ w / (np.linalg.norm(g) * np.linalg.norm(w) + 1e-300))
    assert err <= rel and c >= cos, (err, c)
    return err, c


def packs(ctx, params):
    p = torch.from_numpy(flat_params(params)).cuda()
    packed = torch.empty(ctx.cnn_packed_bytes() // 2, dtype=torch.bfloat16, device="cuda")
    ctx.cnn_pack(p, packed)
    return p, packed


def layer_params(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    params = [(rng.normal(0, scale, size=(9, 32, 32)), rng.normal(0, 0.1, size=32)) for _ in range(cnn.N_LAYERS)]
    return params


@pytest.mark.parametrize("shape", [(1, 8, 32), (2, 19, 45), (1, 33, 70)])
def test_conv_forward_and_epilogues(ctx, shape):
    n, h, w = shape
    say("conv forward", shape)
    rng = np.random.default_rng(h * w)
    params = layer_params(1)
    p, packed = packs(ctx, params)
    rp = rounded(params)
    k = 5
    x = cnn.bf16_round(rng.normal(size=(n, h, w, 32)))
    add = cnn.bf16_round(rng.normal(size=(n, h, w, 32)))
    ref = cnn.bf16_round(rng.normal(size=(n, h, w, 32)))
    xd, addd, refd = to_bf16(x), to_bf16(add), to_bf16(ref)
    fwd = packed[k * 2 * WSZ: k * 2 * WSZ + WSZ]
    bias = p[k * (WSZ + 32) + WSZ: (k + 1) * (WSZ + 32)]
    W, b = rp[k]
    out = torch.empty_like(xd)
    ctx.cnn_diag_conv(xd, fwd, bias, out)
    close(from_dev(out), cnn.conv(x, W, b))
    ctx.cnn_diag_conv(xd, fwd, bias, out, relu=True)
    close(from_dev(out), np.maximum(cnn.conv(x, W, b), 0))
    ctx.cnn_diag_conv(xd, fwd, bias, out, add=addd)
    close(from_dev(out), cnn.conv(x, W, b) + add)
    ctx.cnn_diag_conv(xd, fwd, None, out, ref=refd)
    close(from_dev(out), cnn.conv(x, W) * (ref > 0))
    ctx.cnn_diag_conv(xd, fwd, bias, out, add=addd, ref=refd, relu=True)
    close(from_dev(out), np.maximum(cnn.conv(x, W, b) + add, 0) * (ref > 0))


@pytest.mark.parametrize("shape", [(2, 19, 45), (1, 40, 64)])
def test_conv_input_and_weight_gradients(ctx, shape):
    n, h, w = shape
    say("conv gradients", shape)
    rng = np.random.default_rng(7 + h)
    params = layer_params(2)
    p, packed = packs(ctx, params)
    rp = rounded(params)
    k = 9
    W, _ = rp[k]
    x = cnn.bf16_round(rng.normal(size=(n, h, w, 32)))
    g = cnn.bf16_round(rng.normal(size=(n, h, w, 32)))
    ref = cnn.bf16_round(rng.normal(size=(n, h, w, 32)))
    xd, gd, refd = to_bf16(x), to_bf16(g), to_bf16(ref)
    dgrad = packed[k * 2 * WSZ + WSZ: (k + 1) * 2 * WSZ]
    out = torch.empty_like(xd)
    ctx.cnn_diag_conv(gd, dgrad, None, out)
    close(from_dev(out), cnn.conv_dgrad(g, W))
    ws = torch.empty(256 * 4 * (WSZ + 32) * 4, dtype=torch.uint8, device="cuda")
    grads = torch.zeros(WSZ + 32, dtype=torch.float32, device="cuda")
    ctx.cnn_diag_wgrad(xd, gd, grads, ws)
    dW, db = cnn.conv_wgrad(x, g)
    gr = grads.cpu().numpy().astype(np.float64)
    close(gr[:WSZ].reshape(9, 32, 32), dW, rel=1e-3, cos=0.99999)
    close(gr[WSZ:], db, rel=1e-3, cos=0.99999)
    ctx.cnn_diag_wgrad(xd, gd, grads, ws, gref=refd)
    dW, db = cnn.conv_wgrad(x, g * (ref > 0))
    gr = grads.cpu().numpy().astype(np.float64)
    close(gr[:WSZ].reshape(9, 32, 32), dW, rel=1e-3, cos=0.99999)


def test_network_forward_loss_backward(ctx):
    """Forward, loss and backward of the whole network against the oracle's
    composition with the kernels' bfloat16 storage: the head output and every
    layer's weight and bias gradients within 2e-2 of their largest magnitude,
    cosine >= 0.999."""
    params, phi, sampled, target = network_case(3)
    n, h, w = phi.shape
    p, packed = packs(ctx, params)
    rp = rounded(params)
    phid = torch.from_numpy(phi.astype(np.float32)).cuda()
    sd = torch.from_numpy(sampled).cuda()
    x = torch.empty((n, h, w, 32), dtype=torch.bfloat16, device="cuda")
    ctx.cnn_encode(phid, sd, x)
    xo = cnn.bf16_round(cnn.encode(phi.astype(np.float32).astype(np.float64), sampled.astype(bool)))
    close(from_dev(x), xo, rel=1e-6, cos=0.999999)
    ws = torch.empty(ctx.cnn_workspace_size(n, h, w, True), dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    ctx.cnn_forward(p, packed, x, ws, y, training=True)
    yo, acts = forward_bf16(rp, xo)
    err, c = close(from_dev(y)[..., :2], yo[..., :2])
    say(f"  forward: max rel err {err:.2e}, cosine {c:.6f}")
    gap = sampled == 0
    dy = torch.empty_like(x)
    lw = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    L = ctx.cnn_loss(y, torch.from_numpy(target.astype(np.float32)).cuda(), sd, int(gap.sum()), dy, lw)
    Lo, dyo = cnn.loss(yo, target.astype(np.float32).astype(np.float64), gap)
    say(f"  loss gpu {L:.6f} oracle {Lo:.6f}")
    assert abs(L / Lo - 1) < 1e-3
    dyo = cnn.bf16_round(dyo)
    close(from_dev(dy)[..., :2], dyo[..., :2])
    grads = torch.zeros(ctx.cnn_param_count(), dtype=torch.float32, device="cuda")
    ctx.cnn_backward(p, packed, x, dy, ws, grads)
    go = backward_bf16(rp, acts, dyo)
    g = grads.cpu().numpy().astype(np.float64).reshape(cnn.N_LAYERS, WSZ + 32)
    worst_err, worst_cos = 0.0, 1.0
    for k in range(cnn.N_LAYERS):
        gw = g[k, :WSZ].reshape(9, 32, 32)
        ow = go[k][0]
        gb, ob = g[k, WSZ:], go[k][1]
        if k == 0:
            gw, ow = gw[:, :3], ow[:, :3]
        if k == cnn.N_LAYERS - 1:
            gw, ow, gb, ob = gw[..., :2], ow[..., :2], gb[:2], ob[:2]
        for got, want in ((gw, ow), (gb, ob)):
            e, c = close(got, want)
            worst_err, worst_cos = max(worst_err, e), min(worst_cos, c)
    say(f"  backward: worst per-layer max rel err {worst_err:.2e}, cosine {worst_cos:.6f}")
    # unused channels stay exactly zero
    assert np.all(g[0, :WSZ].reshape(9, 32, 32)[:, 3:] == 0)
    assert np.all(g[-1, :WSZ].reshape(9, 32, 32)[..., 2:] == 0)
    assert np.all(g[-1, WSZ + 2:] == 0)


@pytest.mark.parametrize("shape", [(1, 8, 32), (2, 37, 61), (1, 14, 30), (1, 15, 31), (3, 71, 100)])
def test_fused_residual_blocks_equal_the_layer_by_layer_forward(ctx, shape):
    """Inference runs each residual block as one kernel (the inner
    activation in LDS, rounded to bfloat16 as the layer-by-layer path stores
    it); the training forward runs the convs one by one.  Their outputs must
    be the same bits, on shapes smaller than, equal to, one more than and
    several times the 14 x 30 output tile, and the inference output meets
    the oracle's bar."""
    n, h, w = shape
    params = layer_params(7 + h, scale=0.15)
    p, packed = packs(ctx, params)
    rng = np.random.default_rng(w)
    xo = cnn.bf16_round(rng.normal(0, 1, size=(n, h, w, 32)))
    x = to_bf16(xo)
    y_inf, y_train = torch.empty_like(x), torch.empty_like(x)
    ws_i = torch.empty(ctx.cnn_workspace_size(n, h, w, False), dtype=torch.uint8, device="cuda")
    ws_t = torch.empty(ctx.cnn_workspace_size(n, h, w, True), dtype=torch.uint8, device="cuda")
    ctx.cnn_forward(p, packed, x, ws_i, y_inf, training=False)
    ctx.cnn_forward(p, packed, x, ws_t, y_train, training=True)
    torch.cuda.synchronize()
    a = y_inf.view(torch.int16).cpu().numpy()
    b = y_train.view(torch.int16).cpu().numpy()
    assert np.array_equal(a, b), int((a != b).sum())
    yo, _ = forward_bf16(rounded(params), xo)
    err, c = close(from_dev(y_inf), yo)
    say(f"  {shape}: bit-equal; against the oracle max rel err {err:.2e}, cosine {c:.6f}")


@pytest.mark.parametrize("shape", [(1, 8, 32), (2, 37, 61), (1, 100, 130)])
def test_fused_inference_equals_encode_forward_decode(ctx, shape):
    """mpr_cnn_infer (the encoding done while the stem stages its input, the
    decoding in the head's epilogue) gives the starting angles of
    mpr_cnn_encode, mpr_cnn_forward and mpr_cnn_decode bit for bit."""
    n, h, w = shape
    params = layer_params(11 + w, scale=0.15)
    p, packed = packs(ctx, params)
    rng = np.random.default_rng(h)
    phi = torch.from_numpy(rng.uniform(0, 2 * np.pi, size=shape).astype(np.float32)).cuda()
    sd = torch.from_numpy((rng.random(shape) < 0.4).astype(np.uint8)).cuda()
    ws = torch.empty(ctx.cnn_workspace_size(n, h, w, False), dtype=torch.uint8, device="cuda")
    x = torch.empty((n, h, w, 32), dtype=torch.bfloat16, device="cuda")
    y = torch.empty_like(x)
    a = torch.full_like(phi, -1.0)
    b = torch.full_like(phi, -2.0)
    ctx.cnn_encode(phi, sd, x)
    ctx.cnn_forward(p, packed, x, ws, y, training=False)
    ctx.cnn_decode(y, sd, a)
    ctx.cnn_infer(p, packed, phi, sd, ws, b)
    torch.cuda.synchronize()
    av, bv = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(av.view(np.uint32), bv.view(np.uint32)), int((av != bv).sum())
    assert np.all(bv[sd.cpu().numpy() == 1] == 0)


def test_decode_matches_oracle(ctx):
    rng = np.random.default_rng(4)
    n, h, w = 1, 9, 40
    yv = cnn.bf16_round(rng.normal(size=(n, h, w, 32)))
    sampled = (rng.random((n, h, w)) < 0.3).astype(np.uint8)
    phi = torch.empty((n, h, w), dtype=torch.float32, device="cuda")
    ctx.cnn_decode(to_bf16(yv), torch.from_numpy(sampled).cuda(), phi)
    want = cnn.decode(yv)
    got = phi.cpu().numpy().astype(np.float64)
    g = sampled == 0
    assert np.max(np.abs(got[g] - want[g])) < 1e-5
    assert np.all(got[~g] == 0) and np.all((got[g] >= 0) & (got[g] < 2 * math.pi))


def test_training_steps_reduce_the_loss(ctx):
    """A few Adam steps on a fixed small batch drive the masked loss down."""
    import synth
    n, h, w = 4, 32, 32
    phis, masks = [], []
    for i in range(n):
        z = synth.matern_field(w, h, 2.5, 0.15, 0.0, 1.0, 40 + i)
        phis.append(2 * math.pi * (z - z.min()) / (z.max() - z.min()))
        masks.append(synth.random_mask(w, h, 0.5, 50 + i))
    phi = np.stack(phis)
    sampled = np.stack(masks)
    target = np.stack([np.cos(0.5 * phi), np.sin(0.5 * phi)], -1).astype(np.float32)
    params = cnn.init_params(5)
    p = torch.from_numpy(flat_params(params)).cuda()
    packed = torch.empty(ctx.cnn_packed_bytes() // 2, dtype=torch.bfloat16, device="cuda")
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    grads = torch.zeros_like(p)
    phid = torch.from_numpy(phi.astype(np.float32)).cuda()
    sd = torch.from_numpy(sampled).cuda()
    x = torch.empty((n, h, w, 32), dtype=torch.bfloat16, device="cuda")
    ctx.cnn_encode(phid, sd, x)
    ws = torch.empty(ctx.cnn_workspace_size(n, h, w, True), dtype=torch.uint8, device="cuda")
    y, dy = torch.empty_like(x), torch.empty_like(x)
    lw = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    tg = torch.from_numpy(target).cuda()
    ng = int((sampled == 0).sum())
    losses = []
    for step in range(1, 61):
        ctx.cnn_pack(p, packed)
        ctx.cnn_forward(p, packed, x, ws, y, training=True)
        losses.append(ctx.cnn_loss(y, tg, sd, ng, dy, lw))
        ctx.cnn_backward(p, packed, x, dy, ws, grads)
        ctx.cnn_opt_step(p, grads, m, v, step, lr=2e-3)
    say(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.3 * losses[0]
