"""Pins of the FP64 warm-start network oracle (oracle/cnn.py)."""
import math

import numpy as np
import pytest
import scipy.signal

from cnn_bf16 import backward_bf16, forward_bf16, network_case, rounded
from oracle import cnn


def rand(shape, seed):
    return np.random.default_rng(seed).normal(size=shape)


def test_conv_matches_scipy_correlate():
    """Each output channel is a sum of 2-D correlations with zero fill."""
    x = rand((2, 7, 9, 5), 1)
    W = rand((9, 5, 4), 2)
    b = rand(4, 3)
    out = cnn.conv(x, W, b)
    for n in range(2):
        for o in range(4):
            ref = np.full((7, 9), b[o])
            for i in range(5):
                K = W[:, i, o].reshape(3, 3)
                ref += scipy.signal.correlate2d(x[n, :, :, i], K, mode="same", boundary="fill")
            assert np.max(np.abs(out[n, :, :, o] - ref)) < 1e-12


def test_conv_gradients_by_finite_differences():
    """dgrad and wgrad against central differences of a linear functional."""
    x = rand((1, 5, 6, 3), 4)
    W = rand((9, 3, 2), 5)
    b = rand(2, 6)
    G = rand((1, 5, 6, 2), 7)

    def f(x_, W_, b_):
        return float((cnn.conv(x_, W_, b_) * G).sum())

    dx = cnn.conv_dgrad(G, W)
    dW, db = cnn.conv_wgrad(x, G)
    eps = 1e-6
    rng = np.random.default_rng(8)
    for _ in range(12):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        assert abs((f(xp, W, b) - f(xm, W, b)) / (2 * eps) - dx[idx]) < 1e-6
        idw = tuple(rng.integers(0, s) for s in W.shape)
        Wp, Wm = W.copy(), W.copy()
        Wp[idw] += eps
        Wm[idw] -= eps
        assert abs((f(x, Wp, b) - f(x, Wm, b)) / (2 * eps) - dW[idw]) < 1e-6
    for o in range(2):
        bp, bm = b.copy(), b.copy()
        bp[o] += eps
        bm[o] -= eps
        assert abs((f(x, W, bp) - f(x, W, bm)) / (2 * eps) - db[o]) < 1e-6


def test_network_backward_by_finite_differences():
    """Full residual network: every layer's gradient against central
    differences of the masked loss (relative error <= 1e-6)."""
    rng = np.random.default_rng(11)
    params = cnn.init_params(3)
    # enlarge the small-initialised layers so every path carries signal
    params = [(W * (3.0 if k % 2 == 0 and 0 < k < cnn.N_LAYERS - 1 else 1.0) + 0.0, b + rng.normal(0, 0.05, cnn.C))
              for k, (W, b) in enumerate(params)]
    params[-1][0][:, :, :2] += rng.normal(0, 0.05, size=(9, cnn.C, 2))
    phi = rng.uniform(0, 2 * math.pi, size=(1, 6, 7))
    sampled = (rng.random((1, 6, 7)) < 0.5)
    x = cnn.encode(phi, sampled)
    tgt_phi = rng.uniform(0, 2 * math.pi, size=(1, 6, 7))
    target = np.stack([np.cos(0.5 * tgt_phi), np.sin(0.5 * tgt_phi)], -1)
    gap = ~sampled

    def L(p):
        y, _ = cnn.forward(p, x)
        return cnn.loss(y, target, gap)[0]

    y, acts = cnn.forward(params, x)
    _, dy = cnn.loss(y, target, gap)
    grads = cnn.backward(params, acts, dy)
    eps = 1e-6
    for k in range(cnn.N_LAYERS):
        W, b = params[k]
        for _ in range(2):
            i = (rng.integers(0, 9), rng.integers(0, 3 if k == 0 else cnn.C), rng.integers(0, 2 if k == cnn.N_LAYERS - 1 else cnn.C))
            Wp, Wm = W.copy(), W.copy()
            Wp[i] += eps
            Wm[i] -= eps
            pp = list(params)
            pm = list(params)
            pp[k] = (Wp, b)
            pm[k] = (Wm, b)
            fd = (L(pp) - L(pm)) / (2 * eps)
            an = grads[k][0][i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, i, fd, an)
        o = rng.integers(0, 2 if k == cnn.N_LAYERS - 1 else cnn.C)
        bp, bm = b.copy(), b.copy()
        bp[o] += eps
        bm[o] -= eps
        pp, pm = list(params), list(params)
        pp[k] = (W, bp)
        pm[k] = (W, bm)
        fd = (L(pp) - L(pm)) / (2 * eps)
        assert abs(fd - grads[k][1][o]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, o)


def test_encode_decode_round_trip():
    rng = np.random.default_rng(5)
    phi = rng.uniform(0, 2 * math.pi, size=(2, 4, 5))
    s = np.ones((2, 4, 5), bool)
    x = cnn.encode(phi, s)
    assert np.all(x[..., 2] == 1.0) and np.all(x[..., 3:] == 0.0)
    back = cnn.decode(x)
    assert np.max(np.abs(back - phi)) < 1e-12
    s[0, 0, 0] = False
    x = cnn.encode(phi, s)
    assert np.all(x[0, 0, 0] == 0.0)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 3.14159265, -2.5e-3, 0.0])
    r = cnn.bf16_round(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    assert abs(r[3] - 3.140625) < 1e-12
    assert np.all(np.abs(r - v) <= np.abs(v) * 2 ** -8 + 1e-300)


def test_bf16_network_composition_matches_the_float64_network():
    """The bfloat16 composition the GPU network test uses is the float64
    network up to bfloat16 rounding: with the rounding replaced by the
    identity it is cnn.forward / cnn.backward exactly, and with it the output
    stays within a few bfloat16 steps of the float64 one."""
    params, phi, sampled, target = network_case(3)
    rp = rounded(params)
    x = cnn.bf16_round(cnn.encode(phi, sampled.astype(bool)))
    y64, acts64 = cnn.forward(rp, x)
    y16, _ = forward_bf16(rp, x)
    g, w = y16[..., :2].ravel(), y64[..., :2].ravel()
    assert np.max(np.abs(g - w)) / np.max(np.abs(w)) < 5e-2
    assert g @ w / (np.linalg.norm(g) * np.linalg.norm(w)) > 0.999
    ident = lambda a: np.asarray(a, dtype=np.float64)  # noqa: E731
    orig = cnn.bf16_round
    cnn.bf16_round = ident
    try:
        y_id, acts_id = forward_bf16(rp, x)
        _, dy = cnn.loss(y_id, target, sampled == 0)
        g_id = backward_bf16(rp, acts_id, dy)
    finally:
        cnn.bf16_round = orig
    assert np.array_equal(y_id, y64)
    g64 = cnn.backward(rp, acts64, dy)
    for (a, b), (c, d) in zip(g_id, g64):
        assert np.allclose(a, c, rtol=1e-12, atol=1e-15) and np.allclose(b, d, rtol=1e-12, atol=1e-15)
