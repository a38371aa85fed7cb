"""The oracle's warm-start network composed with bfloat16 storage between
layers, as the GPU kernels store their activations and gradient maps (test
infrastructure: built from the oracle's layer functions only)."""
import math

import numpy as np

from oracle import cnn


def rounded(params):
    """The oracle's view of the packed weights: W in bfloat16, b in float32."""
    return [(cnn.bf16_round(W), np.float32(b).astype(np.float64)) for W, b in params]


def network_case(seed, n=2, h=20, w=36):
    rng = np.random.default_rng(seed)
    params = cnn.init_params(seed)
    # larger residual branches than the initialisation, so every layer matters
    params = [(W * (3.0 if k % 2 == 0 and 0 < k < cnn.N_LAYERS - 1 else 1.0), b + rng.normal(0, 0.02, 32))
              for k, (W, b) in enumerate(params)]
    params[-1][0][:, :, :2] += rng.normal(0, 0.05, size=(9, 32, 2))
    phi = rng.uniform(0, 2 * math.pi, size=(n, h, w))
    sampled = (rng.random((n, h, w)) < 0.5).astype(np.uint8)
    tphi = rng.uniform(0, 2 * math.pi, size=(n, h, w))
    target = np.stack([np.cos(0.5 * tphi), np.sin(0.5 * tphi)], -1)
    return params, phi, sampled, target


def forward_bf16(params, x):
    """The oracle's forward pass with activations stored in bfloat16 where
    the kernels store them: after the stem, after each block's first conv
    (ReLU applied), after each residual sum, and at the head."""
    r = cnn.bf16_round
    acts = {"x": x}
    h = r(np.maximum(cnn.conv(x, *params[0]), 0.0))
    acts["h0"] = h
    for b in range(cnn.N_BLOCKS):
        t = r(np.maximum(cnn.conv(h, *params[1 + 2 * b]), 0.0))
        acts[f"in{b}"], acts[f"t{b}"] = h, t
        h = r(cnn.conv(t, *params[2 + 2 * b]) + h)
    acts["hN"] = h
    return r(cnn.conv(h, *params[-1])), acts


def backward_bf16(params, acts, dy):
    """The oracle's chain rule in the kernels' order, with each gradient map
    rounded to bfloat16 where the kernels store it; weight gradients stay
    unrounded (the kernels accumulate them in float32)."""
    r = cnn.bf16_round
    grads = [None] * cnn.N_LAYERS
    grads[-1] = cnn.conv_wgrad(acts["hN"], dy)
    dh = r(cnn.conv_dgrad(dy, params[-1][0]))
    for b in reversed(range(cnn.N_BLOCKS)):
        t, hin = acts[f"t{b}"], acts[f"in{b}"]
        grads[2 + 2 * b] = cnn.conv_wgrad(t, dh)
        dt = r(cnn.conv_dgrad(dh, params[2 + 2 * b][0]) * (t > 0))
        grads[1 + 2 * b] = cnn.conv_wgrad(hin, dt)
        dh = r(dh + cnn.conv_dgrad(dt, params[1 + 2 * b][0]))
    grads[0] = cnn.conv_wgrad(acts["x"], dh * (acts["h0"] > 0))
    return grads
