"""FP64 reference of the warm-start network (test infrastructure only).

The network maps the sampled angles of an image to initial gap angles for the
Monte Carlo chain:
  input  x = (cos q phi, sin q phi, 1) at sampled sites, 0 at gaps, padded
         with zero channels to C = 32;
  stem   h = relu(conv(x) + b);
  8 residual blocks  h <- h + conv2(relu(conv1(h) + b1)) + b2;
  head   y = conv(h) + b, of which channels 0 and 1 are (cos q phi, sin q phi);
  loss   mean over gap sites of (y0 - c)^2 + (y1 - s)^2 for target angles.
Every conv is 3x3, stride 1, zero padding, C -> C channels; weights are
W[tap, c_in, c_out] with tap = 3 (dy + 1) + (dx + 1), so
  out[y, x, o] = b[o] + sum_{tap, i} in[y + dy, x + dx, i] W[tap, i, o].
Arrays are (N, H, W, C).  Plain numpy in float64: explicit loops over the
nine taps, no fusion.
"""
from __future__ import annotations

import numpy as np

C = 32
N_BLOCKS = 8
N_LAYERS = 2 + 2 * N_BLOCKS
TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shift(a: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """s[n, y, x] = a[n, y + dy, x + dx], zero outside the image."""
    n, h, w, c = a.shape
    out = np.zeros_like(a)
    ys, yd = slice(max(0, -dy), h - max(0, dy)), slice(max(0, dy), h - max(0, -dy))
    xs, xd = slice(max(0, -dx), w - max(0, dx)), slice(max(0, dx), w - max(0, -dx))
    out[:, ys, xs] = a[:, yd, xd]
    return out


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """3x3 convolution (cross-correlation) with zero padding."""
    out = np.zeros(x.shape[:3] + (W.shape[2],), dtype=np.float64)
    for t, (dy, dx) in enumerate(TAPS):
        out += shift(x, dy, dx) @ W[t]
    if b is not None:
        out += b
    return out


def conv_dgrad(g: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Gradient of conv with respect to its input, given the output gradient."""
    out = np.zeros(g.shape[:3] + (W.shape[1],), dtype=np.float64)
    for t, (dy, dx) in enumerate(TAPS):
        out += shift(g @ W[t].T, -dy, -dx)
    return out


def conv_wgrad(x: np.ndarray, g: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Gradients of conv with respect to W[tap, i, o] and b[o]."""
    dW = np.zeros((9, x.shape[3], g.shape[3]))
    for t, (dy, dx) in enumerate(TAPS):
        xs = shift(x, dy, dx)
        dW[t] = np.einsum("nyxi,nyxo->io", xs, g)
    return dW, g.sum(axis=(0, 1, 2))


def encode(phi: np.ndarray, sampled: np.ndarray, q: float = 0.5) -> np.ndarray:
    """(N, H, W) angles and masks -> (N, H, W, C) network input."""
    s = sampled.astype(np.float64)
    x = np.zeros(phi.shape + (C,))
    x[..., 0] = np.cos(q * phi) * s
    x[..., 1] = np.sin(q * phi) * s
    x[..., 2] = s
    return x


def decode(y: np.ndarray, q: float = 0.5) -> np.ndarray:
    """Head output (channels 0, 1 = cos, sin of q phi) -> angle in [0, 2 pi).

    sin(q phi) >= 0 for phi in [0, 2 pi], so the sine is clipped at 0; the
    result is capped just below 2 pi (the largest double below it)."""
    th = np.arctan2(np.maximum(y[..., 1], 0.0), y[..., 0])
    return np.minimum(th / q, np.nextafter(2.0 * np.pi, 0.0))


def init_params(seed: int) -> list[tuple[np.ndarray, np.ndarray]]:
    """He-normal weights; residual second convs and the head start small."""
    rng = np.random.default_rng(seed)
    layers = []
    for k in range(N_LAYERS):
        fan_in = 9 * (3 if k == 0 else C)
        W = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(9, C, C))
        if k == 0:
            W[:, 3:, :] = 0.0
        if k >= 2 and k % 2 == 0 and k < N_LAYERS - 1:
            W *= 0.1  # second conv of each residual block
        if k == N_LAYERS - 1:
            W *= 0.1
            W[:, :, 2:] = 0.0
        layers.append((W, np.zeros(C)))
    return layers


def forward(params, x: np.ndarray):
    """Returns the head output and the activations needed by backward."""
    acts = {}
    h = np.maximum(conv(x, *params[0]), 0.0)
    acts["x"], acts["h0"] = x, h
    for b in range(N_BLOCKS):
        W1, b1 = params[1 + 2 * b]
        W2, b2 = params[2 + 2 * b]
        t = np.maximum(conv(h, W1, b1), 0.0)
        acts[f"in{b}"], acts[f"t{b}"] = h, t
        h = h + conv(t, W2, b2)
    acts["hN"] = h
    return conv(h, *params[-1]), acts


def loss(y: np.ndarray, target: np.ndarray, gap: np.ndarray) -> tuple[float, np.ndarray]:
    """Mean over gap sites of the squared (cos, sin) error, and dL/dy."""
    g = gap.astype(np.float64)
    n = max(g.sum(), 1.0)
    d0 = (y[..., 0] - target[..., 0]) * g
    d1 = (y[..., 1] - target[..., 1]) * g
    L = float((d0 * d0 + d1 * d1).sum() / n)
    dy = np.zeros_like(y)
    dy[..., 0] = 2.0 * d0 / n
    dy[..., 1] = 2.0 * d1 / n
    return L, dy


def backward(params, acts, dy: np.ndarray):
    """Gradients (dW, db) for every layer, by the chain rule through forward."""
    grads = [None] * N_LAYERS
    grads[-1] = conv_wgrad(acts["hN"], dy)
    dh = conv_dgrad(dy, params[-1][0])
    for b in reversed(range(N_BLOCKS)):
        W2 = params[2 + 2 * b][0]
        W1 = params[1 + 2 * b][0]
        t, hin = acts[f"t{b}"], acts[f"in{b}"]
        grads[2 + 2 * b] = conv_wgrad(t, dh)
        dt = conv_dgrad(dh, W2) * (t > 0)
        grads[1 + 2 * b] = conv_wgrad(hin, dt)
        dh = dh + conv_dgrad(dt, W1)
    dh0 = dh * (acts["h0"] > 0)
    grads[0] = conv_wgrad(acts["x"], dh0)
    return grads


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
