"""CPU oracle for the learned angular reconstruction network.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark baseline).  Plain
numpy in double precision with BF16 round-to-nearest-even at exactly the
points where the HIP kernels store BF16: after each layer's activation, the
output, and each propagated gradient.  Shares no code with the HIP path.

Network (a stand-in for 4x angular supersampling, not in the paper): per
pixel, the V rendered views' (R, G, B, d) with d = D/Z - 1 (-1 for background)
form 4V input channels; four 3x3 convolutions 4V -> 32 -> 32 -> 32 -> 3V with
ReLU between them and zero padding; the output adds the input RGB of each
view (residual).  Weights are laid out [tap][cout][cin] with tap = 3*(dy+1) +
(dx+1) reading input pixel (y+dy, x+dx); biases [cout].

Pins (tests/test_net_oracle.py): finite differences of the double-precision
loss; zero weights make the output equal the input RGB; a 1x1 identity
kernel reproduces its input; convolution equals an explicit loop.
"""
from __future__ import annotations

import numpy as np


def bf16(x) -> np.ndarray:
    """Round to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def layer_shapes(V: int, hidden: int = 32):
    return [(4 * V, hidden), (hidden, hidden), (hidden, hidden), (hidden, 3 * V)]


def init_params(V: int, seed: int, hidden: int = 32, scale: float = 1.0):
    """He-style random weights (last layer scaled down), zero biases."""
    rng = np.random.default_rng(seed)
    ps = []
    for k, (ci, co) in enumerate(layer_shapes(V, hidden)):
        std = scale * np.sqrt(2.0 / (9 * ci)) * (0.1 if k == 3 else 1.0)
        ps.append((rng.normal(0.0, std, (9, co, ci)), np.zeros(co)))
    return ps


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Zero-padded 3x3 convolution: x (H, W, Cin), w (9, Cout, Cin), b (Cout)."""
    H, W, _ = x.shape
    xp = np.zeros((H + 2, W + 2, x.shape[2]))
    xp[1:-1, 1:-1] = x
    out = np.broadcast_to(b, (H, W, w.shape[1])).copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            tap = 3 * (dy + 1) + (dx + 1)
            out += xp[1 + dy:1 + dy + H, 1 + dx:1 + dx + W] @ w[tap].T
    return out


def conv3x3_wgrad(x: np.ndarray, dz: np.ndarray):
    """Gradients of conv3x3 w.r.t. w (9, Cout, Cin) and b."""
    H, W, _ = x.shape
    xp = np.zeros((H + 2, W + 2, x.shape[2]))
    xp[1:-1, 1:-1] = x
    dw = np.zeros((9, dz.shape[2], x.shape[2]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            tap = 3 * (dy + 1) + (dx + 1)
            xs = xp[1 + dy:1 + dy + H, 1 + dx:1 + dx + W].reshape(-1, x.shape[2])
            dw[tap] = dz.reshape(-1, dz.shape[2]).T @ xs
    return dw, dz.reshape(-1, dz.shape[2]).sum(axis=0)


def conv3x3_xgrad(dz: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient of conv3x3 w.r.t. its input: the transposed convolution."""
    H, W, _ = dz.shape
    dx_ = np.zeros((H + 2, W + 2, w.shape[2]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            tap = 3 * (dy + 1) + (dx + 1)
            dx_[1 + dy:1 + dy + H, 1 + dx:1 + dx + W] += dz @ w[tap]
    return dx_[1:-1, 1:-1]


def residual_rgb(x: np.ndarray, V: int) -> np.ndarray:
    """Input RGB of every view, in output channel order (3v + c)."""
    H, W, _ = x.shape
    return x.reshape(H, W, V, 4)[..., :3].reshape(H, W, 3 * V)


def forward(x: np.ndarray, params, V: int, round_bf16: bool = True):
    """Returns (pre-activations z1..z4, activations a0..a3, output y)."""
    r = bf16 if round_bf16 else (lambda v: np.asarray(v, np.float64))
    a = [r(x)]
    zs = []
    for k, (w, b) in enumerate(params):
        w = r(w)
        z = conv3x3(a[-1], w, b)
        zs.append(z)
        if k < 3:
            a.append(r(np.maximum(z, 0.0)))
    y = r(zs[-1] + residual_rgb(a[0], V))
    return zs, a, y


def loss_and_grads(x: np.ndarray, target: np.ndarray, params, V: int, round_bf16: bool = True):
    """MSE loss over all output values and gradients of every weight/bias."""
    r = bf16 if round_bf16 else (lambda v: np.asarray(v, np.float64))
    zs, a, y = forward(x, params, V, round_bf16)
    n = y.size
    diff = y - target
    loss = float((diff * diff).mean())
    dz = r(2.0 * diff / n)
    grads = [None] * 4
    for k in (3, 2, 1, 0):
        w = r(params[k][0])
        dw, db = conv3x3_wgrad(a[k], dz)
        grads[k] = (dw, db)
        if k > 0:
            da = conv3x3_xgrad(dz, w)
            dz = r(da * (a[k] > 0))
    return loss, grads, y


def adam(params, grads, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    out = []
    for k in range(len(params)):
        pw, pb = params[k]
        gw, gb = grads[k]
        nw = []
        for p_, g_, key in ((pw, gw, (k, 0)), (pb, gb, (k, 1))):
            m[key] = b1 * m.get(key, 0.0) + (1 - b1) * g_
            v[key] = b2 * v.get(key, 0.0) + (1 - b2) * g_ * g_
            mh = m[key] / (1 - b1 ** step)
            vh = v[key] / (1 - b2 ** step)
            nw.append(p_ - lr * mh / (np.sqrt(vh) + eps))
        out.append((nw[0], nw[1]))
    return out
