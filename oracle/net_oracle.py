"""CPU oracle for the learned angular reconstruction network.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark baseline).  Plain
numpy in double precision with BF16 round-to-nearest-even at exactly the
points where the HIP kernels store BF16: after each layer's activation, the
output, and each propagated gradient.  Shares no code with the HIP path.

Network (a stand-in for 4x angular supersampling, not in the paper): it is
applied to each view v of a frame separately.  4x angular supersampling
followed by the angular filter (Sec. 4) averages sub-views within about one
view interval of view v; a surface at disparity d (d = D/Z - 1) moves by k*d
pixels horizontally per view step (k = fx * 2 tan(cone/2) / V), so the
average is, away from occlusions, a horizontal blur of width proportional to
|d|.  The network therefore sees:

* the disparity blur of view v: sum over t in {-1, -3/4, .., 1} of
  w(t) * view_v(x + t*k*d, y), linear interpolation along x with the border
  pixel repeated, w(t) the angular filter's Gaussian profile (sigma = half a
  view) normalised; pixels with d <= -1 (empty) are not moved;
* (R, G, B, d) of views v-2 .. v+2 (zero beyond the rig),

24 channels in all; four zero-padded 3x3 convolutions 24 -> 32 -> 32 -> 32
-> 3 with ReLU between them, dilated horizontally by 1, 3, 9, 1; the output
adds the blurred RGB (residual).  Weights are laid out [tap][cout][cin] with
tap = 3*(dy+1) + (dx+1) reading input pixel (y+dy, x+dil*dx); biases [cout].

The blur is defined in binary32 with a fixed operation order (below), so it is
reproduced exactly; everything after it is checked within BF16 tolerances.

Pins (tests/test_net_oracle.py): finite differences of the double-precision
loss; zero weights make the output equal the blurred input; a 1x1 identity
kernel reproduces its input; convolution equals an explicit loop; the input
assembly reads the right neighbour views; the blur is the identity at zero
disparity, keeps constants and linear ramps, its impulse response is the
Gaussian profile, and it equals a per-pixel double-precision loop.
"""
from __future__ import annotations

import math

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


NEIGH = 2                 # views v-2 .. v+2
CIN0 = 4 * (2 * NEIGH + 1) + 4  # 24 input channels: five views' (R, G, B, d), blurred RGB of view v, 0
BLUR_T = tuple((j - 4) / 4.0 for j in range(9))  # tap offsets in view steps
DILATION = (1, 3, 9, 1)   # horizontal dilation of the four layers (receptive field +-14 px across, +-4 down)


def layer_shapes(hidden: int = 32):
    return [(CIN0, hidden), (hidden, hidden), (hidden, hidden), (hidden, 3)]


def init_params(seed: int, hidden: int = 32, scale: float = 1.0):
    """He-style random weights (last layer scaled down), zero biases."""
    rng = np.random.default_rng(seed)
    ps = []
    for k, (ci, co) in enumerate(layer_shapes(hidden)):
        std = scale * np.sqrt(2.0 / (9 * ci)) * (0.1 if k == 3 else 1.0)
        ps.append((rng.normal(0.0, std, (9, co, ci)), np.zeros(co)))
    return ps


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray, dil: int = 1) -> np.ndarray:
    """Zero-padded 3x3 convolution with horizontal dilation `dil`: tap (dy, dx)
    reads pixel (y + dy, x + dil*dx).  x (H, W, Cin), w (9, Cout, Cin), b (Cout)."""
    H, W, _ = x.shape
    xp = np.zeros((H + 2, W + 2 * dil, x.shape[2]))
    xp[1:-1, dil:dil + W] = x
    out = np.broadcast_to(b, (H, W, w.shape[1])).copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            tap = 3 * (dy + 1) + (dx + 1)
            out += xp[1 + dy:1 + dy + H, dil + dil * dx:dil + dil * dx + W] @ w[tap].T
    return out


def conv3x3_wgrad(x: np.ndarray, dz: np.ndarray, dil: int = 1):
    """Gradients of conv3x3 w.r.t. w (9, Cout, Cin) and b."""
    H, W, _ = x.shape
    xp = np.zeros((H + 2, W + 2 * dil, x.shape[2]))
    xp[1:-1, dil:dil + W] = x
    dw = np.zeros((9, dz.shape[2], x.shape[2]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            tap = 3 * (dy + 1) + (dx + 1)
            xs = xp[1 + dy:1 + dy + H, dil + dil * dx:dil + dil * dx + W].reshape(-1, x.shape[2])
            dw[tap] = dz.reshape(-1, dz.shape[2]).T @ xs
    return dw, dz.reshape(-1, dz.shape[2]).sum(axis=0)


def conv3x3_xgrad(dz: np.ndarray, w: np.ndarray, dil: int = 1) -> np.ndarray:
    """Gradient of conv3x3 w.r.t. its input: the transposed convolution."""
    H, W, _ = dz.shape
    dx_ = np.zeros((H + 2, W + 2 * dil, w.shape[2]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            tap = 3 * (dy + 1) + (dx + 1)
            dx_[1 + dy:1 + dy + H, dil + dil * dx:dil + dil * dx + W] += dz @ w[tap]
    return dx_[1:-1, dil:dil + W]


def blur_weights() -> np.ndarray:
    """Tap weights of the disparity blur: the integers round(65535 exp(-t^2 /
    (2 * 0.5^2))) (the angular filter's profile), each divided by their sum in
    binary32."""
    wi = [int(round(65535.0 * math.exp(-t * t / 0.5))) for t in BLUR_T]
    tot = np.float32(sum(wi))
    return np.array([np.float32(w) / tot for w in wi], np.float32)


def disparity_blur(x: np.ndarray, k: float) -> np.ndarray:
    """Compact input (V, H, W, 4), BF16 values -> (V, H, W, 4) BF16 (blurred R,
    G, B, 0).  Binary32 steps per pixel (x, y) of view v, with s = k*d if d > -1
    else 0: for each tap t in order, u = min(max(x + t*s, -1), W), x0 =
    floor(u), f = u - x0, c = (1 - f)*C[clamp(x0)] + f*C[clamp(x0 + 1)] (clamp
    to 0..W-1), acc = acc + w_t*c; the result is rounded to BF16."""
    x32 = np.asarray(x, np.float32)
    V, H, W, _ = x32.shape
    d = x32[..., 3]
    s = np.where(d > np.float32(-1.0), np.float32(k) * d, np.float32(0.0)).astype(np.float32)
    wn = blur_weights()
    xs = np.arange(W, dtype=np.float32)[None, None, :]
    vi = np.arange(V)[:, None, None]
    yi = np.arange(H)[None, :, None]
    acc = np.zeros((V, H, W, 3), np.float32)
    for j, t in enumerate(BLUR_T):
        u = xs + np.float32(t) * s
        u = np.minimum(np.maximum(u, np.float32(-1.0)), np.float32(W))
        fl = np.floor(u)
        f = (u - fl)[..., None]
        i0 = fl.astype(np.int64)
        c0 = x32[vi, yi, np.clip(i0, 0, W - 1), :3]
        c1 = x32[vi, yi, np.clip(i0 + 1, 0, W - 1), :3]
        val = (np.float32(1.0) - f) * c0 + f * c1
        acc = acc + wn[j] * val
    out = np.zeros((V, H, W, 4), np.float64)
    out[..., :3] = bf16(acc)
    return out


def assemble(x: np.ndarray, xb: np.ndarray = None) -> np.ndarray:
    """Compact per-view input (V, H, W, 4) and its blur (V, H, W, 4) ->
    per-view network input (V, H, W, 24): views v-2 .. v+2 in that order (zero
    beyond the rig), then the blur of view v (no blur given: zeros)."""
    V, H, W, _ = x.shape
    out = np.zeros((V, H, W, CIN0))
    for v in range(V):
        for k, off in enumerate(range(-NEIGH, NEIGH + 1)):
            if 0 <= v + off < V:
                out[v, :, :, 4 * k:4 * k + 4] = x[v + off]
        if xb is not None:
            out[v, :, :, 20:24] = xb[v]
    return out


def forward(x: np.ndarray, params, round_bf16: bool = True, dil=DILATION, k: float = 0.0):
    """x: compact input (V, H, W, 4), k the disparity scale (pixels per view
    step per unit d).  Returns (pre-activations per layer, activations a0..a3
    with a0 the assembled input, output y (V, H, W, 3))."""
    r = bf16 if round_bf16 else (lambda v: np.asarray(v, np.float64))
    x = r(x)
    xb = disparity_blur(x, k)
    a = [assemble(x, xb)]
    zs = []
    for k, (w, b) in enumerate(params):
        w = r(w)
        z = np.stack([conv3x3(a[-1][v], w, b, dil[k]) for v in range(x.shape[0])])
        zs.append(z)
        if k < 3:
            a.append(r(np.maximum(z, 0.0)))
    y = r(zs[-1] + xb[..., :3])
    return zs, a, y


def loss_and_grads(x: np.ndarray, target: np.ndarray, params, round_bf16: bool = True, dil=DILATION,
                   k: float = 0.0):
    """MSE loss over all output values (V, H, W, 3) and the gradients of every
    weight and bias."""
    r = bf16 if round_bf16 else (lambda v: np.asarray(v, np.float64))
    zs, a, y = forward(x, params, round_bf16, dil, k)
    n = y.size
    diff = y - target
    loss = float((diff * diff).mean())
    dz = r(2.0 * diff / n)
    grads = [None] * 4
    V = x.shape[0]
    for k in (3, 2, 1, 0):
        w = r(params[k][0])
        dw = np.zeros_like(params[k][0], dtype=np.float64)
        db = np.zeros_like(params[k][1], dtype=np.float64)
        for v in range(V):
            gw, gb = conv3x3_wgrad(a[k][v], dz[v], dil[k])
            dw += gw
            db += gb
        grads[k] = (dw, db)
        if k > 0:
            da = np.stack([conv3x3_xgrad(dz[v], w, dil[k]) for v in range(V)])
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
