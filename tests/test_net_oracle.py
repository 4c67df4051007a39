"""Pins of the network oracle: finite differences, identities, explicit loops."""
import math

import numpy as np
import pytest

from oracle import net_oracle as N


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 1e-40, 3.0e38])
    got = N.bf16(x)
    assert got[0] == 1.0 and got[1] == 1.0  # tie to even
    assert got[2] == 1.0 + 2 ** -7           # above the tie rounds up
    assert got[3] == -2.5 and got[4] == 0.0


@pytest.mark.parametrize("dil", [1, 2, 3])
def test_conv_matches_explicit_loop(dil):
    rng = np.random.default_rng(0)
    x = rng.normal(size=(5, 6, 3))
    w = rng.normal(size=(9, 4, 3))
    b = rng.normal(size=4)
    out = N.conv3x3(x, w, b, dil)
    for y in range(5):
        for xx in range(6):
            acc = b.copy()
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    yy, xs = y + dy, xx + dil * dx
                    if 0 <= yy < 5 and 0 <= xs < 6:
                        acc += w[3 * (dy + 1) + (dx + 1)] @ x[yy, xs]
            np.testing.assert_allclose(out[y, xx], acc, rtol=1e-12, atol=1e-12)


def test_zero_weights_give_identity():
    rng = np.random.default_rng(1)
    x = N.bf16(rng.random((5, 4, 6, 4)))
    params = [(np.zeros((9, co, ci)), np.zeros(co)) for ci, co in N.layer_shapes(8)]
    _, _, y = N.forward(x, params)          # no disparity scale: the input RGB
    np.testing.assert_array_equal(y, x[..., :3])
    _, a, y = N.forward(x, params, k=3.0)   # with one: the blurred RGB
    np.testing.assert_array_equal(y, N.disparity_blur(x, 3.0)[..., :3])
    np.testing.assert_array_equal(a[0][..., 20:24], N.disparity_blur(x, 3.0))


def _blur_loop(x, k):
    """Per-pixel double-precision restatement of the disparity blur (no
    binary32 steps): Gaussian taps at t = -1..1 in quarters, linear
    interpolation along the row, border pixel repeated, empty pixels kept."""
    V, H, W, _ = x.shape
    ts = [j / 4.0 - 1.0 for j in range(9)]
    ws = [round(65535.0 * math.exp(-2.0 * t * t)) for t in ts]
    out = np.zeros((V, H, W, 3))
    for v in range(V):
        for y in range(H):
            for xx in range(W):
                d = x[v, y, xx, 3]
                s = k * d if d > -1.0 else 0.0
                acc = np.zeros(3)
                for t, w in zip(ts, ws):
                    u = min(max(xx + t * s, -1.0), float(W))
                    x0 = math.floor(u)
                    f = u - x0
                    a = x[v, y, min(max(x0, 0), W - 1), :3]
                    b = x[v, y, min(max(x0 + 1, 0), W - 1), :3]
                    acc += w * ((1.0 - f) * a + f * b)
                out[v, y, xx] = acc / sum(ws)
    return out


def _within_bf16_ulp(got, want):
    mag = np.maximum(np.abs(got), np.abs(want))
    ulp = 2.0 ** (np.floor(np.log2(np.maximum(mag, 1e-30))) - 7)
    return np.abs(got - want) <= ulp * 1.0001


def test_blur_matches_per_pixel_loop():
    rng = np.random.default_rng(11)
    x = N.bf16(np.concatenate([rng.random((3, 4, 23, 3)), rng.uniform(-1.2, 2.5, (3, 4, 23, 1))], -1))
    x[0, 1, 5:9, 3] = -1.0                      # empty pixels
    for k in (0.0, 1.7, 6.0):
        got = N.disparity_blur(x, k)
        assert (got[..., 3] == 0).all()
        assert _within_bf16_ulp(got[..., :3], _blur_loop(x, k)).all()


def test_blur_zero_disparity_constants_and_ramps():
    rng = np.random.default_rng(12)
    x = N.bf16(rng.random((2, 3, 17, 4)))
    np.testing.assert_array_equal(N.disparity_blur(x, 0.0)[..., :3], x[..., :3])
    c = np.zeros((1, 2, 20, 4))
    c[..., :3] = [0.25, 0.5, 0.75]
    c[..., 3] = N.bf16(rng.uniform(-0.9, 3.0, (1, 2, 20)))
    np.testing.assert_array_equal(N.disparity_blur(c, 4.0)[..., :3], c[..., :3])
    # a linear ramp is kept where every tap stays inside the row (symmetric taps)
    W = 64
    r = np.zeros((1, 1, W, 4))
    r[..., 0] = np.arange(W) / 64.0
    r[..., 3] = 1.0
    got = N.disparity_blur(r, 3.0)[0, 0, :, 0]
    np.testing.assert_array_equal(got[3:W - 4], r[0, 0, 3:W - 4, 0])


def test_blur_impulse_response_is_the_gaussian_profile():
    W = 21
    x = np.zeros((1, 2, W, 4))
    x[0, :, 10, 0] = 1.0           # one bright red pixel per row
    x[..., 3] = 0.5                # k*d = 4: taps land on whole pixels 4t = -4..4
    x[0, 1, :, 3] = -1.0           # second row empty: not moved
    out = N.disparity_blur(x, 8.0)
    prof = np.array([math.exp(-2.0 * (j / 4.0 - 1.0) ** 2) for j in range(9)])
    prof /= prof.sum()
    row = out[0, 0, :, 0]
    # output pixel 10 - m reads input pixel 10 at tap t = m/4
    want = np.zeros(W)
    want[6:15] = prof[::-1]
    assert np.all(np.abs(row - want) <= 2.0 ** -8 * want + 1e-7)   # one BF16 ulp
    assert (out[0, 0, :, 1:3] == 0).all()
    np.testing.assert_array_equal(out[0, 1, :, :3], x[0, 1, :, :3])


def test_assemble_reads_neighbour_views():
    V = 6
    x = np.zeros((V, 2, 3, 4))
    for v in range(V):
        x[v] = v + 1
    a = N.assemble(x)
    for v in range(V):
        for k, off in enumerate(range(-2, 3)):
            want = v + off + 1 if 0 <= v + off < V else 0
            assert (a[v, :, :, 4 * k:4 * k + 4] == want).all()


def test_identity_kernel_passes_input():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(4, 4, 3))
    w = np.zeros((9, 3, 3))
    w[4] = np.eye(3)
    np.testing.assert_allclose(N.conv3x3(x, w, np.zeros(3)), x)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.random((4, 5, 21, 4))
    t = rng.random((4, 5, 21, 3))
    params = N.init_params(7, hidden=6, scale=2.0)
    params = [(w, rng.normal(0, 0.1, b.shape)) for w, b in params]
    kd = 2.5   # the blurred channels take part
    loss, grads, _ = N.loss_and_grads(x, t, params, round_bf16=False, k=kd)
    h = 1e-6
    for k in range(4):
        for which in (0, 1):
            arr = params[k][which]
            for _ in range(6):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp, _, _ = N.loss_and_grads(x, t, params, round_bf16=False, k=kd)
                arr[idx] = old - h
                lm, _, _ = N.loss_and_grads(x, t, params, round_bf16=False, k=kd)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                an = grads[k][which][idx]
                assert an == pytest.approx(fd, rel=2e-4, abs=1e-9), (k, which, idx)


def test_adam_first_step_is_signed_lr():
    p = [(np.ones((9, 2, 2)), np.zeros(2))]
    g = [(np.full((9, 2, 2), 0.3), np.full(2, -2.0))]
    out = N.adam(p, g, {}, {}, 1, lr=0.01)
    np.testing.assert_allclose(out[0][0], 1 - 0.01, rtol=1e-6)
    np.testing.assert_allclose(out[0][1], 0.01, rtol=1e-6)
