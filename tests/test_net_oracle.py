"""Pins of the network oracle: finite differences, identities, explicit loops."""
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
    _, _, y = N.forward(x, params)
    np.testing.assert_array_equal(y, x[..., :3])


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
    loss, grads, _ = N.loss_and_grads(x, t, params, round_bf16=False)
    h = 1e-6
    for k in range(4):
        for which in (0, 1):
            arr = params[k][which]
            for _ in range(6):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp, _, _ = N.loss_and_grads(x, t, params, round_bf16=False)
                arr[idx] = old - h
                lm, _, _ = N.loss_and_grads(x, t, params, round_bf16=False)
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
