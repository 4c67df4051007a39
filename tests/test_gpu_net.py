"""GPU parity of the learned-reconstruction kernels (BF16 MFMA) with the
double-precision oracle.  Each layer is checked from the GPU's own input to
that layer, so one BF16 rounding flip upstream cannot cascade: activations
and propagated gradients within 1 BF16 ulp; FP32 weight gradients within a
relative 2e-3 of the largest entry (FP32 accumulation of BF16 products vs
double)."""
import os
import sys
import tempfile

import numpy as np
import pytest

from oracle import net_oracle as N

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def bits_to_f(h: np.ndarray) -> np.ndarray:
    return (h.astype(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def f_to_bits(x: np.ndarray) -> np.ndarray:
    return (N.bf16(x).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


def assert_bf16_close(got, want, label, max_frac=1e-3, abs_sum=None):
    """|got - want| <= 1 BF16 ulp of the larger magnitude plus, when the sum of
    absolute terms is given, the FP32 accumulation bound 1e-5 * sum|terms|."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    mag = np.maximum(np.abs(got), np.abs(want))
    ulp = np.where(mag > 0, 2.0 ** (np.floor(np.log2(np.maximum(mag, 1e-38))) - 7), 0.0)
    acc = 0.0 if abs_sum is None else 1e-5 * abs_sum
    bad = np.abs(got - want) > ulp * 1.0001 + acc + 1e-30
    exact = (got == want).mean()
    _log(f"[{label}] exact {exact:.5f}, beyond 1 ulp {bad.sum()}")
    assert not bad.any(), f"{label}: {bad.sum()} values beyond one BF16 ulp"
    assert exact > 1 - max_frac * 50


def make_net(torch, V, H, W):
    from paper_2601_19901_amd import lfdpr
    R = lfdpr.Renderer(0)
    return R, lfdpr.Net(R, V, H, W)


@pytest.mark.parametrize("V,H,W", [(16, 24, 40), (48, 16, 64)])
def test_forward_layers_match_oracle(torch_cuda, V, H, W):
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    R, net = make_net(torch, V, H, W)
    rng = np.random.default_rng(V + H)
    params = N.init_params(V, 3, scale=1.5)
    params = [(w, rng.normal(0, 0.05, b.shape)) for w, b in params]
    flat = lfdpr.params_to_flat(params)
    net.set_params(flat)
    P = lfdpr.flat_to_params(flat.astype(np.float64), V)
    xb = f_to_bits(rng.random((H, W, 4 * V)) * 2 - 0.5)
    x = torch.from_numpy(xb.view(np.int16)).cuda()
    y = torch.zeros((H, W, 3 * V), dtype=torch.int16, device="cuda")
    net.forward(x, y, H, W)
    acts = []
    for k in (1, 2, 3):
        a = torch.zeros((H, W, 32), dtype=torch.int16, device="cuda")
        net.copy_state(k, a)
        acts.append(bits_to_f(a.cpu().numpy().view(np.uint16)))
    inp = [bits_to_f(xb)] + acts
    for k in range(3):
        want = N.bf16(np.maximum(N.conv3x3(inp[k], N.bf16(P[k][0]), P[k][1]), 0))
        S = N.conv3x3(np.abs(inp[k]), np.abs(N.bf16(P[k][0])), np.abs(P[k][1]))
        assert_bf16_close(acts[k], want, f"V{V} layer {k + 1}", abs_sum=S)
    want_y = N.bf16(N.conv3x3(acts[2], N.bf16(P[3][0]), P[3][1]) + N.residual_rgb(bits_to_f(xb), V))
    S = N.conv3x3(np.abs(acts[2]), np.abs(N.bf16(P[3][0])), np.abs(P[3][1])) + np.abs(N.residual_rgb(bits_to_f(xb), V))
    assert_bf16_close(bits_to_f(y.cpu().numpy().view(np.uint16)), want_y, f"V{V} output", abs_sum=S)


def test_zero_parameters_are_identity(torch_cuda):
    torch = torch_cuda
    V, H, W = 16, 8, 48
    R, net = make_net(torch, V, H, W)
    rng = np.random.default_rng(0)
    xb = f_to_bits(rng.random((H, W, 4 * V)))
    x = torch.from_numpy(xb.view(np.int16)).cuda()
    y = torch.zeros((H, W, 3 * V), dtype=torch.int16, device="cuda")
    net.forward(x, y, H, W)
    want = f_to_bits(N.residual_rgb(bits_to_f(xb), V))
    np.testing.assert_array_equal(y.cpu().numpy().view(np.uint16), want)


def test_backward_matches_oracle(torch_cuda):
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    V, H, W = 16, 20, 36
    R, net = make_net(torch, V, H, W)
    rng = np.random.default_rng(5)
    params = N.init_params(V, 4, scale=1.5)
    params = [(w, rng.normal(0, 0.05, b.shape)) for w, b in params]
    flat = lfdpr.params_to_flat(params)
    net.set_params(flat)
    P = lfdpr.flat_to_params(flat.astype(np.float64), V)
    xb = f_to_bits(rng.random((H, W, 4 * V)))
    tb = f_to_bits(rng.random((H, W, 3 * V)))
    x = torch.from_numpy(xb.view(np.int16)).cuda()
    t = torch.from_numpy(tb.view(np.int16)).cuda()
    y = torch.zeros((H, W, 3 * V), dtype=torch.int16, device="cuda")
    net.forward(x, y, H, W)
    loss = float(net.backward(t).cpu().numpy()[0])
    yf = bits_to_f(y.cpu().numpy().view(np.uint16))
    want_loss = ((yf - bits_to_f(tb)) ** 2).mean()
    assert loss == pytest.approx(want_loss, rel=1e-4)
    # gradient of the output, then each layer from the GPU's own upstream gradient
    n = yf.size
    dz4 = torch.zeros((H, W, 64), dtype=torch.int16, device="cuda")
    net.copy_state(14, dz4)
    dz4f = bits_to_f(dz4.cpu().numpy().view(np.uint16))
    assert (dz4f[..., 48:] == 0).all()
    assert_bf16_close(dz4f[..., :48], N.bf16(2.0 * (yf - bits_to_f(tb)) / n), "dZ4")
    acts = [bits_to_f(xb)]
    for k in (1, 2, 3):
        a = torch.zeros((H, W, 32), dtype=torch.int16, device="cuda")
        net.copy_state(k, a)
        acts.append(bits_to_f(a.cpu().numpy().view(np.uint16)))
    dzs = {4: dz4f[..., :48]}
    for k in (3, 2, 1):
        d = torch.zeros((H, W, 32), dtype=torch.int16, device="cuda")
        net.copy_state(10 + k, d)
        dzs[k] = bits_to_f(d.cpu().numpy().view(np.uint16))
        want = N.bf16(N.conv3x3_xgrad(dzs[k + 1], N.bf16(P[k][0])) * (acts[k] > 0))
        S = N.conv3x3_xgrad(np.abs(dzs[k + 1]), np.abs(N.bf16(P[k][0])))
        assert_bf16_close(dzs[k], want, f"dZ{k}", abs_sum=S)
    g = torch.zeros(net.n_params, dtype=torch.float32, device="cuda")
    net.copy_state(20, g)
    G = lfdpr.flat_to_params(g.cpu().numpy().astype(np.float64), V)
    for k in range(4):
        dw, db = N.conv3x3_wgrad(acts[k], dzs[k + 1])
        scale = np.abs(dw).max() + 1e-30
        err = np.abs(G[k][0] - dw).max() / scale
        _log(f"dW{k + 1}: max rel err {err:.2e}")
        assert err < 2e-3
        np.testing.assert_allclose(G[k][1], db, rtol=2e-3, atol=2e-3 * (np.abs(db).max() + 1e-30))


def test_adam_step_and_training_reduce_loss(torch_cuda):
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    V, H, W = 16, 16, 32
    R, net = make_net(torch, V, H, W)
    rng = np.random.default_rng(9)
    params = N.init_params(V, 6)
    flat = lfdpr.params_to_flat(params)
    net.set_params(flat)
    xb = f_to_bits(rng.random((H, W, 4 * V)))
    x = torch.from_numpy(xb.view(np.int16)).cuda()
    # target: a smooth function of the input that the network can fit
    tgt = N.residual_rgb(bits_to_f(xb), V) * 0.8 + 0.05
    t = torch.from_numpy(f_to_bits(tgt).view(np.int16)).cuda()
    y = torch.zeros((H, W, 3 * V), dtype=torch.int16, device="cuda")
    net.forward(x, y, H, W)
    net.backward(t)
    g = torch.zeros(net.n_params, dtype=torch.float32, device="cuda")
    net.copy_state(20, g)
    gnp = g.cpu().numpy().astype(np.float64)
    net.adam_step(1e-3)
    after = net.get_params().astype(np.float64)
    # first Adam step moves every parameter by lr * g/(|g| + eps/sqrt(1-b2)) ~ lr sign(g)
    want = flat.astype(np.float64) - 1e-3 * gnp / (np.abs(gnp) + 1e-8)
    np.testing.assert_allclose(after, want, rtol=0, atol=1e-6)
    losses = []
    for it in range(60):
        net.forward(x, y, H, W)
        losses.append(float(net.backward(t).cpu().numpy()[0]))
        net.adam_step(3e-3)
    _log(f"loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    assert losses[-1] < 0.5 * losses[0]
    # checkpoint round trip reproduces parameters and continues identically
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        net.save(path)
        p_before = net.get_params()
        net.forward(x, y, H, W); net.backward(t); net.adam_step(3e-3)
        p_next = net.get_params()
        net.load(path)
        np.testing.assert_array_equal(net.get_params(), p_before)
        net.forward(x, y, H, W); net.backward(t); net.adam_step(3e-3)
        np.testing.assert_array_equal(net.get_params(), p_next)


def test_pack_and_unpack(torch_cuda):
    torch = torch_cuda
    V, H, W = 16, 6, 20
    R, net = make_net(torch, V, H, W)
    rng = np.random.default_rng(2)
    views = rng.integers(0, 2 ** 32, (V, H, W), dtype=np.uint64).astype(np.uint32)
    depth = rng.uniform(2.0, 9.0, (V, H, W)).astype(np.float32)
    depth[0, 0, :5] = np.inf
    D = 4.0
    tv = torch.from_numpy(views.view(np.int32)).cuda()
    td = torch.from_numpy(depth).cuda()
    x = torch.zeros((H, W, 4 * V), dtype=torch.int16, device="cuda")
    net.pack_input(tv, td, x, D)
    xg = bits_to_f(x.cpu().numpy().view(np.uint16)).reshape(H, W, V, 4)
    rgba = views.view(np.uint8).reshape(V, H, W, 4).astype(np.float64)
    for c in range(3):
        want = N.bf16((rgba[..., c].astype(np.float32) / np.float32(255.0)).astype(np.float64))
        np.testing.assert_array_equal(xg[..., c], want.transpose(1, 2, 0))
    dd = np.where(np.isinf(depth), np.float32(-1.0), np.float32(D) / depth - np.float32(1.0)).astype(np.float32)
    np.testing.assert_array_equal(xg[..., 3], N.bf16(dd.astype(np.float64)).transpose(1, 2, 0))
    # unpack: y -> RGBA8
    yb = f_to_bits(rng.uniform(-0.2, 1.2, (H, W, 3 * V)))
    y = torch.from_numpy(yb.view(np.int16)).cuda()
    out = torch.zeros((V, H, W), dtype=torch.int32, device="cuda")
    net.unpack_output(y, out, H, W)
    got = out.cpu().numpy().view(np.uint32).view(np.uint8).reshape(V, H, W, 4)
    yf = bits_to_f(yb).reshape(H, W, V, 3).transpose(2, 0, 1, 3)
    want = np.clip(np.floor(yf.astype(np.float32) * np.float32(255.0) + np.float32(0.5)), 0, 255)
    np.testing.assert_array_equal(got[..., :3], want.astype(np.uint8))
    assert (got[..., 3] == 255).all()
