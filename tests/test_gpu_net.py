"""GPU parity of the learned-reconstruction kernels (BF16 MFMA) with the
double-precision oracle.  Each layer is checked from the GPU's own input to
that layer, so one BF16 rounding flip upstream cannot cascade: activations
and propagated gradients within 1 BF16 ulp plus the FP32 accumulation bound
1e-5 * sum|terms|; FP32 weight and bias gradients within 1e-5 * sum|terms|
of the double-precision sums (products of BF16 values are exact in FP32; the
bound covers the FP32 additions).  Sizes include launches with more tiles
than the persistent grid (768 blocks), so blocks run several tiles through
the prefetch, re-staging and XCD-ordered tile loop, and weight-gradient blocks
loop over several 256-pixel chunks."""
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


def t16(a: np.ndarray, torch):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).cuda()


def get16(t) -> np.ndarray:
    return bits_to_f(t.cpu().numpy().view(np.uint16))


def random_params(seed, scale=1.5):
    rng = np.random.default_rng(seed)
    params = N.init_params(seed, scale=scale)
    return [(w, rng.normal(0, 0.05, b.shape)) for w, b in params]


def random_input(rng, n, H, W):
    """Colours in [-0.5, 1.5), disparities in [-0.5, 3) with some empty (-1) pixels."""
    x = rng.random((n, H, W, 4)) * 2 - 0.5
    x[..., 3] = rng.uniform(-0.5, 3.0, (n, H, W))
    x[..., 3][rng.random((n, H, W)) < 0.1] = -1.0
    return f_to_bits(x)


@pytest.mark.parametrize("V,F,H,W,k", [(6, 1, 24, 40, 2.75), (48, 1, 8, 32, 9.05), (5, 2, 7, 13, 0.0),
                                       (5, 2, 7, 13, 1.3), (2, 1, 3, 4100, 40.0),
                                       (48, 1, 64, 128, 9.05), (48, 1, 21, 200, 4.4)])
def test_forward_layers_match_oracle(torch_cuda, V, F, H, W, k):
    """F frames of V views each, ragged pixel counts; disparity blur bit-exact
    (rows of up to 4096 pixels are blurred from LDS, wider ones by global
    gathers: the fifth case).  The last two cases have 1,536 and 1,152 tiles
    of 4 x 64 pixels for 768 persistent blocks."""
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    R, net = make_net(torch, V, H, W * F)
    net.set_disparity_scale(k)
    params = random_params(V + H)
    flat = lfdpr.params_to_flat(params)
    net.set_params(flat)
    P = lfdpr.flat_to_params(flat.astype(np.float64))
    rng = np.random.default_rng(1)
    xb = random_input(rng, F * V, H, W)
    x = t16(xb, torch)
    y = torch.zeros((F * V, H, W, 4), dtype=torch.int16, device="cuda")
    net.forward(x, y)
    acts = []
    for j in (1, 2, 3):
        a = torch.zeros((F * V, H, W, 32), dtype=torch.int16, device="cuda")
        net.copy_state(j, a)
        acts.append(get16(a))
    xf = bits_to_f(xb)
    blur_g = torch.zeros((F * V, H, W, 4), dtype=torch.int16, device="cuda")
    net.copy_state(4, blur_g)
    blur = N.disparity_blur(xf, np.float32(k))
    np.testing.assert_array_equal(get16(blur_g), blur)
    a0 = np.concatenate([N.assemble(xf[f * V:(f + 1) * V], blur[f * V:(f + 1) * V]) for f in range(F)])
    inp = [a0] + acts
    for k in range(3):
        w = N.bf16(P[k][0])
        d = N.DILATION[k]
        want = N.bf16(np.maximum(np.stack([N.conv3x3(inp[k][n], w, P[k][1], d) for n in range(F * V)]), 0))
        S = np.stack([N.conv3x3(np.abs(inp[k][n]), np.abs(w), np.abs(P[k][1]), d) for n in range(F * V)])
        assert_bf16_close(acts[k], want, f"V{V}x{F} layer {k + 1}", abs_sum=S)
    w = N.bf16(P[3][0])
    d = N.DILATION[3]
    want_y = N.bf16(np.stack([N.conv3x3(acts[2][n], w, P[3][1], d) for n in range(F * V)]) + blur[..., :3])
    S = np.stack([N.conv3x3(np.abs(acts[2][n]), np.abs(w), np.abs(P[3][1]), d) for n in range(F * V)]) + np.abs(blur[..., :3])
    yg = get16(y)
    assert (yg[..., 3] == 0).all()
    assert_bf16_close(yg[..., :3], want_y, f"V{V}x{F} output", abs_sum=S)


def test_zero_parameters_are_identity(torch_cuda):
    """Zero parameters: the output is the input RGB without a disparity scale,
    the oracle's disparity blur with one."""
    torch = torch_cuda
    V, H, W = 8, 8, 48
    R, net = make_net(torch, V, H, W)
    rng = np.random.default_rng(0)
    xb = random_input(rng, V, H, W)
    x = t16(xb, torch)
    y = torch.zeros((V, H, W, 4), dtype=torch.int16, device="cuda")
    net.forward(x, y)
    yb = y.cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(yb[..., :3], xb[..., :3])
    assert (yb[..., 3] == 0).all()
    net.set_disparity_scale(5.5)
    net.forward(x, y)
    np.testing.assert_array_equal(get16(y)[..., :3], N.disparity_blur(bits_to_f(xb), np.float32(5.5))[..., :3])


@pytest.mark.parametrize("V,H,W,seed", [(7, 20, 36, 5), (48, 64, 128, 6)])
def test_backward_matches_oracle(torch_cuda, V, H, W, seed):
    """The second case: 1,536 tiles per propagated-gradient layer for 768
    blocks, and 393,216 pixels for at most 1,024 weight-gradient blocks (two
    256-pixel chunks each)."""
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    R, net = make_net(torch, V, H, W)
    net.set_disparity_scale(3.1)
    params = random_params(seed)
    flat = lfdpr.params_to_flat(params)
    net.set_params(flat)
    P = lfdpr.flat_to_params(flat.astype(np.float64))
    rng = np.random.default_rng(seed)
    xb = random_input(rng, V, H, W)
    tb = f_to_bits(np.concatenate([rng.random((V, H, W, 3)), np.zeros((V, H, W, 1))], axis=-1))
    x, t = t16(xb, torch), t16(tb, torch)
    y = torch.zeros((V, H, W, 4), dtype=torch.int16, device="cuda")
    net.forward(x, y)
    loss = float(net.backward(t).cpu().numpy()[0])
    yf = get16(y)[..., :3]
    tf = bits_to_f(tb)[..., :3]
    assert loss == pytest.approx(((yf - tf) ** 2).mean(), rel=1e-4)
    n = yf.size
    dz4 = torch.zeros((V, H, W, 32), dtype=torch.int16, device="cuda")
    net.copy_state(14, dz4)
    dz4f = get16(dz4)
    assert (dz4f[..., 3:] == 0).all()
    assert_bf16_close(dz4f[..., :3], N.bf16(2.0 * (yf - tf) / n), "dZ4")
    acts = [N.assemble(bits_to_f(xb), N.disparity_blur(bits_to_f(xb), np.float32(3.1)))]
    for k in (1, 2, 3):
        a = torch.zeros((V, H, W, 32), dtype=torch.int16, device="cuda")
        net.copy_state(k, a)
        acts.append(get16(a))
    dzs = {4: dz4f[..., :3]}
    for k in (3, 2, 1):
        d = torch.zeros((V, H, W, 32), dtype=torch.int16, device="cuda")
        net.copy_state(10 + k, d)
        dzs[k] = get16(d)
        w = N.bf16(P[k][0])
        d = N.DILATION[k]
        want = N.bf16(np.stack([N.conv3x3_xgrad(dzs[k + 1][v], w, d) for v in range(V)]) * (acts[k] > 0))
        S = np.stack([N.conv3x3_xgrad(np.abs(dzs[k + 1][v]), np.abs(w), d) for v in range(V)])
        assert_bf16_close(dzs[k], want, f"dZ{k}", abs_sum=S)
    g = torch.zeros(net.n_params, dtype=torch.float32, device="cuda")
    net.copy_state(20, g)
    G = lfdpr.flat_to_params(g.cpu().numpy().astype(np.float64))
    for k in range(4):
        dw = db = Sw = Sb = 0.0
        for v in range(V):
            gw, gb = N.conv3x3_wgrad(acts[k][v], dzs[k + 1][v], N.DILATION[k])
            aw, ab = N.conv3x3_wgrad(np.abs(acts[k][v]), np.abs(dzs[k + 1][v]), N.DILATION[k])
            dw, db, Sw, Sb = dw + gw, db + gb, Sw + aw, Sb + ab
        ew = np.abs(G[k][0] - dw) / (Sw + 1e-30)
        eb = np.abs(G[k][1] - db) / (Sb + 1e-30)
        _log(f"dW{k + 1}: max error / sum|terms| {ew.max():.2e}, db {eb.max():.2e}")
        assert (np.abs(G[k][0] - dw) <= 1e-5 * Sw + 1e-30).all()
        assert (np.abs(G[k][1] - db) <= 1e-5 * Sb + 1e-30).all()


def test_adam_step_and_training_reduce_loss(torch_cuda):
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    V, H, W = 6, 16, 32
    R, net = make_net(torch, V, H, W)
    flat = lfdpr.params_to_flat(N.init_params(6))
    net.set_params(flat)
    rng = np.random.default_rng(9)
    xf = rng.random((V, H, W, 4))
    xb = f_to_bits(xf)
    x = t16(xb, torch)
    # target: each view blended with its neighbours (what the network is for)
    xr = bits_to_f(xb)[..., :3]
    tgt = xr.copy()
    tgt[1:-1] = 0.5 * xr[1:-1] + 0.25 * (xr[:-2] + xr[2:])
    t = t16(f_to_bits(np.concatenate([tgt, np.zeros((V, H, W, 1))], -1)), torch)
    y = torch.zeros((V, H, W, 4), dtype=torch.int16, device="cuda")
    net.forward(x, y)
    net.backward(t)
    g = torch.zeros(net.n_params, dtype=torch.float32, device="cuda")
    net.copy_state(20, g)
    gnp = g.cpu().numpy().astype(np.float64)
    net.adam_step(1e-3)
    after = net.get_params().astype(np.float64)
    want = flat.astype(np.float64) - 1e-3 * gnp / (np.abs(gnp) + 1e-8)
    np.testing.assert_allclose(after, want, rtol=0, atol=1e-6)
    losses = []
    for it in range(150):
        net.forward(x, y)
        losses.append(float(net.backward(t).cpu().numpy()[0]))
        net.adam_step(2e-3)
    _log(f"loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    assert losses[-1] < 0.3 * losses[0]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        net.save(path)
        p_before = net.get_params()
        net.forward(x, y); net.backward(t); net.adam_step(2e-3)
        p_next = net.get_params()
        net.load(path)
        np.testing.assert_array_equal(net.get_params(), p_before)
        net.forward(x, y); net.backward(t); net.adam_step(2e-3)
        np.testing.assert_array_equal(net.get_params(), p_next)


def test_pack_and_unpack(torch_cuda):
    torch = torch_cuda
    V, H, W = 5, 6, 20
    R, net = make_net(torch, V, H, W)
    rng = np.random.default_rng(2)
    views = rng.integers(0, 2 ** 32, (V, H, W), dtype=np.uint64).astype(np.uint32)
    depth = rng.uniform(2.0, 9.0, (V, H, W)).astype(np.float32)
    depth[0, 0, :5] = np.inf
    D = 4.0
    tv = torch.from_numpy(views.view(np.int32)).cuda()
    td = torch.from_numpy(depth).cuda()
    x = torch.zeros((V, H, W, 4), dtype=torch.int16, device="cuda")
    net.pack_input(tv, td, x, D)
    xg = get16(x)
    rgba = views.view(np.uint8).reshape(V, H, W, 4)
    for c in range(3):
        want = N.bf16((rgba[..., c].astype(np.float32) / np.float32(255.0)).astype(np.float64))
        np.testing.assert_array_equal(xg[..., c], want)
    dd = np.where(np.isinf(depth), np.float32(-1.0), np.float32(D) / depth - np.float32(1.0)).astype(np.float32)
    np.testing.assert_array_equal(xg[..., 3], N.bf16(dd.astype(np.float64)))
    net.pack_input(tv, None, x)
    assert (get16(x)[..., 3] == 0).all()
    yb = f_to_bits(rng.uniform(-0.2, 1.2, (V, H, W, 4)))
    y = t16(yb, torch)
    out = torch.zeros((V, H, W), dtype=torch.int32, device="cuda")
    net.unpack_output(y, out)
    got = out.cpu().numpy().view(np.uint32).view(np.uint8).reshape(V, H, W, 4)
    yf = bits_to_f(yb)[..., :3]
    want = np.clip(np.floor(yf.astype(np.float32) * np.float32(255.0) + np.float32(0.5)), 0, 255)
    np.testing.assert_array_equal(got[..., :3], want.astype(np.uint8))
    assert (got[..., 3] == 255).all()


def test_gradients_are_identical_run_to_run(torch_cuda):
    """Parameter gradients are summed per block and then over blocks in a fixed
    order (no atomics): two backward passes over the same 48 x 128 x 128 crop
    (hundreds of blocks per sum) give the same bits.  (The reported loss is a
    sum of per-block atomics and may differ in its last bits.)"""
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    V, H, W = 48, 128, 128
    R, net = make_net(torch, V, H, W)
    net.set_params(lfdpr.params_to_flat(random_params(11, scale=1.0)))
    net.set_disparity_scale(3.3)
    rng = np.random.default_rng(12)
    x = t16(random_input(rng, V, H, W), torch)
    t = t16(f_to_bits(np.concatenate([rng.random((V, H, W, 3)), np.zeros((V, H, W, 1))], -1)), torch)
    y = torch.zeros((V, H, W, 4), dtype=torch.int16, device="cuda")
    grads, losses = [], []
    for _ in range(2):
        net.forward(x, y)
        losses.append(float(net.backward(t).cpu().numpy()[0]))
        g = torch.zeros(net.n_params, dtype=torch.float32, device="cuda")
        net.copy_state(20, g)
        grads.append(g.cpu().numpy())
    np.testing.assert_array_equal(grads[0].view(np.uint32), grads[1].view(np.uint32))
    assert np.any(grads[0] != 0.0)
    _log(f"loss {losses[0]:.6f} / {losses[1]:.6f}, {net.n_params} gradients bit-identical")


def test_forward_from_an_input_only_8_byte_aligned(torch_cuda):
    """Layer 1 reads pixel pairs with 16-byte loads only where the address is
    16-byte aligned: an input that starts 8 bytes into its buffer (and an odd
    image width) gives the same activations and output as an aligned copy."""
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    V, H, W = 6, 9, 77
    R, net = make_net(torch, V, H, W)
    net.set_params(lfdpr.params_to_flat(random_params(21)))
    net.set_disparity_scale(4.5)
    xb = random_input(np.random.default_rng(22), V, H, W)
    x = t16(xb, torch)
    n = x.numel()
    buf = torch.zeros(n + 8, dtype=torch.int16, device="cuda")
    buf[4:4 + n] = x.reshape(-1)
    xm = buf[4:4 + n].view(V, H, W, 4)
    assert xm.data_ptr() % 16 == 8 and x.data_ptr() % 16 == 0
    outs = []
    for inp in (x, xm):
        y = torch.zeros((V, H, W, 4), dtype=torch.int16, device="cuda")
        net.forward(inp, y)
        states = [y.cpu().numpy()]
        for k in (1, 2, 3):
            a = torch.zeros((V, H, W, 32), dtype=torch.int16, device="cuda")
            net.copy_state(k, a)
            states.append(a.cpu().numpy())
        outs.append(states)
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)
