"""The learned angular reconstruction, trained by the library's own forward and
backward kernels on pairs the method renders, beats the plain renders against
4x angular supersampling; poisoned parameters fall back to 4x supersampling.
Untrained (last layer zero) the network is the disparity blur alone."""
import math

import numpy as np
import pytest

from paper_2601_19901_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_19901_amd import learned
    train_w = [scenes.small_display(seed=s, V=16, W=96, H=96) for s in (31, 32, 33)]
    test_w = [scenes.small_display(seed=s, V=16, W=96, H=96) for s in (41,)]
    ss = learned.AngularSS(train_w + test_w, factors=(1, 4, 16))
    model = learned.LearnedReconstruction(ss, 96, 96)
    rng = np.random.default_rng(0)
    frames = [(int(rng.integers(0, 3)), int(rng.integers(0, 1000))) for _ in range(400)]
    test = [(3, int(f)) for f in rng.integers(0, 1000, 12)]
    before = learned.evaluate(model, test, 16)
    loss0 = model.frame_loss(0, 123)
    losses = model.train(frames, steps_per_frame=4, crop=64, lr=1e-3, lr_end=3e-4, log_every=0)
    loss1 = model.frame_loss(0, 123)
    after = learned.evaluate(model, test, 16)
    print("before", before, "\nafter", after, "\nframe loss", loss0, "->", loss1, flush=True)
    return learned, ss, model, before, after, (loss0, loss1)


def test_training_reduces_loss(trained):
    _, _, _, _, _, (loss0, loss1) = trained
    assert loss0[0] < 0.7 * loss0[1]     # the disparity blur alone already helps
    assert loss1[0] < 0.95 * loss0[0]    # and training improves on it


def test_learned_beats_plain_against_supersampling(trained):
    _, _, _, before, after, _ = trained
    assert before["learned_vs_ss4"] > before["plain_vs_ss4"] + 1.0
    assert after["learned_vs_ss4"] > before["learned_vs_ss4"]
    assert after["learned_vs_ss4"] > after["plain_vs_ss4"] + 2.0
    assert after["learned_vs_ref"] > after["plain_vs_ref"] + 2.0


def test_fallback_on_poisoned_parameters(trained):
    learned, ss, model, _, _, _ = trained
    good = model.net.get_params()
    bad = good.copy()
    bad[7] = np.inf
    assert not model.set_params(bad)
    out = model.reconstruct(3, 5).clone()
    ref = ss.render_ss(3, 5, 4)
    assert learned.psnr_views(out, ref) == math.inf
    assert model.set_params(good) and model.healthy


def test_overlapped_frames_equal_serial_frames(trained):
    """LearnedPipeline (network of frame i on its own stream while frame i+1
    renders, two alternating buffers) gives every panel bit for bit as the
    serial path; a poisoned-parameter frame in the middle takes the fallback."""
    learned, ss, model, _, _, _ = trained
    import torch
    lens = ss.workloads[3].lens
    R1 = ss.rigs[1].renderer
    R1.set_lens(lens)
    frames = [5, 6, 7, 300, 301, 999, 0]

    def new_panel():
        return torch.empty((lens.Hp, lens.Wp, 3), dtype=torch.uint8, device="cuda")

    serial = []
    for f in frames:
        p = new_panel()
        R1.reconstruct(model.reconstruct(3, f), p)
        serial.append(p.cpu().numpy())
    pipe = learned.LearnedPipeline(model, lens)
    panels = []
    for f in frames:
        p = new_panel()
        pipe.frame(3, f, p)
        panels.append(p)
    torch.cuda.synchronize()
    for f, a, b in zip(frames, serial, panels):
        np.testing.assert_array_equal(b.cpu().numpy(), a, err_msg=f"frame {f}")
    # fallback in the middle of overlapped frames
    good = model.net.get_params()
    bad = good.copy()
    bad[3] = np.nan
    out = []
    for f, ok in ((10, True), (11, False), (12, True)):
        assert model.set_params(good if ok else bad) == ok
        p = new_panel()
        pipe.frame(3, f, p)
        out.append(p)
    torch.cuda.synchronize()
    want = []
    for f, ok in ((10, True), (11, False), (12, True)):
        model.set_params(good if ok else bad)
        p = new_panel()
        R1.reconstruct(model.reconstruct(3, f), p)
        want.append(p.cpu().numpy())
    model.set_params(good)
    for (f, _), a, b in zip(((10, 0), (11, 0), (12, 0)), want, out):
        np.testing.assert_array_equal(b.cpu().numpy(), a, err_msg=f"frame {f} around the fallback")
    pipe.close()


def test_validation_against_supersampling_switches_off_a_bad_network(trained):
    """The 4x result judges the network: a trained network passes; finite but
    wrong parameters (large random weights) fail the PSNR check, and the
    reconstruction then returns the 4x result."""
    learned, ss, model, _, _, _ = trained
    good = model.net.get_params()
    ok = model.validate([(3, 17), (3, 512)])
    assert ok["healthy"] and ok["gain_db_vs_plain"] > 2.0, ok
    rng = np.random.default_rng(9)
    bad = (rng.normal(0.0, 0.5, good.size)).astype(np.float32)
    assert model.set_params(bad)               # finite: accepted
    res = model.validate([(3, 17), (3, 512)])
    assert not res["healthy"], res
    out = model.reconstruct(3, 40).clone()
    assert learned.psnr_views(out, ss.render_ss(3, 40, 4)) == math.inf
    assert model.set_params(good) and model.healthy
    assert model.validate([(3, 17)])["healthy"]


def test_disparity_scale_from_the_rig(trained):
    """lfdpr_net_set_rig gives the network the scale k = fx 2 tan(cone/2) / V
    of the rig the views come from: forward equals the one with k set
    explicitly from that formula (double, rounded once)."""
    _, ss, model, _, _, _ = trained
    import torch
    vp = ss.rigs[1].views
    # the rig crosses the boundary in binary32
    aspect, fovy, cone = (float(np.float32(v)) for v in (vp.aspect, vp.fovy_deg, vp.cone_deg))
    fx = (vp.W / 2.0) / (aspect * math.tan(fovy * math.pi / 360.0))
    k = np.float32(fx * 2.0 * math.tan(cone * math.pi / 360.0) / vp.V)
    views, depth = ss.render_plain(3, 77)
    x = torch.empty((vp.V, vp.H, vp.W, 4), dtype=torch.int16, device="cuda")
    model.net.pack_input(views, depth, x, ss.D)
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    model.net.set_rig(vp)
    model.net.forward(x, y1)
    model.net.set_disparity_scale(float(k))
    model.net.forward(x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    model.net.set_disparity_scale(float(k) * 1.5)
    model.net.forward(x, y2)
    assert not torch.equal(y1, y2)
    model.net.set_rig(vp)
