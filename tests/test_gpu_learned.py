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
