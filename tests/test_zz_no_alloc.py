"""The no-allocation frame entry point (lfdpr_render_frame_noalloc), called
through the C ABI: every per-frame buffer in the library's static device
scratch.  Its views, depth and statistics must equal lfdpr_render_frame's,
which the parity tests tie to the oracle, bit for bit, on consecutive calls
that shrink the input (the scratch keeps the previous call's contents)."""
import sys

import numpy as np
import pytest

from paper_2601_19901_amd import scenes

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _both(torch, R, sid, model, label):
    """(views, depth, stats) from lfdpr_render_frame and from the no-allocation entry."""
    va, da = R.alloc_views(with_depth=True)
    R.render_frame(sid, model, va, da)
    sa = R.stats()
    vb = torch.full_like(va, 0x5A5A5A5A)
    db = torch.full_like(da, -1.0)
    sb = torch.full((6,), -7, dtype=torch.int64, device="cuda")
    _log(f"[{label}] no-allocation frame: {R.n_views} views of {R.vp.W}x{R.vp.H}")
    R.render_frame_noalloc(sid, model, vb, db, sb)
    torch.cuda.synchronize()
    return (va.cpu().numpy(), da.cpu().numpy(), sa), (vb.cpu().numpy(), db.cpu().numpy(), sb.cpu().numpy())


def _check(a, b, label):
    (va, da, sa), (vb, db, sb) = a, b
    _log(f"[{label}] render_frame stats {sa}; no-allocation stats {sb.tolist()}")
    assert sa["points"] > 0 and sa["written_px"] > 0
    assert sb.tolist() == [sa["points"], sa["active_tris"], sa["point_views"], sa["overflow_tris"],
                           sa["written_px"], 1 << 19]
    np.testing.assert_array_equal(vb, va, err_msg=f"{label}: views")
    np.testing.assert_array_equal(db.view(np.uint32), da.view(np.uint32), err_msg=f"{label}: depth")


def test_noalloc_frames_equal_render_frame(torch_cuda):
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    R = lfdpr.Renderer(0)
    big = scenes.small_display(seed=7)                 # ~7k triangles, 12 views of 96^2
    small = scenes.tiny(V=4, size=64)                  # 1,280 triangles, 4 views of 64^2
    sid_big = R.upload_scene(big.scene)
    sid_small = R.upload_scene(small.scene)
    assert small.scene.n_tris < big.scene.n_tris
    R.set_views(big.views)
    a, b = _both(torch, R, sid_big, big.model(3), "small-display")
    _check(a, b, "small-display")
    # second call: fewer triangles, fewer and smaller views; the scratch still
    # holds the first frame's records, points and keys
    R.set_views(small.views)
    a, b = _both(torch, R, sid_small, small.model(11), "tiny")
    _check(a, b, "tiny")
    # the other key layout, and no depth or statistics output
    R.set_launch(1024, 1)
    va, _ = R.alloc_views()
    R.render_frame(sid_small, small.model(12), va)
    vb = torch.zeros_like(va)
    R.render_frame_noalloc(sid_small, small.model(12), vb)
    np.testing.assert_array_equal(vb.cpu().numpy(), va.cpu().numpy())


def test_noalloc_refusals(torch_cuda):
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    R = lfdpr.Renderer(0)
    w = scenes.tiny(V=4, size=64)
    sid = R.upload_scene(w.scene)
    v = torch.zeros((4, 64, 64), dtype=torch.int32, device="cuda")
    with pytest.raises(lfdpr.LfdprError) as e:       # no rig yet
        R.render_frame_noalloc(sid, w.model(0), v)
    assert e.value.code == lfdpr.LFDPR_ESTATE
    R.set_views(w.views)
    R.set_frames_in_flight(2)
    with pytest.raises(lfdpr.LfdprError) as e:
        R.render_frame_noalloc(sid, w.model(0), v)
    assert e.value.code == lfdpr.LFDPR_ESTATE
    R.set_frames_in_flight(1)
    # more triangles than the scratch holds: refused before any launch
    n = 70_000
    rng = np.random.default_rng(0)
    pos = rng.uniform(-1, 1, (n * 3, 3)).astype(np.float32)
    many = scenes.Scene(pos, np.zeros((n * 3, 2), np.float32), np.arange(n * 3, dtype=np.uint32).reshape(n, 3),
                        np.zeros(n, np.uint16), [scenes.constant_texture(4, (1, 2, 3, 255))]).check()
    sid_many = R.upload_scene(many)
    with pytest.raises(lfdpr.LfdprError) as e:
        R.render_frame_noalloc(sid_many, w.model(0), v)
    assert e.value.code == lfdpr.LFDPR_EINVAL and "65,536" in str(e.value)
    # more keys than the scratch holds
    R.set_views(scenes.ViewParams(V=32, W=512, H=512, fovy_deg=30.0, aspect=1.0, D=3.0, cone_deg=40.0, znear=0.1))
    vv = torch.zeros((32, 512, 512), dtype=torch.int32, device="cuda")
    with pytest.raises(lfdpr.LfdprError) as e:
        R.render_frame_noalloc(sid, w.model(0), vv)
    assert e.value.code == lfdpr.LFDPR_EINVAL and "2,097,152" in str(e.value)
    # still usable afterwards
    R.set_views(w.views)
    va, _ = R.alloc_views()
    R.render_frame(sid, w.model(1), va)
    vb = torch.zeros_like(va)
    R.render_frame_noalloc(sid, w.model(1), vb)
    np.testing.assert_array_equal(vb.cpu().numpy(), va.cpu().numpy())
