"""Two frames in flight (lfdpr_set_frames_in_flight): point generation of a
frame on the context's side stream, overlapping the previous frame's splat.

Bar: every frame of a pipelined sequence bit-exact against the oracle (or
against serial renders at display size); statistics, points, counts, debug
records and material words describe the last frame; mode switches, scene
switches and rig changes between pipelined frames keep every frame exact."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_19901_amd import scenes
from test_gpu_parity import _log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _views(torch, w):
    return torch.empty((w.views.V * w.views.S, w.views.H, w.views.W), dtype=torch.int32, device="cuda")


def test_pipelined_frames_match_the_oracle(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    torch = torch_cuda
    w = scenes.small_display(seed=7)
    nt = w.scene.n_tris
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    R.set_frames_in_flight(2)
    frames = [0, 40, 80, 120, 160, 200, 240]
    outs = []
    for f in frames:
        v = _views(torch, w)
        R.render_frame(sid, w.model(f), v)
        outs.append(v)
    last = O.render(w.scene, w.views, w.model(frames[-1]))
    # statistics, points and counts describe the last frame
    st = R.stats()
    assert st["points"] == last["n_points"] and st["point_views"] == last["stats"]["point_views"]
    np.testing.assert_array_equal(R.counts(nt), last["count"].astype(np.uint32))
    np.testing.assert_array_equal(R.points()["tvmax"], last["points"]["tvmax"])
    for f, v in zip(frames, outs):
        o = O.render(w.scene, w.views, w.model(f))
        np.testing.assert_array_equal(v.cpu().numpy().view(np.uint32), o["rgba"], err_msg=f"frame {f}")
    _log(f"{len(frames)} pipelined frames bit-exact")
    # debug records of the last frame
    df = torch.zeros((nt, 8), dtype=torch.float32, device="cuda")
    di = torch.zeros((nt, 8), dtype=torch.int32, device="cuda")
    R.set_debug_records(df, di)
    v = _views(torch, w)
    R.render_frame(sid, w.model(7), v)
    R.render_frame(sid, w.model(9), v)
    o = O.render(w.scene, w.views, w.model(9))
    np.testing.assert_array_equal(di.cpu().numpy(), o["trii"])
    np.testing.assert_array_equal(df.cpu().numpy().view(np.uint32), o["trif"].view(np.uint32))
    R.close()


def test_scene_and_mode_switches_between_pipelined_frames(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    torch = torch_cuda
    a = scenes.small_display(seed=7)
    b = scenes.with_pbr(scenes.small_display(seed=8), seed=8)
    R = lfdpr.Renderer(0)
    sa, sb = R.upload_scene(a.scene), R.upload_scene(b.scene)
    R.set_views(a.views)
    R.set_frames_in_flight(2)
    seq = [(sa, a, None, 3), (sb, b, None, 5), (sb, b, b.shading, 7), (sa, a, None, 9), (sb, b, b.shading, 11)]
    outs = []
    for sid, w, sh, f in seq:
        R.set_shading(sh)
        v = _views(torch, w)
        R.render_frame(sid, w.model(f), v)
        outs.append(v)
    pm = R.point_materials()
    ob = O.render(b.scene, b.views, b.model(11), shading=b.shading)
    np.testing.assert_array_equal(pm["nmin"], ob["points"]["nmin"])
    np.testing.assert_array_equal(pm["rm"], ob["points"]["rm"])
    for (sid, w, sh, f), v in zip(seq, outs):
        o = O.render(w.scene, w.views, w.model(f), shading=sh)
        np.testing.assert_array_equal(v.cpu().numpy().view(np.uint32), o["rgba"], err_msg=f"frame {f}")
    # back to one frame in flight, then a new rig, then two again
    R.set_shading(None)
    R.set_frames_in_flight(1)
    v = _views(torch, a)
    R.render_frame(sa, a.model(13), v)
    np.testing.assert_array_equal(v.cpu().numpy().view(np.uint32), O.render(a.scene, a.views, a.model(13))["rgba"])
    small = scenes.small_display(seed=7, W=64, H=48, V=6)
    R.set_frames_in_flight(2)
    R.set_views(small.views, point_capacity=1 << 16)
    outs = []
    for f in (2, 4, 6):
        v = _views(torch, small)
        R.render_frame(sa, small.model(f), v)
        outs.append(v)
    for f, v in zip((2, 4, 6), outs):
        o = O.render(a.scene, small.views, small.model(f))
        np.testing.assert_array_equal(v.cpu().numpy().view(np.uint32), o["rgba"], err_msg=f"small rig frame {f}")
    # stage timing covers both streams
    R.timing(True)
    for f in (8, 10, 12):
        R.render_frame(sa, small.model(f), v)
    t = R.timings()
    for k in ("setup", "scan", "emit", "splat", "resolve"):
        assert t[k][0] > 0.0 and t[k][1] == 3, (k, t)
    R.timing(False)
    R.close()


def test_pipelined_display_frames_equal_serial_renders(torch_cuda):
    """Display-size frames with two in flight, in the launch configuration the
    benchmark times, equal serial renders of the same frames bit for bit
    (views and panels)."""
    from paper_2601_19901_amd import lfdpr
    torch = torch_cuda
    _log("generating display-size scene")
    w = scenes.display()
    frames = [0, 1, 2, 3, 50, 51]
    res = {}
    for nf in (1, 2):
        R = lfdpr.Renderer(0)
        sid = R.upload_scene(w.scene)
        R.set_views(w.views)
        R.set_lens(w.lens)
        R.set_frames_in_flight(nf)
        out = []
        for f in frames:
            v = _views(torch, w)
            p = torch.empty((w.lens.Hp, w.lens.Wp, 3), dtype=torch.uint8, device="cuda")
            R.render_frame(sid, w.model(f), v)
            R.reconstruct(v, p)
            out.append((v, p))
        res[nf] = [(v.cpu().numpy(), p.cpu().numpy()) for v, p in out]
        res[f"stats{nf}"] = R.stats()
        R.close()
    for k, f in enumerate(frames):
        np.testing.assert_array_equal(res[1][k][0], res[2][k][0], err_msg=f"views, frame {f}")
        np.testing.assert_array_equal(res[1][k][1], res[2][k][1], err_msg=f"panel, frame {f}")
    assert res["stats1"] == res["stats2"]


@pytest.mark.parametrize("order", ["point", "quilt"])
def test_pipelined_supersampled_frames_with_presentation_match_the_oracle(torch_cuda, order):
    """The benchmark's supersampled loop at a small size: each frame renders
    4x sub-views with two frames in flight, then the angular filter and the
    panel pass are queued on the context's stream before the next frame (so
    the next frame's point generation waits for them); one sub-view buffer
    serves every frame.  Every filtered frame and panel equals the oracle."""
    from paper_2601_19901_amd import lfdpr
    torch = torch_cuda
    w = scenes.small_display(seed=21, S=4, V=8)
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    R.set_lens(w.lens)
    R.set_splat_order(lfdpr.SPLAT_QUILT if order == "quilt" else lfdpr.SPLAT_POINT)
    R.set_frames_in_flight(2)
    sub = _views(torch, w)
    frames = [2, 3, 4, 90, 91]
    outs = []
    for f in frames:
        R.render_frame(sid, w.model(f), sub)
        filt = torch.empty((w.views.V, w.views.H, w.views.W), dtype=torch.int32, device="cuda")
        panel = torch.empty((w.lens.Hp, w.lens.Wp, 3), dtype=torch.uint8, device="cuda")
        R.angular_filter(sub, filt)
        R.reconstruct(filt, panel)
        outs.append((filt, panel))
    torch.cuda.synchronize()
    assert R.stats()["splat_order"] == (lfdpr.SPLAT_QUILT if order == "quilt" else lfdpr.SPLAT_POINT)
    for f, (filt, panel) in zip(frames, outs):
        o = O.render(w.scene, w.views, w.model(f))
        of = O.angular_filter(o["rgba"], w.views)
        np.testing.assert_array_equal(filt.cpu().numpy().view(np.uint32), of, err_msg=f"{order} frame {f} filtered")
        np.testing.assert_array_equal(panel.cpu().numpy(), O.interleave(of, w.lens), err_msg=f"{order} frame {f} panel")
    R.close()
