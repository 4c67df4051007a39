"""The two splat orders (lfdpr_set_splat_order): per point, the default, and
per (triangle, view) for unlit frames.  They visit the same (point, view,
pixel) work in different orders, so views, depth and statistics must be
identical bit for bit; the default order is tied to the oracle by the parity
tests, and here the triangle-view order is tied to it through the default."""
import numpy as np
import pytest

from paper_2601_19901_amd import scenes
from test_gpu_parity import _log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _render(R, sid, model, order):
    from paper_2601_19901_amd import lfdpr  # noqa: F401
    R.set_splat_order(order)
    v, d = R.alloc_views(with_depth=True)
    R.render_frame(sid, model, v, d)
    st = R.stats()
    return v.cpu().numpy(), d.cpu().numpy(), st


def _same(R, sid, model, label):
    from paper_2601_19901_amd import lfdpr
    vt, dt, st = _render(R, sid, model, lfdpr.SPLAT_TRIANGLE_VIEW)
    vp, dp, sp = _render(R, sid, model, lfdpr.SPLAT_POINT)
    _log(f"[{label}] triangle-view {st}; point {sp}")
    # each frame ran the splat of the order asked for
    assert st.pop("splat_order") == lfdpr.SPLAT_TRIANGLE_VIEW and sp.pop("splat_order") == lfdpr.SPLAT_POINT
    # the hole census is observed by the triangle-view order only
    assert sp.pop("covered_px") == -1 and sp.pop("missed_px") == -1
    assert st.pop("covered_px") >= st["written_px"] and st.pop("missed_px") >= 0
    assert st == sp
    assert st["written_px"] > 0
    np.testing.assert_array_equal(vt, vp, err_msg=f"{label}: views")
    np.testing.assert_array_equal(dt.view(np.uint32), dp.view(np.uint32), err_msg=f"{label}: depth")


@pytest.mark.parametrize("seed,frame,mip,S", [(7, 0, True, 1), (8, 333, False, 1), (9, 500, True, 4)])
def test_orders_agree_small_display(torch_cuda, seed, frame, mip, S):
    from paper_2601_19901_amd import lfdpr
    w = scenes.small_display(seed=seed, S=S)
    w.views.mip = mip
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    _same(R, sid, w.model(frame), f"small-display seed {seed} S={S}")
    # the other key layout and a small grid (several chunks per wave)
    R.set_launch(64, 1)
    _same(R, sid, w.model(frame + 1), f"small-display seed {seed}, 64 blocks, [y][view][x] keys")


def test_orders_agree_at_display_size(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    w = scenes.display()
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    for f in (17, 600):
        _same(R, sid, w.model(f), f"display-1M frame {f}")
    # two frames in flight, triangle-view order, against the serial point order
    R.set_splat_order(lfdpr.SPLAT_TRIANGLE_VIEW)
    R.set_frames_in_flight(2)
    outs = []
    for f in (3, 4, 5):
        v, _ = R.alloc_views()
        R.render_frame(sid, w.model(f), v)
        outs.append(v)
    assert R.stats()["splat_order"] == lfdpr.SPLAT_TRIANGLE_VIEW
    R.set_frames_in_flight(1)
    for f, v in zip((3, 4, 5), outs):
        vp, _, _ = _render(R, sid, w.model(f), lfdpr.SPLAT_POINT)
        np.testing.assert_array_equal(v.cpu().numpy(), vp, err_msg=f"pipelined frame {f}")


def test_orders_agree_in_batches(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    torch = torch_cuda
    ws = [scenes.small_display(seed=s, V=12, W=96, H=96, hf_quads=hq) for s, hq in ((70, 24), (71, 48), (72, 8))]
    for k, w in enumerate(ws):
        w.views.cone_deg = 30.0 + 7.0 * k
    R = lfdpr.Renderer(0)
    ids = [R.upload_scene(w.scene) for w in ws]
    R.set_lens(ws[0].lens)
    models = [w.model(50 + 9 * k) for k, w in enumerate(ws)]
    out = {}
    for order in (lfdpr.SPLAT_TRIANGLE_VIEW, lfdpr.SPLAT_POINT):
        R.set_splat_order(order)
        B = lfdpr.Batch(R, ids, [w.views for w in ws])
        v = B.alloc_views()
        panels = torch.empty((len(ws), ws[0].lens.Hp, ws[0].lens.Wp, 3), dtype=torch.uint8, device="cuda")
        B.use_graph(order == lfdpr.SPLAT_TRIANGLE_VIEW)
        for _ in range(2):
            B.render(models, v, panels)
        st = B.stats()
        assert st.pop("splat_order") == order
        cov, mis = st.pop("covered_px"), st.pop("missed_px")
        if order == lfdpr.SPLAT_POINT:
            assert cov == -1 and mis == -1
        else:  # the batch's census: every covered pixel written
            assert cov == st["written_px"] and mis == 0
        out[order] = (v.cpu().numpy(), panels.cpu().numpy(), st)
        B.close()
    a, b = out[lfdpr.SPLAT_TRIANGLE_VIEW], out[lfdpr.SPLAT_POINT]
    assert a[2] == b[2] and a[2]["written_px"] > 0
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("kind,seed,frame", [("tiny", 3, 0), ("small", 7, 0), ("small", 8, 40), ("display", 2, 17)])
def test_hole_census_matches_the_oracle(torch_cuda, kind, seed, frame):
    """Under the triangle-view order the splat counts the pixels inside every
    active (triangle, view) pair's Q8 triangle and, of those, the ones no point
    writes (Sec. 3.2's holes); both equal the oracle's own census, which
    rasterises the triangles independently (display-1M frame 17 had one hole
    before the grazing-margin and zero-area rules)."""
    from oracle import oracle as O
    from paper_2601_19901_amd import lfdpr
    w = {"tiny": scenes.tiny, "small": scenes.small_display, "display": scenes.display}[kind](seed=seed)
    o = O.render(w.scene, w.views, w.model(frame))["stats"]
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    _, _, st = _render(R, sid, w.model(frame), lfdpr.SPLAT_TRIANGLE_VIEW)
    _log(f"[census {kind} {seed} f{frame}] gpu covered {st['covered_px']} missed {st['missed_px']}; oracle {o}")
    assert o["overflow_tris"] == 0 and o["orphans"] == 0
    assert st["covered_px"] == o["fragments"] and st["missed_px"] == o["misses"]
    assert st["written_px"] == o["fragments"] - o["misses"]
