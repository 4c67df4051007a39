"""Batched rendering (one launch per stage for several scenes, hipGraph replay)
and the autotuner: every result bit-identical to single-scene renders, which
the other GPU tests tie to the oracle, and, for some items, to the oracle
directly."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_19901_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_19901_amd import lfdpr
    ws = [scenes.small_display(seed=s, V=12, W=96, H=96, hf_quads=hq) for s, hq in ((60, 24), (61, 48), (62, 80), (63, 16))]
    for k, w in enumerate(ws):            # per-scene cones and distances differ
        w.views.cone_deg = 30.0 + 6.0 * k
        w.views.D = 10.0 + 0.5 * k
    R = lfdpr.Renderer(0)
    ids = [R.upload_scene(w.scene) for w in ws]
    R.set_lens(ws[0].lens)
    return torch, lfdpr, R, ws, ids


def single(torch, R, w, sid, model):
    R.set_views(w.views)
    v, _ = R.alloc_views()
    R.render_frame(sid, model, v)
    panel = torch.empty((w.lens.Hp, w.lens.Wp, 3), dtype=torch.uint8, device="cuda")
    R.reconstruct(v, panel)
    return v.cpu().numpy(), panel.cpu().numpy(), R.stats()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_single_renders(setup, graph):
    torch, lfdpr, R, ws, ids = setup
    B = lfdpr.Batch(R, ids, [w.views for w in ws])
    B.use_graph(graph)
    views = B.alloc_views()
    panels = torch.empty((len(ws), ws[0].lens.Hp, ws[0].lens.Wp, 3), dtype=torch.uint8, device="cuda")
    for frame in (0, 77, 400):
        models = [w.model(frame + 13 * k) for k, w in enumerate(ws)]
        B.render(models, views, panels)
        torch.cuda.synchronize()
        bv, bp = views.cpu().numpy(), panels.cpu().numpy()
        bst = B.stats()
        tot_pts = 0
        for k, w in enumerate(ws):
            sv, sp, st = single(torch, R, w, ids[k], models[k])
            np.testing.assert_array_equal(bv[k], sv, err_msg=f"item {k} frame {frame} views")
            np.testing.assert_array_equal(bp[k], sp, err_msg=f"item {k} frame {frame} panel")
            tot_pts += st["points"]
        assert bst["points"] == tot_pts
        print(f"frame {frame}: {bst['points']} points over {len(ws)} scenes, graph={graph}", flush=True)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_items_match_oracle(setup, graph):
    """Every item of a batch frame (scenes of different sizes, cones and eye
    distances) against the oracle's render of that scene: views, panel (the
    context's lens) and the point and point-view totals."""
    torch, lfdpr, R, ws, ids = setup
    B = lfdpr.Batch(R, ids, [w.views for w in ws])
    B.use_graph(graph)
    views = B.alloc_views()
    panels = torch.empty((len(ws), ws[0].lens.Hp, ws[0].lens.Wp, 3), dtype=torch.uint8, device="cuda")
    models = [w.model(211 + 29 * k) for k, w in enumerate(ws)]
    for _ in range(2 if graph else 1):   # graph: capture, then a replay
        B.render(models, views, panels)
    torch.cuda.synchronize()
    bv, bp, bst = views.cpu().numpy(), panels.cpu().numpy(), B.stats()
    pts = pv = 0
    for k, w in enumerate(ws):
        o = O.render(w.scene, w.views, models[k])
        np.testing.assert_array_equal(bv[k].view(np.uint32), o["rgba"], err_msg=f"item {k} views")
        np.testing.assert_array_equal(bp[k], O.interleave(o["rgba"], ws[0].lens), err_msg=f"item {k} panel")
        pts += o["n_points"]
        pv += o["stats"]["point_views"]
    assert bst["points"] == pts and bst["point_views"] == pv
    B.close()


def test_graph_replays_with_interleaved_eager_work(setup):
    """Several replays, with eager frames and synchronisations between them,
    each equal to an eager batch render of the same models."""
    torch, lfdpr, R, ws, ids = setup
    G = lfdpr.Batch(R, ids, [w.views for w in ws])
    E = lfdpr.Batch(R, ids, [w.views for w in ws])
    E.use_graph(False)
    vg, ve = G.alloc_views(), E.alloc_views()
    for frame in (5, 6, 600, 5):
        models = [w.model(frame * (k + 1)) for k, w in enumerate(ws)]
        G.render(models, vg)
        torch.cuda.synchronize()
        E.render(models, ve)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(vg.cpu().numpy(), ve.cpu().numpy())


@pytest.mark.parametrize("graph", [False, True])
def test_pipelined_batches_equal_serial_batches(setup, graph):
    """Two batch calls in flight (a call's point generation on the batch's
    second stream while the previous call splats): every call's views and
    panels equal a serial batch's bit for bit, statistics describe the last
    call, and switching back to one in flight (graph replay) keeps results."""
    torch, lfdpr, R, ws, ids = setup
    S = lfdpr.Batch(R, ids, [w.views for w in ws])
    S.use_graph(False)
    P = lfdpr.Batch(R, ids, [w.views for w in ws])
    P.use_graph(graph)
    P.set_frames_in_flight(2)

    def panels():
        return torch.empty((len(ws), ws[0].lens.Hp, ws[0].lens.Wp, 3), dtype=torch.uint8, device="cuda")

    frames = [0, 77, 400, 5, 6, 6]
    want = []
    for f in frames:
        models = [w.model(f + 13 * k) for k, w in enumerate(ws)]
        v, p = S.alloc_views(), panels()
        S.render(models, v, p)
        torch.cuda.synchronize()
        want.append((v.cpu().numpy(), p.cpu().numpy()))
    last = S.stats()
    got = []
    for f in frames:
        models = [w.model(f + 13 * k) for k, w in enumerate(ws)]
        v, p = P.alloc_views(), panels()
        P.render(models, v, p)
        got.append((v, p))
    torch.cuda.synchronize()
    assert P.stats() == last
    for f, (wv, wp), (v, p) in zip(frames, want, got):
        np.testing.assert_array_equal(v.cpu().numpy(), wv, err_msg=f"frame {f} views")
        np.testing.assert_array_equal(p.cpu().numpy(), wp, err_msg=f"frame {f} panels")
    # the autotuner with two calls in flight, then a pipelined call in its shape
    models = [w.model(77 + 13 * k) for k, w in enumerate(ws)]
    v = P.alloc_views()
    P.autotune(models, v)
    v, p = P.alloc_views(), panels()
    P.render(models, v, p)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(v.cpu().numpy(), want[1][0])
    np.testing.assert_array_equal(p.cpu().numpy(), want[1][1])
    P.set_frames_in_flight(1)
    P.use_graph(True)
    models = [w.model(31 + 13 * k) for k, w in enumerate(ws)]
    for B in (S, P):
        v, p = B.alloc_views(), panels()
        for _ in range(2):
            B.render(models, v, p)
        torch.cuda.synchronize()
        got.append((v.cpu().numpy(), p.cpu().numpy()))
    np.testing.assert_array_equal(got[-1][0], got[-2][0])
    np.testing.assert_array_equal(got[-1][1], got[-2][1])
    with pytest.raises(lfdpr.LfdprError):
        P.set_frames_in_flight(3)
    S.close()
    P.close()


def test_autotune_keeps_results(setup):
    torch, lfdpr, R, ws, ids = setup
    B = lfdpr.Batch(R, ids, [w.views for w in ws])
    views = B.alloc_views()
    models = [w.model(9) for w in ws]
    B.use_graph(False)
    B.render(models, views)
    torch.cuda.synchronize()
    ref = views.cpu().numpy().copy()
    res = B.autotune(models, views)
    print("batch autotune:", res["best"], flush=True)
    # ten point-order shapes, then the quilt under each band height that fits
    assert 10 < len(res["entries"]) <= 14 and res["best"] in res["entries"]
    assert {e["splat_order"] for e in res["entries"][10:]} == {lfdpr.SPLAT_QUILT}
    B.use_graph(True)
    B.render(models, views)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(views.cpu().numpy(), ref)
    # single-frame autotune + explicit launch shapes give identical views
    w = ws[2]
    R.set_views(w.views)
    v, _ = R.alloc_views()
    outs = []
    for blocks, layout in ((1024, 0), (16384, 1), (3000, 1)):
        R.set_launch(blocks, layout)
        R.render_frame(ids[2], w.model(9), v)
        outs.append(v.cpu().numpy().copy())
    r1 = R.autotune(ids[2], w.model(9), v)
    R.render_frame(ids[2], w.model(9), v)
    outs.append(v.cpu().numpy().copy())
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    print("frame autotune:", r1["best"], flush=True)


def test_batch16_full_size_matches_single_renders():
    """The benchmark's 16-scene batch (10.2M triangles, 50k-4M per scene) in one
    hipGraph replay after the autotuner: every scene's views and panel equal a
    single-scene render of the same frame, which the parity tests tie to the
    oracle."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_19901_amd import lfdpr
    ws = scenes.batch_workloads(seed=400)
    R = lfdpr.Renderer(0)
    ids = [R.upload_scene(w.scene) for w in ws]
    R.set_lens(ws[0].lens)
    B = lfdpr.Batch(R, ids, [w.views for w in ws], point_capacity=96 << 20)
    views = B.alloc_views()
    panels = torch.empty((len(ws), ws[0].lens.Hp, ws[0].lens.Wp, 3), dtype=torch.uint8, device="cuda")
    models = [w.model(7 + 37 * k) for k, w in enumerate(ws)]
    B.use_graph(False)
    print("batch16 autotune:", B.autotune(models, views)["best"], flush=True)
    B.use_graph(True)
    for _ in range(2):   # capture, then a replay
        B.render(models, views, panels)
    torch.cuda.synchronize()
    bst = B.stats()
    bv, bp = views.cpu().numpy(), panels.cpu().numpy()
    tot = 0
    for k, w in enumerate(ws):
        R.set_views(w.views, point_capacity=32 << 20)
        v, _ = R.alloc_views()
        R.render_frame(ids[k], models[k], v)
        panel = torch.empty((w.lens.Hp, w.lens.Wp, 3), dtype=torch.uint8, device="cuda")
        R.reconstruct(v, panel)
        np.testing.assert_array_equal(bv[k], v.cpu().numpy(), err_msg=f"scene {k} views")
        np.testing.assert_array_equal(bp[k], panel.cpu().numpy(), err_msg=f"scene {k} panel")
        tot += R.stats()["point_views"]
    assert bst["point_views"] == tot
    print(f"batch16: {bst['points']} points, {tot} point-views, all scenes identical", flush=True)
    # the two smallest scenes (about 55k triangles, 48 views of 512^2 each)
    # straight against the oracle
    for k in sorted(range(len(ws)), key=lambda k: ws[k].scene.n_tris)[:2]:
        o = O.render(ws[k].scene, ws[k].views, models[k])
        np.testing.assert_array_equal(bv[k].view(np.uint32), o["rgba"], err_msg=f"scene {k} views vs oracle")
        np.testing.assert_array_equal(bp[k], O.interleave(o["rgba"], ws[0].lens), err_msg=f"scene {k} panel vs oracle")
        print(f"batch16 scene {k} ({ws[k].scene.n_tris} triangles): equal to the oracle", flush=True)
    # two batch calls in flight: another frame, then this one, equal to the replay
    B.set_frames_in_flight(2)
    other = B.alloc_views()
    B.render([w.model(900 + k) for k, w in enumerate(ws)], other)
    v2 = B.alloc_views()
    p2 = torch.empty_like(panels)
    B.render(models, v2, p2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(v2.cpu().numpy(), bv)
    np.testing.assert_array_equal(p2.cpu().numpy(), bp)
    assert B.stats() == bst
    B.close()


def test_lifetimes_are_enforced():
    """A scene rendered by a live batch cannot be freed, and a context with live
    batches or networks cannot be destroyed; both work once those are gone."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_19901_amd import lfdpr
    w = scenes.small_display(seed=70, V=8, W=64, H=64)
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    B = lfdpr.Batch(R, [sid], [w.views])
    assert lib_call(lfdpr, "lfdpr_scene_free", R.h, sid) == lfdpr.LFDPR_ESTATE
    net = lfdpr.Net(R, 8, 64, 64)
    assert lfdpr.lib().lfdpr_destroy(R.h) == lfdpr.LFDPR_ESTATE
    B.close()
    assert lfdpr.lib().lfdpr_destroy(R.h) == lfdpr.LFDPR_ESTATE   # the network is still alive
    net.close()
    assert lib_call(lfdpr, "lfdpr_scene_free", R.h, sid) == lfdpr.LFDPR_OK
    R.close()


def lib_call(lfdpr, name, *args):
    return getattr(lfdpr.lib(), name)(*args)
