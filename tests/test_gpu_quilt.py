"""The row-band quilt (lfdpr_set_splat_order(LFDPR_SPLAT_QUILT)): the views'
64-bit keys (Sec. 5.1) resolved in LDS tiles of q_rows pixel rows x q_views
views, the views written straight from the tiles.  It does the point order's
(point, view, pixel) work in another grouping, so views, depth and statistics
must be identical bit for bit: tied to the oracle directly at small sizes and
through the point order (itself tied to the oracle) at display size, for
every tile shape, shaded frames, two frames in flight and the per-point
fallback taken when the band lists overflow."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_19901_amd import scenes
from test_gpu_parity import _log, assert_parity, run_gpu

pytestmark = pytest.mark.gpu

QUILT_KEYS = ("quilt_rows", "quilt_views", "quilt_entries")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _render(R, sid, model, order):
    R.set_splat_order(order)
    v, d = R.alloc_views(with_depth=True)
    R.render_frame(sid, model, v, d)
    return v.cpu().numpy(), d.cpu().numpy(), R.stats()


def _same_as_point(R, sid, model, label, rows=0, views=0):
    """Quilt frame (tile rows x views; 0, 0 = automatic) against the point
    order; returns the quilt's (rows, views, entries)."""
    from paper_2601_19901_amd import lfdpr
    R.set_quilt_tile(rows, views)
    vq, dq, sq = _render(R, sid, model, lfdpr.SPLAT_QUILT)
    vp, dp, sp = _render(R, sid, model, lfdpr.SPLAT_POINT)
    _log(f"[{label}] quilt {sq}; point {sp}")
    assert sq.pop("splat_order") == lfdpr.SPLAT_QUILT and sp.pop("splat_order") == lfdpr.SPLAT_POINT
    q = tuple(sq.pop(k) for k in QUILT_KEYS)
    assert tuple(sp.pop(k) for k in QUILT_KEYS) == (0, 0, -1)
    H, nv = R.vp.H, R.vp.V * R.vp.S
    assert 1 <= q[0] <= H and 1 <= q[1] <= nv and q[2] >= 0
    if rows:
        assert q[:2] == (min(rows, H), min(views, nv))
    assert sq == sp and sp["written_px"] > 0
    np.testing.assert_array_equal(vq, vp, err_msg=f"{label}: views")
    np.testing.assert_array_equal(dq.view(np.uint32), dp.view(np.uint32), err_msg=f"{label}: depth")
    return q


@pytest.mark.parametrize("kind,seed,frame,mip", [("tiny", 1, 0, True), ("tiny", 1, 137, True),
                                                 ("small", 7, 250, True), ("small", 8, 40, False)])
def test_quilt_matches_the_oracle(torch_cuda, kind, seed, frame, mip):
    from paper_2601_19901_amd import lfdpr
    w = {"tiny": scenes.tiny, "small": scenes.small_display}[kind](seed=seed)
    w.views.mip = mip
    o = O.render(w.scene, w.views, w.model(frame))
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    R.set_splat_order(lfdpr.SPLAT_QUILT)
    g = run_gpu(R, sid, w, w.model(frame), w.scene.n_tris)
    assert g["stats"]["splat_order"] == lfdpr.SPLAT_QUILT
    assert_parity(g, o, w.scene.n_tris, f"quilt {kind} s{seed} f{frame}")
    assert g["stats"]["written_px"] == o["stats"]["fragments"] - o["stats"]["misses"]


@pytest.mark.parametrize("rows,views", [(0, 0), (1, 1), (3, 5), (4, 12), (8, 2), (96, 2), (200, 2), (7, 11)])
def test_every_tile_shape_agrees_with_the_point_order(torch_cuda, rows, views):
    """Tiles of one row and one view up to all rows of two views (96 x 96
    views); band heights that do not divide H and view counts that do not
    divide V (partial last band and subset); rows beyond the rig are clipped."""
    from paper_2601_19901_amd import lfdpr
    w = scenes.small_display(seed=11)
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    _same_as_point(R, sid, w.model(77), f"small-display tile {rows}x{views}", rows, views)


def test_band_entries_shrink_with_taller_bands(torch_cuda):
    """Each point is listed once per band its splat's rows reach: taller bands
    list no more entries, and one band over the whole view lists each point
    with rows at most once."""
    from paper_2601_19901_amd import lfdpr
    w = scenes.small_display(seed=12)
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    ents = []
    for rows in (1, 2, 4, 8, w.views.H):
        ents.append(_same_as_point(R, sid, w.model(5), f"entries at {rows} rows", rows, 1)[2])
    _log(f"band entries at 1, 2, 4, 8, H rows: {ents}")
    assert all(a >= b for a, b in zip(ents, ents[1:]))
    assert 0 < ents[-1] <= R.stats()["points"]


def test_a_tile_beyond_the_lds_is_refused(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    w = scenes.small_display(seed=11)
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    R.set_splat_order(lfdpr.SPLAT_QUILT)
    R.set_quilt_tile(96, 12)  # 96 rows x 12 views x 96 columns x 8 B = 864 KiB
    v, _ = R.alloc_views()
    with pytest.raises(lfdpr.LfdprError) as e:
        R.render_frame(sid, w.model(1), v)
    assert e.value.code == lfdpr.LFDPR_EINVAL
    R.set_quilt_tile(0, 0)
    R.render_frame(sid, w.model(1), v)
    assert R.stats()["splat_order"] == lfdpr.SPLAT_QUILT


@pytest.mark.parametrize("S,mip", [(1, False), (4, True)])
def test_quilt_with_sub_views(torch_cuda, S, mip):
    from paper_2601_19901_amd import lfdpr
    w = scenes.small_display(seed=13, S=S)
    w.views.mip = mip
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    _same_as_point(R, sid, w.model(300), f"small-display S={S}")
    _same_as_point(R, sid, w.model(301), f"small-display S={S}, 2 rows x 5 views", 2, 5)


def test_quilt_shaded(torch_cuda):
    """Physically based shading: the shaded colour per (point, view) is the
    same in a tile as in the point order."""
    from paper_2601_19901_amd import lfdpr
    w = scenes.with_pbr(scenes.small_display(seed=14))
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    R.set_shading(w.shading)
    _same_as_point(R, sid, w.model(42), "small-display PBR")
    _same_as_point(R, sid, w.model(43), "small-display PBR, 1 row x 3 views", 1, 3)


def test_overflowed_band_lists_fall_back_to_the_point_order(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    w = scenes.small_display(seed=15)
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    m = w.model(9)
    vp, dp, sp = _render(R, sid, m, lfdpr.SPLAT_POINT)
    R.set_quilt_capacity(1000)
    vq, dq, sq = _render(R, sid, m, lfdpr.SPLAT_QUILT)
    _log(f"quilt with 1000 entries: {sq}")
    assert sq["splat_order"] == lfdpr.SPLAT_POINT and sq["quilt_entries"] > 1000
    np.testing.assert_array_equal(vq, vp)
    np.testing.assert_array_equal(dq.view(np.uint32), dp.view(np.uint32))
    assert sq["written_px"] == sp["written_px"]
    # the next frame with room again takes the quilt; then overflow once more
    R.set_quilt_capacity(0)
    vq2, dq2, sq2 = _render(R, sid, m, lfdpr.SPLAT_QUILT)
    assert sq2["splat_order"] == lfdpr.SPLAT_QUILT and sq2["quilt_entries"] == sq["quilt_entries"]
    np.testing.assert_array_equal(vq2, vp)
    R.set_quilt_capacity(1000)
    vq3, _, sq3 = _render(R, sid, m, lfdpr.SPLAT_QUILT)
    assert sq3["splat_order"] == lfdpr.SPLAT_POINT
    np.testing.assert_array_equal(vq3, vp)


def test_quilt_at_display_size(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    w = scenes.display()
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    for f, (rows, views) in ((17, (0, 0)), (600, (2, 16)), (601, (1, 24))):
        q = _same_as_point(R, sid, w.model(f), f"display-1M frame {f}", rows, views)
        _log(f"display-1M frame {f}: tile {q[0]} rows x {q[1]} views, {q[2]} entries")
    # two frames in flight under the quilt against the serial point order
    R.set_quilt_tile(0, 0)
    R.set_splat_order(lfdpr.SPLAT_QUILT)
    R.set_frames_in_flight(2)
    outs = []
    for f in (3, 4, 5):
        v, _ = R.alloc_views()
        R.render_frame(sid, w.model(f), v)
        outs.append(v)
    assert R.stats()["splat_order"] == lfdpr.SPLAT_QUILT
    R.set_frames_in_flight(1)
    for f, v in zip((3, 4, 5), outs):
        vp, _, _ = _render(R, sid, w.model(f), lfdpr.SPLAT_POINT)
        np.testing.assert_array_equal(v.cpu().numpy(), vp, err_msg=f"pipelined frame {f}")


def test_quilt_shaded_at_display_size(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    w = scenes.with_pbr(scenes.display())
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    R.set_shading(w.shading)
    _same_as_point(R, sid, w.model(17), "display-1M PBR frame 17")


def test_autotune_takes_the_quilt_into_account(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    w = scenes.small_display(seed=16)
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    v, _ = R.alloc_views()
    res = R.autotune(sid, w.model(3), v)
    _log(f"autotune best {res['best']}")
    orders = {e["splat_order"] for e in res["entries"]}
    assert orders == {lfdpr.SPLAT_POINT, lfdpr.SPLAT_QUILT}
    assert all((e["quilt_rows"] > 0) == (e["splat_order"] == lfdpr.SPLAT_QUILT) for e in res["entries"])
    # whatever it kept, the frame equals the point order's
    v1, d1, s1 = _render_current(R, sid, w.model(4))
    assert s1["splat_order"] == res["best"]["splat_order"]
    vp, dp, _ = _render(R, sid, w.model(4), lfdpr.SPLAT_POINT)
    np.testing.assert_array_equal(v1, vp)
    np.testing.assert_array_equal(d1.view(np.uint32), dp.view(np.uint32))


def _render_current(R, sid, model):
    v, d = R.alloc_views(with_depth=True)
    R.render_frame(sid, model, v, d)
    return v.cpu().numpy(), d.cpu().numpy(), R.stats()


def _batch_scenes():
    ws = [scenes.small_display(seed=s, V=12, W=96, H=96, hf_quads=hq) for s, hq in ((70, 24), (71, 48), (72, 8))]
    for k, w in enumerate(ws):
        w.views.cone_deg = 30.0 + 7.0 * k
    return ws


def _batch_run(lfdpr, torch, R, ids, ws, order, tile, graph, in_flight, frames):
    R.set_splat_order(order)
    R.set_quilt_tile(*tile)
    B = lfdpr.Batch(R, ids, [w.views for w in ws])
    B.use_graph(graph)
    if in_flight == 2:
        B.set_frames_in_flight(2)
    outs = []
    for f in frames:
        models = [w.model(f + 9 * k) for k, w in enumerate(ws)]
        v = B.alloc_views()
        p = torch.empty((len(ws), ws[0].lens.Hp, ws[0].lens.Wp, 3), dtype=torch.uint8, device="cuda")
        B.render(models, v, p)
        outs.append((v, p))
    torch.cuda.synchronize()
    st = B.stats()
    res = [(v.cpu().numpy(), p.cpu().numpy()) for v, p in outs]
    B.close()
    return res, st


@pytest.mark.parametrize("tile", [(0, 0), (1, 5), (3, 12)])
def test_quilt_in_batches(torch_cuda, tile):
    """A batch of three scenes with different cones under the quilt (every
    item's bands in one set of lists and one tile launch) against the same
    batch per point: views, panels and statistics, eager, replayed from a
    hipGraph and with two calls in flight."""
    from paper_2601_19901_amd import lfdpr
    torch = torch_cuda
    ws = _batch_scenes()
    R = lfdpr.Renderer(0)
    ids = [R.upload_scene(w.scene) for w in ws]
    R.set_lens(ws[0].lens)
    frames = [50, 51, 52]
    want, sp = _batch_run(lfdpr, torch, R, ids, ws, lfdpr.SPLAT_POINT, (0, 0), False, 1, frames)
    for graph, fif in ((False, 1), (True, 1), (False, 2)):
        got, sq = _batch_run(lfdpr, torch, R, ids, ws, lfdpr.SPLAT_QUILT, tile, graph, fif, frames)
        _log(f"[batch quilt {tile} graph={graph} in flight {fif}] {sq}")
        assert sq.pop("splat_order") == lfdpr.SPLAT_QUILT
        q = tuple(sq.pop(k) for k in QUILT_KEYS)
        assert q[0] >= 1 and q[1] >= 1 and q[2] > 0
        if tile[0]:
            assert q[:2] == tile
        p = dict(sp)
        p.pop("splat_order")
        for k in QUILT_KEYS:
            p.pop(k)
        assert sq == p
        for f, (wv, wp), (gv, gp) in zip(frames, want, got):
            np.testing.assert_array_equal(gv, wv, err_msg=f"frame {f} views ({graph}, {fif})")
            np.testing.assert_array_equal(gp, wp, err_msg=f"frame {f} panels ({graph}, {fif})")


def test_quilt_in_shaded_batches(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    torch = torch_cuda
    ws = [scenes.with_pbr(w) for w in _batch_scenes()]
    R = lfdpr.Renderer(0)
    ids = [R.upload_scene(w.scene) for w in ws]
    R.set_lens(ws[0].lens)
    R.set_shading(ws[0].shading)
    want, _ = _batch_run(lfdpr, torch, R, ids, ws, lfdpr.SPLAT_POINT, (0, 0), False, 1, [7, 8])
    got, sq = _batch_run(lfdpr, torch, R, ids, ws, lfdpr.SPLAT_QUILT, (0, 0), True, 1, [7, 8])
    assert sq["splat_order"] == lfdpr.SPLAT_QUILT
    for (wv, wp), (gv, gp) in zip(want, got):
        np.testing.assert_array_equal(gv, wv)
        np.testing.assert_array_equal(gp, wp)


def test_batch_autotune_takes_the_quilt_into_account(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    torch = torch_cuda
    ws = _batch_scenes()
    R = lfdpr.Renderer(0)
    ids = [R.upload_scene(w.scene) for w in ws]
    R.set_lens(ws[0].lens)
    want, _ = _batch_run(lfdpr, torch, R, ids, ws, lfdpr.SPLAT_POINT, (0, 0), False, 1, [60])
    B = lfdpr.Batch(R, ids, [w.views for w in ws])
    models = [w.model(60 + 9 * k) for k, w in enumerate(ws)]
    v = B.alloc_views()
    res = B.autotune(models, v)
    _log(f"batch autotune best {res['best']}")
    assert lfdpr.SPLAT_QUILT in {e["splat_order"] for e in res["entries"]}
    B.use_graph(True)
    p = torch.empty((len(ws), ws[0].lens.Hp, ws[0].lens.Wp, 3), dtype=torch.uint8, device="cuda")
    for _ in range(2):
        B.render(models, v, p)
    torch.cuda.synchronize()
    assert B.stats()["splat_order"] == res["best"]["splat_order"]
    np.testing.assert_array_equal(v.cpu().numpy(), want[0][0])
    np.testing.assert_array_equal(p.cpu().numpy(), want[0][1])
    B.close()


def test_random_rigs_and_tiles(torch_cuda):
    """Twelve seeded rigs (odd view sizes, one to twenty views, sub-views) and
    tiles (bands that do not divide H, subsets that do not divide the views,
    bands taller than the view): the quilt equals the point order bit for
    bit, with depth and statistics."""
    from paper_2601_19901_amd import lfdpr
    rng = np.random.default_rng(2026)
    for case in range(12):
        W, H = int(rng.integers(17, 161)), int(rng.integers(5, 161))
        S = int(rng.choice([1, 1, 2]))
        V = int(rng.integers(1, 21))
        w = scenes.small_display(seed=100 + case, S=S, V=V, W=W, H=H, hf_quads=int(rng.choice([8, 24, 48])))
        nv = V * S
        rows = int(rng.choice([0, 1, 2, 3, 5, 8, H + 3]))
        views = 0 if rows == 0 else int(rng.integers(1, nv + 3))
        if rows and lfdpr.quilt_tile(W, H, nv, rows=rows, views=views) is None:
            rows, views = 0, 0
        R = lfdpr.Renderer(0)
        sid = R.upload_scene(w.scene)
        R.set_views(w.views)
        q = _same_as_point(R, sid, w.model(int(rng.integers(0, 1000))),
                           f"random rig {case}: {V}x{S} views of {W}x{H}, tile {rows}x{views}", rows, views)
        assert q[:2] == lfdpr.quilt_tile(W, H, nv, rows=rows, views=views)


@pytest.mark.parametrize("pbr", [False, True])
def test_lean_setup_records_equal_the_late_form(torch_cuda, pbr):
    """The quilt order runs the set-up form that stores a triangle's records
    before its lattice count; the point order the form that stores them at
    the end.  Same frame: set-up debug records, counts, points (with the
    material words when shaded) and views identical."""
    from paper_2601_19901_amd import lfdpr
    torch = torch_cuda
    w = scenes.small_display(seed=33, V=12, W=96, H=96)
    if pbr:
        w = scenes.with_pbr(w)
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    if pbr:
        R.set_shading(w.shading)
    nt = w.scene.n_tris
    out = {}
    for order in (lfdpr.SPLAT_POINT, lfdpr.SPLAT_QUILT):
        df = torch.zeros((nt, 8), dtype=torch.float32, device="cuda")
        di = torch.zeros((nt, 8), dtype=torch.int32, device="cuda")
        R.set_debug_records(df, di)
        R.set_splat_order(order)
        v, d = R.alloc_views(with_depth=True)
        R.render_frame(sid, w.model(44), v, d)
        st = R.stats()
        assert st["splat_order"] == order
        out[order] = dict(f=df.cpu().numpy(), i=di.cpu().numpy(), counts=R.counts(nt), points=R.points(),
                          mats=R.point_materials() if pbr else None, v=v.cpu().numpy(), pts=st["points"])
        R.set_debug_records(None, None)
    a, b = out[lfdpr.SPLAT_POINT], out[lfdpr.SPLAT_QUILT]
    np.testing.assert_array_equal(a["f"].view(np.uint32), b["f"].view(np.uint32))
    np.testing.assert_array_equal(a["i"], b["i"])
    np.testing.assert_array_equal(a["counts"], b["counts"])
    assert a["pts"] == b["pts"] > 0
    for k in a["points"]:
        np.testing.assert_array_equal(a["points"][k], b["points"][k], err_msg=f"points.{k}")
    if pbr:
        for k in a["mats"]:
            np.testing.assert_array_equal(a["mats"][k], b["mats"][k], err_msg=f"materials.{k}")
    np.testing.assert_array_equal(a["v"], b["v"])
    R.close()
