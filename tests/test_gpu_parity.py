"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: point counts, the point buffer (triangle, cell, flags, both mip texels),
per-triangle set-up records, per-pixel keys (colour and depth) and panel
indexing are bit-exact.  The image bar of the method (<= 1e-4 differing pixels
and >= 60 dB PSNR) is asserted as well; bit-exactness implies it."""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
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


def _renderer(torch_cuda):
    from paper_2601_19901_amd import lfdpr
    return lfdpr.Renderer(0)


def psnr(a, b):
    a = O.unpack_rgba(a)[..., :3].astype(np.float64)
    b = O.unpack_rgba(b)[..., :3].astype(np.float64)
    mse = ((a - b) ** 2).mean()
    return math.inf if mse == 0 else 10 * math.log10(255.0 ** 2 / mse)


def run_gpu(R, sid, w, model, nt, with_dbg=True):
    torch = R._torch
    if with_dbg:
        df = torch.zeros((nt, 8), dtype=torch.float32, device="cuda")
        di = torch.zeros((nt, 8), dtype=torch.int32, device="cuda")
        R.set_debug_records(df, di)
    views, depth = R.alloc_views(with_depth=True)
    R.render_frame(sid, model, views, depth)
    st = R.stats()
    out = dict(stats=st, rgba=views.cpu().numpy().view(np.uint32), depth=depth.cpu().numpy(),
               counts=R.counts(nt), points=R.points(), views_t=views)
    if with_dbg:
        out["dbgf"] = df.cpu().numpy()
        out["dbgi"] = di.cpu().numpy()
        R.set_debug_records(None, None)
    return out


def assert_parity(g, o, nt, label):
    _log(f"[{label}] gpu stats {g['stats']}  oracle {o['stats']}")
    # per-triangle set-up records and counts: bit-exact
    np.testing.assert_array_equal(g["dbgi"], o["trii"], err_msg=f"{label}: int set-up records")
    np.testing.assert_array_equal(g["dbgf"].view(np.uint32), o["trif"].view(np.uint32), err_msg=f"{label}: float set-up records")
    np.testing.assert_array_equal(g["counts"], o["count"].astype(np.uint32), err_msg=f"{label}: counts")
    assert g["stats"]["points"] == o["n_points"]
    assert g["stats"]["active_tris"] == o["stats"]["active_tris"]
    assert g["stats"]["point_views"] == o["stats"]["point_views"]
    assert g["stats"]["overflow_tris"] == o["stats"]["overflow_tris"]
    gp, op = g["points"], o["points"]
    for k in ("tri", "i", "j", "flags", "tvmin", "tvmax"):
        np.testing.assert_array_equal(gp[k], op[k].astype(gp[k].dtype), err_msg=f"{label}: points.{k}")
    # images: colour and depth bit-exact
    diff = (g["rgba"] != o["rgba"]).mean()
    p = psnr(g["rgba"], o["rgba"])
    _log(f"[{label}] differing pixels {diff:.3e}  PSNR {p}")
    assert diff <= 1e-4 and p >= 60.0
    np.testing.assert_array_equal(g["rgba"], o["rgba"], err_msg=f"{label}: views")
    np.testing.assert_array_equal(g["depth"].view(np.uint32), o["depth"].view(np.uint32), err_msg=f"{label}: depth")


@pytest.mark.parametrize("frame", [0, 137])
def test_tiny_parity(torch_cuda, frame):
    w = scenes.tiny()
    _log(f"tiny frame {frame}: {w.scene.n_tris} tris, {w.views.V} views {w.views.W}x{w.views.H}")
    o = O.render(w.scene, w.views, w.model(frame))
    R = _renderer(torch_cuda)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    g = run_gpu(R, sid, w, w.model(frame), w.scene.n_tris)
    assert_parity(g, o, w.scene.n_tris, f"tiny f{frame}")


@pytest.mark.parametrize("seed,frame,mip", [(7, 0, True), (7, 250, True), (8, 40, False)])
def test_small_display_parity(torch_cuda, seed, frame, mip):
    w = scenes.small_display(seed=seed)
    w.views.mip = mip
    _log(f"small-display seed {seed} frame {frame} mip {mip}: {w.scene.n_tris} tris")
    o = O.render(w.scene, w.views, w.model(frame))
    R = _renderer(torch_cuda)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    g = run_gpu(R, sid, w, w.model(frame), w.scene.n_tris)
    assert_parity(g, o, w.scene.n_tris, f"small s{seed} f{frame}")


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_panel_parity(torch_cuda, mode):
    torch = torch_cuda
    w = scenes.small_display(seed=9)
    o = O.render(w.scene, w.views, w.model(11))
    R = _renderer(torch_cuda)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    R.set_lens(w.lens, mode=mode)
    views, _ = R.alloc_views()
    R.render_frame(sid, w.model(11), views)
    panel = torch.empty((w.lens.Hp, w.lens.Wp, 3), dtype=torch.uint8, device="cuda")
    R.reconstruct(views, panel)
    want = O.interleave(o["rgba"], w.lens, mode=mode)
    got = panel.cpu().numpy()
    _log(f"panel mode {mode}: differing subpixels {(got != want).mean():.3e}")
    np.testing.assert_array_equal(got, want)


def test_interleave_index_map_on_gpu(torch_cuda):
    """View-id fill reads out the lens index map, for the prototype lens."""
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    V, H, W = 48, 64, 80
    views = np.zeros((V, H, W), np.uint32)
    for v in range(V):
        views[v] = v * 0x00010101
    ln = scenes.display().lens if False else scenes.LensParams(Wp=640, Hp=400, pitch_subpx=3 * 3840 / 479.36,
                                                               slope=-math.tan(math.radians(9.66)), offset=0.21)
    R = _renderer(torch_cuda)
    R.set_lens(ln)
    tv = torch.from_numpy(views.view(np.int32)).cuda()
    panel = torch.empty((ln.Hp, ln.Wp, 3), dtype=torch.uint8, device="cuda")
    R.reconstruct(tv, panel)
    np.testing.assert_array_equal(panel.cpu().numpy(), O.interleave(views, ln))


def test_angular_supersampling_parity(torch_cuda):
    torch = torch_cuda
    w = scenes.small_display(seed=12, S=4, V=8)
    _log(f"angular SS: {w.views.V}x{w.views.S} sub-views")
    o = O.render(w.scene, w.views, w.model(3))
    R = _renderer(torch_cuda)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    g = run_gpu(R, sid, w, w.model(3), w.scene.n_tris)
    assert_parity(g, o, w.scene.n_tris, "ss4")
    out = torch.empty((w.views.V, w.views.H, w.views.W), dtype=torch.int32, device="cuda")
    R.angular_filter(g["views_t"], out)
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), O.angular_filter(o["rgba"], w.views))


def test_determinism_and_launch_shape_independence(torch_cuda):
    torch = torch_cuda
    w = scenes.small_display(seed=13)
    R = _renderer(torch_cuda)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    imgs = []
    for k in range(3):
        v, d = R.alloc_views(with_depth=True)
        R.render_frame(sid, w.model(5), v, d)
        imgs.append((v.cpu().numpy().copy(), d.cpu().numpy().copy()))
    for a, b in imgs[1:]:
        np.testing.assert_array_equal(a, imgs[0][0])
        np.testing.assert_array_equal(b.view(np.uint32), imgs[0][1].view(np.uint32))


@pytest.mark.parametrize("in_flight", [1, 2])
def test_edge_cases(torch_cuda, in_flight):
    torch = torch_cuda
    from paper_2601_19901_amd import lfdpr
    w = scenes.tiny()
    R = _renderer(torch_cuda)
    R.set_frames_in_flight(in_flight)
    sid = R.upload_scene(w.scene)
    # render before set_views -> state error
    v = torch.empty((8, 128, 128), dtype=torch.int32, device="cuda")
    with pytest.raises(lfdpr.LfdprError) as e:
        R.render_frame(sid, w.model(0), v)
    assert e.value.code == lfdpr.LFDPR_ESTATE
    R.set_views(w.views)
    # unknown scene
    with pytest.raises(lfdpr.LfdprError):
        R.render_frame(999, w.model(0), v)
    # scene entirely behind the eyes: nothing drawn, no points
    m = w.model(0).copy()
    m[2, 3] = -10.0
    R.render_frame(sid, m, v)
    st = R.stats()
    assert st["points"] == 0 and st["active_tris"] == 0
    assert (v.cpu().numpy() == 0).all()
    # empty scene (no triangles)
    empty = scenes.Scene(w.scene.pos[:3].copy(), w.scene.uv[:3].copy(), np.zeros((0, 3), np.uint32),
                         np.zeros(0, np.uint16), w.scene.textures)
    eid = R.upload_scene(empty)
    R.render_frame(eid, w.model(0), v)
    assert R.stats()["points"] == 0
    # point capacity overflow is reported, not a fault
    R.set_views(w.views, point_capacity=1000)
    R.render_frame(sid, w.model(0), v)
    st = R.stats(allow_overflow=True)
    assert st["point_overflow"] == 1 and st["points"] > 1000
    with pytest.raises(lfdpr.LfdprError) as e:
        R.stats()
    assert e.value.code == lfdpr.LFDPR_EOVERFLOW
    # bad parameters are rejected
    bad = scenes.ViewParams(V=0, W=16, H=16, fovy_deg=30, aspect=1, D=1, cone_deg=40, znear=0.1)
    with pytest.raises(lfdpr.LfdprError) as e:
        R.set_views(bad)
    assert e.value.code == lfdpr.LFDPR_EINVAL
    # after recovery, a normal frame matches the oracle again
    R.set_views(w.views)
    o = O.render(w.scene, w.views, w.model(2))
    g = run_gpu(R, sid, w, w.model(2), w.scene.n_tris)
    assert_parity(g, o, w.scene.n_tris, f"after-errors, {in_flight} in flight")


@pytest.fixture(scope="module")
def display_workload():
    _log("generating display-size scene (1M triangles)")
    return scenes.display()


def _quilt_against_oracle(R, sid, w, model, o, label):
    """The same frame under the quilt order at its automatic tile (the one the
    autotuner times): views, depth and written pixels against the oracle."""
    from paper_2601_19901_amd import lfdpr
    R.set_splat_order(lfdpr.SPLAT_QUILT)
    R.set_quilt_tile(0, 0)
    views, depth = R.alloc_views(with_depth=True)
    R.render_frame(sid, model, views, depth)
    st = R.stats()
    _log(f"[{label} quilt] {st}")
    assert st["splat_order"] == lfdpr.SPLAT_QUILT
    np.testing.assert_array_equal(views.cpu().numpy().view(np.uint32), o["rgba"], err_msg=f"{label} quilt: views")
    np.testing.assert_array_equal(depth.cpu().numpy().view(np.uint32), o["depth"].view(np.uint32),
                                  err_msg=f"{label} quilt: depth")
    assert st["written_px"] == o["stats"]["fragments"] - o["stats"]["misses"]
    R.set_splat_order(lfdpr.SPLAT_POINT)
    return views


def test_display_size_parity(torch_cuda, display_workload):
    """Full display workload (999,168 triangles, 48 views of 512^2) in the
    launch configurations the benchmark times (the point order and the
    quilt, between which its autotuner chooses): everything bit-exact."""
    w = display_workload
    frame = 17
    _log("oracle: display frame", frame)
    o = O.render(w.scene, w.views, w.model(frame))
    R = _renderer(torch_cuda)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    g = run_gpu(R, sid, w, w.model(frame), w.scene.n_tris)
    assert_parity(g, o, w.scene.n_tris, "display")
    torch = torch_cuda
    R.set_lens(w.lens)
    panel = torch.empty((w.lens.Hp, w.lens.Wp, 3), dtype=torch.uint8, device="cuda")
    R.reconstruct(g["views_t"], panel)
    np.testing.assert_array_equal(panel.cpu().numpy(), O.interleave(o["rgba"], w.lens))
    _quilt_against_oracle(R, sid, w, w.model(frame), o, "display")


def test_display_4m_ss4_parity(torch_cuda):
    """The 4M-triangle workload with 4x angular supersampling (192 rendered
    views of 512^2) in the benchmark's launch configurations (its autotuner
    takes the quilt here): counts, points, all 192 sub-views with depth, the
    angular filter to 48 views and the panel, bit-exact against the oracle
    (the oracle takes about a minute)."""
    torch = torch_cuda
    _log("generating display-4M-ss4 scene (3,996,672 triangles)")
    w = scenes.display_4m(seed=3)
    frame = 5
    _log("oracle: display-4M-ss4 frame", frame)
    o = O.render(w.scene, w.views, w.model(frame))
    R = _renderer(torch_cuda)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views, point_capacity=48 << 20)
    g = run_gpu(R, sid, w, w.model(frame), w.scene.n_tris)
    assert g["stats"]["n_views"] == 192
    assert_parity(g, o, w.scene.n_tris, "display-4M-ss4")
    filt = torch.empty((w.views.V, w.views.H, w.views.W), dtype=torch.int32, device="cuda")
    R.angular_filter(g["views_t"], filt)
    of = O.angular_filter(o["rgba"], w.views)
    np.testing.assert_array_equal(filt.cpu().numpy().view(np.uint32), of)
    R.set_lens(w.lens)
    panel = torch.empty((w.lens.Hp, w.lens.Wp, 3), dtype=torch.uint8, device="cuda")
    R.reconstruct(filt, panel)
    np.testing.assert_array_equal(panel.cpu().numpy(), O.interleave(of, w.lens))
    vq = _quilt_against_oracle(R, sid, w, w.model(frame), o, "display-4M-ss4")
    R.angular_filter(vq, filt)
    np.testing.assert_array_equal(filt.cpu().numpy().view(np.uint32), of)


def test_spatial_supersampling_parity(torch_cuda):
    """2x spatial supersampling (views at twice the resolution, panel through
    the spatial Gaussian taps): views, depth, counts and panel bit-exact."""
    torch = torch_cuda
    w = scenes.spatial_ss(scenes.small_display(seed=7))
    assert (w.views.W, w.views.H) == (192, 192)
    o = O.render(w.scene, w.views, w.model(40))
    R = _renderer(torch_cuda)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    g = run_gpu(R, sid, w, w.model(40), w.scene.n_tris)
    assert_parity(g, o, w.scene.n_tris, "spatial-2x")
    R.set_lens(w.lens)
    panel = torch.empty((w.lens.Hp, w.lens.Wp, 3), dtype=torch.uint8, device="cuda")
    R.reconstruct(g["views_t"], panel)
    np.testing.assert_array_equal(panel.cpu().numpy(), O.interleave(o["rgba"], w.lens))


@pytest.mark.parametrize("mode", [scenes.RECON_ANGULAR, scenes.RECON_BOTH])
def test_direct_panel_reconstruction_parity(torch_cuda, mode):
    """The panel reconstructed straight from all S*V sub-views (no angular
    pre-filter), angular taps spanning +-S sub-view intervals: bit-exact."""
    torch = torch_cuda
    w = scenes.small_display(seed=12, S=4, V=8)
    o = O.render(w.scene, w.views, w.model(9))
    R = _renderer(torch_cuda)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views)
    g = run_gpu(R, sid, w, w.model(9), w.scene.n_tris, with_dbg=False)
    np.testing.assert_array_equal(g["rgba"], o["rgba"])
    lens = scenes.direct_panel_lens(w, mode=mode)
    R.set_lens(lens)
    panel = torch.empty((lens.Hp, lens.Wp, 3), dtype=torch.uint8, device="cuda")
    R.reconstruct(g["views_t"], panel)
    assert g["views_t"].shape[0] == 32
    np.testing.assert_array_equal(panel.cpu().numpy(), O.interleave(o["rgba"], lens))
