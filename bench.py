"""Benchmark of the LFDPR per-frame hot path on one MI355X.

Default workload (display-1M): one step = one whole frame of the hot path on
999,168 triangles, 16 RGBA8 2048^2 textures, 48 views of 512^2 and a
2560x1600 tilted-lenticular panel: triangle set-up, scan, point emission,
splat into all 48 views, resolve, interleave.  The scene rotates by 2*pi/1000
per frame.  Inputs are resident in HBM before the timed region starts.

--workload display-4M-ss4: 3,996,672 triangles rendered into 192 views (4x
angular supersampling), angular filter to 48 views, interleave;
display-4M-ss4-direct reconstructs the panel straight from the 192 sub-views.
--workload display-1M-spatial2x: 48 views of 1024^2 (2x spatial
supersampling), spatial reconstruction at the panel.
--workload batch16: 16 scenes of 50k-4M triangles per step, one hipGraph
replay after the launch autotuner.
--workload learned-display: display-1M rendered once plus the learned
angular reconstruction, beside the plain and 4x angular-SS frames.

Before the timed frames the library's autotuner chooses the splat order
(--splat-order auto, the default): the point order under each launch shape
and key layout, or the row-band quilt (keys resolved in LDS tiles) under each
band height; the line's splat_order holds the choice and every candidate's
time.

Prints one JSON line: value = point-view splats per second of whole-step
time (sum over points of the views their triangle is active in, divided by
step time), ms_per_step; per-stage ms, the roofline of the dominant kernel
(HIP events on the library's stream, inside the timed region) and, for the
default workload, the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
# VALU: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s (one FP32/INT op per lane per clock)
VALU_PEAK_GOPS = 256 * 64 * 2.4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic work of the splat, as the method's own operation count: about 25
# operations per (point, active view) (the splat's projected box and its colour,
# Eqs. 8-9) plus about 40 per written pixel (pixel ray, plane depth, lattice
# coordinates, ownership, 64-bit key and depth test).  Written pixels come from
# the GPU's own count of depth-test updates (lfdpr_stats.written_px).
SPLAT_OPS_PER_POINT_VIEW_ALG = 25
SPLAT_OPS_PER_WRITTEN_PX_ALG = 40
# A finer census of the definition as evaluated (visibility 2, vertex
# projection + Q8 + guard 12, area 7, triangle box 8, splat box 20, Eqs. 8-9
# colour 26, lattice offsets 6, edge set-up 12 per point-view; ray 1, plane 4,
# divide 1, checks 2, ur/wr 8, s/t 8, ownership 4, key 2, atomic 1 per
# written pixel), reported beside the algorithmic fraction.
SPLAT_OPS_PER_POINT_VIEW = 100
SPLAT_OPS_PER_WRITTEN_PX = 37
# physically based shading of a splat (unpack 9, shading normal 25, view and
# half vectors 26, four dot products 24, roughness/metallic 4, D 8, k 3, G 8,
# Fresnel power 5, specular 5, per channel 26 x 3) ~ 205 ops per written pixel
SPLAT_PBR_OPS_PER_WRITTEN_PX = 205
SETUP_OPS_PER_TRI_VIEW = 40        # visibility and the density terms per (triangle, view)
NET_FWD_BYTES_PER_PX = 16 + 80 + 128 + 128 + 80   # blur + four convolution layers, BF16
BYTES = {
    "setup": lambda s: s["nt"] * 78 + s["tris_with_points"] * 176,
    # the tile sums of 256 triangles each (8 B) in, their bases out
    "scan": lambda s: -(-s["nt"] // 256) * 16,
    # counts in, offsets out; emission records in; points out, texels in
    "emit": lambda s: s["nt"] * (4 + 8) + s["tris_with_points"] * 76 + s["points"] * (16 + 2 * 16),
    # point order: points and records in, one 8 B key per written pixel; quilt:
    # points, records and splat rectangles in, the views (4 B per pixel) out
    "splat": lambda s: (s["points"] * (16 + 112 + 48) + s["pixels"] * 4 if s.get("quilt")
                        else s["points"] * (16 + 112) + s["written_px"] * 8),
    "resolve": lambda s: 0 if s.get("quilt") else s["pixels"] * (8 + 8 + 4),
    "quilt_bin": lambda s: s["points"] * (4 + 4 + 4),
    "interleave": lambda s: s["panel_px"] * 3 + s["panel_px"] * 3 * 4,
    "angular_filter": lambda s: s["pixels"] * 4 + s["out_pixels"] * 4,
}


def splat_ops(pv: float, written: float, pbr: bool = False) -> float:
    """Algorithmic lane-operations of one splat launch (see above)."""
    per_px = SPLAT_OPS_PER_WRITTEN_PX_ALG + (SPLAT_PBR_OPS_PER_WRITTEN_PX if pbr else 0)
    return SPLAT_OPS_PER_POINT_VIEW_ALG * pv + per_px * written


def splat_ops_census(pv: float, written: float, pbr: bool = False) -> float:
    per_px = SPLAT_OPS_PER_WRITTEN_PX + (SPLAT_PBR_OPS_PER_WRITTEN_PX if pbr else 0)
    return SPLAT_OPS_PER_POINT_VIEW * pv + per_px * written


def roofline(stage_ms: dict, pv_per_frame: float, shape: dict, traffic=None, pbr: bool = False) -> dict:
    """Roofline object of the dominant kernel of a frame (stage ms from HIP events)."""
    dom = max(("setup", "emit", "splat", "resolve", "interleave", "scan", "angular_filter"),
              key=lambda k: stage_ms.get(k, 0.0))
    dom_ms = stage_ms[dom]
    peak_t = VALU_PEAK_GOPS / 1e3
    if dom == "splat":
        wpx = shape["written_px"]
        ops = splat_ops(pv_per_frame, wpx, pbr)
        achieved = ops / (dom_ms * 1e-3) / 1e12
        census = splat_ops_census(pv_per_frame, wpx, pbr) / (dom_ms * 1e-3) / 1e12
        return {"kernel": "k_splat_quilt" if shape.get("quilt") else "k_splat", "bound": "alu",
                "achieved": round(achieved, 3),
                "peak": round(peak_t, 2), "unit": "Tops/s",
                "frac": round(achieved / peak_t, 4), "traffic": traffic,
                "ops": f"{SPLAT_OPS_PER_POINT_VIEW_ALG} per point-view + "
                       f"{SPLAT_OPS_PER_WRITTEN_PX_ALG + (SPLAT_PBR_OPS_PER_WRITTEN_PX if pbr else 0)} per written pixel",
                "point_views": int(pv_per_frame), "written_px": int(wpx),
                "frac_census": round(census / peak_t, 4), "launch_ms": round(dom_ms, 4)}
    if dom == "setup":
        ops = SETUP_OPS_PER_TRI_VIEW * shape["nt"] * shape["views"]
        achieved = ops / (dom_ms * 1e-3) / 1e12
        return {"kernel": "k_tri_setup", "bound": "alu", "achieved": round(achieved, 3),
                "peak": round(VALU_PEAK_GOPS / 1e3, 2), "unit": "Tops/s",
                "frac": round(achieved / (VALU_PEAK_GOPS / 1e3), 4), "traffic": None, "launch_ms": round(dom_ms, 4)}
    b = BYTES[dom](shape)
    achieved = b / (dom_ms * 1e-3) / 1e9
    return {"kernel": "k_" + dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "launch_ms": round(dom_ms, 4)}


def frame_roofline(stage_ms: dict, pv_per_frame: float, shape: dict, frame_ms: float, pbr: bool = False) -> dict:
    """The frame's achievable time: for every stage the larger of its
    algorithmic bytes at the HBM peak and its algorithmic lane-ops at the ALU
    peak, summed over the stages; frac = that sum / the measured frame time."""
    peak_ops = VALU_PEAK_GOPS * 1e9
    peak_bytes = HBM_PEAK_GBS * 1e9
    ops = {"setup": SETUP_OPS_PER_TRI_VIEW * shape["nt"] * shape["views"],
           "splat": splat_ops(pv_per_frame, shape["written_px"], pbr)}
    bounds = {}
    for k in stage_ms:
        t_mem = BYTES[k](shape) / peak_bytes if k in BYTES else 0.0
        t_alu = ops.get(k, 0.0) / peak_ops
        bounds[k] = round(max(t_mem, t_alu) * 1e3, 4)
    total = sum(bounds.values())
    return {"achievable_ms": round(total, 4), "measured_ms": round(frame_ms, 4), "frac": round(total / frame_ms, 4),
            "bound_ms": bounds}


def profile_traffic(name: str, sources, label: str):
    """HBM bytes (`label: <value>` in profiles/<name>) from a committed
    rocprofv3 counter summary, if it was taken on the current kernel sources
    (the summary's sha256 over `sources` in csrc/ matches; else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_2601_19901_amd", "csrc", f), "rb").read())
    m = re.search(r"kernel sources sha256: ([0-9a-f]{64})", txt)
    t = re.search(re.escape(label) + r": ([0-9.e+]+)", txt)
    if not m or not t or m.group(1) != h.hexdigest():
        return None
    return float(t.group(1))


SPLAT_TRAFFIC_PROFILES = {"display-1M": "display-1M_splat_traffic.md", "display-4M-ss4": "display-4M-ss4_splat_traffic.md"}


def splat_traffic(kind: str, kernel: str):
    """HBM bytes per launch of the splat kernel that ran (k_splat or
    k_splat_quilt) on a workload with a committed counter summary (see
    profile_traffic)."""
    if kind not in SPLAT_TRAFFIC_PROFILES:
        return None
    return profile_traffic(SPLAT_TRAFFIC_PROFILES[kind], ("lfdpr_kernels.hip", "lfdpr_device.h", "lfdpr_internal.h"),
                           f"HBM bytes per launch of {kernel}")


ORDER_NAMES = {0: "point", 1: "triangle-view", 2: "quilt"}


def choose_splat_order(args, lfdpr, R, sid, model, views) -> dict:
    """The splat order of the run: the library's autotuner (point order under
    each launch shape and key layout, the quilt under each band height) or the
    one asked for.  Returns what was chosen."""
    if args.splat_order == "auto":
        tune = R.autotune(sid, model, views)
        b = tune["best"]
        log(f"autotune: {b}")
        return {"order": ORDER_NAMES[b["splat_order"]], "quilt_tile": [b["quilt_rows"], b["quilt_views"]],
                "splat_blocks": b["splat_blocks"], "key_layout": b["key_layout"], "autotuned": True,
                "candidates_ms": {f"{ORDER_NAMES[e['splat_order']]} {e['splat_blocks']}/{e['key_layout']}/"
                                  f"{e['quilt_rows']}x{e['quilt_views']}": round(e["ms"], 4) for e in tune["entries"]}}
    R.set_splat_order({"point": lfdpr.SPLAT_POINT, "triangle-view": lfdpr.SPLAT_TRIANGLE_VIEW,
                       "quilt": lfdpr.SPLAT_QUILT}[args.splat_order])
    return {"order": args.splat_order, "autotuned": False}


def host_cpu() -> dict:
    """The host the CPU baseline ran on: logical CPUs visible to this process,
    all logical CPUs, and the CPU model."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"nproc": usable, "logical_cpus": os.cpu_count(), "cpu_model": model, "oracle_threads": 1}


def stage_avg(R):
    return {k: (v[0] / v[1]) for k, v in R.timings().items() if v[1]}


def run_display(args, torch, lfdpr, scenes, kind: str):
    """kind: display-1M, display-4M-ss4 (angular filter to 48 views, then the
    panel), display-4M-ss4-direct (panel straight from the 192 sub-views),
    display-1M-spatial2x (1024^2 views, spatial reconstruction) or
    display-1M-pbr (physically based shading with four material sets)."""
    four_m = kind.startswith("display-4M")
    t0 = time.time()
    w = scenes.display_4m(seed=3) if four_m else scenes.display(seed=args.seed)
    if kind == "display-1M-spatial2x":
        w = scenes.spatial_ss(w)
    if kind == "display-1M-pbr":
        w = scenes.with_pbr(w)
    lens = scenes.direct_panel_lens(w) if kind == "display-4M-ss4-direct" else w.lens
    log(f"workload generated in {time.time() - t0:.1f}s: {w.scene.n_tris} tris")
    R = lfdpr.Renderer(0)
    sid = R.upload_scene(w.scene)
    R.set_views(w.views, point_capacity=(48 << 20) if kind != "display-1M" else 0)
    R.set_lens(lens)
    R.set_shading(w.shading)
    R.set_frames_in_flight(args.frames_in_flight)
    views, _ = R.alloc_views()
    models = [w.model(f) for f in range(args.warmup + args.steps)]
    chosen = choose_splat_order(args, lfdpr, R, sid, models[0], views)
    filtered = (torch.empty((w.views.V, w.views.H, w.views.W), dtype=torch.int32, device="cuda:0")
                if kind == "display-4M-ss4" else None)
    panel = torch.empty((lens.Hp, lens.Wp, 3), dtype=torch.uint8, device="cuda:0")

    def frame(f):
        R.render_frame(sid, models[f], views)
        if filtered is not None:
            R.angular_filter(views, filtered)
            R.reconstruct(filtered, panel)
        else:
            R.reconstruct(views, panel)

    for f in range(args.warmup):
        frame(f)
    torch.cuda.synchronize()
    R.timing(True)
    # one event per frame on the library's stream after the frame's panel:
    # frame-to-frame intervals give the p50 / p99 frame times
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ends[0].record(R.stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        frame(args.warmup + k)
        ends[k + 1].record(R.stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st_avg = stage_avg(R)
    R.timing(False)
    wall_ms = (t1 - t0) * 1e3 / args.steps
    intervals = np.array([ends[k].elapsed_time(ends[k + 1]) for k in range(args.steps)])
    serial_ms = None
    if args.frames_in_flight > 1:
        # the same frames with one frame in flight, for comparison
        R.set_frames_in_flight(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            frame(args.warmup + k)
        torch.cuda.synchronize()
        serial_ms = (time.perf_counter() - t0) * 1e3 / args.steps

    # the same frames again, untimed, for their statistics (deterministic)
    pv = pts = act = wpx = 0
    for k in range(args.steps):
        R.render_frame(sid, models[args.warmup + k], views)
        s = R.stats()
        pv += s["point_views"]
        pts += s["points"]
        act += s["active_tris"]
        wpx += s["written_px"]
    nfr = args.steps
    quilt = s["splat_order"] == lfdpr.SPLAT_QUILT
    chosen["order"] = ORDER_NAMES[s["splat_order"]]
    if quilt:
        chosen["quilt_tile"] = [s["quilt_rows"], s["quilt_views"]]
        chosen["quilt_entries_per_frame"] = s["quilt_entries"]
    n_rendered = w.views.V * w.views.S
    pbr = kind == "display-1M-pbr"
    shape = dict(nt=w.scene.n_tris, views=n_rendered, points=pts / nfr, pixels=n_rendered * w.views.W * w.views.H,
                 out_pixels=w.views.V * w.views.W * w.views.H,
                 panel_px=w.lens.Wp * w.lens.Hp, tris_with_points=act / nfr, written_px=wpx / nfr, quilt=quilt)
    roof = roofline(st_avg, pv / nfr, shape, splat_traffic(kind, "k_splat_quilt" if quilt else "k_splat"), pbr)
    names = {
        "display-1M": "display-1M: 999,168 tris (512^2-quad heightfield + 200 icospheres), 16 RGBA8 2048^2 textures, "
                      "48 views 512x512 (aspect 1.6, 40 deg cone), 2560x1600 lenticular panel, rotating scene",
        "display-4M-ss4": "display-4M-ss4: 3,996,672 tris (1024^2-quad heightfield + 200 icospheres), 16 RGBA8 2048^2 "
                          "textures, 192 rendered views 512x512 (4x angular supersampling over 48, jittered), angular "
                          "filter to 48 views, 2560x1600 lenticular panel, rotating scene",
        "display-4M-ss4-direct": "display-4M-ss4-direct: the display-4M-ss4 frame with the panel reconstructed straight "
                                 "from the 192 sub-views (angular taps over +-4 sub-view intervals), no filter pass",
        "display-1M-spatial2x": "display-1M-spatial2x: the display-1M scene rendered into 48 views of 1024x1024 (2x "
                                "spatial supersampling), panel through the spatial Gaussian taps",
        "display-1M-pbr": "display-1M-pbr: the display-1M scene with physically based shading (albedo + normal, "
                          "roughness and metallic maps in four material sets, normal maps up to 4096^2; one "
                          "directional light plus ambient), 48 views 512x512, 2560x1600 lenticular panel",
    }
    name = names[kind]
    recon = {"display-1M": "none", "display-4M-ss4": "angular filter", "display-4M-ss4-direct": "angular taps at the panel",
             "display-1M-spatial2x": "spatial taps at the panel", "display-1M-pbr": "none"}[kind]
    out = {
        "metric": METRIC,
        "value": round((pv / nfr) / (wall_ms * 1e-3), 1),
        "unit": "point-view splats/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "views": w.views.V, "rendered_views": n_rendered,
                   "view_px": [w.views.W, w.views.H], "panel_px": [w.lens.Wp, w.lens.Hp],
                   "triangles": w.scene.n_tris, "recon": recon},
        "frame_ms": round(wall_ms, 4),
        "frame_ms_p50": round(float(np.percentile(intervals, 50)), 4),
        "frame_ms_p99": round(float(np.percentile(intervals, 99)), 4),
        "frames_per_s": round(1e3 / wall_ms, 2),
        "frames_in_flight": args.frames_in_flight,
        "splat_order": chosen,
        "frame_ms_one_in_flight": round(serial_ms if serial_ms is not None else wall_ms, 4),
        "points_per_frame": int(pts / nfr), "point_views_per_frame": int(pv / nfr),
        "written_px_per_frame": int(wpx / nfr), "active_tris_per_frame": int(act / nfr),
        "stage_ms": {k: round(v, 4) for k, v in st_avg.items()},
        "roofline": roof,
        "frame_roofline": frame_roofline(st_avg, pv / nfr, shape, wall_ms, pbr),
    }
    if not args.no_learned and kind == "display-1M":
        log("learned reconstruction: checkpoint, PSNR against 16x angular supersampling, frame times")
        out["learned"] = learned_summary(args, torch, lfdpr, scenes, w)
    if not args.no_cpu_baseline and kind == "display-1M":
        from oracle import oracle as O
        nf = 3
        pv_cpu = 0
        t0 = time.perf_counter()
        for k in range(nf):
            o = O.render(w.scene, w.views, models[(args.warmup + k) % len(models)])
            O.interleave(o["rgba"], w.lens)
            pv_cpu += o["stats"]["point_views"]
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(pv_cpu / dt, 1), "unit": "point-view splats/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"{nf} consecutive full display-1M frames (point generation, splat into 48 "
                                         f"views, interleave) on one host core: {dt:.2f} s",
                               "host": host_cpu()}
    return out


LEARNED_CHECKPOINT = os.path.join(ROOT, "paper_2601_19901_amd", "weights", "learned_display-1M.lfnet")


def learned_summary(args, torch, lfdpr, scenes, w) -> dict:
    """The learned angular reconstruction on the benchmark's own scene (never
    trained on: training used scenes of seeds 5000-5003), with the committed
    checkpoint: frame time to the panel of plain 1x, learned and 4x angular
    supersampling in the same run, and PSNR of each against 16x angular
    supersampling + filter on frames spread over the rotation."""
    from paper_2601_19901_amd import learned
    if not os.path.exists(LEARNED_CHECKPOINT):
        return {"error": f"checkpoint {os.path.relpath(LEARNED_CHECKPOINT, ROOT)} missing"}
    t0 = time.time()
    ss = learned.AngularSS([w], factors=(1, 4, 16))
    model = learned.LearnedReconstruction(ss, w.views.H, w.views.W)
    model.net.load(LEARNED_CHECKPOINT)
    check = model.validate([(0, 250), (0, 750)])
    frames = [(0, f) for f in range(0, 1000, 125)]
    psnr = learned.evaluate(model, frames, ref_S=16)
    for S in (1, 4):
        ss.rigs[S].renderer.set_frames_in_flight(args.frames_in_flight)
    times = learned.time_pipelines(model, w.lens, 0, list(range(30)))
    out = {
        "checkpoint": os.path.relpath(LEARNED_CHECKPOINT, ROOT),
        "validated_against_4x": check,
        "frame_ms": {k: round(v, 4) for k, v in times.items()},
        "psnr_db_vs_16x": {k: round(v, 3) for k, v in psnr.items() if k.endswith("vs_ref")},
        "psnr_frames": f"{len(frames)} frames of the benchmark scene (seed {args.seed}), every 125th of the rotation",
        "learned_minus_ss4_db": round(psnr["learned_vs_ref"] - psnr["ss4_vs_ref"], 3),
        "learned_speedup_vs_ss4": round(times["ss4_ms"] / times["learned_ms"], 3),
        "target_met": bool(times["learned_ms"] < times["ss4_ms"]
                           and psnr["learned_vs_ref"] >= psnr["ss4_vs_ref"] - 0.5),
        "seconds": round(time.time() - t0, 1),
    }
    return out


def run_batch(args, torch, lfdpr, scenes):
    t0 = time.time()
    ws = scenes.batch_workloads(seed=400)
    ntri = [w.scene.n_tris for w in ws]
    log(f"batch generated in {time.time() - t0:.1f}s: {sum(ntri)} tris over {len(ws)} scenes")
    R = lfdpr.Renderer(0)
    ids = [R.upload_scene(w.scene) for w in ws]
    R.set_lens(ws[0].lens)
    B = lfdpr.Batch(R, ids, [w.views for w in ws], point_capacity=96 << 20)
    views = B.alloc_views()
    V, W, H = ws[0].views.V, ws[0].views.W, ws[0].views.H
    panels = torch.empty((len(ws), ws[0].lens.Hp, ws[0].lens.Wp, 3), dtype=torch.uint8, device="cuda:0")
    nf = args.warmup + args.steps
    models = [[w.model(f + 37 * k) for k, w in enumerate(ws)] for f in range(nf)]
    B.use_graph(False)
    tune = B.autotune(models[0], views)
    log(f"autotune: {tune['best']}")
    # stage times of eager batch renders (same kernels as the graph)
    for f in range(min(3, nf)):
        B.render(models[f], views, panels)
    torch.cuda.synchronize()
    R.timing(True)
    for k in range(args.steps):
        B.render(models[args.warmup + k], views, panels)
    torch.cuda.synchronize()
    st_avg = stage_avg(R)
    R.timing(False)
    # timed: hipGraph replays
    B.use_graph(True)
    for f in range(args.warmup):
        B.render(models[f], views, panels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        B.render(models[args.warmup + k], views, panels)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall_ms = graph_ms = (t1 - t0) * 1e3 / args.steps
    if args.frames_in_flight == 2:
        # timed: two batch calls in flight (a call's point generation overlaps
        # the previous call's splat; kernels launched directly)
        B.set_frames_in_flight(2)
        for f in range(args.warmup):
            B.render(models[f], views, panels)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            B.render(models[args.warmup + k], views, panels)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    pv = pts = act = wpx = 0
    for k in range(args.steps):
        B.render(models[args.warmup + k], views, panels)
        s = B.stats()
        pv += s["point_views"]
        pts += s["points"]
        act += s["active_tris"]
        wpx += s["written_px"]
    nfr = args.steps
    shape = dict(nt=sum(ntri), views=V, points=pts / nfr, pixels=len(ws) * V * W * H,
                 panel_px=len(ws) * ws[0].lens.Wp * ws[0].lens.Hp, tris_with_points=act / nfr, written_px=wpx / nfr)
    roof = roofline(st_avg, pv / nfr, shape)
    roof["timing"] = "stage events on eager batch renders of the same frames (graph replays carry no events)"
    return {
        "metric": METRIC,
        "value": round((pv / nfr) / (wall_ms * 1e-3), 1),
        "unit": "point-view splats/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch16: 16 independent display-family scenes per batch call, triangle counts "
                               "log-uniform 50k-4M, textures 512^2-2048^2, cones 30-50 deg, 48 views 512x512 each, "
                               "16 2560x1600 panels", "scenes": len(ws), "triangles": ntri,
                   "autotuned": tune["best"],
                   "autotune_candidates_ms": {f"{ORDER_NAMES[e['splat_order']]} {e['splat_blocks']}/{e['key_layout']}/"
                                              f"{e['quilt_rows']}x{e['quilt_views']}": round(e["ms"], 4)
                                              for e in tune["entries"]}},
        "frames_in_flight": args.frames_in_flight,
        "ms_per_step_graph_one_in_flight": round(graph_ms, 4),
        "scene_frames_per_s": round(len(ws) * 1e3 / wall_ms, 2),
        "points_per_step": int(pts / nfr), "point_views_per_step": int(pv / nfr),
        "stage_ms_eager": {k: round(v, 4) for k, v in st_avg.items()},
        "roofline": roof,
    }


METRIC = "48-view panel frame ms & point-view splats/s; learned vs 4× angular SS at PSNR"
BF16_MFMA_PEAK_TFLOPS = 2500.0


def run_learned(args, torch, lfdpr, scenes):
    """The learned reconstruction's frame on display-1M: plain 1x render +
    network (disparity blur, 4 BF16-MFMA convolutions) + panel, beside the plain
    and 4x-angular-SS frames.  Parameters are He-initialised: the cost does not
    depend on their values (the trained network's PSNR is measured by
    paper_2601_19901_amd.learned)."""
    from paper_2601_19901_amd import learned
    t0 = time.time()
    w = scenes.display(seed=args.seed)
    log(f"workload generated in {time.time() - t0:.1f}s: {w.scene.n_tris} tris")
    ss = learned.AngularSS([w], factors=(1, 4))
    model = learned.LearnedReconstruction(ss, w.views.H, w.views.W)
    rng = np.random.default_rng(0)
    flat = model.net.get_params()
    model.net.set_params((rng.normal(0.0, 0.05, flat.size)).astype(np.float32))
    for f in (1, 4):
        ss.rigs[f].renderer.set_frames_in_flight(args.frames_in_flight)
    frames = list(range(args.warmup + args.steps))
    times = learned.time_pipelines(model, w.lens, 0, frames)
    # network forward alone, HIP events on the library's (torch's current) stream
    R1 = ss.rigs[1].renderer
    views, depth = ss.render_plain(0, 0)
    model.net.pack_input(views, depth, model.x, ss.D)
    for _ in range(args.warmup):
        model.net.forward(model.x, model.y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        model.net.forward(model.x, model.y)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / args.steps
    # one training step (forward, backward, Adam) on 48 x 128 x 128 crops, the
    # training configuration; the cost does not depend on the values
    xc = model.x[:, :128, :128].contiguous()
    tc = xc.clone()
    yc = torch.empty_like(xc)
    for _ in range(3):
        model.net.forward(xc, yc)
        model.net.backward(tc)
        model.net.adam_step(1e-6)
    e0.record()
    for _ in range(args.steps):
        model.net.forward(xc, yc)
        model.net.backward(tc)
        model.net.adam_step(1e-6)
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1) / args.steps
    px = w.views.V * w.views.W * w.views.H
    flops = 2 * 9 * sum(ci * co for ci, co in lfdpr.NET_SHAPES) * px
    achieved = flops / (fwd_ms * 1e-3) / 1e12
    # algorithmic HBM bytes per pixel of the forward pass (BF16 activations):
    # blur reads the 4-channel input and writes 4 channels (16); layer 1 reads
    # the input and the blur and writes 32 channels (80); layers 2-3 read and
    # write 32 channels (128 each); the output layer reads 32 channels and the
    # blurred RGB and writes 4 channels (80).  121 flop/B, below the 312 flop/B
    # ridge of MI355X: the forward pass is HBM bound.
    net_bytes = NET_FWD_BYTES_PER_PX * px
    # the method's own input and output: (R, G, B, d) per view pixel in, (R, G, B, 0) out, BF16
    io_bytes = (8 + 8) * px
    gbs = net_bytes / (fwd_ms * 1e-3) / 1e9
    R1.render_frame(ss.rigs[1].scene_ids[0], w.model(args.warmup), ss.views1)
    pv = R1.stats()["point_views"]
    return {
        "metric": METRIC,
        "value": round(pv / (times["learned_ms"] * 1e-3), 1),
        "unit": "point-view splats/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(times["learned_ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f32", "data": "synthetic",
        "config": {"workload": "learned-display: display-1M rendered once (48 views 512x512) + learned angular "
                               "reconstruction (disparity blur + 4 BF16-MFMA 3x3 convolutions 24-32-32-32-3) + "
                               "2560x1600 panel; compared with plain 1x and 4x angular supersampling (192 views + "
                               "angular filter)", "views": w.views.V, "view_px": [w.views.W, w.views.H],
                   "triangles": w.scene.n_tris},
        "frame_ms": {k: round(v, 4) for k, v in times.items()},
        "frames_in_flight": args.frames_in_flight,
        "net_forward_ms": round(fwd_ms, 4),
        "net_train_step_ms": round(train_ms, 4),
        "net_train_step": "forward + backward + Adam on 48 x 128 x 128 crops",
        "roofline": {"kernel": "k_conv3x3 (4 layers) + k_disparity_blur_rows", "bound": "mfma",
                     "achieved": round(achieved, 1), "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / BF16_MFMA_PEAK_TFLOPS, 4),
                     "traffic": profile_traffic("learned-display_forward_traffic.md", ("lfdpr_net.hip",),
                                                "HBM bytes per forward"),
                     "flops_per_frame": flops,
                     "io_bytes_per_frame": io_bytes, "io_hbm_frac": round(io_bytes / (fwd_ms * 1e-3) / 1e9
                                                                          / HBM_PEAK_GBS, 4),
                     "unfused_activation_bytes_per_frame": net_bytes,
                     "unfused_activation_gbs": round(gbs, 1), "launch_ms": round(fwd_ms, 4)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=("display-1M", "display-4M-ss4", "display-4M-ss4-direct",
                                           "display-1M-spatial2x", "display-1M-pbr", "batch16", "learned-display"),
                    default="display-1M")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-reconstruction comparison of the default workload")
    ap.add_argument("--frames-in-flight", type=int, choices=(1, 2), default=2,
                    help="frames whose point generation overlaps the previous frame (display, learned and batch workloads)")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--splat-order", choices=("auto", "point", "triangle-view", "quilt"), default="auto",
                    help="how the splat visits its work (the same results); auto: the library's autotuner "
                         "picks the point order's launch shape or the quilt's tile (display workloads)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 (multi-GPU sharding "
                                   "is not implemented)"}))
        sys.exit(2)

    import torch
    from paper_2601_19901_amd import lfdpr, scenes

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 5}))
        return
    if args.workload == "batch16":
        out = run_batch(args, torch, lfdpr, scenes)
    elif args.workload == "learned-display":
        out = run_learned(args, torch, lfdpr, scenes)
    else:
        out = run_display(args, torch, lfdpr, scenes, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
