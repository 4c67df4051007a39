"""Host logic of bench.py (no GPU): the roofline arithmetic, the frame
roofline, the counter-profile lookup with its source hash, and the refusal
of more than one GPU."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def shape(**kw):
    s = dict(nt=1000, views=48, points=5000, pixels=48 * 64 * 64, panel_px=320 * 200, tris_with_points=600,
             written_px=0, out_pixels=0)
    s.update(kw)
    return s


def test_alu_peak_is_the_chip_lane_rate(bench):
    # 256 CUs x 64 lanes x 2.4 GHz
    assert bench.VALU_PEAK_GOPS == pytest.approx(39321.6)
    assert bench.HBM_PEAK_GBS == 8000.0


def test_splat_dominant_roofline(bench):
    st = {"setup": 0.2, "emit": 0.1, "splat": 2.0, "resolve": 0.05}
    pv, wpx = 1.0e8, 3.0e7
    r = bench.roofline(st, pv, shape(written_px=wpx), traffic=123.0)
    assert r["kernel"] == "k_splat" and r["bound"] == "alu" and r["traffic"] == 123.0
    want = (25 * pv + 40 * wpx) / 2.0e-3 / 1e12        # ~25 ops per point-view + ~40 per written pixel
    assert r["achieved"] == pytest.approx(want, abs=1e-3)
    assert r["frac"] == pytest.approx(want / 39.3216, abs=1e-4)
    census = (100 * pv + 37 * wpx) / 2.0e-3 / 1e12 / 39.3216
    assert r["frac_census"] == pytest.approx(census, abs=1e-4)


def test_splat_fraction_of_the_round_one_display_frame(bench):
    """The algorithmic count on the display-1M frame of the earlier kernels:
    146.85M point-views and 48.0M written pixels in a 1667.5 us splat is 5.59 G
    ops, 0.085 of the 39.32 T lane-op/s peak."""
    r = bench.roofline({"splat": 1.6675}, 146.85e6, shape(written_px=48.0e6))
    assert bench.splat_ops(146.85e6, 48.0e6) == pytest.approx(5.59e9, rel=2e-3)
    assert r["frac"] == pytest.approx(0.085, abs=6e-4)


def test_memory_dominant_roofline(bench):
    s = shape()
    st = {"splat": 0.01, "resolve": 0.5}
    r = bench.roofline(st, 10.0, s)
    assert r["kernel"] == "k_resolve" and r["bound"] == "hbm"
    want = s["pixels"] * 20 / 0.5e-3 / 1e9       # key read + clear (8 + 8) and RGBA8 (4) per pixel
    assert r["achieved"] == pytest.approx(want, abs=0.05)   # reported to 0.1 GB/s
    assert r["frac"] == pytest.approx(want / 8000.0, abs=1e-4)


def test_frame_roofline_sums_the_larger_bound_per_stage(bench):
    s = shape(written_px=6.0e6)
    st = {"setup": 0.3, "splat": 1.5, "resolve": 0.05, "interleave": 0.04}
    pv = 2.0e7
    r = bench.frame_roofline(st, pv, s, frame_ms=2.0)
    peak_ops, peak_b = bench.VALU_PEAK_GOPS * 1e9, bench.HBM_PEAK_GBS * 1e9
    want = {
        "setup": max(bench.BYTES["setup"](s) / peak_b, 40 * s["nt"] * s["views"] / peak_ops),
        "splat": max(bench.BYTES["splat"](s) / peak_b, (25 * pv + 40 * 6.0e6) / peak_ops),
        "resolve": bench.BYTES["resolve"](s) / peak_b,
        "interleave": bench.BYTES["interleave"](s) / peak_b,
    }
    for k, v in want.items():
        assert r["bound_ms"][k] == pytest.approx(v * 1e3, abs=1e-4)
    assert r["achievable_ms"] == pytest.approx(sum(want.values()) * 1e3, abs=4e-4)
    assert r["frac"] == pytest.approx(r["achievable_ms"] / 2.0, abs=1e-4)


def test_quilt_frame_roofline(bench):
    """Under the quilt the splat writes the views from its LDS tiles (points,
    records and splat rectangles in, 4 B per view pixel out), the resolve
    stage has nothing to move, and the band lists read each point's row range
    twice and write an entry."""
    s = shape(written_px=6.0e6, quilt=True)
    st = {"setup": 0.3, "splat": 1.4, "resolve": 0.006, "quilt_bin": 0.07}
    r = bench.roofline(st, 2.0e7, s)
    assert r["kernel"] == "k_splat_quilt" and r["bound"] == "alu"
    assert bench.BYTES["splat"](s) == s["points"] * (16 + 112 + 48) + s["pixels"] * 4
    assert bench.BYTES["resolve"](s) == 0
    assert bench.BYTES["quilt_bin"](s) == s["points"] * 12
    f = bench.frame_roofline(st, 2.0e7, s, frame_ms=2.0)
    assert f["bound_ms"]["resolve"] == 0.0
    assert f["bound_ms"]["quilt_bin"] == pytest.approx(s["points"] * 12 / 8e12 * 1e3, abs=1e-4)


def test_profile_traffic_requires_matching_sources(bench, tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2601_19901_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (csrc / "a.hip").write_bytes(b"kernel source v1\n")
    sha = hashlib.sha256(b"kernel source v1\n").hexdigest()
    (tmp_path / "profiles" / "p.md").write_text(f"HBM bytes per launch: 1.5e+09\n\nkernel sources sha256: {sha}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profile_traffic("p.md", ("a.hip",), "HBM bytes per launch") == 1.5e9
    assert bench.profile_traffic("p.md", ("a.hip",), "HBM bytes per forward") is None   # label absent
    assert bench.profile_traffic("missing.md", ("a.hip",), "HBM bytes per launch") is None
    # one summary can hold the bytes of several kernels, each on its own line
    (tmp_path / "profiles" / "k.md").write_text(f"HBM bytes per launch of k_splat: 1.0e+09\n"
                                                f"HBM bytes per launch of k_splat_quilt: 2.5e+08\n\n"
                                                f"kernel sources sha256: {sha}\n")
    assert bench.profile_traffic("k.md", ("a.hip",), "HBM bytes per launch of k_splat_quilt") == 2.5e8
    assert bench.profile_traffic("k.md", ("a.hip",), "HBM bytes per launch of k_splat") == 1.0e9
    (csrc / "a.hip").write_bytes(b"kernel source v2\n")                                  # sources changed
    assert bench.profile_traffic("p.md", ("a.hip",), "HBM bytes per launch") is None


def test_host_cpu_description(bench):
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and h["logical_cpus"] >= h["nproc"] and h["oracle_threads"] == 1
    assert isinstance(h["cpu_model"], str)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
