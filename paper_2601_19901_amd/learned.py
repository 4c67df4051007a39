"""Learned angular reconstruction: training, evaluation and the 4x fallback.

The network (lfdpr_net_* in include/lfdpr.h) maps the V views rendered once
(plus their depth) to what 4x angular supersampling followed by the angular
filter gives (Sec. 4: angular supersampling projects splats into more views at
random angles inside view intervals).  Training pairs are rendered on the fly
by the method itself; the plain 4x supersampled reconstruction stays available
as the fallback and as the reference the network is measured against.

Everything here is orchestration: rendering, packing, convolutions, loss,
gradients and Adam run in the library's HIP kernels; torch only holds device
buffers, slices crops and computes the PSNR metrics.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import lfdpr, scenes


def psnr_views(a, b) -> float:
    """PSNR (dB) of the RGB channels of two RGBA8 view stacks (int32 tensors)."""
    import torch
    x = a.view(torch.uint8).reshape(*a.shape, 4)[..., :3].float()
    y = b.view(torch.uint8).reshape(*b.shape, 4)[..., :3].float()
    mse = float(((x - y) ** 2).mean())
    return math.inf if mse == 0 else 10.0 * math.log10(255.0 ** 2 / mse)


@dataclasses.dataclass
class Rig:
    """One renderer context per angular supersampling factor, all scenes uploaded."""
    renderer: lfdpr.Renderer
    scene_ids: List[int]
    views: scenes.ViewParams


class AngularSS:
    """Plain, 4x-supersampled and reference renders of a set of workloads."""

    def __init__(self, workloads: Sequence[scenes.Workload], factors=(1, 4), jitter_seed: int = 100):
        import torch
        self.torch = torch
        self.workloads = list(workloads)
        base = self.workloads[0].views
        self.V, self.W, self.H, self.D = base.V, base.W, base.H, base.D
        self.rigs: Dict[int, Rig] = {}
        for S in factors:
            vp = dataclasses.replace(base, S=S, jitter=scenes.subview_jitter(jitter_seed + S, base.V * S) if S > 1 else None)
            R = lfdpr.Renderer(0)
            ids = [R.upload_scene(w.scene) for w in self.workloads]
            R.set_views(vp)
            self.rigs[S] = Rig(R, ids, vp)
        dev = "cuda:0"
        self.views1 = torch.empty((self.V, self.H, self.W), dtype=torch.int32, device=dev)
        self.depth1 = torch.empty((self.V, self.H, self.W), dtype=torch.float32, device=dev)
        self.sub = {S: torch.empty((self.V * S, self.H, self.W), dtype=torch.int32, device=dev)
                    for S in factors if S > 1}
        self.filtered = {S: torch.empty((self.V, self.H, self.W), dtype=torch.int32, device=dev)
                         for S in factors if S > 1}

    def render_plain(self, k: int, frame: int):
        rig = self.rigs[1]
        rig.renderer.render_frame(rig.scene_ids[k], self.workloads[k].model(frame), self.views1, self.depth1)
        return self.views1, self.depth1

    def render_ss(self, k: int, frame: int, S: int):
        rig = self.rigs[S]
        rig.renderer.render_frame(rig.scene_ids[k], self.workloads[k].model(frame), self.sub[S])
        rig.renderer.angular_filter(self.sub[S], self.filtered[S])
        return self.filtered[S]


class LearnedReconstruction:
    """The network plus its health state; falls back to 4x supersampling."""

    def __init__(self, ss: AngularSS, max_h: int, max_w: int, seed: int = 0, fallback_S: int = 4):
        import torch
        self.torch = torch
        self.ss = ss
        self.net = lfdpr.Net(ss.rigs[1].renderer, ss.V, max_h, max_w)
        self.net.set_rig(ss.rigs[1].views)
        self.fallback_S = fallback_S
        self.healthy = True
        rng = np.random.default_rng(seed)
        params = []
        for k, (ci, co) in enumerate(lfdpr.NET_SHAPES):
            std = math.sqrt(2.0 / (9 * ci)) * (0.0 if k == 3 else 1.0)
            params.append((rng.normal(0.0, std, (9, co, ci)), np.zeros(co)))
        self.net.set_params(lfdpr.params_to_flat(params))
        dev = "cuda:0"
        V, H, W = ss.V, ss.H, ss.W
        self.x = torch.empty((V, H, W, 4), dtype=torch.int16, device=dev)
        self.t = torch.empty((V, H, W, 4), dtype=torch.int16, device=dev)
        self.y = torch.empty((V, H, W, 4), dtype=torch.int16, device=dev)
        self.out = torch.empty((V, H, W), dtype=torch.int32, device=dev)

    def set_params(self, flat: np.ndarray) -> bool:
        """Installs parameters; non-finite ones switch to the fallback."""
        if not np.all(np.isfinite(flat)):
            self.healthy = False
            return False
        self.net.set_params(flat)
        self.healthy = True
        return True

    def validate(self, frames: Sequence, min_gain_db: float = 1.0) -> dict:
        """The 4x angular supersampling judges the network (Sec. 4's result is
        what it stands in for): on the given (scene, frame) pairs the learned
        views must be closer to the 4x result than the plain 1x render is, by
        at least min_gain_db of PSNR, or the network is switched off and
        reconstruct() returns the 4x result."""
        if not self.healthy:
            return {"healthy": False, "reason": "parameters refused"}
        gains = []
        for (k, f) in frames:
            s4 = self.ss.render_ss(k, f, self.fallback_S).clone()
            plain, _ = self.ss.render_plain(k, f)
            p_plain = psnr_views(plain, s4)
            p_learned = psnr_views(self.reconstruct(k, f), s4)
            gains.append(p_learned - p_plain)
        gain = float(np.mean(gains))
        self.healthy = bool(np.isfinite(gain) and gain >= min_gain_db)
        return {"healthy": self.healthy, "gain_db_vs_plain": gain, "min_gain_db": min_gain_db,
                "frames": len(frames)}

    def make_pair(self, k: int, frame: int):
        views, depth = self.ss.render_plain(k, frame)
        self.net.pack_input(views, depth, self.x, self.ss.D)
        tgt = self.ss.render_ss(k, frame, self.fallback_S)
        self.net.pack_input(tgt, None, self.t)
        return self.x, self.t

    def frame_loss(self, k: int, frame: int):
        """(network MSE, plain-render MSE) against the 4x target over a whole frame."""
        torch = self.torch
        x, t = self.make_pair(k, frame)
        self.net.forward(x, self.y)
        net_mse = float(self.net.backward(t).item())
        xs = (x[..., :3].to(torch.int32) << 16).view(torch.float32)
        ts = (t[..., :3].to(torch.int32) << 16).view(torch.float32)
        return net_mse, float(((xs - ts) ** 2).mean())

    def train(self, frames: Sequence, steps_per_frame: int = 4, crop: int = 128, lr: float = 1e-3,
              lr_end: float = 3e-4, seed: int = 1, log_every: int = 200) -> List[float]:
        torch = self.torch
        rng = np.random.default_rng(seed)
        losses = []
        total = len(frames) * steps_per_frame
        step = 0
        H, W = self.ss.H, self.ss.W
        ch, cw = min(crop, H), min(crop, W)
        for (k, f) in frames:
            x, t = self.make_pair(k, f)
            for _ in range(steps_per_frame):
                y0 = int(rng.integers(0, H - ch + 1))
                x0 = int(rng.integers(0, W - cw + 1))
                xc = x[:, y0:y0 + ch, x0:x0 + cw].contiguous()
                tc = t[:, y0:y0 + ch, x0:x0 + cw].contiguous()
                yc = torch.empty_like(xc)
                self.net.forward(xc, yc)
                loss = self.net.backward(tc)
                a = step / max(total - 1, 1)
                self.net.adam_step(lr * (lr_end / lr) ** a)
                step += 1
                if step % 50 == 0 or step == total:
                    losses.append(float(loss.item()))
                if log_every and step % log_every == 0:
                    print(f"  step {step}/{total} loss {losses[-1]:.3e}", flush=True)
        return losses

    def reconstruct(self, k: int, frame: int):
        """The V views after learned reconstruction (or the 4x fallback)."""
        if not self.healthy:
            return self.ss.render_ss(k, frame, self.fallback_S)
        views, depth = self.ss.render_plain(k, frame)
        self.net.pack_input(views, depth, self.x, self.ss.D)
        self.net.forward(self.x, self.y)
        self.net.unpack_output(self.y, self.out)
        return self.out


class LearnedPipeline:
    """Learned frames to the panel with the network of frame i overlapping the
    rendering of frame i+1.  Rendering stays on the renderer's stream; input
    packing, the network, unpacking and the interleave run on a second stream
    (default priority) through a context and a copy of the network of their
    own.  Two view / depth buffer pairs alternate between the streams, fenced
    by events: a buffer is rendered into again only after the network side has
    packed it.  The renderer keeps one frame in flight while the pipeline runs
    (its own next-frame point generation would be a third stream competing for
    the same gaps; measured slower) and gets its setting back on close().
    Every panel equals the serial path (reconstruct, then the interleave) bit
    for bit; with poisoned parameters frames take the 4x supersampling fallback
    serially."""

    def __init__(self, lr_: LearnedReconstruction, lens: scenes.LensParams):
        import torch
        self.torch = torch
        self.lr = lr_
        self.ss = lr_.ss
        V, H, W = self.ss.V, self.ss.H, self.ss.W
        dev = "cuda:0"
        self.stream = torch.cuda.Stream(device=0)
        self.R = lfdpr.Renderer(0, stream=self.stream)
        self.R.set_lens(lens)
        self.net = lfdpr.Net(self.R, V, H, W)
        self.net.set_rig(self.ss.rigs[1].views)
        self.views = [torch.empty((V, H, W), dtype=torch.int32, device=dev) for _ in range(2)]
        self.depth = [torch.empty((V, H, W), dtype=torch.float32, device=dev) for _ in range(2)]
        self.x = torch.empty((V, H, W, 4), dtype=torch.int16, device=dev)
        self.y = torch.empty_like(self.x)
        self.out = torch.empty((V, H, W), dtype=torch.int32, device=dev)
        self.rendered = [torch.cuda.Event(), torch.cuda.Event()]
        self.packed = [None, None]
        self.n = 0
        R1 = self.ss.rigs[1].renderer
        self.render_in_flight = R1.frames_in_flight
        R1.set_frames_in_flight(1)
        self.sync_params()

    def sync_params(self):
        """Copies the model's current parameters to the pipeline's network."""
        self.torch.cuda.synchronize()
        if self.lr.healthy:
            self.net.set_params(self.lr.net.get_params())

    def frame(self, k: int, frame: int, panel):
        rig = self.ss.rigs[1]
        rs = rig.renderer.stream
        if not self.lr.healthy:
            rs.wait_stream(self.stream)
            self.ss.rigs[1].renderer.reconstruct(self.lr.reconstruct(k, frame), panel)
            self.stream.wait_stream(rs)
            return
        s = self.n % 2
        self.n += 1
        if self.packed[s] is not None:
            rs.wait_event(self.packed[s])
        rig.renderer.render_frame(rig.scene_ids[k], self.ss.workloads[k].model(frame), self.views[s], self.depth[s])
        self.rendered[s].record(rs)
        self.stream.wait_event(self.rendered[s])
        self.net.pack_input(self.views[s], self.depth[s], self.x, self.ss.D)
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        self.packed[s] = ev
        self.net.forward(self.x, self.y)
        self.net.unpack_output(self.y, self.out)
        self.R.reconstruct(self.out, panel)

    def close(self):
        self.torch.cuda.synchronize()
        self.ss.rigs[1].renderer.set_frames_in_flight(self.render_in_flight)
        self.net.close()
        self.R.close()


def evaluate(lr_: LearnedReconstruction, frames: Sequence, ref_S: int, fallback_S: int = 4) -> dict:
    """PSNR of plain 1x, learned and 4x-supersampled views against a high-factor
    angular supersampling reference, and against the 4x result."""
    ss = lr_.ss
    acc = {"plain_vs_ref": [], "learned_vs_ref": [], "ss4_vs_ref": [], "plain_vs_ss4": [], "learned_vs_ss4": []}
    torch = lr_.torch
    for (k, f) in frames:
        ref = ss.render_ss(k, f, ref_S).clone()
        s4 = ss.render_ss(k, f, fallback_S).clone()
        plain, _ = ss.render_plain(k, f)
        plain = plain.clone()
        learned = lr_.reconstruct(k, f).clone()
        acc["plain_vs_ref"].append(psnr_views(plain, ref))
        acc["learned_vs_ref"].append(psnr_views(learned, ref))
        acc["ss4_vs_ref"].append(psnr_views(s4, ref))
        acc["plain_vs_ss4"].append(psnr_views(plain, s4))
        acc["learned_vs_ss4"].append(psnr_views(learned, s4))
    return {k: float(np.mean(v)) for k, v in acc.items()}


def time_pipelines(lr_: LearnedReconstruction, lens: scenes.LensParams, k: int, frames: Sequence[int],
                   fallback_S: int = 4) -> dict:
    """Frame time (ms) to the panel: 1x plain, learned (network of a frame
    overlapping the next frame's rendering; learned_serial_ms without that
    overlap), and 4x supersampled + filter."""
    torch = lr_.torch
    ss = lr_.ss
    R1 = ss.rigs[1].renderer
    R1.set_lens(lens)
    panel = torch.empty((lens.Hp, lens.Wp, 3), dtype=torch.uint8, device="cuda:0")
    out = {}

    def run(name, fn):
        for f in frames[:3]:
            fn(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in frames:
            fn(f)
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0) * 1e3 / len(frames)

    def plain(f):
        v, _ = ss.render_plain(k, f)
        R1.reconstruct(v, panel)

    def learned(f):
        R1.reconstruct(lr_.reconstruct(k, f), panel)

    def ss4(f):
        R1.reconstruct(ss.render_ss(k, f, fallback_S), panel)

    run("plain_1x_ms", plain)
    run("learned_serial_ms", learned)
    run("ss4_ms", ss4)
    pipe = LearnedPipeline(lr_, lens)

    def learned_overlapped(f):
        pipe.frame(k, f, panel)

    run("learned_ms", learned_overlapped)
    pipe.close()
    return {k2: out[k2] for k2 in ("plain_1x_ms", "learned_ms", "learned_serial_ms", "ss4_ms")}


def main(argv=None):
    ap = argparse.ArgumentParser(description="Train and evaluate the learned angular reconstruction")
    ap.add_argument("--train-scenes", type=int, default=4)
    ap.add_argument("--train-frames", type=int, default=2000)
    ap.add_argument("--test-scenes", type=int, default=2)
    ap.add_argument("--test-frames", type=int, default=200)
    ap.add_argument("--steps-per-frame", type=int, default=48)
    ap.add_argument("--crop", type=int, default=128)
    ap.add_argument("--ref-S", type=int, default=16)
    ap.add_argument("--small", action="store_true", help="small-display family (CPU-oracle size) for a quick run")
    ap.add_argument("--report", type=str, default="")
    ap.add_argument("--save", type=str, default="")
    args = ap.parse_args(argv)
    t_start = time.time()
    make = (lambda s: scenes.small_display(seed=s, V=16, W=96, H=96)) if args.small else (lambda s: scenes.display(seed=s))
    train_w = [make(5000 + i) for i in range(args.train_scenes)]
    test_w = [make(9000 + i) for i in range(args.test_scenes)]
    print(f"scenes generated in {time.time() - t_start:.1f}s", flush=True)
    ss = AngularSS(train_w + test_w, factors=(1, 4, args.ref_S))
    V, H, W = ss.V, ss.H, ss.W
    model = LearnedReconstruction(ss, H, W)
    rng = np.random.default_rng(5)
    ntr = len(train_w)
    train_frames = [(int(rng.integers(0, ntr)), int(rng.integers(0, 1000))) for _ in range(args.train_frames)]
    test_frames = [(ntr + int(rng.integers(0, len(test_w))), int(rng.integers(0, 1000))) for _ in range(args.test_frames)]
    before = evaluate(model, test_frames[:20], args.ref_S)
    t0 = time.time()
    losses = model.train(train_frames, steps_per_frame=args.steps_per_frame, crop=args.crop)
    train_s = time.time() - t0
    after = evaluate(model, test_frames, args.ref_S)
    timing = time_pipelines(model, test_w[0].lens, ntr, list(range(20)))
    # fallback: poisoned parameters are refused and the 4x path takes over
    good = model.net.get_params()
    bad = good.copy()
    bad[0] = np.nan
    accepted = model.set_params(bad)
    fb = model.reconstruct(ntr, 0).clone()
    fallback_ok = (not accepted) and psnr_views(fb, ss.render_ss(ntr, 0, 4)) == math.inf
    model.set_params(good)
    rep = {
        "workload": "small-display V16 96x96" if args.small else "display-1M family, V=48 views 512x512",
        "train": {"scenes": args.train_scenes, "frames": args.train_frames, "steps": len(train_frames) * args.steps_per_frame,
                  "crop": args.crop, "seconds": round(train_s, 1), "loss_first": losses[0] if losses else None,
                  "loss_last": losses[-1] if losses else None},
        "test": {"scenes": args.test_scenes, "frames": args.test_frames, "reference": f"{args.ref_S}x angular SS + filter"},
        "psnr_db_before_training_20_frames": before,
        "psnr_db": after,
        "learned_minus_ss4_vs_ref_db": after["learned_vs_ref"] - after["ss4_vs_ref"],
        "frame_ms": timing,
        "fallback_on_bad_params": fallback_ok,
        "n_params": int(model.net.n_params),
    }
    print(json.dumps(rep, indent=1), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    if args.save:
        model.net.save(args.save)


if __name__ == "__main__":
    main()
