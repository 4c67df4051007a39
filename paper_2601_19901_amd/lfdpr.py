"""Thin ctypes binding of liblfdpr.so (include/lfdpr.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels.  torch supplies device memory (``data_ptr()``) and the stream.
Raises if the library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblfdpr.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "lfdpr.h")

LFDPR_OK, LFDPR_EINVAL, LFDPR_ENOMEM, LFDPR_EOVERFLOW, LFDPR_EDEVICE, LFDPR_ESTATE = 0, -1, -2, -3, -4, -5
SPLAT_POINT, SPLAT_TRIANGLE_VIEW, SPLAT_QUILT = 0, 1, 2


class LfdprError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lfdpr error {code}: {msg}")
        self.code = code


class SceneDesc(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tris", C.c_int32), ("pos", C.c_void_p), ("uv", C.c_void_p),
                ("idx", C.c_void_p), ("tex_id", C.c_void_p), ("n_tex", C.c_int32), ("tex_size", C.c_void_p),
                ("tex_rgba8", C.c_void_p)]


class ViewParams(C.Structure):
    _fields_ = [("V", C.c_int32), ("S", C.c_int32), ("W", C.c_int32), ("H", C.c_int32),
                ("fovy_deg", C.c_float), ("aspect", C.c_float), ("D", C.c_float), ("cone_deg", C.c_float),
                ("znear", C.c_float), ("jitter", C.c_void_p), ("mip", C.c_int32), ("point_capacity", C.c_int64)]


class LensParams(C.Structure):
    _fields_ = [("Wp", C.c_int32), ("Hp", C.c_int32), ("pitch_subpx", C.c_double), ("slope", C.c_double),
                ("offset", C.c_double), ("mode", C.c_int32), ("taps", (C.c_int64 * 3) * 8)]


class ShadingParams(C.Structure):
    _fields_ = [("mode", C.c_int32), ("light_dir", C.c_float * 3), ("light_rgb", C.c_float * 3),
                ("ambient_rgb", C.c_float * 3)]


class TuneEntry(C.Structure):
    _fields_ = [("splat_blocks", C.c_int32), ("key_layout", C.c_int32), ("ms", C.c_float),
                ("splat_order", C.c_int32), ("quilt_rows", C.c_int32), ("quilt_views", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("n", C.c_int32), ("best", C.c_int32), ("entries", TuneEntry * 16)]


class Stats(C.Structure):
    _fields_ = [("points", C.c_int64), ("active_tris", C.c_int64), ("point_views", C.c_int64),
                ("overflow_tris", C.c_int64), ("capacity", C.c_int64), ("point_overflow", C.c_int32),
                ("n_views", C.c_int32), ("written_px", C.c_int64), ("splat_order", C.c_int32),
                ("reserved", C.c_int32), ("covered_px", C.c_int64), ("missed_px", C.c_int64),
                ("quilt_rows", C.c_int32), ("quilt_views", C.c_int32), ("quilt_entries", C.c_int64)]


_lib = None


def declared_symbols():
    """Function names declared in include/lfdpr.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lfdpr_[a-z0-9_]+)\s*\(", txt)))


def declared_arity():
    """Number of parameters of each function include/lfdpr.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    out = {}
    for name, args in re.findall(r"\b(lfdpr_[a-z0-9_]+)\s*\(([^)]*)\)\s*;", txt):
        args = args.strip()
        out[name] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    for name, (args, res) in signatures().items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def signatures():
    """ctypes (argtypes, restype) of every entry point in include/lfdpr.h."""
    vp, i32, i64, p = C.c_void_p, C.c_int32, C.c_int64, C.POINTER
    return {
        "lfdpr_abi_version": ([], C.c_int),
        "lfdpr_strerror": ([C.c_int], C.c_char_p),
        "lfdpr_create": ([C.c_int, vp, p(vp)], C.c_int),
        "lfdpr_destroy": ([vp], C.c_int),
        "lfdpr_last_error": ([vp], C.c_char_p),
        "lfdpr_scene_upload": ([vp, p(SceneDesc), p(i32)], C.c_int),
        "lfdpr_scene_free": ([vp, i32], C.c_int),
        "lfdpr_scene_set_materials": ([vp, i32, vp, vp, vp], C.c_int),
        "lfdpr_set_shading": ([vp, p(ShadingParams)], C.c_int),
        "lfdpr_copy_point_materials": ([vp, vp, i64, p(i64)], C.c_int),
        "lfdpr_set_views": ([vp, p(ViewParams)], C.c_int),
        "lfdpr_set_lens": ([vp, p(LensParams)], C.c_int),
        "lfdpr_set_splat_order": ([vp, i32], C.c_int),
        "lfdpr_set_quilt_tile": ([vp, i32, i32], C.c_int),
        "lfdpr_set_quilt_capacity": ([vp, i64], C.c_int),
        "lfdpr_quilt_tile": ([i32, i32, i32, i32, i32, i32, i32, p(i32), p(i32)], C.c_int),
        "lfdpr_render_frame": ([vp, i32, vp, vp, vp], C.c_int),
        "lfdpr_render_frame_noalloc": ([vp, i32, vp, vp, vp, vp], C.c_int),
        "lfdpr_reconstruct": ([vp, vp, i32, i32, i32, vp], C.c_int),
        "lfdpr_angular_filter": ([vp, vp, vp], C.c_int),
        "lfdpr_get_stats": ([vp, p(Stats)], C.c_int),
        "lfdpr_copy_points": ([vp, vp, i64, p(i64)], C.c_int),
        "lfdpr_copy_counts": ([vp, vp, i64], C.c_int),
        "lfdpr_set_debug_records": ([vp, vp, vp, i64], C.c_int),
        "lfdpr_timing": ([vp, C.c_int], C.c_int),
        "lfdpr_set_launch": ([vp, i32, i32], C.c_int),
        "lfdpr_set_frames_in_flight": ([vp, i32], C.c_int),
        "lfdpr_autotune": ([vp, i32, vp, vp, p(TuneResult)], C.c_int),
        "lfdpr_batch_create": ([vp, i32, vp, vp, i64, p(vp)], C.c_int),
        "lfdpr_batch_destroy": ([vp], C.c_int),
        "lfdpr_batch_last_error": ([vp], C.c_char_p),
        "lfdpr_batch_use_graph": ([vp, C.c_int], C.c_int),
        "lfdpr_batch_set_frames_in_flight": ([vp, C.c_int32], C.c_int),
        "lfdpr_batch_render": ([vp, vp, vp, vp], C.c_int),
        "lfdpr_batch_stats": ([vp, p(Stats)], C.c_int),
        "lfdpr_batch_autotune": ([vp, vp, vp, p(TuneResult)], C.c_int),
        "lfdpr_net_create": ([vp, i32, i32, i32, p(vp)], C.c_int),
        "lfdpr_net_destroy": ([vp], C.c_int),
        "lfdpr_net_last_error": ([vp], C.c_char_p),
        "lfdpr_net_param_count": ([vp, p(i64)], C.c_int),
        "lfdpr_net_set_params": ([vp, vp, i64], C.c_int),
        "lfdpr_net_set_disparity_scale": ([vp, C.c_float], C.c_int),
        "lfdpr_net_set_rig": ([vp, p(ViewParams)], C.c_int),
        "lfdpr_net_get_params": ([vp, vp, i64], C.c_int),
        "lfdpr_net_pack_input": ([vp, vp, vp, i32, i32, i32, C.c_float, vp], C.c_int),
        "lfdpr_net_forward": ([vp, vp, i32, i32, i32, vp], C.c_int),
        "lfdpr_net_backward": ([vp, vp, vp], C.c_int),
        "lfdpr_net_adam_step": ([vp, C.c_float, C.c_float, C.c_float, C.c_float], C.c_int),
        "lfdpr_net_unpack_output": ([vp, vp, i32, i32, i32, vp], C.c_int),
        "lfdpr_net_copy_state": ([vp, i32, vp, i64], C.c_int),
        "lfdpr_net_save": ([vp, C.c_char_p], C.c_int),
        "lfdpr_net_load": ([vp, C.c_char_p], C.c_int),
        "lfdpr_get_timings": ([vp, vp, vp], C.c_int),
    }


def _ptr(t) -> int:
    if t is None:
        return 0
    if isinstance(t, np.ndarray):
        assert t.flags["C_CONTIGUOUS"]
        return t.ctypes.data
    assert t.is_contiguous(), "tensor must be contiguous"
    return t.data_ptr()


def view_params(vp, point_capacity: int = 0):
    """ViewParams (scenes.ViewParams) -> the ABI struct; returns it with the arrays it points into."""
    jit = None
    if vp.S > 1:
        jit = np.ascontiguousarray(vp.jitter, np.float32)
    p = ViewParams(vp.V, vp.S, vp.W, vp.H, vp.fovy_deg, vp.aspect, vp.D, vp.cone_deg, vp.znear,
                   _ptr(jit) if jit is not None else None, int(vp.mip), int(point_capacity))
    return p, jit


def quilt_tile(W: int, H: int, n_views: int, n_items: int = 1, max_lds: int = 160 * 1024, rows: int = 0,
               views: int = 0):
    """The quilt tile (rows, views) the library uses for this rig, or None when
    none fits (host only)."""
    r, v = C.c_int32(), C.c_int32()
    rc = lib().lfdpr_quilt_tile(int(W), int(H), int(n_views), int(n_items), int(max_lds), int(rows), int(views),
                                C.byref(r), C.byref(v))
    return (r.value, v.value) if rc == LFDPR_OK else None


def tune_dict(res) -> dict:
    ents = [dict(splat_blocks=res.entries[k].splat_blocks, key_layout=res.entries[k].key_layout,
                 ms=float(res.entries[k].ms), splat_order=res.entries[k].splat_order,
                 quilt_rows=res.entries[k].quilt_rows, quilt_views=res.entries[k].quilt_views)
            for k in range(res.n)]
    return dict(best=ents[res.best], entries=ents)


def _check_dev(t, dtype, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() < numel:
        raise ValueError(f"{name}: need contiguous {dtype} with >= {numel} elements")


class Renderer:
    """One library context on one device and stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        self._check(lib().lfdpr_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h)), ctx=None)
        self.h = h
        self.vp = None
        self.lens = None
        self.frames_in_flight = 1
        self._keep = {}

    def _check(self, rc: int, ctx="self"):
        if rc != LFDPR_OK:
            msg = lib().lfdpr_strerror(rc).decode()
            if ctx == "self" and getattr(self, "h", None):
                last = lib().lfdpr_last_error(self.h)
                msg += ": " + (last.decode() if last else "")
            raise LfdprError(rc, msg)
        return rc

    def close(self):
        """Frees the context; refused (RuntimeError) while batches or networks
        created on it are alive."""
        if getattr(self, "h", None):
            rc = lib().lfdpr_destroy(self.h)
            if rc != LFDPR_OK:
                raise RuntimeError(f"lfdpr_destroy: {lib().lfdpr_last_error(self.h).decode()}")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- scene ---------------------------------------------------------------
    def upload_scene(self, scene) -> int:
        pos = np.ascontiguousarray(scene.pos, np.float32)
        uv = np.ascontiguousarray(scene.uv, np.float32)
        idx = np.ascontiguousarray(scene.idx, np.uint32)
        tex = np.ascontiguousarray(scene.tex, np.uint16)
        texs = [np.ascontiguousarray(t, np.uint8) for t in scene.textures]
        sizes = np.array([t.shape[0] for t in texs], np.int32)
        ptrs = (C.c_void_p * len(texs))(*[t.ctypes.data for t in texs])
        d = SceneDesc(pos.shape[0], idx.shape[0], _ptr(pos), _ptr(uv), _ptr(idx) if idx.size else None,
                      _ptr(tex) if tex.size else None, len(texs), _ptr(sizes), C.cast(ptrs, C.c_void_p))
        sid = C.c_int32()
        self._check(lib().lfdpr_scene_upload(self.h, C.byref(d), C.byref(sid)))
        mats = getattr(scene, "materials", None)
        if mats is not None:
            m = np.ascontiguousarray(mats, np.uint16).reshape(-1, 3)
            cols = [np.ascontiguousarray(m[:, k]) for k in range(3)]
            self._check(lib().lfdpr_scene_set_materials(self.h, sid.value, *[_ptr(c) for c in cols]))
        return sid.value

    def set_shading(self, shading):
        """Splat shading (scenes.Shading, or None for unlit albedo)."""
        sp = ShadingParams()
        if shading is not None and int(shading.mode) != 0:
            sp.mode = int(shading.mode)
            for k in range(3):
                sp.light_dir[k] = float(np.float32(shading.light_dir[k]))
                sp.light_rgb[k] = float(np.float32(shading.light_rgb[k]))
                sp.ambient_rgb[k] = float(np.float32(shading.ambient_rgb[k]))
        self._check(lib().lfdpr_set_shading(self.h, C.byref(sp)))

    def free_scene(self, sid: int):
        self._check(lib().lfdpr_scene_free(self.h, sid))

    # -- parameters ----------------------------------------------------------
    def set_views(self, vp, point_capacity: int = 0):
        p, keep = view_params(vp, point_capacity)
        self._check(lib().lfdpr_set_views(self.h, C.byref(p)))
        self.vp = vp

    def set_launch(self, splat_blocks: int, key_layout: int):
        self._check(lib().lfdpr_set_launch(self.h, splat_blocks, key_layout))

    def set_frames_in_flight(self, n: int):
        self._check(lib().lfdpr_set_frames_in_flight(self.h, n))
        self.frames_in_flight = int(n)

    def set_splat_order(self, order: int):
        """SPLAT_POINT (default), SPLAT_TRIANGLE_VIEW or SPLAT_QUILT; the same results."""
        self._check(lib().lfdpr_set_splat_order(self.h, int(order)))

    def set_quilt_tile(self, rows: int = 0, views: int = 0):
        """Tile of the quilt order: pixel rows x views in LDS (0, 0: chosen per rig)."""
        self._check(lib().lfdpr_set_quilt_tile(self.h, int(rows), int(views)))

    def set_quilt_capacity(self, entries: int = 0):
        """Band-list entries of the quilt order (0: twice the point capacity + 65536)."""
        self._check(lib().lfdpr_set_quilt_capacity(self.h, int(entries)))

    def autotune(self, sid: int, model: np.ndarray, views) -> dict:
        m = np.ascontiguousarray(model, np.float32).reshape(12)
        res = TuneResult()
        self._check(lib().lfdpr_autotune(self.h, sid, _ptr(m), _ptr(views), C.byref(res)))
        return tune_dict(res)

    def set_lens(self, lp, mode: Optional[int] = None):
        p = LensParams()
        p.Wp, p.Hp = lp.Wp, lp.Hp
        p.pitch_subpx, p.slope, p.offset = float(lp.pitch_subpx), float(lp.slope), float(lp.offset)
        p.mode = int(lp.mode if mode is None else mode)
        if lp.taps is not None:
            for k in range(8):
                for c in range(3):
                    p.taps[k][c] = int(lp.taps[k][c])
        self._check(lib().lfdpr_set_lens(self.h, C.byref(p)))
        self.lens = lp

    # -- per frame -----------------------------------------------------------
    @property
    def n_views(self) -> int:
        return self.vp.V * self.vp.S

    def alloc_views(self, with_depth: bool = False):
        torch = self._torch
        n = self.n_views * self.vp.H * self.vp.W
        v = torch.empty((self.n_views, self.vp.H, self.vp.W), dtype=torch.int32, device=f"cuda:{self.device}")
        d = torch.empty_like(v, dtype=torch.float32) if with_depth else None
        assert v.numel() == n
        return v, d

    def render_frame(self, sid: int, model: np.ndarray, views, depth=None):
        torch = self._torch
        if self.vp is not None:  # without a rig the library itself reports LFDPR_ESTATE
            n = self.n_views * self.vp.H * self.vp.W
            _check_dev(views, torch.int32, n, "views")
            if depth is not None:
                _check_dev(depth, torch.float32, n, "depth")
        m = np.ascontiguousarray(model, np.float32).reshape(12)
        self._check(lib().lfdpr_render_frame(self.h, sid, _ptr(m), _ptr(views), _ptr(depth) if depth is not None else None))

    def render_frame_noalloc(self, sid: int, model: np.ndarray, views, depth=None, stats=None):
        """lfdpr_render_frame_noalloc: the frame with the library's static
        scratch (no device allocation); stats: None or a device int64 tensor
        of >= 6 elements (points, active triangles, point-views, overflowed
        triangles, written pixels, point capacity)."""
        torch = self._torch
        if self.vp is not None:
            n = self.n_views * self.vp.H * self.vp.W
            _check_dev(views, torch.int32, n, "views")
            if depth is not None:
                _check_dev(depth, torch.float32, n, "depth")
        if stats is not None:
            _check_dev(stats, torch.int64, 6, "stats")
        m = np.ascontiguousarray(model, np.float32).reshape(12)
        self._check(lib().lfdpr_render_frame_noalloc(self.h, sid, _ptr(m), _ptr(views),
                                                     _ptr(depth) if depth is not None else None,
                                                     _ptr(stats) if stats is not None else None))

    def reconstruct(self, views, panel, n_views: Optional[int] = None, W: Optional[int] = None,
                    H: Optional[int] = None):
        torch = self._torch
        V = n_views if n_views is not None else views.shape[0]
        Hh = H if H is not None else views.shape[1]
        Ww = W if W is not None else views.shape[2]
        _check_dev(views, torch.int32, V * Hh * Ww, "views")
        _check_dev(panel, torch.uint8, self.lens.Wp * self.lens.Hp * 3, "panel")
        self._check(lib().lfdpr_reconstruct(self.h, _ptr(views), V, Ww, Hh, _ptr(panel)))

    def angular_filter(self, sub_views, out):
        torch = self._torch
        _check_dev(sub_views, torch.int32, self.n_views * self.vp.H * self.vp.W, "sub_views")
        _check_dev(out, torch.int32, self.vp.V * self.vp.H * self.vp.W, "out")
        self._check(lib().lfdpr_angular_filter(self.h, _ptr(sub_views), _ptr(out)))

    def stats(self, allow_overflow: bool = False) -> dict:
        s = Stats()
        rc = lib().lfdpr_get_stats(self.h, C.byref(s))
        if rc != LFDPR_OK and not (allow_overflow and rc == LFDPR_EOVERFLOW):
            self._check(rc)
        return {k: int(getattr(s, k)) for k, _ in Stats._fields_}

    def points(self) -> dict:
        """The last frame's point buffer, unpacked into numpy arrays."""
        torch = self._torch
        s = self.stats(allow_overflow=True)
        n = min(s["points"], s["capacity"])
        buf = torch.empty((max(n, 1), 4), dtype=torch.int32, device=f"cuda:{self.device}")
        got = C.c_int64()
        self._check(lib().lfdpr_copy_points(self.h, _ptr(buf), n, C.byref(got)))
        a = buf[:n].cpu().numpy().view(np.uint32)
        tri = a[:, 0] & 0x0FFFFFFF
        return dict(tri=tri, flags=(a[:, 0] >> 28).astype(np.uint8), i=(a[:, 1] & 0xFFFF).astype(np.uint16).view(np.int16),
                    j=(a[:, 1] >> 16).astype(np.uint16).view(np.int16), tvmin=a[:, 2].copy(), tvmax=a[:, 3].copy(),
                    n=int(got.value))

    def point_materials(self) -> dict:
        """Per-point material words of the last physically shaded frame."""
        torch = self._torch
        s = self.stats(allow_overflow=True)
        n = min(s["points"], s["capacity"])
        buf = torch.empty((max(n, 1), 4), dtype=torch.int32, device=f"cuda:{self.device}")
        got = C.c_int64()
        self._check(lib().lfdpr_copy_point_materials(self.h, _ptr(buf), n, C.byref(got)))
        a = buf[:n].cpu().numpy().view(np.uint32)
        return dict(nmin=a[:, 0].copy(), nmax=a[:, 1].copy(), rm=a[:, 2].copy(), n=int(got.value))

    def counts(self, nt: int) -> np.ndarray:
        torch = self._torch
        buf = torch.empty(max(nt, 1), dtype=torch.int32, device=f"cuda:{self.device}")
        self._check(lib().lfdpr_copy_counts(self.h, _ptr(buf), nt))
        return buf[:nt].cpu().numpy().view(np.uint32)

    STAGES = ("setup", "scan", "emit", "splat", "resolve", "interleave", "angular_filter", "quilt_bin")

    def timing(self, enable: bool):
        self._check(lib().lfdpr_timing(self.h, int(enable)))

    def timings(self) -> dict:
        """Per stage: (summed ms, launches) recorded since timing(True)."""
        ms = np.zeros(len(self.STAGES), np.float64)
        n = np.zeros(len(self.STAGES), np.int64)
        self._check(lib().lfdpr_get_timings(self.h, _ptr(ms), _ptr(n)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.STAGES)}

    def set_debug_records(self, f=None, i=None):
        n = 0
        if f is not None:
            n = min(f.numel(), i.numel()) // 8
        self._check(lib().lfdpr_set_debug_records(self.h, _ptr(f) if f is not None else None,
                                                  _ptr(i) if i is not None else None, n))


class Net:
    """The learned angular reconstruction network of one Renderer context."""

    def __init__(self, renderer: Renderer, V: int, max_h: int, max_w: int):
        self.R = renderer
        self._torch = renderer._torch
        h = C.c_void_p()
        rc = lib().lfdpr_net_create(renderer.h, V, max_h, max_w, C.byref(h))
        if rc != LFDPR_OK:
            raise LfdprError(rc, lib().lfdpr_strerror(rc).decode())
        self.h = h
        self.V = V
        n = C.c_int64()
        self._check(lib().lfdpr_net_param_count(self.h, C.byref(n)))
        self.n_params = n.value
        self.loss_buf = self._torch.zeros(1, dtype=self._torch.float32, device=f"cuda:{renderer.device}")
        self._last_shape = None  # (n, H, W) of the last forward: the shape backward's target must have

    def _check(self, rc: int):
        if rc != LFDPR_OK:
            last = lib().lfdpr_net_last_error(self.h) if getattr(self, "h", None) else b""
            raise LfdprError(rc, lib().lfdpr_strerror(rc).decode() + ": " + (last.decode() if last else ""))

    def close(self):
        if getattr(self, "h", None):
            lib().lfdpr_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat: np.ndarray):
        a = np.ascontiguousarray(flat, np.float32)
        self._check(lib().lfdpr_net_set_params(self.h, _ptr(a), a.size))

    def set_disparity_scale(self, k: float):
        """Pixels per view step per unit d of the input's disparity blur."""
        self._check(lib().lfdpr_net_set_disparity_scale(self.h, float(k)))

    def set_rig(self, vp):
        """The disparity scale of the rig (scenes.ViewParams) the views come from,
        computed by the library."""
        p, keep = view_params(vp)
        self._check(lib().lfdpr_net_set_rig(self.h, C.byref(p)))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.n_params, np.float32)
        self._check(lib().lfdpr_net_get_params(self.h, _ptr(a), a.size))
        return a

    def pack_input(self, views, depth, x, D: float = 1.0):
        """views (n, H, W) int32 RGBA8 (+ depth (n, H, W) float32 or None) -> x (n, H, W, 4) int16 (BF16 bits)."""
        torch = self._torch
        n, H, W = views.shape
        _check_dev(views, torch.int32, n * H * W, "views")
        if depth is not None:
            _check_dev(depth, torch.float32, n * H * W, "depth")
        _check_dev(x, torch.int16, n * H * W * 4, "x")
        self._check(lib().lfdpr_net_pack_input(self.h, _ptr(views), _ptr(depth) if depth is not None else None,
                                               n, H, W, float(D), _ptr(x)))

    def forward(self, x, y):
        """x, y: (n, H, W, 4) int16 BF16 bits, n a multiple of V."""
        torch = self._torch
        n, H, W, _ = x.shape
        _check_dev(x, torch.int16, n * H * W * 4, "x")
        _check_dev(y, torch.int16, n * H * W * 4, "y")
        self._check(lib().lfdpr_net_forward(self.h, _ptr(x), n, H, W, _ptr(y)))
        self._last_shape = (n, H, W)

    def backward(self, target):
        """target: (n, H, W, 4) int16 BF16 bits of the last forward's shape."""
        if self._last_shape is None:
            raise ValueError("backward needs a forward first")
        n, H, W = self._last_shape
        _check_dev(target, self._torch.int16, n * H * W * 4, "target")
        self._check(lib().lfdpr_net_backward(self.h, _ptr(target), _ptr(self.loss_buf)))
        return self.loss_buf

    def adam_step(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self._check(lib().lfdpr_net_adam_step(self.h, lr, b1, b2, eps))

    def unpack_output(self, y, views):
        torch = self._torch
        n, H, W, _ = y.shape
        _check_dev(views, torch.int32, n * H * W, "views")
        self._check(lib().lfdpr_net_unpack_output(self.h, _ptr(y), n, H, W, _ptr(views)))

    def copy_state(self, which: int, dst):
        self._check(lib().lfdpr_net_copy_state(self.h, which, _ptr(dst), dst.numel() * dst.element_size()))

    def save(self, path: str):
        self._check(lib().lfdpr_net_save(self.h, path.encode()))

    def load(self, path: str):
        self._check(lib().lfdpr_net_load(self.h, path.encode()))


def params_to_flat(params) -> np.ndarray:
    """[(W (9, co, ci), b (co)), ...] -> the library's flat FP32 parameter vector."""
    return np.concatenate([np.concatenate([np.asarray(w, np.float32).ravel(), np.asarray(b, np.float32).ravel()])
                           for w, b in params])


NET_SHAPES = [(24, 32), (32, 32), (32, 32), (32, 3)]  # (cin, cout) per layer


def flat_to_params(flat: np.ndarray):
    out, o = [], 0
    for ci, co in NET_SHAPES:
        w = flat[o:o + 9 * co * ci].reshape(9, co, ci)
        o += 9 * co * ci
        b = flat[o:o + co]
        o += co
        out.append((w, b))
    return out


class Batch:
    """Several scene frames rendered with one launch per stage (lfdpr_batch_*)."""

    def __init__(self, renderer: Renderer, scene_ids, view_params_list, point_capacity: int = 0):
        self.R = renderer
        self._torch = renderer._torch
        n = len(scene_ids)
        ids = np.ascontiguousarray(scene_ids, np.int32)
        arr = (ViewParams * n)()
        self._keep = []
        for k, vp in enumerate(view_params_list):
            p, jit = view_params(vp)
            arr[k] = p
            self._keep.append(jit)
        h = C.c_void_p()
        renderer._check(lib().lfdpr_batch_create(renderer.h, n, _ptr(ids), C.cast(arr, C.c_void_p), point_capacity,
                                                 C.byref(h)))
        self.h = h
        self.n = n
        vp0 = view_params_list[0]
        self.shape = (n, vp0.V * vp0.S, vp0.H, vp0.W)

    def _check(self, rc):
        if rc != LFDPR_OK:
            last = lib().lfdpr_batch_last_error(self.h)
            raise LfdprError(rc, lib().lfdpr_strerror(rc).decode() + ": " + (last.decode() if last else ""))

    def close(self):
        if getattr(self, "h", None):
            lib().lfdpr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def use_graph(self, enable: bool):
        self._check(lib().lfdpr_batch_use_graph(self.h, int(enable)))

    def set_frames_in_flight(self, n: int):
        """2: a call's point generation overlaps the previous call's splat."""
        self._check(lib().lfdpr_batch_set_frames_in_flight(self.h, int(n)))

    def alloc_views(self):
        return self._torch.empty(self.shape, dtype=self._torch.int32, device=f"cuda:{self.R.device}")

    def render(self, models, views, panels=None):
        """panels: None, or (n, Hp, Wp, 3) uint8 for the context's lens."""
        m = np.ascontiguousarray(np.asarray(models, np.float32).reshape(self.n, 12))
        _check_dev(views, self._torch.int32, int(np.prod(self.shape)), "views")
        if panels is not None:
            if self.R.lens is None:
                raise ValueError("panels need a lens (Renderer.set_lens) on the batch's context")
            _check_dev(panels, self._torch.uint8, self.n * self.R.lens.Hp * self.R.lens.Wp * 3, "panels")
        self._check(lib().lfdpr_batch_render(self.h, _ptr(m), _ptr(views), _ptr(panels) if panels is not None else None))

    def stats(self) -> dict:
        s = Stats()
        rc = lib().lfdpr_batch_stats(self.h, C.byref(s))
        if rc not in (LFDPR_OK, LFDPR_EOVERFLOW):
            self._check(rc)
        return {k: int(getattr(s, k)) for k, _ in Stats._fields_}

    def autotune(self, models, views) -> dict:
        m = np.ascontiguousarray(np.asarray(models, np.float32).reshape(self.n, 12))
        res = TuneResult()
        self._check(lib().lfdpr_batch_autotune(self.h, _ptr(m), _ptr(views), C.byref(res)))
        return tune_dict(res)
