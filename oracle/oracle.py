"""CPU oracle for the LFDPR hot path: Python front end of ``lfdpr_oracle.c``.

TEST INFRASTRUCTURE ONLY.  Imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg; never by the product path.  It shares no
code with the HIP path: the rig/lens tables below are computed here, in
double, from the paper's description (Sec. 3.1, Sec. 4, Sec. 5.1), and the
HIP library computes its own copies independently.

Functions and what pins them (see tests/test_oracle_pins.py):
  view_table        -- camera rig (parallel off-axis eyes, shared focal plane)
                                                            [pinned: eye offsets recovered
                       from rendered depth, focal-plane invariance]
  lens_constants    -- tilted-lens phase constants (prototype geometry, Sec. 5.1)
  angular_table     -- Gaussian weights for the angular supersampling filter
  build_textures    -- box mip chains                      [pinned: numpy box mean]
  render            -- point generation + splatting         [pinned: brute-force lattice
                       counts, closest-point brute force, reverse-projection geometry,
                       rasteriser coverage identity, constant-texture identity,
                       Eqs. 8-9 in double from ray-cast footprints, no orphans or
                       misses at display size]
  interleave        -- panel interleave + reconstruction    [pinned: index-map readout,
                       lens-independence, slope-0 closed form]
  angular_filter    -- 4x angular SS -> V views             [pinned: focal-plane identity,
                       constant input, weight normalisation]
  rasterise         -- conventional z-buffer multiview renderer (gold standard)
  tangent_frame, pbr_terms, pbr_shade
                    -- physically based shading of the PBR mode [pinned: GGX
                       normalisation integral, Helmholtz reciprocity, rotation
                       invariance, Fresnel and geometry limits, tangent frame of
                       axis-aligned mappings, texture-swap reductions of the
                       point data, unlit-density reduction of Eq. 1's maximum]
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lfdpr_oracle.c")
_LIB = os.path.join(_HERE, "liblfdpr_oracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.orc_lattice_cells.restype = C.c_int
        _lib.orc_trilinear.restype = C.c_uint32
        _lib.orc_lod_q8.restype = C.c_int
        _lib.orc_lod_q8.argtypes = [C.c_float]
    return _lib


# ---------------------------------------------------------------------------
# ctypes mirrors of the oracle's own structs


class _Scene(C.Structure):
    _fields_ = [("nv", C.c_int), ("nt", C.c_int), ("pos", C.c_void_p), ("uv", C.c_void_p),
                ("idx", C.c_void_p), ("tex", C.c_void_p), ("ntex", C.c_int),
                ("tex_size", C.c_void_p), ("tex_levels", C.c_void_p), ("tex_level_off", C.c_void_p),
                ("texels", C.c_void_p), ("mat", C.c_void_p)]


class _Frame(C.Structure):
    _fields_ = [("n_views", C.c_int), ("W", C.c_int), ("H", C.c_int), ("mip", C.c_int),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("rD", C.c_float), ("znear", C.c_float), ("eye", C.c_void_p), ("kshift", C.c_void_p),
                ("model", C.c_float * 12), ("shade", C.c_int), ("light", C.c_float * 9)]


class _Out(C.Structure):
    _fields_ = [("count", C.c_void_p), ("trif", C.c_void_p), ("trii", C.c_void_p),
                ("point_cap", C.c_int64), ("p_tri", C.c_void_p), ("p_i", C.c_void_p), ("p_j", C.c_void_p),
                ("p_flags", C.c_void_p), ("p_tvmin", C.c_void_p), ("p_tvmax", C.c_void_p),
                ("keys", C.c_void_p), ("stats", C.c_void_p), ("unused", C.c_void_p),
                ("p_nmin", C.c_void_p), ("p_nmax", C.c_void_p), ("p_rm", C.c_void_p),
                ("tframe", C.c_void_p), ("tlod", C.c_void_p), ("pv_tq", C.c_void_p), ("pv_col", C.c_void_p)]


class _Lens(C.Structure):
    _fields_ = [("Wp", C.c_int), ("Hp", C.c_int), ("mode", C.c_int), ("K1", C.c_uint32),
                ("Ky", C.c_uint32), ("K0", C.c_uint32), ("taps", C.c_void_p)]


def _p(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# ---------------------------------------------------------------------------
# rig, lens and filter tables (double precision, rounded once)


def subview_positions(vp) -> np.ndarray:
    """Position q of every rendered (sub-)view on the view axis, in view
    intervals: plain views sit at interval centres v + 0.5; with angular
    supersampling factor S, sub-view k of view v sits at v + (k + 0.5 + j)/S
    with a random jitter j in [-0.5, 0.5) (Sec. 4: random angles in view
    intervals)."""
    q = np.empty(vp.V * vp.S, np.float64)
    for v in range(vp.V):
        for k in range(vp.S):
            j = float(vp.jitter[v * vp.S + k]) if (vp.S > 1 and vp.jitter is not None) else 0.0
            q[v * vp.S + k] = v + 0.5 if vp.S == 1 else v + (k + 0.5 + j) / vp.S
    return q


def view_table(vp) -> Dict[str, object]:
    """Parallel off-axis cameras sharing one orientation and the focal plane
    Z = D; eye r sits at (b_r, 0, 0) with b = D tan(cone/2) (2q/V - 1) (Sec. 3.1,
    reading R2).  The rig is given by binary32 parameters, as the library's
    interface takes them: the double evaluation starts from D, cone, field of
    view and aspect rounded to binary32, degrees taken to radians as
    deg * (pi / 180)."""
    D, cone = float(np.float32(vp.D)), float(np.float32(vp.cone_deg))
    fovy, aspect = float(np.float32(vp.fovy_deg)), float(np.float32(vp.aspect))
    B = D * math.tan(cone * (math.pi / 180.0) / 2.0)
    q = subview_positions(vp)
    b = B * (2.0 * q / vp.V - 1.0)
    t = math.tan(fovy * (math.pi / 180.0) / 2.0)
    return dict(
        fx=np.float32((vp.W / 2.0) / (aspect * t)), fy=np.float32((vp.H / 2.0) / t),
        cx=np.float32(vp.W / 2.0), cy=np.float32(vp.H / 2.0), rD=np.float32(1.0 / D),
        znear=np.float32(vp.znear), eye=b.astype(np.float32), kshift=(b / D).astype(np.float32),
        q=q)


def lens_constants(lp, V: int):
    """Q32 lens-phase constants: phase = (subpixel - 3*slope*row)/pitch + offset."""
    two32 = 2.0 ** 32
    K1 = int(round(two32 / lp.pitch_subpx)) % (1 << 32)
    Ky = int(round(-3.0 * lp.slope * two32 / lp.pitch_subpx)) % (1 << 32)
    K0 = int(round(lp.offset * two32)) % (1 << 32)
    return K1, Ky, K0


def angular_table(vp):
    """For output view v: sub-views within one view interval of its centre,
    weighted by round(65535 exp(-d^2 / (2 * 0.5^2)))."""
    q = subview_positions(vp)
    maxe = 3 * vp.S
    cnt = np.zeros(vp.V, np.int32)
    src = np.zeros((vp.V, maxe), np.int32)
    wt = np.zeros((vp.V, maxe), np.uint32)
    for v in range(vp.V):
        for r in range(vp.V * vp.S):
            d = q[r] - (v + 0.5)
            if abs(d) < 1.0:
                src[v, cnt[v]] = r
                wt[v, cnt[v]] = int(round(65535.0 * math.exp(-d * d / (2.0 * 0.25))))
                cnt[v] += 1
    return cnt, src, wt, maxe


# ---------------------------------------------------------------------------


class Textures:
    def __init__(self, scene):
        self.ntex = len(scene.textures)
        self.size = np.array([t.shape[0] for t in scene.textures], np.int32)
        self.levels = np.array([int(math.log2(s)) + 1 for s in self.size], np.int32)
        self.off = np.zeros((max(1, self.ntex), 16), np.int64)
        total = 0
        for k, s in enumerate(self.size):
            o = total
            for lvl in range(self.levels[k]):
                self.off[k, lvl] = o
                o += (int(s) >> lvl) ** 2 * 4
            total = o
        self.texels = np.zeros(max(total, 4), np.uint8)
        for k, t in enumerate(scene.textures):
            s = int(self.size[k])
            chain = np.zeros(sum((s >> l) ** 2 * 4 for l in range(self.levels[k])), np.uint8)
            lib().orc_build_mips(C.c_void_p(_p(np.ascontiguousarray(t))), C.c_int(s), C.c_void_p(_p(chain)))
            self.texels[self.off[k, 0]:self.off[k, 0] + chain.size] = chain

    def level(self, k: int, lvl: int) -> np.ndarray:
        s = int(self.size[k]) >> lvl
        o = int(self.off[k, lvl])
        return self.texels[o:o + s * s * 4].reshape(s, s, 4)


def build_textures(scene) -> Textures:
    return Textures(scene)


def _scene_struct(scene, tx: Textures, keep: list) -> _Scene:
    arrs = [np.ascontiguousarray(scene.pos, np.float32), np.ascontiguousarray(scene.uv, np.float32),
            np.ascontiguousarray(scene.idx, np.uint32), np.ascontiguousarray(scene.tex, np.uint16)]
    mat = getattr(scene, "materials", None)
    if mat is not None:
        mat = np.ascontiguousarray(mat, np.uint16).reshape(-1, 3)
        arrs.append(mat)
    keep += arrs
    return _Scene(scene.n_verts, scene.n_tris, _p(arrs[0]), _p(arrs[1]), _p(arrs[2]), _p(arrs[3]),
                  tx.ntex, _p(tx.size), _p(tx.levels), _p(tx.off), _p(tx.texels),
                  _p(mat) if mat is not None else None)


def _set_shading(f: _Frame, shading) -> None:
    """Shading mode and light (camera space): unit direction towards the light,
    light RGB, ambient RGB."""
    if shading is None or int(shading.mode) == 0:
        f.shade = 0
        return
    f.shade = 1
    vals = list(np.float32(shading.light_dir)) + list(np.float32(shading.light_rgb)) + \
        list(np.float32(shading.ambient_rgb))
    for k in range(9):
        f.light[k] = float(vals[k])


def _frame_struct(vp, vt, model, keep: list) -> _Frame:
    eye = np.ascontiguousarray(vt["eye"], np.float32)
    ks = np.ascontiguousarray(vt["kshift"], np.float32)
    keep += [eye, ks]
    f = _Frame()
    f.n_views, f.W, f.H, f.mip = vp.V * vp.S, vp.W, vp.H, int(vp.mip)
    f.fx, f.fy, f.cx, f.cy = float(vt["fx"]), float(vt["fy"]), float(vt["cx"]), float(vt["cy"])
    f.rD, f.znear = float(vt["rD"]), float(vt["znear"])
    f.eye, f.kshift = _p(eye), _p(ks)
    m = np.ascontiguousarray(model, np.float32).reshape(12)
    for k in range(12):
        f.model[k] = float(m[k])
    return f


def render(scene, vp, model: np.ndarray, tx: Optional[Textures] = None, point_cap: Optional[int] = None,
           shading=None, observe: bool = False):
    """Point generation + splatting of one frame into all V*S rendered views.

    Returns a dict with per-triangle counts and records, the point buffer in
    emission order, RGBA8 views (n_views, H, W) as uint32, FP32 depth and stats.
    With a PBR `shading` the scene must carry materials; the point buffer then
    also holds the normal-map fetches and the roughness/metallic bytes, and the
    per-triangle tangent frames and LODs are returned.  With `observe`, the
    Eq. 9 weight tq and the colour of every (point, view) that writes a pixel
    are returned as `pv_tq` (-1 elsewhere) and `pv_col`, (n_points, n_views)."""
    tx = tx or build_textures(scene)
    vt = view_table(vp)
    keep: list = []
    sc = _scene_struct(scene, tx, keep)
    fr = _frame_struct(vp, vt, model, keep)
    _set_shading(fr, shading)
    pbr = fr.shade == 1
    if pbr and getattr(scene, "materials", None) is None:
        raise ValueError("PBR shading needs scene materials")
    nt = scene.n_tris
    nviews = vp.V * vp.S
    cap = point_cap if point_cap is not None else max(64, 24 * nt)
    o = dict(count=np.zeros(nt, np.int32), trif=np.zeros((nt, 8), np.float32), trii=np.zeros((nt, 8), np.int32),
             p_tri=np.zeros(cap, np.uint32), p_i=np.zeros(cap, np.int16), p_j=np.zeros(cap, np.int16),
             p_flags=np.zeros(cap, np.uint8), p_tvmin=np.zeros(cap, np.uint32), p_tvmax=np.zeros(cap, np.uint32),
             keys=np.full((nviews, vp.H, vp.W), np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64),
             stats=np.zeros(8, np.int64))
    if pbr:
        o.update(p_nmin=np.zeros(cap, np.uint32), p_nmax=np.zeros(cap, np.uint32), p_rm=np.zeros(cap, np.uint32),
                 tframe=np.zeros((nt, 6), np.float32), tlod=np.zeros((nt, 8), np.int32))
    if observe:
        o.update(pv_tq=np.full((cap, nviews), -1, np.int16), pv_col=np.zeros((cap, nviews), np.uint32))
    opt = [_p(o[k]) if k in o else None for k in ("p_nmin", "p_nmax", "p_rm", "tframe", "tlod", "pv_tq", "pv_col")]
    out = _Out(_p(o["count"]), _p(o["trif"]), _p(o["trii"]), cap, _p(o["p_tri"]), _p(o["p_i"]), _p(o["p_j"]),
               _p(o["p_flags"]), _p(o["p_tvmin"]), _p(o["p_tvmax"]), _p(o["keys"]), _p(o["stats"]), None, *opt)
    rc = lib().orc_render(C.byref(sc), C.byref(fr), C.byref(out))
    if rc != 0:
        raise ValueError(f"oracle render failed ({rc})")
    n = int(o["stats"][0])
    if n > cap:
        return render(scene, vp, model, tx, point_cap=n, shading=shading, observe=observe)
    rgba = np.zeros((nviews, vp.H, vp.W), np.uint32)
    depth = np.zeros((nviews, vp.H, vp.W), np.float32)
    lib().orc_resolve(C.c_void_p(_p(o["keys"])), C.c_int64(o["keys"].size), C.c_void_p(_p(rgba)), C.c_void_p(_p(depth)))
    st = o["stats"]
    points = dict(tri=o["p_tri"][:n], i=o["p_i"][:n], j=o["p_j"][:n], flags=o["p_flags"][:n],
                  tvmin=o["p_tvmin"][:n], tvmax=o["p_tvmax"][:n])
    extra = {}
    if pbr:
        points.update(nmin=o["p_nmin"][:n], nmax=o["p_nmax"][:n], rm=o["p_rm"][:n])
        extra = dict(tframe=o["tframe"], tlod=o["tlod"])
    if observe:
        extra.update(pv_tq=o["pv_tq"][:n], pv_col=o["pv_col"][:n])
    return dict(count=o["count"], trif=o["trif"], trii=o["trii"], n_points=n, points=points, **extra,
                keys=o["keys"], rgba=rgba, depth=depth,
                stats=dict(points=int(st[0]), active_tris=int(st[1]), point_views=int(st[2]), orphans=int(st[3]),
                           misses=int(st[4]), overflow_tris=int(st[5]), fragments=int(st[6])),
                view_table=vt)


def rasterise(scene, vp, model: np.ndarray, tx: Optional[Textures] = None):
    """Conventional multiview rendering: one z-buffer pass per view, same vertex
    projection and coverage rule, perspective-correct attributes and per-pixel
    trilinear mipmapping in double."""
    tx = tx or build_textures(scene)
    vt = view_table(vp)
    keep: list = []
    sc = _scene_struct(scene, tx, keep)
    fr = _frame_struct(vp, vt, model, keep)
    nviews = vp.V * vp.S
    rgba = np.zeros((nviews, vp.H, vp.W), np.uint32)
    depth = np.zeros((nviews, vp.H, vp.W), np.float32)
    lib().orc_rasterise(C.byref(sc), C.byref(fr), C.c_void_p(_p(rgba)), C.c_void_p(_p(depth)))
    return rgba, depth


def interleave(views: np.ndarray, lp, taps: Optional[np.ndarray] = None, mode: Optional[int] = None) -> np.ndarray:
    """Interleave V views (V, H, W) RGBA8-as-uint32 into the Hp x Wp x 3 panel."""
    views = np.ascontiguousarray(views, np.uint32)
    V, Hv, Wv = views.shape
    K1, Ky, K0 = lens_constants(lp, V)
    t = np.ascontiguousarray(taps if taps is not None else (lp.taps if lp.taps is not None else np.zeros((8, 3))), np.int64)
    ln = _Lens(lp.Wp, lp.Hp, int(lp.mode if mode is None else mode), K1, Ky, K0, _p(t))
    panel = np.zeros((lp.Hp, lp.Wp, 3), np.uint8)
    lib().orc_interleave(C.c_void_p(_p(views)), C.c_int(V), C.c_int(Wv), C.c_int(Hv), C.byref(ln), C.c_void_p(_p(panel)))
    return panel


def angular_filter(sub_views: np.ndarray, vp) -> np.ndarray:
    sub_views = np.ascontiguousarray(sub_views, np.uint32)
    cnt, src, wt, maxe = angular_table(vp)
    out = np.zeros((vp.V, vp.H, vp.W), np.uint32)
    lib().orc_angular_filter(C.c_void_p(_p(sub_views)), C.c_int(vp.V), C.c_int(vp.W), C.c_int(vp.H),
                             C.c_void_p(_p(cnt)), C.c_void_p(_p(src)), C.c_void_p(_p(wt)), C.c_int(maxe),
                             C.c_void_p(_p(out)))
    return out


def lattice_cells(S, T, cap: int = 1 << 20):
    S = np.ascontiguousarray(S, np.int64)
    T = np.ascontiguousarray(T, np.int64)
    ci = np.zeros(cap, np.int32)
    cj = np.zeros(cap, np.int32)
    n = lib().orc_lattice_cells(C.c_void_p(_p(S)), C.c_void_p(_p(T)), C.c_int(cap), C.c_void_p(_p(ci)), C.c_void_p(_p(cj)))
    if n < 0:
        raise ValueError("cell cap exceeded")
    return ci[:n].copy(), cj[:n].copy()


def closest_point(p, a, b, c) -> np.ndarray:
    arrs = [np.ascontiguousarray(x, np.float32) for x in (p, a, b, c)]
    out = np.zeros(3, np.float32)
    lib().orc_closest_point(*[C.c_void_p(_p(x)) for x in arrs], C.c_void_p(_p(out)))
    return out


def trilinear(tx: Textures, t: int, u: float, v: float, kc: int) -> int:
    sc = _Scene(0, 0, None, None, None, None, tx.ntex, _p(tx.size), _p(tx.levels), _p(tx.off), _p(tx.texels), None)
    return int(lib().orc_trilinear(C.byref(sc), C.c_int(t), C.c_float(u), C.c_float(v), C.c_int(kc)))


def lod_q8(a: float) -> int:
    return int(lib().orc_lod_q8(float(a)))


def unpack_rgba(u32: np.ndarray) -> np.ndarray:
    return u32.view(np.uint8).reshape(*u32.shape, 4)


# ---------------------------------------------------------------------------
# physically based shading pieces (PBR mode)


def _f32(x, n):
    a = np.ascontiguousarray(np.asarray(x, np.float32).reshape(n))
    return a


def tangent_frame(e1, e2, duv, nh, u, w) -> np.ndarray:
    """(T, B) of the texture mapping for edges e1, e2 with UV differences
    duv = (du1, dv1, du2, dv2); u, w = fallback axes."""
    arrs = [_f32(e1, 3), _f32(e2, 3), _f32(duv, 4), _f32(nh, 3), _f32(u, 3), _f32(w, 3)]
    out = np.zeros(6, np.float32)
    lib().orc_tangent_frame(*[C.c_void_p(_p(a)) for a in arrs], C.c_void_p(_p(out)))
    return out


def pbr_terms(n, v, L, rough: float, metal: float, albedo) -> Dict[str, object]:
    """BRDF pieces for unit n, v, L: D, G, n.L, n.V, Fresnel F (RGB) and the
    BRDF value f (RGB)."""
    arrs = [_f32(n, 3), _f32(v, 3), _f32(L, 3)]
    a = _f32(albedo, 3)
    out = np.zeros(10, np.float32)
    lib().orc_pbr_terms(*[C.c_void_p(_p(x)) for x in arrs], C.c_float(rough), C.c_float(metal),
                        C.c_void_p(_p(a)), C.c_void_p(_p(out)))
    return dict(D=out[0], G=out[1], NL=out[2], NV=out[3], F=out[4:7].copy(), f=out[7:10].copy())


def pbr_shade(light, frame, Pc, b: float, albedo: int, normal: int, rough: int, metal: int) -> int:
    """Shaded RGBA8 of one splat: light = 9 floats (direction, RGB, ambient RGB),
    frame = 9 floats (T, B, unit normal), Pc = cell centre, b = eye offset,
    byte inputs already interpolated with tau."""
    lt, fr, pc = _f32(light, 9), _f32(frame, 9), _f32(Pc, 3)
    f = lib().orc_pbr_shade
    f.restype = C.c_uint32
    return int(f(C.c_void_p(_p(lt)), C.c_void_p(_p(fr)), C.c_void_p(_p(pc)), C.c_float(b), C.c_uint32(albedo),
                 C.c_uint32(normal), C.c_uint32(rough), C.c_uint32(metal)))
