"""Seeded synthetic inputs for light field display point rendering.

This module only *makes inputs*: triangle meshes, RGBA8 textures, per-frame
model matrices, view/lens parameter sets, the random sub-view jitter and the
random reconstruction taps.  It holds none of the rendering method's
arithmetic, and both the HIP path and the CPU oracle take their inputs from it.

Scene shapes follow the paper's workloads (Sec. 5.1: 0.3-2M triangles, large
textures, triangles tessellated to at most ~100 px, 48 views, rotating
scenes).  The paper's own scenes are not available; these procedural scenes
stand in for them.

Coordinates: camera space is right-handed with +X right, +Y down, +Z forward.
Triangles are wound so that (P1-P0) x (P2-P0) points out of the surface.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# meshes
# ---------------------------------------------------------------------------


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def icosphere(level: int) -> Tuple[np.ndarray, np.ndarray]:
    """Unit icosphere: 10*4^level+2 vertices, 20*4^level triangles."""
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache = {}
        nf = []

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key in cache:
                return cache[key]
            p = np.add(verts[a], verts[b]) * 0.5
            p = p / np.linalg.norm(p)
            verts.append(tuple(p))
            cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(nf, np.int64)
    v = np.array(verts, np.float64)
    # outward winding: (P1-P0)x(P2-P0) . centroid > 0
    p0, p1, p2 = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(p1 - p0, p2 - p0), p0 + p1 + p2)
    flip = s < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f


def heightfield(n: int, rng: np.random.Generator, amp: float) -> Tuple[np.ndarray, np.ndarray]:
    """n x n quads over [-1,1]^2 in (x, y) with fBm height along -z.

    Vertices are (x, y, h); the surface faces -z (towards a camera at -z)."""
    g = np.linspace(-1.0, 1.0, n + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    H = np.zeros_like(X)
    a = 1.0
    for octave in range(6):
        cells = 4 * 2 ** octave
        grid = rng.standard_normal((cells + 1, cells + 1))
        fx = (X + 1.0) * 0.5 * cells
        fy = (Y + 1.0) * 0.5 * cells
        ix = np.minimum(fx.astype(np.int64), cells - 1)
        iy = np.minimum(fy.astype(np.int64), cells - 1)
        tx = fx - ix
        ty = fy - iy
        tx = tx * tx * (3 - 2 * tx)
        ty = ty * ty * (3 - 2 * ty)
        v00 = grid[iy, ix]
        v10 = grid[iy, ix + 1]
        v01 = grid[iy + 1, ix]
        v11 = grid[iy + 1, ix + 1]
        H += a * ((v00 * (1 - tx) + v10 * tx) * (1 - ty) + (v01 * (1 - tx) + v11 * tx) * ty)
        a *= 0.5
    H *= amp / 2.0
    verts = np.stack([X.ravel(), Y.ravel(), -H.ravel()], axis=1)
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    a0 = idx[:-1, :-1].ravel()
    a1 = idx[:-1, 1:].ravel()
    b0 = idx[1:, :-1].ravel()
    b1 = idx[1:, 1:].ravel()
    # (x right, y down): want normal towards -z.  (a1-a0) = +x, (b0-a0) = +y,
    # +x cross +y = +z, so wind a0, b0, a1 (normal -z).
    t1 = np.stack([a0, b0, a1], axis=1)
    t2 = np.stack([a1, b0, b1], axis=1)
    faces = np.empty((2 * n * n, 3), np.int64)
    faces[0::2] = t1
    faces[1::2] = t2
    return verts, faces


# ---------------------------------------------------------------------------
# textures
# ---------------------------------------------------------------------------


def value_noise_texture(size: int, rng: np.random.Generator, octaves: int = 6) -> np.ndarray:
    """Seeded fBm value noise (smooth-step interpolated lattice noise, separable)
    mapped through a random two-colour ramp, RGBA8."""
    acc = np.zeros((size, size), np.float32)
    amp, tot = 1.0, 0.0
    coords = np.arange(size, dtype=np.float32) + 0.5
    for o in range(octaves):
        cells = 4 * 2 ** o
        if cells > size:
            break
        grid = rng.random((cells, cells)).astype(np.float32)
        f = coords * np.float32(cells / size) - np.float32(0.5)
        i0 = np.floor(f).astype(np.int64)
        t = f - i0
        t = t * t * (3 - 2 * t)
        i0m = i0 % cells
        i1m = (i0 + 1) % cells
        rows = grid[i0m] * (1 - t)[:, None] + grid[i1m] * t[:, None]          # (size, cells)
        val = rows[:, i0m] * (1 - t)[None, :] + rows[:, i1m] * t[None, :]     # (size, size)
        acc += np.float32(amp) * val
        tot += amp
        amp *= 0.5
    acc *= np.float32(2.2 / tot)
    acc += np.float32(0.5 - 1.1)
    np.clip(acc, 0.0, 1.0, out=acc)
    c0 = rng.integers(0, 256, 3).astype(np.float32)
    c1 = rng.integers(0, 256, 3).astype(np.float32)
    out = np.empty((size, size, 4), np.uint8)
    for ch in range(3):
        out[..., ch] = (c0[ch] + (c1[ch] - c0[ch]) * acc + np.float32(0.5)).astype(np.uint8)
    out[..., 3] = 255
    return out


def checker_texture(size: int, rng: np.random.Generator) -> np.ndarray:
    period = int(2 ** rng.uniform(3, 8))  # 8..256 texels
    period = max(1, min(period, size))
    y, x = np.mgrid[0:size, 0:size]
    m = ((x // period + y // period) % 2).astype(bool)
    c0 = rng.integers(0, 256, 3)
    c1 = rng.integers(0, 256, 3)
    out = np.empty((size, size, 4), np.uint8)
    out[..., :3] = np.where(m[..., None], c1[None, None, :], c0[None, None, :])
    out[..., 3] = 255
    return out


def _noise_field(size: int, rng: np.random.Generator, octaves: int = 5) -> np.ndarray:
    """Tileable fBm value noise in [0, 1] (float32, size x size)."""
    acc = np.zeros((size, size), np.float32)
    amp, tot = 1.0, 0.0
    coords = np.arange(size, dtype=np.float32) + 0.5
    for o in range(octaves):
        cells = 4 * 2 ** o
        if cells > size:
            break
        grid = rng.random((cells, cells)).astype(np.float32)
        f = coords * np.float32(cells / size) - np.float32(0.5)
        i0 = np.floor(f).astype(np.int64)
        t = f - i0
        t = t * t * (3 - 2 * t)
        rows = grid[i0 % cells] * (1 - t)[:, None] + grid[(i0 + 1) % cells] * t[:, None]
        acc += np.float32(amp) * (rows[:, i0 % cells] * (1 - t)[None, :] + rows[:, (i0 + 1) % cells] * t[None, :])
        tot += amp
        amp *= 0.5
    return acc / np.float32(tot)


def normal_map_texture(size: int, rng: np.random.Generator, strength: float = 6.0) -> np.ndarray:
    """Tangent-space normal map of a tileable bump field: n = normalize(-dh/dx,
    -dh/dy, 1) with wrap-around central differences, stored as round((n + 1)/2 * 255)."""
    h = _noise_field(size, rng) * np.float32(strength)
    gx = (np.roll(h, -1, axis=1) - np.roll(h, 1, axis=1)) * np.float32(0.5 * size / 64.0)
    gy = (np.roll(h, -1, axis=0) - np.roll(h, 1, axis=0)) * np.float32(0.5 * size / 64.0)
    n = np.stack([-gx, -gy, np.ones_like(h)], axis=-1)
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    out = np.empty((size, size, 4), np.uint8)
    out[..., :3] = np.clip(np.rint((n + 1.0) * 127.5), 0, 255).astype(np.uint8)
    out[..., 3] = 255
    return out


def scalar_texture(size: int, rng: np.random.Generator, lo: float, hi: float) -> np.ndarray:
    """Grey value noise in [lo, hi] (all channels equal; the shader reads R)."""
    v = np.float32(lo) + (np.float32(hi - lo)) * _noise_field(size, rng)
    g = np.clip(np.rint(v * 255.0), 0, 255).astype(np.uint8)
    out = np.empty((size, size, 4), np.uint8)
    out[..., 0] = out[..., 1] = out[..., 2] = g
    out[..., 3] = 255
    return out


def metallic_texture(size: int, rng: np.random.Generator) -> np.ndarray:
    """Metal/dielectric mask: a seeded checker of fully metallic (255) and
    dielectric (0) cells with soft noise on top, in R."""
    period = max(1, min(size, int(2 ** rng.uniform(2, 6))))
    y, x = np.mgrid[0:size, 0:size]
    m = ((x // period + y // period) % 2).astype(np.float32)
    v = np.clip(m * np.float32(0.9) + np.float32(0.1) * _noise_field(size, rng), 0.0, 1.0)
    g = np.rint(v * 255.0).astype(np.uint8)
    out = np.empty((size, size, 4), np.uint8)
    out[..., 0] = out[..., 1] = out[..., 2] = g
    out[..., 3] = 255
    return out


def constant_texture(size: int, rgba) -> np.ndarray:
    out = np.empty((size, size, 4), np.uint8)
    out[...] = np.asarray(rgba, np.uint8)
    return out


# ---------------------------------------------------------------------------
# scene container
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Scene:
    pos: np.ndarray          # (nv, 3) float32, scene coordinates (centred)
    uv: np.ndarray           # (nv, 2) float32
    idx: np.ndarray          # (nt, 3) uint32
    tex: np.ndarray          # (nt,) uint16 texture id per triangle
    textures: List[np.ndarray]  # each (s, s, 4) uint8, s a power of two
    name: str = ""
    materials: Optional[np.ndarray] = None  # (nt, 3) uint16: normal, roughness, metallic texture ids (PBR)

    @property
    def n_tris(self) -> int:
        return int(self.idx.shape[0])

    @property
    def n_verts(self) -> int:
        return int(self.pos.shape[0])

    def check(self):
        assert self.pos.dtype == np.float32 and self.pos.ndim == 2 and self.pos.shape[1] == 3
        assert self.uv.dtype == np.float32 and self.uv.shape == (self.n_verts, 2)
        assert self.idx.dtype == np.uint32 and self.idx.shape[1] == 3
        assert self.tex.dtype == np.uint16 and self.tex.shape == (self.n_tris,)
        assert int(self.idx.max(initial=0)) < self.n_verts
        for t in self.textures:
            s = t.shape[0]
            assert t.dtype == np.uint8 and t.shape == (s, s, 4) and s & (s - 1) == 0
        if self.n_tris:
            assert int(self.tex.max()) < len(self.textures)
        if self.materials is not None:
            assert self.materials.dtype == np.uint16 and self.materials.shape == (self.n_tris, 3)
            if self.n_tris:
                assert int(self.materials.max()) < len(self.textures)
        return self


def _combine(parts):
    pos, uv, idx, tex = [], [], [], []
    base = 0
    for p, u, f, t in parts:
        pos.append(p)
        uv.append(u)
        idx.append(f + base)
        tex.append(np.full(len(f), t, np.int64) if np.isscalar(t) else t)
        base += len(p)
    return (np.concatenate(pos).astype(np.float32), np.concatenate(uv).astype(np.float32),
            np.concatenate(idx).astype(np.uint32), np.concatenate(tex).astype(np.uint16))


def _planar_uv(v: np.ndarray, scale: float, rng: np.random.Generator) -> np.ndarray:
    a = rng.uniform(0, 2 * math.pi)
    d1 = np.array([math.cos(a), math.sin(a) * 0.6, 0.45])
    d2 = np.array([-math.sin(a) * 0.5, math.cos(a), 0.35])
    return np.stack([v @ d1, v @ d2], axis=1) * scale + rng.uniform(0, 1, 2)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class ViewParams:
    """Light-field camera rig: V views (rendered as V*S sub-views) of W x H."""
    V: int
    W: int
    H: int
    fovy_deg: float
    aspect: float           # panel aspect: view pixels are `aspect` times wider than tall
    D: float                # focal (zero-disparity) distance
    cone_deg: float         # full horizontal viewing cone
    znear: float
    S: int = 1              # angular supersampling factor
    jitter: Optional[np.ndarray] = None  # (V*S,) float32 in [-0.5, 0.5), random angles inside view intervals
    mip: bool = True        # multiview mipmapping on/off

    @property
    def n_rendered(self) -> int:
        return self.V * self.S


@dataclasses.dataclass
class LensParams:
    """Tilted lenticular panel: Wp x Hp RGB pixels."""
    Wp: int
    Hp: int
    pitch_subpx: float      # lens pitch in subpixels
    slope: float            # horizontal lens shift in pixels per pixel row
    offset: float = 0.0     # lens phase offset (fraction of a lens)
    mode: int = 0           # 0 none, 1 spatial, 2 angular, 3 angular+spatial
    taps: Optional[np.ndarray] = None  # (8, 3) int64: du (Q32 views), dx, dy (Q8 px)


RECON_NONE, RECON_SPATIAL, RECON_ANGULAR, RECON_BOTH = 0, 1, 2, 3


def gaussian_taps(seed: int, n: int = 8, sigma_u: float = 0.5, trunc_u: float = 1.0,
                  sigma_s: float = 0.5625, trunc_s: float = 1.125) -> np.ndarray:
    """8 random Gaussian reconstruction samples (Sec. 4: spatial diameter 2.25 px,
    angular support of 2 view intervals), drawn once per run and quantised:
    du in Q32 of a view interval, dx/dy in Q8 view pixels."""
    rng = np.random.default_rng(seed)
    out = np.zeros((n, 3), np.int64)
    k = 0
    while k < n:
        du = rng.normal(0.0, sigma_u)
        dx, dy = rng.normal(0.0, sigma_s, 2)
        if abs(du) >= trunc_u or dx * dx + dy * dy >= trunc_s * trunc_s:
            continue
        out[k] = (int(round(du * 2.0 ** 32)), int(round(dx * 256.0)), int(round(dy * 256.0)))
        k += 1
    return out


def subview_jitter(seed: int, n: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.random(n) - 0.5).astype(np.float32)


def model_matrix(frame: int, D: float, tilt_deg: float = 0.0, period: int = 1000) -> np.ndarray:
    """3x4 float32 camera-from-scene matrix: the scene turns about its vertical
    axis by 2*pi*frame/period (Sec. 5.1: scenes rotate about their centres),
    after a fixed tilt about X, and sits at depth D in front of the rig."""
    th = 2.0 * math.pi * frame / period
    c, s = math.cos(th), math.sin(th)
    ry = np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    a = math.radians(tilt_deg)
    ca, sa = math.cos(a), math.sin(a)
    rx = np.array([[1, 0, 0], [0, ca, -sa], [0, sa, ca]])
    r = ry @ rx
    m = np.zeros((3, 4))
    m[:, :3] = r
    m[:, 3] = (0.0, 0.0, D)
    return m.astype(np.float32)


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    views: ViewParams
    lens: LensParams
    tilt_deg: float = 0.0
    shading: Optional["Shading"] = None

    def model(self, frame: int) -> np.ndarray:
        return model_matrix(frame, self.views.D, self.tilt_deg)


SHADE_UNLIT, SHADE_PBR = 0, 1


@dataclasses.dataclass
class Shading:
    """Splat shading: unlit albedo, or physically based with one directional
    light plus ambient (camera space; light_dir points towards the light)."""
    mode: int = SHADE_UNLIT
    light_dir: Tuple[float, float, float] = (0.0, 0.0, -1.0)
    light_rgb: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    ambient_rgb: Tuple[float, float, float] = (0.0, 0.0, 0.0)


def default_light() -> Shading:
    d = np.array([0.35, -0.55, -0.75])
    d = (d / np.linalg.norm(d)).astype(np.float32)
    return Shading(SHADE_PBR, tuple(float(x) for x in d), (3.0, 2.9, 2.7), (0.12, 0.13, 0.15))


def with_pbr(w: Workload, seed: int = 0, n_mat: int = 4, normal_scale: int = 2) -> Workload:
    """PBR variant of a workload (Sec. 3.3 with albedo, roughness, metallic and
    normal textures): n_mat material sets, chosen by albedo texture id mod
    n_mat.  Set m has a normal map of normal_scale x the largest albedo size
    for even m and 1x for odd m, roughness at half and metallic at a quarter of
    that size, so Eq. 1's maximum and the per-texture LODs differ from the
    unlit scene."""
    rng = np.random.default_rng(seed + 900)
    sc = w.scene
    base = max(t.shape[0] for t in sc.textures)
    textures = list(sc.textures)
    sets = []
    for m in range(n_mat):
        sn = base * (normal_scale if m % 2 == 0 else 1)
        ids = []
        for tex in (normal_map_texture(sn, rng), scalar_texture(max(1, sn // 2), rng, 0.15, 0.95),
                    metallic_texture(max(1, sn // 4), rng)):
            ids.append(len(textures))
            textures.append(tex)
        sets.append(ids)
    sets = np.asarray(sets, np.uint16)
    mats = sets[sc.tex.astype(np.int64) % n_mat]
    scene = dataclasses.replace(sc, textures=textures, materials=np.ascontiguousarray(mats, np.uint16),
                                name=sc.name + "-pbr").check()
    return dataclasses.replace(w, name=w.name + "-pbr", scene=scene, shading=default_light())


def tiny(seed: int = 1, V: int = 8, size: int = 128, S: int = 1) -> Workload:
    """Icosphere level 3 (1,280 triangles), vertices jittered +-1% of the radius,
    one 256^2 value-noise texture; V horizontal views over a 40 degree cone,
    panel 512^2 with lens pitch 8 subpixels and slope 0.2."""
    rng = np.random.default_rng(seed)
    v, f = icosphere(3)
    R = 1.0
    v = v * R + rng.uniform(-0.01 * R, 0.01 * R, v.shape)
    uv = _planar_uv(v, 1.3, rng)
    tex = [value_noise_texture(256, rng)]
    pos, uvs, idx, tid = _combine([(v, uv, f, 0)])
    scene = Scene(pos, uvs, idx, tid, tex, "icosphere3").check()
    views = ViewParams(V=V, W=size, H=size, fovy_deg=45.0, aspect=1.0, D=3.0 * R,
                       cone_deg=40.0, znear=0.1, S=S,
                       jitter=subview_jitter(seed + 100, V * S) if S > 1 else None)
    lens = LensParams(Wp=512, Hp=512, pitch_subpx=8.0, slope=0.2, offset=0.0,
                      mode=RECON_NONE, taps=gaussian_taps(seed + 200))
    return Workload("tiny-icosphere", scene, views, lens, tilt_deg=0.0)


def display_scene(seed: int = 2, hf_quads: int = 512, levels=(4, 3), counts=(57, 143),
                  tex_size: int = 2048, n_tex: int = 16, name: str = "display") -> Scene:
    """Heightfield of hf_quads^2 quads (fBm heights) plus instanced icospheres at
    random poses, with n_tex RGBA8 textures (half value noise, half checkers).
    Defaults give 999,168 triangles (512^2 quads, 57 level-4 + 143 level-3 spheres)."""
    rng = np.random.default_rng(seed)
    textures = []
    for k in range(n_tex):
        textures.append(value_noise_texture(tex_size, rng) if k % 2 == 0 else checker_texture(tex_size, rng))
    parts = []
    # heightfield: 12 x 12 units, tilted back so it recedes from 0.5D to 1.5D
    hv, hf = heightfield(hf_quads, rng, amp=0.08)
    half = 6.0
    hpos = hv * np.array([half, half, half])
    hpos[:, 1] += 0.0
    uv_scale = 2.0 ** rng.uniform(0.0, 3.0)
    huv = np.stack([hv[:, 0], hv[:, 1]], axis=1) * uv_scale
    parts.append((hpos, huv, hf, 0))
    # spheres above the heightfield (towards the camera, -z in scene space)
    base = {lvl: icosphere(lvl) for lvl in set(levels)}
    for lvl, cnt in zip(levels, counts):
        sv, sf = base[lvl]
        edge = 2.4 / (2 ** lvl)  # rough unit-sphere edge length
        for _ in range(cnt):
            # radius log-uniform so projected edges span ~0.2-50 px at depth ~D
            r = math.exp(rng.uniform(math.log(0.02), math.log(1.6 if lvl <= 3 else 2.4)))
            c = np.array([rng.uniform(-4.5, 4.5), rng.uniform(-4.5, 4.5), -rng.uniform(0.2, 3.5) - r])
            q = rng.standard_normal(4)
            q /= np.linalg.norm(q)
            w, x, y, z = q
            rot = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
            p = (sv @ rot.T) * r + c
            uv = _planar_uv(sv, 2.0 ** rng.uniform(-1.0, 3.0) * (1.0 + 0 * edge), rng)
            parts.append((p, uv, sf, int(rng.integers(0, n_tex))))
    pos, uvs, idx, tid = _combine(parts)
    return Scene(pos, uvs, idx, tid, textures, name).check()


def display(seed: int = 2, S: int = 1, V: int = 48, W: int = 512, H: int = 512,
            hf_quads: int = 512, levels=(4, 3), counts=(57, 143), tex_size: int = 2048,
            n_tex: int = 16, cone_deg: float = 40.0, mode: int = RECON_NONE) -> Workload:
    """Display-size workload: ~1M triangles, 16 2048^2 textures, V=48 views of
    512^2, 2560x1600 tilted-lenticular panel (prototype lens: pitch 0.72 mm at
    0.03 mm subpixels over 479.36 lenses per 3840 px, tilt -9.66 degrees)."""
    scene = display_scene(seed, hf_quads, levels, counts, tex_size, n_tex)
    D = 10.0
    views = ViewParams(V=V, W=W, H=H, fovy_deg=30.0, aspect=1.6, D=D, cone_deg=cone_deg,
                       znear=0.5, S=S, jitter=subview_jitter(seed + 100, V * S) if S > 1 else None)
    pitch = 3.0 * 3840.0 / 479.36
    lens = LensParams(Wp=2560, Hp=1600, pitch_subpx=pitch, slope=-math.tan(math.radians(9.66)),
                      offset=0.0, mode=mode, taps=gaussian_taps(seed + 200))
    return Workload("display-1M", scene, views, lens, tilt_deg=-55.0)


def display_4m(seed: int = 3, S: int = 4) -> Workload:
    """Same family with one more subdivision: 1024^2 quads + 57 level-5 + 143
    level-4 spheres = 3,996,672 triangles; 4x angular supersampling (192 views)."""
    w = display(seed=seed, S=S, hf_quads=1024, levels=(5, 4), counts=(57, 143))
    w.name = "display-4M-ss4"
    return w


def spatial_ss(w: Workload, factor: int = 2, seed: int = 0) -> Workload:
    """Spatial supersampling of a workload (Table 2 "Spatial"): views rendered
    at `factor` times the resolution, and the panel reconstructed with the
    spatial Gaussian taps, whose footprint stays 2.25 pixels of the original
    views (so `factor` times as many rendered pixels)."""
    v = w.views
    views = dataclasses.replace(v, W=v.W * factor, H=v.H * factor)
    taps = gaussian_taps(seed + 300, sigma_s=0.5625 * factor, trunc_s=1.125 * factor)
    lens = dataclasses.replace(w.lens, mode=RECON_SPATIAL, taps=taps)
    out = dataclasses.replace(w, views=views, lens=lens)
    out.name = f"{w.name}-spatial{factor}x"
    return out


def direct_panel_lens(w: Workload, seed: int = 0, mode: int = RECON_ANGULAR) -> LensParams:
    """Lens for reconstructing the panel directly from the S*V sub-views of an
    angularly supersampled workload (Sec. 4, instead of filtering down to V
    views first): the sub-views are taken at their nominal positions and the
    angular taps span +-1 original view interval, i.e. +-S sub-view intervals."""
    S = w.views.S
    taps = gaussian_taps(seed + 400, sigma_u=0.5 * S, trunc_u=1.0 * S)
    return dataclasses.replace(w.lens, mode=mode, taps=taps)


def small_display(seed: int = 7, S: int = 1, V: int = 12, W: int = 96, H: int = 96,
                  hf_quads: int = 48, tex_size: int = 128) -> Workload:
    """A small member of the display family (same geometry kinds, anisotropic
    pixels, lenticular panel) that the oracle finishes in seconds."""
    w = display(seed=seed, S=S, V=V, W=W, H=H, hf_quads=hf_quads, levels=(2, 1), counts=(6, 10),
                tex_size=tex_size, n_tex=4)
    w.lens = LensParams(Wp=320, Hp=200, pitch_subpx=w.lens.pitch_subpx, slope=w.lens.slope,
                        offset=0.13, mode=RECON_NONE, taps=w.lens.taps)
    w.name = "small-display"
    return w


def edge_length_px_stats(scene: Scene, model: np.ndarray, fx: float, fy: float) -> np.ndarray:
    """Approximate projected edge lengths (px) for histogram checks of a workload."""
    p = scene.pos.astype(np.float64) @ model[:, :3].T.astype(np.float64) + model[:, 3]
    q = np.stack([p[:, 0] / p[:, 2] * fx, p[:, 1] / p[:, 2] * fy], axis=1)
    e = q[scene.idx[:, 1]] - q[scene.idx[:, 0]]
    return np.hypot(e[:, 0], e[:, 1])


def batch_workloads(seed: int = 400, n: int = 16, lo: float = 5e4, hi: float = 4e6, n_tex: int = 4) -> List[Workload]:
    """n independent display-family scenes for one batch: triangle counts
    log-uniform in [lo, hi] (half heightfield, half icospheres), textures of
    512^2..2048^2, per-scene view cones 30-50 degrees, V = 48 views of 512^2."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        target = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        quads = max(8, int(round(math.sqrt(target / 4.0))))       # heightfield: 2*quads^2 ~ target/2
        per_sphere = max(20.0, (target - 2 * quads * quads) / 200.0)
        la = max(0, min(5, int(math.floor(math.log(per_sphere / 20.0, 4)))))
        lb = min(la + 1, 6)
        ta, tb = 20 * 4 ** la, 20 * 4 ** lb
        cb = int(round(200 * min(1.0, max(0.0, (per_sphere - ta) / (tb - ta)))))
        tex_size = int(2 ** rng.integers(9, 12))
        w = display(seed=seed + k, hf_quads=quads, levels=(lb, la), counts=(cb, 200 - cb), tex_size=tex_size,
                    n_tex=n_tex, cone_deg=float(rng.uniform(30.0, 50.0)))
        w.name = f"batch-{k}"
        out.append(w)
    return out
