"""Pins of the CPU oracle against facts that do not come from the oracle itself:
exact rational geometry, textbook routines, closed forms, ray casting in
double, the paper's printed constants, and invariants of the method."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_19901_amd import scenes

GOLD = os.path.join(os.path.dirname(__file__), "golden")
IDENT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float32)


def one_tri_scene(P, uv, tex_size=64, tex=None):
    rng = np.random.default_rng(5)
    t = tex if tex is not None else scenes.value_noise_texture(tex_size, rng)
    return scenes.Scene(np.asarray(P, np.float32), np.asarray(uv, np.float32),
                        np.array([[0, 1, 2]], np.uint32), np.zeros(1, np.uint16), [t]).check()


def rig(V=8, W=64, H=64, aspect=1.0, D=4.0, cone=40.0, fovy=40.0, S=1, mip=True, jitter=None):
    return scenes.ViewParams(V=V, W=W, H=H, fovy_deg=fovy, aspect=aspect, D=D, cone_deg=cone, znear=0.1, S=S,
                             jitter=jitter, mip=mip)


# ---------------------------------------------------------------------------
# textures (Sec. 3.3: the hardware mipmap the fragment stage fetches from)


def test_mip_chain_is_rounded_box_mean():
    rng = np.random.default_rng(0)
    t = rng.integers(0, 256, (32, 32, 4), dtype=np.uint8)
    sc = scenes.Scene(np.zeros((3, 3), np.float32), np.zeros((3, 2), np.float32), np.array([[0, 1, 2]], np.uint32),
                      np.zeros(1, np.uint16), [t])
    tx = O.build_textures(sc)
    lvl = t.astype(np.int64)
    for k in range(1, 6):
        s = lvl.shape[0] // 2
        lvl = (lvl.reshape(s, 2, s, 2, 4).sum(axis=(1, 3)) + 2) >> 2
        assert np.array_equal(tx.level(0, k), lvl.astype(np.uint8))


def test_trilinear_special_cases():
    rng = np.random.default_rng(1)
    t = rng.integers(0, 256, (16, 16, 4), dtype=np.uint8)
    sc = scenes.Scene(np.zeros((3, 3), np.float32), np.zeros((3, 2), np.float32), np.array([[0, 1, 2]], np.uint32),
                      np.zeros(1, np.uint16), [t, scenes.constant_texture(16, (10, 200, 30, 255))])
    tx = O.build_textures(sc)
    # texel centres at level 0 return the texel itself
    for (x, y) in [(0, 0), (3, 7), (15, 15), (8, 1)]:
        got = O.trilinear(tx, 0, (x + 0.5) / 16, (y + 0.5) / 16, 0)
        assert got == int(t[y, x].view(np.uint32)[0])
    # wrap addressing: u + 1 samples the same place
    assert O.trilinear(tx, 0, 3.5 / 16 + 1.0, 7.5 / 16 - 2.0, 0) == int(t[7, 3].view(np.uint32)[0])
    # midpoint between two texels = rounded mean
    got = np.frombuffer(np.uint32(O.trilinear(tx, 0, 4.0 / 16, 2.5 / 16, 0)).tobytes(), np.uint8)
    want = (t[2, 3].astype(int) + t[2, 4].astype(int) + 1) // 2
    assert np.array_equal(got, want)
    # a constant texture is constant at every position and level of detail
    for kc in (0, 100, 256, 3 * 256 + 17, 4 * 256):
        for u, v in [(0.1, 0.9), (-3.3, 7.25), (0.5, 0.5)]:
            assert O.trilinear(tx, 1, u, v, kc) == int(np.array([10, 200, 30, 255], np.uint8).view(np.uint32)[0])
    # level of detail exactly on level 1: equals the level-1 texel at its centre
    l1 = tx.level(0, 1)
    assert O.trilinear(tx, 0, 2.5 / 8, 5.5 / 8, 256) == int(l1[5, 2].view(np.uint32)[0])


def test_lod_units():
    # Eqs. 6-7: LOD = 0.5 log2(size * X * Y); quantised to 1/256 level
    for m in range(-6, 12):
        assert O.lod_q8(4.0 ** m) == 256 * m
    assert O.lod_q8(2.0) == 128
    assert O.lod_q8(0.0) < -10 ** 6


# ---------------------------------------------------------------------------
# closest point (Fig. 4: pixel edges are reverse-projected around the point of
# the polygon closest to the eye)


def test_closest_point_matches_brute_force():
    rng = np.random.default_rng(2)
    g = np.linspace(0, 1, 401)
    B1, B2 = np.meshgrid(g, g)
    m = (B1 + B2) <= 1
    b1, b2 = B1[m], B2[m]
    for _ in range(60):
        a, b, c, p = (rng.normal(0, 1, 3) for _ in range(4))
        q = O.closest_point(p, a, b, c).astype(np.float64)
        pts = a[None] + b1[:, None] * (b - a)[None] + b2[:, None] * (c - a)[None]
        d = np.linalg.norm(pts - p[None], axis=1)
        best = pts[np.argmin(d)]
        assert np.linalg.norm(q - p) <= d.min() + 1e-5
        assert np.linalg.norm(q - best) < 0.02 * (1 + np.linalg.norm(b - a) + np.linalg.norm(c - a))
        # on the triangle: barycentrics in [0,1]
        M = np.stack([b - a, c - a], axis=1)
        sol, *_ = np.linalg.lstsq(M, q - a, rcond=None)
        assert sol.min() > -1e-4 and sol.sum() < 1 + 1e-4


# ---------------------------------------------------------------------------
# lattice emission (point generation of the aligned triangle)


def _clip_area(poly, x0, x1, y0, y1):
    def clip(pts, inside, inter):
        out = []
        for k in range(len(pts)):
            a, b = pts[k - 1], pts[k]
            ia, ib = inside(a), inside(b)
            if ib:
                if not ia:
                    out.append(inter(a, b))
                out.append(b)
            elif ia:
                out.append(inter(a, b))
        return out

    def ix(xc):
        return lambda a, b: (xc, a[1] + (b[1] - a[1]) * (xc - a[0]) / (b[0] - a[0]))

    def iy(yc):
        return lambda a, b: (a[0] + (b[0] - a[0]) * (yc - a[1]) / (b[1] - a[1]), yc)

    pts = list(poly)
    for inside, inter in [(lambda p: p[0] >= x0, ix(x0)), (lambda p: p[0] <= x1, ix(x1)),
                          (lambda p: p[1] >= y0, iy(y0)), (lambda p: p[1] <= y1, iy(y1))]:
        pts = clip(pts, inside, inter)
        if not pts:
            return Fraction(0)
    a = Fraction(0)
    for k in range(len(pts)):
        a += pts[k - 1][0] * pts[k][1] - pts[k][0] * pts[k - 1][1]
    return abs(a) / 2


def _exact_cells(S, T):
    poly = [(Fraction(int(S[k]), 256), Fraction(int(T[k]), 256)) for k in range(3)]
    eps = Fraction(4, 256)
    out = []
    lo_i, hi_i = math.floor(min(S) / 256) - 2, math.floor(max(S) / 256) + 2
    lo_j, hi_j = math.floor(min(T) / 256) - 2, math.floor(max(T) / 256) + 2
    for j in range(lo_j, hi_j + 1):
        for i in range(lo_i, hi_i + 1):
            if _clip_area(poly, i - eps, i + 1 + eps, j - eps, j + 1 + eps) > 0:
                out.append((i, j))
    return out


def _exact_cells_degenerate(S, T):
    """A snapped lattice triangle of zero area (a point or a segment) keeps the
    cells whose eps-dilated open box meets the closed bounding box of its
    vertices (exact rationals)."""
    eps = Fraction(4, 256)
    s0, s1 = Fraction(min(S), 256), Fraction(max(S), 256)
    t0, t1 = Fraction(min(T), 256), Fraction(max(T), 256)
    out = []
    for j in range(math.floor(t0) - 2, math.floor(t1) + 3):
        for i in range(math.floor(s0) - 2, math.floor(s1) + 3):
            if i - eps < s1 and i + 1 + eps > s0 and j - eps < t1 and j + 1 + eps > t0:
                out.append((i, j))
    return out


def test_lattice_cells_equal_exact_rational_clipping():
    rng = np.random.default_rng(3)
    n_checked = 0
    for k in range(220):
        kind = k % 4
        if kind == 0:   # tiny triangles near vertex 0 at (128,128)
            S = [128] + list(rng.integers(-300, 600, 2))
            T = [128] + list(rng.integers(-300, 600, 2))
        elif kind == 1:  # slivers
            d = rng.integers(-2000, 2000, 2)
            S = [128, 128 + int(d[0]), 128 + int(d[0]) // 2 + int(rng.integers(-3, 4))]
            T = [128, 128 + int(d[1]), 128 + int(d[1]) // 2 + int(rng.integers(-3, 4))]
        elif kind == 2:  # vertices on cell boundaries / dilation edges
            S = [128] + list(256 * rng.integers(-3, 4, 2) + rng.choice([-4, 0, 4, 252, 256, 260], 2))
            T = [128] + list(256 * rng.integers(-3, 4, 2) + rng.choice([-4, 0, 4, 252, 256, 260], 2))
        else:            # medium
            S = [128] + list(rng.integers(-1500, 1500, 2))
            T = [128] + list(rng.integers(-1500, 1500, 2))
        area2 = (S[1] - S[0]) * (T[2] - T[0]) - (T[1] - T[0]) * (S[2] - S[0])
        ci, cj = O.lattice_cells(S, T)
        got = list(zip(ci.tolist(), cj.tolist()))
        want = _exact_cells(S, T) if area2 != 0 else _exact_cells_degenerate(S, T)
        assert got == want, (S, T)
        n_checked += 1
    assert n_checked == 220


def test_degenerate_lattice_keeps_the_cells_along_it():
    """Zero-area snapped lattices (Sec. 3.2: splats must leave no holes, so a
    visible triangle never emits nothing): a point keeps exactly the cell that
    holds it, a segment the cells along its bounding box, each cell once and
    covering the segment."""
    cases = [([128, 128, 128], [128, 128, 128], [(0, 0)]),
             ([128, 128, 128], [128, 127, 129], [(0, 0)]),
             ([128, 151, 141], [128, 128, 128], [(0, 0)]),
             ([128, 600, 1000], [128, 128, 128], [(0, 0), (1, 0), (2, 0), (3, 0)]),
             ([128, 128, 128], [128, -300, -700], [(0, -3), (0, -2), (0, -1), (0, 0)])]
    for S, T, want in cases:
        ci, cj = O.lattice_cells(S, T)
        got = list(zip(ci.tolist(), cj.tolist()))
        assert got == want, (S, T)
    # a diagonal segment: every point on it lies in an emitted cell
    S, T = [128, 1280, 2432], [128, 704, 1280]
    ci, cj = O.lattice_cells(S, T)
    cells = set(zip(ci.tolist(), cj.tolist()))
    assert len(cells) == len(ci)
    for k in range(0, 1001):
        s = Fraction(128, 256) + Fraction(k, 1000) * Fraction(2432 - 128, 256)
        t = Fraction(128, 256) + Fraction(k, 1000) * Fraction(1280 - 128, 256)
        assert any(i <= s <= i + 1 and j <= t <= j + 1 for i, j in cells)


def test_lattice_right_triangle_golden():
    d = json.load(open(os.path.join(GOLD, "lattice_right_triangle.json")))
    for c in d["cases"]:
        a, b = c["a"], c["b"]
        ci, cj = O.lattice_cells([128, 128 + 256 * a, 128], [128, 128, 128 + 256 * b])
        assert len(ci) == c["count"]
        if "rows" in c:
            assert [int((cj == j).sum()) for j in range(len(c["rows"]))] == c["rows"]


# ---------------------------------------------------------------------------
# sampling densities (Sec. 3.1): LFD-biased H/V densities from reverse-projected
# pixel edges, texture-based coarsening (Eqs. 1-3), mip setup (Eqs. 4-7)


def _active_views_double(P, vt, vp):
    """Views that see the triangle, computed independently in double."""
    P = np.asarray(P, np.float64)
    n = np.cross(P[1] - P[0], P[2] - P[0])
    act = []
    nh = n / np.linalg.norm(n)
    for r, b in enumerate(vt["eye"].astype(np.float64)):
        e = np.array([b, 0, 0])
        # front facing, and the eye direction at least asin(1/256) off the plane
        if np.dot(nh, e - P[0]) < np.linalg.norm(e - P[0]) / 256.0:
            act.append(False)
            continue
        x = vt["cx"] + vt["fx"] * ((P[:, 0] - b) / P[:, 2] + b / vp.D)
        y = vt["cy"] + vt["fy"] * P[:, 1] / P[:, 2]
        act.append(not ((x < 0).all() or (x > vp.W).all() or (y < 0).all() or (y > vp.H).all()))
    return np.array(act)


def _ray_hit(px, py, b, vt, vp, P0, n):
    d = np.array([(px - float(vt["cx"])) / float(vt["fx"]) - b / vp.D, (py - float(vt["cy"])) / float(vt["fy"]), 1.0])
    e = np.array([b, 0.0, 0.0])
    t = np.dot(n, P0 - e) / np.dot(n, d)
    return e + t * d


def test_density_from_reverse_projected_pixel_edges():
    """Sx, Sy, size_xy equal what ray casting the pixel edges around the
    closest point gives (double precision geometry, no closed form)."""
    rng = np.random.default_rng(4)
    vp = rig(V=8, W=64, H=48, aspect=1.6, D=4.0)
    vt = O.view_table(vp)
    checked = 0
    for _ in range(40):
        c = np.array([rng.uniform(-0.6, 0.6), rng.uniform(-0.4, 0.4), rng.uniform(3.0, 5.0)])
        P = c + rng.normal(0, 0.15, (3, 3))
        n = np.cross(P[1] - P[0], P[2] - P[0])
        if n[2] > 0:
            P = P[[0, 2, 1]]
            n = -n
        act = _active_views_double(P, vt, vp)
        if not act.all():
            continue
        # texture fine enough that Eq. 3 does not coarsen
        sc = one_tri_scene(P, [[0, 0], [1, 0], [0, 1]], tex_size=1024)
        res = O.render(sc, vp, IDENT)
        if res["trii"][0, 6] == 0:
            continue
        Sx, Sy, size_xy = (float(v) for v in res["trif"][0, [0, 1, 6]])
        nn = n / np.linalg.norm(n)
        lx, ly, area = [], [], []
        for r, b in enumerate(vt["eye"].astype(np.float64)):
            Ps = O.closest_point([b, 0, 0], *P.astype(np.float32)).astype(np.float64)
            x = float(vt["cx"]) + float(vt["fx"]) * ((Ps[0] - b) / Ps[2] + b / vp.D)
            y = float(vt["cy"]) + float(vt["fy"]) * Ps[1] / Ps[2]
            h = 1e-3
            X0 = _ray_hit(x, y, b, vt, vp, P[0], nn)
            ax = (_ray_hit(x + h, y, b, vt, vp, P[0], nn) - X0) / h
            ay = (_ray_hit(x, y + h, b, vt, vp, P[0], nn) - X0) / h
            lx.append(np.linalg.norm(ax))
            ly.append(np.linalg.norm(ay))
            area.append(np.linalg.norm(np.cross(ax, ay)))
        Ats = 0.5
        Aws = 0.5 * np.linalg.norm(n)
        size_uv = Aws / (Ats * 1024 * 1024)
        f = math.sqrt(min(area) / size_uv) if size_uv > min(area) else 1.0
        assert Sx == pytest.approx(f / min(lx), rel=2e-3)
        assert Sy == pytest.approx(f / min(ly), rel=2e-3)
        assert size_xy == pytest.approx(min(area), rel=2e-3)
        checked += 1
    assert checked >= 10


def test_lfd_bias_halves_horizontal_density():
    """Pixels `aspect` times wider than tall: horizontal density drops by the
    aspect ratio, vertical density does not (Sec. 3.1)."""
    P = [[-0.3, -0.3, 4.0], [0.3, -0.3, 4.0], [-0.3, 0.3, 4.0]]
    if np.cross(np.subtract(P[1], P[0]), np.subtract(P[2], P[0]))[2] > 0:
        P = [P[0], P[2], P[1]]
    sc = one_tri_scene(P, [[0, 0], [4, 0], [0, 4]], tex_size=1024)
    r1 = O.render(sc, rig(aspect=1.0, W=64, H=64), IDENT)
    r2 = O.render(sc, rig(aspect=1.6, W=64, H=64), IDENT)
    assert r2["trif"][0, 0] / r1["trif"][0, 0] == pytest.approx(1 / 1.6, rel=1e-5)
    assert r2["trif"][0, 1] == pytest.approx(r1["trif"][0, 1], rel=1e-6)
    assert r2["count"][0] / r1["count"][0] == pytest.approx(1 / 1.6, rel=0.08)


def test_texture_based_density_matches_texel_count():
    """Eqs. 1-3: with a coarse texture the cell count in the triangle's area
    equals the texel count it spans."""
    P = [[-0.5, -0.5, 4.0], [0.5, -0.5, 4.0], [-0.5, 0.5, 4.0]]
    if np.cross(np.subtract(P[1], P[0]), np.subtract(P[2], P[0]))[2] > 0:
        P = [P[0], P[2], P[1]]
    X = 16
    sc = one_tri_scene(P, [[0, 0], [0.5, 0], [0, 0.5]], tex_size=X)
    res = O.render(sc, rig(W=128, H=128, aspect=1.0), IDENT)
    Sx, Sy = (float(v) for v in res["trif"][0, :2])
    Aws = 0.5 * 1.0
    n_tex = 0.5 * 0.25 * X * X
    assert Sx * Sy * Aws == pytest.approx(n_tex, rel=1e-4)
    # the emitted count is the texel count plus the conservative boundary ring
    assert n_tex <= res["count"][0] <= 4 * n_tex + 12


def _footprint(X, b, vt, vp, nh, h=1e-2):
    """Area on the plane (unit normal nh through X) of the pixel around X's
    projection in the view with eye offset b, by casting rays through the
    pixel's neighbourhood (central differences), double precision."""
    x = float(vt["cx"]) + float(vt["fx"]) * ((X[0] - b) / X[2] + b / vp.D)
    y = float(vt["cy"]) + float(vt["fy"]) * X[1] / X[2]
    ax = (_ray_hit(x + h, y, b, vt, vp, X, nh) - _ray_hit(x - h, y, b, vt, vp, X, nh)) / (2 * h)
    ay = (_ray_hit(x, y + h, b, vt, vp, X, nh) - _ray_hit(x, y - h, b, vt, vp, X, nh)) / (2 * h)
    return float(np.linalg.norm(np.cross(ax, ay)))


def _random_texture(size, seed=0):
    t = np.random.default_rng(seed).integers(0, 256, (size, size, 4), dtype=np.uint8)
    t[..., 3] = 255
    return t


TILTED = np.array([[-0.8, -0.6, 3.0], [-0.3, 0.8, 4.2], [0.9, -0.5, 5.5]])


def _check_eq8_eq9(tex_size):
    """Per (point, view): Eqs. 8-9 evaluated in double from ray-cast geometry
    against the oracle's quantised weight tq and splat colour.  Returns the
    number of pairs checked and how many took each branch of Eq. 8."""
    P = TILTED
    n = np.cross(P[1] - P[0], P[2] - P[0])
    assert n[2] < 0
    uv = np.array([[0.0, 0.0], [0.0, 1.0], [1.0, 0.0]])
    sc = one_tri_scene(P, uv, tex=_random_texture(tex_size))
    vp = rig(V=8, W=64, H=64, aspect=1.6, D=4.0)
    vt = O.view_table(vp)
    r = O.render(sc, vp, IDENT, observe=True)
    Sx, Sy, smin_o, smax_o = (float(v) for v in r["trif"][0, :4])
    nh = n / np.linalg.norm(n)
    Ats = 0.5 * abs((uv[1, 0] - uv[0, 0]) * (uv[2, 1] - uv[0, 1]) - (uv[1, 1] - uv[0, 1]) * (uv[2, 0] - uv[0, 0]))
    ruv = Ats / (0.5 * np.linalg.norm(n))
    eyes = vt["eye"].astype(np.float64)
    act = _active_views_double(P, vt, vp)
    # Eqs. 4-5: extremes of the pixel footprint over the vertices and active views
    foot = [_footprint(P[k], eyes[v], vt, vp, nh) for k in range(3) for v in range(len(eyes)) if act[v]]
    smin, smax = min(foot) * ruv, max(foot) * ruv
    assert smin_o == pytest.approx(smin, rel=1e-4) and smax_o == pytest.approx(smax, rel=1e-4)
    # lattice axes: camera X projected into the plane, and n x u
    u = np.array([1.0, 0.0, 0.0]) - nh * nh[0]
    u /= np.linalg.norm(u)
    w = np.cross(nh, u)
    Acell = 1.0 / (Sx * Sy)
    suv = Acell * ruv
    pts = r["points"]
    tq_o, col_o = r["pv_tq"], r["pv_col"]
    checked, branch = 0, [0, 0]
    for p, v in zip(*np.nonzero(tq_o >= 0)):
        Xc = P[0] + (int(pts["i"][p]) / Sx) * u + (int(pts["j"][p]) / Sy) * w   # cell centre
        av = Acell / _footprint(Xc, eyes[v], vt, vp, nh)    # splat size in view pixels
        vse = suv / min(1.0, av)                             # Eq. 8
        vs = min(max(vse, smin), smax)
        tau = (vs - smin) / (smax - smin)                    # Eq. 9
        tq = min(max(math.floor(256 * tau + 0.5), 0), 256)
        assert abs(int(tq_o[p, v]) - tq) <= 1, (p, v, int(tq_o[p, v]), tq)
        lo = np.frombuffer(np.uint32(pts["tvmin"][p]).tobytes(), np.uint8).astype(float)
        hi = np.frombuffer(np.uint32(pts["tvmax"][p]).tobytes(), np.uint8).astype(float)
        got = np.frombuffer(np.uint32(col_o[p, v]).tobytes(), np.uint8).astype(float)
        assert np.abs(got - np.floor(lo + (hi - lo) * tau + 0.5)).max() <= 1, (p, v, got, lo, hi, tau)
        branch[int(av >= 1.0)] += 1
        checked += 1
    # every written pixel carries the colour of one of the point-views of its view
    for v in range(len(eyes)):
        cols = set(col_o[tq_o[:, v] >= 0, v].tolist())
        drawn = r["rgba"][v][np.isfinite(r["depth"][v])]
        assert set(drawn.tolist()) <= cols
    return checked, branch, tq_o[tq_o >= 0]


def test_eq8_eq9_interpolation_weight_on_a_tilted_triangle():
    """Eqs. 8-9 (multiview mipmapping: per view, the splat's texture footprint
    picks a blend between the triangle's finest and coarsest mip colours).  A
    tilted triangle has smin < smax; with a fine texture the splat is smaller
    than a pixel (Eq. 8 divides by the splat's pixel size), with a coarse one
    (Eq. 3 coarsens the lattice) larger (Eq. 8 keeps the splat's UV area)."""
    n1, b1, tq1 = _check_eq8_eq9(1024)
    assert n1 > 1000 and b1[0] > 0.9 * n1
    assert len(np.unique(tq1)) > 100 and tq1.min() < 16 and tq1.max() > 200
    n2, b2, _ = _check_eq8_eq9(16)
    assert n2 > 500 and b2[1] > 0.5 * n2


def _compile_variant(tmp_path, old, new):
    """The oracle with one planted mistake, compiled into a separate library."""
    import ctypes as C
    import subprocess
    src = open(os.path.join(os.path.dirname(O.__file__), "lfdpr_oracle.c")).read()
    assert old in src
    path = tmp_path / "variant.c"
    path.write_text(src.replace(old, new, 1))
    so = tmp_path / "libvariant.so"
    subprocess.check_call(["gcc", *O.CFLAGS, "-o", str(so), str(path), "-lm"])
    lib = C.CDLL(str(so))
    lib.orc_lattice_cells.restype = C.c_int
    lib.orc_trilinear.restype = C.c_uint32
    lib.orc_lod_q8.restype = C.c_int
    lib.orc_lod_q8.argtypes = [C.c_float]
    return lib


@pytest.mark.parametrize("old,new", [
    ("lerp_rgba8(tvmin[c], tvmax[c], tq)", "lerp_rgba8(tvmax[c], tvmin[c], tq)"),          # tau swapped
    ("float vse = Acell < Ar ?", "float vse = Acell > Ar ?"),                               # Eq. 8 branch
    ("float vs = vse < ts->smin ? ts->smin : (vse > ts->smax ? ts->smax : vse);",
     "float vs = vse < ts->smax ? ts->smax : (vse > ts->smin ? ts->smin : vse);"),         # clamp
    ("float Ar = ((Zc * Zc) * Zc) / (fxfy * ad);", "float Ar = (Zc * Zc) / (fxfy * ad);"),  # footprint
])
def test_eq8_eq9_pin_catches_planted_mistakes(tmp_path, monkeypatch, old, new):
    monkeypatch.setattr(O, "_lib", _compile_variant(tmp_path, old, new))
    with pytest.raises(AssertionError):
        _check_eq8_eq9(1024)
        _check_eq8_eq9(16)


def _rendered_eye_offsets(vp, Z=2.0):
    """Eye offset of every view recovered from the rendered depth of a tilted
    plane at depth ~Z: the pixel ray from eye (b, 0, 0) through pixel x meets
    the plane n.X = h at depth Zp, which fixes b (double precision)."""
    n = np.array([0.35, 0.2, -1.0])
    n /= np.linalg.norm(n)
    c = np.array([0.0, 0.0, Z])
    h = float(np.dot(n, c))
    a = np.cross(n, [0.0, 1.0, 0.0])
    a /= np.linalg.norm(a)
    bb = np.cross(n, a)
    L = 0.6 * Z
    quad = [c - L * a - L * bb, c + L * a - L * bb, c - L * a + L * bb, c + L * a + L * bb]
    P = np.array(quad, np.float32)
    idx = np.array([[0, 1, 2], [1, 3, 2]], np.uint32)
    if np.cross(P[1] - P[0], P[2] - P[0]) @ n < 0:
        idx = idx[:, [0, 2, 1]]
    sc = scenes.Scene(P, np.zeros((4, 2), np.float32), idx, np.zeros(2, np.uint16),
                      [scenes.constant_texture(4, (200, 10, 10, 255))]).check()
    r = O.render(sc, vp, IDENT)
    t = math.tan(math.radians(vp.fovy_deg) / 2.0)
    fx, fy = (vp.W / 2.0) / (vp.aspect * t), (vp.H / 2.0) / t
    out = []
    for v in range(vp.V * vp.S):
        ys, xs = np.nonzero(np.isfinite(r["depth"][v]))
        k = len(xs) // 2
        x, y, Zp = xs[k] + 0.5, ys[k] + 0.5, float(r["depth"][v][ys[k], xs[k]])
        # Zp (n.d) = h - n_x b with d = ((x - W/2)/fx - b/D, (y - H/2)/fy, 1)
        px, py = (x - vp.W / 2.0) / fx, (y - vp.H / 2.0) / fy
        b = (h - Zp * (n[0] * px + n[1] * py + n[2])) / (n[0] * (1.0 - Zp / vp.D))
        out.append(b)
    return np.array(out)


def _check_rig(V=8, D=4.0, cone=40.0):
    vp = rig(V=V, W=96, H=64, aspect=1.6, D=D, cone=cone)
    b = _rendered_eye_offsets(vp)
    half = D * math.tan(math.radians(cone) / 2.0)
    assert np.allclose(np.diff(b), 2.0 * half / V, rtol=2e-4), np.diff(b)     # eye spacing
    assert b[0] == pytest.approx(-half * (1 - 1.0 / V), rel=2e-4)             # outer eyes
    assert b[-1] == pytest.approx(half * (1 - 1.0 / V), rel=2e-4)


def test_rig_eye_offsets_from_rendered_depth():
    """Sec. 3.1/5.1: V parallel eyes spread evenly over the horizontal viewing
    cone, one per view interval at its centre: spacing 2 D tan(cone/2) / V,
    outer eyes at +-D tan(cone/2) (1 - 1/V); recovered from rendered depth."""
    _check_rig(V=8, D=4.0, cone=40.0)
    _check_rig(V=5, D=3.0, cone=30.0)


def test_focal_plane_point_is_in_the_same_pixel_in_every_view():
    """The views share the zero-disparity plane Z = D: a surface on it covers
    the same pixels, at the same depth, in every view."""
    D = 4.0
    P = np.array([[-0.3, -0.25, D], [0.35, -0.2, D], [-0.1, 0.3, D]], np.float32)
    if np.cross(P[1] - P[0], P[2] - P[0])[2] > 0:
        P = P[[0, 2, 1]]
    sc = one_tri_scene(P, [[0, 0], [1, 0], [0, 1]], tex=scenes.constant_texture(4, (1, 2, 3, 255)))
    r = O.render(sc, rig(V=8, W=64, H=48, aspect=1.6, D=D), IDENT)
    cover = np.isfinite(r["depth"])
    assert cover[0].sum() > 30
    assert all(np.array_equal(cover[v], cover[0]) for v in range(8))
    assert np.allclose(r["depth"][cover[0][None].repeat(8, 0)], D, rtol=1e-6)


def test_rig_pin_catches_a_planted_cone_error(monkeypatch):
    real = O.view_table

    def wrong(vp):   # tan(cone) where the rig needs tan(cone/2)
        t = real(vp)
        B, Bw = vp.D * math.tan(math.radians(vp.cone_deg) / 2.0), vp.D * math.tan(math.radians(vp.cone_deg))
        t["eye"] = (t["eye"].astype(np.float64) * (Bw / B)).astype(np.float32)
        t["kshift"] = (t["eye"].astype(np.float64) / vp.D).astype(np.float32)
        return t

    monkeypatch.setattr(O, "view_table", wrong)
    with pytest.raises(AssertionError):
        _check_rig(V=8, D=4.0, cone=40.0)


def test_rig_takes_binary32_parameters():
    """Reading R2: the rig is given by binary32 parameters (as the C ABI holds
    them): a cone, distance, field of view or aspect that is not a binary32
    value gives the tables of its binary32 rounding, and the next binary32
    value gives different eye offsets; the double evaluation uses
    deg * (pi / 180) for the radians."""
    base = rig(V=48, W=512, H=512, aspect=1.6, D=10.0, cone=48.89048503827306, fovy=30.0)
    r32 = rig(V=48, W=512, H=512, aspect=float(np.float32(1.6)), D=10.0,
              cone=float(np.float32(48.89048503827306)), fovy=30.0)
    t, t32 = O.view_table(base), O.view_table(r32)
    for k in ("eye", "kshift", "fx", "fy", "rD"):
        assert np.array_equal(np.asarray(t[k]).view(np.uint32), np.asarray(t32[k]).view(np.uint32)), k
    # the binary32 value above it: one ulp of the cone moves some eyes
    up = rig(V=48, W=512, H=512, aspect=1.6, D=10.0,
             cone=float(np.nextafter(np.float32(48.89048503827306), np.float32(90))), fovy=30.0)
    assert not np.array_equal(O.view_table(up)["eye"], t["eye"])
    # the eye offsets from that definition, written out in double
    c = float(np.float32(48.89048503827306))
    B = 10.0 * math.tan(c * (math.pi / 180.0) / 2.0)
    q = np.arange(48) + 0.5
    assert np.array_equal(t["eye"], (B * (2.0 * q / 48 - 1.0)).astype(np.float32))


def test_multiview_mip_setup_closed_form():
    """Eqs. 4-7 for a fronto-parallel triangle at depth Z: every view's pixel
    footprint on it is Z^2/(fx fy), so size_min = size_max = Z^2/(fx fy) A_ts/A_ws."""
    Z = 4.0
    P = [[-0.2, -0.2, Z], [0.2, -0.2, Z], [-0.2, 0.2, Z]]
    if np.cross(np.subtract(P[1], P[0]), np.subtract(P[2], P[0]))[2] > 0:
        P = [P[0], P[2], P[1]]
    uv = [[0, 0], [2, 0], [0, 2]]
    sc = one_tri_scene(P, uv, tex_size=256)
    vp = rig(W=64, H=64)
    vt = O.view_table(vp)
    res = O.render(sc, vp, IDENT)
    ruv = (0.5 * 4) / (0.5 * 0.16)
    want = Z * Z / (float(vt["fx"]) * float(vt["fy"])) * ruv
    assert res["trif"][0, 2] == pytest.approx(want, rel=1e-5)
    assert res["trif"][0, 3] == pytest.approx(want, rel=1e-5)
    k = int(math.floor(128 * math.log2(want * 256 * 256) + 0.5))
    assert res["trii"][0, 4] == min(max(k, 0), 256 * 8) == res["trii"][0, 5]


# ---------------------------------------------------------------------------
# splatting (Sec. 3.2) against the conventional rasteriser


@pytest.fixture(scope="module")
def tiny():
    w = scenes.tiny()
    tx = O.build_textures(w.scene)
    m = w.model(0)
    return w, tx, O.render(w.scene, w.views, m, tx), O.rasterise(w.scene, w.views, m, tx)


def test_splat_coverage_equals_rasteriser(tiny):
    w, tx, r, (g, gd) = tiny
    assert r["stats"]["orphans"] == 0 and r["stats"]["misses"] == 0
    assert np.array_equal(np.isfinite(r["depth"]), np.isfinite(gd))
    assert r["stats"]["overflow_tris"] == 0


def test_small_display_coverage_and_sanity():
    w = scenes.small_display()
    tx = O.build_textures(w.scene)
    m = w.model(3)
    r = O.render(w.scene, w.views, m, tx)
    g, gd = O.rasterise(w.scene, w.views, m, tx)
    assert r["stats"]["orphans"] == 0 and r["stats"]["misses"] == 0
    assert np.array_equal(np.isfinite(r["depth"]), np.isfinite(gd))
    a = O.unpack_rgba(r["rgba"])[..., :3].astype(np.float64)
    b = O.unpack_rgba(g)[..., :3].astype(np.float64)
    psnr = 10 * np.log10(255.0 ** 2 / ((a - b) ** 2).mean())
    assert psnr > 30.0


def test_constant_textures_reproduce_rasteriser_exactly(tiny):
    w, _, _, _ = tiny
    sc = scenes.Scene(w.scene.pos, w.scene.uv, w.scene.idx, w.scene.tex,
                      [scenes.constant_texture(256, (90, 140, 200, 255))])
    tx = O.build_textures(sc)
    m = w.model(5)
    r = O.render(sc, w.views, m, tx)
    g, _ = O.rasterise(sc, w.views, m, tx)
    assert np.array_equal(r["rgba"], g)


def test_depth_is_nearest_surface(tiny):
    """Where both cover a pixel, the splat depth equals the rasteriser's
    double-precision depth to float rounding (64-bit key holds depth high)."""
    w, tx, r, (g, gd) = tiny
    m = np.isfinite(gd)
    rel = np.abs(r["depth"][m] - gd[m]) / gd[m]
    assert np.quantile(rel, 0.999) < 1e-5


def test_multiview_mipmapping_improves_quality():
    """Fig. 7 ablation: with multiview mipmapping the views are closer to the
    mipmapped rasteriser than without."""
    w = scenes.small_display(seed=11)
    tx = O.build_textures(w.scene)
    m = w.model(0)
    g, _ = O.rasterise(w.scene, w.views, m, tx)
    b = O.unpack_rgba(g)[..., :3].astype(np.float64)
    err = []
    for mip in (True, False):
        w.views.mip = mip
        r = O.render(w.scene, w.views, m, tx)
        a = O.unpack_rgba(r["rgba"])[..., :3].astype(np.float64)
        err.append(((a - b) ** 2).mean())
    w.views.mip = True
    assert err[0] < err[1]


def test_point_counts_follow_density():
    """More views closer/denser sampling: counts scale with the densities."""
    w = scenes.tiny()
    tx = O.build_textures(w.scene)
    r = O.render(w.scene, w.views, w.model(0), tx)
    Sx, Sy = r["trif"][:, 0], r["trif"][:, 1]
    act = r["count"] > 0
    # cells within the lattice triangle area ~ Sx*Sy*A_ws (plus the boundary ring)
    P = w.scene.pos.astype(np.float64)
    idx = w.scene.idx
    Aws = 0.5 * np.linalg.norm(np.cross(P[idx[:, 1]] - P[idx[:, 0]], P[idx[:, 2]] - P[idx[:, 0]]), axis=1)
    inner = Sx.astype(np.float64) * Sy * Aws
    c = r["count"].astype(np.float64)
    assert (c[act] >= np.floor(inner[act]) * 0.999 - 1).all()
    assert np.sum(c[act]) < 2.5 * np.sum(inner[act]) + 8 * act.sum()


# ---------------------------------------------------------------------------
# interleave and reconstruction (Sec. 4)


def _lens(Wp=96, Hp=64, pitch=8.0, slope=0.2, offset=0.0, mode=0, seed=9):
    return scenes.LensParams(Wp=Wp, Hp=Hp, pitch_subpx=pitch, slope=slope, offset=offset, mode=mode,
                             taps=scenes.gaussian_taps(seed))


def test_interleave_reads_out_view_index():
    V, H, W = 8, 16, 24
    views = np.zeros((V, H, W), np.uint32)
    for v in range(V):
        views[v] = v * 0x00010101
    ln = _lens(pitch=8.0, slope=0.0)
    panel = O.interleave(views, ln)
    X = np.arange(ln.Wp)[None, :, None]
    c = np.arange(3)[None, None, :]
    assert np.array_equal(panel, np.broadcast_to((3 * X + c) % V, panel.shape).astype(np.uint8))
    # with a slope the index map follows floor(frac((3X + c - 3 s Y)/P) V)
    ln = _lens(pitch=8.0, slope=0.2)
    panel = O.interleave(views, ln).astype(np.int64)
    Y = np.arange(ln.Hp)[:, None, None]
    ph = ((3 * X + c) - 3 * 0.2 * Y) / 8.0
    frac = (ph - np.floor(ph)) * V
    want = np.floor(frac).astype(np.int64)
    safe = np.abs(frac - np.round(frac)) > 1e-6   # away from phase boundaries
    assert safe.mean() > 0.5
    assert np.array_equal(panel[safe], want[safe])


def test_identical_views_make_panel_lens_independent():
    rng = np.random.default_rng(3)
    one = rng.integers(0, 2 ** 32, (16, 24), dtype=np.uint64).astype(np.uint32)
    views = np.repeat(one[None], 8, axis=0)
    p1 = O.interleave(views, _lens(pitch=8.0, slope=0.2, offset=0.3))
    p2 = O.interleave(views, _lens(pitch=24.03, slope=-0.17, offset=0.0))
    assert np.array_equal(p1, p2)
    for mode in (1, 2, 3):
        q = O.interleave(views, _lens(mode=2))
        assert np.array_equal(q, p1)  # angular-only taps over identical views change nothing


def test_reconstruction_of_constant_views_is_constant():
    views = np.full((6, 16, 24), np.uint32(0xFF204080), np.uint32)
    for mode in (0, 1, 2, 3):
        p = O.interleave(views, _lens(mode=mode))
        assert (p[..., 0] == 0x80).all() and (p[..., 1] == 0x40).all() and (p[..., 2] == 0x20).all()


def test_prototype_lens_constants():
    d = json.load(open(os.path.join(GOLD, "prototype_display.json")))
    pitch_subpx = 3 * d["panel_px"][0] / d["lens_count"]
    assert pitch_subpx == pytest.approx(24.032, abs=1e-3)
    # lens width over subpixel pitch gives the ideal pitch; the measured lens count differs slightly
    assert d["lens_width_mm"] / d["subpixel_pitch_mm"] == pytest.approx(24.0, abs=1e-9)
    assert 3 * d["panel_px"][0] / d["ideal_lens_count"] == pytest.approx(24.014, abs=1e-3)
    ln = scenes.LensParams(Wp=2560, Hp=1600, pitch_subpx=pitch_subpx, slope=-math.tan(math.radians(9.66)))
    K1, Ky, K0 = O.lens_constants(ln, 48)
    assert K1 == round(2 ** 32 / pitch_subpx)
    ky_signed = Ky - (1 << 32) if Ky >= (1 << 31) else Ky
    assert ky_signed == pytest.approx(3 * math.tan(math.radians(9.66)) * 2 ** 32 / pitch_subpx, abs=1)


def test_view_buffer_memory_matches_paper():
    """Sec. 5.2: 64-bit view-buffer pixels give 1.32 MB per 480x360 view and
    63.36 MB for 48 views."""
    d = json.load(open(os.path.join(GOLD, "prototype_display.json")))
    key_bytes = np.dtype(np.uint64).itemsize
    per_view = d["view_px"][0] * d["view_px"][1] * key_bytes / 2 ** 20
    assert round(per_view, 2) == d["view_buffer_MB"]
    assert round(round(per_view, 2) * d["views"], 2) == d["view_buffers_48_MB"]


# ---------------------------------------------------------------------------
# angular supersampling (Sec. 4) and its filter


def test_angular_filter_constant_and_normalised():
    vp = rig(V=6, W=8, H=4, S=4, jitter=scenes.subview_jitter(1, 24))
    cnt, src, wt, maxe = O.angular_table(vp)
    assert (cnt >= 4).all() and (cnt <= 12).all()
    sub = np.full((24, 4, 8), np.uint32(0x11223344), np.uint32)
    assert (O.angular_filter(sub, vp) == 0x11223344).all()
    # each output view weights its own sub-views most
    for v in range(6):
        k = np.argmax(wt[v, :cnt[v]])
        assert src[v, k] // 4 == v


def test_focal_plane_scene_makes_supersampling_exact():
    """A scene lying on the zero-disparity plane looks the same from every
    eye, so 4x angular supersampling + filter reproduces the 1x views."""
    D = 4.0
    P = np.array([[-1.0, -1.0, D], [1.0, -1.0, D], [-1.0, 1.0, D], [1.0, 1.0, D]], np.float32)
    uv = np.array([[0, 0], [3, 0], [0, 3], [3, 3]], np.float32)
    idx = np.array([[0, 2, 1], [1, 2, 3]], np.uint32)
    n = np.cross(P[2] - P[0], P[1] - P[0])
    assert n[2] < 0
    rng = np.random.default_rng(8)
    sc = scenes.Scene(P, uv, idx, np.zeros(2, np.uint16), [scenes.value_noise_texture(64, rng)]).check()
    vp1 = rig(V=6, W=32, H=32, D=D)
    vp4 = rig(V=6, W=32, H=32, D=D, S=4, jitter=scenes.subview_jitter(2, 24))
    r1 = O.render(sc, vp1, IDENT)
    r4 = O.render(sc, vp4, IDENT)
    assert np.isfinite(r1["depth"]).any()
    assert np.array_equal(O.angular_filter(r4["rgba"], vp4), r1["rgba"])


def test_taps_are_gaussian_and_truncated():
    t = np.concatenate([scenes.gaussian_taps(s) for s in range(400)])
    du = t[:, 0] / 2.0 ** 32
    dx = t[:, 1] / 256.0
    assert np.abs(du).max() < 1.0 and np.hypot(t[:, 1], t[:, 2]).max() / 256 < 1.125 + 1 / 256
    assert abs(du.mean()) < 0.03 and abs(dx.mean()) < 0.03
    assert 0.35 < du.std() < 0.5


# ---------------------------------------------------------------------------
# no holes at display size (Sec. 3.2: splats are sized to avoid holes)


@pytest.fixture(scope="module")
def display_1m():
    w = scenes.display()
    return w, O.build_textures(w.scene)


@pytest.mark.parametrize("frame", [0, 17, 111])
def test_display_frames_have_no_orphans_or_misses(display_1m, frame):
    """On the 1M-triangle, 48-view display workload every pixel covered by a
    visible triangle is owned by one of its points and lies in that point's
    splat (frames that had an orphaned zero-area lattice or an edge-on miss
    before the rules for those cases)."""
    w, tx = display_1m
    st = O.render(w.scene, w.views, w.model(frame), tx)["stats"]
    assert st["orphans"] == 0 and st["misses"] == 0 and st["overflow_tris"] == 0, st
    assert st["fragments"] > 40_000_000
