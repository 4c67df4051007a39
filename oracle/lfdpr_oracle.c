/*
 * CPU oracle for light field display point rendering (LFDPR).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header or table generator with the HIP path.
 *
 * Structure: triangle-major.  For each triangle it does the paper's point
 * generation (Sec. 3.1 and 3.3: culling, LFD-aligned frame, horizontal and
 * vertical sampling densities, texture-based density of Eqs. 1-3, the sample
 * lattice, multiview-mip setup of Eqs. 4-7 with two mip fetches per point), then
 * rasterises the triangle into every active view and, for each covered pixel,
 * finds the point whose splat owns it (Sec. 3.2: a projected world-space cell,
 * clipped to the triangle) and applies the per-view texture interpolation of
 * Eqs. 8-9 and the 64-bit (depth, colour) minimum.  The interleave and
 * reconstruction of Sec. 4 and the angular supersampling filter are separate
 * functions.  A conventional per-view z-buffer rasteriser (the paper's
 * multiview-rendering comparison, Sec. 5.1) is included as an independent
 * gold standard.
 *
 * Shading: unlit (the splat's colour is the interpolated albedo of Eq. 9) or
 * physically based (Sec. 3.3: shading happens while the views are rendered,
 * with albedo, roughness, metallic and normal textures).  In the PBR mode each
 * triangle names three more textures; the texture-based density of Eq. 1 takes
 * the largest of the four; every texture gets its own LOD pair (Eqs. 6-7) and
 * its own two mip fetches per point; per view all four are interpolated with
 * the same tau (Eq. 9) and shaded with a Cook-Torrance microfacet BRDF (GGX
 * distribution, Smith-Schlick geometry, Schlick Fresnel) under one directional
 * light plus ambient, then tone mapped (x/(1+x), square-root gamma).
 *
 * Numerics: IEEE binary32, round-to-nearest-even, no contraction (built with
 * -ffp-contract=off), every expression evaluated as parenthesised.  Integer
 * parts (lattice, coverage, texture filtering, interleave) are exact.
 *
 * Parity status per function is listed with the pins in the test-suite; the
 * whole-image comparison with the z-buffer rasteriser is a sanity bound only
 * ("parity unpinned": point rendering differs from rasterisation by design).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define F_ILO 1u
#define F_IHI 2u
#define F_JLO 4u
#define F_JHI 8u
#define CELL_CAP 65536
#define EPS_Q8 4
#define BOX_CAP (1 << 22)

typedef struct {
    int nv, nt;
    const float *pos;      /* nv*3 scene coordinates */
    const float *uv;       /* nv*2 */
    const uint32_t *idx;   /* nt*3 */
    const uint16_t *tex;   /* nt */
    int ntex;
    const int32_t *tex_size;    /* ntex, square power of two */
    const int32_t *tex_levels;  /* ntex */
    const int64_t *tex_level_off; /* ntex*16 byte offsets into texels */
    const uint8_t *texels;
    const uint16_t *mat;   /* nt*3 texture ids (normal, roughness, metallic) or NULL */
} orc_scene;

typedef struct {
    int n_views, W, H, mip;
    float fx, fy, cx, cy, rD, znear;
    const float *eye;      /* n_views: horizontal eye offset b_r */
    const float *kshift;   /* n_views: b_r / D */
    float model[12];       /* camera-from-scene, row-major 3x4 */
    int shade;             /* 0 unlit albedo, 1 physically based */
    float light[9];        /* unit direction towards the light, light RGB, ambient RGB (camera space) */
} orc_frame;

typedef struct {
    /* per triangle */
    int32_t *count;        /* nt */
    float *trif;           /* nt*8: Sx, Sy, smin, smax, ruv, h, size_xy, n_active */
    int32_t *trii;         /* nt*8: S1, T1, S2, T2 (Q8 lattice), kmin, kmax, active?, overflow */
    /* points (emission order) */
    int64_t point_cap;
    uint32_t *p_tri;
    int16_t *p_i, *p_j;
    uint8_t *p_flags;
    uint32_t *p_tvmin, *p_tvmax;
    /* views */
    uint64_t *keys;        /* n_views*H*W, caller-initialised to ~0 */
    /* statistics: [0] points, [1] active tris, [2] point-views, [3] orphans,
       [4] misses, [5] overflow tris, [6] covered fragments */
    int64_t *stats;
    const float *lod_thresholds_unused;
    /* PBR mode only (may be NULL otherwise): per point normal-map fetches and
       roughness/metallic bytes rmin | rmax<<8 | mmin<<16 | mmax<<24; per
       triangle the tangent frame (T, B) and the 8 LODs (albedo, normal,
       roughness, metallic; min, max) */
    uint32_t *p_nmin, *p_nmax, *p_rm;
    float *tframe;         /* nt*6 */
    int32_t *tlod;         /* nt*8 */
    /* optional observation of Eqs. 8-9 (may be NULL): for every (point, view)
       that writes a pixel, the quantised interpolation weight tq (else -1) and
       the splat's RGBA8 colour in that view; point_cap x n_views each */
    int16_t *pv_tq;
    uint32_t *pv_col;
} orc_out;

/* ------------------------------------------------------------------ */
/* small float helpers (expression order is part of the definition)     */

typedef struct { float x, y, z; } v3;

static v3 v3sub(v3 a, v3 b) { v3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static float v3dot(v3 a, v3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
static v3 v3cross(v3 a, v3 b) {
    v3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}
static v3 v3madd(v3 a, float s, v3 d) { v3 r = {a.x + s * d.x, a.y + s * d.y, a.z + s * d.z}; return r; }

/* Closest point on triangle abc to p: the textbook Voronoi-region walk
 * (Ericson, Real-Time Collision Detection, Sec. 5.1.5). */
static v3 closest_on_triangle(v3 p, v3 a, v3 b, v3 c) {
    v3 ab = v3sub(b, a), ac = v3sub(c, a), ap = v3sub(p, a);
    float d1 = v3dot(ab, ap), d2 = v3dot(ac, ap);
    if (d1 <= 0.0f && d2 <= 0.0f) return a;
    v3 bp = v3sub(p, b);
    float d3 = v3dot(ab, bp), d4 = v3dot(ac, bp);
    if (d3 >= 0.0f && d4 <= d3) return b;
    float vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f) {
        float t = d1 / (d1 - d3);
        return v3madd(a, t, ab);
    }
    v3 cp = v3sub(p, c);
    float d5 = v3dot(ab, cp), d6 = v3dot(ac, cp);
    if (d6 >= 0.0f && d5 <= d6) return c;
    float vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) {
        float t = d2 / (d2 - d6);
        return v3madd(a, t, ac);
    }
    float va = d3 * d6 - d5 * d4;
    if (va <= 0.0f && (d4 - d3) >= 0.0f && (d5 - d6) >= 0.0f) {
        float t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        return v3madd(b, t, v3sub(c, b));
    }
    float inv = 1.0f / ((va + vb) + vc);
    float v = vb * inv, w = vc * inv;
    v3 r = v3madd(v3madd(a, v, ab), w, ac);
    return r;
}

static float clampf_big(float x) {
    if (!(x > -1073741824.0f)) return -1073741824.0f;
    if (x > 1073741824.0f) return 1073741824.0f;
    return x;
}

static int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t imax64(int64_t a, int64_t b) { return a > b ? a : b; }
static int64_t floordiv64(int64_t a, int64_t b) { /* b > 0 */
    int64_t q = a / b;
    if ((a % b) != 0 && (a < 0)) q -= 1;
    return q;
}

/* ------------------------------------------------------------------ */
/* textures: box mips and fixed-point trilinear                          */

/* Mip level k+1 is the rounded 2x2 box mean of level k, per channel. */
void orc_build_mips(const uint8_t *level0, int size, uint8_t *chain) {
    memcpy(chain, level0, (size_t)size * size * 4);
    const uint8_t *src = chain;
    uint8_t *dst = chain + (size_t)size * size * 4;
    for (int s = size; s > 1; s >>= 1) {
        int h = s >> 1;
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < h; ++x)
                for (int c = 0; c < 4; ++c) {
                    int a = src[((size_t)(2 * y) * s + 2 * x) * 4 + c];
                    int b = src[((size_t)(2 * y) * s + 2 * x + 1) * 4 + c];
                    int d = src[((size_t)(2 * y + 1) * s + 2 * x) * 4 + c];
                    int e = src[((size_t)(2 * y + 1) * s + 2 * x + 1) * 4 + c];
                    dst[((size_t)y * h + x) * 4 + c] = (uint8_t)((a + b + d + e + 2) >> 2);
                }
        src = dst;
        dst += (size_t)h * h * 4;
    }
}

/* Bilinear sample of one level with 8-bit weights and wrap addressing.
 * Writes 4 channel sums scaled by 2^16. */
static void bilinear_q16(const uint8_t *lev, int Wl, float u, float v, uint32_t out[4]) {
    float sc = (float)(Wl * 256);
    float tx = clampf_big(u * sc - 128.0f);
    float ty = clampf_big(v * sc - 128.0f);
    int ix = (int)floorf(tx), iy = (int)floorf(ty);
    int x0 = (ix >> 8) & (Wl - 1), y0 = (iy >> 8) & (Wl - 1);
    int x1 = (x0 + 1) & (Wl - 1), y1 = (y0 + 1) & (Wl - 1);
    uint32_t ax = (uint32_t)(ix & 255), ay = (uint32_t)(iy & 255);
    uint32_t w00 = (256 - ax) * (256 - ay), w10 = ax * (256 - ay);
    uint32_t w01 = (256 - ax) * ay, w11 = ax * ay;
    for (int c = 0; c < 4; ++c) {
        uint32_t t00 = lev[((size_t)y0 * Wl + x0) * 4 + c];
        uint32_t t10 = lev[((size_t)y0 * Wl + x1) * 4 + c];
        uint32_t t01 = lev[((size_t)y1 * Wl + x0) * 4 + c];
        uint32_t t11 = lev[((size_t)y1 * Wl + x1) * 4 + c];
        out[c] = w00 * t00 + w10 * t10 + w01 * t01 + w11 * t11;
    }
}

/* Trilinear fetch at level-of-detail kc (units of 1/256 level, already
 * clamped to [0, 256*(L-1)]), result RGBA8 packed R | G<<8 | B<<16 | A<<24. */
static uint32_t trilinear(const orc_scene *sc, int t, float u, float v, int kc) {
    int size = sc->tex_size[t], L = sc->tex_levels[t];
    int l0 = kc >> 8, f = kc & 255;
    int l1 = l0 + 1 < L ? l0 + 1 : L - 1;
    uint32_t c0[4], c1[4];
    bilinear_q16(sc->texels + sc->tex_level_off[t * 16 + l0], size >> l0, u, v, c0);
    if (l1 != l0 && f != 0)
        bilinear_q16(sc->texels + sc->tex_level_off[t * 16 + l1], size >> l1, u, v, c1);
    else
        memset(c1, 0, sizeof c1);
    uint32_t out = 0;
    for (int c = 0; c < 4; ++c) {
        uint32_t acc = (uint32_t)(256 - f) * c0[c] + (uint32_t)f * c1[c];
        out |= ((acc + (1u << 23)) >> 24) << (8 * c);
    }
    return out;
}

/* Eqs. 6-7: LOD = 0.5*log2(a), quantised to 1/256 level (round to nearest). */
static int lod_q8(float a) {
    if (!(a > 0.0f)) return -(1 << 30);
    if (isinf(a)) return (1 << 30);
    double k = floor(128.0 * log2((double)a) + 0.5);
    return (int)k;
}

/* ------------------------------------------------------------------ */
/* projection shared by culling, coverage and splat boxes               */

typedef struct { float A, C, Yp; } vproj;

static vproj vertex_proj(const orc_frame *fr, v3 P) {
    vproj r;
    r.A = fr->cx + fr->fx * (P.x / P.z);
    r.C = fr->fx * (1.0f / P.z - fr->rD);
    r.Yp = fr->cy + fr->fy * (P.y / P.z);
    return r;
}

/* Q8 screen position of a projected vertex in view with eye offset b.
 * Returns 0 when outside the +-2^15 px guard band. */
static int q8_xy(vproj p, float b, int64_t *qx, int64_t *qy) {
    float x = p.A - b * p.C;
    if (!(fabsf(x) < 32768.0f) || !(fabsf(p.Yp) < 32768.0f)) return 0;
    *qx = (int64_t)rintf(x * 256.0f);
    *qy = (int64_t)rintf(p.Yp * 256.0f);
    return 1;
}

/* Sec. 3 (the vertex stage checks visibility per LFD view): the triangle faces
 * the eye at (b, 0, 0) by more than a grazing margin.  delta = n.(P0 - e) is
 * the signed distance of the eye from the triangle's plane; the view is kept
 * when delta < 0 (front facing) and |delta| >= |P0 - e| / 256, i.e. the eye
 * direction to vertex 0 is at least asin(1/256) (0.22 degrees) off the plane.
 * Views closer to edge-on project the triangle to (almost) nothing, and the
 * pixel rays that the 1/256-px vertex snap still lets into it meet the plane
 * far outside it (the ray-plane map magnifies by 1/cos). */
static int faces_eye(v3 P0, float delta, float b) {
    float dx = P0.x - b;
    float d2 = (dx * dx + P0.y * P0.y) + P0.z * P0.z;
    return delta < 0.0f && delta * delta >= d2 * 0x1p-16f;
}

/* ------------------------------------------------------------------ */
/* per-triangle state                                                     */

typedef struct {
    v3 P[3];
    v3 nh, u, w;
    float h, Sx, Sy, smin, smax, ruv;
    int64_t S[3], T[3], area2;
    int count;
    int jlo, jhi;
    int *ilo, *ihi;       /* per row, indexed j - jlo */
    int64_t first_point;  /* index of (jlo, ilo(jlo)) in emission order */
    int *rowstart;        /* per row */
    vproj pr[3];
    int tex;
    int texm[4];          /* albedo, normal, roughness, metallic (PBR) */
    int kq[8];            /* LOD min/max per texture (1/256 level) */
    v3 tt, tb;            /* tangent frame (PBR) */
} tri_state;

static int cell_overlaps(const tri_state *ts, int64_t i, int64_t j) {
    int64_t bx0 = 256 * i - EPS_Q8, bx1 = 256 * i + 256 + EPS_Q8;
    int64_t by0 = 256 * j - EPS_Q8, by1 = 256 * j + 256 + EPS_Q8;
    int64_t mins = imin64(ts->S[0], imin64(ts->S[1], ts->S[2]));
    int64_t maxs = imax64(ts->S[0], imax64(ts->S[1], ts->S[2]));
    int64_t mint = imin64(ts->T[0], imin64(ts->T[1], ts->T[2]));
    int64_t maxt = imax64(ts->T[0], imax64(ts->T[1], ts->T[2]));
    if (!(bx1 > mins && bx0 < maxs && by1 > mint && by0 < maxt)) return 0;
    /* a snapped lattice of zero area (a point or a segment) keeps every cell
       whose dilated box meets the bounding box of its vertices */
    if (ts->area2 == 0) return 1;
    int64_t sg = ts->area2 > 0 ? 1 : -1;
    for (int e = 0; e < 3; ++e) {
        int a = e, b = (e + 1) % 3;
        int64_t dx = ts->S[b] - ts->S[a], dy = ts->T[b] - ts->T[a];
        int64_t cx[4] = {bx0, bx1, bx0, bx1}, cy[4] = {by0, by0, by1, by1};
        int any = 0;
        for (int k = 0; k < 4; ++k) {
            int64_t E = sg * (dx * (cy[k] - ts->T[a]) - dy * (cx[k] - ts->S[a]));
            if (E > 0) any = 1;
        }
        if (!any) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------ */

/* Eqs. 8-9: interpolation weight tau of the splat of cell (i, j) in the view
 * with eye offset b, quantised to tq/256. */
static int splat_tq(const tri_state *ts, const orc_frame *fr, float b, int i, int j) {
    float fxfy = fr->fx * fr->fy;
    float cs = (float)i / ts->Sx, ct = (float)j / ts->Sy;
    float Zc = (ts->P[0].z + cs * ts->u.z) + ct * ts->w.z;
    float delta = ts->h - ts->nh.x * b;
    float ad = fabsf(delta);
    float Ar = ((Zc * Zc) * Zc) / (fxfy * ad);   /* pixel footprint at the cell centre */
    float Acell = 1.0f / (ts->Sx * ts->Sy);      /* splat (cell) area */
    /* Eq. 8: the splat's texture area suv = Acell*ruv, divided by min(1, Acell/Ar) */
    float vse = Acell < Ar ? ts->ruv * Ar : Acell * ts->ruv;
    float vs = vse < ts->smin ? ts->smin : (vse > ts->smax ? ts->smax : vse); /* clamp */
    float irange = ts->smax > ts->smin ? 1.0f / (ts->smax - ts->smin) : 0.0f;
    float tau = (vs - ts->smin) * irange;          /* Eq. 9 */
    int tq = (int)floorf(tau * 256.0f + 0.5f);
    if (tq < 0) tq = 0;
    if (tq > 256) tq = 256;
    return tq;
}

/* ------------------------------------------------------------------ */
/* physically based shading (PBR mode)                                     */

#define K255 0x1.010102p-8f     /* float nearest 1/255 */
#define K2_255 0x1.010102p-7f   /* float nearest 2/255 (exactly 2*K255) */
#define PI_F 0x1.921fb6p+1f     /* float nearest pi */
#define INV_PI_F 0x1.45f306p-2f /* float nearest 1/pi */

/* Tangent frame of the texture mapping: T = dP/du and B = dP/dv solved from
 * the two edges and their UV differences, T made orthogonal to the unit normal
 * and normalised, B = n x T with the sign of dP/dv.  A degenerate mapping
 * falls back to the lattice axes u, w. */
static void tangent_frame(v3 e1, v3 e2, float du1, float dv1, float du2, float dv2, v3 nh, v3 u, v3 w,
                          v3 *T, v3 *B) {
    float det = du1 * dv2 - dv1 * du2;
    v3 t = u, bb = w;
    if (det != 0.0f) {
        float rd = 1.0f / det;
        t.x = (e1.x * dv2 - e2.x * dv1) * rd;
        t.y = (e1.y * dv2 - e2.y * dv1) * rd;
        t.z = (e1.z * dv2 - e2.z * dv1) * rd;
        bb.x = (e2.x * du1 - e1.x * du2) * rd;
        bb.y = (e2.y * du1 - e1.y * du2) * rd;
        bb.z = (e2.z * du1 - e1.z * du2) * rd;
    }
    float tn = v3dot(nh, t);
    v3 tp = {t.x - nh.x * tn, t.y - nh.y * tn, t.z - nh.z * tn};
    float tl = sqrtf((tp.x * tp.x + tp.y * tp.y) + tp.z * tp.z);
    if (tl > 0.0f && !isinf(tl)) {
        float it = 1.0f / tl;
        tp.x = tp.x * it; tp.y = tp.y * it; tp.z = tp.z * it;
    } else {
        tp = u;
    }
    v3 bp = v3cross(nh, tp);
    if (v3dot(bp, bb) < 0.0f) { bp.x = -bp.x; bp.y = -bp.y; bp.z = -bp.z; }
    *T = tp;
    *B = bp;
}

typedef struct { float D, G, NL, NV, F[3], f[3]; } pbr_terms;

/* Cook-Torrance BRDF for unit normal n, unit view v and unit light L:
 * f = kd a / pi + F D G / (4 (n.L)(n.V) + 1e-4), GGX D with alpha = r^2,
 * Smith-Schlick G with k = (r+1)^2/8, Schlick F with F0 = 0.04 (1-m) + a m,
 * kd = (1 - F)(1 - m). */
static void pbr_eval(v3 n, v3 v, v3 L, float rgh, float mtl, const float a[3], pbr_terms *o) {
    v3 h = {L.x + v.x, L.y + v.y, L.z + v.z};
    float hl = sqrtf((h.x * h.x + h.y * h.y) + h.z * h.z);
    v3 H = n;
    if (hl > 0.0f && !isinf(hl)) {
        float ih = 1.0f / hl;
        H.x = h.x * ih; H.y = h.y * ih; H.z = h.z * ih;
    }
    float NL = v3dot(n, L), NV = v3dot(n, v), NH = v3dot(n, H), VH = v3dot(v, H);
    NL = NL > 0.0f ? NL : 0.0f;
    NV = NV > 0.0f ? NV : 0.0f;
    NH = NH > 0.0f ? NH : 0.0f;
    VH = VH > 0.0f ? VH : 0.0f;
    float al = rgh * rgh, a2 = al * al;
    float dd = (NH * NH) * (a2 - 1.0f) + 1.0f;
    float D = a2 / ((PI_F * dd) * dd);
    float kk = ((rgh + 1.0f) * (rgh + 1.0f)) * 0.125f;
    float G = (NL / (NL * (1.0f - kk) + kk)) * (NV / (NV * (1.0f - kk) + kk));
    float fr = 1.0f - VH;
    float f5 = ((fr * fr) * (fr * fr)) * fr;
    float sp = (D * G) / (((4.0f * NL) * NV) + 1e-4f);
    o->D = D; o->G = G; o->NL = NL; o->NV = NV;
    for (int c = 0; c < 3; ++c) {
        float F0 = 0.04f * (1.0f - mtl) + a[c] * mtl;
        float F = F0 + (1.0f - F0) * f5;
        float kd = (1.0f - F) * (1.0f - mtl);
        o->F[c] = F;
        o->f[c] = (kd * a[c]) * INV_PI_F + F * sp;
    }
}

/* Shaded RGBA8 of a splat in the view with eye offset b: albedo, normal-map,
 * roughness and metallic bytes already interpolated with tau (Eq. 9); the
 * surface point is the cell centre Pc; alpha is the albedo's. */
static uint32_t pbr_shade(const float light[9], v3 nh, v3 tt, v3 tb, v3 Pc, float b, uint32_t alb,
                          uint32_t nrm, uint32_t rq, uint32_t mq) {
    float a[3];
    for (int c = 0; c < 3; ++c) a[c] = (float)((alb >> (8 * c)) & 255u) * K255;
    float nr = (float)(nrm & 255u) * K2_255 - 1.0f;
    float ng = (float)((nrm >> 8) & 255u) * K2_255 - 1.0f;
    float nb = (float)((nrm >> 16) & 255u) * K2_255 - 1.0f;
    v3 sn = {(nr * tt.x + ng * tb.x) + nb * nh.x, (nr * tt.y + ng * tb.y) + nb * nh.y,
             (nr * tt.z + ng * tb.z) + nb * nh.z};
    float sl = sqrtf((sn.x * sn.x + sn.y * sn.y) + sn.z * sn.z);
    v3 n = nh;
    if (sl > 0.0f && !isinf(sl)) {
        float is = 1.0f / sl;
        n.x = sn.x * is; n.y = sn.y * is; n.z = sn.z * is;
    }
    v3 vv = {b - Pc.x, 0.0f - Pc.y, 0.0f - Pc.z};
    float vl = sqrtf((vv.x * vv.x + vv.y * vv.y) + vv.z * vv.z);
    v3 v = {0.0f, 0.0f, -1.0f};
    if (vl > 0.0f && !isinf(vl)) {
        float iv = 1.0f / vl;
        v.x = vv.x * iv; v.y = vv.y * iv; v.z = vv.z * iv;
    }
    v3 L = {light[0], light[1], light[2]};
    float rgh = (float)rq * K255;
    rgh = rgh > 0.03f ? rgh : 0.03f;
    float mtl = (float)mq * K255;
    pbr_terms T;
    pbr_eval(n, v, L, rgh, mtl, a, &T);
    uint32_t out = alb & 0xFF000000u;
    for (int c = 0; c < 3; ++c) {
        float lo = T.f[c] * (light[3 + c] * T.NL) + light[6 + c] * a[c];
        float t = lo / (1.0f + lo);
        float y = floorf(sqrtf(t) * 255.0f + 0.5f);
        uint32_t q = y >= 255.0f ? 255u : (y > 0.0f ? (uint32_t)y : 0u);
        out |= q << (8 * c);
    }
    return out;
}

/* Eq. 9 interpolation of one byte, and of four packed bytes, with weight tq/256. */
static uint32_t lerp8(uint32_t a, uint32_t z, int tq) {
    return (a * (uint32_t)(256 - tq) + z * (uint32_t)tq + 128u) >> 8;
}

static uint32_t lerp_rgba8(uint32_t lo, uint32_t hi, int tq) {
    uint32_t out = 0;
    for (int c = 0; c < 4; ++c) out |= lerp8((lo >> (8 * c)) & 255u, (hi >> (8 * c)) & 255u, tq) << (8 * c);
    return out;
}

/* Pixel range that the splat of point (i, j, flags) may write in a view. */
static void splat_box(const tri_state *ts, const orc_frame *fr, float b, int i, int j, unsigned flags,
                      int tx0, int tx1, int ty0, int ty1, int box[4]) {
    int s0 = i - ((flags & F_ILO) ? 1 : 0), s1 = i + 1 + ((flags & F_IHI) ? 1 : 0);
    int t0 = j - ((flags & F_JLO) ? 1 : 0), t1 = j + 1 + ((flags & F_JHI) ? 1 : 0);
    int ss[4] = {s0, s1, s0, s1}, tt[4] = {t0, t0, t1, t1};
    float xmin = 0, xmax = 0, ymin = 0, ymax = 0;
    for (int k = 0; k < 4; ++k) {
        float a = ((float)ss[k] - 0.5f) / ts->Sx;
        float c = ((float)tt[k] - 0.5f) / ts->Sy;
        v3 X;
        X.x = (ts->P[0].x + a * ts->u.x) + c * ts->w.x;
        X.y = (ts->P[0].y + a * ts->u.y) + c * ts->w.y;
        X.z = (ts->P[0].z + a * ts->u.z) + c * ts->w.z;
        if (!(X.z >= 0.5f * fr->znear)) { box[0] = tx0; box[1] = tx1; box[2] = ty0; box[3] = ty1; return; }
        vproj p = vertex_proj(fr, X);
        float x = p.A - b * p.C, y = p.Yp;
        if (k == 0) { xmin = xmax = x; ymin = ymax = y; }
        else {
            xmin = x < xmin ? x : xmin; xmax = x > xmax ? x : xmax;
            ymin = y < ymin ? y : ymin; ymax = y > ymax ? y : ymax;
        }
    }
    box[0] = (int)ceilf(clampf_big(xmin - 0.515625f));
    box[1] = (int)floorf(clampf_big(xmax - 0.484375f));
    box[2] = (int)ceilf(clampf_big(ymin - 0.515625f));
    box[3] = (int)floorf(clampf_big(ymax - 0.484375f));
}

/* Main entry: point generation + splatting for one frame. */
int orc_render(const orc_scene *sc, const orc_frame *fr, orc_out *out) {
    const float *m = fr->model;
    float fxfy = fr->fx * fr->fy;
    int64_t npts = 0;
    int nviews = fr->n_views;
    int64_t px_per_view = (int64_t)fr->W * fr->H;
    if (fr->shade == 1 && !sc->mat) return -2;
    int *vactive = (int *)malloc(sizeof(int) * (size_t)nviews);
    for (int t = 0; t < sc->nt; ++t) {
        tri_state ts;
        memset(&ts, 0, sizeof ts);
        out->count[t] = 0;
        for (int k = 0; k < 8; ++k) { out->trif[t * 8 + k] = 0.0f; out->trii[t * 8 + k] = 0; }
        /* frame transform */
        int zbad = 0;
        for (int k = 0; k < 3; ++k) {
            uint32_t vi = sc->idx[t * 3 + k];
            float px = sc->pos[vi * 3 + 0], py = sc->pos[vi * 3 + 1], pz = sc->pos[vi * 3 + 2];
            ts.P[k].x = ((m[0] * px + m[1] * py) + m[2] * pz) + m[3];
            ts.P[k].y = ((m[4] * px + m[5] * py) + m[6] * pz) + m[7];
            ts.P[k].z = ((m[8] * px + m[9] * py) + m[10] * pz) + m[11];
            if (!(ts.P[k].z >= fr->znear)) zbad = 1;
        }
        if (zbad) continue;
        v3 e1 = v3sub(ts.P[1], ts.P[0]), e2 = v3sub(ts.P[2], ts.P[0]);
        v3 n = v3cross(e1, e2);
        float nl = sqrtf((n.x * n.x + n.y * n.y) + n.z * n.z);
        if (!(nl > 0.0f) || isinf(nl)) continue;
        ts.nh.x = n.x / nl; ts.nh.y = n.y / nl; ts.nh.z = n.z / nl;
        ts.h = v3dot(ts.nh, ts.P[0]);
        for (int k = 0; k < 3; ++k) ts.pr[k] = vertex_proj(fr, ts.P[k]);
        /* Sec. 3: visibility of the triangle in each LFD view */
        int nact = 0;
        for (int r = 0; r < nviews; ++r) {
            float b = fr->eye[r];
            float delta = ts.h - ts.nh.x * b;
            int act = faces_eye(ts.P[0], delta, b);
            int64_t qx[3], qy[3];
            for (int k = 0; k < 3 && act; ++k) act = q8_xy(ts.pr[k], b, &qx[k], &qy[k]);
            if (act) {
                int64_t W8 = 256 * (int64_t)fr->W, H8 = 256 * (int64_t)fr->H;
                if (qx[0] < 0 && qx[1] < 0 && qx[2] < 0) act = 0;
                if (qx[0] > W8 && qx[1] > W8 && qx[2] > W8) act = 0;
                if (qy[0] < 0 && qy[1] < 0 && qy[2] < 0) act = 0;
                if (qy[0] > H8 && qy[1] > H8 && qy[2] > H8) act = 0;
            }
            vactive[r] = act;
            nact += act;
        }
        if (nact == 0) continue;
        out->stats[1] += 1;
        /* LFD-aligned sampling frame (T_align): normal, camera-X in plane, and their cross */
        v3 up;
        if (fabsf(ts.nh.x) > 0.99999f) {
            up.x = 0.0f - ts.nh.x * ts.nh.y; up.y = 1.0f - ts.nh.y * ts.nh.y; up.z = 0.0f - ts.nh.z * ts.nh.y;
        } else {
            up.x = 1.0f - ts.nh.x * ts.nh.x; up.y = 0.0f - ts.nh.y * ts.nh.x; up.z = 0.0f - ts.nh.z * ts.nh.x;
        }
        float ul = sqrtf((up.x * up.x + up.y * up.y) + up.z * up.z);
        ts.u.x = up.x / ul; ts.u.y = up.y / ul; ts.u.z = up.z / ul;
        ts.w = v3cross(ts.nh, ts.u);
        /* Horizontal / vertical densities from reverse-projected pixel edges at
           the closest point to each active eye (Sec. 3.1, Fig. 4) */
        float lxmin = INFINITY, lymin = INFINITY, Amin = INFINITY, admin = INFINITY, admax = 0.0f;
        for (int r = 0; r < nviews; ++r) {
            if (!vactive[r]) continue;
            float b = fr->eye[r];
            v3 e = {b, 0.0f, 0.0f};
            v3 Ps = closest_on_triangle(e, ts.P[0], ts.P[1], ts.P[2]);
            v3 d = v3sub(Ps, e);
            float delta = ts.h - ts.nh.x * b;
            float ad = fabsf(delta);
            float Zs = Ps.z;
            float g = ts.nh.x / delta;
            float vx = 1.0f - d.x * g, vy = 0.0f - d.y * g, vz = 0.0f - d.z * g;
            float lx = (Zs / fr->fx) * sqrtf((vx * vx + vy * vy) + vz * vz);
            float g2 = ts.nh.y / delta;
            float wx = 0.0f - d.x * g2, wy = 1.0f - d.y * g2, wz = 0.0f - d.z * g2;
            float ly = (Zs / fr->fy) * sqrtf((wx * wx + wy * wy) + wz * wz);
            float A = ((Zs * Zs) * Zs) / (fxfy * ad);
            lxmin = lx < lxmin ? lx : lxmin;
            lymin = ly < lymin ? ly : lymin;
            Amin = A < Amin ? A : Amin;
            admin = ad < admin ? ad : admin;
            admax = ad > admax ? ad : admax;
        }
        ts.Sx = 1.0f / lxmin;
        ts.Sy = 1.0f / lymin;
        float size_xy = Amin;
        /* Texture-based sampling, Eqs. 1-3: one albedo texture per triangle, or
           the four textures of the PBR mode with Eq. 1's maximum over them */
        const int pbr = fr->shade == 1;
        ts.tex = sc->tex[t];
        ts.texm[0] = ts.tex;
        for (int k = 1; k < 4; ++k) ts.texm[k] = pbr ? (int)sc->mat[t * 3 + k - 1] : ts.tex;
        float uv0u, uv0v, du1, dv1, du2, dv2;
        {
            uint32_t i0 = sc->idx[t * 3], i1 = sc->idx[t * 3 + 1], i2 = sc->idx[t * 3 + 2];
            uv0u = sc->uv[i0 * 2]; uv0v = sc->uv[i0 * 2 + 1];
            du1 = sc->uv[i1 * 2] - uv0u; dv1 = sc->uv[i1 * 2 + 1] - uv0v;
            du2 = sc->uv[i2 * 2] - uv0u; dv2 = sc->uv[i2 * 2 + 1] - uv0v;
        }
        float Ats = 0.5f * fabsf(du1 * dv2 - dv1 * du2);
        float Aws = 0.5f * nl;
        float Xt = (float)sc->tex_size[ts.tex];
        float ntex = (Ats * Xt) * Xt;                 /* Eq. 1 */
        for (int k = 1; k < 4 && pbr; ++k) {
            float Xk = (float)sc->tex_size[ts.texm[k]];
            float nk = (Ats * Xk) * Xk;
            ntex = nk > ntex ? nk : ntex;
        }
        if (ntex > 0.0f) {
            float size_uv = Aws / ntex;               /* Eq. 2 */
            if (size_uv > size_xy) {                  /* Eq. 3 */
                float f = sqrtf(size_xy / size_uv);
                ts.Sx = ts.Sx * f;
                ts.Sy = ts.Sy * f;
            }
        }
        ts.ruv = Ats / Aws;
        /* Multiview-mip setup, Eqs. 4-5: extremes of the per-view pixel footprint
           on the triangle (over its vertices and the active views) */
        float Zmin = ts.P[0].z, Zmax = ts.P[0].z;
        for (int k = 1; k < 3; ++k) {
            Zmin = ts.P[k].z < Zmin ? ts.P[k].z : Zmin;
            Zmax = ts.P[k].z > Zmax ? ts.P[k].z : Zmax;
        }
        ts.smin = (((Zmin * Zmin) * Zmin) / (fxfy * admax)) * ts.ruv;
        ts.smax = (((Zmax * Zmax) * Zmax) / (fxfy * admin)) * ts.ruv;
        /* Eqs. 6-7 per texture (its own size and level count) */
        for (int k = 0; k < 4; ++k) {
            int tk = ts.texm[k];
            float Xk = (float)sc->tex_size[tk];
            int k0 = 0, k1 = 0;
            if (fr->mip) {
                k0 = lod_q8((ts.smin * Xk) * Xk);     /* Eq. 6 */
                k1 = lod_q8((ts.smax * Xk) * Xk);     /* Eq. 7 */
                int top = 256 * (sc->tex_levels[tk] - 1);
                k0 = k0 < 0 ? 0 : (k0 > top ? top : k0);
                k1 = k1 < 0 ? 0 : (k1 > top ? top : k1);
            }
            ts.kq[2 * k] = k0;
            ts.kq[2 * k + 1] = k1;
        }
        int kmin = ts.kq[0], kmax = ts.kq[1];
        if (pbr) {
            tangent_frame(e1, e2, du1, dv1, du2, dv2, ts.nh, ts.u, ts.w, &ts.tt, &ts.tb);
            if (out->tframe) {
                float *tf = out->tframe + (int64_t)t * 6;
                tf[0] = ts.tt.x; tf[1] = ts.tt.y; tf[2] = ts.tt.z; tf[3] = ts.tb.x; tf[4] = ts.tb.y; tf[5] = ts.tb.z;
            }
            if (out->tlod)
                for (int k = 0; k < 8; ++k) out->tlod[(int64_t)t * 8 + k] = ts.kq[k];
        }
        /* sample lattice in the aligned, density-scaled plane; vertex 0 at cell (0,0) centre */
        int overflow = 0;
        ts.S[0] = 128; ts.T[0] = 128;
        for (int k = 1; k < 3; ++k) {
            v3 ek = k == 1 ? e1 : e2;
            float s = ts.Sx * v3dot(ts.u, ek) + 0.5f;
            float tt = ts.Sy * v3dot(ts.w, ek) + 0.5f;
            if (!(fabsf(s) < 16384.0f) || !(fabsf(tt) < 16384.0f)) { overflow = 1; break; }
            ts.S[k] = (int64_t)rintf(s * 256.0f);
            ts.T[k] = (int64_t)rintf(tt * 256.0f);
        }
        out->trif[t * 8 + 0] = ts.Sx; out->trif[t * 8 + 1] = ts.Sy;
        out->trif[t * 8 + 2] = ts.smin; out->trif[t * 8 + 3] = ts.smax;
        out->trif[t * 8 + 4] = ts.ruv; out->trif[t * 8 + 5] = ts.h;
        out->trif[t * 8 + 6] = size_xy; out->trif[t * 8 + 7] = (float)nact;
        out->trii[t * 8 + 4] = kmin; out->trii[t * 8 + 5] = kmax; out->trii[t * 8 + 6] = 1;
        ts.area2 = 0;
        if (!overflow) {
            out->trii[t * 8 + 0] = (int32_t)ts.S[1]; out->trii[t * 8 + 1] = (int32_t)ts.T[1];
            out->trii[t * 8 + 2] = (int32_t)ts.S[2]; out->trii[t * 8 + 3] = (int32_t)ts.T[2];
            ts.area2 = (ts.S[1] - ts.S[0]) * (ts.T[2] - ts.T[0]) - (ts.T[1] - ts.T[0]) * (ts.S[2] - ts.S[0]);
        }
        /* emission by exhaustive cell test over the lattice bounding box */
        int *cells_i = NULL, *cells_j = NULL;
        int ncell = 0;
        if (!overflow) {
            int64_t mins = imin64(ts.S[0], imin64(ts.S[1], ts.S[2])), maxs = imax64(ts.S[0], imax64(ts.S[1], ts.S[2]));
            int64_t mint = imin64(ts.T[0], imin64(ts.T[1], ts.T[2])), maxt = imax64(ts.T[0], imax64(ts.T[1], ts.T[2]));
            /* cells whose dilated box overlaps the lattice bounding box with positive length */
            int64_t i0 = floordiv64(mins - EPS_Q8, 256), i1 = floordiv64(maxs + EPS_Q8 - 1, 256);
            int64_t j0 = floordiv64(mint - EPS_Q8, 256), j1 = floordiv64(maxt + EPS_Q8 - 1, 256);
            int64_t nb = (i1 - i0 + 1) * (j1 - j0 + 1);
            if (nb > BOX_CAP) overflow = 1;
            else {
                int cap = 1024;
                cells_i = (int *)malloc(sizeof(int) * cap);
                cells_j = (int *)malloc(sizeof(int) * cap);
                for (int64_t j = j0; j <= j1 && !overflow; ++j)
                    for (int64_t i = i0; i <= i1; ++i)
                        if (cell_overlaps(&ts, i, j)) {
                            if (ncell == CELL_CAP) { overflow = 1; break; }
                            if (ncell == cap) {
                                cap *= 2;
                                cells_i = (int *)realloc(cells_i, sizeof(int) * cap);
                                cells_j = (int *)realloc(cells_j, sizeof(int) * cap);
                            }
                            cells_i[ncell] = (int)i; cells_j[ncell] = (int)j; ++ncell;
                        }
            }
        }
        if (overflow) { ncell = 0; out->stats[5] += 1; out->trii[t * 8 + 7] = 1; }
        ts.count = ncell;
        out->count[t] = ncell;
        /* row structure (rows are j-major in emission order) */
        if (ncell > 0) {
            ts.jlo = cells_j[0]; ts.jhi = cells_j[ncell - 1];
            int nrow = ts.jhi - ts.jlo + 1;
            ts.ilo = (int *)malloc(sizeof(int) * nrow);
            ts.ihi = (int *)malloc(sizeof(int) * nrow);
            ts.rowstart = (int *)malloc(sizeof(int) * nrow);
            for (int r = 0; r < nrow; ++r) { ts.ilo[r] = 1 << 30; ts.ihi[r] = -(1 << 30); ts.rowstart[r] = -1; }
            for (int c = 0; c < ncell; ++c) {
                int r = cells_j[c] - ts.jlo;
                if (ts.rowstart[r] < 0) ts.rowstart[r] = c;
                if (cells_i[c] < ts.ilo[r]) ts.ilo[r] = cells_i[c];
                if (cells_i[c] > ts.ihi[r]) ts.ihi[r] = cells_i[c];
            }
        }
        ts.first_point = npts;
        /* per-point attributes: UV at the cell centre, two mip fetches */
        uint32_t *tvmin = NULL, *tvmax = NULL, *nmin = NULL, *nmax = NULL, *rm = NULL;
        unsigned *flg = NULL;
        if (ncell > 0) {
            tvmin = (uint32_t *)malloc(sizeof(uint32_t) * ncell);
            tvmax = (uint32_t *)malloc(sizeof(uint32_t) * ncell);
            flg = (unsigned *)malloc(sizeof(unsigned) * ncell);
            if (pbr) {
                nmin = (uint32_t *)malloc(sizeof(uint32_t) * ncell);
                nmax = (uint32_t *)malloc(sizeof(uint32_t) * ncell);
                rm = (uint32_t *)malloc(sizeof(uint32_t) * ncell);
            }
        }
        for (int c = 0; c < ncell; ++c) {
            int i = cells_i[c], j = cells_j[c];
            int r = j - ts.jlo;
            unsigned f = 0;
            if (i == ts.ilo[r]) f |= F_ILO;
            if (i == ts.ihi[r]) f |= F_IHI;
            if (j == ts.jlo) f |= F_JLO;
            if (j == ts.jhi) f |= F_JHI;
            int64_t cxq = 256 * (int64_t)i + 128, cyq = 256 * (int64_t)j + 128;
            int64_t w1 = (cxq - ts.S[0]) * (ts.T[2] - ts.T[0]) - (cyq - ts.T[0]) * (ts.S[2] - ts.S[0]);
            int64_t w2 = (ts.S[1] - ts.S[0]) * (cyq - ts.T[0]) - (ts.T[1] - ts.T[0]) * (cxq - ts.S[0]);
            /* a zero-area lattice has no barycentrics: its points take vertex 0's UV */
            float b1 = ts.area2 != 0 ? (float)((double)w1 / (double)ts.area2) : 0.0f;
            float b2 = ts.area2 != 0 ? (float)((double)w2 / (double)ts.area2) : 0.0f;
            float uu = (uv0u + b1 * du1) + b2 * du2;
            float vv = (uv0v + b1 * dv1) + b2 * dv2;
            tvmin[c] = trilinear(sc, ts.tex, uu, vv, kmin);
            tvmax[c] = trilinear(sc, ts.tex, uu, vv, kmax);
            if (pbr) {
                nmin[c] = trilinear(sc, ts.texm[1], uu, vv, ts.kq[2]);
                nmax[c] = trilinear(sc, ts.texm[1], uu, vv, ts.kq[3]);
                uint32_t r0 = trilinear(sc, ts.texm[2], uu, vv, ts.kq[4]) & 255u;
                uint32_t r1 = trilinear(sc, ts.texm[2], uu, vv, ts.kq[5]) & 255u;
                uint32_t m0 = trilinear(sc, ts.texm[3], uu, vv, ts.kq[6]) & 255u;
                uint32_t m1 = trilinear(sc, ts.texm[3], uu, vv, ts.kq[7]) & 255u;
                rm[c] = r0 | (r1 << 8) | (m0 << 16) | (m1 << 24);
            }
            flg[c] = f;
            int64_t gi = npts + c;
            if (gi < out->point_cap) {
                out->p_tri[gi] = (uint32_t)t;
                out->p_i[gi] = (int16_t)i; out->p_j[gi] = (int16_t)j;
                out->p_flags[gi] = (uint8_t)f;
                out->p_tvmin[gi] = tvmin[c]; out->p_tvmax[gi] = tvmax[c];
                if (pbr && out->p_nmin) { out->p_nmin[gi] = nmin[c]; out->p_nmax[gi] = nmax[c]; out->p_rm[gi] = rm[c]; }
            }
        }
        npts += ncell;
        out->stats[2] += (int64_t)ncell * nact;
        /* Splatting into every active view (Sec. 3.2) */
        for (int r = 0; r < nviews; ++r) {
            if (!vactive[r]) continue;
            float b = fr->eye[r];
            int64_t qx[3], qy[3];
            for (int k = 0; k < 3; ++k) q8_xy(ts.pr[k], b, &qx[k], &qy[k]);
            int64_t a2 = (qx[1] - qx[0]) * (qy[2] - qy[0]) - (qy[1] - qy[0]) * (qx[2] - qx[0]);
            if (a2 == 0) continue;
            if (a2 < 0) {
                int64_t tx = qx[1]; qx[1] = qx[2]; qx[2] = tx;
                int64_t ty = qy[1]; qy[1] = qy[2]; qy[2] = ty;
            }
            int64_t xmin = imin64(qx[0], imin64(qx[1], qx[2])), xmax = imax64(qx[0], imax64(qx[1], qx[2]));
            int64_t ymin = imin64(qy[0], imin64(qy[1], qy[2])), ymax = imax64(qy[0], imax64(qy[1], qy[2]));
            int64_t X0 = imax64(0, -floordiv64(-(xmin - 128), 256)), X1 = imin64(fr->W - 1, floordiv64(xmax - 128, 256));
            int64_t Y0 = imax64(0, -floordiv64(-(ymin - 128), 256)), Y1 = imin64(fr->H - 1, floordiv64(ymax - 128, 256));
            float ks = fr->kshift[r];
            float delta = ts.h - ts.nh.x * b;
            float cu = ts.u.x * (b - ts.P[0].x) - (ts.u.y * ts.P[0].y + ts.u.z * ts.P[0].z);
            float cw = ts.w.x * (b - ts.P[0].x) - (ts.w.y * ts.P[0].y + ts.w.z * ts.P[0].z);
            for (int64_t y = Y0; y <= Y1; ++y)
                for (int64_t x = X0; x <= X1; ++x) {
                    int64_t pxq = 256 * x + 128, pyq = 256 * y + 128;
                    int in = 1;
                    for (int e = 0; e < 3 && in; ++e) {
                        int a = e, bb = (e + 1) % 3;
                        int64_t dx = qx[bb] - qx[a], dy = qy[bb] - qy[a];
                        int64_t E = dx * (pyq - qy[a]) - dy * (pxq - qx[a]);
                        int owns = dy > 0 || (dy == 0 && dx > 0);
                        in = E > 0 || (E == 0 && owns);
                    }
                    if (!in) continue;
                    out->stats[6] += 1;
                    /* the eye ray through the pixel centre meets the triangle's plane */
                    float fxp = (float)x + 0.5f, fyp = (float)y + 0.5f;
                    float rx = (fxp - fr->cx) / fr->fx - ks;
                    float ry = (fyp - fr->cy) / fr->fy;
                    float den = (ts.nh.x * rx + ts.nh.y * ry) + ts.nh.z;
                    float Z = delta / den;
                    if (!(Z > 0.0f) || isinf(Z)) { out->stats[4] += 1; continue; }
                    /* hit - P0 = (b - P0x, -P0y, -P0z) + Z*(rx, ry, 1), projected on the lattice axes */
                    float ur = (ts.u.x * rx + ts.u.y * ry) + ts.u.z;
                    float wr = (ts.w.x * rx + ts.w.y * ry) + ts.w.z;
                    float s = ts.Sx * (Z * ur + cu) + 0.5f;
                    float tt = ts.Sy * (Z * wr + cw) + 0.5f;
                    if (ts.count == 0) { out->stats[3] += 1; continue; }
                    int fi = (int)floorf(clampf_big(s)), fj = (int)floorf(clampf_big(tt));
                    int cj = fj < ts.jlo ? ts.jlo : (fj > ts.jhi ? ts.jhi : fj);
                    int rr = cj - ts.jlo;
                    int ci = fi < ts.ilo[rr] ? ts.ilo[rr] : (fi > ts.ihi[rr] ? ts.ihi[rr] : fi);
                    int c = ts.rowstart[rr] + (ci - ts.ilo[rr]);
                    int box[4];
                    splat_box(&ts, fr, b, ci, cj, flg[c], (int)X0, (int)X1, (int)Y0, (int)Y1, box);
                    if (x < box[0] || x > box[1] || y < box[2] || y > box[3]) { out->stats[4] += 1; continue; }
                    int tq = splat_tq(&ts, fr, b, ci, cj);
                    uint32_t col = lerp_rgba8(tvmin[c], tvmax[c], tq);
                    if (pbr) {
                        /* cell centre of the owning point (vertex 0 sits at the centre of cell (0,0)) */
                        float cs = (float)ci / ts.Sx, ct = (float)cj / ts.Sy;
                        v3 Pc = {(ts.P[0].x + cs * ts.u.x) + ct * ts.w.x, (ts.P[0].y + cs * ts.u.y) + ct * ts.w.y,
                                 (ts.P[0].z + cs * ts.u.z) + ct * ts.w.z};
                        uint32_t nrm = lerp_rgba8(nmin[c], nmax[c], tq);
                        uint32_t rq = lerp8(rm[c] & 255u, (rm[c] >> 8) & 255u, tq);
                        uint32_t mq = lerp8((rm[c] >> 16) & 255u, rm[c] >> 24, tq);
                        col = pbr_shade(fr->light, ts.nh, ts.tt, ts.tb, Pc, b, col, nrm, rq, mq);
                    }
                    if (out->pv_tq && ts.first_point + c < out->point_cap) {
                        int64_t o = (ts.first_point + c) * nviews + r;
                        out->pv_tq[o] = (int16_t)tq;
                        out->pv_col[o] = col;
                    }
                    uint32_t zb;
                    memcpy(&zb, &Z, 4);
                    uint64_t key = ((uint64_t)zb << 32) | col;
                    uint64_t *dst = out->keys + (int64_t)r * px_per_view + y * fr->W + x;
                    if (key < *dst) *dst = key;
                }
        }
        free(cells_i); free(cells_j); free(tvmin); free(tvmax); free(flg); free(nmin); free(nmax); free(rm);
        free(ts.ilo); free(ts.ihi); free(ts.rowstart);
    }
    out->stats[0] = npts;
    free(vactive);
    return 0;
}

/* Key buffer -> RGBA8 colour and FP32 depth (cleared pixels: 0 and +inf). */
void orc_resolve(const uint64_t *keys, int64_t n, uint32_t *rgba, float *depth) {
    for (int64_t k = 0; k < n; ++k) {
        uint64_t key = keys[k];
        if (key == ~(uint64_t)0) { rgba[k] = 0; depth[k] = INFINITY; continue; }
        rgba[k] = (uint32_t)(key & 0xffffffffu);
        uint32_t zb = (uint32_t)(key >> 32);
        memcpy(&depth[k], &zb, 4);
    }
}

/* ------------------------------------------------------------------ */
/* Sec. 4: interleaving into the lenticular panel and reconstruction      */

typedef struct {
    int Wp, Hp, mode;
    uint32_t K1, Ky, K0;     /* lens phase constants, Q32 */
    const int64_t *taps;     /* 8 x (du Q32 view, dx Q8, dy Q8) */
} orc_lens;

void orc_interleave(const uint32_t *views, int V, int Wv, int Hv, const orc_lens *ln, uint8_t *panel) {
    for (int64_t Y = 0; Y < ln->Hp; ++Y)
        for (int64_t X = 0; X < ln->Wp; ++X) {
            int64_t xq = ((2 * X + 1) * (int64_t)Wv * 128) / ln->Wp;
            int64_t yq = ((2 * Y + 1) * (int64_t)Hv * 128) / ln->Hp;
            for (int c = 0; c < 3; ++c) {
                uint32_t phi = (uint32_t)((uint32_t)(3 * X + c) * ln->K1 + (uint32_t)Y * ln->Ky + ln->K0);
                uint64_t U = (uint64_t)phi * (uint64_t)V;
                uint32_t val;
                if (ln->mode == 0) {
                    int64_t v = (int64_t)(U >> 32), x = xq >> 8, y = yq >> 8;
                    val = (views[(v * Hv + y) * Wv + x] >> (8 * c)) & 255u;
                } else {
                    uint32_t sum = 0;
                    for (int k = 0; k < 8; ++k) {
                        int64_t du = (ln->mode & 2) ? ln->taps[k * 3] : 0;
                        int64_t dx = (ln->mode & 1) ? ln->taps[k * 3 + 1] : 0;
                        int64_t dy = (ln->mode & 1) ? ln->taps[k * 3 + 2] : 0;
                        int64_t v = ((int64_t)U + du) >> 32;
                        int64_t x = (xq + dx) >> 8, y = (yq + dy) >> 8;
                        v = v < 0 ? 0 : (v > V - 1 ? V - 1 : v);
                        x = x < 0 ? 0 : (x > Wv - 1 ? Wv - 1 : x);
                        y = y < 0 ? 0 : (y > Hv - 1 ? Hv - 1 : y);
                        sum += (views[(v * Hv + y) * Wv + x] >> (8 * c)) & 255u;
                    }
                    val = (sum + 4) >> 3;
                }
                panel[(Y * ln->Wp + X) * 3 + c] = (uint8_t)val;
            }
        }
}

/* Angular supersampling filter: n_sub sub-views -> V views with integer
 * Gaussian weights (host table: for view v, entries [v*maxe, v*maxe+cnt[v])). */
void orc_angular_filter(const uint32_t *sub, int V, int Wv, int Hv, const int32_t *cnt,
                        const int32_t *src, const uint32_t *wt, int maxe, uint32_t *outv) {
    int64_t npx = (int64_t)Wv * Hv;
    for (int v = 0; v < V; ++v) {
        uint64_t wsum = 0;
        for (int e = 0; e < cnt[v]; ++e) wsum += wt[v * maxe + e];
        for (int64_t p = 0; p < npx; ++p) {
            uint32_t o = 0;
            for (int c = 0; c < 4; ++c) {
                uint64_t acc = 0;
                for (int e = 0; e < cnt[v]; ++e)
                    acc += (uint64_t)wt[v * maxe + e] * ((sub[(int64_t)src[v * maxe + e] * npx + p] >> (8 * c)) & 255u);
                o |= (uint32_t)((acc + wsum / 2) / wsum) << (8 * c);
            }
            outv[(int64_t)v * npx + p] = o;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Gold standard: a conventional per-view z-buffer rasteriser (multiview   */
/* rendering, one pass per view) with perspective-correct attributes and   */
/* per-pixel trilinear mipmapping, all in double.                           */

static void trilinear_d(const orc_scene *sc, int t, double u, double v, double lod, double out[4]) {
    int size = sc->tex_size[t], L = sc->tex_levels[t];
    if (!(lod > 0.0)) lod = 0.0;
    if (lod > L - 1) lod = L - 1;
    int l0 = (int)floor(lod);
    int l1 = l0 + 1 < L ? l0 + 1 : L - 1;
    double f = lod - l0;
    double acc[2][4];
    int ls[2] = {l0, l1};
    for (int q = 0; q < 2; ++q) {
        int Wl = size >> ls[q];
        const uint8_t *lev = sc->texels + sc->tex_level_off[t * 16 + ls[q]];
        double x = u * Wl - 0.5, y = v * Wl - 0.5;
        double fx0 = floor(x), fy0 = floor(y);
        double ax = x - fx0, ay = y - fy0;
        int64_t ix = (int64_t)fx0, iy = (int64_t)fy0;
        int x0 = (int)(((ix % Wl) + Wl) % Wl), y0 = (int)(((iy % Wl) + Wl) % Wl);
        int x1 = (x0 + 1) % Wl, y1 = (y0 + 1) % Wl;
        for (int c = 0; c < 4; ++c) {
            double t00 = lev[((size_t)y0 * Wl + x0) * 4 + c], t10 = lev[((size_t)y0 * Wl + x1) * 4 + c];
            double t01 = lev[((size_t)y1 * Wl + x0) * 4 + c], t11 = lev[((size_t)y1 * Wl + x1) * 4 + c];
            acc[q][c] = (t00 * (1 - ax) + t10 * ax) * (1 - ay) + (t01 * (1 - ax) + t11 * ax) * ay;
        }
    }
    for (int c = 0; c < 4; ++c) out[c] = acc[0][c] * (1 - f) + acc[1][c] * f;
}

int orc_rasterise(const orc_scene *sc, const orc_frame *fr, uint32_t *rgba, float *depth) {
    const float *m = fr->model;
    int64_t npx = (int64_t)fr->W * fr->H;
    double *zbuf = (double *)malloc(sizeof(double) * (size_t)(npx * fr->n_views));
    for (int64_t k = 0; k < npx * fr->n_views; ++k) { zbuf[k] = INFINITY; rgba[k] = 0; depth[k] = INFINITY; }
    for (int t = 0; t < sc->nt; ++t) {
        v3 P[3];
        int zbad = 0;
        for (int k = 0; k < 3; ++k) {
            uint32_t vi = sc->idx[t * 3 + k];
            float px = sc->pos[vi * 3 + 0], py = sc->pos[vi * 3 + 1], pz = sc->pos[vi * 3 + 2];
            P[k].x = ((m[0] * px + m[1] * py) + m[2] * pz) + m[3];
            P[k].y = ((m[4] * px + m[5] * py) + m[6] * pz) + m[7];
            P[k].z = ((m[8] * px + m[9] * py) + m[10] * pz) + m[11];
            if (!(P[k].z >= fr->znear)) zbad = 1;
        }
        if (zbad) continue;
        v3 e1 = v3sub(P[1], P[0]), e2 = v3sub(P[2], P[0]);
        v3 n = v3cross(e1, e2);
        float nl = sqrtf((n.x * n.x + n.y * n.y) + n.z * n.z);
        if (!(nl > 0.0f) || isinf(nl)) continue;
        v3 nh = {n.x / nl, n.y / nl, n.z / nl};
        float h = v3dot(nh, P[0]);
        vproj pr[3];
        for (int k = 0; k < 3; ++k) pr[k] = vertex_proj(fr, P[k]);
        int tex = sc->tex[t];
        uint32_t i0 = sc->idx[t * 3], i1 = sc->idx[t * 3 + 1], i2 = sc->idx[t * 3 + 2];
        double u0 = sc->uv[i0 * 2], v0 = sc->uv[i0 * 2 + 1];
        double u1 = sc->uv[i1 * 2], v1 = sc->uv[i1 * 2 + 1];
        double u2 = sc->uv[i2 * 2], v2 = sc->uv[i2 * 2 + 1];
        double Ats = 0.5 * fabs((u1 - u0) * (v2 - v0) - (v1 - v0) * (u2 - u0));
        /* double-precision plane */
        double dP0[3] = {P[0].x, P[0].y, P[0].z}, dP1[3] = {P[1].x, P[1].y, P[1].z}, dP2[3] = {P[2].x, P[2].y, P[2].z};
        double de1[3] = {dP1[0] - dP0[0], dP1[1] - dP0[1], dP1[2] - dP0[2]};
        double de2[3] = {dP2[0] - dP0[0], dP2[1] - dP0[1], dP2[2] - dP0[2]};
        double dn[3] = {de1[1] * de2[2] - de1[2] * de2[1], de1[2] * de2[0] - de1[0] * de2[2], de1[0] * de2[1] - de1[1] * de2[0]};
        double dnl = sqrt(dn[0] * dn[0] + dn[1] * dn[1] + dn[2] * dn[2]);
        double Aws = 0.5 * dnl;
        double Xt = sc->tex_size[tex];
        for (int r = 0; r < fr->n_views; ++r) {
            float b = fr->eye[r];
            float delta = h - nh.x * b;
            if (!faces_eye(P[0], delta, b)) continue;
            int64_t qx[3], qy[3];
            int ok = 1;
            for (int k = 0; k < 3 && ok; ++k) ok = q8_xy(pr[k], b, &qx[k], &qy[k]);
            if (!ok) continue;
            int64_t a2 = (qx[1] - qx[0]) * (qy[2] - qy[0]) - (qy[1] - qy[0]) * (qx[2] - qx[0]);
            if (a2 == 0) continue;
            if (a2 < 0) {
                int64_t tx = qx[1]; qx[1] = qx[2]; qx[2] = tx;
                int64_t ty = qy[1]; qy[1] = qy[2]; qy[2] = ty;
            }
            int64_t xmin = imin64(qx[0], imin64(qx[1], qx[2])), xmax = imax64(qx[0], imax64(qx[1], qx[2]));
            int64_t ymin = imin64(qy[0], imin64(qy[1], qy[2])), ymax = imax64(qy[0], imax64(qy[1], qy[2]));
            int64_t X0 = imax64(0, -floordiv64(-(xmin - 128), 256)), X1 = imin64(fr->W - 1, floordiv64(xmax - 128, 256));
            int64_t Y0 = imax64(0, -floordiv64(-(ymin - 128), 256)), Y1 = imin64(fr->H - 1, floordiv64(ymax - 128, 256));
            double bd = b;
            double ddelta = (dn[0] * dP0[0] + dn[1] * dP0[1] + dn[2] * dP0[2]) / dnl - dn[0] / dnl * bd;
            for (int64_t y = Y0; y <= Y1; ++y)
                for (int64_t x = X0; x <= X1; ++x) {
                    int64_t pxq = 256 * x + 128, pyq = 256 * y + 128;
                    int in = 1;
                    for (int e = 0; e < 3 && in; ++e) {
                        int a = e, bb = (e + 1) % 3;
                        int64_t dx = qx[bb] - qx[a], dy = qy[bb] - qy[a];
                        int64_t E = dx * (pyq - qy[a]) - dy * (pxq - qx[a]);
                        int owns = dy > 0 || (dy == 0 && dx > 0);
                        in = E > 0 || (E == 0 && owns);
                    }
                    if (!in) continue;
                    double rx = (x + 0.5 - (double)fr->cx) / (double)fr->fx - bd / (1.0 / (double)fr->rD);
                    double ry = (y + 0.5 - (double)fr->cy) / (double)fr->fy;
                    double den = (dn[0] * rx + dn[1] * ry + dn[2]) / dnl;
                    double Z = ddelta / den;
                    if (!(Z > 0.0)) continue;
                    int64_t k = (int64_t)r * npx + y * fr->W + x;
                    if (!(Z < zbuf[k])) continue;
                    double X[3] = {bd + Z * rx, Z * ry, Z};
                    /* barycentrics of the hit point */
                    double q[3] = {X[0] - dP0[0], X[1] - dP0[1], X[2] - dP0[2]};
                    double c1[3] = {q[1] * de2[2] - q[2] * de2[1], q[2] * de2[0] - q[0] * de2[2], q[0] * de2[1] - q[1] * de2[0]};
                    double c2[3] = {de1[1] * q[2] - de1[2] * q[1], de1[2] * q[0] - de1[0] * q[2], de1[0] * q[1] - de1[1] * q[0]};
                    double nn = dn[0] * dn[0] + dn[1] * dn[1] + dn[2] * dn[2];
                    double b1 = (c1[0] * dn[0] + c1[1] * dn[1] + c1[2] * dn[2]) / nn;
                    double b2 = (c2[0] * dn[0] + c2[1] * dn[1] + c2[2] * dn[2]) / nn;
                    double uu = u0 + b1 * (u1 - u0) + b2 * (u2 - u0);
                    double vv = v0 + b1 * (v1 - v0) + b2 * (v2 - v0);
                    double lod = 0.0;
                    if (fr->mip) {
                        double foot = Z * Z * Z / ((double)fr->fx * (double)fr->fy * fabs(ddelta));
                        double a = foot * (Ats / Aws) * Xt * Xt;
                        lod = a > 0 ? 0.5 * log2(a) : 0.0;
                    }
                    double col[4];
                    trilinear_d(sc, tex, uu, vv, lod, col);
                    uint32_t o = 0;
                    for (int c = 0; c < 4; ++c) {
                        long vq = lround(col[c]);
                        vq = vq < 0 ? 0 : (vq > 255 ? 255 : vq);
                        o |= (uint32_t)vq << (8 * c);
                    }
                    zbuf[k] = Z;
                    rgba[k] = o;
                    depth[k] = (float)Z;
                }
        }
    }
    free(zbuf);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Helpers exposed for the pins in the test-suite.                        */

/* Emission rule on given Q8 lattice vertices: writes the emitted cells in
 * emission order (row-major, rows ascending) and returns their number, or -1
 * when more than `cap` cells would be written. */
int orc_lattice_cells(const int64_t S[3], const int64_t T[3], int cap, int32_t *ci, int32_t *cj) {
    tri_state ts;
    memset(&ts, 0, sizeof ts);
    for (int k = 0; k < 3; ++k) { ts.S[k] = S[k]; ts.T[k] = T[k]; }
    ts.area2 = (S[1] - S[0]) * (T[2] - T[0]) - (T[1] - T[0]) * (S[2] - S[0]);
    int64_t mins = imin64(S[0], imin64(S[1], S[2])), maxs = imax64(S[0], imax64(S[1], S[2]));
    int64_t mint = imin64(T[0], imin64(T[1], T[2])), maxt = imax64(T[0], imax64(T[1], T[2]));
    int n = 0;
    for (int64_t j = floordiv64(mint, 256) - 1; j <= floordiv64(maxt, 256) + 1; ++j)
        for (int64_t i = floordiv64(mins, 256) - 1; i <= floordiv64(maxs, 256) + 1; ++i)
            if (cell_overlaps(&ts, i, j)) {
                if (n == cap) return -1;
                ci[n] = (int32_t)i; cj[n] = (int32_t)j; ++n;
            }
    return n;
}

void orc_closest_point(const float p[3], const float a[3], const float b[3], const float c[3], float out[3]) {
    v3 P = {p[0], p[1], p[2]}, A = {a[0], a[1], a[2]}, B = {b[0], b[1], b[2]}, C = {c[0], c[1], c[2]};
    v3 r = closest_on_triangle(P, A, B, C);
    out[0] = r.x; out[1] = r.y; out[2] = r.z;
}

uint32_t orc_trilinear(const orc_scene *sc, int t, float u, float v, int kc) { return trilinear(sc, t, u, v, kc); }
int orc_lod_q8(float a) { return lod_q8(a); }

/* PBR pieces for the pins: tangent frame, BRDF terms, shaded RGBA8. */
void orc_tangent_frame(const float e1[3], const float e2[3], const float uv[4], const float nh[3], const float u[3],
                       const float w[3], float out[6]) {
    v3 a = {e1[0], e1[1], e1[2]}, b = {e2[0], e2[1], e2[2]}, n = {nh[0], nh[1], nh[2]};
    v3 uu = {u[0], u[1], u[2]}, ww = {w[0], w[1], w[2]}, T, B;
    tangent_frame(a, b, uv[0], uv[1], uv[2], uv[3], n, uu, ww, &T, &B);
    out[0] = T.x; out[1] = T.y; out[2] = T.z; out[3] = B.x; out[4] = B.y; out[5] = B.z;
}

void orc_pbr_terms(const float n[3], const float v[3], const float L[3], float rgh, float mtl, const float a[3],
                   float out[10]) {
    v3 nn = {n[0], n[1], n[2]}, vv = {v[0], v[1], v[2]}, LL = {L[0], L[1], L[2]};
    pbr_terms T;
    pbr_eval(nn, vv, LL, rgh, mtl, a, &T);
    out[0] = T.D; out[1] = T.G; out[2] = T.NL; out[3] = T.NV;
    for (int c = 0; c < 3; ++c) { out[4 + c] = T.F[c]; out[7 + c] = T.f[c]; }
}

uint32_t orc_pbr_shade(const float light[9], const float frame[9], const float Pc[3], float b, uint32_t alb,
                       uint32_t nrm, uint32_t rq, uint32_t mq) {
    v3 nh = {frame[6], frame[7], frame[8]}, tt = {frame[0], frame[1], frame[2]}, tb = {frame[3], frame[4], frame[5]};
    v3 P = {Pc[0], Pc[1], Pc[2]};
    return pbr_shade(light, nh, tt, tb, P, b, alb, nrm, rq, mq);
}
