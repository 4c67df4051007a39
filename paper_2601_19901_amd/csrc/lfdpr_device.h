// Device-side arithmetic of the LFDPR hot path for gfx950.
//
// Every floating-point expression is binary32 with round-to-nearest-even, no
// contraction (the library is built with -ffp-contract=off and correctly
// rounded division/sqrt), evaluated exactly as parenthesised, so that point
// counts, point attributes and per-pixel keys are reproducible bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define LF_HD __host__ __device__ __forceinline__

namespace lfdpr {

constexpr uint32_t F_ILO = 1u, F_IHI = 2u, F_JLO = 4u, F_JHI = 8u;
constexpr int kCellCap = 65536;          // cells per triangle before overflow
constexpr uint32_t kBigCells = 96;       // triangles with more cells are emitted by a whole workgroup
constexpr int64_t kBoxCap = 1ll << 22;   // lattice bounding-box cells before overflow
constexpr int64_t kEpsQ8 = 4;            // cell dilation, 4/256 of a cell
constexpr float kGuard = 32768.0f;       // screen guard band, pixels

// Per-triangle record read by the splat kernel (128 B, 8 x float4).
struct alignas(16) TriRec {
  float p0x, p0y, p0z, h;      // camera-space vertex 0; plane offset n.P0
  float nx, ny, nz, sx;        // unit normal; horizontal sampling density
  float ux, uy, uz, sy;        // lattice s axis; vertical sampling density
  float wx, wy, wz, ruv;       // lattice t axis; texture/world area ratio
  float a0, c0, y0, smin;      // projected vertex 0 (x = a - b*c), Eqs. 4-5 minimum
  float a1, c1, y1, smax;      // projected vertex 1, Eqs. 4-5 maximum
  float a2, c2, y2, irange;    // projected vertex 2; 1/(smax - smin) (0 when equal)
  float cu0, cw0;              // u.P0 and w.P0 without their x terms
  int32_t item, pad1;          // batch item the triangle belongs to
};

// Per-triangle emission data (64 B).
struct alignas(16) TriEmit {
  float uv0u, uv0v, du1, dv1;
  float du2, dv2;
  int32_t s1, t1;
  int32_t s2, t2, kmin, kmax;
  int32_t tex, item;
  int32_t jlo, jhi;  // first and last lattice rows with cells
};

// One point: 16 B.  tri | flags<<28, (u16)i | (u16)j<<16, tv_min, tv_max (RGBA8).
struct alignas(16) Point {
  uint32_t tri_flags, ij, tvmin, tvmax;
};

// Per-point splat data (48 B) for the triangle-major splat, written with the
// point's mip colours: the four corners of the point's splat rectangle
// (lattice cell, extended by one cell beyond a row or column end) projected
// except for the eye offset (x = cA - b*cC in the view with eye offset b),
// the pixel rows the rectangle covers (view independent; kAllRows when a
// corner lies behind z_near/2: then no box limit), the cube of the cell-centre
// depth (Eq. 8) and the two mip colours (Eq. 9).
struct alignas(16) PointBox {
  float cA[4];
  float cC[4];
  float zc3;
  int32_t rows;  // (u16)first row | (u16)last row << 16
  uint32_t tvmin, tvmax;
};
constexpr int32_t kAllRows = (int32_t)0x7FFF8000;  // first row -32768, last 32767

// One row j of a triangle's lattice, stored at (triangle's first point) + (j -
// jlo): the row's first point relative to the triangle's first point, and the
// row's cell range [ilo, ihi].
struct alignas(8) RowEntry {
  uint32_t start;
  int16_t ilo, ihi;
};

struct TexInfo {
  int32_t size, levels;
  int64_t off[16];  // byte offset of each level in the texel pool
};

// Per-triangle material record of the physically based mode (64 B): normal,
// roughness and metallic textures with their LOD pairs (Eqs. 6-7, 1/256
// level) and the tangent frame (T, B) of the texture mapping, camera space.
struct alignas(16) TriMat {
  int32_t texn, texr, texm, pad0;
  int32_t kn0, kn1, kr0, kr1;
  int32_t km0, km1;
  float tx, ty;
  float tz, bx, by, bz;
};

// One directional light (unit direction towards it, camera space), its RGB
// radiance and the ambient RGB.
struct Shading {
  float lx, ly, lz, lr, lg, lb, ar, ag, ab;
};

struct Rig {
  int32_t n_views, W, H, mip;
  float fx, fy, cx, cy, rD, znear, fxfy;
  float eye_lo, eye_hi;  // smallest and largest eye offset of the table
  const float* eye;     // n_views
  const float* kshift;  // n_views
};

struct Model {
  float m[12];
};

LF_HD float clamp_big(float x) {
  if (!(x > -1073741824.0f)) return -1073741824.0f;
  if (x > 1073741824.0f) return 1073741824.0f;
  return x;
}

LF_HD int64_t floor_div(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  if ((a % b) != 0 && a < 0) q -= 1;
  return q;
}
// floor(a / b) for b > 0 and |a| < 2^53, b < 2^53: the correctly rounded double
// quotient is within one of the floor (|a / b| < 2^48 here, so its error is
// below 1/32), and one integer check settles it; q * b stays near a.  Much
// cheaper on the GPU than a 64-bit integer division.
LF_HD int64_t floor_div_53(int64_t a, int64_t b) {
  int64_t q = (int64_t)floor((double)a / (double)b);
  const int64_t r = a - q * b;
  if (r < 0) q -= 1;
  else if (r >= b) q += 1;
  return q;
}

LF_HD int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
LF_HD int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }

// ---------------------------------------------------------------- projection
// x = A - b*C with A = cx + fx*(X/Z), C = fx*(1/Z - 1/D); y = cy + fy*(Y/Z).
LF_HD void vertex_proj(const Rig& rg, float X, float Y, float Z, float& A, float& C, float& Yp) {
  A = rg.cx + rg.fx * (X / Z);
  C = rg.fx * (1.0f / Z - rg.rD);
  Yp = rg.cy + rg.fy * (Y / Z);
}

LF_HD bool q8_xy(float A, float C, float Yp, float b, int32_t& qx, int32_t& qy) {
  float x = A - b * C;
  if (!(fabsf(x) < kGuard) || !(fabsf(Yp) < kGuard)) return false;
  qx = (int32_t)rintf(x * 256.0f);
  qy = (int32_t)rintf(Yp * 256.0f);
  return true;
}

// The eye at (b, 0, 0) sees the triangle's front more than edge-on: delta =
// n.(P0 - e) < 0 and |delta| >= |P0 - e|/256 (the eye direction at least
// asin(1/256) off the plane; nearer edge-on the ray-plane map magnifies the
// 1/256-px vertex snap without bound).  p0y2 = P0y*P0y, p0z2 = P0z*P0z.
LF_HD bool faces_eye(float p0x, float p0y2, float p0z2, float delta, float b) {
  const float dx = p0x - b;
  const float d2 = (dx * dx + p0y2) + p0z2;
  return delta < 0.0f && delta * delta >= d2 * 0x1p-16f;
}

// View r is active for the triangle: facing the eye (above), inside the guard
// band, and not entirely beyond one screen edge.  Fills the Q8 vertices on
// success.
LF_HD bool view_active(const Rig& rg, const TriRec& t, float b, int32_t qx[3], int32_t qy[3]) {
  float delta = t.h - t.nx * b;
  if (!faces_eye(t.p0x, t.p0y * t.p0y, t.p0z * t.p0z, delta, b)) return false;
  if (!q8_xy(t.a0, t.c0, t.y0, b, qx[0], qy[0])) return false;
  if (!q8_xy(t.a1, t.c1, t.y1, b, qx[1], qy[1])) return false;
  if (!q8_xy(t.a2, t.c2, t.y2, b, qx[2], qy[2])) return false;
  int32_t W8 = 256 * rg.W, H8 = 256 * rg.H;
  if (qx[0] < 0 && qx[1] < 0 && qx[2] < 0) return false;
  if (qx[0] > W8 && qx[1] > W8 && qx[2] > W8) return false;
  if (qy[0] < 0 && qy[1] < 0 && qy[2] < 0) return false;
  if (qy[0] > H8 && qy[1] > H8 && qy[2] > H8) return false;
  return true;
}

// ---------------------------------------------------------------- geometry
struct F3 {
  float x, y, z;
};
LF_HD F3 sub3(F3 a, F3 b) { return F3{a.x - b.x, a.y - b.y, a.z - b.z}; }
LF_HD float dot3(F3 a, F3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
LF_HD F3 axpy3(F3 a, float s, F3 d) { return F3{a.x + s * d.x, a.y + s * d.y, a.z + s * d.z}; }

// False only for a triangle that no view of the rig can see (view_active is
// false for every eye offset in [eye_lo, eye_hi]), told from the two ends of
// the range: the plane distance delta = h - nx*b and each projected x = a - b*c
// are monotone in b (a product with a fixed factor and a difference with a
// fixed term keep their order under rounding), and the projected rows do not
// depend on b.  So the triangle is behind its plane for every eye, or its rows
// are off the view or outside the guard band, or all its vertices are left of
// (right of) the view at both ends and hence for every eye.  The record needs
// h, nx, a/c/y of the three vertices.
LF_HD bool may_be_seen(const Rig& rg, const TriRec& R) {
  if (R.h - R.nx * rg.eye_lo >= 0.0f && R.h - R.nx * rg.eye_hi >= 0.0f) return false;
  if (!(fabsf(R.y0) < kGuard) || !(fabsf(R.y1) < kGuard) || !(fabsf(R.y2) < kGuard)) return false;
  const int32_t H8 = 256 * rg.H;
  const int32_t qy0 = (int32_t)rintf(R.y0 * 256.0f), qy1 = (int32_t)rintf(R.y1 * 256.0f),
                qy2 = (int32_t)rintf(R.y2 * 256.0f);
  if ((qy0 < 0 && qy1 < 0 && qy2 < 0) || (qy0 > H8 && qy1 > H8 && qy2 > H8)) return false;
  // x * 256 < -0.5 rounds below 0; x * 256 > W8 + 0.5 rounds above W8
  const float W8h = (float)(256 * rg.W) + 0.5f;
  const float xl0 = R.a0 - rg.eye_lo * R.c0, xh0 = R.a0 - rg.eye_hi * R.c0;
  const float xl1 = R.a1 - rg.eye_lo * R.c1, xh1 = R.a1 - rg.eye_hi * R.c1;
  const float xl2 = R.a2 - rg.eye_lo * R.c2, xh2 = R.a2 - rg.eye_hi * R.c2;
  if (fmaxf(xl0, xh0) * 256.0f < -0.5f && fmaxf(xl1, xh1) * 256.0f < -0.5f && fmaxf(xl2, xh2) * 256.0f < -0.5f)
    return false;
  if (fminf(xl0, xh0) * 256.0f > W8h && fminf(xl1, xh1) * 256.0f > W8h && fminf(xl2, xh2) * 256.0f > W8h)
    return false;
  return true;
}

// Point of triangle abc nearest to p, by the Voronoi regions of its vertices,
// edges and face (Ericson, Real-Time Collision Detection, Sec. 5.1.5).
LF_HD F3 nearest_on_triangle(F3 p, F3 a, F3 b, F3 c) {
  F3 ab = sub3(b, a), ac = sub3(c, a);
  F3 ap = sub3(p, a);
  float d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  if (d1 <= 0.0f && d2 <= 0.0f) return a;
  F3 bp = sub3(p, b);
  float d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  if (d3 >= 0.0f && d4 <= d3) return b;
  float vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f) return axpy3(a, d1 / (d1 - d3), ab);
  F3 cp = sub3(p, c);
  float d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  if (d6 >= 0.0f && d5 <= d6) return c;
  float vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) return axpy3(a, d2 / (d2 - d6), ac);
  float va = d3 * d6 - d5 * d4;
  float e43 = d4 - d3, e56 = d5 - d6;
  if (va <= 0.0f && e43 >= 0.0f && e56 >= 0.0f) return axpy3(b, e43 / (e43 + e56), sub3(c, b));
  float inv = 1.0f / ((va + vb) + vc);
  return axpy3(axpy3(a, vb * inv, ab), vc * inv, ac);
}

// ---------------------------------------------------------------- lattice
// Conservative cell rule: cell (i,j)'s box [256i-4, 256i+260] x [256j-4, 256j+260]
// (Q8) overlaps the snapped triangle with positive area.  The two box axes give
// the bounding ranges below; each of the three edges bounds i within a row.  A
// snapped triangle of zero area (a point or a segment) keeps every cell that
// passes the box-axis test.
struct Lattice {
  int64_t S[3], T[3];
  int64_t sg;                 // sign of the doubled area (0: degenerate)
  int64_t iA, iB, jA, jB;     // cells passing the box-axis test
};

LF_HD void lattice_init(Lattice& L, int32_t s1, int32_t t1, int32_t s2, int32_t t2) {
  L.S[0] = 128; L.T[0] = 128;
  L.S[1] = s1; L.T[1] = t1;
  L.S[2] = s2; L.T[2] = t2;
  int64_t a2 = (L.S[1] - L.S[0]) * (L.T[2] - L.T[0]) - (L.T[1] - L.T[0]) * (L.S[2] - L.S[0]);
  L.sg = a2 > 0 ? 1 : (a2 < 0 ? -1 : 0);
  int64_t mins = imin(L.S[0], imin(L.S[1], L.S[2])), maxs = imax(L.S[0], imax(L.S[1], L.S[2]));
  int64_t mint = imin(L.T[0], imin(L.T[1], L.T[2])), maxt = imax(L.T[0], imax(L.T[1], L.T[2]));
  L.iA = floor_div(mins - kEpsQ8, 256);
  L.iB = floor_div(maxs + kEpsQ8 - 1, 256);
  L.jA = floor_div(mint - kEpsQ8, 256);
  L.jB = floor_div(maxt + kEpsQ8 - 1, 256);
}

// Emitted i-range [lo, hi] of row j (empty when lo > hi).
// Cell range [lo, hi] of lattice row j.  Magnitudes: Q8 vertices below 2^22
// (|s|, |t| < 16384 cells), so edge coefficients stay below 2^23, the row's
// edge offsets below 2^48 and the divisors below 2^31 (floor_div_53's range).
LF_HD void lattice_row(const Lattice& L, int64_t j, int64_t& lo, int64_t& hi) {
  lo = L.iA;
  hi = L.iB;
  if (L.sg == 0) return;
  int64_t y0 = 256 * j - kEpsQ8, y1 = 256 * j + 256 + kEpsQ8;
  for (int e = 0; e < 3; ++e) {
    int a = e, b = e == 2 ? 0 : e + 1;
    int64_t dx = L.S[b] - L.S[a], dy = L.T[b] - L.T[a];
    // E(x,y) = alpha*x + beta*y + gamma, interior positive
    int64_t alpha = -L.sg * dy, beta = L.sg * dx;
    int64_t gamma = L.sg * (dy * L.S[a] - dx * L.T[a]);
    int64_t c = beta * (beta > 0 ? y1 : y0) + gamma;
    if (alpha > 0) {
      // alpha*(256 i + 260) + c > 0
      lo = imax(lo, floor_div_53(-c - (256 + kEpsQ8) * alpha, 256 * alpha) + 1);
    } else if (alpha < 0) {
      // -a'*(256 i - 4) + c > 0  <=>  256 a' i < c + 4 a'
      int64_t ap = -alpha;
      int64_t num = c + kEpsQ8 * ap;
      // i < num / (256 ap)  <=>  i <= ceil(num / (256 ap)) - 1
      hi = imin(hi, floor_div_53(num - 1, 256 * ap));
    } else if (!(c > 0)) {
      lo = 1;
      hi = 0;
      return;
    }
  }
}

// ---------------------------------------------------------------- level of detail
// Eqs. 6-7: LOD = 0.5 log2(a), in units of 1/256 level, rounded to nearest:
// round(128 log2 a) = 128 e - 128 + #{k : thr[k] <= m} for a = m 2^e with
// m in [0.5, 1), where thr[k] is 2^((k - 127.5)/128) rounded up to a float
// (so the comparison with the float m is exact).
LF_HD int32_t lod_q8(const float* thr, float a) {
  if (!(a > 0.0f)) return -(1 << 30);
  if (__builtin_isinf(a)) return 1 << 30;
  int e;
  float m = frexpf(a, &e);
  int lo = 0, hi = 128;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (thr[mid] <= m) lo = mid + 1; else hi = mid;
  }
  return 128 * e - 128 + lo;
}

// ---------------------------------------------------------------- textures
LF_HD void bilinear_q16(const uint8_t* lev, int Wl, float u, float v, uint32_t out[4]) {
  float sc = (float)(Wl * 256);
  float tx = clamp_big(u * sc - 128.0f);
  float ty = clamp_big(v * sc - 128.0f);
  int32_t ix = (int32_t)floorf(tx), iy = (int32_t)floorf(ty);
  int32_t m = Wl - 1;
  int32_t x0 = (ix >> 8) & m, y0 = (iy >> 8) & m;
  int32_t x1 = (x0 + 1) & m, y1 = (y0 + 1) & m;
  uint32_t ax = (uint32_t)(ix & 255), ay = (uint32_t)(iy & 255);
  uint32_t w00 = (256u - ax) * (256u - ay), w10 = ax * (256u - ay);
  uint32_t w01 = (256u - ax) * ay, w11 = ax * ay;
  const uint32_t* t = reinterpret_cast<const uint32_t*>(lev);
  uint32_t t00 = t[(int64_t)y0 * Wl + x0], t10 = t[(int64_t)y0 * Wl + x1];
  uint32_t t01 = t[(int64_t)y1 * Wl + x0], t11 = t[(int64_t)y1 * Wl + x1];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int sh = 8 * c;
    out[c] = w00 * ((t00 >> sh) & 255u) + w10 * ((t10 >> sh) & 255u) + w01 * ((t01 >> sh) & 255u) +
             w11 * ((t11 >> sh) & 255u);
  }
}

LF_HD uint32_t trilinear(const uint8_t* pool, const TexInfo& ti, float u, float v, int32_t kc) {
  int32_t l0 = kc >> 8, f = kc & 255;
  int32_t l1 = l0 + 1 < ti.levels ? l0 + 1 : ti.levels - 1;
  uint32_t c0[4], c1[4] = {0u, 0u, 0u, 0u};
  bilinear_q16(pool + ti.off[l0], ti.size >> l0, u, v, c0);
  if (l1 != l0 && f != 0) bilinear_q16(pool + ti.off[l1], ti.size >> l1, u, v, c1);
  uint32_t r = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uint32_t acc = (uint32_t)(256 - f) * c0[c] + (uint32_t)f * c1[c];
    r |= ((acc + (1u << 23)) >> 24) << (8 * c);
  }
  return r;
}

// ---------------------------------------------------------------- shading
constexpr float kInv255 = 0x1.010102p-8f;     // binary32 nearest 1/255
constexpr float kTwoInv255 = 0x1.010102p-7f;  // binary32 nearest 2/255 (= 2 kInv255 exactly)
constexpr float kPiF = 0x1.921fb6p+1f;        // binary32 nearest pi
constexpr float kInvPiF = 0x1.45f306p-2f;     // binary32 nearest 1/pi

LF_HD F3 scale3(F3 a, float s) { return F3{a.x * s, a.y * s, a.z * s}; }

// Tangent frame of a triangle's texture mapping: dP/du and dP/dv from the two
// edges and their UV differences; T = dP/du without its normal component,
// normalised; B = n x T, turned to the side of dP/dv.  Degenerate mappings
// take the lattice axes (u, w).
LF_HD void texture_frame(F3 e1, F3 e2, float du1, float dv1, float du2, float dv2, F3 n, F3 u, F3 w, F3& T,
                         F3& B) {
  const float det = du1 * dv2 - dv1 * du2;
  F3 dpu = u, dpv = w;
  if (det != 0.0f) {
    const float rd = 1.0f / det;
    dpu = F3{(e1.x * dv2 - e2.x * dv1) * rd, (e1.y * dv2 - e2.y * dv1) * rd, (e1.z * dv2 - e2.z * dv1) * rd};
    dpv = F3{(e2.x * du1 - e1.x * du2) * rd, (e2.y * du1 - e1.y * du2) * rd, (e2.z * du1 - e1.z * du2) * rd};
  }
  const float along = dot3(n, dpu);
  F3 t{dpu.x - n.x * along, dpu.y - n.y * along, dpu.z - n.z * along};
  const float len = sqrtf(dot3(t, t));
  if (len > 0.0f && !__builtin_isinf(len)) t = scale3(t, 1.0f / len);
  else t = u;
  F3 b{n.y * t.z - n.z * t.y, n.z * t.x - n.x * t.z, n.x * t.y - n.y * t.x};
  if (dot3(b, dpv) < 0.0f) b = F3{-b.x, -b.y, -b.z};
  T = t;
  B = b;
}

// Unit vector along v, or `fallback` when v has no finite non-zero length.
LF_HD F3 unit_or(F3 v, F3 fallback) {
  const float len = sqrtf(dot3(v, v));
  if (len > 0.0f && !__builtin_isinf(len)) return scale3(v, 1.0f / len);
  return fallback;
}

// Physically based colour of a splat in the view whose eye sits at (b, 0, 0):
// Cook-Torrance with a GGX distribution (alpha = roughness^2), Smith-Schlick
// geometry (k = (r+1)^2/8), Schlick Fresnel (F0 = 0.04 (1-m) + albedo m), a
// diffuse share (1-F)(1-m) albedo/pi, one directional light plus ambient,
// tone mapped as sqrt(x/(1+x)).  Inputs: albedo, tangent-space normal (RGB =
// (n+1)/2), roughness and metallic bytes, interpolated with tau (Eq. 9); the
// surface point is the cell centre pc; alpha is the albedo's.
LF_HD uint32_t shade_splat(const Shading& L, F3 ng, F3 T, F3 B, F3 pc, float b, uint32_t alb, uint32_t nrm,
                           uint32_t rq, uint32_t mq) {
  const float ar = (float)(alb & 255u) * kInv255;
  const float ag = (float)((alb >> 8) & 255u) * kInv255;
  const float ab = (float)((alb >> 16) & 255u) * kInv255;
  const float tr = (float)(nrm & 255u) * kTwoInv255 - 1.0f;
  const float tg = (float)((nrm >> 8) & 255u) * kTwoInv255 - 1.0f;
  const float tb = (float)((nrm >> 16) & 255u) * kTwoInv255 - 1.0f;
  const F3 n = unit_or(F3{(tr * T.x + tg * B.x) + tb * ng.x, (tr * T.y + tg * B.y) + tb * ng.y,
                          (tr * T.z + tg * B.z) + tb * ng.z}, ng);
  const F3 v = unit_or(F3{b - pc.x, 0.0f - pc.y, 0.0f - pc.z}, F3{0.0f, 0.0f, -1.0f});
  const F3 l{L.lx, L.ly, L.lz};
  const F3 h = unit_or(F3{l.x + v.x, l.y + v.y, l.z + v.z}, n);
  float nl = dot3(n, l), nv = dot3(n, v), nh = dot3(n, h), vh = dot3(v, h);
  nl = nl > 0.0f ? nl : 0.0f;
  nv = nv > 0.0f ? nv : 0.0f;
  nh = nh > 0.0f ? nh : 0.0f;
  vh = vh > 0.0f ? vh : 0.0f;
  float r = (float)rq * kInv255;
  r = r > 0.03f ? r : 0.03f;
  const float m = (float)mq * kInv255;
  const float alpha = r * r, a2 = alpha * alpha;
  const float dd = (nh * nh) * (a2 - 1.0f) + 1.0f;
  const float D = a2 / ((kPiF * dd) * dd);
  const float k = ((r + 1.0f) * (r + 1.0f)) * 0.125f;
  const float G = (nl / (nl * (1.0f - k) + k)) * (nv / (nv * (1.0f - k) + k));
  const float c1 = 1.0f - vh;
  const float c5 = ((c1 * c1) * (c1 * c1)) * c1;
  const float spec = (D * G) / (((4.0f * nl) * nv) + 1e-4f);
  const float alb3[3] = {ar, ag, ab}, rad[3] = {L.lr, L.lg, L.lb}, amb[3] = {L.ar, L.ag, L.ab};
  uint32_t out = alb & 0xFF000000u;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float F0 = 0.04f * (1.0f - m) + alb3[c] * m;
    const float F = F0 + (1.0f - F0) * c5;
    const float kd = (1.0f - F) * (1.0f - m);
    const float f = (kd * alb3[c]) * kInvPiF + F * spec;
    const float lo = f * (rad[c] * nl) + amb[c] * alb3[c];
    const float t = lo / (1.0f + lo);
    const float y = floorf(sqrtf(t) * 255.0f + 0.5f);
    const uint32_t q = y >= 255.0f ? 255u : (y > 0.0f ? (uint32_t)y : 0u);
    out |= q << (8 * c);
  }
  return out;
}

}  // namespace lfdpr
