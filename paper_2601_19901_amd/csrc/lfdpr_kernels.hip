// HIP kernels of the LFDPR hot path for gfx950 (wave64).
//
//   k_tri_setup   one lane per triangle: frame transform, visibility in every
//                 LFD view, T_align frame, LFD-biased H/V densities, Eqs. 1-7,
//                 lattice snap and cell count; each workgroup's count sum
//                 and the list of triangles with many cells    (Sec. 3, 3.1, 3.3)
//   k_scan_top    one workgroup: the workgroups' count sums -> point offset bases
//   k_emit        one lane per triangle: its point offset and its cells in
//                 deterministic order; triangles with many cells: one
//                 workgroup each, rows over lanes (same launch)
//   k_fetch       one lane per point: UV at the cell centre, two trilinear
//                 mip fetches (tv_min, tv_max)                (Sec. 3.3); for
//                 the triangle-view order and the quilt also the point's
//                 splat rectangle (and, for the quilt, its pixel rows)
//   k_splat       one lane per point, looping over the views: splat box,
//                 inside-triangle test, cell ownership, Eqs. 8-9, 64-bit
//                 atomicMin of (depth, colour)                (Sec. 3.2, 3.3, 5.1)
//   k_qcount, k_qplan, k_qscatter   the quilt's band lists: points binned by
//                 the pixel rows their splat reaches           (Sec. 3.2)
//   k_splat_quilt one workgroup per tile (a band of rows x a subset of the
//                 views): the same splat with the 64-bit keys in LDS, the
//                 tile written out as RGBA8 (+ depth)          (Sec. 3.2, 5.1)
//   k_splat_tv    per (triangle, view): covered pixels find their owning point
//   k_resolve     keys -> RGBA8 (+ depth), keys re-cleared for the next frame
//   k_interleave  one lane per four panel pixels: tilted-lens phase, view and
//                 pixel index, optional 8-tap Gaussian reconstruction (Sec. 4)
//   k_angular_filter  sub-views -> views (angular supersampling, Sec. 4), one
//                 lane per four pixels
#include "lfdpr_device.h"
#include "lfdpr_internal.h"

namespace lfdpr {

// ------------------------------------------------------------------ utilities

__global__ void k_fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// The single-frame item table, written from a kernel argument (no host staging).
__global__ void k_store_item(Item it, Item* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = it;
}

// Frame statistics for the caller: points, active triangles, point-views,
// overflowed triangles, written pixels, point capacity.
__global__ void k_export_stats(const uint64_t* __restrict__ st, int64_t cap, int64_t* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[0] = (int64_t)st[STAT_TOTAL];
    out[1] = (int64_t)st[STAT_ACTIVE];
    out[2] = (int64_t)st[STAT_POINT_VIEWS];
    out[3] = (int64_t)st[STAT_OVERFLOW];
    out[4] = (int64_t)st[STAT_WRITTEN];
    out[5] = cap;
  }
}

__global__ void k_build_mip(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int s) {
  int h = s >> 1;
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)h * h) return;
  int y = (int)(k / h), x = (int)(k % h);
  uint32_t a = src[(int64_t)(2 * y) * s + 2 * x], b = src[(int64_t)(2 * y) * s + 2 * x + 1];
  uint32_t c = src[(int64_t)(2 * y + 1) * s + 2 * x], d = src[(int64_t)(2 * y + 1) * s + 2 * x + 1];
  uint32_t r = 0;
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
    int sh = 8 * ch;
    uint32_t m = (((a >> sh) & 255u) + ((b >> sh) & 255u) + ((c >> sh) & 255u) + ((d >> sh) & 255u) + 2u) >> 2;
    r |= m << sh;
  }
  dst[k] = r;
}

// wave64 inclusive scan of one uint64 per lane
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Slot of this lane in a list shared by the grid when `take`: one atomic per wave.
__device__ __forceinline__ uint64_t wave_append(bool take, uint64_t* counter) {
  const uint64_t mask = __builtin_amdgcn_ballot_w64(take);
  if (!mask) return 0;
  const int lane = threadIdx.x & 63;
  const int leader = __builtin_ctzll(mask);
  uint64_t base = 0;
  if (lane == leader) base = atomicAdd((unsigned long long*)counter, (unsigned long long)__builtin_popcountll(mask));
  base = __shfl(base, leader, 64);
  const uint64_t below = lane ? (mask & (~0ull >> (64 - lane))) : 0ull;
  return base + (uint64_t)__builtin_popcountll(below);
}

// ------------------------------------------------------------------ a1/a2: triangle setup

// kMulti: triangles of several items (a batch), each lane finds its own; else
// every triangle belongs to items[0], whose rig then sits in scalar registers.
// kLean: the triangle's records are stored before its lattice count (only the
// row range after it), so none of them is held in registers across the row
// loop: 88 VGPRs (5 waves per SIMD) instead of 158 (3 waves).  A triangle
// whose count then overflows keeps records that nothing reads.  Which form
// makes the faster frame depends on the splat that runs beside the next
// frame's set-up: next to the quilt's whole-CU tiles the set-up gets whole
// CUs between tiles and the lean form is faster; next to the point splat,
// whose workgroups retire one at a time, the lean form fits into each freed
// slot and then slows the splat more than it gains.
template <bool kMulti, bool kLean>
__global__ void __launch_bounds__(256) k_tri_setup(SetupArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t act_cnt = 0, ovf_cnt = 0, pv_cnt = 0;
  uint32_t cnt = 0;
  if (t < a.nt) {
    if (a.dbgf) {
      for (int k = 0; k < 8; ++k) { a.dbgf[t * 8 + k] = 0.0f; a.dbgi[t * 8 + k] = 0; }
    }
    const int item = kMulti ? find_item(a.items, a.n_items, t) : 0;
    const Item& it = a.items[item];
    const int64_t lt = t - it.tri_base;
    const Rig rg = it.rig;  // in registers: the view loop reads it every iteration
    const float* m = a.models ? a.models[item].m : a.model.m;
    float P[3][3];
    bool ok = true;
    uint32_t vi[3];
    for (int k = 0; k < 3; ++k) {
      vi[k] = it.idx[lt * 3 + k];
      float px = it.pos[(int64_t)vi[k] * 3], py = it.pos[(int64_t)vi[k] * 3 + 1], pz = it.pos[(int64_t)vi[k] * 3 + 2];
      P[k][0] = ((m[0] * px + m[1] * py) + m[2] * pz) + m[3];
      P[k][1] = ((m[4] * px + m[5] * py) + m[6] * pz) + m[7];
      P[k][2] = ((m[8] * px + m[9] * py) + m[10] * pz) + m[11];
      if (!(P[k][2] >= rg.znear)) ok = false;
    }
    F3 P0{P[0][0], P[0][1], P[0][2]}, P1{P[1][0], P[1][1], P[1][2]}, P2{P[2][0], P[2][1], P[2][2]};
    F3 e1 = sub3(P1, P0), e2 = sub3(P2, P0);
    F3 n{e1.y * e2.z - e1.z * e2.y, e1.z * e2.x - e1.x * e2.z, e1.x * e2.y - e1.y * e2.x};
    float nl = sqrtf((n.x * n.x + n.y * n.y) + n.z * n.z);
    if (ok && (!(nl > 0.0f) || isinf(nl))) ok = false;
    TriRec R;
    if (ok) {
      R.nx = n.x / nl; R.ny = n.y / nl; R.nz = n.z / nl;
      R.p0x = P0.x; R.p0y = P0.y; R.p0z = P0.z;
      R.h = (R.nx * P0.x + R.ny * P0.y) + R.nz * P0.z;
      vertex_proj(rg, P0.x, P0.y, P0.z, R.a0, R.c0, R.y0);
      vertex_proj(rg, P1.x, P1.y, P1.z, R.a1, R.c1, R.y1);
      vertex_proj(rg, P2.x, P2.y, P2.z, R.a2, R.c2, R.y2);
    }
    // triangles that no view can see skip the view loop (see may_be_seen)
    const bool seen = ok && may_be_seen(rg, R);
    // visibility in each view + LFD-biased densities over the active views
    int nact = 0;
    float lxmin = INFINITY, lymin = INFINITY, Amin = INFINITY, admin = INFINITY, admax = 0.0f;
    if (seen) {
      // the next view's eye offset is fetched one iteration ahead
      float b_next = rg.eye[0];
      for (int r = 0; r < rg.n_views; ++r) {
        const float b = b_next;
        if (r + 1 < rg.n_views) b_next = rg.eye[r + 1];
        int32_t qx[3], qy[3];
        if (!view_active(rg, R, b, qx, qy)) continue;
        ++nact;
        F3 e{b, 0.0f, 0.0f};
        F3 Ps = nearest_on_triangle(e, P0, P1, P2);
        F3 d = sub3(Ps, e);
        float delta = R.h - R.nx * b;
        float ad = fabsf(delta);
        float Zs = Ps.z;
        float g = R.nx / delta;
        float vx = 1.0f - d.x * g, vy = 0.0f - d.y * g, vz = 0.0f - d.z * g;
        float lx = (Zs / rg.fx) * sqrtf((vx * vx + vy * vy) + vz * vz);
        float g2 = R.ny / delta;
        float wx = 0.0f - d.x * g2, wy = 1.0f - d.y * g2, wz = 0.0f - d.z * g2;
        float ly = (Zs / rg.fy) * sqrtf((wx * wx + wy * wy) + wz * wz);
        float A = ((Zs * Zs) * Zs) / (rg.fxfy * ad);
        lxmin = lx < lxmin ? lx : lxmin;
        lymin = ly < lymin ? ly : lymin;
        Amin = A < Amin ? A : Amin;
        admin = ad < admin ? ad : admin;
        admax = ad > admax ? ad : admax;
      }
    }
    if (ok && nact > 0) {
      act_cnt = 1;
      // T_align: s axis = camera X projected into the plane, t axis = n x s
      float upx, upy, upz;
      if (fabsf(R.nx) > 0.99999f) {
        upx = 0.0f - R.nx * R.ny; upy = 1.0f - R.ny * R.ny; upz = 0.0f - R.nz * R.ny;
      } else {
        upx = 1.0f - R.nx * R.nx; upy = 0.0f - R.ny * R.nx; upz = 0.0f - R.nz * R.nx;
      }
      float ul = sqrtf((upx * upx + upy * upy) + upz * upz);
      R.ux = upx / ul; R.uy = upy / ul; R.uz = upz / ul;
      R.wx = R.ny * R.uz - R.nz * R.uy;
      R.wy = R.nz * R.ux - R.nx * R.uz;
      R.wz = R.nx * R.uy - R.ny * R.ux;
      float Sx = 1.0f / lxmin, Sy = 1.0f / lymin;
      float size_xy = Amin;
      // texture-based sampling, Eqs. 1-3
      const int tex = it.tex[lt];
      const TexInfo& ti = it.texinfo[tex];
      // physically based mode: three more textures; Eq. 1 takes the largest
      const bool pbr = a.tm != nullptr;
      int32_t texk[4] = {tex, tex, tex, tex};
      if (pbr) {
        texk[1] = it.mat[lt * 3];
        texk[2] = it.mat[lt * 3 + 1];
        texk[3] = it.mat[lt * 3 + 2];
      }
      float uv0u = it.uv[(int64_t)vi[0] * 2], uv0v = it.uv[(int64_t)vi[0] * 2 + 1];
      float du1 = it.uv[(int64_t)vi[1] * 2] - uv0u, dv1 = it.uv[(int64_t)vi[1] * 2 + 1] - uv0v;
      float du2 = it.uv[(int64_t)vi[2] * 2] - uv0u, dv2 = it.uv[(int64_t)vi[2] * 2 + 1] - uv0v;
      float Ats = 0.5f * fabsf(du1 * dv2 - dv1 * du2);
      float Aws = 0.5f * nl;
      float Xt = (float)ti.size;
      float ntex = (Ats * Xt) * Xt;
      if (pbr) {
        for (int k = 1; k < 4; ++k) {
          const float Xk = (float)it.texinfo[texk[k]].size;
          const float nk = (Ats * Xk) * Xk;
          ntex = nk > ntex ? nk : ntex;
        }
      }
      if (ntex > 0.0f) {
        float size_uv = Aws / ntex;
        if (size_uv > size_xy) {
          float f = sqrtf(size_xy / size_uv);
          Sx = Sx * f;
          Sy = Sy * f;
        }
      }
      R.sx = Sx; R.sy = Sy;
      R.ruv = Ats / Aws;
      // multiview-mip setup, Eqs. 4-7
      float Zmin = P0.z, Zmax = P0.z;
      Zmin = P1.z < Zmin ? P1.z : Zmin; Zmax = P1.z > Zmax ? P1.z : Zmax;
      Zmin = P2.z < Zmin ? P2.z : Zmin; Zmax = P2.z > Zmax ? P2.z : Zmax;
      R.smin = (((Zmin * Zmin) * Zmin) / (rg.fxfy * admax)) * R.ruv;
      R.smax = (((Zmax * Zmax) * Zmax) / (rg.fxfy * admin)) * R.ruv;
      R.irange = R.smax > R.smin ? 1.0f / (R.smax - R.smin) : 0.0f;
      R.cu0 = R.uy * P0.y + R.uz * P0.z;
      R.cw0 = R.wy * P0.y + R.wz * P0.z;
      R.item = item;
      R.pad1 = 0;
      int32_t kmin = 0, kmax = 0;
      if (rg.mip) {
        int32_t top = 256 * (ti.levels - 1);
        kmin = lod_q8(a.lod_thr, (R.smin * Xt) * Xt);
        kmax = lod_q8(a.lod_thr, (R.smax * Xt) * Xt);
        kmin = kmin < 0 ? 0 : (kmin > top ? top : kmin);
        kmax = kmax < 0 ? 0 : (kmax > top ? top : kmax);
      }
      TriMat M{};
      if (pbr) {
        // Eqs. 6-7 for each material texture at its own size and level count
        int32_t kq[6] = {0, 0, 0, 0, 0, 0};
        if (rg.mip) {
          for (int k = 1; k < 4; ++k) {
            const TexInfo& tk = it.texinfo[texk[k]];
            const float Xk = (float)tk.size;
            const int32_t top = 256 * (tk.levels - 1);
            int32_t k0 = lod_q8(a.lod_thr, (R.smin * Xk) * Xk);
            int32_t k1 = lod_q8(a.lod_thr, (R.smax * Xk) * Xk);
            kq[2 * k - 2] = k0 < 0 ? 0 : (k0 > top ? top : k0);
            kq[2 * k - 1] = k1 < 0 ? 0 : (k1 > top ? top : k1);
          }
        }
        F3 Tf, Bf;
        texture_frame(e1, e2, du1, dv1, du2, dv2, F3{R.nx, R.ny, R.nz}, F3{R.ux, R.uy, R.uz},
                      F3{R.wx, R.wy, R.wz}, Tf, Bf);
        M.texn = texk[1]; M.texr = texk[2]; M.texm = texk[3];
        M.kn0 = kq[0]; M.kn1 = kq[1]; M.kr0 = kq[2]; M.kr1 = kq[3]; M.km0 = kq[4]; M.km1 = kq[5];
        M.tx = Tf.x; M.ty = Tf.y; M.tz = Tf.z; M.bx = Bf.x; M.by = Bf.y; M.bz = Bf.z;
      }
      // sample lattice, vertex 0 at the centre of cell (0,0)
      bool ovf = false;
      int32_t sq[3] = {128, 0, 0}, tq[3] = {128, 0, 0};
      F3 ek[2] = {e1, e2};
      F3 uh{R.ux, R.uy, R.uz}, wh{R.wx, R.wy, R.wz};
      for (int k = 0; k < 2; ++k) {
        float s = Sx * dot3(uh, ek[k]) + 0.5f;
        float tt = Sy * dot3(wh, ek[k]) + 0.5f;
        if (!(fabsf(s) < 16384.0f) || !(fabsf(tt) < 16384.0f)) { ovf = true; break; }
        sq[k + 1] = (int32_t)rintf(s * 256.0f);
        tq[k + 1] = (int32_t)rintf(tt * 256.0f);
      }
      if (a.dbgf) {
        float* df = a.dbgf + t * 8;
        int32_t* di = a.dbgi + t * 8;
        df[0] = Sx; df[1] = Sy; df[2] = R.smin; df[3] = R.smax; df[4] = R.ruv; df[5] = R.h;
        df[6] = size_xy; df[7] = (float)nact;
        if (!ovf) { di[0] = sq[1]; di[1] = tq[1]; di[2] = sq[2]; di[3] = tq[2]; }
        di[4] = kmin; di[5] = kmax; di[6] = 1;
      }
      int64_t count = 0, jfirst = 0, jlast = -1;
      Lattice L;
      TriEmit E;
      E.uv0u = uv0u; E.uv0v = uv0v; E.du1 = du1; E.dv1 = dv1; E.du2 = du2; E.dv2 = dv2;
      E.s1 = sq[1]; E.t1 = tq[1]; E.s2 = sq[2]; E.t2 = tq[2];
      E.kmin = kmin; E.kmax = kmax; E.tex = tex; E.item = item;
      E.jlo = 0; E.jhi = -1;
      if (!ovf) {
        if constexpr (kLean) {
          a.rec[t] = R;
          if (pbr) a.tm[t] = M;
          a.em[t] = E;
        }
        lattice_init(L, sq[1], tq[1], sq[2], tq[2]);
        int64_t nb = (L.iB - L.iA + 1) * (L.jB - L.jA + 1);
        if (nb > kBoxCap) {
          ovf = true;
        } else {
          for (int64_t j = L.jA; j <= L.jB; ++j) {
            int64_t lo, hi;
            lattice_row(L, j, lo, hi);
            if (hi >= lo) {
              if (count == 0) jfirst = j;
              jlast = j;
              count += hi - lo + 1;
            }
          }
          if (count > kCellCap) ovf = true;
        }
      }
      if (ovf) {
        count = 0;
        ovf_cnt = 1;
        if (a.dbgi) a.dbgi[t * 8 + 7] = 1;
      }
      cnt = (uint32_t)count;
      pv_cnt = (uint64_t)count * (uint64_t)nact;
      if (cnt > 0) {
        if constexpr (kLean) {
          *reinterpret_cast<int2*>(&a.em[t].jlo) = make_int2((int32_t)jfirst, (int32_t)jlast);
        } else {
          E.jlo = (int32_t)jfirst;
          E.jhi = (int32_t)jlast;
          a.rec[t] = R;
          a.em[t] = E;
          if (pbr) a.tm[t] = M;
        }
      }
    }
    a.counts[t] = cnt;
  }
  // triangles with more cells than one lane emits go to the workgroup list
  const bool big = cnt > kBigCells;
  const uint64_t bslot = wave_append(big, a.n_big);
  if (big) a.big[bslot] = (uint32_t)t;
  // this workgroup's point count (its 256 triangles form one scan tile)
  __shared__ uint64_t tsum[4];
  const uint64_t wcnt = wave_sum((uint64_t)cnt);
  if ((threadIdx.x & 63) == 0) tsum[threadIdx.x >> 6] = wcnt;
  // per-wave statistics, one atomic per wave
  act_cnt = wave_sum(act_cnt);
  ovf_cnt = wave_sum(ovf_cnt);
  pv_cnt = wave_sum(pv_cnt);
  if ((threadIdx.x & 63) == 0) {
    if (act_cnt) atomicAdd((unsigned long long*)&a.stats[STAT_ACTIVE], (unsigned long long)act_cnt);
    if (ovf_cnt) atomicAdd((unsigned long long*)&a.stats[STAT_OVERFLOW], (unsigned long long)ovf_cnt);
    if (pv_cnt) atomicAdd((unsigned long long*)&a.stats[STAT_POINT_VIEWS], (unsigned long long)pv_cnt);
  }
  __syncthreads();
  if (threadIdx.x == 0) a.tile_sum[blockIdx.x] = (tsum[0] + tsum[1]) + (tsum[2] + tsum[3]);
}

// ------------------------------------------------------------------ scan (counts -> offsets)
// The point offsets are an exclusive prefix sum of the per-triangle counts over
// tiles of 256 triangles: the set-up writes each tile's sum (one tile per
// set-up workgroup), k_scan_top turns the tile sums into tile bases (one
// workgroup; also the grand total), and the emission kernel, whose workgroups
// take the same tiles, adds the prefix within its tile.

constexpr int kScanTile = 256;  // triangles per tile: one set-up / emission workgroup

__global__ void __launch_bounds__(1024) k_scan_top(uint64_t* __restrict__ tile_sum, int64_t ntiles,
                                                    uint64_t* __restrict__ total) {
  __shared__ uint64_t ws[16];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < ntiles; b0 += 1024) {
    int64_t i = b0 + threadIdx.x;
    uint64_t v = i < ntiles ? tile_sum[i] : 0;
    uint64_t inc = wave_incl_scan(v);
    if ((threadIdx.x & 63) == 63) ws[threadIdx.x >> 6] = inc;
    __syncthreads();
    uint64_t wbase = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wbase += ws[w];
    uint64_t excl = carry + wbase + inc - v;
    __syncthreads();
    if (i < ntiles) tile_sum[i] = excl;
    if (threadIdx.x == 1023) carry = excl + v;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

// ------------------------------------------------------------------ a1/a2: emission

__device__ __forceinline__ void write_head(Point* pts, uint64_t gi, uint32_t t, uint32_t f, int64_t i, int64_t j) {
  uint2 head;
  head.x = t | (f << 28);
  head.y = (uint32_t)(uint16_t)(int16_t)i | ((uint32_t)(uint16_t)(int16_t)j << 16);
  *reinterpret_cast<uint2*>(&pts[gi]) = head;
}

// Exclusive prefix of v over the 256 lanes of the workgroup (every lane calls).
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t* ws4) {
  const uint64_t inc = wave_incl_scan(v);
  if ((threadIdx.x & 63) == 63) ws4[threadIdx.x >> 6] = inc;
  __syncthreads();
  uint64_t before = 0;
  for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) before += ws4[w];
  __syncthreads();  // ws4 may be rewritten after this
  return before + inc - v;
}

// Emission, one launch: workgroups [0, kEmitBigBlocks) take the queued
// triangles with more than kBigCells cells, one triangle per workgroup at a
// time (lanes take rows, a block scan places them); the others take the
// set-up's tiles of 256 triangles: each lane writes its triangle's point offset
// (tile base + prefix within the tile) and emits the points of a small
// triangle.
constexpr unsigned kEmitBigBlocks = 1024;

__device__ __forceinline__ void emit_big(const EmitArgs& a, uint64_t* ws4) {
  const uint64_t nbig = *a.n_big;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (uint64_t b = blockIdx.x; b < nbig; b += kEmitBigBlocks) {
    const uint32_t t = a.big[b];
    const TriEmit& E = a.em[t];
    // the triangle's first point: the tile base plus the earlier counts in the tile
    const int64_t t0 = (int64_t)t - (int64_t)t % kScanTile;
    const int64_t u = t0 + threadIdx.x;
    const uint64_t cu = u < (int64_t)t ? a.counts[u] : 0u;
    uint64_t wsum = wave_sum(cu);
    if (lane == 0) ws4[wv] = wsum;
    __syncthreads();
    const uint64_t base = a.tile_base[t0 / kScanTile] + (ws4[0] + ws4[1]) + (ws4[2] + ws4[3]);
    __syncthreads();
    Lattice L;
    lattice_init(L, E.s1, E.t1, E.s2, E.t2);
    const int64_t jlo = E.jlo, jhi = E.jhi;  // rows with cells, found by the set-up
    uint64_t run = 0;
    for (int64_t j0 = jlo; j0 <= jhi; j0 += blockDim.x) {
      const int64_t j = j0 + threadIdx.x;
      int64_t lo = 1, hi = 0;
      if (j <= jhi) lattice_row(L, j, lo, hi);
      const uint64_t c = hi >= lo ? (uint64_t)(hi - lo + 1) : 0;
      uint64_t inc = wave_incl_scan(c);
      if (lane == 63) ws4[wv] = inc;
      __syncthreads();
      uint64_t before = 0, total = 0;
      for (int w = 0; w < 4; ++w) {
        if (w < wv) before += ws4[w];
        total += ws4[w];
      }
      const uint64_t start = base + run + before + inc - c;
      const uint32_t fj = (j == jlo ? F_JLO : 0u) | (j == jhi ? F_JHI : 0u);
      const uint64_t ri = base + (uint64_t)(j - jlo);
      if (a.rows && j <= jhi && ri < (uint64_t)a.cap)
        a.rows[ri] = RowEntry{(uint32_t)(start - base), (int16_t)lo, (int16_t)hi};
      for (int64_t i = lo; i <= hi; ++i) {
        uint64_t gi = start + (uint64_t)(i - lo);
        if (gi < (uint64_t)a.cap)
          write_head(a.points, gi, t, fj | (i == lo ? F_ILO : 0u) | (i == hi ? F_IHI : 0u), i, j);
      }
      run += total;
      __syncthreads();  // the wave sums are rewritten by the next pass
    }
  }
}

__global__ void __launch_bounds__(256) k_emit(EmitArgs a) {
  __shared__ uint64_t ws4[4];
  if (blockIdx.x < kEmitBigBlocks) {
    emit_big(a, ws4);
    return;
  }
  const int64_t tile = (int64_t)blockIdx.x - kEmitBigBlocks;
  const int64_t t = tile * kScanTile + threadIdx.x;
  const uint32_t cnt = t < a.nt ? a.counts[t] : 0u;
  const uint64_t base = a.tile_base[tile] + block_excl_scan(cnt, ws4);
  if (t < a.nt) a.offsets[t] = base;
  if (a.tris) {
    const uint64_t slot = wave_append(cnt > 0, a.n_tris);
    if (cnt > 0) a.tris[slot] = (uint32_t)t;
  }
  if (cnt == 0 || cnt > kBigCells) return;  // the big ones are queued by the set-up
  const TriEmit& E = a.em[t];
  Lattice L;
  lattice_init(L, E.s1, E.t1, E.s2, E.t2);
  const int64_t jlo = E.jlo, jhi = E.jhi;  // rows with cells, found by the set-up
  uint64_t k = 0;
  for (int64_t j = jlo; j <= jhi; ++j) {
    int64_t lo, hi;
    lattice_row(L, j, lo, hi);
    uint32_t fj = (j == jlo ? F_JLO : 0u) | (j == jhi ? F_JHI : 0u);
    const uint64_t ri = base + (uint64_t)(j - jlo);  // rows never outnumber points
    if (a.rows && ri < (uint64_t)a.cap) a.rows[ri] = RowEntry{(uint32_t)k, (int16_t)lo, (int16_t)hi};
    for (int64_t i = lo; i <= hi; ++i, ++k) {
      uint64_t gi = base + k;
      if (gi >= (uint64_t)a.cap) return;
      write_head(a.points, gi, (uint32_t)t, fj | (i == lo ? F_ILO : 0u) | (i == hi ? F_IHI : 0u), i, j);
    }
  }
}

// Splat rectangle of point (i, j): its lattice cell, extended by one cell
// beyond the end of its row (F_ILO / F_IHI) or of the lattice (F_JLO / F_JHI),
// with the corners projected except for the eye offset (x = cA - b*cC) and the
// range of their projected rows; `full` when a corner lies behind z_near/2.
__device__ __forceinline__ void splat_corners(const Rig& rg, const TriRec& T, int32_t i, int32_t j, uint32_t flags,
                                              float cA[4], float cC[4], float& ymn, float& ymx, bool& full) {
  const int32_t s0 = i - ((flags & F_ILO) ? 1 : 0), s1 = i + 1 + ((flags & F_IHI) ? 1 : 0);
  const int32_t t0 = j - ((flags & F_JLO) ? 1 : 0), t1 = j + 1 + ((flags & F_JHI) ? 1 : 0);
  const float zlim = 0.5f * rg.znear;
  ymn = ymx = 0.0f;
  full = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float aa = ((float)((k & 1) ? s1 : s0) - 0.5f) / T.sx;
    float cc = ((float)((k & 2) ? t1 : t0) - 0.5f) / T.sy;
    float X = (T.p0x + aa * T.ux) + cc * T.wx;
    float Y = (T.p0y + aa * T.uy) + cc * T.wy;
    float Z = (T.p0z + aa * T.uz) + cc * T.wz;
    if (!(Z >= zlim)) full = true;
    float Yp;
    vertex_proj(rg, X, Y, Z, cA[k], cC[k], Yp);
    if (k == 0) { ymn = ymx = Yp; }
    else { ymn = Yp < ymn ? Yp : ymn; ymx = Yp > ymx ? Yp : ymx; }
  }
}

// Rows that splat_point can write for a point in any view: the triangle's rows
// (guard band, the whole triangle above or below the view) met with the splat
// rectangle's rows `rows` (PointBox).  False when none.
__device__ __forceinline__ bool quilt_point_rows(int32_t H, const TriRec& T, int32_t rows, int32_t& r0, int32_t& r1) {
  if (!(fabsf(T.y0) < kGuard) || !(fabsf(T.y1) < kGuard) || !(fabsf(T.y2) < kGuard)) return false;
  const int32_t H8 = 256 * H;
  const int32_t qy0 = (int32_t)rintf(T.y0 * 256.0f), qy1 = (int32_t)rintf(T.y1 * 256.0f),
                qy2 = (int32_t)rintf(T.y2 * 256.0f);
  if ((qy0 < 0 && qy1 < 0 && qy2 < 0) || (qy0 > H8 && qy1 > H8 && qy2 > H8)) return false;
  const int32_t ymin = min(qy0, min(qy1, qy2)), ymax = max(qy0, max(qy1, qy2));
  r0 = max(0, -((128 - ymin) >> 8));
  r1 = min(H - 1, (ymax - 128) >> 8);
  if (rows != kAllRows) {
    r0 = max(r0, (int32_t)(int16_t)(rows & 0xFFFF));
    r1 = min(r1, (int32_t)(int16_t)((uint32_t)rows >> 16));
  }
  return r0 <= r1;
}

// Per point: UV at the cell centre and the two mip fetches (Eqs. 6-7); for the
// triangle-major splat and the quilt (kBox) also the point's splat rectangle
// (PointBox), for the quilt the pixel rows its splat can write; kPBR: the
// material fetches.  The plain form holds 46 VGPRs (8 waves per SIMD, for a
// kernel that waits on its texel gathers) instead of the 75 of all branches.
template <bool kBox, bool kPBR>
__global__ void __launch_bounds__(256) k_fetch(EmitArgs a) {
  const uint64_t npts = imin((int64_t)*a.n_points, a.cap);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += stride) {
    uint2 head = *reinterpret_cast<const uint2*>(&a.points[p]);
    const uint32_t t = head.x & 0x0FFFFFFFu;
    const int64_t i = (int16_t)(head.y & 0xFFFFu), j = (int16_t)(head.y >> 16);
    const TriEmit& E = a.em[t];
    const int64_t S1 = E.s1, T1 = E.t1, S2 = E.s2, T2 = E.t2;
    const int64_t area2 = (S1 - 128) * (T2 - 128) - (T1 - 128) * (S2 - 128);
    int64_t cxq = 256 * i + 128, cyq = 256 * j + 128;
    int64_t w1 = (cxq - 128) * (T2 - 128) - (cyq - 128) * (S2 - 128);
    int64_t w2 = (S1 - 128) * (cyq - 128) - (T1 - 128) * (cxq - 128);
    // a zero-area lattice has no barycentrics: its points take vertex 0's UV
    float b1 = area2 != 0 ? (float)((double)w1 / (double)area2) : 0.0f;
    float b2 = area2 != 0 ? (float)((double)w2 / (double)area2) : 0.0f;
    float u = (E.uv0u + b1 * E.du1) + b2 * E.du2;
    float v = (E.uv0v + b1 * E.dv1) + b2 * E.dv2;
    const Item& it = a.items[E.item];
    const TexInfo& ti = it.texinfo[E.tex];
    uint2 tv;
    tv.x = trilinear(it.texels, ti, u, v, E.kmin);
    tv.y = E.kmax == E.kmin ? tv.x : trilinear(it.texels, ti, u, v, E.kmax);
    *reinterpret_cast<uint2*>(&a.points[p].tvmin) = tv;
    if constexpr (kBox) {
      const TriRec& T = a.rec[t];
      PointBox B;
      float ymn, ymx;
      bool full;
      splat_corners(it.rig, T, (int32_t)i, (int32_t)j, head.x >> 28, B.cA, B.cC, ymn, ymx, full);
      if (full) {
        B.rows = kAllRows;
      } else {
        // rows whose centres lie within 1/64 px of the corners' range, clamped
        // to [-1, H] (rows outside the view never matter)
        int32_t r0 = (int32_t)ceilf(clamp_big(ymn - 0.515625f)), r1 = (int32_t)floorf(clamp_big(ymx - 0.484375f));
        r0 = r0 < -1 ? -1 : (r0 > it.rig.H ? it.rig.H : r0);
        r1 = r1 < -1 ? -1 : (r1 > it.rig.H ? it.rig.H : r1);
        B.rows = (int32_t)((uint32_t)(uint16_t)(int16_t)r0 | ((uint32_t)(uint16_t)(int16_t)r1 << 16));
      }
      const float cs = (float)i / T.sx, ct = (float)j / T.sy;
      const float Zc = (T.p0z + cs * T.uz) + ct * T.wz;
      B.zc3 = (Zc * Zc) * Zc;
      B.tvmin = tv.x;
      B.tvmax = tv.y;
      a.pbox[p] = B;
      if (a.prows) {
        int32_t r0, r1;
        const uint32_t base = (uint32_t)E.item * (uint32_t)it.rig.H;
        a.prows[p] = quilt_point_rows(it.rig.H, T, B.rows, r0, r1) ? make_uint2(base + (uint32_t)r0, base + (uint32_t)r1)
                                                                   : make_uint2(~0u, ~0u);
      }
    }
    if constexpr (kPBR) {
      // physically based mode: normal map (RGBA8) and the R bytes of the
      // roughness and metallic maps, each at its own LOD pair
      const TriMat& M = a.tm[t];
      const TexInfo& tn = it.texinfo[M.texn];
      const TexInfo& tr = it.texinfo[M.texr];
      const TexInfo& tm = it.texinfo[M.texm];
      uint4 pm;
      pm.x = trilinear(it.texels, tn, u, v, M.kn0);
      pm.y = M.kn1 == M.kn0 ? pm.x : trilinear(it.texels, tn, u, v, M.kn1);
      const uint32_t r0 = trilinear(it.texels, tr, u, v, M.kr0) & 255u;
      const uint32_t r1 = M.kr1 == M.kr0 ? r0 : trilinear(it.texels, tr, u, v, M.kr1) & 255u;
      const uint32_t m0 = trilinear(it.texels, tm, u, v, M.km0) & 255u;
      const uint32_t m1 = M.km1 == M.km0 ? m0 : trilinear(it.texels, tm, u, v, M.km1) & 255u;
      pm.z = r0 | (r1 << 8) | (m0 << 16) | (m1 << 24);
      pm.w = 0u;
      a.pmat[p] = pm;
    }
  }
}

// ------------------------------------------------------------------ a3: splat

// One lane per point, looping over the views.  Everything that does not depend
// on the eye offset b is computed once per point: the cell's corner projections
// (x = A - b*C is affine in b), the row range, the cell-centre depth.  Pixel
// ray slopes (x+0.5-cx)/fx and (y+0.5-cy)/fy come from per-block LDS tables
// holding exactly the values the inline expressions give.  The integer edge
// functions are evaluated in double, which represents every value exactly
// (|E| < 2^50), and stepped along x.
// An item table entry read by all active lanes of a wave from one address,
// moved to scalar registers word by word.
__device__ __forceinline__ Item load_uniform(const Item* p) {
  static_assert(sizeof(Item) % 4 == 0, "Item is a whole number of words");
  Item out;
  const int32_t* src = reinterpret_cast<const int32_t*>(p);
  int32_t* dst = reinterpret_cast<int32_t*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(Item) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
  return out;
}

// 64-bit depth-test update (relaxed, device scope); the key buffers are global
// memory, which lets the compiler issue a global rather than a flat atomic.
__device__ __forceinline__ void key_min(uint64_t* p, uint64_t v) {
  typedef __attribute__((address_space(1))) unsigned long long global_u64;
  __hip_atomic_fetch_min((global_u64*)p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 64-bit depth-test update of a key held in LDS (a quilt tile).
__device__ __forceinline__ void lds_key_min(uint64_t* p, uint64_t v) {
  typedef __attribute__((address_space(3))) unsigned long long lds_u64;
  __hip_atomic_fetch_min((lds_u64*)p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One tile of the row-band quilt: views [r_lo, r_hi) and rows [y_lo, y_hi] of
// every view, all W columns, as keys[((r - r_lo) * rows + (y - y_lo)) * W + x]
// in LDS; `box` is the point's splat rectangle written at emission.
struct QuiltTile {
  uint64_t* keys;
  int32_t r_lo, r_hi, y_lo, y_hi, rows;
  const PointBox* box;
};

// Element i (wave-uniform) of a table that no kernel of the launch writes, as a
// scalar-cache read straight into a scalar register.
__device__ __forceinline__ float table_f32(const float* p, int i) {
  typedef const __attribute__((address_space(4))) float const_f32;
  return ((const_f32*)p)[i];
}

__device__ __forceinline__ float uniform_f32(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// One point against every view of its item's rig; `item` is wave-uniform.
// kPBR: the colour is shaded (material record tm[tri], point words pm).
// kQuilt: only the views and rows of tile *qt, keys in its LDS; the splat
// rectangle's corners, rows and cell-centre depth come from the point's
// PointBox (the same values, computed at emission).
template <bool kPBR, bool kQuilt = false>
__device__ __forceinline__ void splat_point(const Item& item, const Point& pt, const TriRec& T, uint32_t flags,
                                            int32_t i, int32_t j, const float* tx, const float* ty,
                                            const SplatArgs& a, uint64_t p, uint32_t& written,
                                            const QuiltTile* qt = nullptr) {
  const int64_t vpx = (int64_t)item.rig.W * item.rig.H;
  const int32_t H8 = 256 * item.rig.H, W8 = 256 * item.rig.W;
  const Rig& rg = item.rig;
  uint64_t* const keys = item.keys;
  const bool rowmajor = item.key_layout != 0;
  const int64_t row_stride = rowmajor ? (int64_t)rg.n_views * rg.W : rg.W;
  // view-independent vertex rows (guard band on y) and triangle row range
  if (!(fabsf(T.y0) < kGuard) || !(fabsf(T.y1) < kGuard) || !(fabsf(T.y2) < kGuard)) return;
  const int32_t qy0 = (int32_t)rintf(T.y0 * 256.0f), qy1 = (int32_t)rintf(T.y1 * 256.0f),
                qy2 = (int32_t)rintf(T.y2 * 256.0f);
  if ((qy0 < 0 && qy1 < 0 && qy2 < 0) || (qy0 > H8 && qy1 > H8 && qy2 > H8)) return;
  const int32_t ymin = min(qy0, min(qy1, qy2)), ymax = max(qy0, max(qy1, qy2));
  const int32_t Y0 = max(0, -((128 - ymin) >> 8));
  const int32_t Y1 = min(rg.H - 1, (ymax - 128) >> 8);
  if (Y0 > Y1) return;
  // splat box corners (row-end extended cell), projected except for the eye offset
  float cA[4], cC[4];
  bool full;
  int32_t by0 = Y0, by1 = Y1;
  if constexpr (kQuilt) {
    // the stored rows are clamped to [-1, H], which leaves their intersection
    // with [Y0, Y1] (inside [0, H-1]) unchanged or empty as before
    const PointBox& B = *qt->box;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      cA[k] = B.cA[k];
      cC[k] = B.cC[k];
    }
    full = B.rows == kAllRows;
    if (!full) {
      by0 = max((int32_t)(int16_t)(B.rows & 0xFFFF), by0);
      by1 = min((int32_t)(int16_t)((uint32_t)B.rows >> 16), by1);
    }
    by0 = max(by0, qt->y_lo);
    by1 = min(by1, qt->y_hi);
  } else {
    float ymn, ymx;
    splat_corners(rg, T, i, j, flags, cA, cC, ymn, ymx, full);
    if (!full) {
      int32_t r0 = (int32_t)ceilf(clamp_big(ymn - 0.515625f)), r1 = (int32_t)floorf(clamp_big(ymx - 0.484375f));
      by0 = max(r0, by0);
      by1 = min(r1, by1);
    }
  }
  if (by0 > by1) return;
  // cell-centre terms of Eqs. 8-9 and the ownership bounds
  float cs = 0.0f, ct = 0.0f, Zc = 0.0f, Zc3;
  if (kQuilt && !kPBR) {
    Zc3 = qt->box->zc3;
  } else {
    cs = (float)i / T.sx;
    ct = (float)j / T.sy;
    Zc = (T.p0z + cs * T.uz) + ct * T.wz;
    Zc3 = (Zc * Zc) * Zc;
  }
  F3 pc{0.0f, 0.0f, Zc}, Tf{0.0f, 0.0f, 0.0f}, Bf{0.0f, 0.0f, 0.0f};
  uint4 pm{0u, 0u, 0u, 0u};
  if constexpr (kPBR) {
    // cell centre in camera space, tangent frame, material bytes of the point
    pc.x = (T.p0x + cs * T.ux) + ct * T.wx;
    pc.y = (T.p0y + cs * T.uy) + ct * T.wy;
    const TriMat& M = a.tm[pt.tri_flags & 0x0FFFFFFFu];
    Tf = F3{M.tx, M.ty, M.tz};
    Bf = F3{M.bx, M.by, M.bz};
    pm = a.pmat[p];
  }
  const float Acell = 1.0f / (T.sx * T.sy);
  const float suv = Acell * T.ruv;
  const float fi0 = (float)i, fi1 = (float)(i + 1), fj0 = (float)j, fj1 = (float)(j + 1);
  const bool oilo = flags & F_ILO, oihi = flags & F_IHI, ojlo = flags & F_JLO, ojhi = flags & F_JHI;
  const uint32_t lo02 = pt.tvmin & 0x00FF00FFu, lo13 = (pt.tvmin >> 8) & 0x00FF00FFu;
  const uint32_t hi02 = pt.tvmax & 0x00FF00FFu, hi13 = (pt.tvmax >> 8) & 0x00FF00FFu;
  const float p0y2 = T.p0y * T.p0y, p0z2 = T.p0z * T.p0z;
  const int r_begin = kQuilt ? qt->r_lo : 0, r_end = kQuilt ? qt->r_hi : rg.n_views;
  float b_next = table_f32(rg.eye, r_begin);  // the next view's eye offset, one iteration ahead
  for (int r = r_begin; r < r_end; ++r) {
    const float b = b_next;
    if (r + 1 < r_end) b_next = table_f32(rg.eye, r + 1);
    const float delta = T.h - T.nx * b;
    if (!faces_eye(T.p0x, p0y2, p0z2, delta, b)) continue;
    // splat box columns first: empty for about a third of the (point, view) pairs
    int32_t cbx0 = 0, cbx1 = rg.W - 1;
    if (!full) {
      float xmn = cA[0] - b * cC[0], xmx = xmn;
#pragma unroll
      for (int k = 1; k < 4; ++k) {
        float xx = cA[k] - b * cC[k];
        xmn = xx < xmn ? xx : xmn;
        xmx = xx > xmx ? xx : xmx;
      }
      cbx0 = max(cbx0, (int32_t)ceilf(clamp_big(xmn - 0.515625f)));
      cbx1 = min(cbx1, (int32_t)floorf(clamp_big(xmx - 0.484375f)));
      if (cbx0 > cbx1) continue;
    }
    const float x0 = T.a0 - b * T.c0, x1 = T.a1 - b * T.c1, x2 = T.a2 - b * T.c2;
    if (!(fabsf(x0) < kGuard) || !(fabsf(x1) < kGuard) || !(fabsf(x2) < kGuard)) continue;
    int32_t qx[3] = {(int32_t)rintf(x0 * 256.0f), (int32_t)rintf(x1 * 256.0f), (int32_t)rintf(x2 * 256.0f)};
    int32_t qy[3] = {qy0, qy1, qy2};
    if ((qx[0] < 0 && qx[1] < 0 && qx[2] < 0) || (qx[0] > W8 && qx[1] > W8 && qx[2] > W8)) continue;
    const double a2 = (double)(qx[1] - qx[0]) * (double)(qy[2] - qy[0]) -
                      (double)(qy[1] - qy[0]) * (double)(qx[2] - qx[0]);
    if (a2 == 0.0) continue;
    if (a2 < 0.0) {
      int32_t u = qx[1]; qx[1] = qx[2]; qx[2] = u;
      u = qy[1]; qy[1] = qy[2]; qy[2] = u;
    }
    const int32_t xmin = min(qx[0], min(qx[1], qx[2])), xmax = max(qx[0], max(qx[1], qx[2]));
    const int32_t bx0 = max(cbx0, -((128 - xmin) >> 8));
    const int32_t bx1 = min(cbx1, (xmax - 128) >> 8);
    const int32_t ry0 = kQuilt ? by0 : (full ? Y0 : by0), ry1 = kQuilt ? by1 : (full ? Y1 : by1);
    if (bx0 > bx1 || ry0 > ry1) continue;
    // colour of this point in this view (Eqs. 8-9)
    const float ad = fabsf(delta);
    const float Ar = Zc3 / (rg.fxfy * ad);
    const float vse = Acell < Ar ? T.ruv * Ar : suv;
    const float vs = vse < T.smin ? T.smin : (vse > T.smax ? T.smax : vse);
    const float tau = (vs - T.smin) * T.irange;
    int32_t tq = (int32_t)floorf(tau * 256.0f + 0.5f);
    tq = tq < 0 ? 0 : (tq > 256 ? 256 : tq);
    const uint32_t wa = (uint32_t)(256 - tq), wz = (uint32_t)tq;
    uint32_t col = (((lo02 * wa + hi02 * wz + 0x00800080u) >> 8) & 0x00FF00FFu) |
                   ((((lo13 * wa + hi13 * wz + 0x00800080u) >> 8) & 0x00FF00FFu) << 8);
    if constexpr (kPBR) {
      // the normal map and the roughness / metallic bytes take the same tau
      auto lerp_even = [&](uint32_t lo, uint32_t hi) {  // bytes 0 and 2 of each word
        return (((lo & 0x00FF00FFu) * wa + (hi & 0x00FF00FFu) * wz + 0x00800080u) >> 8) & 0x00FF00FFu;
      };
      const uint32_t nrm = lerp_even(pm.x, pm.y) | (lerp_even(pm.x >> 8, pm.y >> 8) << 8);
      const uint32_t rq = ((pm.z & 255u) * wa + ((pm.z >> 8) & 255u) * wz + 128u) >> 8;
      const uint32_t mq = (((pm.z >> 16) & 255u) * wa + (pm.z >> 24) * wz + 128u) >> 8;
      col = shade_splat(a.sh, F3{T.nx, T.ny, T.nz}, Tf, Bf, pc, b, col, nrm, rq, mq);
    }
    const float ks = table_f32(rg.kshift, r);
    const float cu = T.ux * (b - T.p0x) - T.cu0;
    const float cw = T.wx * (b - T.p0x) - T.cw0;
    // edge functions with the tie rule folded in as +0.5 (E integer: E+0.5 > 0 <=> E >= 0)
    double edx[3], edy[3], bias[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int eb = e == 2 ? 0 : e + 1;
      const int32_t dx = qx[eb] - qx[e], dy = qy[eb] - qy[e];
      edx[e] = (double)dx;
      edy[e] = (double)dy;
      bias[e] = (dy > 0 || (dy == 0 && dx > 0)) ? 0.5 : 0.0;
    }
    uint64_t* kv = keys + (rowmajor ? (int64_t)r * rg.W : (int64_t)r * vpx);
    const int32_t kq = kQuilt ? ((r - qt->r_lo) * qt->rows - qt->y_lo) * rg.W : 0;  // tile key of (y, x): kq + y*W + x
    const int32_t pxq0 = 256 * bx0 + 128, pyq0 = 256 * ry0 + 128;
    // edge functions at (bx0, ry0), stepped by whole pixels (all values are
    // integers + 0.5 below 2^51, so every step is exact)
    double R0 = edx[0] * (double)(pyq0 - qy[0]) - edy[0] * (double)(pxq0 - qx[0]) + bias[0];
    double R1 = edx[1] * (double)(pyq0 - qy[1]) - edy[1] * (double)(pxq0 - qx[1]) + bias[1];
    double R2 = edx[2] * (double)(pyq0 - qy[2]) - edy[2] * (double)(pxq0 - qx[2]) + bias[2];
    const double st0 = edy[0] * 256.0, st1 = edy[1] * 256.0, st2 = edy[2] * 256.0;
    const double sr0 = edx[0] * 256.0, sr1 = edx[1] * 256.0, sr2 = edx[2] * 256.0;
    for (int32_t y = ry0; y <= ry1; ++y, R0 += sr0, R1 += sr1, R2 += sr2) {
      double E0 = R0, E1 = R1, E2 = R2;
      const float ry = ty[y];
      const float nyr = T.ny * ry, uyr = T.uy * ry, wyr = T.wy * ry;
      for (int32_t x = bx0; x <= bx1; ++x) {
        const bool in = E0 > 0.0 && E1 > 0.0 && E2 > 0.0;
        E0 -= st0;
        E1 -= st1;
        E2 -= st2;
        if (!in) continue;
        const float rx = tx[x] - ks;
        const float den = (T.nx * rx + nyr) + T.nz;
        const float Z = delta / den;
        if (!(Z > 0.0f) || isinf(Z)) continue;
        const float ur = (T.ux * rx + uyr) + T.uz;
        const float wr = (T.wx * rx + wyr) + T.wz;
        const float sv = T.sx * (Z * ur + cu) + 0.5f;
        const float tv = T.sy * (Z * wr + cw) + 0.5f;
        const bool own = (oilo || sv >= fi0) && (oihi || sv < fi1) && (ojlo || tv >= fj0) && (ojhi || tv < fj1);
        if (own) {
          if constexpr (kQuilt)
            lds_key_min(qt->keys + (kq + y * rg.W + x), ((uint64_t)__float_as_uint(Z) << 32) | col);
          else
            key_min(&kv[(int64_t)y * row_stride + x], ((uint64_t)__float_as_uint(Z) << 32) | col);
          ++written;
        }
      }
    }
  }
}

// kMulti: points of several items (a batch); otherwise every point belongs to
// items[0] and the item is read once.  kPBR: shaded colours;
// held to 128 VGPRs (4 waves per SIMD instead of 3 at its natural 138), which
// measured faster despite an 8-byte spill.  The batch instantiation keeps 139:
// capped, it spills 40 bytes and slows down.
template <bool kMulti, bool kPBR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kPBR && !kMulti ? 4 : 1))) k_splat(SplatArgs a) {
  if (a.gate && *a.gate == 0) return;
  extern __shared__ float ray_tab[];  // W column slopes, then H row slopes
  const Rig& trg = a.table_rig;
  float* tx = ray_tab;
  float* ty = ray_tab + trg.W;
  for (int k = threadIdx.x; k < trg.W; k += blockDim.x) tx[k] = ((float)k + 0.5f - trg.cx) / trg.fx;
  for (int k = threadIdx.x; k < trg.H; k += blockDim.x) ty[k] = ((float)k + 0.5f - trg.cy) / trg.fy;
  __syncthreads();
  const uint64_t npts = imin((int64_t)*a.n_points, a.cap);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const Item it0 = load_uniform(a.items);
  uint32_t written = 0;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += stride) {
    const Point pt = a.points[p];
    const uint32_t tri = pt.tri_flags & 0x0FFFFFFFu, flags = pt.tri_flags >> 28;
    const int32_t i = (int16_t)(pt.ij & 0xFFFFu), j = (int16_t)(pt.ij >> 16);
    if (!kMulti) {
      const TriRec T = a.rec[tri];
      splat_point<kPBR>(it0, pt, T, flags, i, j, tx, ty, a, p, written);
      continue;
    }
    // points of one wave nearly always belong to one item: take the items one at
    // a time, each pass with a uniform item.  The loop runs on a ballot mask, so
    // its trip count is the same in every lane and the body stays inside it.
    // Only the record's item is read before the loop (the whole record inside).
    const int32_t my = a.rec[tri].item;
    uint64_t todo = __builtin_amdgcn_ballot_w64(true);
    while (todo) {
      const int32_t cur = __builtin_amdgcn_readlane(my, (int32_t)__builtin_ctzll(todo));
      const bool mine = my == cur;
      if (mine) {
        const Item it = load_uniform(a.items + cur);
        const TriRec T = a.rec[tri];
        splat_point<kPBR>(it, pt, T, flags, i, j, tx, ty, a, p, written);
      }
      todo &= ~__builtin_amdgcn_ballot_w64(mine);
    }
  }
  const uint64_t wsum = wave_sum((uint64_t)written);
  if ((threadIdx.x & 63) == 0 && wsum) atomicAdd((unsigned long long*)&a.stats[STAT_WRITTEN], (unsigned long long)wsum);
}

// ------------------------------------------------------------------ a3: splat, row-band quilt
//
// The keys of one tile -- q_rows pixel rows of q_views views, all W columns --
// stay in LDS while every point whose splat reaches those rows is splatted
// into them (64-bit ds_min), and the finished tile is written out as the
// views' RGBA8 (+ depth): the key buffer in HBM is neither updated nor
// resolved.  The views differ only by a horizontal eye offset (Sec. 3.2), so a
// point's pixel rows are the same in every view and each point is binned once
// per frame, into every band of q_rows rows that its splat can reach (in a
// batch, the bands of its own item).  A workgroup takes one tile; tiles are
// launched by decreasing band size.  Workgroups have 1024 threads (16 waves,
// one tile per CU), or 512 when two tiles fit the CU's LDS.

constexpr int kQChunk = 4096;  // points per workgroup pass in the band kernels

// Band (over all items) of stacked row g = item * H + row.
__device__ __forceinline__ uint32_t quilt_band(const QuiltBinArgs& a, uint32_t g) {
  const uint32_t item = g / (uint32_t)a.H;
  return item * (uint32_t)a.bands_item + (g - item * (uint32_t)a.H) / (uint32_t)a.rows;
}

// Pass 1: entries per band (a workgroup histogram in LDS, one global add per
// band it touched).
__global__ void __launch_bounds__(256) k_qcount(QuiltBinArgs a) {
  extern __shared__ uint32_t qhist[];
  for (int k = threadIdx.x; k < a.bands; k += blockDim.x) qhist[k] = 0u;
  __syncthreads();
  const uint64_t npts = imin((int64_t)*a.n_points, a.cap);
  for (uint64_t c = (uint64_t)blockIdx.x * kQChunk; c < npts; c += (uint64_t)gridDim.x * kQChunk) {
    const uint64_t end = c + kQChunk < npts ? c + kQChunk : npts;
    for (uint64_t p = c + threadIdx.x; p < end; p += blockDim.x) {
      const uint2 pr = a.prows[p];
      if (pr.x != ~0u)
        for (uint32_t b = quilt_band(a, pr.x), b1 = quilt_band(a, pr.y); b <= b1; ++b) atomicAdd(&qhist[b], 1u);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < a.bands; k += blockDim.x)
    if (qhist[k]) atomicAdd(&a.band_cnt[k], qhist[k]);
}

// Pass 2 (one workgroup): band offsets and cursors, the overflow flag, and
// the bands sorted by decreasing entries (bitonic sort in LDS) so that the
// largest tiles start first.  Leaves the band counts at zero.
__global__ void __launch_bounds__(1024) k_qplan(QuiltBinArgs a) {
  constexpr int kPer = kQuiltBandCap / 1024;  // bands per thread
  __shared__ uint64_t sk[kQuiltBandCap];
  __shared__ uint64_t wtot[16];
  const int nb = a.bands, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t c[kPer];
  uint64_t t = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int b = tid * kPer + k;
    c[k] = b < nb ? a.band_cnt[b] : 0u;
    t += c[k];
  }
  const uint64_t inc = wave_incl_scan(t);
  if (lane == 63) wtot[wv] = inc;
  __syncthreads();
  uint64_t run = inc - t, total = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wv) run += wtot[w];
    total += wtot[w];
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int b = tid * kPer + k;
    if (b < nb) {
      const uint32_t o = run < 0xFFFFFFFFull ? (uint32_t)run : 0xFFFFFFFFu;
      a.band_off[b] = o;
      a.band_cur[b] = o;
      a.band_cnt[b] = 0u;
      sk[b] = ((uint64_t)c[k] << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)b);
    }
    run += c[k];
  }
  if (tid == 0) {
    const bool over = total > (uint64_t)a.entry_cap;
    a.band_off[nb] = over ? 0xFFFFFFFFu : (uint32_t)total;
    a.state[0] = over ? 1u : 0u;
    a.state[1] = total < 0xFFFFFFFFull ? (uint32_t)total : 0xFFFFFFFFu;
  }
  int n2 = 1;
  while (n2 < nb) n2 <<= 1;
  for (int b = nb + tid; b < n2; b += blockDim.x) sk[b] = 0ull;  // below every band's key
  __syncthreads();
  for (int size = 2; size <= n2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < n2; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const uint64_t x = sk[i], y = sk[j];
          const bool desc = (i & size) == 0;
          if (desc ? x < y : x > y) {
            sk[i] = y;
            sk[j] = x;
          }
        }
      }
      __syncthreads();
    }
  for (int k = tid; k < nb; k += blockDim.x) a.order[k] = 0xFFFFFFFFu - (uint32_t)sk[k];
}

// Pass 3: the band lists.  A workgroup counts its points' entries per band in
// LDS, reserves each band's share with one global add, then places them.
__global__ void __launch_bounds__(256) k_qscatter(QuiltBinArgs a) {
  if (a.state[0]) return;  // overflow: the point splat takes the frame
  extern __shared__ uint32_t qsh[];
  uint32_t* hist = qsh;
  uint32_t* base = qsh + a.bands;
  for (int k = threadIdx.x; k < a.bands; k += blockDim.x) hist[k] = 0u;
  __syncthreads();
  const uint64_t npts = imin((int64_t)*a.n_points, a.cap);
  const uint64_t step = (uint64_t)gridDim.x * kQChunk;
  for (uint64_t c = (uint64_t)blockIdx.x * kQChunk; c < npts; c += step) {
    const uint64_t end = c + kQChunk < npts ? c + kQChunk : npts;
    for (uint64_t p = c + threadIdx.x; p < end; p += blockDim.x) {
      const uint2 pr = a.prows[p];
      if (pr.x != ~0u)
        for (uint32_t b = quilt_band(a, pr.x), b1 = quilt_band(a, pr.y); b <= b1; ++b) atomicAdd(&hist[b], 1u);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < a.bands; k += blockDim.x)
    if (hist[k]) {
      base[k] = atomicAdd(&a.band_cur[k], hist[k]);
      hist[k] = 0u;
    }
  __syncthreads();
  for (uint64_t c = (uint64_t)blockIdx.x * kQChunk; c < npts; c += step) {
    const uint64_t end = c + kQChunk < npts ? c + kQChunk : npts;
    for (uint64_t p = c + threadIdx.x; p < end; p += blockDim.x) {
      const uint2 pr = a.prows[p];
      if (pr.x != ~0u)
        for (uint32_t b = quilt_band(a, pr.x), b1 = quilt_band(a, pr.y); b <= b1; ++b)
          a.entries[base[b] + atomicAdd(&hist[b], 1u)] = (uint32_t)p;
    }
  }
}

// One tile per workgroup: clear the keys, splat the band's points into the
// tile's views and rows, write the tile out into its item's views.  kPBR:
// shaded colours.  Held to 128 VGPRs: four waves per SIMD.
template <bool kPBR, int kBlock>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) k_splat_quilt(SplatArgs a) {
  extern __shared__ uint64_t qtile[];  // the tile's keys, then W column and H row ray slopes
  __shared__ uint32_t qnext;           // next unclaimed entry of the band
  if (*a.q_state != 0) return;         // overflow: the point splat takes the frame
  const Rig& trg = a.table_rig;
  const int32_t W = trg.W, H = trg.H;
  // Workgroups go to the 8 XCDs round robin (block b on XCD b % 8).  XCD x
  // takes the bands of rank x, x + 8, ... (ranks by decreasing size, so the
  // XCDs get equal shares), each band's view subsets on consecutive blocks of
  // that XCD: the subsets read the same points through one L2.  The grid is
  // padded to whole rounds of 8 bands; blocks past the last band exit.
  const uint32_t xcd = blockIdx.x & 7u, k = blockIdx.x >> 3;
  const uint32_t rank = (k / (uint32_t)a.q_subsets) * 8u + xcd, sub = k % (uint32_t)a.q_subsets;
  if (rank >= (uint32_t)a.q_bands) return;
  const int32_t band = (int32_t)a.q_order[rank];
  const int32_t item = band / a.q_bands_item, lband = band - item * a.q_bands_item;  // the band within its item
  QuiltTile qt;
  qt.keys = qtile;
  qt.rows = a.q_rows;
  qt.y_lo = lband * a.q_rows;
  qt.y_hi = min(H - 1, qt.y_lo + a.q_rows - 1);
  qt.r_lo = (int32_t)sub * a.q_views;
  qt.r_hi = min(trg.n_views, qt.r_lo + a.q_views);
  const int32_t nkeys = a.q_rows * a.q_views * W;
  float* tx = reinterpret_cast<float*>(qtile + nkeys);
  float* ty = tx + W;
  for (int32_t k = threadIdx.x; k < nkeys; k += blockDim.x) qtile[k] = ~0ull;
  for (int k = threadIdx.x; k < W; k += blockDim.x) tx[k] = ((float)k + 0.5f - trg.cx) / trg.fx;
  for (int k = threadIdx.x; k < H; k += blockDim.x) ty[k] = ((float)k + 0.5f - trg.cy) / trg.fy;
  if (threadIdx.x == 0) qnext = 0u;
  __syncthreads();
  const uint32_t e0 = a.q_band_off[band], e1 = a.q_band_off[band + 1];
  const Item it0 = load_uniform(a.items + item);
  const int lane = threadIdx.x & 63;
  uint32_t written = 0;
  // the band's entries in chunks of 64, one chunk per wave at a time, taken
  // from an LDS counter as the waves free up: the tile ends when its last
  // chunk does, whatever the per-point work
  for (;;) {
    uint32_t c = 0;
    if (lane == 0) c = atomicAdd(&qnext, 64u);
    c = (uint32_t)__shfl((int)c, 0, 64);
    if (c >= e1 - e0) break;
    const uint32_t e = e0 + c + (uint32_t)lane;
    if (e < e1) {
      const uint32_t p = a.q_entries[e];
      const Point pt = a.points[p];
      const uint32_t tri = pt.tri_flags & 0x0FFFFFFFu, flags = pt.tri_flags >> 28;
      const int32_t i = (int16_t)(pt.ij & 0xFFFFu), j = (int16_t)(pt.ij >> 16);
      const TriRec T = a.rec[tri];
      qt.box = a.pbox + p;
      splat_point<kPBR, true>(it0, pt, T, flags, i, j, tx, ty, a, p, written, &qt);
    }
  }
  __syncthreads();
  // the tile as RGBA8 (+ depth): one pixel row of one view per wave at a time
  const int32_t nrows = qt.y_hi - qt.y_lo + 1, nvt = qt.r_hi - qt.r_lo;
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int32_t q = wv; q < nvt * nrows; q += nw) {
    const int32_t rv = q / nrows, yy = q - rv * nrows;
    const uint64_t* src = qtile + (rv * a.q_rows + yy) * W;
    const int64_t o = (((int64_t)item * trg.n_views + qt.r_lo + rv) * H + (qt.y_lo + yy)) * W;
    for (int32_t x = lane; x < W; x += 64) {
      const uint64_t key = src[x];
      const bool empty = key == ~0ull;
      a.out_rgba[o + x] = empty ? 0u : (uint32_t)key;
      if (a.out_depth) a.out_depth[o + x] = empty ? __uint_as_float(0x7f800000u) : __uint_as_float((uint32_t)(key >> 32));
    }
  }
  const uint64_t wsum = wave_sum((uint64_t)written);
  if (lane == 0 && wsum) atomicAdd((unsigned long long*)&a.stats[STAT_WRITTEN], (unsigned long long)wsum);
}

// ------------------------------------------------------------------ a3: splat, triangle-major
//
// The same splats and keys as k_splat, visited per (triangle, view) instead of
// per point.  A wave takes 64 (triangle, view) pairs; each lane sets its pair
// up (visibility, Q8 vertices, edge functions, pixel bounding box) and the
// wave then walks the concatenated bounding boxes 64 pixels at a time, so that
// every lane works whatever the boxes' sizes.  A pixel inside the triangle
// finds its owning cell by the clamped lattice coordinates of its ray hit
// (row table of the triangle), then applies that point's splat rectangle and
// colour (Eqs. 8-9) from the point's PointBox, and the 64-bit depth test.

// Everything the pixel pass needs of one (triangle, view) pair, in LDS.
struct alignas(16) PairData {
  int32_t qx0, qx1, qx2, qy0;    // Q8 vertices, positively oriented
  int32_t qy1, qy2, xy0, w;      // bounding box origin (x | y << 16) and width
  float delta, cu, cw, ks;       // plane distance of the eye, lattice offsets, lens shift
  float fxfy_ad, b, inv_w, acell;  // fx*fy*|delta| (Eq. 8), eye offset, 1/width, 1/(Sx*Sy)
  uint64_t* kv;                  // keys of this view
  int32_t row_stride;            // keys per pixel row
  float suv;                     // acell * ruv (Eq. 8)
  float nx, ny, nz, ux;          // the triangle's plane and lattice axes
  float uy, uz, wx, wy;
  float wz, sx, sy, ruv;
  float smin, smax, irange;      // Eqs. 4-5, 9
  int32_t jlo;                   // first lattice row
  uint64_t first;                // the triangle's first point
  int32_t jhi, pad;
};
static_assert(sizeof(PairData) == 160, "PairData is ten 16-byte words");
constexpr int kPairWords = 10;

// The pair records of a wave are kept in LDS word-major: word g of pair o at
// [g][o], so that lanes reading consecutive pairs hit consecutive banks.
__device__ __forceinline__ void store_pair(uint4 (*pw)[64], int o, const PairData& P) {
  const uint4* w = reinterpret_cast<const uint4*>(&P);
#pragma unroll
  for (int g = 0; g < kPairWords; ++g) pw[g][o] = w[g];
}

__device__ __forceinline__ PairData load_pair(const uint4 (*pw)[64], int o) {
  PairData P;
  uint4* w = reinterpret_cast<uint4*>(&P);
#pragma unroll
  for (int g = 0; g < kPairWords; ++g) w[g] = pw[g][o];
  return P;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One covered pixel of pair Q: ray hit, owning cell, its splat rectangle and
// colour (Eqs. 8-9), the 64-bit depth test.  Returns 1 when a key was written.
__device__ __forceinline__ uint32_t splat_fragment(const PairData& Q, int32_t x, int32_t y, const float* tx,
                                                   const float* ty, const RowEntry* __restrict__ rows,
                                                   const PointBox* __restrict__ pbox) {
  const float rx = tx[x] - Q.ks, ry = ty[y];
  const float den = (Q.nx * rx + Q.ny * ry) + Q.nz;
  const float Z = Q.delta / den;
  if (!(Z > 0.0f) || isinf(Z)) return 0;
  const float ur = (Q.ux * rx + Q.uy * ry) + Q.uz;
  const float wr = (Q.wx * rx + Q.wy * ry) + Q.wz;
  const float sv = Q.sx * (Z * ur + Q.cu) + 0.5f;
  const float tv = Q.sy * (Z * wr + Q.cw) + 0.5f;
  // owning cell: clamp to the lattice rows, then to the row's cells
  int32_t cj = (int32_t)floorf(clamp_big(tv));
  cj = cj < Q.jlo ? Q.jlo : (cj > Q.jhi ? Q.jhi : cj);
  const RowEntry R = rows[Q.first + (uint64_t)(cj - Q.jlo)];
  int32_t ci = (int32_t)floorf(clamp_big(sv));
  ci = ci < R.ilo ? R.ilo : (ci > R.ihi ? R.ihi : ci);
  const PointBox& B = pbox[Q.first + R.start + (uint32_t)(ci - R.ilo)];
  const int32_t rws = B.rows;
  if (rws != kAllRows) {
    const int32_t r0 = (int16_t)(rws & 0xFFFF), r1 = (int16_t)((uint32_t)rws >> 16);
    if (y < r0 || y > r1) return 0;
    const float b = Q.b;
    float xmn = B.cA[0] - b * B.cC[0], xmx = xmn;
#pragma unroll
    for (int kk = 1; kk < 4; ++kk) {
      const float xx = B.cA[kk] - b * B.cC[kk];
      xmn = xx < xmn ? xx : xmn;
      xmx = xx > xmx ? xx : xmx;
    }
    if (x < (int32_t)ceilf(clamp_big(xmn - 0.515625f)) || x > (int32_t)floorf(clamp_big(xmx - 0.484375f))) return 0;
  }
  // colour of the point in this view (Eqs. 8-9)
  const float Ar = B.zc3 / Q.fxfy_ad;
  const float vse = Q.acell < Ar ? Q.ruv * Ar : Q.suv;
  const float vs = vse < Q.smin ? Q.smin : (vse > Q.smax ? Q.smax : vse);
  const float tau = (vs - Q.smin) * Q.irange;
  int32_t tq = (int32_t)floorf(tau * 256.0f + 0.5f);
  tq = tq < 0 ? 0 : (tq > 256 ? 256 : tq);
  const uint32_t wa = (uint32_t)(256 - tq), wz = (uint32_t)tq;
  const uint32_t lo = B.tvmin, hi = B.tvmax;
  const uint32_t col =
      ((((lo & 0x00FF00FFu) * wa + (hi & 0x00FF00FFu) * wz + 0x00800080u) >> 8) & 0x00FF00FFu) |
      (((((lo >> 8) & 0x00FF00FFu) * wa + ((hi >> 8) & 0x00FF00FFu) * wz + 0x00800080u) >> 8) & 0x00FF00FFu) << 8;
  key_min(&Q.kv[(int64_t)y * Q.row_stride + x], ((uint64_t)__float_as_uint(Z) << 32) | col);
  return 1;
}

template <bool kMulti>
__global__ void __launch_bounds__(256) k_splat_tv(SplatArgs a) {
  extern __shared__ float ray_tab[];  // W column slopes, then H row slopes
  __shared__ uint4 pd[4][kPairWords][64];
  __shared__ uint32_t poff[4][64];
  __shared__ uint32_t fq[4][128];     // covered pixels waiting: pair | x << 6 | y << 19
  const Rig& trg = a.table_rig;
  float* tx = ray_tab;
  float* ty = ray_tab + trg.W;
  for (int k = threadIdx.x; k < trg.W; k += blockDim.x) tx[k] = ((float)k + 0.5f - trg.cx) / trg.fx;
  for (int k = threadIdx.x; k < trg.H; k += blockDim.x) ty[k] = ((float)k + 0.5f - trg.cy) / trg.fy;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int32_t V = trg.n_views;
  const int64_t npairs = (int64_t)imin((int64_t)*a.n_tris, a.nt) * V;
  const Item it0 = load_uniform(a.items);
  uint4 (*const mypd)[64] = pd[wv];
  uint32_t* const myoff = poff[wv];
  uint32_t* const myq = fq[wv];
  uint32_t written = 0, covered = 0;  // key updates; covered pixels visited (the hole census)
  const int64_t chunks = (npairs + 63) >> 6;
  for (int64_t c = (int64_t)blockIdx.x * 4 + wv; c < chunks; c += (int64_t)gridDim.x * 4) {
    // ---- phase A: one (triangle, view) pair per lane
    const int64_t k = c * 64 + lane;
    uint32_t npx = 0;
    PairData P;
    if (k < npairs) {
      const uint32_t ti = (uint32_t)k / (uint32_t)V;
      const int32_t r = (int32_t)((uint32_t)k - ti * (uint32_t)V);
      const uint32_t tri = a.tris[ti];
      const TriRec& T = a.rec[tri];
      const Item& it = kMulti ? a.items[T.item] : it0;
      const Rig& rg = it.rig;
      // every point of the triangle must be in the buffer (else the frame
      // overflowed and the triangle is left out)
      const uint64_t first = a.offsets[tri];
      const bool fits = first + a.counts[tri] <= (uint64_t)a.cap;
      const float b = fits && r < rg.n_views ? rg.eye[r] : 0.0f;
      const float delta = T.h - T.nx * b;
      const int32_t H8 = 256 * rg.H, W8 = 256 * rg.W;
      bool act = fits && r < rg.n_views && faces_eye(T.p0x, T.p0y * T.p0y, T.p0z * T.p0z, delta, b);
      int32_t qx[3], qy[3];
      if (act) act = q8_xy(T.a0, T.c0, T.y0, b, qx[0], qy[0]) && q8_xy(T.a1, T.c1, T.y1, b, qx[1], qy[1]) &&
                     q8_xy(T.a2, T.c2, T.y2, b, qx[2], qy[2]);
      if (act && ((qx[0] < 0 && qx[1] < 0 && qx[2] < 0) || (qx[0] > W8 && qx[1] > W8 && qx[2] > W8) ||
                  (qy[0] < 0 && qy[1] < 0 && qy[2] < 0) || (qy[0] > H8 && qy[1] > H8 && qy[2] > H8)))
        act = false;
      if (act) {
        const int64_t a2 = (int64_t)(qx[1] - qx[0]) * (qy[2] - qy[0]) - (int64_t)(qy[1] - qy[0]) * (qx[2] - qx[0]);
        if (a2 == 0) act = false;
        if (a2 < 0) {
          int32_t u = qx[1]; qx[1] = qx[2]; qx[2] = u;
          u = qy[1]; qy[1] = qy[2]; qy[2] = u;
        }
      }
      if (act) {
        const int32_t xmin = min(qx[0], min(qx[1], qx[2])), xmax = max(qx[0], max(qx[1], qx[2]));
        const int32_t ymin = min(qy[0], min(qy[1], qy[2])), ymax = max(qy[0], max(qy[1], qy[2]));
        const int32_t X0 = max(0, -((128 - xmin) >> 8)), X1 = min(rg.W - 1, (xmax - 128) >> 8);
        const int32_t Y0 = max(0, -((128 - ymin) >> 8)), Y1 = min(rg.H - 1, (ymax - 128) >> 8);
        if (X0 <= X1 && Y0 <= Y1) {
          const int32_t w = X1 - X0 + 1;
          npx = (uint32_t)(w * (Y1 - Y0 + 1));
          P.qx0 = qx[0]; P.qx1 = qx[1]; P.qx2 = qx[2];
          P.qy0 = qy[0]; P.qy1 = qy[1]; P.qy2 = qy[2];
          P.xy0 = X0 | (Y0 << 16);
          P.w = w;
          P.delta = delta;
          P.cu = T.ux * (b - T.p0x) - T.cu0;
          P.cw = T.wx * (b - T.p0x) - T.cw0;
          P.ks = rg.kshift[r];
          P.fxfy_ad = rg.fxfy * fabsf(delta);
          P.b = b;
          P.inv_w = 1.0f / (float)w;
          const bool rowmajor = it.key_layout != 0;
          P.kv = it.keys + (rowmajor ? (int64_t)r * rg.W : (int64_t)r * rg.W * rg.H);
          P.row_stride = rowmajor ? rg.n_views * rg.W : rg.W;
          P.acell = 1.0f / (T.sx * T.sy);
          P.suv = P.acell * T.ruv;
          P.nx = T.nx; P.ny = T.ny; P.nz = T.nz;
          P.ux = T.ux; P.uy = T.uy; P.uz = T.uz;
          P.wx = T.wx; P.wy = T.wy; P.wz = T.wz;
          P.sx = T.sx; P.sy = T.sy; P.ruv = T.ruv;
          P.smin = T.smin; P.smax = T.smax; P.irange = T.irange;
          const int2 jr = *reinterpret_cast<const int2*>(&a.em[tri].jlo);
          P.jlo = jr.x;
          P.jhi = jr.y;
          P.first = first;
          P.pad = 0;
        }
      }
    }
    // exclusive offsets of the pixel boxes; pair data to LDS
    uint32_t inc = npx;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    const uint32_t total = __shfl(inc, 63, 64);
    if (total == 0) continue;
    myoff[lane] = inc - npx;
    if (npx) store_pair(mypd, lane, P);
    wave_sync_lds();
    // ---- phase B: 64 box pixels per round over the concatenated boxes; the
    // covered ones queue up and are splatted 64 at a time
    uint32_t qn = 0;
    for (uint32_t base = 0; base < total; base += 64) {
      const uint32_t u = base + lane;
      bool cov = false;
      uint32_t entry = 0;
      if (u < total) {
        int o = 0;
#pragma unroll
        for (int st = 32; st >= 1; st >>= 1)
          if (myoff[o + st] <= u) o += st;
        const uint4 g0 = mypd[0][o], g1 = mypd[1][o];
        const float inv_w = __uint_as_float(mypd[3][o].z);
        const int32_t q = (int32_t)(u - myoff[o]);
        const int32_t w = (int32_t)g1.w, xy0 = (int32_t)g1.z;
        int32_t yq = (int32_t)((float)q * inv_w);
        int32_t xq = q - yq * w;
        if (xq < 0) { yq -= 1; xq += w; }
        else if (xq >= w) { yq += 1; xq -= w; }
        const int32_t x = (xy0 & 0xFFFF) + xq, y = (xy0 >> 16) + yq;
        const int32_t pxq = 256 * x + 128, pyq = 256 * y + 128;
        const int32_t qx0 = (int32_t)g0.x, qx1 = (int32_t)g0.y, qx2 = (int32_t)g0.z, qy0 = (int32_t)g0.w,
                      qy1 = (int32_t)g1.x, qy2 = (int32_t)g1.y;
        // edge functions in 64-bit integers; an edge owns its ties iff dy > 0 || (dy == 0 && dx > 0)
        auto inside = [](int32_t ax, int32_t ay, int32_t bx, int32_t by, int32_t px, int32_t py) {
          const int32_t dx = bx - ax, dy = by - ay;
          const int64_t E = (int64_t)dx * (py - ay) - (int64_t)dy * (px - ax);
          return E > 0 || (E == 0 && (dy > 0 || (dy == 0 && dx > 0)));
        };
        cov = inside(qx0, qy0, qx1, qy1, pxq, pyq) && inside(qx1, qy1, qx2, qy2, pxq, pyq) &&
              inside(qx2, qy2, qx0, qy0, pxq, pyq);
        entry = (uint32_t)o | ((uint32_t)x << 6) | ((uint32_t)y << 19);
      }
      const uint64_t m = __builtin_amdgcn_ballot_w64(cov);
      if (cov) myq[qn + (uint32_t)__builtin_popcountll(m & below)] = entry;
      qn += (uint32_t)__builtin_popcountll(m);
      if (qn >= 64) {
        wave_sync_lds();
        const uint32_t e = myq[lane];
        covered += 1;
        written += splat_fragment(load_pair(mypd, (int)(e & 63)), (int32_t)((e >> 6) & 0x1FFF), (int32_t)(e >> 19), tx,
                                  ty, a.rows, a.pbox);
        const uint32_t rest = qn - 64;
        const uint32_t moved = lane < rest ? myq[64 + lane] : 0u;
        wave_sync_lds();
        if (lane < rest) myq[lane] = moved;
        qn = rest;
      }
    }
    if (qn) {
      wave_sync_lds();
      if ((uint32_t)lane < qn) {
        const uint32_t e = myq[lane];
        covered += 1;
        written += splat_fragment(load_pair(mypd, (int)(e & 63)), (int32_t)((e >> 6) & 0x1FFF), (int32_t)(e >> 19), tx,
                                  ty, a.rows, a.pbox);
      }
    }
    wave_sync_lds();  // the pair data and the queue are rewritten for the next chunk
  }
  const uint64_t wsum = wave_sum((uint64_t)written), csum = wave_sum((uint64_t)covered);
  if (lane == 0 && wsum) atomicAdd((unsigned long long*)&a.stats[STAT_WRITTEN], (unsigned long long)wsum);
  if (lane == 0 && csum) atomicAdd((unsigned long long*)&a.stats[STAT_COVERED], (unsigned long long)csum);
}

// keys -> RGBA8 (+ depth) in [item][view][y][x] order; keys re-cleared.
__global__ void k_resolve(uint64_t* __restrict__ keys, int64_t n, int32_t nv, int32_t H, int32_t W, int32_t layout,
                          uint32_t* __restrict__ rgba, float* __restrict__ depth, const uint32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t per_view = (int64_t)W * H, per_item = per_view * nv;
  for (; i < n; i += stride) {
    int64_t k = i;
    if (layout) {
      const int64_t b = i / per_item, rem = i % per_item;
      const int64_t r = rem / per_view, q = rem % per_view;
      const int64_t y = q / W, x = q % W;
      k = b * per_item + (y * nv + r) * W + x;
    }
    const uint64_t key = keys[k];
    const bool empty = key == ~0ull;
    rgba[i] = empty ? 0u : (uint32_t)key;
    if (depth) depth[i] = empty ? __uint_as_float(0x7f800000u) : __uint_as_float((uint32_t)(key >> 32));
    keys[k] = ~0ull;
  }
}

// ------------------------------------------------------------------ a4: interleave + reconstruction

// Logical block of a 1-D launch of nb blocks such that the blocks the
// hardware places on one XCD (round robin over 8) take one contiguous eighth
// of the logical order: neighbouring tiles share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t per = nb / 8, extra = nb % 8, xcd = b % 8, k = b / 8;
  // XCD x takes per (+1 for the first `extra`) consecutive logical blocks
  return xcd * per + (xcd < extra ? xcd : extra) + k;
}

// One lane per four consecutive panel pixels (12 bytes, written as three
// 32-bit words when they are aligned and whole).  Panel rows are spread over
// the XCDs in contiguous bands so that each view row is fetched into one L2.
__global__ void __launch_bounds__(256) k_interleave(InterleaveArgs a, uint32_t blocks_per_row, uint32_t nblocks) {
  const uint32_t L = xcd_block(blockIdx.x, nblocks);
  const int64_t Y = L / blocks_per_row;
  const int64_t X0 = ((int64_t)(L % blocks_per_row) * blockDim.x + threadIdx.x) * 4;
  if (Y >= a.Hp || X0 >= a.Wp) return;
  const int64_t yq = ((2 * Y + 1) * (int64_t)a.Hv * 128) / a.Hp;
  uint32_t bytes[12];
  const int nx = a.Wp - X0 < 4 ? (int)(a.Wp - X0) : 4;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t X = X0 + k;
    const int64_t xq = ((2 * X + 1) * (int64_t)a.Wv * 128) / a.Wp;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uint32_t val = 0;
      if (k < nx) {
        const uint32_t phi = (uint32_t)(3 * X + c) * a.K1 + (uint32_t)Y * a.Ky + a.K0;
        const uint64_t U = (uint64_t)phi * (uint64_t)a.V;
        if (a.mode == 0) {
          const int64_t v = (int64_t)(U >> 32);
          val = (a.views[(v * a.Hv + (yq >> 8)) * a.Wv + (xq >> 8)] >> (8 * c)) & 255u;
        } else {
          uint32_t sum = 0;
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            int64_t v = ((int64_t)U + a.du[t]) >> 32;
            int64_t x = (xq + a.dx[t]) >> 8, y = (yq + a.dy[t]) >> 8;
            v = v < 0 ? 0 : (v > a.V - 1 ? a.V - 1 : v);
            x = x < 0 ? 0 : (x > a.Wv - 1 ? a.Wv - 1 : x);
            y = y < 0 ? 0 : (y > a.Hv - 1 ? a.Hv - 1 : y);
            sum += (a.views[(v * a.Hv + y) * a.Wv + x] >> (8 * c)) & 255u;
          }
          val = (sum + 4u) >> 3;
        }
      }
      bytes[3 * k + c] = val;
    }
  }
  uint8_t* dst = a.panel + (Y * a.Wp + X0) * 3;
  if (nx == 4 && ((uintptr_t)dst & 3) == 0) {
    uint32_t* d32 = reinterpret_cast<uint32_t*>(dst);
    d32[0] = bytes[0] | (bytes[1] << 8) | (bytes[2] << 16) | (bytes[3] << 24);
    d32[1] = bytes[4] | (bytes[5] << 8) | (bytes[6] << 16) | (bytes[7] << 24);
    d32[2] = bytes[8] | (bytes[9] << 8) | (bytes[10] << 16) | (bytes[11] << 24);
  } else {
    for (int k = 0; k < 3 * nx; ++k) dst[k] = (uint8_t)bytes[k];
  }
}

// Angular supersampling filter, one lane per four consecutive pixels of an
// output view (16-byte loads and stores where whole).  Per channel the
// weighted sum fits 32 bits (weights < 2^16, at most 3S sub-views); the
// rounded quotient (acc + ws/2) div ws is taken exactly from a double
// reciprocal and one integer correction step.
__global__ void __launch_bounds__(256) k_angular_filter(AngularArgs a) {
  const int v = blockIdx.y;
  const int64_t npx = (int64_t)a.W * a.H;
  const int64_t p0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (p0 >= npx) return;
  const int n = a.cnt[v];
  uint32_t ws = 0;
  for (int e = 0; e < n; ++e) ws += a.wt[v * a.maxe + e];
  const double rcp = 1.0 / (double)ws;
  const uint32_t half = ws / 2;
  const bool whole = p0 + 4 <= npx && (npx & 3) == 0;
  uint32_t acc[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[k][c] = 0u;
  for (int e = 0; e < n; ++e) {
    const uint32_t w = a.wt[v * a.maxe + e];
    const uint32_t* row = a.sub + (int64_t)a.src[v * a.maxe + e] * npx + p0;
    uint32_t px[4];
    if (whole) {
      const uint4 q = *reinterpret_cast<const uint4*>(row);
      px[0] = q.x; px[1] = q.y; px[2] = q.z; px[3] = q.w;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) px[k] = p0 + k < npx ? row[k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[k][c] += w * ((px[k] >> (8 * c)) & 255u);
  }
  uint32_t o[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o[k] = 0u;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t num = acc[k][c] + half;
      uint32_t q = (uint32_t)((double)num * rcp);
      const int64_t r = (int64_t)num - (int64_t)q * ws;
      if (r >= (int64_t)ws) q += 1;
      else if (r < 0) q -= 1;
      o[k] |= q << (8 * c);
    }
  }
  uint32_t* dst = a.out + (int64_t)v * npx + p0;
  if (whole) {
    *reinterpret_cast<uint4*>(dst) = make_uint4(o[0], o[1], o[2], o[3]);
  } else {
    for (int k = 0; k < 4; ++k)
      if (p0 + k < npx) dst[k] = o[k];
  }
}

// ------------------------------------------------------------------ launchers

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = (unsigned)imin(nblk(n, 256), 256 * 64);
  k_fill_u64<<<g, 256, 0, s>>>(p, n, v);
}

void launch_store_item(const Item& it, Item* dst, hipStream_t s) { k_store_item<<<1, 64, 0, s>>>(it, dst); }

void launch_export_stats(const uint64_t* st, int64_t cap, int64_t* out, hipStream_t s) {
  k_export_stats<<<1, 64, 0, s>>>(st, cap, out);
}

void launch_build_mip(const uint32_t* src, uint32_t* dst, int s, hipStream_t st) {
  int64_t n = (int64_t)(s >> 1) * (s >> 1);
  k_build_mip<<<nblk(n, 256), 256, 0, st>>>(src, dst, s);
}

void launch_tri_setup(const SetupArgs& a, bool lean, hipStream_t s) {
  if (a.nt <= 0) return;
  const unsigned g = nblk(a.nt, 256);
  if (a.n_items > 1 && lean)
    k_tri_setup<true, true><<<g, 256, 0, s>>>(a);
  else if (a.n_items > 1)
    k_tri_setup<true, false><<<g, 256, 0, s>>>(a);
  else if (lean)
    k_tri_setup<false, true><<<g, 256, 0, s>>>(a);
  else
    k_tri_setup<false, false><<<g, 256, 0, s>>>(a);
}

void launch_interleave_batch(const InterleaveArgs& a, int n_items, int64_t view_stride, int64_t panel_stride,
                             hipStream_t s) {
  for (int b = 0; b < n_items; ++b) {
    InterleaveArgs c = a;
    c.views = a.views + view_stride * b;
    c.panel = a.panel + panel_stride * b;
    launch_interleave(c, s);
  }
}

void launch_scan(uint64_t* tile_sum, int64_t nt, uint64_t* total, hipStream_t s) {
  k_scan_top<<<1, 1024, 0, s>>>(tile_sum, (nt + kScanTile - 1) / kScanTile, total);
}

void launch_emit(const EmitArgs& a, int fetch_blocks, hipStream_t s) {
  if (a.nt <= 0) return;
  k_emit<<<kEmitBigBlocks + nblk(a.nt, kScanTile), 256, 0, s>>>(a);
  if (a.pbox && a.tm)
    k_fetch<true, true><<<fetch_blocks, 256, 0, s>>>(a);
  else if (a.pbox)
    k_fetch<true, false><<<fetch_blocks, 256, 0, s>>>(a);
  else if (a.tm)
    k_fetch<false, true><<<fetch_blocks, 256, 0, s>>>(a);
  else
    k_fetch<false, false><<<fetch_blocks, 256, 0, s>>>(a);
}

void launch_splat(const SplatArgs& a, int grid_blocks, hipStream_t s) {
  size_t lds = sizeof(float) * (size_t)(a.table_rig.W + a.table_rig.H);
  if (a.pbox && !a.tm) {
    if (a.n_items > 1)
      k_splat_tv<true><<<grid_blocks, 256, lds, s>>>(a);
    else
      k_splat_tv<false><<<grid_blocks, 256, lds, s>>>(a);
    return;
  }
  if (a.n_items > 1 && a.tm)
    k_splat<true, true><<<grid_blocks, 256, lds, s>>>(a);
  else if (a.n_items > 1)
    k_splat<true, false><<<grid_blocks, 256, lds, s>>>(a);
  else if (a.tm)
    k_splat<false, true><<<grid_blocks, 256, lds, s>>>(a);
  else
    k_splat<false, false><<<grid_blocks, 256, lds, s>>>(a);
}

void launch_resolve(uint64_t* keys, int64_t n_items, int32_t n_views, int32_t H, int32_t W, int32_t key_layout,
                    uint32_t* rgba, float* depth, hipStream_t s, const uint32_t* gate) {
  const int64_t n = n_items * n_views * (int64_t)H * W;
  // a gated resolve is a fallback that nearly always exits at once: a small grid
  unsigned g = (unsigned)imin(nblk(n, 256), gate ? 1024 : 256 * 64);
  k_resolve<<<g, 256, 0, s>>>(keys, n, n_views, H, W, key_layout, rgba, depth, gate);
}

constexpr size_t kQuiltStaticLds = 16;  // the workgroup's entry counter

size_t quilt_lds_bytes(int32_t rows, int32_t views, int32_t W, int32_t H) {
  return (size_t)rows * (size_t)views * (size_t)W * 8u + (size_t)(W + H) * 4u + kQuiltStaticLds;
}

void launch_quilt_bin(const QuiltBinArgs& a, hipStream_t s) {
  const unsigned g = (unsigned)imin(nblk(a.cap, kQChunk), 1024);
  k_qcount<<<g, 256, sizeof(uint32_t) * (size_t)a.bands, s>>>(a);
  k_qplan<<<1, 1024, 0, s>>>(a);
  k_qscatter<<<g, 256, 2 * sizeof(uint32_t) * (size_t)a.bands, s>>>(a);
}

hipError_t prepare_quilt_kernels(size_t lds) {
  const int dyn = (int)(lds - kQuiltStaticLds);
  const void* ks[] = {(const void*)k_splat_quilt<false, 512>, (const void*)k_splat_quilt<false, 1024>,
                      (const void*)k_splat_quilt<true, 512>, (const void*)k_splat_quilt<true, 1024>};
  for (const void* k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_splat_quilt(const SplatArgs& a, hipStream_t s) {
  const size_t lds = quilt_lds_bytes(a.q_rows, a.q_views, a.table_rig.W, a.table_rig.H) - kQuiltStaticLds;
  const unsigned g = (unsigned)((a.q_bands + 7) / 8) * 8u * (unsigned)a.q_subsets;
  if (a.q_block == 512) {
    if (a.tm) k_splat_quilt<true, 512><<<g, 512, lds, s>>>(a);
    else k_splat_quilt<false, 512><<<g, 512, lds, s>>>(a);
  } else {
    if (a.tm) k_splat_quilt<true, 1024><<<g, 1024, lds, s>>>(a);
    else k_splat_quilt<false, 1024><<<g, 1024, lds, s>>>(a);
  }
  // the error stays set for callers that check it after the frame's launches
  return hipPeekAtLastError();
}

void launch_interleave(const InterleaveArgs& a, hipStream_t s) {
  const uint32_t per_row = nblk(a.Wp, 256 * 4);
  const uint32_t nb = per_row * (uint32_t)a.Hp;
  k_interleave<<<nb, 256, 0, s>>>(a, per_row, nb);
}

void launch_angular_filter(const AngularArgs& a, hipStream_t s) {
  dim3 g(nblk(((int64_t)a.W * a.H + 3) / 4, 256), (unsigned)a.V);
  k_angular_filter<<<g, 256, 0, s>>>(a);
}

}  // namespace lfdpr
