// C ABI of the LFDPR hot path: context, scene store, rig/lens tables and the
// per-frame launch sequence.  See include/lfdpr.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <string>
#include <algorithm>
#include <vector>

#include "../../include/lfdpr.h"
#include "lfdpr_internal.h"

using namespace lfdpr;

namespace {

struct SceneDev {
  int32_t nv = 0, nt = 0, ntex = 0;
  float* pos = nullptr;
  float* uv = nullptr;
  uint32_t* idx = nullptr;
  uint16_t* tex = nullptr;
  TexInfo* texinfo = nullptr;
  uint8_t* texels = nullptr;
  uint16_t* mat = nullptr;  // nt x (normal, roughness, metallic) texture ids, or null
  int32_t batch_refs = 0;   // live batches rendering this scene
};

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

// Scratch of lfdpr_render_frame_noalloc: every per-frame buffer of one
// unlit frame of at most kNoAllocTris triangles, kNoAllocPoints points and
// kNoAllocKeys keys (views x H x W), at 256-byte aligned offsets.
constexpr int64_t kNoAllocTris = 65536;
constexpr int64_t kNoAllocPoints = 1 << 19;
constexpr int64_t kNoAllocKeys = 1 << 21;
constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kOffItem = 0;
constexpr size_t kOffStats = kOffItem + align256(sizeof(Item));
constexpr size_t kOffCounts = kOffStats + align256(8 * STAT_SLOTS);
constexpr size_t kOffOffsets = kOffCounts + align256(4 * kNoAllocTris);
constexpr size_t kOffTiles = kOffOffsets + align256(8 * kNoAllocTris);
constexpr size_t kOffRec = kOffTiles + align256(8 * (kNoAllocTris / 256 + 1));
constexpr size_t kOffEm = kOffRec + align256(sizeof(TriRec) * kNoAllocTris);
constexpr size_t kOffBig = kOffEm + align256(sizeof(TriEmit) * kNoAllocTris);
constexpr size_t kOffTris = kOffBig + align256(4 * kNoAllocTris);
constexpr size_t kOffPoints = kOffTris + align256(4 * kNoAllocTris);
constexpr size_t kOffRows = kOffPoints + align256(sizeof(Point) * kNoAllocPoints);
constexpr size_t kOffPbox = kOffRows + align256(sizeof(RowEntry) * kNoAllocPoints);
constexpr size_t kOffKeys = kOffPbox + align256(sizeof(PointBox) * kNoAllocPoints);
constexpr size_t kScratchBytes = kOffKeys + 8 * kNoAllocKeys;  // 65.5 MiB
static_assert(kScratchBytes <= (66u << 20), "no-allocation scratch stays within 66 MiB");

}  // namespace

// One copy per device, held until the process ends.  Host code never uses this
// name as an address: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), resolved once.
void* scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device] && g_scratch_err[device] == hipSuccess) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    else g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

}  // namespace

struct lfdpr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  void* scratch = nullptr;  // device address of this device's no-allocation scratch
  std::string err;
  std::map<int32_t, SceneDev> scenes;
  int32_t next_scene = 1;
  int32_t live_children = 0;  // batches and networks created on this context
  // rig
  bool views_set = false;
  lfdpr_view_params vp{};
  std::vector<float> jitter;
  Rig rig{};
  float* d_eye = nullptr;
  float* d_kshift = nullptr;
  float* d_lod_thr = nullptr;
  int64_t cap = 0;
  Point* d_points = nullptr;
  RowEntry* d_rows = nullptr;   // triangle-major splat: lattice row table and
  PointBox* d_pbox = nullptr;   // per-point splat rectangles (point capacity each)
  uint2* d_prows = nullptr;     // quilt: per point its splat's pixel rows (first, last), or ~0
  uint64_t* d_keys = nullptr;
  int64_t n_keys = 0;
  // angular supersampling filter table
  int32_t* d_acnt = nullptr;
  int32_t* d_asrc = nullptr;
  uint32_t* d_awt = nullptr;
  int32_t amaxe = 0;
  // per-triangle buffers
  int64_t tri_cap = 0;
  uint32_t* d_counts = nullptr;
  uint64_t* d_offsets = nullptr;
  TriRec* d_rec = nullptr;
  TriEmit* d_em = nullptr;
  uint64_t* d_tiles = nullptr;
  uint32_t* d_big = nullptr;
  uint32_t* d_tris = nullptr;   // triangles with points
  uint64_t* d_stats = nullptr;
  int64_t last_nt = 0;
  // lens
  bool lens_set = false;
  lfdpr_lens_params lens{};
  // debug records
  float* dbgf = nullptr;
  int32_t* dbgi = nullptr;
  int64_t dbg_cap = 0;
  // single-frame item table (device) and its host copy
  Item* d_item1 = nullptr;
  Item h_item1{};
  // shading: unlit albedo or physically based (material records and per-point
  // material words allocated on first use)
  lfdpr_shading shading{};
  TriMat* d_tm = nullptr;
  int64_t tm_cap = 0;
  uint4* d_pmat = nullptr;
  int64_t pmat_cap = 0;
  bool last_pbr = false;
  int64_t points_alloc = 0;  // points the current d_points holds
  // Frames in flight (lfdpr_set_frames_in_flight).  With 2, a frame's point
  // generation runs on `side` into the second set of per-frame buffers while
  // the previous frame splats on `stream`; the sets are swapped with the
  // fields above at every frame, so the fields always hold the last frame's.
  int frames_in_flight = 1;
  hipStream_t side = nullptr;
  int slot = 0;  // which set the fields hold
  hipEvent_t ev_emitted[2] = {nullptr, nullptr}, ev_splatted[2] = {nullptr, nullptr};
  hipEvent_t ev_caller = nullptr;  // the caller's stream, for debug records written on `side`
  bool splatted_pending[2] = {false, false};
  // the library stream at the start of the last frame: after the caller's
  // work on the frame before it (its presentation), which the next frame's
  // point generation waits for
  hipEvent_t ev_start = nullptr;
  bool start_pending = false;
  struct FrameBufs {
    int64_t points_alloc = 0, tri_cap = 0, tm_cap = 0, pmat_cap = 0, last_nt = 0;
    Point* d_points = nullptr;
    RowEntry* d_rows = nullptr;
    PointBox* d_pbox = nullptr;
    uint2* d_prows = nullptr;
    uint32_t* d_counts = nullptr;
    uint64_t* d_offsets = nullptr;
    TriRec* d_rec = nullptr;
    TriEmit* d_em = nullptr;
    uint64_t* d_tiles = nullptr;
    uint32_t* d_big = nullptr;
    uint32_t* d_tris = nullptr;
    uint64_t* d_stats = nullptr;
    TriMat* d_tm = nullptr;
    uint4* d_pmat = nullptr;
    uint32_t* d_qentries = nullptr;
    uint32_t* d_qband = nullptr;
    int64_t q_entry_cap = 0;
    bool last_pbr = false;
  } other;
  // launch shape of the splat kernel and key layout (autotuned); splat order:
  // LFDPR_SPLAT_POINT or LFDPR_SPLAT_TRIANGLE_VIEW (unlit frames; shaded frames
  // always go point by point)
  int splat_blocks = 4096;
  int key_layout = 0;
  int splat_order = LFDPR_SPLAT_POINT;
  int last_order = LFDPR_SPLAT_POINT;  // the order the last frame's splat used
  // row-band quilt: tile shape asked for (0, 0: chosen per rig), the last
  // frame's, the device's LDS per workgroup, and the band lists (a per-frame
  // buffer, built with the point generation): the entries, and per band
  // counts | offsets (+1) | cursors | order, then the overflow flag and the
  // number of entries
  int quilt_rows = 0, quilt_views = 0;
  int64_t quilt_cap_req = 0;  // band-list entries asked for (0: twice the point capacity + 65536)
  int last_qrows = 0, last_qviews = 0;
  int max_lds = 65536;
  uint32_t* d_qentries = nullptr;
  uint32_t* d_qband = nullptr;
  int64_t q_entry_cap = 0;
  // stage timing: event pairs recorded on the stream
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_marks;
};

namespace {

int fail(lfdpr_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPOK(call)                                                                              \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fail(ctx, LFDPR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
hipError_t dalloc(T*& p, size_t n) {
  p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void**)&p, n * sizeof(T));
}

void free_scene(SceneDev& s) {
  dfree(s.pos);
  dfree(s.uv);
  dfree(s.idx);
  dfree(s.tex);
  dfree(s.texinfo);
  dfree(s.texels);
  dfree(s.mat);
}

// Waits for everything the context enqueued, on its stream and its side stream.
hipError_t sync_all(lfdpr_ctx* ctx) {
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess && ctx->side) e = hipStreamSynchronize(ctx->side);
  return e;
}

// Exchanges the per-frame buffers held in the context's fields with the other set.
void swap_frame_buffers(lfdpr_ctx* ctx) {
  auto& o = ctx->other;
  std::swap(ctx->points_alloc, o.points_alloc);
  std::swap(ctx->tri_cap, o.tri_cap);
  std::swap(ctx->tm_cap, o.tm_cap);
  std::swap(ctx->pmat_cap, o.pmat_cap);
  std::swap(ctx->last_nt, o.last_nt);
  std::swap(ctx->d_points, o.d_points);
  std::swap(ctx->d_rows, o.d_rows);
  std::swap(ctx->d_pbox, o.d_pbox);
  std::swap(ctx->d_prows, o.d_prows);
  std::swap(ctx->d_tris, o.d_tris);
  std::swap(ctx->d_counts, o.d_counts);
  std::swap(ctx->d_offsets, o.d_offsets);
  std::swap(ctx->d_rec, o.d_rec);
  std::swap(ctx->d_em, o.d_em);
  std::swap(ctx->d_tiles, o.d_tiles);
  std::swap(ctx->d_big, o.d_big);
  std::swap(ctx->d_stats, o.d_stats);
  std::swap(ctx->d_tm, o.d_tm);
  std::swap(ctx->d_pmat, o.d_pmat);
  std::swap(ctx->d_qentries, o.d_qentries);
  std::swap(ctx->d_qband, o.d_qband);
  std::swap(ctx->q_entry_cap, o.q_entry_cap);
  std::swap(ctx->last_pbr, o.last_pbr);
  ctx->slot ^= 1;
}

int ensure_tri_buffers(lfdpr_ctx* ctx, int64_t nt);

// The quilt tile for the context's rig: the shape asked for, clipped to the
// rig, or the automatic one (4 rows, else 2, else 1, as long as at least
// min(8, views) views fit; the views spread evenly over the subsets).  False
// when the keys do not fit the device's LDS.
bool quilt_shape_for(const Rig& rg, int max_lds, int want_rows, int want_views, int n_items, int& rows, int& views) {
  auto fits = [&](int r, int v) {
    return quilt_lds_bytes(r, v, rg.W, rg.H) <= (size_t)max_lds &&
           (int64_t)n_items * ((rg.H + r - 1) / r) <= kQuiltBandCap;
  };
  if (want_rows > 0) {
    rows = std::min(want_rows, rg.H);
    views = std::min(want_views, rg.n_views);
    return fits(rows, views);
  }
  for (int r : {4, 2, 1}) {
    if (r > rg.H && r > 1) continue;
    int vmax = 0;
    while (vmax < rg.n_views && fits(r, vmax + 1)) ++vmax;
    if (vmax >= std::min(8, rg.n_views) || (r == 1 && vmax >= 1)) {
      const int subsets = (rg.n_views + vmax - 1) / vmax;
      rows = r;
      views = (rg.n_views + subsets - 1) / subsets;
      return true;
    }
  }
  return false;
}

bool quilt_shape(const lfdpr_ctx* ctx, int& rows, int& views) {
  return quilt_shape_for(ctx->rig, ctx->max_lds, ctx->quilt_rows, ctx->quilt_views, 1, rows, views);
}

// Band lists sized for the context's point capacity: twice as many entries
// as points unless set (a frame that needs more is splatted per point).
int ensure_quilt_buffers(lfdpr_ctx* ctx) {
  // entries and band offsets are 32-bit
  const int64_t ecap = ctx->quilt_cap_req > 0 ? ctx->quilt_cap_req : std::min<int64_t>(2 * ctx->cap + 65536, 0xFFFFFFFFll);
  if (ctx->d_qentries && ctx->q_entry_cap == ecap) return LFDPR_OK;
  if (sync_all(ctx) != hipSuccess) return fail(ctx, LFDPR_EDEVICE, "synchronising before reallocation");
  dfree(ctx->d_qentries);
  dfree(ctx->d_qband);
  ctx->q_entry_cap = 0;
  if (dalloc(ctx->d_qentries, (size_t)ecap) != hipSuccess || dalloc(ctx->d_qband, (size_t)(4 * kQuiltBandCap + 8)) != hipSuccess)
    return fail(ctx, LFDPR_ENOMEM, "quilt band lists");
  if (hipMemset(ctx->d_qband, 0, (4 * kQuiltBandCap + 8) * sizeof(uint32_t)) != hipSuccess)
    return fail(ctx, LFDPR_EDEVICE, "clearing the quilt band counts");
  ctx->q_entry_cap = ecap;
  return LFDPR_OK;
}

// Band-list kernels' arguments over the lists at qb (per band counts |
// offsets (+1) | cursors | order, then the overflow flag and the entries).
QuiltBinArgs quilt_bin_args(uint32_t* qb, uint32_t* entries, int64_t entry_cap, const uint2* prows,
                            const uint64_t* n_points, int64_t cap, int H, int rows, int n_items) {
  QuiltBinArgs qa{};
  qa.n_points = n_points;
  qa.cap = cap;
  qa.prows = prows;
  qa.H = H;
  qa.rows = rows;
  qa.bands_item = (H + rows - 1) / rows;
  qa.bands = qa.bands_item * n_items;
  qa.band_cnt = qb;
  qa.band_off = qb + kQuiltBandCap;
  qa.band_cur = qb + 2 * kQuiltBandCap + 1;
  qa.order = qb + 3 * kQuiltBandCap + 1;
  qa.entries = entries;
  qa.entry_cap = entry_cap;
  qa.state = qb + 4 * kQuiltBandCap + 1;
  return qa;
}

// The tile kernel's arguments: those of the point splat pa plus the lists.
SplatArgs quilt_tile_args(const SplatArgs& pa, const QuiltBinArgs& qa, PointBox* pbox, int views, int max_lds,
                          uint32_t* out_rgba, float* out_depth) {
  SplatArgs qp = pa;
  qp.pbox = pbox;
  qp.q_entries = qa.entries;
  qp.q_band_off = qa.band_off;
  qp.q_order = qa.order;
  qp.q_state = qa.state;
  qp.q_rows = qa.rows;
  qp.q_views = views;
  qp.q_bands = qa.bands;
  qp.q_bands_item = qa.bands_item;
  qp.q_subsets = (pa.table_rig.n_views + views - 1) / views;
  // two tiles per CU when their LDS allows (the device's per-workgroup
  // figure is the CU's LDS on this architecture)
  qp.q_block = 2 * quilt_lds_bytes(qa.rows, views, pa.table_rig.W, pa.table_rig.H) <= (size_t)max_lds ? 512 : 1024;
  qp.out_rgba = out_rgba;
  qp.out_depth = out_depth;
  return qp;
}

// Per-frame buffers of the set in the context's fields, sized for a frame of
// nt triangles (material buffers only for physically based shading).
int prepare_frame_buffers(lfdpr_ctx* ctx, int64_t nt, bool pbr) {
  int rc = ensure_tri_buffers(ctx, nt);
  if (rc) return rc;
  if (!ctx->d_points || !ctx->d_rows || !ctx->d_pbox || !ctx->d_prows || ctx->points_alloc != ctx->cap) {
    if (sync_all(ctx) != hipSuccess) return fail(ctx, LFDPR_EDEVICE, "synchronising before reallocation");
    dfree(ctx->d_points);
    dfree(ctx->d_rows);
    dfree(ctx->d_pbox);
    dfree(ctx->d_prows);
    ctx->points_alloc = 0;
    if (dalloc(ctx->d_points, (size_t)ctx->cap) != hipSuccess || dalloc(ctx->d_rows, (size_t)ctx->cap) != hipSuccess ||
        dalloc(ctx->d_pbox, (size_t)ctx->cap) != hipSuccess || dalloc(ctx->d_prows, (size_t)ctx->cap) != hipSuccess)
      return fail(ctx, LFDPR_ENOMEM, "point buffers");
    ctx->points_alloc = ctx->cap;
  }
  if (!ctx->d_stats) {
    if (dalloc(ctx->d_stats, STAT_SLOTS) != hipSuccess) return fail(ctx, LFDPR_ENOMEM, "statistics");
    if (hipMemset(ctx->d_stats, 0, STAT_SLOTS * sizeof(uint64_t)) != hipSuccess)
      return fail(ctx, LFDPR_EDEVICE, "clearing statistics");
  }
  if (pbr && (ctx->tm_cap < ctx->tri_cap || ctx->pmat_cap != ctx->cap)) {
    if (sync_all(ctx) != hipSuccess) return fail(ctx, LFDPR_EDEVICE, "synchronising before reallocation");
    dfree(ctx->d_tm);
    dfree(ctx->d_pmat);
    ctx->tm_cap = ctx->pmat_cap = 0;
    if (dalloc(ctx->d_tm, (size_t)ctx->tri_cap) != hipSuccess || dalloc(ctx->d_pmat, (size_t)ctx->cap) != hipSuccess)
      return fail(ctx, LFDPR_ENOMEM, "material buffers");
    ctx->tm_cap = ctx->tri_cap;
    ctx->pmat_cap = ctx->cap;
  }
  return LFDPR_OK;
}

int ensure_tri_buffers(lfdpr_ctx* ctx, int64_t nt) {
  if (nt <= ctx->tri_cap && ctx->d_counts) return LFDPR_OK;
  if (sync_all(ctx) != hipSuccess) return fail(ctx, LFDPR_EDEVICE, "synchronising before reallocation");
  int64_t n = nt > 1024 ? nt : 1024;
  dfree(ctx->d_counts);
  dfree(ctx->d_offsets);
  dfree(ctx->d_rec);
  dfree(ctx->d_em);
  dfree(ctx->d_tiles);
  dfree(ctx->d_big);
  dfree(ctx->d_tris);
  if (dalloc(ctx->d_counts, n) != hipSuccess || dalloc(ctx->d_offsets, n) != hipSuccess ||
      dalloc(ctx->d_rec, n) != hipSuccess || dalloc(ctx->d_em, n) != hipSuccess ||
      dalloc(ctx->d_tiles, (n + 255) / 256 + 1) != hipSuccess || dalloc(ctx->d_big, n) != hipSuccess ||
      dalloc(ctx->d_tris, n) != hipSuccess) {
    ctx->tri_cap = 0;
    return fail(ctx, LFDPR_ENOMEM, "per-triangle buffers");
  }
  ctx->tri_cap = n;
  return LFDPR_OK;
}

// Event recorded on `st` when timing is on (nullptr otherwise).
hipEvent_t mark_on(lfdpr_ctx* ctx, hipStream_t st) {
  if (!ctx->timing) return nullptr;
  if (ctx->ev_used == ctx->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->ev_pool.push_back(e);
  }
  hipEvent_t e = ctx->ev_pool[ctx->ev_used++];
  (void)hipEventRecord(e, st);
  return e;
}

hipEvent_t mark(lfdpr_ctx* ctx) { return mark_on(ctx, ctx->stream); }

void stage(lfdpr_ctx* ctx, int id, hipEvent_t a, hipEvent_t b) {
  if (a && b) ctx->ev_marks.push_back({id, {a, b}});
}

}  // namespace

hipStream_t ctx_stream_of(lfdpr_ctx* c) { return c->stream; }

namespace {

// Rig in double, rounded once: eye offsets b_r = D tan(cone/2) (2 q_r / V - 1),
// kshift_r = b_r / D, and the shared projection constants.
void build_rig(const lfdpr_view_params& v, Rig& rg, std::vector<float>& eye, std::vector<float>& ks,
               std::vector<double>& q) {
  const int64_t nviews = (int64_t)v.V * v.S;
  const double D = v.D;
  // degrees to radians as deg * (pi / 180), then halved
  const double B = D * std::tan((double)v.cone_deg * (M_PI / 180.0) / 2.0);
  const double tf = std::tan((double)v.fovy_deg * (M_PI / 180.0) / 2.0);
  eye.assign(nviews, 0.0f);
  ks.assign(nviews, 0.0f);
  q.assign(nviews, 0.0);
  for (int vv = 0; vv < v.V; ++vv)
    for (int k = 0; k < v.S; ++k) {
      int r = vv * v.S + k;
      q[r] = v.S == 1 ? vv + 0.5 : vv + (k + 0.5 + (double)v.jitter[r]) / v.S;
      double b = B * (2.0 * q[r] / v.V - 1.0);
      eye[r] = (float)b;
      ks[r] = (float)(b / D);
    }
  rg = Rig{};
  rg.n_views = (int32_t)nviews;
  rg.W = v.W;
  rg.H = v.H;
  rg.mip = v.mip ? 1 : 0;
  rg.fx = (float)((v.W / 2.0) / ((double)v.aspect * tf));
  rg.fy = (float)((v.H / 2.0) / tf);
  rg.cx = (float)(v.W / 2.0);
  rg.cy = (float)(v.H / 2.0);
  rg.rD = (float)(1.0 / D);
  rg.znear = v.znear;
  rg.fxfy = rg.fx * rg.fy;
  rg.eye_lo = *std::min_element(eye.begin(), eye.end());
  rg.eye_hi = *std::max_element(eye.begin(), eye.end());
}

bool view_params_ok(const lfdpr_view_params* v) {
  const int64_t nviews = (int64_t)v->V * v->S;
  if (v->V < 1 || v->S < 1 || nviews > 1024 || v->W < 1 || v->H < 1 || v->W > 4096 || v->H > 4096 ||
      !(v->fovy_deg > 0.0f && v->fovy_deg < 180.0f) || !(v->aspect > 0.0f) || !(v->D > 0.0f) ||
      !(v->cone_deg >= 0.0f && v->cone_deg < 180.0f) || !(v->znear > 0.0f) || (v->S > 1 && !v->jitter) ||
      v->point_capacity < 0 || v->point_capacity > (1ll << 31))
    return false;
  if (v->S > 1)
    for (int64_t k = 0; k < nviews; ++k)
      if (!(v->jitter[k] >= -0.5f && v->jitter[k] < 0.5f)) return false;
  return true;
}

InterleaveArgs interleave_args(const lfdpr_lens_params& l, const uint32_t* views, int32_t n_views, int32_t W,
                               int32_t H, uint8_t* panel) {
  const double two32 = 4294967296.0;
  auto mod32 = [](long long v) { return (uint32_t)((unsigned long long)v & 0xFFFFFFFFull); };
  InterleaveArgs a{};
  a.views = views;
  a.V = n_views;
  a.Wv = W;
  a.Hv = H;
  a.Wp = l.Wp;
  a.Hp = l.Hp;
  a.mode = l.mode;
  a.K1 = mod32(std::llround(two32 / l.pitch_subpx));
  a.Ky = mod32(std::llround(-3.0 * l.slope * two32 / l.pitch_subpx));
  a.K0 = mod32(std::llround(l.offset * two32));
  for (int k = 0; k < 8; ++k) {
    a.du[k] = (l.mode & LFDPR_RECON_ANGULAR) ? l.taps[k][0] : 0;
    a.dx[k] = (l.mode & LFDPR_RECON_SPATIAL) ? (int32_t)l.taps[k][1] : 0;
    a.dy[k] = (l.mode & LFDPR_RECON_SPATIAL) ? (int32_t)l.taps[k][2] : 0;
  }
  a.panel = panel;
  return a;
}

}  // namespace
int ctx_device_of(lfdpr_ctx* c) { return c->device; }
void ctx_children_add(lfdpr_ctx* c, int delta) { c->live_children += delta; }

extern "C" {

int lfdpr_abi_version(void) { return LFDPR_ABI_VERSION; }

const char* lfdpr_strerror(int code) {
  switch (code) {
    case LFDPR_OK: return "ok";
    case LFDPR_EINVAL: return "invalid argument";
    case LFDPR_ENOMEM: return "out of device memory";
    case LFDPR_EOVERFLOW: return "point capacity exceeded";
    case LFDPR_EDEVICE: return "HIP runtime error";
    case LFDPR_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

int lfdpr_create(int device, void* stream, lfdpr_ctx** out) {
  lfdpr_ctx* ctx = nullptr;
  if (!out) return LFDPR_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LFDPR_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return LFDPR_EDEVICE;
  ctx = new lfdpr_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)stream;
  ctx->scratch = scratch_on(device);  // null: lfdpr_render_frame_noalloc reports LFDPR_EDEVICE
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    ctx->max_lds = lds;
  // the quilt's tile kernels may take that much LDS (set once, outside any
  // capture); if the device refuses, tiles stay within 64 KiB
  if (prepare_quilt_kernels((size_t)ctx->max_lds) != hipSuccess) {
    (void)hipGetLastError();
    ctx->max_lds = 65536;
    if (prepare_quilt_kernels((size_t)ctx->max_lds) != hipSuccess) {
      (void)hipGetLastError();
      ctx->max_lds = 0;  // no tile fits: the quilt order is refused
    }
  }
  if (dalloc(ctx->d_stats, STAT_SLOTS) != hipSuccess || dalloc(ctx->d_item1, 1) != hipSuccess) {
    dfree(ctx->d_stats);
    delete ctx;
    return LFDPR_ENOMEM;
  }
  // LOD thresholds: 2^((k - 127.5)/128) rounded up to the next float
  float thr[128];
  for (int k = 0; k < 128; ++k) {
    double t = std::exp2((k - 127.5) / 128.0);
    float f = (float)t;
    if ((double)f < t) f = std::nextafter(f, INFINITY);
    thr[k] = f;
  }
  if (dalloc(ctx->d_lod_thr, 128) != hipSuccess ||
      hipMemcpy(ctx->d_lod_thr, thr, sizeof thr, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(ctx->d_stats, 0, STAT_SLOTS * sizeof(uint64_t)) != hipSuccess) {
    lfdpr_destroy(ctx);
    return LFDPR_EDEVICE;
  }
  *out = ctx;
  return LFDPR_OK;
}

int lfdpr_destroy(lfdpr_ctx* ctx) {
  if (!ctx) return LFDPR_OK;
  if (ctx->live_children > 0) return fail(ctx, LFDPR_ESTATE, "destroy the context's batches and networks first");
  (void)hipSetDevice(ctx->device);
  (void)sync_all(ctx);
  for (auto& kv : ctx->scenes) free_scene(kv.second);
  {
    auto& o = ctx->other;
    dfree(o.d_points);
    dfree(o.d_rows);
    dfree(o.d_pbox);
    dfree(o.d_prows);
    dfree(o.d_tris);
    dfree(o.d_counts);
    dfree(o.d_offsets);
    dfree(o.d_rec);
    dfree(o.d_em);
    dfree(o.d_tiles);
    dfree(o.d_big);
    dfree(o.d_stats);
    dfree(o.d_tm);
    dfree(o.d_pmat);
    dfree(o.d_qentries);
    dfree(o.d_qband);
  }
  for (int k = 0; k < 2; ++k) {
    if (ctx->ev_emitted[k]) (void)hipEventDestroy(ctx->ev_emitted[k]);
    if (ctx->ev_splatted[k]) (void)hipEventDestroy(ctx->ev_splatted[k]);
  }
  if (ctx->ev_caller) (void)hipEventDestroy(ctx->ev_caller);
  if (ctx->ev_start) (void)hipEventDestroy(ctx->ev_start);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  dfree(ctx->d_eye);
  dfree(ctx->d_kshift);
  dfree(ctx->d_lod_thr);
  dfree(ctx->d_points);
  dfree(ctx->d_rows);
  dfree(ctx->d_pbox);
  dfree(ctx->d_prows);
  dfree(ctx->d_tris);
  dfree(ctx->d_keys);
  dfree(ctx->d_acnt);
  dfree(ctx->d_asrc);
  dfree(ctx->d_awt);
  dfree(ctx->d_counts);
  dfree(ctx->d_offsets);
  dfree(ctx->d_rec);
  dfree(ctx->d_em);
  dfree(ctx->d_tiles);
  dfree(ctx->d_big);
  dfree(ctx->d_stats);
  dfree(ctx->d_item1);
  dfree(ctx->d_tm);
  dfree(ctx->d_pmat);
  dfree(ctx->d_qentries);
  dfree(ctx->d_qband);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
  return LFDPR_OK;
}

const char* lfdpr_last_error(lfdpr_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int lfdpr_scene_upload(lfdpr_ctx* ctx, const lfdpr_scene_desc* d, int32_t* scene_id) {
  if (!ctx || !d || !scene_id) return fail(ctx, LFDPR_EINVAL, "null argument");
  if (d->n_verts < 3 || d->n_tris < 0 || d->n_tris > (1 << 28) - 1 || d->n_tex < 1 || d->n_tex > 65535 ||
      !d->pos || !d->uv || (d->n_tris > 0 && (!d->idx || !d->tex_id)) || !d->tex_size || !d->tex_rgba8)
    return fail(ctx, LFDPR_EINVAL, "scene descriptor out of range");
  for (int64_t k = 0; k < 3ll * d->n_tris; ++k)
    if (d->idx[k] >= (uint32_t)d->n_verts) return fail(ctx, LFDPR_EINVAL, "vertex index out of range");
  for (int64_t k = 0; k < d->n_tris; ++k)
    if (d->tex_id[k] >= d->n_tex) return fail(ctx, LFDPR_EINVAL, "texture id out of range");
  std::vector<TexInfo> ti(d->n_tex);
  int64_t pool = 0;
  for (int k = 0; k < d->n_tex; ++k) {
    int s = d->tex_size[k];
    if (s < 1 || s > 16384 || (s & (s - 1)) || !d->tex_rgba8[k]) return fail(ctx, LFDPR_EINVAL, "texture size");
    ti[k].size = s;
    ti[k].levels = 0;
    for (int q = s; q >= 1; q >>= 1) {
      ti[k].off[ti[k].levels++] = pool;
      pool += (int64_t)q * q * 4;
    }
    for (int l = ti[k].levels; l < 16; ++l) ti[k].off[l] = 0;
  }
  HIPOK(hipSetDevice(ctx->device));
  SceneDev s;
  s.nv = d->n_verts;
  s.nt = d->n_tris;
  s.ntex = d->n_tex;
  if (dalloc(s.pos, 3ll * s.nv) != hipSuccess || dalloc(s.uv, 2ll * s.nv) != hipSuccess ||
      dalloc(s.idx, 3ll * s.nt) != hipSuccess || dalloc(s.tex, (size_t)s.nt) != hipSuccess ||
      dalloc(s.texinfo, (size_t)s.ntex) != hipSuccess || dalloc(s.texels, (size_t)pool) != hipSuccess) {
    free_scene(s);
    return fail(ctx, LFDPR_ENOMEM, "scene buffers");
  }
  hipError_t e = hipMemcpyAsync(s.pos, d->pos, 12ll * s.nv, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s.uv, d->uv, 8ll * s.nv, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && s.nt) e = hipMemcpyAsync(s.idx, d->idx, 12ll * s.nt, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && s.nt) e = hipMemcpyAsync(s.tex, d->tex_id, 2ll * s.nt, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s.texinfo, ti.data(), sizeof(TexInfo) * s.ntex, hipMemcpyHostToDevice, ctx->stream);
  for (int k = 0; k < s.ntex && e == hipSuccess; ++k) {
    int sz = ti[k].size;
    e = hipMemcpyAsync(s.texels + ti[k].off[0], d->tex_rgba8[k], (size_t)sz * sz * 4, hipMemcpyHostToDevice, ctx->stream);
    for (int l = 1; l < ti[k].levels && e == hipSuccess; ++l) {
      launch_build_mip((const uint32_t*)(s.texels + ti[k].off[l - 1]), (uint32_t*)(s.texels + ti[k].off[l]),
                       sz >> (l - 1), ctx->stream);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    free_scene(s);
    return fail(ctx, LFDPR_EDEVICE, std::string("scene upload: ") + hipGetErrorString(e));
  }
  int32_t id = ctx->next_scene++;
  ctx->scenes[id] = s;
  *scene_id = id;
  return LFDPR_OK;
}

int lfdpr_scene_free(lfdpr_ctx* ctx, int32_t scene_id) {
  if (!ctx) return LFDPR_EINVAL;
  auto it = ctx->scenes.find(scene_id);
  if (it == ctx->scenes.end()) return fail(ctx, LFDPR_EINVAL, "unknown scene id");
  if (it->second.batch_refs > 0) return fail(ctx, LFDPR_ESTATE, "the scene is rendered by a live batch");
  HIPOK(sync_all(ctx));
  free_scene(it->second);
  ctx->scenes.erase(it);
  return LFDPR_OK;
}

int lfdpr_scene_set_materials(lfdpr_ctx* ctx, int32_t scene_id, const uint16_t* normal_id,
                              const uint16_t* roughness_id, const uint16_t* metallic_id) {
  if (!ctx) return LFDPR_EINVAL;
  auto it = ctx->scenes.find(scene_id);
  if (it == ctx->scenes.end()) return fail(ctx, LFDPR_EINVAL, "unknown scene id");
  SceneDev& s = it->second;
  if (s.batch_refs > 0) return fail(ctx, LFDPR_ESTATE, "the scene is rendered by a live batch");
  const int given = (normal_id != nullptr) + (roughness_id != nullptr) + (metallic_id != nullptr);
  if (given != 0 && given != 3) return fail(ctx, LFDPR_EINVAL, "all three material arrays or none");
  std::vector<uint16_t> m;
  if (given == 3) {
    m.resize((size_t)s.nt * 3);
    for (int64_t t = 0; t < s.nt; ++t) {
      const uint16_t ids[3] = {normal_id[t], roughness_id[t], metallic_id[t]};
      for (int k = 0; k < 3; ++k) {
        if (ids[k] >= s.ntex) return fail(ctx, LFDPR_EINVAL, "material texture id out of range");
        m[(size_t)t * 3 + k] = ids[k];
      }
    }
  }
  HIPOK(hipSetDevice(ctx->device));
  HIPOK(sync_all(ctx));  // earlier frames may still read the old table
  dfree(s.mat);
  if (given == 3) {
    if (dalloc(s.mat, m.size()) != hipSuccess) return fail(ctx, LFDPR_ENOMEM, "material table");
    HIPOK(hipMemcpy(s.mat, m.data(), m.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  }
  return LFDPR_OK;
}

int lfdpr_set_shading(lfdpr_ctx* ctx, const lfdpr_shading* sh) {
  if (!ctx || !sh) return fail(ctx, LFDPR_EINVAL, "null argument");
  if (sh->mode != LFDPR_SHADE_UNLIT && sh->mode != LFDPR_SHADE_PBR) return fail(ctx, LFDPR_EINVAL, "shading mode");
  if (sh->mode == LFDPR_SHADE_PBR) {
    double len2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const float c[3] = {sh->light_dir[k], sh->light_rgb[k], sh->ambient_rgb[k]};
      for (float x : c)
        if (!std::isfinite(x)) return fail(ctx, LFDPR_EINVAL, "non-finite light");
      if (!(sh->light_rgb[k] >= 0.0f && sh->light_rgb[k] <= 1e4f && sh->ambient_rgb[k] >= 0.0f &&
            sh->ambient_rgb[k] <= 1e4f))
        return fail(ctx, LFDPR_EINVAL, "light and ambient RGB must lie in [0, 1e4]");
      len2 += (double)sh->light_dir[k] * sh->light_dir[k];
    }
    if (std::fabs(std::sqrt(len2) - 1.0) > 1e-3) return fail(ctx, LFDPR_EINVAL, "light direction is not a unit vector");
  }
  ctx->shading = *sh;
  return LFDPR_OK;
}

int lfdpr_set_views(lfdpr_ctx* ctx, const lfdpr_view_params* v) {
  if (!ctx || !v) return fail(ctx, LFDPR_EINVAL, "null argument");
  if (!view_params_ok(v)) return fail(ctx, LFDPR_EINVAL, "view parameters out of range");
  const int64_t nviews = (int64_t)v->V * v->S;
  HIPOK(hipSetDevice(ctx->device));
  HIPOK(sync_all(ctx));
  Rig rg{};
  std::vector<float> eye, ks;
  std::vector<double> q;
  build_rig(*v, rg, eye, ks, q);
  // angular filter table: sub-views within one interval of each view centre
  int32_t maxe = 3 * v->S;
  std::vector<int32_t> acnt(v->V, 0), asrc((size_t)v->V * maxe, 0);
  std::vector<uint32_t> awt((size_t)v->V * maxe, 0);
  for (int vv = 0; vv < v->V; ++vv)
    for (int r = 0; r < nviews; ++r) {
      double dlt = q[r] - (vv + 0.5);
      if (std::fabs(dlt) < 1.0 && acnt[vv] < maxe) {
        asrc[(size_t)vv * maxe + acnt[vv]] = r;
        awt[(size_t)vv * maxe + acnt[vv]] = (uint32_t)std::llround(65535.0 * std::exp(-dlt * dlt / (2.0 * 0.25)));
        ++acnt[vv];
      }
    }
  int64_t cap = v->point_capacity ? v->point_capacity : (8ll << 20);
  int64_t nkeys = nviews * (int64_t)v->W * v->H;
  dfree(ctx->d_eye);
  dfree(ctx->d_kshift);
  dfree(ctx->d_acnt);
  dfree(ctx->d_asrc);
  dfree(ctx->d_awt);
  if (dalloc(ctx->d_eye, nviews) != hipSuccess || dalloc(ctx->d_kshift, nviews) != hipSuccess ||
      dalloc(ctx->d_acnt, v->V) != hipSuccess || dalloc(ctx->d_asrc, (size_t)v->V * maxe) != hipSuccess ||
      dalloc(ctx->d_awt, (size_t)v->V * maxe) != hipSuccess)
    return fail(ctx, LFDPR_ENOMEM, "rig tables");
  if (cap != ctx->cap || !ctx->d_points) {
    // the point buffer with the splat data sized like it (row table, point rectangles)
    dfree(ctx->d_points);
    dfree(ctx->d_rows);
    dfree(ctx->d_pbox);
    dfree(ctx->d_prows);
    ctx->cap = ctx->points_alloc = 0;
    if (dalloc(ctx->d_points, (size_t)cap) != hipSuccess || dalloc(ctx->d_rows, (size_t)cap) != hipSuccess ||
        dalloc(ctx->d_pbox, (size_t)cap) != hipSuccess || dalloc(ctx->d_prows, (size_t)cap) != hipSuccess)
      return fail(ctx, LFDPR_ENOMEM, "point buffers");
    ctx->cap = ctx->points_alloc = cap;
  }
  if (ctx->other.points_alloc != cap) {  // the second set (two frames in flight) follows on first use
    dfree(ctx->other.d_points);
    dfree(ctx->other.d_rows);
    dfree(ctx->other.d_pbox);
    dfree(ctx->other.d_prows);
    ctx->other.points_alloc = 0;
  }
  if (nkeys != ctx->n_keys || !ctx->d_keys) {
    dfree(ctx->d_keys);
    ctx->n_keys = 0;
    if (dalloc(ctx->d_keys, (size_t)nkeys) != hipSuccess) return fail(ctx, LFDPR_ENOMEM, "key buffer");
    ctx->n_keys = nkeys;
  }
  HIPOK(hipMemcpy(ctx->d_eye, eye.data(), 4 * nviews, hipMemcpyHostToDevice));
  HIPOK(hipMemcpy(ctx->d_kshift, ks.data(), 4 * nviews, hipMemcpyHostToDevice));
  HIPOK(hipMemcpy(ctx->d_acnt, acnt.data(), 4 * acnt.size(), hipMemcpyHostToDevice));
  HIPOK(hipMemcpy(ctx->d_asrc, asrc.data(), 4 * asrc.size(), hipMemcpyHostToDevice));
  HIPOK(hipMemcpy(ctx->d_awt, awt.data(), 4 * awt.size(), hipMemcpyHostToDevice));
  launch_fill_u64(ctx->d_keys, nkeys, ~0ull, ctx->stream);
  HIPOK(hipGetLastError());
  HIPOK(sync_all(ctx));
  rg.eye = ctx->d_eye;
  rg.kshift = ctx->d_kshift;
  ctx->rig = rg;
  ctx->vp = *v;
  ctx->amaxe = maxe;
  ctx->views_set = true;
  return LFDPR_OK;
}

int lfdpr_set_splat_order(lfdpr_ctx* ctx, int32_t order) {
  if (!ctx) return LFDPR_EINVAL;
  if (order != LFDPR_SPLAT_TRIANGLE_VIEW && order != LFDPR_SPLAT_POINT && order != LFDPR_SPLAT_QUILT)
    return fail(ctx, LFDPR_EINVAL, "unknown splat order");
  ctx->splat_order = order;
  return LFDPR_OK;
}

int lfdpr_set_quilt_tile(lfdpr_ctx* ctx, int32_t rows, int32_t views) {
  if (!ctx) return LFDPR_EINVAL;
  if (!((rows == 0 && views == 0) || (rows >= 1 && rows <= 4096 && views >= 1 && views <= 1024)))
    return fail(ctx, LFDPR_EINVAL, "quilt tile: rows in [1, 4096] and views in [1, 1024], or both 0");
  ctx->quilt_rows = rows;
  ctx->quilt_views = views;
  return LFDPR_OK;
}

int lfdpr_quilt_tile(int32_t W, int32_t H, int32_t n_views, int32_t n_items, int32_t max_lds, int32_t rows,
                     int32_t views, int32_t* out_rows, int32_t* out_views) {
  if (!out_rows || !out_views || W < 1 || H < 1 || W > 4096 || H > 4096 || n_views < 1 || n_views > 1024 ||
      n_items < 1 || n_items > 256 || max_lds < 0 || !((rows == 0 && views == 0) || (rows >= 1 && views >= 1)))
    return LFDPR_EINVAL;
  Rig rg{};
  rg.W = W;
  rg.H = H;
  rg.n_views = n_views;
  int r = 0, v = 0;
  if (!quilt_shape_for(rg, max_lds, rows, views, n_items, r, v)) return LFDPR_EINVAL;
  *out_rows = r;
  *out_views = v;
  return LFDPR_OK;
}

int lfdpr_set_quilt_capacity(lfdpr_ctx* ctx, int64_t entries) {
  if (!ctx) return LFDPR_EINVAL;
  if (entries < 0 || entries > 0xFFFFFFFFll) return fail(ctx, LFDPR_EINVAL, "quilt capacity in [0, 2^32 - 1]");
  ctx->quilt_cap_req = entries;
  return LFDPR_OK;
}

int lfdpr_set_lens(lfdpr_ctx* ctx, const lfdpr_lens_params* l) {
  if (!ctx || !l) return fail(ctx, LFDPR_EINVAL, "null argument");
  if (l->Wp < 1 || l->Hp < 1 || l->Wp > 16384 || l->Hp > 16384 || !(l->pitch_subpx > 0.0) || l->mode < 0 ||
      l->mode > 3 || !std::isfinite(l->slope) || !std::isfinite(l->offset))
    return fail(ctx, LFDPR_EINVAL, "lens parameters out of range");
  for (int k = 0; k < 8; ++k)
    if (l->taps[k][0] <= -(1ll << 34) || l->taps[k][0] >= (1ll << 34) || l->taps[k][1] < -65536 ||
        l->taps[k][1] > 65536 || l->taps[k][2] < -65536 || l->taps[k][2] > 65536)
      return fail(ctx, LFDPR_EINVAL, "reconstruction tap out of range");
  ctx->lens = *l;
  ctx->lens_set = true;
  return LFDPR_OK;
}

int lfdpr_set_debug_records(lfdpr_ctx* ctx, float* f, int32_t* i, int64_t n_tris) {
  if (!ctx) return LFDPR_EINVAL;
  if ((f == nullptr) != (i == nullptr)) return fail(ctx, LFDPR_EINVAL, "both or neither debug buffers");
  if (f && n_tris < 0) return fail(ctx, LFDPR_EINVAL, "negative debug record capacity");
  ctx->dbgf = f;
  ctx->dbgi = i;
  ctx->dbg_cap = f ? n_tris : 0;
  return LFDPR_OK;
}

int lfdpr_render_frame(lfdpr_ctx* ctx, int32_t scene_id, const float* model, uint32_t* views, float* depth) {
  if (!ctx || !model || !views) return fail(ctx, LFDPR_EINVAL, "null argument");
  if (!ctx->views_set) return fail(ctx, LFDPR_ESTATE, "lfdpr_set_views first");
  auto it = ctx->scenes.find(scene_id);
  if (it == ctx->scenes.end()) return fail(ctx, LFDPR_EINVAL, "unknown scene id");
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(model[k])) return fail(ctx, LFDPR_EINVAL, "non-finite model matrix");
  const SceneDev& s = it->second;
  if (ctx->dbgf && s.nt > ctx->dbg_cap) return fail(ctx, LFDPR_EINVAL, "debug record buffers smaller than the scene");
  const bool pbr = ctx->shading.mode == LFDPR_SHADE_PBR;
  if (pbr && s.nt > 0 && !s.mat) return fail(ctx, LFDPR_ESTATE, "physically based shading needs lfdpr_scene_set_materials");
  HIPOK(hipSetDevice(ctx->device));
  const bool quilt = ctx->splat_order == LFDPR_SPLAT_QUILT;
  int qrows = 0, qviews = 0;
  if (quilt && !quilt_shape(ctx, qrows, qviews)) return fail(ctx, LFDPR_EINVAL, "quilt tile does not fit the device's LDS");
  // two frames in flight: this frame takes the other set of per-frame buffers
  const bool piped = ctx->frames_in_flight == 2;
  if (piped) swap_frame_buffers(ctx);
  int rc = prepare_frame_buffers(ctx, s.nt, pbr);
  if (!rc && quilt) rc = ensure_quilt_buffers(ctx);
  if (rc) {
    if (piped) swap_frame_buffers(ctx);
    return rc;
  }
  hipStream_t st = ctx->stream;
  // point generation runs on the side stream when two frames are in flight;
  // it first waits for the splat that last read this set of buffers
  hipStream_t gen = piped ? ctx->side : st;
  const int sl = ctx->slot;
  if (piped && ctx->splatted_pending[sl]) HIPOK(hipStreamWaitEvent(gen, ctx->ev_splatted[sl], 0));
  if (piped) {
    // and for the caller's work queued before the previous frame began (the
    // frame before it presented: filter, panel), so that this generation does
    // not take the CUs that work needs while the previous frame waits on it.
    // With the wait, the generation's first launch also reaches the GPU after
    // the previous frame's splat has taken the CUs, and the set-up then takes
    // only slots that splat workgroups free (measured faster than starting
    // beside the splat's first workgroups)
    if (ctx->start_pending) HIPOK(hipStreamWaitEvent(gen, ctx->ev_start, 0));
    HIPOK(hipEventRecord(ctx->ev_start, st));
    ctx->start_pending = true;
  }
  if (piped && ctx->dbgf) {
    // the set-up writes the caller's debug record buffers: after the caller's earlier work
    HIPOK(hipEventRecord(ctx->ev_caller, st));
    HIPOK(hipStreamWaitEvent(gen, ctx->ev_caller, 0));
  }
  Item one;
  std::memset(&one, 0, sizeof one);  // padding too: the table is compared bytewise
  one.pos = s.pos;
  one.uv = s.uv;
  one.idx = s.idx;
  one.tex = s.tex;
  one.texinfo = s.texinfo;
  one.texels = s.texels;
  one.tri_base = 0;
  one.nt = s.nt;
  one.rig = ctx->rig;
  one.keys = ctx->d_keys;
  one.key_layout = ctx->key_layout;
  one.mat = pbr ? s.mat : nullptr;
  if (std::memcmp(&one, &ctx->h_item1, sizeof one) != 0) {
    HIPOK(sync_all(ctx));  // earlier frames may still read the table
    HIPOK(hipMemcpy(ctx->d_item1, &one, sizeof one, hipMemcpyHostToDevice));
    std::memcpy(&ctx->h_item1, &one, sizeof one);
  }
  launch_fill_u64(ctx->d_stats, STAT_SLOTS, 0ull, gen);
  SetupArgs sa{};
  sa.items = ctx->d_item1;
  sa.n_items = 1;
  sa.nt = s.nt;
  std::memcpy(sa.model.m, model, sizeof sa.model.m);
  sa.models = nullptr;
  sa.lod_thr = ctx->d_lod_thr;
  sa.counts = ctx->d_counts;
  sa.rec = ctx->d_rec;
  sa.em = ctx->d_em;
  sa.dbgf = ctx->dbgf;
  sa.dbgi = ctx->dbgi;
  sa.stats = ctx->d_stats;
  sa.tm = pbr ? ctx->d_tm : nullptr;
  sa.tile_sum = ctx->d_tiles;
  sa.big = ctx->d_big;
  sa.n_big = ctx->d_stats + STAT_BIG;
  hipEvent_t e0 = mark_on(ctx, gen);
  launch_tri_setup(sa, quilt, gen);
  hipEvent_t e1 = mark_on(ctx, gen);
  launch_scan(ctx->d_tiles, s.nt, ctx->d_stats + STAT_TOTAL, gen);
  hipEvent_t e2 = mark_on(ctx, gen);
  EmitArgs ea{};
  ea.items = ctx->d_item1;
  ea.nt = s.nt;
  ea.counts = ctx->d_counts;
  ea.tile_base = ctx->d_tiles;
  ea.offsets = ctx->d_offsets;
  ea.em = ctx->d_em;
  ea.points = ctx->d_points;
  ea.n_points = ctx->d_stats + STAT_TOTAL;
  ea.big = ctx->d_big;
  ea.n_big = ctx->d_stats + STAT_BIG;
  ea.cap = ctx->cap;
  ea.tm = pbr ? ctx->d_tm : nullptr;
  ea.pmat = pbr ? ctx->d_pmat : nullptr;
  const bool tv = !pbr && ctx->splat_order == LFDPR_SPLAT_TRIANGLE_VIEW;
  ea.rec = ctx->d_rec;
  ea.rows = tv ? ctx->d_rows : nullptr;
  ea.pbox = tv || quilt ? ctx->d_pbox : nullptr;
  ea.prows = quilt ? ctx->d_prows : nullptr;
  ea.tris = tv ? ctx->d_tris : nullptr;
  ea.n_tris = ctx->d_stats + STAT_EMITTING;
  launch_emit(ea, ctx->splat_blocks, gen);
  hipEvent_t e3 = mark_on(ctx, gen);
  QuiltBinArgs qa{};
  if (quilt) {
    // the quilt's band lists, built with the point generation
    qa = quilt_bin_args(ctx->d_qband, ctx->d_qentries, ctx->q_entry_cap, ctx->d_prows, ctx->d_stats + STAT_TOTAL,
                        ctx->cap, ctx->rig.H, qrows, 1);
    launch_quilt_bin(qa, gen);
  }
  hipEvent_t ebin = quilt ? mark_on(ctx, gen) : e3;
  if (piped) {
    HIPOK(hipEventRecord(ctx->ev_emitted[sl], gen));
    HIPOK(hipStreamWaitEvent(st, ctx->ev_emitted[sl], 0));
  }
  hipEvent_t e3s = piped ? mark(ctx) : ebin;
  SplatArgs pa{};
  pa.items = ctx->d_item1;
  pa.n_items = 1;
  pa.table_rig = ctx->rig;
  pa.points = ctx->d_points;
  pa.n_points = ctx->d_stats + STAT_TOTAL;
  pa.stats = ctx->d_stats;
  pa.em = ctx->d_em;
  pa.offsets = ctx->d_offsets;
  pa.counts = ctx->d_counts;
  pa.rows = ctx->d_rows;
  pa.pbox = tv ? ctx->d_pbox : nullptr;
  pa.tris = ctx->d_tris;
  pa.n_tris = ctx->d_stats + STAT_EMITTING;
  pa.nt = s.nt;
  pa.cap = ctx->cap;
  pa.rec = ctx->d_rec;
  pa.tm = pbr ? ctx->d_tm : nullptr;
  pa.pmat = pbr ? ctx->d_pmat : nullptr;
  const lfdpr_shading& sh = ctx->shading;
  pa.sh = Shading{sh.light_dir[0], sh.light_dir[1], sh.light_dir[2], sh.light_rgb[0], sh.light_rgb[1],
                  sh.light_rgb[2], sh.ambient_rgb[0], sh.ambient_rgb[1], sh.ambient_rgb[2]};
  const uint32_t* qstate = nullptr;
  if (quilt) {
    // the tiles, which write the views; the point splat and the resolve
    // below run only if the band lists overflowed
    const SplatArgs qp = quilt_tile_args(pa, qa, ctx->d_pbox, qviews, ctx->max_lds, views, depth);
    HIPOK(launch_splat_quilt(qp, st));
    qstate = qa.state;
    pa.gate = qstate;
  }
  // under the quilt this is the overflow fallback, which nearly always exits at once: a small grid
  launch_splat(pa, quilt ? 256 : ctx->splat_blocks, st);
  ctx->last_order = quilt ? LFDPR_SPLAT_QUILT : (pa.pbox && !pa.tm ? LFDPR_SPLAT_TRIANGLE_VIEW : LFDPR_SPLAT_POINT);
  ctx->last_qrows = qrows;
  ctx->last_qviews = qviews;
  hipEvent_t e4 = mark(ctx);
  launch_resolve(ctx->d_keys, 1, ctx->rig.n_views, ctx->rig.H, ctx->rig.W, ctx->key_layout, views, depth, st, qstate);
  hipEvent_t e5 = mark(ctx);
  if (piped) {
    // after the resolve, which reads this set's overflow flag under the quilt
    HIPOK(hipEventRecord(ctx->ev_splatted[sl], st));
    ctx->splatted_pending[sl] = true;
  }
  HIPOK(hipGetLastError());
  stage(ctx, 0, e0, e1);
  stage(ctx, 1, e1, e2);
  stage(ctx, 2, e2, e3);
  if (quilt) stage(ctx, 7, e3, ebin);
  stage(ctx, 3, e3s, e4);
  stage(ctx, 4, e4, e5);
  ctx->last_nt = s.nt;
  ctx->last_pbr = pbr;
  return LFDPR_OK;
}

int lfdpr_render_frame_noalloc(lfdpr_ctx* ctx, int32_t scene_id, const float* model, uint32_t* views, float* depth,
                               int64_t* stats) {
  if (!ctx || !model || !views) return fail(ctx, LFDPR_EINVAL, "null argument");
  if (!ctx->views_set) return fail(ctx, LFDPR_ESTATE, "lfdpr_set_views first");
  if (ctx->frames_in_flight != 1) return fail(ctx, LFDPR_ESTATE, "one frame in flight only");
  if (ctx->shading.mode == LFDPR_SHADE_PBR)
    return fail(ctx, LFDPR_ESTATE, "physically based shading needs lfdpr_render_frame");
  auto it = ctx->scenes.find(scene_id);
  if (it == ctx->scenes.end()) return fail(ctx, LFDPR_EINVAL, "unknown scene id");
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(model[k])) return fail(ctx, LFDPR_EINVAL, "non-finite model matrix");
  const SceneDev& s = it->second;
  if (s.nt > kNoAllocTris) return fail(ctx, LFDPR_EINVAL, "scene above the no-allocation limit of 65,536 triangles");
  const int64_t nkeys = (int64_t)ctx->rig.n_views * ctx->rig.W * ctx->rig.H;
  if (nkeys > kNoAllocKeys)
    return fail(ctx, LFDPR_EINVAL, "views x H x W above the no-allocation limit of 2,097,152 keys");
  if (!ctx->scratch) return fail(ctx, LFDPR_EDEVICE, "no-allocation scratch unavailable on this device");
  HIPOK(hipSetDevice(ctx->device));
  unsigned char* base = (unsigned char*)ctx->scratch;
  Item* d_item = (Item*)(base + kOffItem);
  uint64_t* d_st = (uint64_t*)(base + kOffStats);
  uint32_t* d_counts = (uint32_t*)(base + kOffCounts);
  uint64_t* d_offsets = (uint64_t*)(base + kOffOffsets);
  uint64_t* d_tiles = (uint64_t*)(base + kOffTiles);
  TriRec* d_rec = (TriRec*)(base + kOffRec);
  TriEmit* d_em = (TriEmit*)(base + kOffEm);
  uint32_t* d_big = (uint32_t*)(base + kOffBig);
  uint32_t* d_tris = (uint32_t*)(base + kOffTris);
  Point* d_points = (Point*)(base + kOffPoints);
  RowEntry* d_rows = (RowEntry*)(base + kOffRows);
  PointBox* d_pbox = (PointBox*)(base + kOffPbox);
  uint64_t* d_keys = (uint64_t*)(base + kOffKeys);
  hipStream_t st = ctx->stream;
  Item one;
  std::memset(&one, 0, sizeof one);
  one.pos = s.pos;
  one.uv = s.uv;
  one.idx = s.idx;
  one.tex = s.tex;
  one.texinfo = s.texinfo;
  one.texels = s.texels;
  one.tri_base = 0;
  one.nt = s.nt;
  one.rig = ctx->rig;
  one.keys = d_keys;
  one.key_layout = ctx->key_layout;
  one.mat = nullptr;
  // the scratch keeps the last call's contents: statistics start at 0, keys at ~0
  launch_store_item(one, d_item, st);
  launch_fill_u64(d_st, STAT_SLOTS, 0ull, st);
  launch_fill_u64(d_keys, nkeys, ~0ull, st);
  SetupArgs sa{};
  sa.items = d_item;
  sa.n_items = 1;
  sa.nt = s.nt;
  std::memcpy(sa.model.m, model, sizeof sa.model.m);
  sa.models = nullptr;
  sa.lod_thr = ctx->d_lod_thr;
  sa.counts = d_counts;
  sa.rec = d_rec;
  sa.em = d_em;
  sa.dbgf = nullptr;
  sa.dbgi = nullptr;
  sa.stats = d_st;
  sa.tm = nullptr;
  sa.tile_sum = d_tiles;
  sa.big = d_big;
  sa.n_big = d_st + STAT_BIG;
  launch_tri_setup(sa, false, st);
  launch_scan(d_tiles, s.nt, d_st + STAT_TOTAL, st);
  EmitArgs ea{};
  ea.items = d_item;
  ea.nt = s.nt;
  ea.counts = d_counts;
  ea.tile_base = d_tiles;
  ea.offsets = d_offsets;
  ea.em = d_em;
  ea.points = d_points;
  ea.n_points = d_st + STAT_TOTAL;
  ea.big = d_big;
  ea.n_big = d_st + STAT_BIG;
  ea.cap = kNoAllocPoints;
  ea.tm = nullptr;
  ea.pmat = nullptr;
  const bool tv = ctx->splat_order == LFDPR_SPLAT_TRIANGLE_VIEW;
  ea.rec = d_rec;
  ea.rows = tv ? d_rows : nullptr;
  ea.pbox = tv ? d_pbox : nullptr;
  ea.tris = tv ? d_tris : nullptr;
  ea.n_tris = d_st + STAT_EMITTING;
  launch_emit(ea, ctx->splat_blocks, st);
  SplatArgs pa{};
  pa.items = d_item;
  pa.n_items = 1;
  pa.table_rig = ctx->rig;
  pa.points = d_points;
  pa.n_points = d_st + STAT_TOTAL;
  pa.cap = kNoAllocPoints;
  pa.rec = d_rec;
  pa.tm = nullptr;
  pa.pmat = nullptr;
  pa.sh = Shading{};
  pa.stats = d_st;
  pa.em = d_em;
  pa.offsets = d_offsets;
  pa.counts = d_counts;
  pa.rows = d_rows;
  pa.pbox = tv ? d_pbox : nullptr;
  pa.tris = d_tris;
  pa.n_tris = d_st + STAT_EMITTING;
  pa.nt = s.nt;
  launch_splat(pa, ctx->splat_blocks, st);
  launch_resolve(d_keys, 1, ctx->rig.n_views, ctx->rig.H, ctx->rig.W, ctx->key_layout, views, depth, st);
  if (stats) launch_export_stats(d_st, kNoAllocPoints, stats, st);
  HIPOK(hipGetLastError());
  return LFDPR_OK;
}

int lfdpr_reconstruct(lfdpr_ctx* ctx, const uint32_t* views, int32_t n_views, int32_t W, int32_t H, uint8_t* panel) {
  if (!ctx || !views || !panel) return fail(ctx, LFDPR_EINVAL, "null argument");
  if (!ctx->lens_set) return fail(ctx, LFDPR_ESTATE, "lfdpr_set_lens first");
  if (n_views < 1 || n_views > 4096 || W < 1 || H < 1 || W > 16384 || H > 16384)
    return fail(ctx, LFDPR_EINVAL, "view stack size out of range");
  InterleaveArgs a = interleave_args(ctx->lens, views, n_views, W, H, panel);
  HIPOK(hipSetDevice(ctx->device));
  hipEvent_t e0 = mark(ctx);
  launch_interleave(a, ctx->stream);
  hipEvent_t e1 = mark(ctx);
  HIPOK(hipGetLastError());
  stage(ctx, 5, e0, e1);
  return LFDPR_OK;
}

int lfdpr_angular_filter(lfdpr_ctx* ctx, const uint32_t* sub, uint32_t* out) {
  if (!ctx || !sub || !out) return fail(ctx, LFDPR_EINVAL, "null argument");
  if (!ctx->views_set) return fail(ctx, LFDPR_ESTATE, "lfdpr_set_views first");
  AngularArgs a{};
  a.sub = sub;
  a.out = out;
  a.V = ctx->vp.V;
  a.W = ctx->vp.W;
  a.H = ctx->vp.H;
  a.maxe = ctx->amaxe;
  a.cnt = ctx->d_acnt;
  a.src = ctx->d_asrc;
  a.wt = ctx->d_awt;
  HIPOK(hipSetDevice(ctx->device));
  hipEvent_t e0 = mark(ctx);
  launch_angular_filter(a, ctx->stream);
  hipEvent_t e1 = mark(ctx);
  HIPOK(hipGetLastError());
  stage(ctx, 6, e0, e1);
  return LFDPR_OK;
}

int lfdpr_get_stats(lfdpr_ctx* ctx, lfdpr_stats* out) {
  if (!ctx || !out) return fail(ctx, LFDPR_EINVAL, "null argument");
  uint64_t st[STAT_SLOTS];
  HIPOK(hipSetDevice(ctx->device));
  HIPOK(sync_all(ctx));
  HIPOK(hipMemcpy(st, ctx->d_stats, sizeof st, hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof *out);
  out->points = (int64_t)st[STAT_TOTAL];
  out->active_tris = (int64_t)st[STAT_ACTIVE];
  out->point_views = (int64_t)st[STAT_POINT_VIEWS];
  out->overflow_tris = (int64_t)st[STAT_OVERFLOW];
  out->written_px = (int64_t)st[STAT_WRITTEN];
  out->splat_order = ctx->last_order;
  out->covered_px = ctx->last_order == LFDPR_SPLAT_TRIANGLE_VIEW ? (int64_t)st[STAT_COVERED] : -1;
  out->missed_px = out->covered_px >= 0 ? out->covered_px - out->written_px : -1;
  out->quilt_entries = -1;
  if (ctx->last_order == LFDPR_SPLAT_QUILT) {
    uint32_t qs[2];
    HIPOK(hipMemcpy(qs, ctx->d_qband + 4 * kQuiltBandCap + 1, sizeof qs, hipMemcpyDeviceToHost));
    out->quilt_rows = ctx->last_qrows;
    out->quilt_views = ctx->last_qviews;
    out->quilt_entries = (int64_t)qs[1];
    if (qs[0]) out->splat_order = LFDPR_SPLAT_POINT;  // the lists overflowed: splatted per point
  }
  out->capacity = ctx->cap;
  out->point_overflow = out->points > ctx->cap ? 1 : 0;
  out->n_views = ctx->rig.n_views;
  return out->point_overflow ? LFDPR_EOVERFLOW : LFDPR_OK;
}

int lfdpr_copy_points(lfdpr_ctx* ctx, void* dst, int64_t cap, int64_t* n_points) {
  if (!ctx || !dst || !n_points || cap < 0) return fail(ctx, LFDPR_EINVAL, "null argument");
  uint64_t total = 0;
  HIPOK(hipSetDevice(ctx->device));
  HIPOK(sync_all(ctx));
  HIPOK(hipMemcpy(&total, ctx->d_stats + STAT_TOTAL, 8, hipMemcpyDeviceToHost));
  int64_t n = (int64_t)total < ctx->cap ? (int64_t)total : ctx->cap;
  *n_points = (int64_t)total;
  if (n > cap) n = cap;
  if (n > 0) HIPOK(hipMemcpy(dst, ctx->d_points, (size_t)n * sizeof(Point), hipMemcpyDeviceToDevice));
  return LFDPR_OK;
}

int lfdpr_copy_point_materials(lfdpr_ctx* ctx, void* dst, int64_t cap, int64_t* n_points) {
  if (!ctx || !dst || !n_points || cap < 0) return fail(ctx, LFDPR_EINVAL, "null argument");
  if (!ctx->last_pbr) return fail(ctx, LFDPR_ESTATE, "the last frame was not rendered with physically based shading");
  uint64_t total = 0;
  HIPOK(hipSetDevice(ctx->device));
  HIPOK(sync_all(ctx));
  HIPOK(hipMemcpy(&total, ctx->d_stats + STAT_TOTAL, 8, hipMemcpyDeviceToHost));
  int64_t n = (int64_t)total < ctx->cap ? (int64_t)total : ctx->cap;
  *n_points = (int64_t)total;
  if (n > cap) n = cap;
  if (n > 0) HIPOK(hipMemcpy(dst, ctx->d_pmat, (size_t)n * sizeof(uint4), hipMemcpyDeviceToDevice));
  return LFDPR_OK;
}

int lfdpr_copy_counts(lfdpr_ctx* ctx, uint32_t* dst, int64_t n) {
  if (!ctx || !dst || n < 0) return fail(ctx, LFDPR_EINVAL, "null argument");
  if (n > ctx->last_nt) return fail(ctx, LFDPR_EINVAL, "more counts than triangles");
  HIPOK(hipSetDevice(ctx->device));
  HIPOK(sync_all(ctx));
  if (n > 0) HIPOK(hipMemcpy(dst, ctx->d_counts, (size_t)n * 4, hipMemcpyDeviceToDevice));
  return LFDPR_OK;
}

int lfdpr_timing(lfdpr_ctx* ctx, int enable) {
  if (!ctx) return LFDPR_EINVAL;
  HIPOK(sync_all(ctx));
  ctx->timing = enable != 0;
  ctx->ev_used = 0;
  ctx->ev_marks.clear();
  return LFDPR_OK;
}

int lfdpr_get_timings(lfdpr_ctx* ctx, double* ms_sum, int64_t* n) {
  if (!ctx || !ms_sum || !n) return fail(ctx, LFDPR_EINVAL, "null argument");
  HIPOK(sync_all(ctx));
  for (int k = 0; k < LFDPR_N_STAGES; ++k) { ms_sum[k] = 0.0; n[k] = 0; }
  for (auto& m : ctx->ev_marks) {
    float ms = 0.0f;
    HIPOK(hipEventElapsedTime(&ms, m.second.first, m.second.second));
    ms_sum[m.first] += ms;
    n[m.first] += 1;
  }
  return LFDPR_OK;
}

}  // extern "C"

// ============================================================================
// Batches: several scenes rendered by the same kernels over one concatenated
// triangle index space (one launch per stage for the whole batch), optionally
// captured once into a hipGraph and replayed with new model matrices.
// ============================================================================

struct lfdpr_batch {
  lfdpr_ctx* ctx = nullptr;
  int n = 0;
  std::vector<int32_t> scene_ids;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_stage = nullptr;
  std::vector<Item> items;
  Item* d_items = nullptr;
  std::vector<float*> eyes;
  Model* d_models = nullptr;
  Model* h_models = nullptr;  // pinned staging
  uint64_t* keys = nullptr;
  int64_t nt = 0, per_item_px = 0;
  uint32_t* counts = nullptr;
  uint64_t* offsets = nullptr;
  TriRec* rec = nullptr;
  TriEmit* em = nullptr;
  uint64_t* tiles = nullptr;
  uint32_t* big = nullptr;
  uint32_t* tris = nullptr;
  uint64_t* stats = nullptr;
  Point* points = nullptr;
  RowEntry* rows = nullptr;
  PointBox* pbox = nullptr;
  int64_t cap = 0;
  int splat_order = LFDPR_SPLAT_POINT;
  int last_order = LFDPR_SPLAT_POINT;
  // quilt: tile asked for (0, 0: chosen for the batch), the tile of the
  // calls being enqueued, and this set's per-point rows and band lists
  // (allocated on the first quilt call)
  int quilt_rows = 0, quilt_views = 0, cur_qrows = 0, cur_qviews = 0;
  uint2* prows = nullptr;
  uint32_t* qentries = nullptr;
  uint32_t* qband = nullptr;
  int64_t q_entry_cap = 0;
  TriMat* tm = nullptr;  // physically based shading: material records and
  uint4* pmat = nullptr; // per-point material words (allocated on first use)
  Rig table_rig{};
  int splat_blocks = 4096, key_layout = 0;
  bool use_graph = true, g_valid = false;
  bool g_pbr = false;    // shading the graph was captured with
  lfdpr_shading g_sh{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t* g_views = nullptr;
  uint8_t* g_panels = nullptr;
  // Two batch frames in flight: a second set of generation buffers, swapped
  // with the fields above at every call, point generation on `gen` while the
  // previous call splats on `stream`.
  struct GenSet {
    Model* d_models = nullptr;
    Model* h_models = nullptr;
    hipEvent_t ev_stage = nullptr;
    uint32_t* counts = nullptr;
    uint64_t* offsets = nullptr;
    TriRec* rec = nullptr;
    TriEmit* em = nullptr;
    uint64_t* tiles = nullptr;
    uint32_t* big = nullptr;
    uint32_t* tris = nullptr;
    uint64_t* stats = nullptr;
    Point* points = nullptr;
    RowEntry* rows = nullptr;
    PointBox* pbox = nullptr;
    TriMat* tm = nullptr;
    uint4* pmat = nullptr;
    uint2* prows = nullptr;
    uint32_t* qentries = nullptr;
    uint32_t* qband = nullptr;
    int64_t q_entry_cap = 0;
  } alt;
  int in_flight = 1, slot = 0;
  hipStream_t gen = nullptr;
  hipEvent_t ev_gen[2] = {nullptr, nullptr}, ev_spl[2] = {nullptr, nullptr};
  bool spl_pending[2] = {false, false};
  std::string err;
};

namespace {

int bfail(lfdpr_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}

#define BHIP(call)                                                                                  \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) return bfail(b, LFDPR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// The second buffer set, the generation stream and its events.
void batch_free_alt(lfdpr_batch* b) {
  lfdpr_batch::GenSet& a = b->alt;
  dfree(a.d_models);
  if (a.h_models) (void)hipHostFree(a.h_models);
  a.h_models = nullptr;
  if (a.ev_stage) (void)hipEventDestroy(a.ev_stage);
  a.ev_stage = nullptr;
  dfree(a.counts);
  dfree(a.offsets);
  dfree(a.rec);
  dfree(a.em);
  dfree(a.tiles);
  dfree(a.big);
  dfree(a.tris);
  dfree(a.stats);
  dfree(a.points);
  dfree(a.rows);
  dfree(a.pbox);
  dfree(a.tm);
  dfree(a.pmat);
  dfree(a.prows);
  dfree(a.qentries);
  dfree(a.qband);
  a.q_entry_cap = 0;
  for (int k = 0; k < 2; ++k) {
    if (b->ev_gen[k]) (void)hipEventDestroy(b->ev_gen[k]);
    if (b->ev_spl[k]) (void)hipEventDestroy(b->ev_spl[k]);
    b->ev_gen[k] = b->ev_spl[k] = nullptr;
    b->spl_pending[k] = false;
  }
  if (b->gen) (void)hipStreamDestroy(b->gen);
  b->gen = nullptr;
}

void batch_swap_sets(lfdpr_batch* b) {
  lfdpr_batch::GenSet& a = b->alt;
  std::swap(b->d_models, a.d_models);
  std::swap(b->h_models, a.h_models);
  std::swap(b->ev_stage, a.ev_stage);
  std::swap(b->counts, a.counts);
  std::swap(b->offsets, a.offsets);
  std::swap(b->rec, a.rec);
  std::swap(b->em, a.em);
  std::swap(b->tiles, a.tiles);
  std::swap(b->big, a.big);
  std::swap(b->tris, a.tris);
  std::swap(b->stats, a.stats);
  std::swap(b->points, a.points);
  std::swap(b->rows, a.rows);
  std::swap(b->pbox, a.pbox);
  std::swap(b->tm, a.tm);
  std::swap(b->pmat, a.pmat);
  std::swap(b->prows, a.prows);
  std::swap(b->qentries, a.qentries);
  std::swap(b->qband, a.qband);
  std::swap(b->q_entry_cap, a.q_entry_cap);
}

// Every stream of the batch idle.
hipError_t batch_sync(lfdpr_batch* b) {
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess && b->gen) e = hipStreamSynchronize(b->gen);
  return e;
}

void batch_free(lfdpr_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (float* e : b->eyes) dfree(e);
  dfree(b->d_items);
  dfree(b->d_models);
  if (b->h_models) (void)hipHostFree(b->h_models);
  dfree(b->keys);
  dfree(b->counts);
  dfree(b->offsets);
  dfree(b->rec);
  dfree(b->em);
  dfree(b->tiles);
  dfree(b->big);
  dfree(b->tris);
  dfree(b->stats);
  dfree(b->points);
  dfree(b->rows);
  dfree(b->pbox);
  dfree(b->tm);
  dfree(b->pmat);
  dfree(b->prows);
  dfree(b->qentries);
  dfree(b->qband);
  batch_free_alt(b);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->ev_stage) (void)hipEventDestroy(b->ev_stage);
  if (b->stream) (void)hipStreamDestroy(b->stream);
}

// Point generation of a batch frame (statistics reset, set-up, scan, emission)
// on stream st: only kernel launches (capturable), plus stage events when
// `timed` (never while capturing).  Returns the mark at its end (timed).
hipEvent_t batch_gen(lfdpr_batch* b, hipStream_t st, bool timed) {
  lfdpr_ctx* ctx = b->ctx;
  const bool pbr = ctx->shading.mode == LFDPR_SHADE_PBR;
  auto ev = [&]() { return timed ? mark_on(ctx, st) : nullptr; };
  launch_fill_u64(b->stats, STAT_SLOTS, 0ull, st);
  hipEvent_t e0 = ev();
  SetupArgs sa{};
  sa.items = b->d_items;
  sa.n_items = b->n;
  sa.nt = b->nt;
  sa.models = b->d_models;
  sa.lod_thr = b->ctx->d_lod_thr;
  sa.counts = b->counts;
  sa.rec = b->rec;
  sa.em = b->em;
  sa.stats = b->stats;
  sa.tm = pbr ? b->tm : nullptr;
  sa.tile_sum = b->tiles;
  sa.big = b->big;
  sa.n_big = b->stats + STAT_BIG;
  launch_tri_setup(sa, b->splat_order == LFDPR_SPLAT_QUILT, st);
  hipEvent_t e1 = ev();
  launch_scan(b->tiles, b->nt, b->stats + STAT_TOTAL, st);
  hipEvent_t e2 = ev();
  EmitArgs ea{};
  ea.items = b->d_items;
  ea.nt = b->nt;
  ea.counts = b->counts;
  ea.tile_base = b->tiles;
  ea.offsets = b->offsets;
  ea.em = b->em;
  ea.points = b->points;
  ea.n_points = b->stats + STAT_TOTAL;
  ea.big = b->big;
  ea.n_big = b->stats + STAT_BIG;
  ea.cap = b->cap;
  ea.tm = pbr ? b->tm : nullptr;
  ea.pmat = pbr ? b->pmat : nullptr;
  const bool tv = !pbr && b->splat_order == LFDPR_SPLAT_TRIANGLE_VIEW;
  const bool quilt = b->splat_order == LFDPR_SPLAT_QUILT;
  ea.rec = b->rec;
  ea.rows = tv ? b->rows : nullptr;
  ea.pbox = tv || quilt ? b->pbox : nullptr;
  ea.prows = quilt ? b->prows : nullptr;
  ea.tris = tv ? b->tris : nullptr;
  ea.n_tris = b->stats + STAT_EMITTING;
  launch_emit(ea, b->splat_blocks, st);
  hipEvent_t e3 = ev();
  hipEvent_t ebin = e3;
  if (quilt) {
    launch_quilt_bin(quilt_bin_args(b->qband, b->qentries, b->q_entry_cap, b->prows, b->stats + STAT_TOTAL, b->cap,
                                    b->table_rig.H, b->cur_qrows, b->n),
                     st);
    ebin = ev();
    stage(ctx, 7, e3, ebin);
  }
  stage(ctx, 0, e0, e1);
  stage(ctx, 1, e1, e2);
  stage(ctx, 2, e2, e3);
  return ebin;
}

// Splat, resolve and interleave of a batch frame on stream st; e3 marks the
// start of the splat stage when `timed`.
void batch_splat(lfdpr_batch* b, uint32_t* views, uint8_t* panels, hipStream_t st, bool timed, hipEvent_t e3) {
  lfdpr_ctx* ctx = b->ctx;
  const bool pbr = ctx->shading.mode == LFDPR_SHADE_PBR;
  auto ev = [&]() { return timed ? mark_on(ctx, st) : nullptr; };
  SplatArgs pa{};
  pa.items = b->d_items;
  pa.n_items = b->n;
  pa.table_rig = b->table_rig;
  pa.points = b->points;
  pa.n_points = b->stats + STAT_TOTAL;
  pa.stats = b->stats;
  pa.cap = b->cap;
  pa.rec = b->rec;
  pa.em = b->em;
  pa.offsets = b->offsets;
  pa.counts = b->counts;
  pa.rows = b->rows;
  pa.pbox = !pbr && b->splat_order == LFDPR_SPLAT_TRIANGLE_VIEW ? b->pbox : nullptr;
  pa.tris = b->tris;
  pa.n_tris = b->stats + STAT_EMITTING;
  pa.nt = b->nt;
  pa.tm = pbr ? b->tm : nullptr;
  pa.pmat = pbr ? b->pmat : nullptr;
  const lfdpr_shading& sh = ctx->shading;
  pa.sh = Shading{sh.light_dir[0], sh.light_dir[1], sh.light_dir[2], sh.light_rgb[0], sh.light_rgb[1],
                  sh.light_rgb[2], sh.ambient_rgb[0], sh.ambient_rgb[1], sh.ambient_rgb[2]};
  const bool quilt = b->splat_order == LFDPR_SPLAT_QUILT;
  const uint32_t* qstate = nullptr;
  if (quilt) {
    // the tiles write every item's views; the point splat and the resolve
    // below run only if the band lists overflowed
    const QuiltBinArgs qa = quilt_bin_args(b->qband, b->qentries, b->q_entry_cap, b->prows, b->stats + STAT_TOTAL,
                                           b->cap, b->table_rig.H, b->cur_qrows, b->n);
    (void)launch_splat_quilt(quilt_tile_args(pa, qa, b->pbox, b->cur_qviews, ctx->max_lds, views, nullptr), st);
    qstate = qa.state;
    pa.gate = qstate;
  }
  launch_splat(pa, quilt ? 256 : b->splat_blocks, st);
  b->last_order = quilt ? LFDPR_SPLAT_QUILT : (pa.pbox && !pa.tm ? LFDPR_SPLAT_TRIANGLE_VIEW : LFDPR_SPLAT_POINT);
  hipEvent_t e4 = ev();
  launch_resolve(b->keys, b->n, b->table_rig.n_views, b->table_rig.H, b->table_rig.W, b->key_layout, views, nullptr, st,
                 qstate);
  hipEvent_t e5 = ev();
  if (panels) {
    InterleaveArgs ia = interleave_args(b->ctx->lens, views, b->table_rig.n_views, b->table_rig.W, b->table_rig.H, panels);
    launch_interleave_batch(ia, b->n, b->per_item_px, (int64_t)b->ctx->lens.Wp * b->ctx->lens.Hp * 3, st);
    stage(ctx, 5, e5, ev());
  }
  stage(ctx, 3, e3, e4);
  stage(ctx, 4, e4, e5);
}

// The whole batch frame on b->stream.
void batch_enqueue(lfdpr_batch* b, uint32_t* views, uint8_t* panels, bool timed) {
  const hipEvent_t e3 = batch_gen(b, b->stream, timed);
  batch_splat(b, views, panels, b->stream, timed, e3);
}

// Rows and band lists of the batch's buffer set(s) for the quilt (entries:
// twice the point capacity + 65536, at most 2^32 - 1).
int ensure_batch_quilt(lfdpr_batch* b) {
  const int64_t ecap = std::min<int64_t>(2 * b->cap + 65536, 0xFFFFFFFFll);
  const int64_t nq = 4 * kQuiltBandCap + 8;
  auto need = [&](uint2* pr) { return pr == nullptr; };
  if (!need(b->prows) && !(b->in_flight == 2 && need(b->alt.prows))) return LFDPR_OK;
  BHIP(batch_sync(b));
  bool ok = true;
  if (need(b->prows)) {
    ok = dalloc(b->prows, (size_t)b->cap) == hipSuccess && dalloc(b->qentries, (size_t)ecap) == hipSuccess &&
         dalloc(b->qband, (size_t)nq) == hipSuccess &&
         hipMemset(b->qband, 0, (size_t)nq * sizeof(uint32_t)) == hipSuccess;
    b->q_entry_cap = ecap;
  }
  if (ok && b->in_flight == 2 && need(b->alt.prows)) {
    lfdpr_batch::GenSet& a = b->alt;
    ok = dalloc(a.prows, (size_t)b->cap) == hipSuccess && dalloc(a.qentries, (size_t)ecap) == hipSuccess &&
         dalloc(a.qband, (size_t)nq) == hipSuccess &&
         hipMemset(a.qband, 0, (size_t)nq * sizeof(uint32_t)) == hipSuccess;
    a.q_entry_cap = ecap;
  }
  if (!ok) {
    dfree(b->prows);
    dfree(b->qentries);
    dfree(b->qband);
    dfree(b->alt.prows);
    dfree(b->alt.qentries);
    dfree(b->alt.qband);
    return bfail(b, LFDPR_ENOMEM, "quilt band lists");
  }
  return LFDPR_OK;
}

int batch_set_shape(lfdpr_batch* b, int splat_blocks, int key_layout) {
  if (splat_blocks == b->splat_blocks && key_layout == b->key_layout) return LFDPR_OK;
  BHIP(batch_sync(b));
  b->splat_blocks = splat_blocks;
  if (key_layout != b->key_layout) {
    b->key_layout = key_layout;
    for (auto& it : b->items) it.key_layout = key_layout;
    BHIP(hipMemcpy(b->d_items, b->items.data(), sizeof(Item) * b->n, hipMemcpyHostToDevice));
  }
  b->g_valid = false;
  return LFDPR_OK;
}

}  // namespace

extern "C" {

int lfdpr_batch_create(lfdpr_ctx* ctx, int32_t n, const int32_t* scene_ids, const lfdpr_view_params* views,
                       int64_t point_capacity, lfdpr_batch** out) {
  if (!ctx || !out || !scene_ids || !views || n < 1 || n > 256 || point_capacity < 0 || point_capacity > (1ll << 31))
    return fail(ctx, LFDPR_EINVAL, "batch arguments out of range");
  *out = nullptr;
  for (int k = 0; k < n; ++k) {
    if (!view_params_ok(&views[k])) return fail(ctx, LFDPR_EINVAL, "view parameters out of range");
    if (views[k].V * views[k].S != views[0].V * views[0].S || views[k].W != views[0].W || views[k].H != views[0].H ||
        views[k].fovy_deg != views[0].fovy_deg || views[k].aspect != views[0].aspect)
      return fail(ctx, LFDPR_EINVAL, "batch items must share views, size, field of view and aspect");
    if (ctx->scenes.find(scene_ids[k]) == ctx->scenes.end()) return fail(ctx, LFDPR_EINVAL, "unknown scene id");
  }
  HIPOK(hipSetDevice(ctx->device));
  lfdpr_batch* b = new lfdpr_batch();
  b->ctx = ctx;
  b->n = n;
  b->splat_order = ctx->splat_order;
  b->quilt_rows = ctx->quilt_rows;
  b->quilt_views = ctx->quilt_views;
  bool ok = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_stage, hipEventDisableTiming) == hipSuccess;
  b->items.resize(n);
  int64_t tri_base = 0;
  for (int k = 0; k < n && ok; ++k) {
    const SceneDev& s = ctx->scenes[scene_ids[k]];
    Rig rg{};
    std::vector<float> eye, ks;
    std::vector<double> q;
    build_rig(views[k], rg, eye, ks, q);
    float* d = nullptr;
    ok = dalloc(d, 2 * eye.size()) == hipSuccess;
    if (!ok) break;
    b->eyes.push_back(d);
    ok = hipMemcpy(d, eye.data(), 4 * eye.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(d + eye.size(), ks.data(), 4 * ks.size(), hipMemcpyHostToDevice) == hipSuccess;
    rg.eye = d;
    rg.kshift = d + eye.size();
    Item& it = b->items[k];
    it = Item{};
    it.pos = s.pos;
    it.uv = s.uv;
    it.idx = s.idx;
    it.tex = s.tex;
    it.texinfo = s.texinfo;
    it.texels = s.texels;
    it.tri_base = tri_base;
    it.nt = s.nt;
    it.rig = rg;
    it.key_layout = 0;
    tri_base += s.nt;
    if (k == 0) b->table_rig = rg;
  }
  b->nt = tri_base;
  if (b->nt >= (1ll << 28)) ok = false;  // points carry a 28-bit triangle index
  b->per_item_px = (int64_t)b->table_rig.n_views * b->table_rig.W * b->table_rig.H;
  b->cap = point_capacity ? point_capacity : (32ll << 20);
  const int64_t ntb = b->nt > 1024 ? b->nt : 1024;
  if (ok)
    ok = dalloc(b->keys, (size_t)(b->per_item_px * n)) == hipSuccess && dalloc(b->counts, ntb) == hipSuccess &&
         dalloc(b->offsets, ntb) == hipSuccess && dalloc(b->rec, ntb) == hipSuccess && dalloc(b->em, ntb) == hipSuccess &&
         dalloc(b->tiles, (ntb + 255) / 256 + 1) == hipSuccess && dalloc(b->big, ntb) == hipSuccess &&
         dalloc(b->tris, ntb) == hipSuccess && dalloc(b->rows, (size_t)b->cap) == hipSuccess &&
         dalloc(b->pbox, (size_t)b->cap) == hipSuccess &&
         dalloc(b->stats, STAT_SLOTS) == hipSuccess && dalloc(b->points, (size_t)b->cap) == hipSuccess &&
         dalloc(b->d_items, n) == hipSuccess && dalloc(b->d_models, n) == hipSuccess &&
         hipHostMalloc((void**)&b->h_models, sizeof(Model) * n, hipHostMallocDefault) == hipSuccess;
  if (ok) {
    for (int k = 0; k < n; ++k) b->items[k].keys = b->keys + b->per_item_px * k;
    ok = hipMemcpy(b->d_items, b->items.data(), sizeof(Item) * n, hipMemcpyHostToDevice) == hipSuccess;
    launch_fill_u64(b->keys, b->per_item_px * n, ~0ull, b->stream);
    ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(b->ev_stage, b->stream) == hipSuccess &&
         hipStreamSynchronize(b->stream) == hipSuccess;
  }
  if (!ok) {
    const bool too_many = b->nt >= (1ll << 28);
    batch_free(b);
    delete b;
    return too_many ? fail(ctx, LFDPR_EINVAL, "more than 2^28 - 1 triangles in one batch")
                    : fail(ctx, LFDPR_ENOMEM, "batch buffers");
  }
  for (int k = 0; k < n; ++k) {
    ctx->scenes[scene_ids[k]].batch_refs += 1;
    b->scene_ids.push_back(scene_ids[k]);
  }
  ctx->live_children += 1;
  *out = b;
  return LFDPR_OK;
}

int lfdpr_batch_destroy(lfdpr_batch* b) {
  if (!b) return LFDPR_OK;
  (void)hipSetDevice(b->ctx->device);
  (void)batch_sync(b);
  for (int32_t id : b->scene_ids) {
    auto it = b->ctx->scenes.find(id);
    if (it != b->ctx->scenes.end()) it->second.batch_refs -= 1;
  }
  b->ctx->live_children -= 1;
  batch_free(b);
  delete b;
  return LFDPR_OK;
}

const char* lfdpr_batch_last_error(lfdpr_batch* b) { return b ? b->err.c_str() : "null batch"; }

int lfdpr_batch_use_graph(lfdpr_batch* b, int enable) {
  if (!b) return LFDPR_EINVAL;
  b->use_graph = enable != 0;
  return LFDPR_OK;
}

int lfdpr_batch_set_frames_in_flight(lfdpr_batch* b, int32_t n) {
  if (!b) return LFDPR_EINVAL;
  if (n != 1 && n != 2) return bfail(b, LFDPR_EINVAL, "frames in flight must be 1 or 2");
  if (n == b->in_flight) return LFDPR_OK;
  BHIP(hipSetDevice(b->ctx->device));
  BHIP(batch_sync(b));
  b->g_valid = false;  // a captured graph names the buffers of one set
  if (n == 1) {
    batch_free_alt(b);
    b->in_flight = 1;
    return LFDPR_OK;
  }
  const int64_t ntb = b->nt > 1024 ? b->nt : 1024;
  lfdpr_batch::GenSet& a = b->alt;
  bool ok = hipStreamCreateWithFlags(&b->gen, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&a.ev_stage, hipEventDisableTiming) == hipSuccess &&
            hipEventRecord(a.ev_stage, b->gen) == hipSuccess;
  for (int k = 0; k < 2 && ok; ++k)
    ok = hipEventCreateWithFlags(&b->ev_gen[k], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&b->ev_spl[k], hipEventDisableTiming) == hipSuccess;
  if (ok)
    ok = dalloc(a.counts, ntb) == hipSuccess && dalloc(a.offsets, ntb) == hipSuccess && dalloc(a.rec, ntb) == hipSuccess &&
         dalloc(a.em, ntb) == hipSuccess && dalloc(a.tiles, (ntb + 255) / 256 + 1) == hipSuccess &&
         dalloc(a.big, ntb) == hipSuccess && dalloc(a.stats, STAT_SLOTS) == hipSuccess &&
         dalloc(a.tris, ntb) == hipSuccess && dalloc(a.rows, (size_t)b->cap) == hipSuccess &&
         dalloc(a.pbox, (size_t)b->cap) == hipSuccess &&
         dalloc(a.points, (size_t)b->cap) == hipSuccess && dalloc(a.d_models, b->n) == hipSuccess &&
         hipHostMalloc((void**)&a.h_models, sizeof(Model) * b->n, hipHostMallocDefault) == hipSuccess;
  if (ok && b->tm) ok = dalloc(a.tm, (size_t)ntb) == hipSuccess && dalloc(a.pmat, (size_t)b->cap) == hipSuccess;
  if (ok) ok = hipStreamSynchronize(b->gen) == hipSuccess;
  if (!ok) {
    batch_free_alt(b);
    return bfail(b, LFDPR_ENOMEM, "second batch buffer set");
  }
  b->slot = 0;
  b->in_flight = 2;
  return LFDPR_OK;
}

int lfdpr_batch_render(lfdpr_batch* b, const float* models, uint32_t* views, uint8_t* panels) {
  if (!b || !models || !views) return bfail(b, LFDPR_EINVAL, "null argument");
  const bool pbr = b->ctx->shading.mode == LFDPR_SHADE_PBR;
  if (pbr)
    for (int k = 0; k < b->n; ++k) {
      const SceneDev& s = b->ctx->scenes[b->scene_ids[k]];
      if (s.nt > 0 && !s.mat)
        return bfail(b, LFDPR_ESTATE, "physically based shading needs lfdpr_scene_set_materials on every scene");
    }
  if (panels && (!b->ctx->lens_set || b->table_rig.n_views < 1))
    return bfail(b, LFDPR_ESTATE, "lfdpr_set_lens on the context first");
  for (int k = 0; k < 12 * b->n; ++k)
    if (!std::isfinite(models[k])) return bfail(b, LFDPR_EINVAL, "non-finite model matrix");
  BHIP(hipSetDevice(b->ctx->device));
  // shading: material buffers on first use, the items' material tables, and a
  // new graph when the captured shading differs
  if (pbr && (!b->tm || (b->in_flight == 2 && !b->alt.tm))) {
    BHIP(batch_sync(b));
    const int64_t ntb = b->nt > 1024 ? b->nt : 1024;
    bool ok = true;
    if (!b->tm) ok = dalloc(b->tm, (size_t)ntb) == hipSuccess && dalloc(b->pmat, (size_t)b->cap) == hipSuccess;
    if (ok && b->in_flight == 2 && !b->alt.tm)
      ok = dalloc(b->alt.tm, (size_t)ntb) == hipSuccess && dalloc(b->alt.pmat, (size_t)b->cap) == hipSuccess;
    if (!ok) {
      dfree(b->tm);
      dfree(b->pmat);
      dfree(b->alt.tm);
      dfree(b->alt.pmat);
      return bfail(b, LFDPR_ENOMEM, "material buffers");
    }
  }
  bool items_changed = false;
  for (int k = 0; k < b->n; ++k) {
    const uint16_t* m = pbr ? b->ctx->scenes[b->scene_ids[k]].mat : nullptr;
    if (b->items[k].mat != m) {
      b->items[k].mat = m;
      items_changed = true;
    }
  }
  if (items_changed) {
    BHIP(batch_sync(b));  // earlier replays may still read the table
    BHIP(hipMemcpy(b->d_items, b->items.data(), sizeof(Item) * b->n, hipMemcpyHostToDevice));
  }
  if (items_changed || b->g_pbr != pbr ||
      (pbr && std::memcmp(&b->g_sh, &b->ctx->shading, sizeof b->g_sh) != 0))
    b->g_valid = false;
  if (b->splat_order == LFDPR_SPLAT_QUILT) {
    int qr = 0, qv = 0;
    if (!quilt_shape_for(b->table_rig, b->ctx->max_lds, b->quilt_rows, b->quilt_views, b->n, qr, qv))
      return bfail(b, LFDPR_EINVAL, "quilt tile does not fit the device's LDS or the batch's band lists");
    if (qr != b->cur_qrows || qv != b->cur_qviews) b->g_valid = false;
    b->cur_qrows = qr;
    b->cur_qviews = qv;
    int rc = ensure_batch_quilt(b);
    if (rc) return rc;
  }
  if (b->in_flight == 2) {
    // this call's generation buffers; generation waits only for the splat
    // that last read them, the splat for earlier work on the context's stream
    batch_swap_sets(b);
    b->slot ^= 1;
    const int sl = b->slot;
    const bool timed = b->ctx->timing;
    BHIP(hipEventSynchronize(b->ev_stage));
    std::memcpy(b->h_models, models, sizeof(Model) * b->n);
    if (b->spl_pending[sl]) BHIP(hipStreamWaitEvent(b->gen, b->ev_spl[sl], 0));
    BHIP(hipMemcpyAsync(b->d_models, b->h_models, sizeof(Model) * b->n, hipMemcpyHostToDevice, b->gen));
    BHIP(hipEventRecord(b->ev_stage, b->gen));
    (void)batch_gen(b, b->gen, timed);
    BHIP(hipGetLastError());
    BHIP(hipEventRecord(b->ev_gen[sl], b->gen));
    BHIP(hipEventRecord(b->ev_in, b->ctx->stream));
    BHIP(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    BHIP(hipStreamWaitEvent(b->stream, b->ev_gen[sl], 0));
    batch_splat(b, views, panels, b->stream, timed, timed ? mark_on(b->ctx, b->stream) : nullptr);
    BHIP(hipGetLastError());
    BHIP(hipEventRecord(b->ev_spl[sl], b->stream));
    b->spl_pending[sl] = true;
    BHIP(hipEventRecord(b->ev_out, b->stream));
    BHIP(hipStreamWaitEvent(b->ctx->stream, b->ev_out, 0));
    return LFDPR_OK;
  }
  // model matrices: pinned staging -> device, outside any graph
  BHIP(hipEventSynchronize(b->ev_stage));
  std::memcpy(b->h_models, models, sizeof(Model) * b->n);
  BHIP(hipEventRecord(b->ev_in, b->ctx->stream));
  BHIP(hipStreamWaitEvent(b->stream, b->ev_in, 0));
  BHIP(hipMemcpyAsync(b->d_models, b->h_models, sizeof(Model) * b->n, hipMemcpyHostToDevice, b->stream));
  BHIP(hipEventRecord(b->ev_stage, b->stream));
  if (b->use_graph) {
    if (!b->g_valid || b->g_views != views || b->g_panels != panels) {
      if (b->exec) { BHIP(hipGraphExecDestroy(b->exec)); b->exec = nullptr; }
      if (b->graph) { BHIP(hipGraphDestroy(b->graph)); b->graph = nullptr; }
      BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      batch_enqueue(b, views, panels, false);
      hipError_t ce = hipStreamEndCapture(b->stream, &b->graph);
      if (ce != hipSuccess) return bfail(b, LFDPR_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
      BHIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      b->g_views = views;
      b->g_panels = panels;
      b->g_pbr = pbr;
      b->g_sh = b->ctx->shading;
      b->g_valid = true;
    }
    BHIP(hipGraphLaunch(b->exec, b->stream));
  } else {
    batch_enqueue(b, views, panels, b->ctx->timing);
    BHIP(hipGetLastError());
  }
  BHIP(hipEventRecord(b->ev_out, b->stream));
  BHIP(hipStreamWaitEvent(b->ctx->stream, b->ev_out, 0));
  return LFDPR_OK;
}

int lfdpr_batch_stats(lfdpr_batch* b, lfdpr_stats* out) {
  if (!b || !out) return LFDPR_EINVAL;
  uint64_t st[STAT_SLOTS];
  BHIP(hipSetDevice(b->ctx->device));
  BHIP(hipStreamSynchronize(b->stream));
  BHIP(hipMemcpy(st, b->stats, sizeof st, hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof *out);
  out->points = (int64_t)st[STAT_TOTAL];
  out->active_tris = (int64_t)st[STAT_ACTIVE];
  out->point_views = (int64_t)st[STAT_POINT_VIEWS];
  out->overflow_tris = (int64_t)st[STAT_OVERFLOW];
  out->written_px = (int64_t)st[STAT_WRITTEN];
  out->splat_order = b->last_order;
  out->covered_px = b->last_order == LFDPR_SPLAT_TRIANGLE_VIEW ? (int64_t)st[STAT_COVERED] : -1;
  out->missed_px = out->covered_px >= 0 ? out->covered_px - out->written_px : -1;
  out->quilt_entries = -1;
  if (b->last_order == LFDPR_SPLAT_QUILT) {
    uint32_t qs[2];
    BHIP(hipMemcpy(qs, b->qband + 4 * kQuiltBandCap + 1, sizeof qs, hipMemcpyDeviceToHost));
    out->quilt_rows = b->cur_qrows;
    out->quilt_views = b->cur_qviews;
    out->quilt_entries = (int64_t)qs[1];
    if (qs[0]) out->splat_order = LFDPR_SPLAT_POINT;  // the lists overflowed: splatted per point
  }
  out->capacity = b->cap;
  out->point_overflow = out->points > b->cap ? 1 : 0;
  out->n_views = b->table_rig.n_views;
  return out->point_overflow ? LFDPR_EOVERFLOW : LFDPR_OK;
}

// Times every candidate (splat launch blocks x key layout) on the batch's own
// workload and keeps the fastest; the results are returned per candidate.
int lfdpr_batch_autotune(lfdpr_batch* b, const float* models, uint32_t* views, lfdpr_tune_result* res) {
  if (!b || !models || !views || !res) return bfail(b, LFDPR_EINVAL, "null argument");
  static const int kBlocks[] = {1024, 2048, 4096, 8192, 16384};
  static const int kQuiltRows[] = {1, 2, 4, 8};
  // candidates: the batch's per-point (or triangle-view) order under every
  // launch shape and key layout, then the quilt under each band height with
  // the most views that fit (its band lists hold every item's bands)
  struct Cand {
    int order, blocks, layout, qrows, qviews;
  };
  std::vector<Cand> cands;
  const int base_order = b->splat_order == LFDPR_SPLAT_QUILT ? LFDPR_SPLAT_POINT : b->splat_order;
  for (int layout = 0; layout < 2; ++layout)
    for (int blocks : kBlocks) cands.push_back({base_order, blocks, layout, 0, 0});
  for (int r : kQuiltRows) {
    int qr = 0, qv = 0, v = 0;
    while (v < b->table_rig.n_views && quilt_lds_bytes(r, v + 1, b->table_rig.W, b->table_rig.H) <= (size_t)b->ctx->max_lds) ++v;
    if (v == 0) continue;
    const int subsets = (b->table_rig.n_views + v - 1) / v;
    if (!quilt_shape_for(b->table_rig, b->ctx->max_lds, r, (b->table_rig.n_views + subsets - 1) / subsets, b->n, qr, qv))
      continue;
    cands.push_back({LFDPR_SPLAT_QUILT, b->splat_blocks, b->key_layout, qr, qv});
  }
  const int saved[5] = {b->splat_order, b->splat_blocks, b->key_layout, b->quilt_rows, b->quilt_views};
  const bool graph = b->use_graph;
  b->use_graph = false;
  hipEvent_t t0, t1;
  BHIP(hipEventCreate(&t0));
  BHIP(hipEventCreate(&t1));
  std::memset(res, 0, sizeof *res);
  float best = INFINITY;
  int rc = LFDPR_OK;
  for (const Cand& c : cands) {
    if (res->n >= (int)(sizeof res->entries / sizeof res->entries[0])) break;
    rc = batch_set_shape(b, c.blocks, c.layout);
    if (rc) break;
    b->splat_order = c.order;
    b->quilt_rows = c.qrows;
    b->quilt_views = c.qviews;
    for (int w = 0; w < 2 && !rc; ++w) rc = lfdpr_batch_render(b, models, views, nullptr);
    if (rc) break;
    (void)hipEventRecord(t0, b->stream);
    for (int w = 0; w < 3 && !rc; ++w) rc = lfdpr_batch_render(b, models, views, nullptr);
    (void)hipEventRecord(t1, b->stream);
    (void)hipEventSynchronize(t1);
    if (rc) break;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    lfdpr_tune_entry& e = res->entries[res->n++];
    e.splat_blocks = c.blocks;
    e.key_layout = c.layout;
    e.ms = ms / 3.0f;
    e.splat_order = b->last_order;
    e.quilt_rows = c.qrows;
    e.quilt_views = c.qviews;
    if (e.ms < best) {
      best = e.ms;
      res->best = res->n - 1;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  b->use_graph = graph;
  b->g_valid = false;
  if (rc || res->n == 0) {
    b->splat_order = saved[0];
    b->quilt_rows = saved[3];
    b->quilt_views = saved[4];
    const int rc2 = batch_set_shape(b, saved[1], saved[2]);
    return rc ? rc : (rc2 ? rc2 : bfail(b, LFDPR_ESTATE, "no candidate ran"));
  }
  const lfdpr_tune_entry& e = res->entries[res->best];
  b->splat_order = e.splat_order == LFDPR_SPLAT_QUILT ? LFDPR_SPLAT_QUILT : base_order;
  b->quilt_rows = e.quilt_rows;
  b->quilt_views = e.quilt_views;
  return batch_set_shape(b, e.splat_blocks, e.key_layout);
}

// Same search for single frames of one scene on the context.
int lfdpr_autotune(lfdpr_ctx* ctx, int32_t scene_id, const float* model, uint32_t* views, lfdpr_tune_result* res) {
  if (!ctx || !model || !views || !res) return fail(ctx, LFDPR_EINVAL, "null argument");
  static const int kBlocks[] = {1024, 2048, 4096, 8192, 16384};
  static const int kQuiltRows[] = {1, 2, 4, 8};
  // candidates: the per-point (or per triangle-view) order under every launch
  // shape and key layout, then the quilt under each band height with the most
  // views that fit
  struct Cand {
    int order, blocks, layout, qrows, qviews;
  };
  std::vector<Cand> cands;
  const int base_order = ctx->splat_order == LFDPR_SPLAT_QUILT ? LFDPR_SPLAT_POINT : ctx->splat_order;
  for (int layout = 0; layout < 2; ++layout)
    for (int blocks : kBlocks) cands.push_back({base_order, blocks, layout, 0, 0});
  if (ctx->views_set)
    for (int r : kQuiltRows) {
      if (r > ctx->rig.H) continue;
      int v = 0;
      while (v < ctx->rig.n_views && quilt_lds_bytes(r, v + 1, ctx->rig.W, ctx->rig.H) <= (size_t)ctx->max_lds) ++v;
      if (v == 0) continue;
      const int subsets = (ctx->rig.n_views + v - 1) / v;
      cands.push_back({LFDPR_SPLAT_QUILT, ctx->splat_blocks, ctx->key_layout, r, (ctx->rig.n_views + subsets - 1) / subsets});
    }
  const int saved[5] = {ctx->splat_order, ctx->splat_blocks, ctx->key_layout, ctx->quilt_rows, ctx->quilt_views};
  hipEvent_t t0, t1;
  HIPOK(hipEventCreate(&t0));
  HIPOK(hipEventCreate(&t1));
  std::memset(res, 0, sizeof *res);
  float best = INFINITY;
  int rc = LFDPR_OK;
  for (const Cand& c : cands) {
    if (res->n >= (int)(sizeof res->entries / sizeof res->entries[0])) break;
    ctx->splat_order = c.order;
    ctx->splat_blocks = c.blocks;
    ctx->key_layout = c.layout;
    ctx->quilt_rows = c.qrows;
    ctx->quilt_views = c.qviews;
    for (int w = 0; w < 2 && !rc; ++w) rc = lfdpr_render_frame(ctx, scene_id, model, views, nullptr);
    if (rc) break;
    (void)hipEventRecord(t0, ctx->stream);
    for (int w = 0; w < 3 && !rc; ++w) rc = lfdpr_render_frame(ctx, scene_id, model, views, nullptr);
    (void)hipEventRecord(t1, ctx->stream);
    (void)hipEventSynchronize(t1);
    if (rc) break;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    lfdpr_tune_entry& e = res->entries[res->n++];
    e.splat_blocks = c.blocks;
    e.key_layout = c.layout;
    e.ms = ms / 3.0f;
    e.splat_order = c.order;
    e.quilt_rows = c.qrows;
    e.quilt_views = c.qviews;
    if (e.ms < best) {
      best = e.ms;
      res->best = res->n - 1;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (rc || res->n == 0) {
    ctx->splat_order = saved[0];
    ctx->splat_blocks = saved[1];
    ctx->key_layout = saved[2];
    ctx->quilt_rows = saved[3];
    ctx->quilt_views = saved[4];
    return rc ? rc : fail(ctx, LFDPR_ESTATE, "no candidate ran");
  }
  const lfdpr_tune_entry& b = res->entries[res->best];
  ctx->splat_order = b.splat_order;
  ctx->splat_blocks = b.splat_blocks;
  ctx->key_layout = b.key_layout;
  ctx->quilt_rows = b.quilt_rows;
  ctx->quilt_views = b.quilt_views;
  return LFDPR_OK;
}

int lfdpr_set_frames_in_flight(lfdpr_ctx* ctx, int32_t n) {
  if (!ctx || n < 1 || n > 2) return fail(ctx, LFDPR_EINVAL, "frames in flight must be 1 or 2");
  HIPOK(hipSetDevice(ctx->device));
  HIPOK(sync_all(ctx));
  if (n == 2 && !ctx->side) {
    // created together or not at all: the context keeps them only on success
    hipStream_t side = nullptr;
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool ok = hipStreamCreateWithFlags(&side, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; k < 6 && ok; ++k) ok = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
      if (side) (void)hipStreamDestroy(side);
      return fail(ctx, LFDPR_EDEVICE, "creating the second stream and its events");
    }
    ctx->side = side;
    ctx->ev_emitted[0] = ev[0];
    ctx->ev_emitted[1] = ev[1];
    ctx->ev_splatted[0] = ev[2];
    ctx->ev_splatted[1] = ev[3];
    ctx->ev_caller = ev[4];
    ctx->ev_start = ev[5];
  }
  ctx->frames_in_flight = n;
  ctx->splatted_pending[0] = ctx->splatted_pending[1] = false;
  ctx->start_pending = false;
  return LFDPR_OK;
}

int lfdpr_set_launch(lfdpr_ctx* ctx, int32_t splat_blocks, int32_t key_layout) {
  if (!ctx || splat_blocks < 1 || splat_blocks > (1 << 20) || key_layout < 0 || key_layout > 1)
    return fail(ctx, LFDPR_EINVAL, "launch shape out of range");
  HIPOK(sync_all(ctx));
  ctx->splat_blocks = splat_blocks;
  ctx->key_layout = key_layout;
  return LFDPR_OK;
}

}  // extern "C"
