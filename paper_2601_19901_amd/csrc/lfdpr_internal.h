// Internal interface between the C ABI and the kernels (not exported).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lfdpr_device.h"

namespace lfdpr {

enum StatSlot { STAT_ACTIVE = 0, STAT_OVERFLOW = 1, STAT_POINT_VIEWS = 2, STAT_TOTAL = 3, STAT_BIG = 4,
                STAT_WRITTEN = 5, STAT_EMITTING = 6, STAT_COVERED = 7, STAT_SLOTS = 8 };

// One frame of one scene inside a (possibly single-element) batch.  Items share
// the view size and projection (W, H, fovy, aspect); eye tables may differ.
struct Item {
  const float* pos;
  const float* uv;
  const uint32_t* idx;
  const uint16_t* tex;
  const TexInfo* texinfo;
  const uint8_t* texels;
  int64_t tri_base;  // first batch-wide triangle index of this item
  int32_t nt;
  int32_t key_layout;  // 0: keys [view][y][x]; 1: keys [y][view][x] (views of a row adjacent)
  Rig rig;
  uint64_t* keys;    // rig.n_views * H * W keys of this item
  const uint16_t* mat;  // physically based mode: nt x (normal, roughness, metallic) texture ids; else null
};

__device__ __forceinline__ int find_item(const Item* items, int n, int64_t t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (items[mid].tri_base <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct SetupArgs {
  const Item* items;
  int32_t n_items;
  int64_t nt;              // triangles over all items
  Model model;             // used when models == nullptr (single frame)
  const Model* models;     // per item (batch)
  const float* lod_thr;    // 128 mantissa thresholds
  uint32_t* counts;
  TriRec* rec;
  TriEmit* em;
  float* dbgf;     // optional nt*8
  int32_t* dbgi;   // optional nt*8
  uint64_t* stats;
  TriMat* tm;      // physically based mode: per-triangle material records; else null
  uint64_t* tile_sum;  // per workgroup (256 triangles): the sum of their counts
  uint32_t* big;       // triangles with more than kBigCells cells (capacity nt)
  uint64_t* n_big;     // and their number
};

struct EmitArgs {
  const Item* items;
  int64_t nt;
  const uint32_t* big;       // triangles emitted cooperatively, queued by the set-up
  const uint64_t* n_big;
  const uint32_t* counts;
  const uint64_t* tile_base;  // exclusive point offset of each tile of 256 triangles
  uint64_t* offsets;          // written: first point of each triangle
  const TriEmit* em;
  Point* points;
  const uint64_t* n_points;  // device count (total emitted)
  int64_t cap;
  const TriMat* tm;          // physically based mode: material records, and
  uint4* pmat;               // per point normal min/max and roughness/metallic bytes; else null
  // triangle-major splat data (null when the point-major splat is used):
  const TriRec* rec;         // set-up records (for the point boxes)
  RowEntry* rows;            // per lattice row, at the triangle's first point + (j - jlo)
  PointBox* pbox;            // per point
  uint32_t* tris;            // triangles with points (any order) and their number
  uint64_t* n_tris;
  // row-band quilt: per point the pixel rows its splat can write in any view,
  // as rows of the batch's stacked views (item * H + row; first, last), or
  // (~0, ~0) for none; null otherwise
  uint2* prows;
};

struct SplatArgs {
  const Item* items;
  int32_t n_items;
  Rig table_rig;             // view size and projection shared by all items
  const Point* points;
  const uint64_t* n_points;  // device count (total emitted)
  int64_t cap;
  const TriRec* rec;
  const TriMat* tm;          // physically based mode; else null
  const uint4* pmat;
  Shading sh;
  uint64_t* stats;           // STAT_WRITTEN: pixels written (64-bit key updates issued);
                             // STAT_COVERED: covered pixels visited (triangle-view order)
  // triangle-major splat (used when pbox is not null)
  const TriEmit* em;
  const uint64_t* offsets;   // first point of each triangle
  const uint32_t* counts;    // points of each triangle
  const RowEntry* rows;
  const PointBox* pbox;
  const uint32_t* tris;
  const uint64_t* n_tris;
  int64_t nt;                // triangles of the launch (capacity of tris)
  // point-major splat: runs only when gate is null or *gate != 0 (the
  // quilt's fallback when its band lists overflowed)
  const uint32_t* gate;
  // row-band quilt (k_splat_quilt): per-point splat rectangles in pbox, the
  // band lists, and the views it writes directly
  const uint32_t* q_entries;   // point indices grouped by band
  const uint32_t* q_band_off;  // q_bands + 1 offsets into q_entries
  const uint32_t* q_order;     // bands by decreasing number of entries
  const uint32_t* q_state;     // [0] != 0: the lists overflowed, the point splat takes the frame
  int32_t q_rows, q_views, q_bands, q_subsets;  // tile: q_rows rows x q_views views x W
  int32_t q_bands_item;        // bands per item (q_bands over all items)
  int32_t q_block;             // threads per quilt workgroup: 1024, or 512 (two tiles per CU)
  uint32_t* out_rgba;          // the views, [view][y][x]
  float* out_depth;            // optional, [view][y][x]
};

// Band lists of the row-band quilt: every point goes to each band of q_rows
// pixel rows that its splat can write in some view (its rows do not depend
// on the eye offset).
struct QuiltBinArgs {
  const uint64_t* n_points;  // device count (total emitted)
  int64_t cap;
  const uint2* prows;        // per point: first and last stacked row (item * H + row), or ~0
  int32_t H, rows;           // view height, rows per band
  int32_t bands_item, bands; // bands per item, over all items
  uint32_t* band_cnt;  // entries per band (zero on entry; left zero)
  uint32_t* band_off;  // bands + 1 exclusive offsets
  uint32_t* band_cur;  // scatter cursors
  uint32_t* order;     // bands by decreasing entries, ties by band
  uint32_t* entries;
  int64_t entry_cap;
  uint32_t* state;     // [0]: 1 when the entries exceed entry_cap; [1]: entries
};

struct InterleaveArgs {
  const uint32_t* views;
  int32_t V, Wv, Hv, Wp, Hp, mode;
  uint32_t K1, Ky, K0;
  int64_t du[8];
  int32_t dx[8], dy[8];
  uint8_t* panel;
};

struct AngularArgs {
  const uint32_t* sub;
  uint32_t* out;
  int32_t V, W, H, maxe;
  const int32_t* cnt;
  const int32_t* src;
  const uint32_t* wt;
};

void launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
void launch_store_item(const Item& it, Item* dst, hipStream_t s);
void launch_export_stats(const uint64_t* st, int64_t cap, int64_t* out, hipStream_t s);
void launch_build_mip(const uint32_t* src, uint32_t* dst, int s, hipStream_t st);
// lean: the set-up form that stores its records before the lattice count
// (fewer registers; used beside the quilt splat)
void launch_tri_setup(const SetupArgs& a, bool lean, hipStream_t s);
// tile sums (written by the set-up) -> exclusive tile bases, and the total
void launch_scan(uint64_t* tile_sum, int64_t nt, uint64_t* total, hipStream_t s);
void launch_emit(const EmitArgs& a, int fetch_blocks, hipStream_t s);
void launch_splat(const SplatArgs& a, int grid_blocks, hipStream_t s);
// the quilt: band lists (bins), then one workgroup per (band, view subset)
// tile in decreasing band size; the tile's LDS bytes
size_t quilt_lds_bytes(int32_t rows, int32_t views, int32_t W, int32_t H);
constexpr int kQuiltBandCap = 8192;  // bands of a frame or batch frame
// Lets the tile kernels take up to lds bytes of LDS (once per device, before
// any launch or graph capture).
hipError_t prepare_quilt_kernels(size_t lds);
void launch_quilt_bin(const QuiltBinArgs& a, hipStream_t s);
hipError_t launch_splat_quilt(const SplatArgs& a, hipStream_t s);
void launch_resolve(uint64_t* keys, int64_t n_items, int32_t n_views, int32_t H, int32_t W, int32_t key_layout,
                    uint32_t* rgba, float* depth, hipStream_t s, const uint32_t* gate = nullptr);
void launch_interleave_batch(const InterleaveArgs& a, int n_items, int64_t view_stride, int64_t panel_stride, hipStream_t s);
void launch_interleave(const InterleaveArgs& a, hipStream_t s);
void launch_angular_filter(const AngularArgs& a, hipStream_t s);

}  // namespace lfdpr

struct lfdpr_ctx;
hipStream_t ctx_stream_of(lfdpr_ctx* c);
int ctx_device_of(lfdpr_ctx* c);
// networks count as children of their context (it is not destroyed under them)
void ctx_children_add(lfdpr_ctx* c, int delta);
