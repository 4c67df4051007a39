/*
 * lfdpr.h — C ABI of the light field display point rendering (LFDPR) hot path
 * on AMD Instinct MI355X (gfx950).
 *
 * One frame (Gavane & Watson, Light Field Display Point Rendering, Sec. 3-4):
 *   1. point generation from textured triangles with LFD-biased horizontal /
 *      vertical sampling densities and texture-based coarsening (Sec. 3.1,
 *      Eqs. 1-3), multiview-mip set-up and two mip fetches per point
 *      (Sec. 3.3, Eqs. 4-7);
 *   2. splatting of every point into every light-field view with per-view
 *      texture interpolation (Sec. 3.2, Eqs. 8-9) and a 64-bit (depth,
 *      colour) minimum per pixel (Sec. 5.1);
 *   3. interleaving of the views into the tilted-lenticular panel with
 *      optional Gaussian reconstruction, and the angular supersampling filter
 *      (Sec. 4).
 *
 * Conventions shared by every entry point:
 *   - Every function returns an int status: LFDPR_OK (0) or a negative
 *     LFDPR_E* code.  lfdpr_strerror() names a code; lfdpr_last_error() gives
 *     the message of the context's last failure.  Nothing else crosses the ABI
 *     on error (no exceptions, no aborts); a failed call leaves the context
 *     usable unless it returned LFDPR_EDEVICE.
 *   - "device" pointers are HIP device memory on the context's device, owned
 *     by the caller; "host" pointers are ordinary process memory, owned by the
 *     caller and only read during the call.  Memory the library allocates
 *     (scene copies, mip chains, per-triangle records, the point buffer, the
 *     64-bit key buffer) belongs to the context and is freed by lfdpr_destroy.
 *   - Work is enqueued on the stream given to lfdpr_create and is asynchronous
 *     unless stated otherwise; device outputs are valid once that stream has
 *     been synchronised.  A context is used from one host thread at a time.
 *   - Images: views are RGBA8 packed in uint32 (R in the low byte), laid out
 *     [view][row][column]; depth is FP32 camera-space Z, +inf where empty;
 *     the panel is RGB8, [row][column][3].
 */
#ifndef LFDPR_H
#define LFDPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LFDPR_ABI_VERSION 6

enum {
  LFDPR_OK = 0,
  LFDPR_EINVAL = -1,    /* bad argument (null pointer, size out of range, unknown id) */
  LFDPR_ENOMEM = -2,    /* device allocation failed */
  LFDPR_EOVERFLOW = -3, /* point capacity exceeded in the last frame (reported by lfdpr_get_stats) */
  LFDPR_EDEVICE = -4,   /* a HIP runtime call failed */
  LFDPR_ESTATE = -5     /* call out of order (e.g. render before lfdpr_set_views) */
};

enum { LFDPR_RECON_NONE = 0, LFDPR_RECON_SPATIAL = 1, LFDPR_RECON_ANGULAR = 2, LFDPR_RECON_BOTH = 3 };
/* Order in which the splat visits its work (lfdpr_set_splat_order); all give
 * the same keys, hence the same views, bit for bit. */
enum { LFDPR_SPLAT_POINT = 0, LFDPR_SPLAT_TRIANGLE_VIEW = 1, LFDPR_SPLAT_QUILT = 2 };
enum { LFDPR_SHADE_UNLIT = 0, LFDPR_SHADE_PBR = 1 };

typedef struct lfdpr_ctx lfdpr_ctx;

/* Scene: a flat indexed triangle mesh in scene coordinates with one RGBA8
 * albedo texture per triangle (Sec. 3.1, Eq. 1 with |T| = 1).  Triangles are
 * wound so that (P1-P0) x (P2-P0) points out of the surface.  All pointers
 * are host pointers; the data is copied. */
typedef struct {
  int32_t n_verts, n_tris;
  const float* pos;            /* host, n_verts*3 (x, y, z) */
  const float* uv;             /* host, n_verts*2 */
  const uint32_t* idx;         /* host, n_tris*3, each < n_verts */
  const uint16_t* tex_id;      /* host, n_tris, each < n_tex */
  int32_t n_tex;               /* 1..65535 */
  const int32_t* tex_size;     /* host, n_tex; square edge, power of two in [1, 16384] */
  const uint8_t* const* tex_rgba8; /* host, n_tex pointers to level-0 RGBA8 texels, row-major */
} lfdpr_scene_desc;

/* Light-field rig (Sec. 3.1: centres of projection distributed horizontally;
 * Sec. 4: angular supersampling).  V views of W x H pixels, rendered as V*S
 * sub-views; parallel off-axis cameras sharing the focal plane Z = D; eye r at
 * x = D tan(cone/2) (2 q_r / V - 1) with q = v + 0.5 (S = 1) or
 * q = v + (k + 0.5 + jitter[v*S+k]) / S.  Pixels are `aspect` times wider than
 * tall (the LFD anisotropy of Sec. 3.1). */
typedef struct {
  int32_t V, S, W, H;          /* V*S in [1, 1024]; W, H in [1, 4096] */
  float fovy_deg, aspect, D, cone_deg, znear;
  const float* jitter;         /* host, V*S values in [-0.5, 0.5); may be NULL when S == 1 */
  int32_t mip;                 /* multiview mipmapping (Sec. 3.3) on (1) or off (0) */
  int64_t point_capacity;      /* points per frame the context reserves; 0 = 8M */
} lfdpr_view_params;

/* Tilted lenticular panel (Sec. 4, prototype of Sec. 5.1): Wp x Hp RGB
 * pixels; lens phase of subpixel X' in row Y is frac((X' - 3*slope*Y)/pitch +
 * offset).  Reconstruction taps (Sec. 4: Gaussian, 8 random samples): du in
 * Q32 view intervals, dx/dy in Q8 view pixels. */
typedef struct {
  int32_t Wp, Hp;              /* in [1, 16384] */
  double pitch_subpx, slope, offset;
  int32_t mode;                /* LFDPR_RECON_* */
  int64_t taps[8][3];
} lfdpr_lens_params;

typedef struct {
  int64_t points;          /* points emitted by the last frame (may exceed capacity) */
  int64_t active_tris;     /* triangles visible in at least one view */
  int64_t point_views;     /* sum over points of the views their triangle is active in */
  int64_t overflow_tris;   /* triangles whose lattice exceeded the cell caps (no points) */
  int64_t capacity;        /* point capacity of the context */
  int32_t point_overflow;  /* 1 when points > capacity (frame incomplete) */
  int32_t n_views;         /* rendered (sub-)views */
  int64_t written_px;      /* (point, view, pixel) depth-test updates the splat issued: every
                              covered pixel of a visible triangle, owned by one point (Sec. 3.2) */
  int32_t splat_order;     /* LFDPR_SPLAT_* the last frame's splat used */
  int32_t reserved;
  /* Hole census (Sec. 3.2), observed by the triangle-view splat order only (-1
   * under the point order, which never visits a pixel no point covers):
   * covered_px counts the pixels inside an active (triangle, view) pair's Q8
   * triangle, over the triangles that have points; missed_px those that no point
   * writes -- the eye ray meets the plane behind the eye, or the pixel lies
   * outside the splat box of the point owning its cell.  A triangle without
   * points (an orphan: only an overflowed lattice, counted in overflow_tris) is
   * not visited. */
  int64_t covered_px;
  int64_t missed_px;
  /* Row-band quilt (LFDPR_SPLAT_QUILT): the last frame's tile (pixel rows x
   * views per LDS tile; 0 under the other orders) and its band-list entries,
   * one per (point, band of quilt_rows rows its splat reaches) (-1 under the
   * other orders).  When the entries exceed the context's list capacity the
   * frame is splatted per point instead and splat_order says so. */
  int32_t quilt_rows;
  int32_t quilt_views;
  int64_t quilt_entries;
} lfdpr_stats;

/* Version of this ABI (LFDPR_ABI_VERSION). */
int lfdpr_abi_version(void);

/* Static text for a status code; never NULL. */
const char* lfdpr_strerror(int code);

/* Creates a context on HIP device `device`, enqueuing on `stream` (a
 * hipStream_t; NULL = the null stream).  *out receives the context. */
int lfdpr_create(int device, void* stream, lfdpr_ctx** out);

/* Frees the context and every device buffer it owns.  NULL is accepted.
 * LFDPR_ESTATE (nothing freed) while batches or networks created on it are
 * alive: destroy those first. */
int lfdpr_destroy(lfdpr_ctx* ctx);

/* Message of the last failure on this context (empty when none); the string
 * is owned by the context and valid until its next call. */
const char* lfdpr_last_error(lfdpr_ctx* ctx);

/* Copies a scene into device memory and builds its box mip chains on the
 * device (the "hardware mipmap" of Sec. 3.3).  *scene_id receives a handle.
 * Synchronises the stream before returning (host buffers are then free). */
int lfdpr_scene_upload(lfdpr_ctx* ctx, const lfdpr_scene_desc* desc, int32_t* scene_id);

/* Releases a scene's device memory; LFDPR_ESTATE while a live batch renders it. */
int lfdpr_scene_free(lfdpr_ctx* ctx, int32_t scene_id);

/* Materials of the physically based mode (Sec. 3.3: the shader reads albedo,
 * roughness, metallic and normal textures, each with its own LOD pair).  Three
 * host arrays of n_tris texture ids into the scene's texture list: a
 * tangent-space normal map (RGB = (n + 1)/2 * 255), a roughness map and a
 * metallic map (both read from R).  The triangle's albedo stays tex_id.  All
 * three NULL removes the materials.  Copied; synchronises the stream.
 * LFDPR_EINVAL for an unknown scene, an id >= n_tex or only some arrays;
 * LFDPR_ESTATE while a live batch renders the scene. */
int lfdpr_scene_set_materials(lfdpr_ctx* ctx, int32_t scene_id, const uint16_t* normal_id,
                              const uint16_t* roughness_id, const uint16_t* metallic_id);

/* Splat shading (Sec. 3.3: shading while the views are rendered).
 * LFDPR_SHADE_UNLIT (the default): the colour is the interpolated albedo of
 * Eq. 9.  LFDPR_SHADE_PBR: Eq. 1 takes the largest of a triangle's four
 * textures; each texture gets its LOD pair (Eqs. 6-7) and two mip fetches per
 * point; per view the four are interpolated with the same tau (Eq. 9) and
 * shaded at the cell centre with a Cook-Torrance BRDF (GGX distribution with
 * alpha = roughness^2 (roughness at least 0.03), Smith-Schlick geometry with
 * k = (roughness+1)^2/8, Schlick Fresnel with F0 = 0.04 (1-m) + albedo m,
 * diffuse (1-F)(1-m) albedo/pi) under one directional light plus ambient, then
 * tone mapped as sqrt(x/(1+x)) and rounded to 8 bits; alpha is the albedo's.
 * light_dir is the camera-space unit vector towards the light (length within
 * 1e-3 of 1); light_rgb and ambient_rgb lie in [0, 1e4].  Batches shade with
 * the context's mode too: every scene of the batch then needs materials
 * (LFDPR_ESTATE otherwise), and a batch graph is captured again when the mode
 * or the light changes. */
typedef struct {
  int32_t mode;                /* LFDPR_SHADE_* */
  float light_dir[3];
  float light_rgb[3];
  float ambient_rgb[3];
} lfdpr_shading;
int lfdpr_set_shading(lfdpr_ctx* ctx, const lfdpr_shading* shading);

/* Sets the rig and (re)allocates the per-view key buffer (8 B per pixel of
 * every rendered view, the 64-bit view buffer of Sec. 5.1) and the point
 * buffer (16 B per point).  Synchronous. */
int lfdpr_set_views(lfdpr_ctx* ctx, const lfdpr_view_params* views);

/* How the splat (Sec. 3.2) visits its (point, view, pixel) work:
 *   LFDPR_SPLAT_POINT (default)  per point, looping over the views and its
 *     splat rectangle's pixels, 64-bit atomicMin into the key buffer in HBM;
 *   LFDPR_SPLAT_TRIANGLE_VIEW  per (triangle, view): the pixels inside the
 *     triangle's projection find their owning point through the lattice row
 *     table and apply its splat rectangle and colour (unlit frames; physically
 *     shaded frames always splat per point);
 *   LFDPR_SPLAT_QUILT  per tile of the views' key space (a band of pixel rows
 *     of a subset of the views, all columns; lfdpr_set_quilt_tile): the tile's
 *     64-bit keys (Sec. 5.1) stay in LDS while the points whose splat reaches
 *     its rows are splatted into it, then it is written out as the views
 *     (unlit and physically shaded frames and batches, whose band lists
 *     hold every item's bands; lfdpr_render_frame_noalloc splats per point
 *     under this order).
 * The keys, views and depth are identical.  Applies to the context's frames
 * and to batches created on it afterwards. */
int lfdpr_set_splat_order(lfdpr_ctx* ctx, int32_t order);

/* Tile of the quilt order (the 64-bit view buffers of Sec. 5.1, a tile at a
 * time): `rows` pixel rows of `views` views, all W columns, 8 B per key in
 * LDS (plus 4 B per view column and row for the ray slopes).  0, 0 (the
 * default) chooses per rig: 4 rows, else 2, else 1, with the most views that
 * fit the device's LDS per workgroup, spread evenly over the subsets.  rows
 * and views beyond the rig are clipped to it.  Host only; returns
 * LFDPR_EINVAL for rows outside [1, 4096] or views outside [1, 1024] (unless
 * both are 0).  A shape whose keys do not fit, or a batch whose bands (items
 * x ceil(H / rows)) exceed 8192, is refused by the frame (LFDPR_EINVAL).
 * Results do not depend on it.  Batches created afterwards start from it. */
int lfdpr_set_quilt_tile(lfdpr_ctx* ctx, int32_t rows, int32_t views);

/* The tile a frame (n_items = 1) or a batch of n_items would use for views of
 * W x H pixels, n_views (sub-)views, with max_lds bytes of LDS per
 * workgroup, when rows x views is asked for (0, 0: the automatic choice
 * described above); a tile takes rows * views * W * 8 + (W + H) * 4 + 16
 * bytes.  Host only (no device, no context).  LFDPR_EINVAL when no tile fits
 * or an argument is out of range (W, H in [1, 4096], n_views in [1, 1024],
 * n_items in [1, 256]). */
int lfdpr_quilt_tile(int32_t W, int32_t H, int32_t n_views, int32_t n_items, int32_t max_lds, int32_t rows,
                     int32_t views, int32_t* out_rows, int32_t* out_views);

/* Capacity of the quilt's band lists in entries (4 B each, device memory
 * the context owns, one set per frame in flight; one entry per point and
 * band of rows its splat reaches, Sec. 3.2); 0 (the default) = twice the
 * point capacity + 65536, at most 2^32 - 1; LFDPR_EINVAL outside [0, 2^32 -
 * 1].  A frame with more entries is splatted per point into the key buffer
 * instead (same results; lfdpr_get_stats reports it).  Reallocated by the
 * next quilt frame (which synchronises then). */
int lfdpr_set_quilt_capacity(lfdpr_ctx* ctx, int64_t entries);

/* Sets the panel and reconstruction parameters used by lfdpr_reconstruct. */
int lfdpr_set_lens(lfdpr_ctx* ctx, const lfdpr_lens_params* lens);

/* Renders one frame of a scene into all V*S rendered views (Sec. 3):
 *   model      host, 12 floats, row-major 3x4 camera-from-scene transform;
 *   views_rgba device, V*S*H*W uint32 (RGBA8);
 *   depth      device, V*S*H*W float, or NULL.
 * Asynchronous.  A point-capacity overflow is reported by lfdpr_get_stats
 * (the frame's views are then incomplete).  With LFDPR_SHADE_PBR the scene
 * needs materials (LFDPR_ESTATE otherwise); the first such frame allocates
 * 64 B per triangle and 16 B per point of material buffers (synchronous). */
int lfdpr_render_frame(lfdpr_ctx* ctx, int32_t scene_id, const float* model, uint32_t* views_rgba, float* depth);

/* lfdpr_render_frame for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with every per-frame buffer
 * (triangle records, counts, offsets, points and their splat data, 64-bit
 * keys, statistics) in one 65.5 MiB array of the library's device image that
 * each GPU holds until the process ends.  This call allocates nothing.
 *   model, views_rgba, depth  as for lfdpr_render_frame;
 *   stats  device, 6 int64 (points, active triangles, point-views, overflowed
 *          triangles, written pixels, point capacity), or NULL.
 * Limits: unlit shading (LFDPR_ESTATE with LFDPR_SHADE_PBR), one frame in
 * flight (LFDPR_ESTATE otherwise), at most 65,536 triangles and V*S*H*W at
 * most 2,097,152 (LFDPR_EINVAL beyond), at most 524,288 points (more leave
 * the frame incomplete: stats[0] > stats[5]).  Asynchronous.  All calls on one
 * GPU share the array, so calls that overlap in time on one GPU (other
 * streams, other contexts) race; calls ordered on one stream do not.
 * lfdpr_get_stats / lfdpr_copy_points keep describing the last
 * lfdpr_render_frame.  LFDPR_EDEVICE when the array's address could not be
 * resolved for the device at lfdpr_create. */
int lfdpr_render_frame_noalloc(lfdpr_ctx* ctx, int32_t scene_id, const float* model, uint32_t* views_rgba,
                               float* depth, int64_t* stats);

/* Interleaves n_views views of W x H (device, [view][row][col] RGBA8) into the
 * lenticular panel (device, Hp*Wp*3 bytes) with the lens and reconstruction
 * mode of lfdpr_set_lens (Sec. 4).  Asynchronous. */
int lfdpr_reconstruct(lfdpr_ctx* ctx, const uint32_t* views_rgba, int32_t n_views, int32_t W, int32_t H,
                      uint8_t* panel_rgb);

/* Angular supersampling filter (Sec. 4): V*S sub-views (device, as rendered
 * by lfdpr_render_frame with S > 1) to V views (device, V*H*W) with Gaussian
 * weights over sub-views within one view interval.  Asynchronous. */
int lfdpr_angular_filter(lfdpr_ctx* ctx, const uint32_t* sub_views, uint32_t* views_out);

/* Statistics of the last rendered frame.  Synchronises the stream.  Returns
 * LFDPR_EOVERFLOW (with *stats filled) when the point capacity overflowed. */
int lfdpr_get_stats(lfdpr_ctx* ctx, lfdpr_stats* stats);

/* Copies the last frame's point buffer (device, 16 B per point:
 * tri | flags<<28, (u16)i | (u16)j<<16, tv_min, tv_max) into dst (device,
 * room for cap points) and its length into *n_points (host).  Synchronises. */
int lfdpr_copy_points(lfdpr_ctx* ctx, void* dst, int64_t cap, int64_t* n_points);

/* Copies the last frame's per-point material words (device, 16 B per point in
 * point order: normal-map fetch at LOD_min and at LOD_max (RGBA8), then
 * rough_min | rough_max<<8 | metal_min<<16 | metal_max<<24, then 0) into dst
 * (device, room for cap points) and the point count into *n_points (host).
 * LFDPR_ESTATE when the last frame was not shaded physically.  Synchronises. */
int lfdpr_copy_point_materials(lfdpr_ctx* ctx, void* dst, int64_t cap, int64_t* n_points);

/* Copies the last frame's per-triangle point counts (device, uint32 per
 * triangle of the scene last rendered) into dst.  Synchronises. */
int lfdpr_copy_counts(lfdpr_ctx* ctx, uint32_t* dst, int64_t n);

/* Enables (dst_f/dst_i non-NULL, device, 8 values per triangle each for up to
 * n_tris triangles) or disables (both NULL) the per-triangle set-up record
 * written by the next frames; rendering a scene with more than n_tris
 * triangles while enabled fails with LFDPR_EINVAL.  Record:
 * f = {Sx, Sy, size_min, size_max, A_ts/A_ws, n.P0, size_xy, active views},
 * i = {lattice s1, t1, s2, t2 (Q8), LOD_min, LOD_max (1/256), active, overflow}. */
int lfdpr_set_debug_records(lfdpr_ctx* ctx, float* dst_f, int32_t* dst_i, int64_t n_tris);

/* Frames in flight: 1 (the default) or 2.  With 2, render_frame runs the
 * frame's point generation (set-up, scan, emission, mip fetches) on a stream
 * of the context's own, into a second set of per-frame buffers, while the
 * previous frame's splat runs on the context's stream; the splat and the
 * resolve of each frame stay on the context's stream, ordered after that
 * frame's point generation, so the views are complete when the context's
 * stream reaches them (as with 1).  Point generation reads only the scene,
 * the model matrix (passed by value) and the rig.  It waits for the splat
 * that last read its buffers and for the work the caller enqueued on the
 * context's stream before the previous render_frame call (typically the
 * presentation of the frame before: filter, panel), so that it does not
 * compete with that work for the GPU; not for work enqueued after it (except
 * while debug records are enabled: the set-up writes those caller buffers,
 * so it then waits for all of it).  Statistics, copies and debug records refer to the
 * last frame as before.  A render_frame enqueued while a stream is being
 * captured into a hipGraph needs 1.  The second set of buffers is allocated
 * on first use (per-triangle records, point buffer, statistics).
 * Synchronises both streams. */
int lfdpr_set_frames_in_flight(lfdpr_ctx* ctx, int32_t n);

/* Stage timing with HIP events recorded on the context's stream.
 * lfdpr_timing(ctx, 1) clears and starts recording; every following
 * render_frame / reconstruct / angular_filter records one event pair per
 * stage.  lfdpr_get_timings() synchronises the stream and writes, per stage,
 * the summed milliseconds and the number of recorded launches (host arrays of
 * LFDPR_N_STAGES); stages: 0 triangle set-up, 1 scan, 2 emission, 3 splat,
 * 4 resolve, 5 interleave, 6 angular filter, 7 the quilt's band lists (quilt
 * frames; their splat stage is then the tile kernel alone).  Batch renders on
 * the context that are not replayed from a graph record their stages the same
 * way (on the batch's stream).  lfdpr_timing(ctx, 0) stops. */
#define LFDPR_N_STAGES 8
int lfdpr_timing(lfdpr_ctx* ctx, int enable);
int lfdpr_get_timings(lfdpr_ctx* ctx, double* ms_sum, int64_t* n_launches);

/* ------------------------------------------------------------------------
 * Launch shape, autotuning and batches (not part of the paper).
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t splat_blocks;  /* workgroups of the splat and fetch launches */
  int32_t key_layout;    /* 0: 64-bit keys [view][y][x]; 1: [y][view][x] (a row of every view adjacent) */
  float ms;              /* measured time of one frame (or one batch) */
  int32_t splat_order;   /* LFDPR_SPLAT_POINT or LFDPR_SPLAT_QUILT (single frames) */
  int32_t quilt_rows, quilt_views;  /* the quilt tile (0, 0 under the point order) */
} lfdpr_tune_entry;
typedef struct {
  int32_t n, best;       /* entries tried; index of the fastest (now in use) */
  lfdpr_tune_entry entries[16];
} lfdpr_tune_result;

/* Sets the splat launch shape and key layout of the context's single frames.
 * Results do not depend on them (keys are exact integers; layout only moves
 * them in memory).  Synchronises the stream. */
int lfdpr_set_launch(lfdpr_ctx* ctx, int32_t splat_blocks, int32_t key_layout);

/* Renders a scene (model: host 3x4; views: device as in lfdpr_render_frame)
 * under every candidate: the point order (or the triangle-view order, if
 * set) under each launch shape and key layout, and the quilt with bands of
 * 1, 2, 4 and 8 rows (each with the most views that fit); times each with
 * HIP events on the stream and keeps the fastest (order, shape and tile).
 * Synchronous. */
int lfdpr_autotune(lfdpr_ctx* ctx, int32_t scene_id, const float* model, uint32_t* views, lfdpr_tune_result* res);

typedef struct lfdpr_batch lfdpr_batch;

/* A batch renders n scene frames with one launch per pipeline stage over all
 * of them.  views[k] is the rig of item k (host array of n): every item must
 * have the same V*S, W, H, fovy and aspect; cones, D and jitter may differ.
 * The batch owns its key, triangle and point buffers (point_capacity points in
 * total; 0 = 32M) and a stream of its own.  The scenes stay uploaded while the
 * batch lives (lfdpr_scene_free refuses them); at most 2^28 - 1 triangles in
 * all (LFDPR_EINVAL beyond). */
int lfdpr_batch_create(lfdpr_ctx* ctx, int32_t n, const int32_t* scene_ids, const lfdpr_view_params* views,
                       int64_t point_capacity, lfdpr_batch** out);
int lfdpr_batch_destroy(lfdpr_batch* batch);
const char* lfdpr_batch_last_error(lfdpr_batch* batch);
/* 1 (default): the first lfdpr_batch_render captures the launch sequence into a
 * hipGraph and later calls with the same output pointers replay it; 0: plain
 * launches. */
int lfdpr_batch_use_graph(lfdpr_batch* batch, int enable);
/* 2: the point generation of a batch call (set-up, scan, emission; Sec. 3.1)
 * runs on a stream of the batch's own while the previous call's splat runs,
 * into a second set of generation buffers (allocated here: points, triangle
 * records, counts; as much device memory again); the splat still follows
 * earlier work on the context's stream, so results are identical.  Pipelined
 * calls launch their kernels directly (no graph).  1 (default): one set, the
 * graph replay of lfdpr_batch_use_graph.  Synchronises the batch; statistics
 * describe the last call either way.  LFDPR_EINVAL for other values,
 * LFDPR_ENOMEM (nothing changed) if the second set cannot be allocated. */
int lfdpr_batch_set_frames_in_flight(lfdpr_batch* batch, int32_t n);
/* models: host n*12 floats (row-major 3x4 per item); views: device
 * n*(V*S)*H*W uint32 RGBA8, item-major; panels: device n*Hp*Wp*3 bytes
 * interleaved with the context's lens (requires S == 1), or NULL.  Ordered
 * after earlier work on the context's stream; later work on that stream sees
 * the results. */
int lfdpr_batch_render(lfdpr_batch* batch, const float* models, uint32_t* views, uint8_t* panels);
/* Totals of the last batch frame.  Synchronous. */
int lfdpr_batch_stats(lfdpr_batch* batch, lfdpr_stats* stats);
/* The autotuner for a batch (see lfdpr_autotune).  Synchronous. */
int lfdpr_batch_autotune(lfdpr_batch* batch, const float* models, uint32_t* views, lfdpr_tune_result* res);

/* ------------------------------------------------------------------------
 * Learned angular reconstruction (a stand-in for 4x angular supersampling,
 * Sec. 4; not part of the paper).  The network is applied to every view v of
 * a frame of V views.  Its input at a pixel is (R, G, B, d = D/Z - 1; d = -1
 * where empty) of views v-2 .. v+2 (zero beyond the rig) and the disparity
 * blur of view v: with s = k*d (k from lfdpr_net_set_disparity_scale; s = 0
 * where d <= -1), the sum over t = -1, -3/4, .., 1 of w_t * view_v(x + t*s, y)
 * (linear interpolation along the row, border pixel repeated; w_t the
 * normalised weights round(65535 exp(-2 t^2)), the angular filter's profile),
 * evaluated in binary32 in that order and rounded to BF16 -- 24 channels.
 * Four zero-padded 3x3 convolutions 24 -> 32 -> 32 -> 32 -> 3 with ReLU
 * between them, dilated horizontally by 1, 3, 9, 1 (tap (dy, dx) reads pixel
 * (y+dy, x+dil*dx)), FP32 accumulation on BF16 MFMA, BF16 activations; the
 * output is the blurred RGB plus the network.  Tensors: compact input x
 * [view][H][W][4] BF16 (as written by lfdpr_net_pack_input), output y
 * [view][H][W][4] BF16 (R, G, B, 0).  Parameters: an FP32 vector, per layer W
 * [9][cout][cin] (tap 3*(dy+1)+(dx+1) reads pixel (y+dy, x+dx)) followed by
 * b [cout].  All tensors are device
 * memory unless stated; calls are asynchronous on the context's stream unless
 * stated.
 * ------------------------------------------------------------------------ */
typedef struct lfdpr_net lfdpr_net;

/* V views per frame; calls process whole frames, up to V*max_h*max_w pixels
 * in total (<= 2^26).  Parameters start at zero (output = input RGB).  The
 * network uses the context's device and stream. */
int lfdpr_net_create(lfdpr_ctx* ctx, int32_t V, int32_t max_h, int32_t max_w, lfdpr_net** out);
int lfdpr_net_destroy(lfdpr_net* net);
const char* lfdpr_net_last_error(lfdpr_net* net);
/* Number of FP32 parameters (host int64). */
int lfdpr_net_param_count(lfdpr_net* net, int64_t* n);
/* Pixels a surface at d = 1 moves across per view step: k = fx * 2 tan(cone/2) / V
 * for the rig of R2 (k >= 0; 0, the default, turns the blur into the identity).
 * Applies from the next forward. */
int lfdpr_net_set_disparity_scale(lfdpr_net* net, float k);
/* The same k computed by the library from the rig the views were rendered with
 * (R2: fx = (W/2) / (aspect tan(fovy/2)); k = fx * 2 tan(cone/2) / V, in
 * double, rounded once).  views->V must equal the network's V. */
int lfdpr_net_set_rig(lfdpr_net* net, const lfdpr_view_params* views);
/* Host FP32 parameters in / out (n must equal the count); set resets Adam.  Synchronous. */
int lfdpr_net_set_params(lfdpr_net* net, const float* host_params, int64_t n);
int lfdpr_net_get_params(lfdpr_net* net, float* host_params, int64_t n);
/* n_views views (n_views, H, W) RGBA8 and depth (same shape, FP32; NULL gives
 * d = 0, the layout of a training target) -> x [n_views][H][W][4] BF16 with
 * (R/255, G/255, B/255, D/Z - 1). */
int lfdpr_net_pack_input(lfdpr_net* net, const uint32_t* views, const float* depth, int32_t n_views, int32_t H,
                         int32_t W, float D, void* x);
/* x -> y for n_views (a multiple of V) views of H x W; keeps the activations
 * for lfdpr_net_backward. */
int lfdpr_net_forward(lfdpr_net* net, const void* x, int32_t n_views, int32_t H, int32_t W, void* y);
/* Mean-squared error of the last forward output's RGB against target (same
 * layout as y), written to *loss (device float, may be NULL), and the gradient
 * of every parameter (kept inside the network). */
int lfdpr_net_backward(lfdpr_net* net, const void* target, float* loss);
/* One Adam step on the FP32 parameters, then the BF16 copies are refreshed. */
int lfdpr_net_adam_step(lfdpr_net* net, float lr, float beta1, float beta2, float eps);
/* y -> RGBA8 views (n_views, H, W): clamp(floor(255 y + 0.5)), alpha 255. */
int lfdpr_net_unpack_output(lfdpr_net* net, const void* y, int32_t n_views, int32_t H, int32_t W, uint32_t* views);
/* Copies internal state of the last forward/backward into dst (device, n_bytes
 * room): which = 1..3 activation of hidden layer k ([view][H][W][32] BF16),
 * 4 the disparity blur of the input ([view][H][W][4] BF16, (R, G, B, 0)),
 * 11..13 gradient of hidden pre-activation k, 14 gradient of the output
 * ([view][H][W][32] BF16, channels 0..2), 20 parameter gradients (FP32).
 * Synchronous. */
int lfdpr_net_copy_state(lfdpr_net* net, int32_t which, void* dst, int64_t n_bytes);
/* Checkpoint (parameters + Adam moments + step) to / from a host file.  Synchronous. */
int lfdpr_net_save(lfdpr_net* net, const char* path);
int lfdpr_net_load(lfdpr_net* net, const char* path);

#ifdef __cplusplus
}
#endif

#endif /* LFDPR_H */
