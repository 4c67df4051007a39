// Learned angular reconstruction: a small 3x3 convolutional network whose
// inference and training run on BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32
// accumulate).  It stands in for 4x angular supersampling (Sec. 4) and is
// applied to every view v of a frame.  Angular supersampling plus the angular
// filter averages sub-views within about one view interval; a surface at
// disparity d = D/Z - 1 moves k*d pixels across per view step, so away from
// occlusions that average is a horizontal blur of width proportional to |d|.
// The input at a pixel is (R, G, B, d) of views v-2 .. v+2 (zero beyond the
// rig) and the disparity blur of view v (9 Gaussian taps over +-1 view step,
// the angular filter's profile): 24 channels; layers 24 -> 32 -> 32 -> 32 -> 3
// with ReLU, 3x3 kernels dilated horizontally by 1, 3, 9, 1; output = blurred
// RGB + network.
//
// Layouts: the compact input is [view][H][W][4] BF16 and layer 1 gathers the
// neighbour views from it directly, and the blur from its own [view][H][W][4]
// buffer; hidden activations are [view][H][W][32]
// BF16; the output [view][H][W][4] (RGB, 0).  Parameters: FP32 master vector,
// per layer W [tap][cout][cin] then b [cout] (unpadded); BF16 copies padded
// to 32 input channels (layer 1) and 16 output channels (layer 4).
//
// MFMA 16x16x32 lane layout used throughout: lane l feeds row (l % 16) of A
// and column (l % 16) of B with 8 K-values each (group l / 16); the 4 results
// of lane l are D[4*(l/16) + e][l % 16].  A and B take their K-values in the
// same order, so the K ordering inside a group does not matter.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lfdpr.h"
#include "lfdpr_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace lfdpr {
namespace net {

constexpr int kHidden = 32;
enum Mode { MODE_RELU = 0, MODE_OUT = 1, MODE_BWD = 2 };

__device__ __forceinline__ uint16_t to_bf16(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// Two values rounded to BF16 (nearest, ties to even) by one v_cvt_pk_bf16_f32,
// lo in bits 0-15.  For every non-NaN binary32 input it gives the same bits as
// to_bf16 (checked exhaustively on gfx950).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}

union Frag {
  uint4 u;
  bf16x8 v;
};

// ---------------------------------------------------------------- 3x3 convolution
constexpr int kNeigh = 2;   // views v-2 .. v+2
constexpr int kViewCh = 4 * (2 * kNeigh + 1);  // 20 channels of the five views
constexpr int kCin0 = kViewCh + 4;             // + blurred (R, G, B, 0) of view v
constexpr int kK = 32;      // padded input channels of every layer (one MFMA K step per tap)
// Horizontal dilation per layer: one view step shifts content by several
// pixels across, so the stack sees +-14 px horizontally and +-4 px vertically.
constexpr int kDilation[4] = {1, 3, 9, 1};

// Loads the 8 K-values of lane group g for input pixel (n, yy, xx), zero
// outside the image.  GATHER: from the compact [n][H][W][4] input, channels
// 8g..8g+7 = views n+2g-2, n+2g-1; the slot after view n+2 (channels 20..23)
// takes the blur XB of view n.  Pixel indices fit in 32 bits: a network holds
// at most 2^26 pixels.
template <bool GATHER>
__device__ __forceinline__ uint4 load_a(const uint16_t* __restrict__ X, const uint16_t* __restrict__ XB, int n, int yy,
                                        int xx, int H, int W, int g, int V) {
  if (yy < 0 || yy >= H || xx < 0 || xx >= W) return uint4{0u, 0u, 0u, 0u};
  if (!GATHER) return *reinterpret_cast<const uint4*>(X + (size_t)((n * H + yy) * W + xx) * kK + 8 * g);
  const int v = n % V, f0 = n - v;
  uint2 lo = {0u, 0u}, hi = {0u, 0u};
  const int o0 = 2 * g - kNeigh, o1 = 2 * g + 1 - kNeigh;
  if (o0 <= kNeigh && v + o0 >= 0 && v + o0 < V)
    lo = *reinterpret_cast<const uint2*>(X + (size_t)(((f0 + v + o0) * H + yy) * W + xx) * 4);
  if (o1 <= kNeigh) {
    if (v + o1 >= 0 && v + o1 < V)
      hi = *reinterpret_cast<const uint2*>(X + (size_t)(((f0 + v + o1) * H + yy) * W + xx) * 4);
  } else if (o1 == kNeigh + 1) {
    hi = *reinterpret_cast<const uint2*>(XB + (size_t)((n * H + yy) * W + xx) * 4);
  }
  return uint4{lo.x, lo.y, hi.x, hi.y};
}

// One block = 4 waves, persistent over output tiles of kTY rows x kTX pixels of
// one image (wave w computes row w: four 16-pixel M tiles); NT = COUT/16
// output-channel tiles.  All nine taps' [COUT][32] weights stay in LDS; each
// tile's input, rows y0-1 .. y0+kTY and columns x0-DIL .. x0+kTX-1+DIL with
// zero padding, is staged in LDS once and read by all nine taps.  LDS rows of
// 32 channels are four 16-byte groups stored at slot g ^ ((px >> 1) & 3): LDS
// serves 16-byte reads eight lanes (128 bytes) at a time, and any 8
// consecutive pixels then fall into 8 distinct bank groups (no conflicts on
// gfx950 by the SQ_LDS_BANK_CONFLICT counter).  aux: GATHER, the blur buffer;
// MODE_OUT, the residual (stride AUX_C); MODE_BWD, the activation whose ReLU
// masks the gradient.
constexpr int kTX = 64, kTY = 4;
constexpr int kMaxDil = 9;  // the staging registers are sized for it
static_assert(kDilation[0] <= kMaxDil && kDilation[1] <= kMaxDil && kDilation[2] <= kMaxDil &&
                  kDilation[3] <= kMaxDil,
              "dilation beyond the staged halo");
constexpr int kStagePerThread = ((kTY + 2) * (kTX + 2 * kMaxDil) * 4 + 255) / 256;
constexpr int kPlanes = 2 * kNeigh + 2;  // layer 1's sources: five views and the blur
constexpr int kGatherPerThread = ((kTY + 2) * (kTX / 2 + kMaxDil + 1) * kPlanes + 255) / 256;  // pixel pairs

__device__ __forceinline__ int swz(int row, int g) { return row * 4 + (g ^ ((row >> 1) & 3)); }

template <int NT>
constexpr size_t conv_lds_bytes(int dil) {
  return (size_t)9 * NT * 16 * 4 * 16 + (size_t)(kTY + 2) * (kTX + 2 * dil) * 4 * 16;
}

template <int NT, int MODE, bool GATHER>
__global__ void __launch_bounds__(256) k_conv3x3(const uint16_t* __restrict__ X, const uint16_t* __restrict__ Wt,
                                                  const float* __restrict__ bias, int N, int H, int W, int V, int DIL,
                                                  uint16_t* __restrict__ Y, int YS, const uint16_t* __restrict__ aux,
                                                  int AUX_C) {
  constexpr int COUT = NT * 16;
  extern __shared__ uint4 smem[];
  uint4* wlds = smem;                  // [9 * COUT rows][4 groups]
  uint4* tl = smem + 9 * COUT * 4;     // [(kTY + 2) rows][TW pixels][4 groups]
  const int TW = kTX + 2 * DIL;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  for (int k = threadIdx.x; k < 9 * COUT * 4; k += blockDim.x)
    wlds[swz(k >> 2, k & 3)] = reinterpret_cast<const uint4*>(Wt)[k];
  // Loads whose results the epilogue uses are unconditional (clamped indices):
  // a load issued under a branch leaves the compiler unsure that a later wait
  // covered it, and it would then wait for all memory traffic in the epilogue.
  // The MFMA computes D = W x A (rows: output channels, columns: pixels), so
  // lane (g, r16) ends with channels t*16 + 4g .. +3 of pixel r16 of each M tile.
  float bco[NT][4];  // their biases (3 in the output layer)
  const int nbias = MODE == MODE_BWD ? 0 : (MODE == MODE_OUT ? 3 : YS);
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = t * 16 + 4 * g + e;
      if (MODE == MODE_BWD) {
        bco[t][e] = 0.0f;
      } else {
        const float bv = bias[c < nbias ? c : 0];
        bco[t][e] = c < nbias ? bv : 0.0f;
      }
    }
  const int tiles_x = (W + kTX - 1) / kTX, tiles_y = (H + kTY - 1) / kTY;
  const int ntile = N * tiles_x * tiles_y;
  const int nstage = (kTY + 2) * TW * 4;  // <= kStagePerThread * 256 for DIL <= kMaxDil
  // Tile order.  Image-major ([n][row band][column]), except for the gathering
  // first layer: position-major with the view fastest, so the five output views
  // that read one input view's tile follow each other.  Workgroups are handed to
  // the 8 XCDs round robin and each XCD has its own L2, so the blocks of XCD c
  // (blockIdx % 8 == c) take the c-th eighth of that order, in order: tiles that
  // share halo rows and columns (or input views) then run at about the same time
  // on the XCD that caches them.  Any other grid takes tiles blockIdx + k*grid.
  const bool by_xcd = gridDim.x % 8 == 0 && ntile >= (int)gridDim.x;
  const int xc = blockIdx.x % 8;
  const int t_end = by_xcd ? (int)((int64_t)ntile * (xc + 1) / 8) : ntile;
  const int t_first = by_xcd ? (int)((int64_t)ntile * xc / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  const int t_step = by_xcd ? (int)(gridDim.x / 8) : (int)gridDim.x;
  auto decode = [&](int tile, int& n, int& y0, int& x0) {
    int pos;
    if (GATHER) {
      n = tile % N;
      pos = tile / N;
    } else {
      n = tile / (tiles_x * tiles_y);
      pos = tile % (tiles_x * tiles_y);
    }
    y0 = (pos / tiles_x) * kTY;
    x0 = (pos % tiles_x) * kTX;
  };
  // Staging items of this thread, the same for every tile.  Layers 2-4: item j
  // is 16-byte group threadIdx % 4 of LDS pixel q = threadIdx / 4 + 64 j, at
  // tile row q / TW and column q % TW (rows from kTY + 2 on lie past the staged
  // tile).  Layer 1 (GATHER) stages plane by plane -- views v-2 .. v+2 of the
  // compact input, then the blur, 8 bytes per pixel -- in pairs of pixels from
  // an even column xs = x0 - DIL - (DIL & 1), so each wave load reads 128
  // consecutive pixels of one plane (16 bytes a lane where the pair is inside
  // the image and 16-byte aligned, else two 8-byte loads): item j' = threadIdx
  // + 256 j is plane j' / ((kTY + 2) NP), then row and pair (NP pairs a row);
  // plane p fills half p % 2 of group p / 2, pixels outside the tile's columns
  // are dropped, and group 3 (channels 24-31) stays zero.
  constexpr int kSlots = GATHER ? kGatherPerThread : kStagePerThread;
  const int NP = kTX / 2 + DIL + (DIL & 1);  // pixel pairs per staged row (layer 1)
  int geo[kSlots];
#pragma unroll
  for (int j = 0; j < kSlots; ++j) {
    if (GATHER) {
      const int i = (int)threadIdx.x + 256 * j, m = (kTY + 2) * NP;
      const int pl = i / m, rem = i % m;
      geo[j] = (pl << 24) | ((rem / NP) << 16) | (rem % NP);
    } else {
      const int q = (int)(threadIdx.x >> 2) + 64 * j;
      geo[j] = ((q / TW) << 16) | (q % TW);
    }
  }
  const int sg = threadIdx.x & 3;
  if (GATHER) {  // the zero group: the whole tile once, before any staging
    for (int k = threadIdx.x; k < nstage; k += blockDim.x) tl[k] = uint4{0u, 0u, 0u, 0u};
    __syncthreads();
  }
  // the next tile's input is fetched into registers while this one computes
  uint4 pre[kSlots];
  auto fetch = [&](int tile) {
    int n, y0, x0;
    decode(tile, n, y0, x0);
    if constexpr (GATHER) {
      const int vv = n % V, f0 = n - vv;
      const int xs = x0 - DIL - (DIL & 1);
#pragma unroll
      for (int j = 0; j < kSlots; ++j) {
        const int pl = geo[j] >> 24, r = (geo[j] >> 16) & 0xFF, q = geo[j] & 0xFFFF;
        const int yy = y0 - 1 + r, xx = xs + 2 * q;
        uint4 val = {0u, 0u, 0u, 0u};
        const int vo = vv + pl - kNeigh;
        const bool plane_ok = pl < kPlanes - 1 ? (vo >= 0 && vo < V) : pl == kPlanes - 1;
        if (plane_ok && yy >= 0 && yy < H) {
          const uint16_t* src = pl < kPlanes - 1 ? X : aux;
          const int img = pl < kPlanes - 1 ? f0 + vo : n;
          const bool ok0 = xx >= 0 && xx < W, ok1 = xx + 1 >= 0 && xx + 1 < W;
          const int p0 = (img * H + yy) * W + xx;  // dereferenced only where in the image
          const uint16_t* a0 = src + (size_t)p0 * 4;
          if (ok0 && ok1 && ((uintptr_t)a0 & 15) == 0) {
            val = *reinterpret_cast<const uint4*>(a0);
          } else {
            if (ok0) {
              const uint2 a = *reinterpret_cast<const uint2*>(src + (size_t)p0 * 4);
              val.x = a.x;
              val.y = a.y;
            }
            if (ok1) {
              const uint2 b = *reinterpret_cast<const uint2*>(src + (size_t)(p0 + 1) * 4);
              val.z = b.x;
              val.w = b.y;
            }
          }
        }
        pre[j] = val;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kSlots; ++j) {
        const int r = geo[j] >> 16, c = geo[j] & 0xFFFF;
        pre[j] = r < kTY + 2 ? load_a<false>(X, nullptr, n, y0 - 1 + r, x0 - DIL + c, H, W, sg, V) : uint4{0u, 0u, 0u, 0u};
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
      if constexpr (GATHER) {
        const int pl = geo[j] >> 24, r = (geo[j] >> 16) & 0xFF, q = geo[j] & 0xFFFF;
        const int c0 = 2 * q - (DIL & 1);  // tile column of the pair's first pixel
        if (pl < kPlanes) {
          if (c0 >= 0) reinterpret_cast<uint2*>(&tl[swz(r * TW + c0, pl >> 1)])[pl & 1] = uint2{pre[j].x, pre[j].y};
          if (c0 + 1 < TW)
            reinterpret_cast<uint2*>(&tl[swz(r * TW + c0 + 1, pl >> 1)])[pl & 1] = uint2{pre[j].z, pre[j].w};
        }
      } else {
        const int k = threadIdx.x + j * 256;
        if (k < nstage) tl[swz(k >> 2, k & 3)] = pre[j];
      }
    }
  };
  // Software pipeline per tile: MFMAs on the staged tile; then the next tile
  // (already in registers) goes to LDS, the one after it is requested, and only
  // then do this tile's results leave.  Vector-memory waits count stores as well
  // as loads, so each wait (before staging) covers requests that have had a
  // whole tile of MFMAs to complete, never the stores just issued.
  if (t_first < t_end) {
    fetch(t_first);
    stage();
    __syncthreads();  // weights and the first tile in LDS
    if (t_first + t_step < t_end) fetch(t_first + t_step);
  }
  for (int tile = t_first; tile < t_end; tile += t_step) {
    int n, y0, x0;
    decode(tile, n, y0, x0);
    const int y = y0 + wv;
    // the epilogue's side input (residual or ReLU mask), clamped into the image
    // and used only where in range: the residual is requested before the MFMAs;
    // the mask (two 32-channel tiles) after them, which keeps the backward
    // instantiation at three waves per SIMD
    uint2 side[4][NT];
    auto load_side = [&]() {
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int x = min(x0 + m * 16 + r16, W - 1), yc = min(y, H - 1), c0 = t * 16 + 4 * g;
          side[m][t] = *reinterpret_cast<const uint2*>(aux + (((size_t)n * H + yc) * W + x) * AUX_C +
                                                       (c0 < YS ? c0 : 0));
        }
    };
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) side[m][t] = uint2{0u, 0u};
    if (MODE == MODE_OUT) load_side();
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // all nine taps unrolled: in a rolled loop the compiler moves the
    // accumulators between AGPRs on every iteration (about 40 moves per 8 MFMAs)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      Frag b[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) b[t].u = wlds[swz(tap * COUT + t * 16 + r16, g)];
      const int rowbase = (wv + 1 + dy) * TW + DIL + dx * DIL + r16;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        Frag a;
        a.u = tl[swz(rowbase + m * 16, g)];
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[t].v, a.v, acc[m][t], 0, 0, 0);
      }
    }
    if (MODE == MODE_BWD) load_side();
    const int next = tile + t_step;
    __syncthreads();  // every wave has finished reading this tile
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) on every path: all requests so far have landed
    if (next < t_end) stage();
    __syncthreads();
    if (next + t_step < t_end) fetch(next + t_step);
    // epilogue: lane holds D[4g+e][r16] = channel t*16 + 4g + e of pixel x0 + 16m + r16
    // (row y0 + wv); four consecutive channels leave as one 8-byte store
    if (y < H) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int x = x0 + m * 16 + r16;
        if (x >= W) continue;
        const size_t p = ((size_t)n * H + y) * W + x;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int c0 = t * 16 + 4 * g;
          if (c0 >= YS) continue;
          float v[4];
          const uint16_t sh[4] = {(uint16_t)(side[m][t].x & 0xFFFFu), (uint16_t)(side[m][t].x >> 16),
                                  (uint16_t)(side[m][t].y & 0xFFFFu), (uint16_t)(side[m][t].y >> 16)};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int co = c0 + e;
            float u = acc[m][t][e];
            if (MODE == MODE_RELU) {
              u = fmaxf(u + bco[t][e], 0.0f);
            } else if (MODE == MODE_OUT) {
              u = co < 3 ? (u + bco[t][e]) + from_bf16(sh[e]) : 0.0f;
            } else {
              u = from_bf16(sh[e]) > 0.0f ? u : 0.0f;
            }
            v[e] = u;
          }
          uint2 o;
          o.x = pack_bf16x2(v[0], v[1]);
          o.y = pack_bf16x2(v[2], v[3]);
          *reinterpret_cast<uint2*>(Y + p * YS + c0) = o;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- weight gradient
// dW[tap][co][ci] = sum_p dZ[p][co] * A[p + off(tap)][ci].  A block owns a
// chunk of pixels; 256 of them at a time it stages dZ, and for each tap the
// shifted activations, in LDS channel-major (rows of 256 pixels padded by 16
// bytes, so the 8 lanes of a 128-byte read group hit distinct banks); wave w
// then reduces its (co tile w/2, ci tile w%2) over the pixels with one MFMA
// per 32 pixels (M = co, N = ci, K = pixels).  Each block writes its sums to
// its own row of a partials buffer, which k_sum_partials adds in block order.
constexpr int kWgPix = 256;
constexpr int kMaxGradBlocks = 1024;  // blocks of one gradient sum (partials buffer rows)
constexpr int kWgPitch = kWgPix + 8;  // bf16 per LDS row

__device__ __forceinline__ void put_cols(uint16_t* T, int col, const uint4 (&v)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t w[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      T[(8 * q + 2 * h) * kWgPitch + col] = (uint16_t)(w[h] & 0xFFFFu);
      T[(8 * q + 2 * h + 1) * kWgPitch + col] = (uint16_t)(w[h] >> 16);
    }
  }
}

template <bool GATHER>
__global__ void __launch_bounds__(256) k_conv_wgrad(const uint16_t* __restrict__ dZ, int CO,
                                                     const uint16_t* __restrict__ A, const uint16_t* __restrict__ AB,
                                                     int CI, int N, int H, int W, int V, int DIL,
                                                     float* __restrict__ dW, int chunk) {
  __shared__ uint16_t dzT[kK * kWgPitch];
  __shared__ uint16_t aT[kK * kWgPitch];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int ct = wv >> 1, it = wv & 1;
  const bool active = ct * 16 < CO && it * 16 < CI;  // wave-uniform
  const int hw = H * W, npx = N * hw;
  const int c0 = blockIdx.x * chunk, c1 = min(npx, c0 + chunk);
  f32x4 acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int base = c0; base < c1; base += kWgPix) {
    const int p = base + (int)threadIdx.x;
    const bool pv = p < c1;
    const int n = pv ? p / hw : 0, q = pv ? p % hw : 0;
    const int y = q / W, x = q % W;
    __syncthreads();  // the previous chunk's reads are done
    {
      uint4 v[4] = {};
      if (pv) {
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) v[c4] = reinterpret_cast<const uint4*>(dZ + (size_t)p * kK)[c4];
      }
      put_cols(dzT, threadIdx.x, v);
    }
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {  // unrolled: acc[tap] stays in registers
      const int yy = y + tap / 3 - 1, xx = x + (tap % 3 - 1) * DIL;
      uint4 v[4] = {};
      if (pv) {
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) v[c4] = load_a<GATHER>(A, AB, n, yy, xx, H, W, c4, V);
      }
      __syncthreads();  // the previous tap's reads of aT are done
      put_cols(aT, threadIdx.x, v);
      __syncthreads();
      if (active) {
#pragma unroll
        for (int k = 0; k < kWgPix / 32; ++k) {
          Frag fa, fb;
          fa.u = *reinterpret_cast<const uint4*>(&dzT[(ct * 16 + r16) * kWgPitch + k * 32 + 8 * g]);
          fb.u = *reinterpret_cast<const uint4*>(&aT[(it * 16 + r16) * kWgPitch + k * 32 + 8 * g]);
          acc[tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa.v, fb.v, acc[tap], 0, 0, 0);
        }
      }
    }
  }
  // lane holds D[4g+e][r16]: co = ct*16 + 4g + e, ci = it*16 + r16
  if (active) {
    const int ci = it * 16 + r16;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int co = ct * 16 + 4 * g + e;
        if (co < CO && ci < CI) dW[(size_t)blockIdx.x * 9 * CO * CI + ((size_t)tap * CO + co) * CI + ci] = acc[tap][e];
      }
  }
}

__global__ void __launch_bounds__(256) k_bias_grad(const uint16_t* __restrict__ dZ, int CO, int npx, int chunk,
                                                    float* __restrict__ db) {
  // db[block][c] = sum over the block's pixels of dZ[p][c] (dZ [p][32] BF16):
  // thread t adds channels 8(t % 4) .. +7 of pixels t / 4, t / 4 + 64, .. from
  // 16-byte loads; the 64 partial sums of each channel meet in LDS
  __shared__ float red[8][256];
  const int g = threadIdx.x & 3, q = threadIdx.x >> 2;
  const int p0 = blockIdx.x * chunk, p1 = min(npx, p0 + chunk);
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int p = p0 + q; p < p1; p += 64) {
    const uint4 v = *reinterpret_cast<const uint4*>(dZ + (size_t)p * kK + 8 * g);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      acc[2 * h] += from_bf16((uint16_t)(w[h] & 0xFFFFu));
      acc[2 * h + 1] += from_bf16((uint16_t)(w[h] >> 16));
    }
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) red[e][threadIdx.x] = acc[e];
  __syncthreads();
  if ((int)threadIdx.x < CO) {
    const int c = threadIdx.x, gg = c >> 3, e = c & 7;
    float sum = 0.0f;
    for (int k = 0; k < 64; ++k) sum += red[e][gg + 4 * k];
    db[(size_t)blockIdx.x * CO + c] = sum;
  }
}

// out[i] = sum over the nblk rows of part[b][i] in a fixed order, so gradients
// come out the same on every run (no atomics in their sums): in a block of 256,
// lane (phase f = t / 16, column j = t % 16) adds rows f, f + 16, .. in
// ascending order, then the 16 phase sums of each column are added in phase
// order.  Grid: ceil(n / 16) blocks.
__global__ void __launch_bounds__(256) k_sum_partials(const float* __restrict__ part, int nblk, int n,
                                                       float* __restrict__ out) {
  __shared__ float red[16][17];
  const int j = threadIdx.x & 15, f = threadIdx.x >> 4;
  const int i = blockIdx.x * 16 + j;
  float sum = 0.0f;
  if (i < n) {
#pragma unroll 8
    for (int b = f; b < nblk; b += 16) sum += part[(size_t)b * n + i];
  }
  red[f][j] = sum;
  __syncthreads();
  if (f == 0 && i < n) {
    float total = 0.0f;
    for (int k = 0; k < 16; ++k) total += red[k][j];
    out[i] = total;
  }
}

// loss = mean((y - t)^2) over the 3 colour channels of npx pixels (inputs
// [p][4]); dZ = bf16(2 (y - t) / n) into a [p][32] buffer (other channels 0),
// one pixel (four 16-byte stores) per thread.  Grid-stride, one loss atomic per
// block.
__global__ void __launch_bounds__(256) k_mse(const uint16_t* __restrict__ Yb, const uint16_t* __restrict__ T, int npx,
                                              uint16_t* __restrict__ dZ, float* __restrict__ loss) {
  const int64_t n = (int64_t)npx * 3;
  float sq = 0.0f;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (int64_t)gridDim.x * blockDim.x) {
    const uint2 yv = *reinterpret_cast<const uint2*>(Yb + p * 4);
    const uint2 tv = *reinterpret_cast<const uint2*>(T + p * 4);
    const float d0 = from_bf16((uint16_t)(yv.x & 0xFFFFu)) - from_bf16((uint16_t)(tv.x & 0xFFFFu));
    const float d1 = from_bf16((uint16_t)(yv.x >> 16)) - from_bf16((uint16_t)(tv.x >> 16));
    const float d2 = from_bf16((uint16_t)(yv.y & 0xFFFFu)) - from_bf16((uint16_t)(tv.y & 0xFFFFu));
    sq += d0 * d0;
    sq += d1 * d1;
    sq += d2 * d2;
    uint4* out = reinterpret_cast<uint4*>(dZ + p * kK);
    out[0] = uint4{(uint32_t)to_bf16((2.0f * d0) / (float)n) | ((uint32_t)to_bf16((2.0f * d1) / (float)n) << 16),
                   (uint32_t)to_bf16((2.0f * d2) / (float)n), 0u, 0u};
    out[1] = uint4{0u, 0u, 0u, 0u};
    out[2] = uint4{0u, 0u, 0u, 0u};
    out[3] = uint4{0u, 0u, 0u, 0u};
  }
  __shared__ float red[256];
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) atomicAdd(loss, red[0] / (float)n);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 weights for the forward pass ([tap][cof][32], zero-padded from the
// master [tap][co][ci]) and the flipped, transposed copy for the input
// gradient ([8 - tap][ci][32], zero beyond co).
__global__ void k_pack_w(const float* __restrict__ master, int CO, int CI, int COF, uint16_t* __restrict__ wf,
                         uint16_t* __restrict__ wb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)9 * COF * kK) {
    const int tap = (int)(i / (COF * kK)), rem = (int)(i % (COF * kK));
    const int co = rem / kK, ci = rem % kK;
    wf[i] = (co < CO && ci < CI) ? to_bf16(master[((int64_t)tap * CO + co) * CI + ci]) : (uint16_t)0;
  }
  if (wb && i < (int64_t)9 * CI * kK) {
    const int tapb = (int)(i / (CI * kK)), rem = (int)(i % (CI * kK));
    const int ci = rem / kK, co = rem % kK;
    wb[i] = co < CO ? to_bf16(master[((int64_t)(8 - tapb) * CO + co) * CI + ci]) : (uint16_t)0;
  }
}

// views (V, H, W) RGBA8 + depth -> x[v][p][4] = (R/255, G/255, B/255, D/Z - 1), d = -1 when empty
__global__ void k_pack_input(const uint32_t* __restrict__ views, const float* __restrict__ depth, int64_t n, float D,
                             uint16_t* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = views[i];
  const float z = depth ? depth[i] : INFINITY;
  const float d = z < INFINITY ? D / z - 1.0f : -1.0f;
  uint2 o;
  o.x = (uint32_t)to_bf16((float)(c & 255u) / 255.0f) | ((uint32_t)to_bf16((float)((c >> 8) & 255u) / 255.0f) << 16);
  o.y = (uint32_t)to_bf16((float)((c >> 16) & 255u) / 255.0f) | ((uint32_t)(depth ? to_bf16(d) : 0u) << 16);
  reinterpret_cast<uint2*>(x)[i] = o;
}

// Disparity blur of each view (the binary32 steps are fixed, so the result is
// reproducible bit for bit): per pixel, s = k*d (0 where d <= -1, empty); for
// tap t = -1, -3/4, .., 1: u = min(max(x + t*s, -1), W), x0 = floor(u),
// f = u - x0, c = (1 - f)*C[x0] + f*C[x0 + 1] (indices clamped to the row),
// acc += w_t*c; XB = (bf16(acc_R), bf16(acc_G), bf16(acc_B), 0).
struct BlurTaps {
  float w[9];
};

// One output pixel of the blur; px(i) returns input pixel i of the row.
template <typename RowPx>
__device__ __forceinline__ uint2 blur_pixel(RowPx px, int x, int W, float k, const BlurTaps& bw) {
  const float d = from_bf16((uint16_t)(px(x).y >> 16));
  const float s = d > -1.0f ? k * d : 0.0f;
  float acc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const float t = (float)(j - 4) * 0.25f;
    float u = (float)x + t * s;
    u = fminf(fmaxf(u, -1.0f), (float)W);
    const float fl = floorf(u);
    const float f = u - fl;
    const int i0 = (int)fl;
    const int a = min(max(i0, 0), W - 1), b = min(max(i0 + 1, 0), W - 1);
    const uint2 ca = px(a);
    const uint2 cb = px(b);
    const float g = 1.0f - f;
    const float a0 = from_bf16((uint16_t)(ca.x & 0xFFFFu)), a1 = from_bf16((uint16_t)(ca.x >> 16)),
                a2 = from_bf16((uint16_t)(ca.y & 0xFFFFu));
    const float b0 = from_bf16((uint16_t)(cb.x & 0xFFFFu)), b1 = from_bf16((uint16_t)(cb.x >> 16)),
                b2 = from_bf16((uint16_t)(cb.y & 0xFFFFu));
    acc[0] = acc[0] + bw.w[j] * (g * a0 + f * b0);
    acc[1] = acc[1] + bw.w[j] * (g * a1 + f * b1);
    acc[2] = acc[2] + bw.w[j] * (g * a2 + f * b2);
  }
  uint2 o;
  o.x = pack_bf16x2(acc[0], acc[1]);
  o.y = pack_bf16x2(acc[2], 0.0f);
  return o;
}

// Rows of up to kBlurRowMax pixels: a block stages a whole row (8 bytes per
// pixel) in LDS with coalesced loads, and every tap is gathered from there.
constexpr int kBlurRowMax = 4096;

__global__ void __launch_bounds__(256) k_disparity_blur_rows(const uint16_t* __restrict__ X, int64_t nrows, int W,
                                                              float k, BlurTaps bw, uint16_t* __restrict__ XB) {
  extern __shared__ uint2 lrow[];  // W pixels
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const uint2* src = reinterpret_cast<const uint2*>(X) + r * W;
    __syncthreads();  // the previous row's gathers are finished
    for (int i = threadIdx.x; i < W; i += blockDim.x) lrow[i] = src[i];
    __syncthreads();
    uint2* dst = reinterpret_cast<uint2*>(XB) + r * W;
    for (int x = threadIdx.x; x < W; x += blockDim.x)
      dst[x] = blur_pixel([&](int i) { return lrow[i]; }, x, W, k, bw);
  }
}

// Wider rows: one thread per pixel, taps gathered from global memory.
__global__ void __launch_bounds__(256) k_disparity_blur(const uint16_t* __restrict__ X, int64_t npx, int W, float k,
                                                         BlurTaps bw, uint16_t* __restrict__ XB) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npx) return;
  const int x = (int)(p % W);
  const uint2* row = reinterpret_cast<const uint2*>(X) + (p - x);
  reinterpret_cast<uint2*>(XB)[p] = blur_pixel([&](int i) { return row[i]; }, x, W, k, bw);
}

// y[v][p][4] -> RGBA8, clamp(floor(255 y + 0.5)), alpha 255
__global__ void k_unpack_output(const uint16_t* __restrict__ y, int64_t n, uint32_t* __restrict__ views) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t o = 0xFF000000u;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float f = floorf(from_bf16(y[i * 4 + c]) * 255.0f + 0.5f);
    f = f < 0.0f ? 0.0f : (f > 255.0f ? 255.0f : f);
    o |= (uint32_t)f << (8 * c);
  }
  views[i] = o;
}

__global__ void k_zero_f32(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

}  // namespace net
}  // namespace lfdpr

using namespace lfdpr;
using namespace lfdpr::net;

struct lfdpr_net {
  lfdpr_ctx* ctx = nullptr;
  bool counted = false;  // registered as a child of ctx
  hipStream_t stream = nullptr;
  int device = 0;
  int V = 0;
  int64_t maxpx = 0;  // views * H * W
  int ci[4], co[4], cof[4];
  int64_t off_w[4], off_b[4], nparams = 0;
  float* master = nullptr;
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  int64_t step = 0;
  uint16_t* wf[4] = {nullptr, nullptr, nullptr, nullptr};
  uint16_t* wb[4] = {nullptr, nullptr, nullptr, nullptr};
  uint16_t* act[4] = {nullptr, nullptr, nullptr, nullptr};  // act[1..3]
  uint16_t* dz[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  uint16_t* xb = nullptr;  // disparity blur of the last forward input, [view][H][W][4]
  float kscale = 0.0f;     // pixels per view step per unit d
  BlurTaps taps{};
  const uint16_t* last_x = nullptr;
  const uint16_t* last_y = nullptr;
  int last_n = 0, last_h = 0, last_w = 0;
  float* d_loss = nullptr;
  float* part = nullptr;   // per-block partial gradients: kMaxGradBlocks x (9*32*32 + 32)
  std::string err;
};

namespace {

int nfail(lfdpr_net* n, int code, const std::string& m) {
  if (n) n->err = m;
  return code;
}

#define NHIP(call)                                                                                    \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess) return nfail(net, LFDPR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <int NT, int MODE, bool GATHER>
void launch_conv(const uint16_t* X, const uint16_t* Wt, const float* b, int N, int H, int W, int V, int dil,
                 uint16_t* Y, int YS, const uint16_t* aux, int AUXC, hipStream_t s) {
  const int64_t tiles = (int64_t)N * ((H + kTY - 1) / kTY) * ((W + kTX - 1) / kTX);
  const int grid = (int)(tiles < 768 ? tiles : 768);  // persistent: about three blocks per CU
  k_conv3x3<NT, MODE, GATHER><<<grid, 256, conv_lds_bytes<NT>(dil), s>>>(X, Wt, b, N, H, W, V, dil, Y, YS, aux, AUXC);
}

void pack_weights(lfdpr_net* net) {
  for (int k = 0; k < 4; ++k) {
    const int64_t n = 9ll * kK * (net->cof[k] > net->ci[k] ? net->cof[k] : net->ci[k]);
    k_pack_w<<<(unsigned)((n + 255) / 256), 256, 0, net->stream>>>(net->master + net->off_w[k], net->co[k], net->ci[k],
                                                                   net->cof[k], net->wf[k], net->wb[k]);
  }
}

}  // namespace

extern "C" {

int lfdpr_net_create(lfdpr_ctx* ctx, int32_t V, int32_t max_h, int32_t max_w, lfdpr_net** out) {
  if (!ctx || !out) return LFDPR_EINVAL;
  *out = nullptr;
  if (V < 1 || V > 4096 || max_h < 1 || max_w < 1 || (int64_t)V * max_h * max_w > (1ll << 26)) return LFDPR_EINVAL;
  lfdpr_net* net = new lfdpr_net();
  net->ctx = ctx;
  net->stream = ctx_stream_of(ctx);
  net->device = ctx_device_of(ctx);
  net->V = V;
  net->maxpx = (int64_t)V * max_h * max_w;
  const int ci[4] = {kCin0, kHidden, kHidden, kHidden}, co[4] = {kHidden, kHidden, kHidden, 3};
  int64_t off = 0;
  for (int k = 0; k < 4; ++k) {
    net->ci[k] = ci[k];
    net->co[k] = co[k];
    net->cof[k] = k == 3 ? 16 : kHidden;
    net->off_w[k] = off;
    off += 9ll * co[k] * ci[k];
    net->off_b[k] = off;
    off += co[k];
  }
  net->nparams = off;
  bool ok = hipSetDevice(net->device) == hipSuccess;
  auto al = [&](auto*& p, size_t n) { if (ok) ok = hipMalloc((void**)&p, n * sizeof(*p)) == hipSuccess; };
  al(net->master, off);
  al(net->grad, off);
  al(net->adam_m, off);
  al(net->adam_v, off);
  al(net->d_loss, 1);
  al(net->part, (size_t)kMaxGradBlocks * (9 * kHidden * kHidden + kHidden));
  for (int k = 0; k < 4; ++k) {
    al(net->wf[k], 9ll * net->cof[k] * kK);
    if (k > 0) al(net->wb[k], 9ll * ci[k] * kK);
    if (k > 0) al(net->act[k], (size_t)net->maxpx * kHidden);
  }
  for (int k = 1; k <= 4; ++k) al(net->dz[k], (size_t)net->maxpx * kK);
  al(net->xb, (size_t)net->maxpx * 4);
  {  // the angular filter's Gaussian profile (sigma = half a view step), normalised in binary32
    long long wi[9], tot = 0;
    for (int j = 0; j < 9; ++j) {
      const double t = (j - 4) / 4.0;
      wi[j] = std::llround(65535.0 * std::exp(-t * t / 0.5));
      tot += wi[j];
    }
    for (int j = 0; j < 9; ++j) net->taps.w[j] = (float)wi[j] / (float)tot;
  }
  if (!ok) {
    lfdpr_net_destroy(net);
    return LFDPR_ENOMEM;
  }
  if (hipMemset(net->master, 0, off * 4) != hipSuccess) {
    lfdpr_net_destroy(net);
    return LFDPR_EDEVICE;
  }
  *out = net;
  ctx_children_add(ctx, 1);
  net->counted = true;
  int rc = lfdpr_net_set_params(net, nullptr, 0);
  if (rc) {
    lfdpr_net_destroy(net);
    *out = nullptr;
  }
  return rc;
}

int lfdpr_net_destroy(lfdpr_net* net) {
  if (!net) return LFDPR_OK;
  (void)hipSetDevice(net->device);
  (void)hipStreamSynchronize(net->stream);
  if (net->counted) ctx_children_add(net->ctx, -1);
  (void)hipFree(net->master);
  (void)hipFree(net->grad);
  (void)hipFree(net->adam_m);
  (void)hipFree(net->adam_v);
  (void)hipFree(net->d_loss);
  (void)hipFree(net->part);
  for (int k = 0; k < 4; ++k) { (void)hipFree(net->wf[k]); (void)hipFree(net->wb[k]); (void)hipFree(net->act[k]); }
  for (int k = 0; k < 5; ++k) (void)hipFree(net->dz[k]);
  (void)hipFree(net->xb);
  delete net;
  return LFDPR_OK;
}

const char* lfdpr_net_last_error(lfdpr_net* net) { return net ? net->err.c_str() : "null network"; }

int lfdpr_net_param_count(lfdpr_net* net, int64_t* n) {
  if (!net || !n) return LFDPR_EINVAL;
  *n = net->nparams;
  return LFDPR_OK;
}

int lfdpr_net_set_params(lfdpr_net* net, const float* host, int64_t n) {
  if (!net) return LFDPR_EINVAL;
  if (host && n != net->nparams) return nfail(net, LFDPR_EINVAL, "parameter count mismatch");
  for (int64_t k = 0; host && k < n; ++k)
    if (!std::isfinite(host[k])) return nfail(net, LFDPR_EINVAL, "non-finite parameter");
  NHIP(hipSetDevice(net->device));
  NHIP(hipStreamSynchronize(net->stream));
  if (host) NHIP(hipMemcpy(net->master, host, n * 4, hipMemcpyHostToDevice));
  NHIP(hipMemset(net->adam_m, 0, net->nparams * 4));
  NHIP(hipMemset(net->adam_v, 0, net->nparams * 4));
  net->step = 0;
  pack_weights(net);
  NHIP(hipGetLastError());
  NHIP(hipStreamSynchronize(net->stream));
  return LFDPR_OK;
}

int lfdpr_net_get_params(lfdpr_net* net, float* host, int64_t n) {
  if (!net || !host || n != net->nparams) return LFDPR_EINVAL;
  NHIP(hipSetDevice(net->device));
  NHIP(hipStreamSynchronize(net->stream));
  NHIP(hipMemcpy(host, net->master, n * 4, hipMemcpyDeviceToHost));
  return LFDPR_OK;
}

int lfdpr_net_set_disparity_scale(lfdpr_net* net, float k) {
  if (!net) return LFDPR_EINVAL;
  if (!(k >= 0.0f) || !(k < 1.0e6f)) return nfail(net, LFDPR_EINVAL, "disparity scale out of range");
  net->kscale = k;
  return LFDPR_OK;
}

int lfdpr_net_set_rig(lfdpr_net* net, const lfdpr_view_params* v) {
  if (!net || !v) return LFDPR_EINVAL;
  if (v->V != net->V || v->W < 1 || !(v->aspect > 0.0f) || !(v->fovy_deg > 0.0f && v->fovy_deg < 180.0f) ||
      !(v->cone_deg >= 0.0f && v->cone_deg < 180.0f))
    return nfail(net, LFDPR_EINVAL, "rig does not match the network or is out of range");
  // a view step moves the eye by 2 D tan(cone/2) / V, which shifts a surface at
  // depth Z by fx * 2 D tan(cone/2) / V * (1/Z - 1/D) pixels = k * d, d = D/Z - 1
  const double fx = (v->W / 2.0) / ((double)v->aspect * std::tan((double)v->fovy_deg * M_PI / 360.0));
  const double k = fx * 2.0 * std::tan((double)v->cone_deg * M_PI / 360.0) / v->V;
  return lfdpr_net_set_disparity_scale(net, (float)k);
}

int lfdpr_net_pack_input(lfdpr_net* net, const uint32_t* views, const float* depth, int32_t n_views, int32_t H,
                         int32_t W, float D, void* x) {
  if (!net || !views || !x || n_views < 1 || H < 1 || W < 1 || !(D > 0.0f)) return LFDPR_EINVAL;
  NHIP(hipSetDevice(net->device));
  const int64_t n = (int64_t)n_views * H * W;
  k_pack_input<<<(unsigned)((n + 255) / 256), 256, 0, net->stream>>>(views, depth, n, D, (uint16_t*)x);
  NHIP(hipGetLastError());
  return LFDPR_OK;
}

int lfdpr_net_forward(lfdpr_net* net, const void* x, int32_t n_views, int32_t H, int32_t W, void* y) {
  if (!net || !x || !y) return LFDPR_EINVAL;
  if (n_views < 1 || n_views % net->V || H < 1 || W < 1 || (int64_t)n_views * H * W > net->maxpx)
    return nfail(net, LFDPR_EINVAL, "views must be whole frames of V views and fit the network's maximum");
  NHIP(hipSetDevice(net->device));
  const uint16_t* in = (const uint16_t*)x;
  hipStream_t s = net->stream;
  const int N = n_views, V = net->V;
  const int* d = kDilation;
  const int64_t npx = (int64_t)N * H * W;
  if (W <= kBlurRowMax) {
    const int64_t rows = (int64_t)N * H;
    k_disparity_blur_rows<<<(unsigned)(rows < 4096 ? rows : 4096), 256, (size_t)W * sizeof(uint2), s>>>(
        in, rows, W, net->kscale, net->taps, net->xb);
  } else {
    k_disparity_blur<<<(unsigned)((npx + 255) / 256), 256, 0, s>>>(in, npx, W, net->kscale, net->taps, net->xb);
  }
  launch_conv<2, MODE_RELU, true>(in, net->wf[0], net->master + net->off_b[0], N, H, W, V, d[0], net->act[1], kHidden, net->xb, 4, s);
  launch_conv<2, MODE_RELU, false>(net->act[1], net->wf[1], net->master + net->off_b[1], N, H, W, V, d[1], net->act[2], kHidden, nullptr, 0, s);
  launch_conv<2, MODE_RELU, false>(net->act[2], net->wf[2], net->master + net->off_b[2], N, H, W, V, d[2], net->act[3], kHidden, nullptr, 0, s);
  launch_conv<1, MODE_OUT, false>(net->act[3], net->wf[3], net->master + net->off_b[3], N, H, W, V, d[3], (uint16_t*)y, 4, net->xb, 4, s);
  NHIP(hipGetLastError());
  net->last_x = in;
  net->last_y = (const uint16_t*)y;
  net->last_n = N;
  net->last_h = H;
  net->last_w = W;
  return LFDPR_OK;
}

int lfdpr_net_backward(lfdpr_net* net, const void* target, float* loss) {
  if (!net || !target) return LFDPR_EINVAL;
  if (!net->last_x) return nfail(net, LFDPR_ESTATE, "lfdpr_net_forward first");
  NHIP(hipSetDevice(net->device));
  hipStream_t s = net->stream;
  const int N = net->last_n, H = net->last_h, W = net->last_w, V = net->V;
  const int npx = N * H * W;
  k_zero_f32<<<(unsigned)((net->nparams + 255) / 256), 256, 0, s>>>(net->grad, net->nparams);
  k_zero_f32<<<1, 64, 0, s>>>(net->d_loss, 1);
  const int64_t mse_blocks = ((int64_t)npx + 255) / 256;
  k_mse<<<(unsigned)(mse_blocks < 2048 ? mse_blocks : 2048), 256, 0, s>>>(net->last_y, (const uint16_t*)target, npx,
                                                                           net->dz[4], net->d_loss);
  // Gradient sums: at most kMaxGradBlocks blocks each (multiples of 256 pixels
  // for the weights, of 64 for the biases), then k_sum_partials in block order.
  const int chunk = (int)((((int64_t)npx + kMaxGradBlocks - 1) / kMaxGradBlocks + 255) / 256 * 256);
  const unsigned nch = (unsigned)((npx + chunk - 1) / chunk);
  const int bchunk = (int)((((int64_t)npx + kMaxGradBlocks - 1) / kMaxGradBlocks + 63) / 64 * 64);
  const unsigned nbch = (unsigned)((npx + bchunk - 1) / bchunk);
  float* const part_w = net->part;
  float* const part_b = net->part + (size_t)kMaxGradBlocks * 9 * kHidden * kHidden;
  for (int k = 3; k >= 0; --k) {
    const int CO = net->co[k], CI = net->ci[k];
    if (k == 0)
      k_conv_wgrad<true><<<nch, 256, 0, s>>>(net->dz[1], CO, net->last_x, net->xb, CI, N, H, W, V, kDilation[0],
                                             part_w, chunk);
    else
      k_conv_wgrad<false><<<nch, 256, 0, s>>>(net->dz[k + 1], CO, net->act[k], nullptr, CI, N, H, W, V, kDilation[k],
                                              part_w, chunk);
    const int nw = 9 * CO * CI;
    k_sum_partials<<<(unsigned)((nw + 15) / 16), 256, 0, s>>>(part_w, (int)nch, nw, net->grad + net->off_w[k]);
    k_bias_grad<<<nbch, 256, 0, s>>>(net->dz[k + 1], CO, npx, bchunk, part_b);
    k_sum_partials<<<(unsigned)((CO + 15) / 16), 256, 0, s>>>(part_b, (int)nbch, CO, net->grad + net->off_b[k]);
    if (k > 0)  // input gradient through the flipped, transposed weights (same dilation), masked by the ReLU
      launch_conv<2, MODE_BWD, false>(net->dz[k + 1], net->wb[k], nullptr, N, H, W, V, kDilation[k], net->dz[k], kHidden,
                                      net->act[k], kHidden, s);
  }
  NHIP(hipGetLastError());
  if (loss) NHIP(hipMemcpyAsync(loss, net->d_loss, 4, hipMemcpyDeviceToDevice, s));
  return LFDPR_OK;
}

int lfdpr_net_adam_step(lfdpr_net* net, float lr, float b1, float b2, float eps) {
  if (!net || !(lr >= 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps > 0.0f))
    return nfail(net, LFDPR_EINVAL, "Adam hyper-parameters out of range");
  NHIP(hipSetDevice(net->device));
  net->step += 1;
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)net->step));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)net->step));
  k_adam<<<(unsigned)((net->nparams + 255) / 256), 256, 0, net->stream>>>(net->master, net->grad, net->adam_m,
                                                                          net->adam_v, net->nparams, lr, b1, b2, eps,
                                                                          c1, c2);
  pack_weights(net);
  NHIP(hipGetLastError());
  return LFDPR_OK;
}

int lfdpr_net_unpack_output(lfdpr_net* net, const void* y, int32_t n_views, int32_t H, int32_t W, uint32_t* views) {
  if (!net || !y || !views || n_views < 1 || H < 1 || W < 1) return LFDPR_EINVAL;
  NHIP(hipSetDevice(net->device));
  const int64_t n = (int64_t)n_views * H * W;
  k_unpack_output<<<(unsigned)((n + 255) / 256), 256, 0, net->stream>>>((const uint16_t*)y, n, views);
  NHIP(hipGetLastError());
  return LFDPR_OK;
}

int lfdpr_net_copy_state(lfdpr_net* net, int32_t which, void* dst, int64_t n_bytes) {
  if (!net || !dst) return LFDPR_EINVAL;
  const int64_t npx = (int64_t)net->last_n * net->last_h * net->last_w;
  const void* src = nullptr;
  int64_t bytes = 0;
  if (which >= 1 && which <= 3) { src = net->act[which]; bytes = npx * kHidden * 2; }
  else if (which == 4) { src = net->xb; bytes = npx * 4 * 2; }
  else if (which >= 11 && which <= 14) { src = net->dz[which - 10]; bytes = npx * kK * 2; }
  else if (which == 20) { src = net->grad; bytes = net->nparams * 4; }
  else return nfail(net, LFDPR_EINVAL, "unknown state");
  if (n_bytes < bytes) return nfail(net, LFDPR_EINVAL, "destination too small");
  NHIP(hipSetDevice(net->device));
  NHIP(hipStreamSynchronize(net->stream));
  NHIP(hipMemcpy(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice));
  return LFDPR_OK;
}

int lfdpr_net_save(lfdpr_net* net, const char* path) {
  if (!net || !path) return LFDPR_EINVAL;
  std::vector<float> buf(3 * net->nparams);
  NHIP(hipSetDevice(net->device));
  NHIP(hipStreamSynchronize(net->stream));
  NHIP(hipMemcpy(buf.data(), net->master, net->nparams * 4, hipMemcpyDeviceToHost));
  NHIP(hipMemcpy(buf.data() + net->nparams, net->adam_m, net->nparams * 4, hipMemcpyDeviceToHost));
  NHIP(hipMemcpy(buf.data() + 2 * net->nparams, net->adam_v, net->nparams * 4, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  if (!f) return nfail(net, LFDPR_EINVAL, "cannot open file for writing");
  const char magic[8] = {'L', 'F', 'D', 'P', 'R', 'N', 'E', '1'};
  int64_t hdr[3] = {net->V, net->nparams, net->step};
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 8, 3, f) == 3 &&
            std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? LFDPR_OK : nfail(net, LFDPR_EINVAL, "write failed");
}

int lfdpr_net_load(lfdpr_net* net, const char* path) {
  if (!net || !path) return LFDPR_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return nfail(net, LFDPR_EINVAL, "cannot open file");
  char magic[8];
  int64_t hdr[3];
  std::vector<float> buf(3 * net->nparams);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "LFDPRNE1", 8) == 0 && std::fread(hdr, 8, 3, f) == 3 &&
            hdr[0] == net->V && hdr[1] == net->nparams && hdr[2] >= 0 &&
            std::fread(buf.data(), 4, buf.size(), f) == buf.size();
  std::fclose(f);
  if (!ok) return nfail(net, LFDPR_EINVAL, "not a checkpoint of this network");
  int rc = lfdpr_net_set_params(net, buf.data(), net->nparams);
  if (rc) return rc;
  NHIP(hipMemcpy(net->adam_m, buf.data() + net->nparams, net->nparams * 4, hipMemcpyHostToDevice));
  NHIP(hipMemcpy(net->adam_v, buf.data() + 2 * net->nparams, net->nparams * 4, hipMemcpyHostToDevice));
  net->step = hdr[2];
  return LFDPR_OK;
}

}  // extern "C"
