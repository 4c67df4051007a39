// Learned angular reconstruction: a small 3x3 convolutional network whose
// inference and training run on BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32
// accumulate).  It stands in for 4x angular supersampling (Sec. 4): input per
// pixel = the V rendered views' (R, G, B, d = D/Z - 1), 4V channels; layers
// 4V -> 32 -> 32 -> 32 -> 3V with ReLU; output = input RGB + network.
//
// Layouts: activations NHWC (channels innermost) in BF16; weights
// [tap][cout][cin] in BF16 with an FP32 master copy; tap = 3*(dy+1) + (dx+1)
// reads input pixel (y+dy, x+dx), zero padding.
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

union Frag {
  uint4 u;
  bf16x8 v;
};

// ---------------------------------------------------------------- 3x3 convolution
// One block = 4 waves = 256 output pixels of one image row segment (4 M-tiles of
// 16 pixels per wave); NT = COUT/16 output-channel tiles per M-tile.  Per tap,
// the block stages that tap's [COUT][CIN] weights in LDS.
template <int NT, int MODE>
__global__ void __launch_bounds__(256) k_conv3x3(const uint16_t* __restrict__ X, int CIN,
                                                  const uint16_t* __restrict__ Wt, const float* __restrict__ bias,
                                                  int H, int W, uint16_t* __restrict__ Y, int COUT_STORE,
                                                  const uint16_t* __restrict__ aux, int AUX_C) {
  constexpr int COUT = NT * 16;
  extern __shared__ uint4 wlds[];  // [COUT][CIN] bf16 of one tap
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int npx = H * W;
  const int ntile = (npx + 255) / 256;
  const int cin_q = CIN / 8;  // uint4 per weight row
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int pbase = tile * 256 + wv * 64;
    int py[4], px[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int p = pbase + m * 16 + r16;
      py[m] = p < npx ? p / W : -100;
      px[m] = p < npx ? p % W : -100;
    }
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      __syncthreads();
      const uint4* wsrc = reinterpret_cast<const uint4*>(Wt + (size_t)tap * COUT * CIN);
      for (int k = threadIdx.x; k < COUT * cin_q; k += blockDim.x) wlds[k] = wsrc[k];
      __syncthreads();
      for (int c0 = 0; c0 < CIN; c0 += 32) {
        Frag b[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) b[n].u = wlds[(n * 16 + r16) * cin_q + (c0 >> 3) + g];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int yy = py[m] + dy, xx = px[m] + dx;
          Frag a;
          a.u = uint4{0u, 0u, 0u, 0u};
          if (yy >= 0 && yy < H && xx >= 0 && xx < W)
            a.u = *reinterpret_cast<const uint4*>(X + ((size_t)yy * W + xx) * CIN + c0 + 8 * g);
#pragma unroll
          for (int n = 0; n < NT; ++n)
            acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b[n].v, acc[m][n], 0, 0, 0);
        }
      }
    }
    // epilogue: lane holds D[4g+e][r16] = pixel pbase + 16m + 4g + e, channel n*16 + r16
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const int co = n * 16 + r16;
        if (co >= COUT_STORE) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int p = pbase + m * 16 + 4 * g + e;
          if (p >= npx) continue;
          float v = acc[m][n][e];
          if (MODE == MODE_RELU) {
            v = fmaxf(v + bias[co], 0.0f);
          } else if (MODE == MODE_OUT) {
            v = (v + bias[co]) + from_bf16(aux[(size_t)p * AUX_C + 4 * (co / 3) + co % 3]);
          } else {
            v = from_bf16(aux[(size_t)p * AUX_C + co]) > 0.0f ? v : 0.0f;
          }
          Y[(size_t)p * COUT_STORE + co] = to_bf16(v);
        }
      }
  }
}

// ---------------------------------------------------------------- weight gradient
// dW[tap][co][ci] += sum_p dZ[p][co] * A[p + off(tap)][ci]: one wave per
// (tap, 16 co, 16 ci) tile and pixel chunk; M = co, N = ci, K = pixels.
__global__ void __launch_bounds__(64) k_conv_wgrad(const uint16_t* __restrict__ dZ, int DZS, int CO,
                                                    const uint16_t* __restrict__ A, int CI, int H, int W,
                                                    float* __restrict__ dW, int chunk) {
  const int lane = threadIdx.x, g = lane >> 4, r16 = lane & 15;
  const int nct = CO / 16, nit = CI / 16;
  int t = blockIdx.x;
  const int it = t % nit; t /= nit;
  const int ct = t % nct; t /= nct;
  const int tap = t;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int npx = H * W;
  const int p0 = blockIdx.y * chunk, p1 = min(npx, p0 + chunk);
  const int co = ct * 16 + r16, ci = it * 16 + r16;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = p0; k0 < p1; k0 += 32) {
    union { uint16_t h[8]; bf16x8 v; } fa, fb;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int p = k0 + 8 * g + e;
      uint16_t za = 0, zb = 0;
      if (p < p1) {
        za = dZ[(size_t)p * DZS + co];
        const int y = p / W, x = p % W;
        const int yy = y + dy, xx = x + dx;
        if (yy >= 0 && yy < H && xx >= 0 && xx < W) zb = A[((size_t)yy * W + xx) * CI + ci];
      }
      fa.h[e] = za;
      fb.h[e] = zb;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa.v, fb.v, acc, 0, 0, 0);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) atomicAdd(&dW[((size_t)tap * CO + ct * 16 + 4 * g + e) * CI + ci], acc[e]);
}

__global__ void k_bias_grad(const uint16_t* __restrict__ dZ, int DZS, int npx, float* __restrict__ db) {
  const int co = blockIdx.x;
  float s = 0.0f;
  for (int p = threadIdx.x; p < npx; p += blockDim.x) s += from_bf16(dZ[(size_t)p * DZS + co]);
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(&db[co], red[0]);
}

// loss = mean((y - t)^2) over npx*C values; dZ = bf16(2 (y - t) / n) into a
// [p][CP] buffer (channels C..CP-1 zero).
__global__ void k_mse(const uint16_t* __restrict__ Yb, const uint16_t* __restrict__ T, int C, int CP, int npx,
                      uint16_t* __restrict__ dZ, float* __restrict__ loss) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)npx * C;
  float sq = 0.0f;
  if (i < (int64_t)npx * CP) {
    const int64_t p = i / CP;
    const int c = (int)(i % CP);
    uint16_t out = 0;
    if (c < C) {
      const float d = from_bf16(Yb[p * C + c]) - from_bf16(T[p * C + c]);
      sq = d * d;
      out = to_bf16((2.0f * d) / (float)n);
    }
    dZ[i] = out;
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

// BF16 weights for the forward pass ([tap][co][ci]) and the flipped, transposed
// copy for the input gradient ([8 - tap][ci][co_pad], zero beyond co).
__global__ void k_pack_w(const float* __restrict__ master, int CO, int CI, int COP, uint16_t* __restrict__ wf,
                         uint16_t* __restrict__ wb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)9 * CO * CI;
  if (i < n) wf[i] = to_bf16(master[i]);
  if (wb) {
    const int64_t nb = (int64_t)9 * CI * COP;
    if (i < nb) {
      const int tapb = (int)(i / ((int64_t)CI * COP));
      const int rem = (int)(i % ((int64_t)CI * COP));
      const int ci = rem / COP, co = rem % COP;
      const int tap = 8 - tapb;
      wb[i] = co < CO ? to_bf16(master[((int64_t)tap * CO + co) * CI + ci]) : (uint16_t)0;
    }
  }
}

// views (V, H, W) RGBA8 + depth -> x[p][4v + c] = c/255, x[p][4v+3] = D/Z - 1 (-1 when empty)
__global__ void k_pack_input(const uint32_t* __restrict__ views, const float* __restrict__ depth, int V, int npx,
                             float D, uint16_t* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)V * npx) return;
  const int64_t p = i % npx;
  const int v = (int)(i / npx);
  const uint32_t c = views[(int64_t)v * npx + p];
  const float z = depth[(int64_t)v * npx + p];
  const float d = z < INFINITY ? D / z - 1.0f : -1.0f;
  uint16_t* o = x + p * (4 * V) + 4 * v;
  o[0] = to_bf16((float)(c & 255u) / 255.0f);
  o[1] = to_bf16((float)((c >> 8) & 255u) / 255.0f);
  o[2] = to_bf16((float)((c >> 16) & 255u) / 255.0f);
  o[3] = to_bf16(d);
}

// y[p][3v + c] -> RGBA8 views, clamp(floor(255 y + 0.5)), alpha 255
__global__ void k_unpack_output(const uint16_t* __restrict__ y, int V, int npx, uint32_t* __restrict__ views) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)V * npx) return;
  const int64_t p = i % npx;
  const int v = (int)(i / npx);
  uint32_t o = 0xFF000000u;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float f = floorf(from_bf16(y[p * (3 * V) + 3 * v + c]) * 255.0f + 0.5f);
    f = f < 0.0f ? 0.0f : (f > 255.0f ? 255.0f : f);
    o |= (uint32_t)f << (8 * c);
  }
  views[(int64_t)v * npx + p] = o;
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
  hipStream_t stream = nullptr;
  int device = 0;
  int V = 0, maxpx = 0;
  int ci[4], co[4], cop[4];
  int64_t off_w[4], off_b[4], nparams = 0;
  float* master = nullptr;
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  int64_t step = 0;
  uint16_t* wf[4] = {nullptr, nullptr, nullptr, nullptr};
  uint16_t* wb[4] = {nullptr, nullptr, nullptr, nullptr};
  uint16_t* act[4] = {nullptr, nullptr, nullptr, nullptr};  // act[0] unused (input is the caller's)
  uint16_t* dz[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const uint16_t* last_x = nullptr;
  const uint16_t* last_y = nullptr;
  int last_h = 0, last_w = 0;
  float* d_loss = nullptr;
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

template <int NT, int MODE>
void launch_conv(const uint16_t* X, int CIN, const uint16_t* Wt, const float* b, int H, int W, uint16_t* Y, int CS,
                 const uint16_t* aux, int AUXC, hipStream_t s) {
  const int tiles = (H * W + 255) / 256;
  const size_t lds = (size_t)NT * 16 * CIN * 2;
  const int grid = tiles < 2048 ? tiles : 2048;
  k_conv3x3<NT, MODE><<<grid, 256, lds, s>>>(X, CIN, Wt, b, H, W, Y, CS, aux, AUXC);
}

// forward conv dispatch on the output tile count
int conv_fwd(lfdpr_net* net, int layer, const uint16_t* X, int H, int W, uint16_t* Y, const uint16_t* resid) {
  const int CIN = net->ci[layer], COUT = net->co[layer];
  const float* b = net->master + net->off_b[layer];
  hipStream_t s = net->stream;
  if (layer < 3) {
    launch_conv<2, MODE_RELU>(X, CIN, net->wf[layer], b, H, W, Y, COUT, nullptr, 0, s);
  } else if (COUT == 48) {
    launch_conv<3, MODE_OUT>(X, CIN, net->wf[layer], b, H, W, Y, COUT, resid, net->ci[0], s);
  } else if (COUT == 144) {
    launch_conv<9, MODE_OUT>(X, CIN, net->wf[layer], b, H, W, Y, COUT, resid, net->ci[0], s);
  } else {
    return nfail(net, LFDPR_EINVAL, "unsupported output width");
  }
  return LFDPR_OK;
}

}  // namespace

extern "C" {

int lfdpr_net_create(lfdpr_ctx* ctx, int32_t V, int32_t max_h, int32_t max_w, lfdpr_net** out) {
  if (!ctx || !out) return LFDPR_EINVAL;
  *out = nullptr;
  if (!(V == 16 || V == 48) || max_h < 1 || max_w < 1 || (int64_t)max_h * max_w > (1 << 22))
    return LFDPR_EINVAL;
  lfdpr_net* net = new lfdpr_net();
  net->ctx = ctx;
  net->stream = ctx_stream_of(ctx);
  net->device = ctx_device_of(ctx);
  net->V = V;
  net->maxpx = max_h * max_w;
  const int ci[4] = {4 * V, kHidden, kHidden, kHidden}, co[4] = {kHidden, kHidden, kHidden, 3 * V};
  int64_t off = 0;
  for (int k = 0; k < 4; ++k) {
    net->ci[k] = ci[k];
    net->co[k] = co[k];
    net->cop[k] = (co[k] + 31) / 32 * 32;
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
  for (int k = 0; k < 4; ++k) {
    al(net->wf[k], 9ll * co[k] * ci[k]);
    if (k > 0) al(net->wb[k], 9ll * ci[k] * net->cop[k]);
    if (k > 0) al(net->act[k], (size_t)net->maxpx * kHidden);
  }
  for (int k = 1; k <= 4; ++k) al(net->dz[k], (size_t)net->maxpx * (k == 4 ? net->cop[3] : kHidden));
  if (!ok) {
    lfdpr_net_destroy(net);
    return LFDPR_ENOMEM;
  }
  if (hipMemset(net->master, 0, off * 4) != hipSuccess || hipMemset(net->adam_m, 0, off * 4) != hipSuccess ||
      hipMemset(net->adam_v, 0, off * 4) != hipSuccess) {
    lfdpr_net_destroy(net);
    return LFDPR_EDEVICE;
  }
  *out = net;
  return lfdpr_net_set_params(net, nullptr, 0);
}

int lfdpr_net_destroy(lfdpr_net* net) {
  if (!net) return LFDPR_OK;
  hipSetDevice(net->device);
  hipStreamSynchronize(net->stream);
  hipFree(net->master);
  hipFree(net->grad);
  hipFree(net->adam_m);
  hipFree(net->adam_v);
  hipFree(net->d_loss);
  for (int k = 0; k < 4; ++k) { hipFree(net->wf[k]); hipFree(net->wb[k]); hipFree(net->act[k]); }
  for (int k = 0; k < 5; ++k) hipFree(net->dz[k]);
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
  for (int k = 0; k < 4; ++k) {
    int64_t cnt = 9ll * net->co[k] * net->ci[k];
    int64_t cb = 9ll * net->ci[k] * net->cop[k];
    int64_t m = cnt > cb ? cnt : cb;
    k_pack_w<<<(unsigned)((m + 255) / 256), 256, 0, net->stream>>>(net->master + net->off_w[k], net->co[k], net->ci[k],
                                                                   net->cop[k], net->wf[k], net->wb[k]);
  }
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

int lfdpr_net_pack_input(lfdpr_net* net, const uint32_t* views, const float* depth, int32_t H, int32_t W, float D,
                         void* x) {
  if (!net || !views || !depth || !x || H < 1 || W < 1 || !(D > 0.0f)) return LFDPR_EINVAL;
  NHIP(hipSetDevice(net->device));
  const int64_t n = (int64_t)net->V * H * W;
  k_pack_input<<<(unsigned)((n + 255) / 256), 256, 0, net->stream>>>(views, depth, net->V, H * W, D, (uint16_t*)x);
  NHIP(hipGetLastError());
  return LFDPR_OK;
}

int lfdpr_net_forward(lfdpr_net* net, const void* x, int32_t H, int32_t W, void* y) {
  if (!net || !x || !y) return LFDPR_EINVAL;
  if (H < 1 || W < 1 || (int64_t)H * W > net->maxpx)
    return nfail(net, LFDPR_EINVAL, "image larger than the network's maximum");
  NHIP(hipSetDevice(net->device));
  const uint16_t* in = (const uint16_t*)x;
  int rc = conv_fwd(net, 0, in, H, W, net->act[1], nullptr);
  if (!rc) rc = conv_fwd(net, 1, net->act[1], H, W, net->act[2], nullptr);
  if (!rc) rc = conv_fwd(net, 2, net->act[2], H, W, net->act[3], nullptr);
  if (!rc) rc = conv_fwd(net, 3, net->act[3], H, W, (uint16_t*)y, in);
  if (rc) return rc;
  NHIP(hipGetLastError());
  net->last_x = in;
  net->last_y = (const uint16_t*)y;
  net->last_h = H;
  net->last_w = W;
  return LFDPR_OK;
}

int lfdpr_net_backward(lfdpr_net* net, const void* target, float* loss) {
  if (!net || !target) return LFDPR_EINVAL;
  if (!net->last_x) return nfail(net, LFDPR_ESTATE, "lfdpr_net_forward first");
  NHIP(hipSetDevice(net->device));
  hipStream_t s = net->stream;
  const int H = net->last_h, W = net->last_w, npx = H * W;
  k_zero_f32<<<(unsigned)((net->nparams + 255) / 256), 256, 0, s>>>(net->grad, net->nparams);
  k_zero_f32<<<1, 64, 0, s>>>(net->d_loss, 1);
  const int C4 = net->co[3], C4P = net->cop[3];
  const int64_t ne = (int64_t)npx * C4P;
  k_mse<<<(unsigned)((ne + 255) / 256), 256, 0, s>>>(net->last_y, (const uint16_t*)target, C4, C4P, npx, net->dz[4],
                                                     net->d_loss);
  const int chunk = 2048;
  const unsigned nch = (unsigned)((npx + chunk - 1) / chunk);
  for (int k = 3; k >= 0; --k) {
    const int CO = net->co[k], DZS = k == 3 ? C4P : kHidden, CI = net->ci[k];
    const uint16_t* A = k == 0 ? net->last_x : net->act[k];
    dim3 gw((unsigned)(9 * (CO / 16) * (CI / 16)), nch);
    k_conv_wgrad<<<gw, 64, 0, s>>>(net->dz[k + 1], DZS, CO, A, CI, H, W, net->grad + net->off_w[k], chunk);
    k_bias_grad<<<(unsigned)CO, 256, 0, s>>>(net->dz[k + 1], DZS, npx, net->grad + net->off_b[k]);
    if (k > 0)  // input gradient through the flipped, transposed weights, masked by the ReLU
      launch_conv<2, MODE_BWD>(net->dz[k + 1], DZS, net->wb[k], nullptr, H, W, net->dz[k], kHidden, net->act[k],
                               kHidden, s);
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
  for (int k = 0; k < 4; ++k) {
    int64_t cnt = 9ll * net->co[k] * net->ci[k];
    int64_t cb = 9ll * net->ci[k] * net->cop[k];
    int64_t m = cnt > cb ? cnt : cb;
    k_pack_w<<<(unsigned)((m + 255) / 256), 256, 0, net->stream>>>(net->master + net->off_w[k], net->co[k], net->ci[k],
                                                                   net->cop[k], net->wf[k], net->wb[k]);
  }
  NHIP(hipGetLastError());
  return LFDPR_OK;
}

int lfdpr_net_unpack_output(lfdpr_net* net, const void* y, int32_t H, int32_t W, uint32_t* views) {
  if (!net || !y || !views || H < 1 || W < 1) return LFDPR_EINVAL;
  NHIP(hipSetDevice(net->device));
  const int64_t n = (int64_t)net->V * H * W;
  k_unpack_output<<<(unsigned)((n + 255) / 256), 256, 0, net->stream>>>((const uint16_t*)y, net->V, H * W, views);
  NHIP(hipGetLastError());
  return LFDPR_OK;
}

int lfdpr_net_copy_state(lfdpr_net* net, int32_t which, void* dst, int64_t n_bytes) {
  if (!net || !dst) return LFDPR_EINVAL;
  const int64_t npx = (int64_t)net->last_h * net->last_w;
  const void* src = nullptr;
  int64_t bytes = 0;
  if (which >= 1 && which <= 3) { src = net->act[which]; bytes = npx * kHidden * 2; }
  else if (which >= 11 && which <= 13) { src = net->dz[which - 10]; bytes = npx * kHidden * 2; }
  else if (which == 14) { src = net->dz[4]; bytes = npx * net->cop[3] * 2; }
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
