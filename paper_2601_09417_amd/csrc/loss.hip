// vbm_image_loss: the fine-tuning image loss (Sec. 4.4 uses the loss of the cited 3DGS) and its
// gradient with respect to the rendered image.
//
//   L1    = mean |x - y| over all views, channels and pixels
//   SSIM  = mean of the SSIM map; per channel, 11x11 Gaussian window (sigma 1.5), zero-padded
//           "same" filtering, C1 = 0.01^2, C2 = 0.03^2
//   loss  = L1 (kind 0) or (1 - lambda) L1 + lambda (1 - SSIM) (kind 1)
//
// SSIM gradient: with mu = w * x, Sxx = w * x^2, Sxy = w * (x y) the map value s(q) depends on x
// through (mu_x, Sxx, Sxy), so dSSIM/dx(p) = (1/n) [w * ds/dmu_x + 2 x(p) (w * ds/dSxx) + y(p) (w * ds/dSxy)](p)
// (the window is symmetric, so the adjoint of the zero-padded filter is the filter itself):
//   ds/dmu_x = s (2 mu_y / A1 - 2 mu_y / A2 - 2 mu_x / B1 + 2 mu_x / B2),  ds/dSxx = -s / B2,
//   ds/dSxy = 2 s / A2,  A1 = 2 mu_x mu_y + C1, A2 = 2 sigma_xy + C2, B1 = mu_x^2 + mu_y^2 + C1,
//   B2 = sigma_x^2 + sigma_y^2 + C2.
// Two LDS-tiled passes over 32x32 output tiles (256 threads, each filtering a 4-row strip of one
// column vertically): (1) the four filtered maps (x, y, x^2 + y^2, x y) -> s and the three
// partials, (2) the filtered partials -> dL/dx.  Partial sums go to per-block slots reduced in two
// fixed-order stages (256 contiguous chunks, then one block), so the loss value is deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"

// Scratch of vbm_image_loss_static: one copy per GPU, held by the loaded code object until the
// process ends.  In host code this name is only a stand-in for the symbol: the device address of
// each GPU's copy comes from hipGetSymbolAddress (static_scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[VBM_IMAGE_LOSS_STATIC_SCRATCH_BYTES];

namespace vbm {
namespace {

constexpr int TX = 32;             // output tile width (one column per lane of a half wave)
constexpr int TY = 32;             // output tile height
constexpr int RAD = 5;             // window radius
constexpr int EX = TX + 2 * RAD;   // tile with halo
constexpr int EY = TY + 2 * RAD;
constexpr int RPT = 4;             // output rows per thread in the vertical pass (256 threads)
constexpr int kRedBlocks = 256;    // first stage of the partial-sum reduction
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;
constexpr int kRowLoads = (EY + 3) / 4;        // halo rows per wave (a lane per halo column)
static_assert(TX * (TY / RPT) == 256, "vertical pass covers the tile with 256 threads");
static_assert(EX <= 64, "a halo row fits one wave");

struct Window {
  float w[2 * RAD + 1];
};

Window make_window() {
  Window W;
  double s = 0, g[2 * RAD + 1];
  for (int i = 0; i < 2 * RAD + 1; ++i) {
    const double x = i - RAD;
    g[i] = std::exp(-x * x / (2.0 * 1.5 * 1.5));
    s += g[i];
  }
  for (int i = 0; i < 2 * RAD + 1; ++i) W.w[i] = static_cast<float>(g[i] / s);
  return W;
}

__device__ __forceinline__ float block_sum(float v, float* s_red) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) s_red[w] = v;
  __syncthreads();
  float t = 0.0f;
  if (threadIdx.x == 0)
    for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) t += s_red[i];
  return t;
}

// Block order of the SSIM passes.  A run of equal-size views has n_blocks = tiles x 3 channels x
// views logical blocks (tile fastest).  Consecutive dispatches go to the 8 XCDs in turn and each XCD
// has its own L2, so dispatch L takes logical block (L mod 8) * ceil(n_blocks / 8) + L / 8: every
// XCD works through a contiguous run of tiles, and the halo rows and columns that neighbouring
// tiles share are fetched once into that XCD's L2 instead of once per XCD.  Returns false for the
// few padding dispatches past the end.
constexpr int kXcds = 8;

struct SsimBlock {
  int tile, c, z, bid;
};

__device__ __forceinline__ bool ssim_block(int tiles, int n_blocks, SsimBlock& b) {
  const int per = (n_blocks + kXcds - 1) / kXcds;
  const int d = static_cast<int>(blockIdx.x);
  const int logical = (d % kXcds) * per + d / kXcds;
  if (logical >= n_blocks) return false;
  b.tile = logical % tiles;
  b.c = (logical / tiles) % 3;
  b.z = logical / (3 * tiles);
  b.bid = logical;
  return true;
}

// L1 only: dL/dx = scale * sign(x - y); per-block partial of |x - y|.
__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ x, const float* __restrict__ y, int64_t n,
                                            float scale, float* __restrict__ grad, float* __restrict__ partial) {
  __shared__ float s_red[4];
  float acc = 0.0f;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * 256) {
    const float d = x[i] - y[i];
    acc += fabsf(d);
    grad[i] = d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
  }
  const float t = block_sum(acc, s_red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Loads the (TY + 10) x (TX + 10) halo of one channel into LDS: wave w takes halo rows w, w + 4,
// ..., a lane per column; every load is issued before the first store so their latencies overlap.
// The loads are range-checked buffer loads over the channel plane: a lane outside the image (or
// the halo) asks for an offset past the plane and reads 0, so no lane needs its own branch.
template <int NF>
__device__ __forceinline__ void load_halo(const float* const (&src)[NF], int W, int H, int ox, int oy,
                                          float (*dst)[EY][EX + 1]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int gx = ox + lane;
  const int plane_bytes = W * H * 4;   // the plan bounds a view to 16384^2 pixels: below 2^31
  __amdgpu_buffer_rsrc_t rs[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f)
    rs[f] = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(src[f]), (short)0, plane_bytes, 0x00020000);
  float v[NF][kRowLoads];
#pragma unroll
  for (int k = 0; k < kRowLoads; ++k) {
    const int r = w + 4 * k, gy = oy + r;
    const bool in = lane < EX && r < EY && gx >= 0 && gx < W && gy >= 0 && gy < H;
    const int off = in ? 4 * (gy * W + gx) : plane_bytes;
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f][k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs[f], off, 0, 0));
  }
#pragma unroll
  for (int k = 0; k < kRowLoads; ++k) {
    const int r = w + 4 * k;
    if (lane < EX && r < EY)
#pragma unroll
      for (int f = 0; f < NF; ++f) dst[f][r][lane] = v[f][k];
  }
}

// Pass 1 of SSIM over a run of views of equal size: one block per (tile, channel, view) in the
// order of ssim_block, 256 threads, 32x32 outputs per block.  SSIM needs E[x^2] and E[y^2] only through their sum (in
// sigma_x^2 + sigma_y^2, and d/dx of the sum is that of E[x^2]), so four signals are filtered:
// x, y, x^2 + y^2 and x y.  Their horizontally filtered maps over the (TY + 10) x TX halo rows are
// staged in LDS; each thread then filters a 4-row strip of one column vertically.
__global__ __launch_bounds__(256) void k_ssim_maps(const float* __restrict__ x, const float* __restrict__ y, int W,
                                                   int H, int tiles_x, int tiles, int n_blocks, Window win,
                                                   float* __restrict__ p1,
                                                   float* __restrict__ p2, float* __restrict__ p3,
                                                   float* __restrict__ partial_s, float* __restrict__ partial_l1) {
  // The filtered maps 2 and 3 overlay the input halo: the horizontal pass holds them in registers
  // until every thread has read the halo.
  constexpr int kHalo = EY * (EX + 1), kMap = EY * TX;
  __shared__ float lds[2 * kMap + 2 * kHalo];
  __shared__ float s_red[4];
  auto sxy = reinterpret_cast<float(*)[EY][EX + 1]>(lds + 2 * kMap);
  auto hb = reinterpret_cast<float(*)[EY][TX]>(lds);
  auto sx = sxy[0];
  auto sy = sxy[1];
  SsimBlock blk;
  if (!ssim_block(tiles, n_blocks, blk)) return;
  const int c = blk.c;
  const int bx = blk.tile % tiles_x, by = blk.tile / tiles_x;
  const int64_t HW = static_cast<int64_t>(W) * H;
  const int64_t chan = (3 * static_cast<int64_t>(blk.z) + c) * HW;
  const int ox = bx * TX - RAD, oy = by * TY - RAD;
  {
    const float* const src[2] = {x + chan, y + chan};
    load_halo<2>(src, W, H, ox, oy, sxy);
  }
  __syncthreads();
  const int col = threadIdx.x % TX;
  const int r0 = (threadIdx.x / TX) * RPT;
  float l1 = 0.0f;   // |x - y| of the thread's outputs (zero outside the image)
#pragma unroll
  for (int o = 0; o < RPT; ++o) l1 += fabsf(sx[r0 + o + RAD][col + RAD] - sy[r0 + o + RAD][col + RAD]);
  // Horizontal pass: a task filters four adjacent columns of one halo row, so each of the 14 input
  // values it reads forms its two products once for all four outputs.
  constexpr int CPT = 4;                          // columns per task
  constexpr int kTasks = EY * (TX / CPT);
  static_assert(kTasks <= 512, "two rounds of tasks");
  float keep[2][2][CPT];
#pragma unroll
  for (int rd = 0; rd < 2; ++rd) {
    const int task = threadIdx.x + 256 * rd;
    if (task >= kTasks) break;
    const int r = task / (TX / CPT), c0 = (task % (TX / CPT)) * CPT;
    float acc[4][CPT];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int o = 0; o < CPT; ++o) acc[f][o] = 0.0f;
#pragma unroll
    for (int t = 0; t < CPT + 2 * RAD; ++t) {
      const float u = sx[r][c0 + t], v = sy[r][c0 + t];
      const float qq = fmaf(u, u, v * v), uv = u * v;
#pragma unroll
      for (int o = 0; o < CPT; ++o) {
        if (t - o < 0 || t - o > 2 * RAD) continue;
        const float wk = win.w[t - o];
        acc[0][o] = fmaf(wk, u, acc[0][o]);
        acc[1][o] = fmaf(wk, v, acc[1][o]);
        acc[2][o] = fmaf(wk, qq, acc[2][o]);
        acc[3][o] = fmaf(wk, uv, acc[3][o]);
      }
    }
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int o = 0; o < CPT; ++o) hb[f][r][c0 + o] = acc[f][o];
#pragma unroll
    for (int o = 0; o < CPT; ++o) {
      keep[rd][0][o] = acc[2][o];
      keep[rd][1][o] = acc[3][o];
    }
  }
  __syncthreads();
#pragma unroll
  for (int rd = 0; rd < 2; ++rd) {
    const int task = threadIdx.x + 256 * rd;
    if (task >= kTasks) break;
    const int r = task / (TX / CPT), c0 = (task % (TX / CPT)) * CPT;
#pragma unroll
    for (int o = 0; o < CPT; ++o) {
      hb[2][r][c0 + o] = keep[rd][0][o];
      hb[3][r][c0 + o] = keep[rd][1][o];
    }
  }
  __syncthreads();
  const int gx = bx * TX + col;
  // the three partial maps of this channel plane, stored through range-checked buffer stores
  const int plane_bytes = W * H * 4;
  const __amdgpu_buffer_rsrc_t r1 = __builtin_amdgcn_make_buffer_rsrc(p1 + chan, (short)0, plane_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t r2 = __builtin_amdgcn_make_buffer_rsrc(p2 + chan, (short)0, plane_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t r3 = __builtin_amdgcn_make_buffer_rsrc(p3 + chan, (short)0, plane_bytes, 0x00020000);
  float m[RPT][4];
#pragma unroll
  for (int o = 0; o < RPT; ++o)
#pragma unroll
    for (int f = 0; f < 4; ++f) m[o][f] = 0.0f;
#pragma unroll
  for (int t = 0; t < RPT + 2 * RAD; ++t) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const float h = hb[f][r0 + t][col];
#pragma unroll
      for (int o = 0; o < RPT; ++o)
        if (t - o >= 0 && t - o <= 2 * RAD) m[o][f] = fmaf(win.w[t - o], h, m[o][f]);
    }
  }
  float sval = 0.0f;
#pragma unroll
  for (int o = 0; o < RPT; ++o) {
    const int gy = by * TY + r0 + o;
    if (gx < W && gy < H) {
      const float mx = m[o][0], my = m[o][1];
      const float mm = mx * mx + my * my, cxy = m[o][3] - mx * my;
      const float A1 = 2.0f * mx * my + kC1, A2 = 2.0f * cxy + kC2;
      const float B1 = mm + kC1, B2 = (m[o][2] - mm) + kC2;   // sigma_x^2 + sigma_y^2 + C2
      // two hardware reciprocals (about 1 ulp), of A1 A2 and B1 B2, instead of six divisions
      const float AA = A1 * A2, iA = __builtin_amdgcn_rcpf(AA), iB = __builtin_amdgcn_rcpf(B1 * B2);
      const float iA1 = A2 * iA, iA2 = A1 * iA, iB1 = B2 * iB, iB2 = B1 * iB;
      const float sv = AA * iB;
      const int off = 4 * (gy * W + gx);
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, 2.0f * sv * (my * (iA1 - iA2) + mx * (iB2 - iB1))),
                                            r1, off, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, -sv * iB2), r2, off, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, 2.0f * sv * iA2), r3, off, 0, 0);
      sval += sv;
    }
  }
  const int64_t bid = blk.bid;
  const float ts = block_sum(sval, s_red);
  if (threadIdx.x == 0) partial_s[bid] = ts;
  __syncthreads();
  const float tl = block_sum(l1, s_red);
  if (threadIdx.x == 0) partial_l1[bid] = tl;
}

// Pass 2: dL/dx = w_l1 sign(x - y) - w_ssim [w*p1 + 2 x (w*p2) + y (w*p3)], same tiling; the
// horizontal pass filters four adjacent columns per task, reading each input once for all four.
__global__ __launch_bounds__(256) void k_ssim_grad(const float* __restrict__ x, const float* __restrict__ y, int W,
                                                   int H, int tiles_x, int tiles, int n_blocks, Window win,
                                                   const float* __restrict__ p1,
                                                   const float* __restrict__ p2, const float* __restrict__ p3,
                                                   float w_l1, float w_ssim, float* __restrict__ grad) {
  // Filtered maps 1 and 2 overlay the input halo (held in registers until it has been read).
  constexpr int kHalo = EY * (EX + 1), kMap = EY * TX;
  __shared__ float lds[kMap + 3 * kHalo];
  auto sp = reinterpret_cast<float(*)[EY][EX + 1]>(lds + kMap);
  auto hb = reinterpret_cast<float(*)[EY][TX]>(lds);
  SsimBlock blk;
  if (!ssim_block(tiles, n_blocks, blk)) return;
  const int c = blk.c;
  const int bx = blk.tile % tiles_x, by = blk.tile / tiles_x;
  const int64_t HW = static_cast<int64_t>(W) * H;
  const int64_t chan = (3 * static_cast<int64_t>(blk.z) + c) * HW;
  const int ox = bx * TX - RAD, oy = by * TY - RAD;
  {
    const float* const src[3] = {p1 + chan, p2 + chan, p3 + chan};
    load_halo<3>(src, W, H, ox, oy, sp);
  }
  // The thread's own outputs need x and y at its RPT pixels: requested now, so that the loads
  // complete while the block filters (range-checked: a pixel outside the plane reads 0, unused).
  const int col = threadIdx.x % TX;
  const int r0 = (threadIdx.x / TX) * RPT;
  const int gx = bx * TX + col;
  const int plane_bytes = W * H * 4;
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(x + chan), (short)0,
                                                                      plane_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(y + chan), (short)0,
                                                                      plane_bytes, 0x00020000);
  float xv[RPT], yv[RPT];
#pragma unroll
  for (int o = 0; o < RPT; ++o) {
    const int gy = by * TY + r0 + o;
    const int off = gx < W && gy < H ? 4 * (gy * W + gx) : plane_bytes;
    xv[o] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, off, 0, 0));
    yv[o] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ry, off, 0, 0));
  }
  __syncthreads();
  constexpr int CPT = 4;
  constexpr int kTasks = EY * (TX / CPT);
  static_assert(kTasks <= 512, "two rounds of tasks");
  float keep[2][2][CPT];
#pragma unroll
  for (int rd = 0; rd < 2; ++rd) {
    const int task = threadIdx.x + 256 * rd;
    if (task >= kTasks) break;
    const int r = task / (TX / CPT), c0 = (task % (TX / CPT)) * CPT;
    float a[3][CPT];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
      for (int o = 0; o < CPT; ++o) a[f][o] = 0.0f;
#pragma unroll
    for (int t = 0; t < CPT + 2 * RAD; ++t) {
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        const float u = sp[f][r][c0 + t];
#pragma unroll
        for (int o = 0; o < CPT; ++o)
          if (t - o >= 0 && t - o <= 2 * RAD) a[f][o] = fmaf(win.w[t - o], u, a[f][o]);
      }
    }
#pragma unroll
    for (int o = 0; o < CPT; ++o) {
      hb[0][r][c0 + o] = a[0][o];
      keep[rd][0][o] = a[1][o];
      keep[rd][1][o] = a[2][o];
    }
  }
  __syncthreads();
#pragma unroll
  for (int rd = 0; rd < 2; ++rd) {
    const int task = threadIdx.x + 256 * rd;
    if (task >= kTasks) break;
    const int r = task / (TX / CPT), c0 = (task % (TX / CPT)) * CPT;
#pragma unroll
    for (int o = 0; o < CPT; ++o) {
      hb[1][r][c0 + o] = keep[rd][0][o];
      hb[2][r][c0 + o] = keep[rd][1][o];
    }
  }
  __syncthreads();
  float b[RPT][3];
#pragma unroll
  for (int o = 0; o < RPT; ++o)
#pragma unroll
    for (int f = 0; f < 3; ++f) b[o][f] = 0.0f;
#pragma unroll
  for (int t = 0; t < RPT + 2 * RAD; ++t) {
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const float h = hb[f][r0 + t][col];
#pragma unroll
      for (int o = 0; o < RPT; ++o)
        if (t - o >= 0 && t - o <= 2 * RAD) b[o][f] = fmaf(win.w[t - o], h, b[o][f]);
    }
  }
  if (gx >= W) return;
  const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(grad + chan, (short)0, plane_bytes, 0x00020000);
#pragma unroll
  for (int o = 0; o < RPT; ++o) {
    const int gy = by * TY + r0 + o;
    if (gy >= H) continue;
    const int off = 4 * (gy * W + gx);
    const float d = xv[o] - yv[o];
    const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
    __builtin_amdgcn_raw_buffer_store_b32(
        __builtin_bit_cast(uint32_t, w_l1 * sg - w_ssim * (b[o][0] + 2.0f * xv[o] * b[o][1] + yv[o] * b[o][2])), rg,
        off, 0, 0);
  }
}

// First stage of the deterministic reduction: block b sums the fixed chunk
// [b * chunk, min((b + 1) * chunk, n)) of each partial array in double, in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_stage(const float* __restrict__ l1p, const float* __restrict__ sp,
                                                      int64_t n, int64_t chunk, double* __restrict__ out) {
  __shared__ double s_l[256], s_s[256];
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t hi = min(lo + chunk, n);
  double al = 0.0, as = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    al += l1p[i];
    if (sp) as += sp[i];
  }
  s_l[threadIdx.x] = al;
  s_s[threadIdx.x] = as;
  __syncthreads();
  for (int st = 128; st >= 1; st >>= 1) {
    if (static_cast<int>(threadIdx.x) < st) {
      s_l[threadIdx.x] += s_l[threadIdx.x + st];
      s_s[threadIdx.x] += s_s[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = s_l[0];
    out[2 * blockIdx.x + 1] = s_s[0];
  }
}

// Second stage: loss = a * sum(l1 parts) + b * sum(ssim parts) + c, summed in a fixed order.
__global__ void k_finalize(const double* __restrict__ parts, double a, double b, double c0,
                           float* __restrict__ loss) {
  __shared__ double s_red[kRedBlocks];
  s_red[threadIdx.x] = a * parts[2 * threadIdx.x] + b * parts[2 * threadIdx.x + 1];
  __syncthreads();
  for (int st = kRedBlocks / 2; st >= 1; st >>= 1) {
    if (static_cast<int>(threadIdx.x) < st) s_red[threadIdx.x] += s_red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = static_cast<float>(s_red[0] + c0);
}

constexpr int kL1Blocks = 1024;

}  // namespace
}  // namespace vbm

using namespace vbm;

extern "C" size_t vbm_image_loss_workspace_size(const int32_t* dims, int32_t n_views, int32_t kind) {
  if (!dims || n_views < 1) return 0;
  int64_t px = 0, blocks = 0;
  for (int v = 0; v < n_views; ++v) {
    const int64_t W = dims[2 * v], H = dims[2 * v + 1];
    px += W * H;
    blocks += ceil_div(W, TX) * ceil_div(H, TY) * 3;
  }
  const size_t red = align_up(2 * kRedBlocks * sizeof(double), 256);
  if (kind == 0) return align_up(kL1Blocks * 4, 256) + red;
  return 3 * align_up(3 * px * 4, 256) + 2 * align_up(blocks * 4, 256) + red;
}

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's copy of `scratch`, looked up once per device (with that
// device current) and kept; nullptr with the error set when the lookup fails.
void* static_scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error("vbm_image_loss_static: no current device (or device index %d beyond %d)", dev, kMaxDevices);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      hip_check(e == hipSuccess ? hipErrorInvalidSymbol : e, "vbm_image_loss_static: hipGetSymbolAddress(scratch)");
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" vbm_status vbm_image_loss(const float* image, const float* target, const int32_t* dims, int32_t n_views,
                                     int32_t kind, float lambda, float* grad, float* loss, void* ws, size_t ws_bytes,
                                     void* stream) {
  if (!image || !target || !dims || !grad || !loss || (!ws && vbm_image_loss_workspace_size(dims, n_views, kind))) {
    set_error("vbm_image_loss: null argument");
    return VBM_ERR_INVALID;
  }
  if (n_views < 1 || (kind != 0 && kind != 1) || !(lambda >= 0.0f && lambda <= 1.0f)) {
    set_error("vbm_image_loss: need n_views >= 1, kind 0 or 1, 0 <= lambda <= 1");
    return VBM_ERR_INVALID;
  }
  int64_t px = 0;
  for (int v = 0; v < n_views; ++v) {
    if (dims[2 * v] < 1 || dims[2 * v + 1] < 1) {
      set_error("vbm_image_loss: view %d has an empty image", v);
      return VBM_ERR_INVALID;
    }
    px += static_cast<int64_t>(dims[2 * v]) * dims[2 * v + 1];
  }
  if (ws_bytes < vbm_image_loss_workspace_size(dims, n_views, kind)) {
    set_error("vbm_image_loss: workspace too small");
    return VBM_ERR_WORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = 3 * px;
  const double dn = static_cast<double>(n);
  Carver c(ws);
  if (kind == 0) {
    float* partial = c.take<float>(kL1Blocks);
    double* parts = c.take<double>(2 * kRedBlocks);
    hipLaunchKernelGGL(k_l1, dim3(kL1Blocks), dim3(256), 0, s, image, target, n, 1.0f / static_cast<float>(n), grad,
                       partial);
    VBM_LAUNCH_CHECK("loss_l1");
    hipLaunchKernelGGL(k_reduce_stage, dim3(kRedBlocks), dim3(256), 0, s, partial, static_cast<const float*>(nullptr),
                       static_cast<int64_t>(kL1Blocks), ceil_div(kL1Blocks, kRedBlocks), parts);
    VBM_LAUNCH_CHECK("loss_reduce");
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedBlocks), 0, s, parts, 1.0 / dn, 0.0, 0.0, loss);
    VBM_LAUNCH_CHECK("loss_finalize");
    return VBM_OK;
  }
  float* p1 = c.take<float>(n);
  float* p2 = c.take<float>(n);
  float* p3 = c.take<float>(n);
  int64_t blocks = 0;
  for (int v = 0; v < n_views; ++v) blocks += ceil_div(dims[2 * v], TX) * ceil_div(dims[2 * v + 1], TY) * 3;
  float* ps = c.take<float>(blocks);
  float* pl = c.take<float>(blocks);
  double* parts = c.take<double>(2 * kRedBlocks);
  const Window win = make_window();
  const float w_l1 = (1.0f - lambda) / static_cast<float>(n);
  const float w_ss = lambda / static_cast<float>(n);
  // One launch of each pass per run of consecutive views of equal size (their images are
  // consecutive); the partial slots keep the view, channel, tile order.
  int64_t off = 0, boff = 0;
  for (int v = 0; v < n_views;) {
    const int W = dims[2 * v], H = dims[2 * v + 1];
    int nv = 1;
    while (v + nv < n_views && nv < 65535 && dims[2 * (v + nv)] == W && dims[2 * (v + nv) + 1] == H) ++nv;
    const int tx = static_cast<int>(ceil_div(W, TX)), ty = static_cast<int>(ceil_div(H, TY));
    const int64_t nb64 = static_cast<int64_t>(tx) * ty * 3 * nv;
    if (nb64 > (int64_t{1} << 30)) {
      set_error("vbm_image_loss: %lld SSIM tiles in one run of views", static_cast<long long>(nb64));
      return VBM_ERR_UNSUPPORTED;
    }
    const int nb = static_cast<int>(nb64);
    const dim3 grid(static_cast<unsigned>(kXcds * ceil_div(nb, kXcds)));
    hipLaunchKernelGGL(k_ssim_maps, grid, dim3(256), 0, s, image + off, target + off, W, H, tx, tx * ty, nb, win,
                       p1 + off, p2 + off, p3 + off, ps + boff, pl + boff);
    VBM_LAUNCH_CHECK("ssim_maps");
    hipLaunchKernelGGL(k_ssim_grad, grid, dim3(256), 0, s, image + off, target + off, W, H, tx, tx * ty, nb, win,
                       p1 + off, p2 + off, p3 + off, w_l1, w_ss, grad + off);
    VBM_LAUNCH_CHECK("ssim_grad");
    off += 3 * static_cast<int64_t>(W) * H * nv;
    boff += static_cast<int64_t>(tx) * ty * 3 * nv;
    v += nv;
  }
  hipLaunchKernelGGL(k_reduce_stage, dim3(kRedBlocks), dim3(256), 0, s, pl, ps, blocks,
                     ceil_div(blocks, kRedBlocks), parts);
  VBM_LAUNCH_CHECK("loss_reduce");
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedBlocks), 0, s, parts, (1.0 - lambda) / dn, -lambda / dn,
                     static_cast<double>(lambda), loss);
  VBM_LAUNCH_CHECK("loss_finalize");
  return VBM_OK;
}

extern "C" vbm_status vbm_image_loss_static(const float* image, const float* target, const int32_t* dims,
                                            int32_t n_views, int32_t kind, float lambda, float* grad, float* loss,
                                            void* stream) {
  if (!dims || n_views < 1) {
    set_error("vbm_image_loss_static: null view sizes or n_views < 1");
    return VBM_ERR_INVALID;
  }
  const size_t need = vbm_image_loss_workspace_size(dims, n_views, kind);
  if (need > static_cast<size_t>(VBM_IMAGE_LOSS_STATIC_SCRATCH_BYTES)) {
    set_error("vbm_image_loss_static: this loss needs %zu bytes of scratch, more than the fixed %zu; use "
              "vbm_image_loss with a workspace",
              need, static_cast<size_t>(VBM_IMAGE_LOSS_STATIC_SCRATCH_BYTES));
    return VBM_ERR_CAPACITY;
  }
  void* ws = static_scratch_ptr();
  if (!ws) return VBM_ERR_HIP;
  // The passes write every scratch value before they read it (maps, per-block partial sums, the
  // reduction stage), so nothing is cleared first.
  return vbm_image_loss(image, target, dims, n_views, kind, lambda, grad, loss, ws,
                        static_cast<size_t>(VBM_IMAGE_LOSS_STATIC_SCRATCH_BYTES), stream);
}
