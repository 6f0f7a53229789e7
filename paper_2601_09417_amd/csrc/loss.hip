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
// Two LDS-tiled passes per view: (1) the five filtered maps -> s and the three partials, (2) the
// filtered partials -> dL/dx.  Partial sums go to per-block slots reduced in a fixed order, so the
// loss value is deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "common.h"

namespace vbm {
namespace {

constexpr int TS = 16;             // output tile edge
constexpr int RAD = 5;             // window radius
constexpr int EXT = TS + 2 * RAD;  // tile with halo
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

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

// Pass 1 of SSIM for one view: grid (tiles_x, tiles_y, 3 channels), 256 threads.
__global__ __launch_bounds__(256) void k_ssim_maps(const float* __restrict__ x, const float* __restrict__ y, int W,
                                                   int H, Window win, float* __restrict__ p1, float* __restrict__ p2,
                                                   float* __restrict__ p3, float* __restrict__ partial_s,
                                                   float* __restrict__ partial_l1) {
  __shared__ float sx[EXT][EXT], sy[EXT][EXT];
  __shared__ float hb[5][EXT][TS];
  __shared__ float s_red[4];
  const int c = blockIdx.z;
  const int64_t HW = static_cast<int64_t>(W) * H;
  const float* xc = x + c * HW;
  const float* yc = y + c * HW;
  const int ox = blockIdx.x * TS - RAD, oy = blockIdx.y * TS - RAD;
  for (int i = threadIdx.x; i < EXT * EXT; i += 256) {
    const int r = i / EXT, q = i % EXT;
    const int gx = ox + q, gy = oy + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    sx[r][q] = in ? xc[static_cast<int64_t>(gy) * W + gx] : 0.0f;
    sy[r][q] = in ? yc[static_cast<int64_t>(gy) * W + gx] : 0.0f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < EXT * TS; i += 256) {
    const int r = i / TS, q = i % TS;
    float a = 0, b = 0, aa = 0, bb = 0, ab = 0;
    for (int k = 0; k < 2 * RAD + 1; ++k) {
      const float u = sx[r][q + k], v = sy[r][q + k], wk = win.w[k];
      a += wk * u;
      b += wk * v;
      aa += wk * u * u;
      bb += wk * v * v;
      ab += wk * u * v;
    }
    hb[0][r][q] = a;
    hb[1][r][q] = b;
    hb[2][r][q] = aa;
    hb[3][r][q] = bb;
    hb[4][r][q] = ab;
  }
  __syncthreads();
  const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
  const int gx = blockIdx.x * TS + tx, gy = blockIdx.y * TS + ty;
  float m[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < 2 * RAD + 1; ++k)
    for (int f = 0; f < 5; ++f) m[f] += win.w[k] * hb[f][ty + k][tx];
  float sval = 0.0f, l1 = 0.0f;
  if (gx < W && gy < H) {
    const float mx = m[0], my = m[1];
    const float vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
    const float A1 = 2.0f * mx * my + kC1, A2 = 2.0f * cxy + kC2;
    const float B1 = mx * mx + my * my + kC1, B2 = vx + vy + kC2;
    const float s = (A1 * A2) / (B1 * B2);
    const int64_t pix = c * HW + static_cast<int64_t>(gy) * W + gx;
    p1[pix] = s * (2.0f * my / A1 - 2.0f * my / A2 - 2.0f * mx / B1 + 2.0f * mx / B2);
    p2[pix] = -s / B2;
    p3[pix] = 2.0f * s / A2;
    sval = s;
    l1 = fabsf(sx[ty + RAD][tx + RAD] - sy[ty + RAD][tx + RAD]);
  }
  const int64_t bid = (static_cast<int64_t>(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const float ts = block_sum(sval, s_red);
  if (threadIdx.x == 0) partial_s[bid] = ts;
  __syncthreads();
  const float tl = block_sum(l1, s_red);
  if (threadIdx.x == 0) partial_l1[bid] = tl;
}

// Pass 2: dL/dx = w_l1 sign(x - y) - w_ssim [w*p1 + 2 x (w*p2) + y (w*p3)].
__global__ __launch_bounds__(256) void k_ssim_grad(const float* __restrict__ x, const float* __restrict__ y, int W,
                                                   int H, Window win, const float* __restrict__ p1,
                                                   const float* __restrict__ p2, const float* __restrict__ p3,
                                                   float w_l1, float w_ssim, float* __restrict__ grad) {
  __shared__ float sp[3][EXT][EXT];
  __shared__ float hb[3][EXT][TS];
  const int c = blockIdx.z;
  const int64_t HW = static_cast<int64_t>(W) * H;
  const int ox = blockIdx.x * TS - RAD, oy = blockIdx.y * TS - RAD;
  const float* P[3] = {p1 + c * HW, p2 + c * HW, p3 + c * HW};
  for (int i = threadIdx.x; i < EXT * EXT; i += 256) {
    const int r = i / EXT, q = i % EXT;
    const int gx = ox + q, gy = oy + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    for (int f = 0; f < 3; ++f) sp[f][r][q] = in ? P[f][static_cast<int64_t>(gy) * W + gx] : 0.0f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < EXT * TS; i += 256) {
    const int r = i / TS, q = i % TS;
    float a[3] = {0, 0, 0};
    for (int k = 0; k < 2 * RAD + 1; ++k)
      for (int f = 0; f < 3; ++f) a[f] += win.w[k] * sp[f][r][q + k];
    for (int f = 0; f < 3; ++f) hb[f][r][q] = a[f];
  }
  __syncthreads();
  const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
  const int gx = blockIdx.x * TS + tx, gy = blockIdx.y * TS + ty;
  if (gx >= W || gy >= H) return;
  float b[3] = {0, 0, 0};
  for (int k = 0; k < 2 * RAD + 1; ++k)
    for (int f = 0; f < 3; ++f) b[f] += win.w[k] * hb[f][ty + k][tx];
  const int64_t pix = c * HW + static_cast<int64_t>(gy) * W + gx;
  const float xv = x[pix], yv = y[pix];
  const float d = xv - yv;
  const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
  grad[pix] = w_l1 * sg - w_ssim * (b[0] + 2.0f * xv * b[1] + yv * b[2]);
}

// Sums the per-block partials in a fixed order: loss = a * sum(l1 parts) + b * sum(ssim parts) + c.
__global__ void k_finalize(const float* __restrict__ l1p, int64_t nl1, const float* __restrict__ sp, int64_t ns,
                           double a, double b, double c0, float* __restrict__ loss) {
  __shared__ double s_red[256];
  double acc_l = 0.0, acc_s = 0.0;
  for (int64_t i = threadIdx.x; i < nl1; i += 256) acc_l += l1p[i];
  for (int64_t i = threadIdx.x; i < ns; i += 256) acc_s += sp[i];
  s_red[threadIdx.x] = a * acc_l + b * acc_s;
  __syncthreads();
  for (int st = 128; st >= 1; st >>= 1) {
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
    blocks += ceil_div(W, TS) * ceil_div(H, TS) * 3;
  }
  if (kind == 0) return align_up(kL1Blocks * 4, 256);
  return 3 * align_up(3 * px * 4, 256) + 2 * align_up(blocks * 4, 256);
}

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
  if (kind == 0) {
    float* partial = static_cast<float*>(ws);
    hipLaunchKernelGGL(k_l1, dim3(kL1Blocks), dim3(256), 0, s, image, target, n, 1.0f / static_cast<float>(n), grad,
                       partial);
    VBM_LAUNCH_CHECK("loss_l1");
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partial, static_cast<int64_t>(kL1Blocks), partial,
                       static_cast<int64_t>(0), 1.0 / static_cast<double>(n), 0.0, 0.0, loss);
    VBM_LAUNCH_CHECK("loss_finalize");
    return VBM_OK;
  }
  Carver c(ws);
  float* p1 = c.take<float>(n);
  float* p2 = c.take<float>(n);
  float* p3 = c.take<float>(n);
  int64_t blocks = 0;
  for (int v = 0; v < n_views; ++v) blocks += ceil_div(dims[2 * v], TS) * ceil_div(dims[2 * v + 1], TS) * 3;
  float* ps = c.take<float>(blocks);
  float* pl = c.take<float>(blocks);
  const Window win = make_window();
  const float w_l1 = (1.0f - lambda) / static_cast<float>(n);
  const float w_ss = lambda / static_cast<float>(n);
  int64_t off = 0, boff = 0;
  for (int v = 0; v < n_views; ++v) {
    const int W = dims[2 * v], H = dims[2 * v + 1];
    const dim3 grid(static_cast<unsigned>(ceil_div(W, TS)), static_cast<unsigned>(ceil_div(H, TS)), 3);
    hipLaunchKernelGGL(k_ssim_maps, grid, dim3(256), 0, s, image + off, target + off, W, H, win, p1 + off, p2 + off,
                       p3 + off, ps + boff, pl + boff);
    VBM_LAUNCH_CHECK("ssim_maps");
    hipLaunchKernelGGL(k_ssim_grad, grid, dim3(256), 0, s, image + off, target + off, W, H, win, p1 + off, p2 + off,
                       p3 + off, w_l1, w_ss, grad + off);
    VBM_LAUNCH_CHECK("ssim_grad");
    off += 3 * static_cast<int64_t>(W) * H;
    boff += static_cast<int64_t>(grid.x) * grid.y * 3;
  }
  const double dn = static_cast<double>(n);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, pl, blocks, ps, blocks, (1.0 - lambda) / dn, -lambda / dn,
                     static_cast<double>(lambda), loss);
  VBM_LAUNCH_CHECK("loss_finalize");
  return VBM_OK;
}
