// Front-to-back alpha compositing and its reverse-order backward (Sec. 3, the Gaussian mixture
// rendered by the 3DGS rasteriser cited in Sec. 4.4).
//
// One workgroup per (view, tile), one thread per pixel.  The tile's depth-sorted list is staged
// through LDS in batches of one record per thread (mean2d, conic, opacity, rgb); each pixel walks
// the batch in order, and the workgroup leaves as soon as every pixel has terminated
// (__syncthreads_count).  The backward starts from the largest n_contrib of the tile, walks the list
// in reverse, recomputes each pixel's transmittance from final_T by division, reduces the nine
// per-Gaussian partial derivatives across each wave and accumulates the four waves' sums in LDS,
// so a tile issues at most nine global atomics per Gaussian.
#include <hip/hip_runtime.h>

#include "common.h"

namespace vbm {

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

__device__ __forceinline__ int find_view(const DevView* __restrict__ views, int n_views, int tile) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_offset <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Measurement aid: adds the block's evaluated / contributing (pixel, Gaussian) counts to stats[0..1].
__device__ __forceinline__ void add_stats(unsigned long long* stats, uint32_t n_eval, uint32_t n_used) {
  unsigned long long e = n_eval, u = n_used;
  for (int d = 32; d >= 1; d >>= 1) {
    e += __shfl_xor(e, d, 64);
    u += __shfl_xor(u, d, 64);
  }
  if (lane_id() == 0) {
    atomicAdd(&stats[0], e);
    atomicAdd(&stats[1], u);
  }
}

template <int TILE>
__global__ __launch_bounds__(TILE* TILE) void k_composite_fwd(const DevView* __restrict__ views, int n_views,
                                                               const uint2* __restrict__ ranges,
                                                               const uint32_t* __restrict__ pair_item,
                                                               const float4* __restrict__ rec,
                                                               const float* __restrict__ blue,
                                                               float* __restrict__ image, float* __restrict__ final_T,
                                                               int32_t* __restrict__ n_contrib,
                                                               unsigned long long* __restrict__ stats) {
  constexpr int NT = TILE * TILE;
  __shared__ float4 sA[NT];
  __shared__ float4 sB[NT];
  __shared__ float sBlue[NT];
  uint32_t n_eval = 0, n_used = 0;
  const int tile = blockIdx.x;
  const DevView& v = views[find_view(views, n_views, tile)];
  const int local = tile - v.tile_offset;
  const int tx = local % v.tiles_x, ty = local / v.tiles_x;
  const int px = tx * TILE + static_cast<int>(threadIdx.x) % TILE;
  const int py = ty * TILE + static_cast<int>(threadIdx.x) / TILE;
  const bool inside = px < v.width && py < v.height;
  const float fx = static_cast<float>(px) + 0.5f, fy = static_cast<float>(py) + 0.5f;
  const uint2 rg = ranges[tile];
  const int start = static_cast<int>(rg.x), end = static_cast<int>(rg.y);
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  int last = 0;
  bool done = !inside;
  for (int base = start; base < end; base += NT) {
    if (__syncthreads_count(done) == NT) break;
    const int idx = base + static_cast<int>(threadIdx.x);
    if (idx < end) {
      const uint32_t it = pair_item[idx];
      sA[threadIdx.x] = rec[2 * static_cast<int64_t>(it)];
      sB[threadIdx.x] = rec[2 * static_cast<int64_t>(it) + 1];
      sBlue[threadIdx.x] = blue[it];
    }
    __syncthreads();
    const int cnt = min(NT, end - base);
    for (int j = 0; j < cnt && !done; ++j) {
      const float4 a = sA[j];
      const float4 b = sB[j];
      const float dx = a.x - fx, dy = a.y - fy;
      const float power = -0.5f * (a.z * dx * dx + b.x * dy * dy) - a.w * dx * dy;
      ++n_eval;
      if (power > 0.0f) continue;
      const float alpha = fminf(kAlphaMax, b.y * __expf(power));
      if (alpha < kAlphaMin) continue;
      const float Tn = T * (1.0f - alpha);
      if (Tn < kTMin) {
        done = true;
        break;
      }
      const float w = alpha * T;
      cr += b.z * w;
      cg += b.w * w;
      cb += sBlue[j] * w;
      T = Tn;
      last = base + j - start + 1;
      ++n_used;
    }
  }
  if (stats) add_stats(stats, n_eval, n_used);
  if (inside) {
    const int64_t HW = static_cast<int64_t>(v.width) * v.height;
    const int64_t pix = static_cast<int64_t>(py) * v.width + px;
    float* img = image + 3 * static_cast<int64_t>(v.pixel_offset);
    img[pix] = cr + T * v.bg[0];
    img[HW + pix] = cg + T * v.bg[1];
    img[2 * HW + pix] = cb + T * v.bg[2];
    final_T[v.pixel_offset + pix] = T;
    n_contrib[v.pixel_offset + pix] = last;
  }
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

template <int TILE>
__global__ __launch_bounds__(TILE* TILE) void k_composite_bwd(const DevView* __restrict__ views, int n_views,
                                                               const uint2* __restrict__ ranges,
                                                               const uint32_t* __restrict__ pair_item,
                                                               const float4* __restrict__ rec,
                                                               const float* __restrict__ blue,
                                                               const float* __restrict__ final_T,
                                                               const int32_t* __restrict__ n_contrib,
                                                               const float* __restrict__ dL_dimg,
                                                               float* __restrict__ grad2d, int64_t n_items,
                                                               unsigned long long* __restrict__ stats) {
  uint32_t n_eval = 0, n_used = 0;
  constexpr int NT = TILE * TILE;
  __shared__ float4 sA[NT];
  __shared__ float4 sB[NT];
  __shared__ float sBlue[NT];
  __shared__ uint32_t sItem[NT];
  __shared__ float sG[9][NT];
  __shared__ int sMax;
  const int tile = blockIdx.x;
  const DevView& v = views[find_view(views, n_views, tile)];
  const int local = tile - v.tile_offset;
  const int tx = local % v.tiles_x, ty = local / v.tiles_x;
  const int px = tx * TILE + static_cast<int>(threadIdx.x) % TILE;
  const int py = ty * TILE + static_cast<int>(threadIdx.x) / TILE;
  const bool inside = px < v.width && py < v.height;
  const float fx = static_cast<float>(px) + 0.5f, fy = static_cast<float>(py) + 0.5f;
  const int start = static_cast<int>(ranges[tile].x);
  float T = 1.0f;
  int nc = 0;
  float dr = 0.0f, dg = 0.0f, db = 0.0f;
  if (inside) {
    const int64_t HW = static_cast<int64_t>(v.width) * v.height;
    const int64_t pix = static_cast<int64_t>(py) * v.width + px;
    T = final_T[v.pixel_offset + pix];
    nc = n_contrib[v.pixel_offset + pix];
    const float* g = dL_dimg + 3 * static_cast<int64_t>(v.pixel_offset);
    dr = g[pix];
    dg = g[HW + pix];
    db = g[2 * HW + pix];
  }
  if (threadIdx.x == 0) sMax = 0;
  __syncthreads();
  atomicMax(&sMax, nc);
  __syncthreads();
  const int maxn = sMax;
  float accr = v.bg[0], accg = v.bg[1], accb = v.bg[2];
  float last_a = 0.0f, last_r = 0.0f, last_g = 0.0f, last_b = 0.0f;
  for (int bend = maxn; bend > 0; bend -= NT) {
    const int bstart = bend > NT ? bend - NT : 0;
    const int cnt = bend - bstart;
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < cnt) {
      const uint32_t it = pair_item[start + bstart + threadIdx.x];
      sItem[threadIdx.x] = it;
      sA[threadIdx.x] = rec[2 * static_cast<int64_t>(it)];
      sB[threadIdx.x] = rec[2 * static_cast<int64_t>(it) + 1];
      sBlue[threadIdx.x] = blue[it];
#pragma unroll
      for (int k = 0; k < 9; ++k) sG[k][threadIdx.x] = 0.0f;
    }
    __syncthreads();
    for (int j = cnt - 1; j >= 0; --j) {
      const int pos = bstart + j;
      float g[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) g[k] = 0.0f;
      bool contrib = false;
      if (pos < nc) {
        ++n_eval;
        const float4 a = sA[j];
        const float4 b = sB[j];
        const float dx = a.x - fx, dy = a.y - fy;
        const float power = -0.5f * (a.z * dx * dx + b.x * dy * dy) - a.w * dx * dy;
        if (power <= 0.0f) {
          const float G = __expf(power);
          const float og = b.y * G;
          const float alpha = fminf(kAlphaMax, og);
          if (alpha >= kAlphaMin) {
            contrib = true;
            ++n_used;
            T = T / (1.0f - alpha);
            accr = last_a * last_r + (1.0f - last_a) * accr;
            accg = last_a * last_g + (1.0f - last_a) * accg;
            accb = last_a * last_b + (1.0f - last_a) * accb;
            const float cr = b.z, cg = b.w, cb = sBlue[j];
            const float w = alpha * T;
            g[6] = w * dr;
            g[7] = w * dg;
            g[8] = w * db;
            const float dL_da = T * (dr * (cr - accr) + dg * (cg - accg) + db * (cb - accb));
            last_a = alpha;
            last_r = cr;
            last_g = cg;
            last_b = cb;
            if (og <= kAlphaMax) {
              g[5] = dL_da * G;
              const float dp = dL_da * alpha;
              g[0] = dp * -(a.z * dx + a.w * dy);
              g[1] = dp * -(b.x * dy + a.w * dx);
              g[2] = dp * (-0.5f * dx * dx);
              g[3] = dp * (-dx * dy);
              g[4] = dp * (-0.5f * dy * dy);
            }
          }
        }
      }
      if (__any(contrib)) {
#pragma unroll
        for (int k = 0; k < 9; ++k) g[k] = wave_sum(g[k]);
        if (lane_id() == 0) {
#pragma unroll
          for (int k = 0; k < 9; ++k)
            if (g[k] != 0.0f) atomicAdd(&sG[k][j], g[k]);
        }
      }
    }
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < cnt) {
      const uint32_t it = sItem[threadIdx.x];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const float x = sG[k][threadIdx.x];
        if (x != 0.0f) unsafeAtomicAdd(&grad2d[k * n_items + it], x);
      }
    }
  }
  if (stats) add_stats(stats, n_eval, n_used);
}

template <int TILE>
static vbm_status launch_fwd_t(const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges,
                               const uint32_t* pair_item, const float4* rec, const float* blue, float* image,
                               float* final_T, int32_t* n_contrib, unsigned long long* stats, hipStream_t s) {
  hipLaunchKernelGGL(k_composite_fwd<TILE>, dim3(n_tiles), dim3(TILE * TILE), 0, s, views, n_views, ranges, pair_item,
                     rec, blue, image, final_T, n_contrib, stats);
  VBM_LAUNCH_CHECK("composite_fwd");
  return VBM_OK;
}

template <int TILE>
static vbm_status launch_bwd_t(const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges,
                               const uint32_t* pair_item, const float4* rec, const float* blue, const float* final_T,
                               const int32_t* n_contrib, const float* dL_dimg, float* grad2d, int64_t n_items,
                               unsigned long long* stats, hipStream_t s) {
  hipLaunchKernelGGL(k_composite_bwd<TILE>, dim3(n_tiles), dim3(TILE * TILE), 0, s, views, n_views, ranges, pair_item,
                     rec, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats);
  VBM_LAUNCH_CHECK("composite_bwd");
  return VBM_OK;
}

vbm_status launch_composite_fwd(int tile, const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges,
                                const uint32_t* pair_item, const float4* rec, const float* blue, float* image,
                                float* final_T, int32_t* n_contrib, unsigned long long* stats, hipStream_t s) {
  switch (tile) {
    case 8: return launch_fwd_t<8>(views, n_views, n_tiles, ranges, pair_item, rec, blue, image, final_T, n_contrib, stats, s);
    case 16: return launch_fwd_t<16>(views, n_views, n_tiles, ranges, pair_item, rec, blue, image, final_T, n_contrib, stats, s);
    case 32: return launch_fwd_t<32>(views, n_views, n_tiles, ranges, pair_item, rec, blue, image, final_T, n_contrib, stats, s);
  }
  set_error("unsupported tile size %d", tile);
  return VBM_ERR_UNSUPPORTED;
}

vbm_status launch_composite_bwd(int tile, const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges,
                                const uint32_t* pair_item, const float4* rec, const float* blue, const float* final_T,
                                const int32_t* n_contrib, const float* dL_dimg, float* grad2d, int64_t n_items,
                                unsigned long long* stats, hipStream_t s) {
  switch (tile) {
    case 8: return launch_bwd_t<8>(views, n_views, n_tiles, ranges, pair_item, rec, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats, s);
    case 16: return launch_bwd_t<16>(views, n_views, n_tiles, ranges, pair_item, rec, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats, s);
    case 32: return launch_bwd_t<32>(views, n_views, n_tiles, ranges, pair_item, rec, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats, s);
  }
  set_error("unsupported tile size %d", tile);
  return VBM_ERR_UNSUPPORTED;
}

}  // namespace vbm
