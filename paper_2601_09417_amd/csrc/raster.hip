// Front-to-back alpha compositing and its reverse-order backward (Sec. 3, the Gaussian mixture
// rendered by the 3DGS rasteriser cited in Sec. 4.4).
//
// Work decomposition: one wave64 per 256 pixels of a tile (a 16x16 tile is one wave, a 32x32 tile
// four independent waves, an 8x8 tile one wave with one pixel per lane), each lane owning
// PPL = 4 pixels of rows that are contiguous across the wave.  The tile's depth-sorted list is
// walked by every wave in lockstep: a Gaussian's item id and its 36-byte record are wave-uniform,
// so they are fetched with scalar loads into SGPRs and broadcast to the VALU for free -- no LDS
// staging, no workgroup barriers, and the per-Gaussian load cost is amortised over 256 pixels.
// Per-pixel updates are branch-free (predicated selects), and a wave leaves the list as soon as
// every one of its pixels has terminated.
//
// The backward walks the list in reverse from the wave's largest n_contrib, recomputes each
// pixel's transmittance from final_T by division, sums the nine partial derivatives over the lane's
// pixels in registers, reduces them across the wave with DPP row operations plus four lane reads,
// and issues one float atomic per value per (Gaussian, wave) -- only when some pixel contributed.
#include <hip/hip_runtime.h>

#include "common.h"

namespace vbm {

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

typedef __attribute__((address_space(4))) const float cfloat;
typedef __attribute__((address_space(4))) const uint32_t cuint;

template <int TILE>
struct TileCfg {
  static constexpr int kPix = TILE * TILE;
  static constexpr int kWaves = kPix >= 256 ? kPix / 256 : 1;
  static constexpr int kPPL = kPix / (64 * kWaves);  // pixels per lane
  static constexpr int kThreads = 64 * kWaves;
};

__device__ __forceinline__ int find_view(const DevView* __restrict__ views, int n_views, int tile) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_offset <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The Gaussian's exponent at one pixel, written once with explicit fused operations so the forward
// and the backward take bit-identical skip/contribute decisions.
__device__ __forceinline__ float gauss_power(const float4 a, const float conic_c, float dx, float dy) {
  const float q = fmaf(a.z * dx, dx, conic_c * dy * dy);
  return fmaf(-0.5f, q, -(a.w * dx) * dy);
}

// The 32-byte record of item `it` (mean2d.xy, conic.ab | conic.c, opacity, r, g) as two float4.
__device__ __forceinline__ void load_record(cfloat* r, uint32_t it, float4& a, float4& b) {
  const size_t o = 8 * static_cast<size_t>(it);
  a = make_float4(r[o], r[o + 1], r[o + 2], r[o + 3]);
  b = make_float4(r[o + 4], r[o + 5], r[o + 6], r[o + 7]);
}

template <int DPP_CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), DPP_CTRL, 0xF, 0xF, false));
}

// Sum over the 64 lanes (every lane must be active): quad swaps, half-row and row mirrors leave
// each 16-lane row holding its row sum; four lane reads add the rows.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}

// Measurement aid: adds the wave's evaluated / contributing (pixel, Gaussian) counts to stats[0..1].
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

template <int TILE, bool STATS>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_composite_fwd(
    const DevView* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ pair_item, const float4* __restrict__ rec, const float* __restrict__ blue,
    float* __restrict__ image, float* __restrict__ final_T, int32_t* __restrict__ n_contrib,
    unsigned long long* __restrict__ stats) {
  using C = TileCfg<TILE>;
  constexpr int PPL = C::kPPL;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int wave = static_cast<int>(threadIdx.x) >> 6;
  const int tile = blockIdx.x;
  const DevView& v = views[find_view(views, n_views, tile)];
  const int local = tile - v.tile_offset;
  const int tx = local % v.tiles_x, ty = local / v.tiles_x;
  float fx[PPL], fy[PPL], T[PPL], cr[PPL], cg[PPL], cb[PPL];
  int last[PPL];
  bool live[PPL], inside[PPL];
  int px[PPL], py[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int q = wave * (C::kPix / C::kWaves) + k * 64 + lane;
    px[k] = tx * TILE + q % TILE;
    py[k] = ty * TILE + q / TILE;
    inside[k] = px[k] < v.width && py[k] < v.height;
    live[k] = inside[k];
    fx[k] = static_cast<float>(px[k]) + 0.5f;
    fy[k] = static_cast<float>(py[k]) + 0.5f;
    T[k] = 1.0f;
    cr[k] = cg[k] = cb[k] = 0.0f;
    last[k] = 0;
  }
  const uint2 rg = ranges[tile];
  const int start = static_cast<int>(rg.x), end = static_cast<int>(rg.y);
  cuint* items = (cuint*)(pair_item);
  cfloat* recs = (cfloat*)(rec);
  cfloat* blues = (cfloat*)(blue);
  uint32_t n_eval = 0, n_used = 0;
  // Software pipeline over the list: item ids are fetched two positions ahead and records one
  // position ahead, so the scalar-load latency overlaps the current Gaussian's arithmetic.
  const int lastj = end > start ? end - 1 : start;
  // An empty list touches no pair entry; item 0 always exists, so its record is a safe dummy.
  uint32_t it_n = end > start ? items[start] : 0u;
  uint32_t it_nn = end > start ? items[min(start + 1, lastj)] : 0u;
  float4 a_n, b_n;
  load_record(recs, it_n, a_n, b_n);
  float bl_n = blues[it_n];
  for (int j = start; j < end; ++j) {
    bool any_live = false;
#pragma unroll
    for (int k = 0; k < PPL; ++k) any_live |= live[k];
    if (!__any(any_live)) break;
    const float4 a = a_n;
    const float4 b = b_n;
    const float bl = bl_n;
    it_n = it_nn;
    it_nn = items[min(j + 2, lastj)];
    load_record(recs, it_n, a_n, b_n);
    bl_n = blues[it_n];
    const int pos = j - start + 1;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const float dx = a.x - fx[k], dy = a.y - fy[k];
      const float power = gauss_power(a, b.x, dx, dy);
      const float alpha = fminf(kAlphaMax, b.y * __expf(power));
      const bool ok = live[k] && power <= 0.0f && alpha >= kAlphaMin;
      const float Tn = T[k] * (1.0f - alpha);
      const bool stop = ok && Tn < kTMin;
      const bool use = ok && !stop;
      if (STATS) {
        n_eval += live[k] ? 1u : 0u;
        n_used += use ? 1u : 0u;
      }
      live[k] = live[k] && !stop;
      const float w = use ? alpha * T[k] : 0.0f;
      cr[k] = fmaf(b.z, w, cr[k]);
      cg[k] = fmaf(b.w, w, cg[k]);
      cb[k] = fmaf(bl, w, cb[k]);
      T[k] = use ? Tn : T[k];
      last[k] = use ? pos : last[k];
    }
  }
  if (STATS) add_stats(stats, n_eval, n_used);
  const int64_t HW = static_cast<int64_t>(v.width) * v.height;
  float* img = image + 3 * static_cast<int64_t>(v.pixel_offset);
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    if (!inside[k]) continue;
    const int64_t pix = static_cast<int64_t>(py[k]) * v.width + px[k];
    img[pix] = cr[k] + T[k] * v.bg[0];
    img[HW + pix] = cg[k] + T[k] * v.bg[1];
    img[2 * HW + pix] = cb[k] + T[k] * v.bg[2];
    final_T[v.pixel_offset + pix] = T[k];
    n_contrib[v.pixel_offset + pix] = last[k];
  }
}

template <int TILE, bool STATS>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_composite_bwd(
    const DevView* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ pair_item, const float4* __restrict__ rec, const float* __restrict__ blue,
    const float* __restrict__ final_T, const int32_t* __restrict__ n_contrib, const float* __restrict__ dL_dimg,
    float* __restrict__ grad2d, int64_t n_items, unsigned long long* __restrict__ stats) {
  using C = TileCfg<TILE>;
  constexpr int PPL = C::kPPL;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int wave = static_cast<int>(threadIdx.x) >> 6;
  const int tile = blockIdx.x;
  const DevView& v = views[find_view(views, n_views, tile)];
  const int local = tile - v.tile_offset;
  const int tx = local % v.tiles_x, ty = local / v.tiles_x;
  const int64_t HW = static_cast<int64_t>(v.width) * v.height;
  float fx[PPL], fy[PPL], T[PPL], dr[PPL], dg[PPL], db[PPL];
  float accr[PPL], accg[PPL], accb[PPL], la[PPL], lr[PPL], lg[PPL], lb[PPL];
  int nc[PPL];
  int maxn = 0;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int q = wave * (C::kPix / C::kWaves) + k * 64 + lane;
    const int px = tx * TILE + q % TILE;
    const int py = ty * TILE + q / TILE;
    const bool inside = px < v.width && py < v.height;
    fx[k] = static_cast<float>(px) + 0.5f;
    fy[k] = static_cast<float>(py) + 0.5f;
    T[k] = 1.0f;
    nc[k] = 0;
    dr[k] = dg[k] = db[k] = 0.0f;
    if (inside) {
      const int64_t pix = static_cast<int64_t>(py) * v.width + px;
      T[k] = final_T[v.pixel_offset + pix];
      nc[k] = n_contrib[v.pixel_offset + pix];
      const float* g = dL_dimg + 3 * static_cast<int64_t>(v.pixel_offset);
      dr[k] = g[pix];
      dg[k] = g[HW + pix];
      db[k] = g[2 * HW + pix];
    }
    accr[k] = v.bg[0];
    accg[k] = v.bg[1];
    accb[k] = v.bg[2];
    la[k] = lr[k] = lg[k] = lb[k] = 0.0f;
    maxn = max(maxn, nc[k]);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) maxn = max(maxn, __shfl_xor(maxn, d, 64));
  const int start = static_cast<int>(ranges[tile].x);
  cuint* items = (cuint*)(pair_item);
  cfloat* recs = (cfloat*)(rec);
  cfloat* blues = (cfloat*)(blue);
  uint32_t n_eval = 0, n_used = 0;
  // Same two-deep software pipeline as the forward, walking the list backwards.
  const int top = maxn > 0 ? maxn - 1 : 0;
  uint32_t it_n = maxn > 0 ? items[start + top] : 0u;
  uint32_t it_nn = maxn > 0 ? items[start + max(top - 1, 0)] : 0u;
  float4 a_n, b_n;
  load_record(recs, it_n, a_n, b_n);
  float bl_n = blues[it_n];
  for (int j = maxn - 1; j >= 0; --j) {
    const uint32_t it = it_n;
    const float4 a = a_n;
    const float4 b = b_n;
    const float bl = bl_n;
    it_n = it_nn;
    it_nn = items[start + max(j - 2, 0)];
    load_record(recs, it_n, a_n, b_n);
    bl_n = blues[it_n];
    float power[PPL], G[PPL], alpha[PPL];
    bool c[PPL];
    bool anyc = false;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const float dx = a.x - fx[k], dy = a.y - fy[k];
      power[k] = gauss_power(a, b.x, dx, dy);
      G[k] = __expf(power[k]);
      alpha[k] = fminf(kAlphaMax, b.y * G[k]);
      c[k] = j < nc[k] && power[k] <= 0.0f && alpha[k] >= kAlphaMin;
      anyc |= c[k];
      if (STATS) {
        n_eval += j < nc[k] ? 1u : 0u;
        n_used += c[k] ? 1u : 0u;
      }
    }
    if (!__any(anyc)) continue;
    float g0 = 0, g1 = 0, g2 = 0, g3 = 0, g4 = 0, g5 = 0, g6 = 0, g7 = 0, g8 = 0;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const bool ck = c[k];
      const float dx = a.x - fx[k], dy = a.y - fy[k];
      const float Tk = ck ? T[k] * __builtin_amdgcn_rcpf(1.0f - alpha[k]) : T[k];
      T[k] = Tk;
      const float ar = la[k] * lr[k] + (1.0f - la[k]) * accr[k];
      const float ag = la[k] * lg[k] + (1.0f - la[k]) * accg[k];
      const float ab = la[k] * lb[k] + (1.0f - la[k]) * accb[k];
      accr[k] = ck ? ar : accr[k];
      accg[k] = ck ? ag : accg[k];
      accb[k] = ck ? ab : accb[k];
      const float w = ck ? alpha[k] * Tk : 0.0f;
      g6 = fmaf(w, dr[k], g6);
      g7 = fmaf(w, dg[k], g7);
      g8 = fmaf(w, db[k], g8);
      const float dL_da = Tk * (dr[k] * (b.z - ar) + dg[k] * (b.w - ag) + db[k] * (bl - ab));
      la[k] = ck ? alpha[k] : la[k];
      lr[k] = ck ? b.z : lr[k];
      lg[k] = ck ? b.w : lg[k];
      lb[k] = ck ? bl : lb[k];
      const bool unclamped = ck && b.y * G[k] <= kAlphaMax;
      const float dp = unclamped ? dL_da * alpha[k] : 0.0f;
      g5 = fmaf(unclamped ? dL_da : 0.0f, G[k], g5);
      g0 = fmaf(dp, -(a.z * dx + a.w * dy), g0);
      g1 = fmaf(dp, -(b.x * dy + a.w * dx), g1);
      g2 = fmaf(dp, -0.5f * dx * dx, g2);
      g3 = fmaf(dp, -dx * dy, g3);
      g4 = fmaf(dp, -0.5f * dy * dy, g4);
    }
    const float s[9] = {wave_sum(g0), wave_sum(g1), wave_sum(g2), wave_sum(g3), wave_sum(g4),
                        wave_sum(g5), wave_sum(g6), wave_sum(g7), wave_sum(g8)};
    if (lane < 9) {
      float x = s[0];
#pragma unroll
      for (int q = 1; q < 9; ++q) x = lane == q ? s[q] : x;
      if (x != 0.0f) unsafeAtomicAdd(&grad2d[lane * n_items + it], x);
    }
  }
  if (STATS) add_stats(stats, n_eval, n_used);
}

template <int TILE>
static vbm_status launch_fwd_t(const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges,
                               const uint32_t* pair_item, const float4* rec, const float* blue, float* image,
                               float* final_T, int32_t* n_contrib, unsigned long long* stats, hipStream_t s) {
  const dim3 block(TileCfg<TILE>::kThreads);
  if (stats)
    hipLaunchKernelGGL((k_composite_fwd<TILE, true>), dim3(n_tiles), block, 0, s, views, n_views, ranges, pair_item,
                       rec, blue, image, final_T, n_contrib, stats);
  else
    hipLaunchKernelGGL((k_composite_fwd<TILE, false>), dim3(n_tiles), block, 0, s, views, n_views, ranges, pair_item,
                       rec, blue, image, final_T, n_contrib, stats);
  VBM_LAUNCH_CHECK("composite_fwd");
  return VBM_OK;
}

template <int TILE>
static vbm_status launch_bwd_t(const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges,
                               const uint32_t* pair_item, const float4* rec, const float* blue, const float* final_T,
                               const int32_t* n_contrib, const float* dL_dimg, float* grad2d, int64_t n_items,
                               unsigned long long* stats, hipStream_t s) {
  const dim3 block(TileCfg<TILE>::kThreads);
  if (stats)
    hipLaunchKernelGGL((k_composite_bwd<TILE, true>), dim3(n_tiles), block, 0, s, views, n_views, ranges, pair_item,
                       rec, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats);
  else
    hipLaunchKernelGGL((k_composite_bwd<TILE, false>), dim3(n_tiles), block, 0, s, views, n_views, ranges, pair_item,
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
