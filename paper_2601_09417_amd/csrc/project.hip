// EWA projection, binning and the projection backward of the fine-tuning renderer (Sec. 4.4
// fine-tunes with the 3DGS rasteriser the paper cites; Sec. 3 defines the Gaussian set).
//
// Every decision that fixes the pair lists -- camera depth, culling, the 2D covariance, the radius
// and the tile rectangle -- is computed in float32 in one fixed order with contraction disabled and
// correctly rounded division and square root, so that the lists are reproducible bit for bit by
// any implementation following the same order.
#include <hip/hip_runtime.h>

#include "block_scan.h"
#include "common.h"

#pragma clang fp contract(off)

namespace vbm {

struct ProjResult {
  float depth;
  float px, py;
  float ca, cb, cc;
  uint32_t x0, y0, x1, y1;
  bool visible;
};

__device__ __forceinline__ void rot_from_quat(float qw, float qx, float qy, float qz, float Rq[3][3], float qn[4]) {
  const float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  const float nq = sqrt_rn_f32(n2);
  const float w = __fdiv_rn(qw, nq), x = __fdiv_rn(qx, nq), y = __fdiv_rn(qy, nq), z = __fdiv_rn(qz, nq);
  qn[0] = w;
  qn[1] = x;
  qn[2] = y;
  qn[3] = z;
  const float xx = x * x, yy = y * y, zz = z * z;
  const float xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  Rq[0][0] = 1.0f - 2.0f * (yy + zz);
  Rq[0][1] = 2.0f * (xy - wz);
  Rq[0][2] = 2.0f * (xz + wy);
  Rq[1][0] = 2.0f * (xy + wz);
  Rq[1][1] = 1.0f - 2.0f * (xx + zz);
  Rq[1][2] = 2.0f * (yz - wx);
  Rq[2][0] = 2.0f * (xz - wy);
  Rq[2][1] = 2.0f * (yz + wx);
  Rq[2][2] = 1.0f - 2.0f * (xx + yy);
}

// Opacity-aware footprint.  A pixel receives alpha = o exp(-q/2) >= 1/255 only where
// q = d^T Sigma2^-1 d <= 2 ln(255 o).  tau bounds that from above without transcendental functions,
// ln x <= 32 (x^(1/32) - 1) (five correctly rounded square roots), widened by 1% and 0.01 to absorb
// the float32 evaluation error of the compositing kernels; a Gaussian with o < 1/255 reaches nothing.
__device__ __forceinline__ float footprint_tau(float o) {
  float y = 255.0f * o;
  y = sqrt_rn_f32(y);
  y = sqrt_rn_f32(y);
  y = sqrt_rn_f32(y);
  y = sqrt_rn_f32(y);
  y = sqrt_rn_f32(y);
  const float u = 32.0f * (y - 1.0f);
  return (2.0f * u) * 1.01f + 0.01f;
}

__device__ __forceinline__ float quad_form(float A, float B2, float C, float dx, float dy) {
  return ((A * dx) * dx + (B2 * dx) * dy) + (C * dy) * dy;
}

// True when the footprint {q <= tau} can reach a pixel centre of the tile (tx, ty): the minimum of
// q over the rectangle spanned by the tile's pixel centres (clipped to the image) is <= tau.  The
// minimum is 0 with the centre inside; otherwise it lies on one of the four edges, where q is a
// 1D quadratic minimised at a clamped stationary point: dy = dx nBC on a vertical edge and
// dx = dy nBA on a horizontal one, with nBC = -(B/C) and nBA = -(B/A) rounded once per Gaussian.
__device__ __forceinline__ bool tile_reached(float mx, float my, float A, float B, float C, float nBA, float nBC,
                                             float tau, int tx, int ty, int tile, int W, int H) {
  const float X0 = static_cast<float>(tx * tile) + 0.5f;
  const float X1 = static_cast<float>(min((tx + 1) * tile, W)) - 0.5f;
  const float Y0 = static_cast<float>(ty * tile) + 0.5f;
  const float Y1 = static_cast<float>(min((ty + 1) * tile, H)) - 0.5f;
  const float dx0 = X0 - mx, dx1 = X1 - mx, dy0 = Y0 - my, dy1 = Y1 - my;
  if (dx0 <= 0.0f && dx1 >= 0.0f && dy0 <= 0.0f && dy1 >= 0.0f) return true;
  const float B2 = 2.0f * B;
  // Clamps to [d0, d1] with d0 <= d1 (the centres span at least one pixel): for finite values the
  // median of three is min(max(v, d0), d1), in one instruction.
  const float ya = __builtin_amdgcn_fmed3f(dx0 * nBC, dy0, dy1);
  const float yb = __builtin_amdgcn_fmed3f(dx1 * nBC, dy0, dy1);
  const float xa = __builtin_amdgcn_fmed3f(dy0 * nBA, dx0, dx1);
  const float xb = __builtin_amdgcn_fmed3f(dy1 * nBA, dx0, dx1);
  const float q = fminf(fminf(quad_form(A, B2, C, dx0, ya), quad_form(A, B2, C, dx1, yb)),
                        fminf(quad_form(A, B2, C, xa, dy0), quad_form(A, B2, C, xb, dy1)));
  return q <= tau;
}

// Lane groups of a 16x16 tile are its 4-row bands.  The footprint {q <= tau} spans the pixel rows
// whose centre lies within ey of the mean, ey^2 = tau A / (A C - B^2) for the conic (A, B, C) as
// rounded (the determinant in float64, where both products are exact, so a thin ellipse loses
// nothing to cancellation), widened by 0.2% and 0.1 pixel.  Returns the first band it can reach in
// the rectangle's first tile row y0 (bits 12..13) and the last band in its last tile row y1 - 1
// (bits 28..29), to be ORed into the bin entry's row word (tile rows stay below 2^12); every band
// of the rows between can be reached.
__device__ __forceinline__ uint32_t band_bits(float py, float A, float B, float C, float tau, uint32_t y0,
                                              uint32_t y1) {
  constexpr uint32_t kAll = 3u << 28;   // first band 0, last band 3
  const double den = fma(static_cast<double>(A), static_cast<double>(C),
                         -(static_cast<double>(B) * static_cast<double>(B)));
  const float e2 = tau * A / static_cast<float>(den);
  if (!(den > 0.0 && e2 >= 0.0f && e2 < 1e30f)) return kAll;
  const float ey = sqrtf(e2) * 1.002f + 0.1f;
  const float f = floorf((py - ey - 0.5f - 16.0f * static_cast<float>(y0)) * 0.25f);
  const float l = floorf((py + ey - 0.5f - 16.0f * static_cast<float>(y1 - 1)) * 0.25f);
  const uint32_t kf = static_cast<uint32_t>(fminf(fmaxf(f, 0.0f), 3.0f));
  const uint32_t kl = static_cast<uint32_t>(fminf(fmaxf(l, 0.0f), 3.0f));
  return (kf << 12) | (kl << 28);
}

// The pair-value group mask (bits kItemBits..) of tile row r (0-based) of a rectangle h rows tall
// whose bin entry row word is by.
__device__ __forceinline__ uint32_t band_mask(uint32_t by, uint32_t r, uint32_t h) {
  uint32_t m = 0xFu;
  if (r == 0) m &= 0xFu << ((by >> 12) & 3u);
  if (r + 1 == h) m &= 0xFu >> (3u - ((by >> 28) & 3u));
  return (m & 0xFu) << kItemBits;
}

// Rectangles of more than this many tiles are tested by a whole wave (64 tiles per round) after
// the per-thread pass of the block, so that one large footprint does not hold up 63 lanes.
constexpr uint32_t kSmallRect = 32;

// A large rectangle's reached tiles are kept as the projection's 64-tile ballots, one 64-bit word
// per round, in a bump-allocated word buffer that the emission reads back; bin.z holds the item's
// first word, or kNoWords when the buffer was full and the emission repeats the tests.
constexpr uint32_t kNoWords = 0xFFFFFFFFu;

// Column and row of tile t (row-major) of a rectangle w tiles wide, with inv_w = 1/w rounded: the
// float quotient is off by at most one and corrected.
__device__ __forceinline__ void rect_tile(uint32_t t, uint32_t w, float inv_w, uint32_t& tx, uint32_t& ty) {
  int r = static_cast<int>((static_cast<float>(t) + 0.5f) * inv_w);
  int c = static_cast<int>(t) - r * static_cast<int>(w);
  if (c < 0) {
    --r;
    c += static_cast<int>(w);
  } else if (c >= static_cast<int>(w)) {
    ++r;
    c -= static_cast<int>(w);
  }
  tx = static_cast<uint32_t>(c);
  ty = static_cast<uint32_t>(r);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ ProjResult project_one(const DevView& v, int tile, float mx, float my, float mz, float sx,
                                                  float sy, float sz, float qw, float qx, float qy, float qz,
                                                  float opacity) {
  ProjResult o;
  const float* R = v.R;
  const float Xc = ((R[0] * mx + R[1] * my) + R[2] * mz) + v.t[0];
  const float Yc = ((R[3] * mx + R[4] * my) + R[5] * mz) + v.t[1];
  const float Zc = ((R[6] * mx + R[7] * my) + R[8] * mz) + v.t[2];
  bool vis = Zc > v.near_plane;
  float Rq[3][3], qn[4];
  rot_from_quat(qw, qx, qy, qz, Rq, qn);
  const float s[3] = {sx, sy, sz};
  float M[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[i][k] = Rq[i][k] * s[k];
  const float limx = v.lim_x, limy = v.lim_y;
  const float txz = __fdiv_rn(Xc, Zc);
  const float tyz = __fdiv_rn(Yc, Zc);
  const float Xt = fminf(limx, fmaxf(-limx, txz)) * Zc;
  const float Yt = fminf(limy, fmaxf(-limy, tyz)) * Zc;
  const float z2 = Zc * Zc;
  const float J00 = __fdiv_rn(v.fx, Zc);
  const float J02 = -__fdiv_rn(v.fx * Xt, z2);
  const float J11 = __fdiv_rn(v.fy, Zc);
  const float J12 = -__fdiv_rn(v.fy * Yt, z2);
  float A0[3], A1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    A0[k] = J00 * R[k] + J02 * R[6 + k];
    A1[k] = J11 * R[3 + k] + J12 * R[6 + k];
  }
  float V0[3], V1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    V0[k] = (A0[0] * M[0][k] + A0[1] * M[1][k]) + A0[2] * M[2][k];
    V1[k] = (A1[0] * M[0][k] + A1[1] * M[1][k]) + A1[2] * M[2][k];
  }
  const float a = ((V0[0] * V0[0] + V0[1] * V0[1]) + V0[2] * V0[2]) + 0.3f;
  const float b = (V0[0] * V1[0] + V0[1] * V1[1]) + V0[2] * V1[2];
  const float c = ((V1[0] * V1[0] + V1[1] * V1[1]) + V1[2] * V1[2]) + 0.3f;
  const float det = a * c - b * b;
  vis = vis && det > 0.0f;
  const float mid = 0.5f * (a + c);
  const float disc = fmaxf(0.1f, mid * mid - det);
  const float lam = mid + sqrt_rn_f32(disc);
  const float r = ceilf(3.0f * sqrt_rn_f32(lam));
  const float px = v.fx * txz + v.cx;
  const float py = v.fy * tyz + v.cy;
  // the tile edge is a power of two, so multiplying by its reciprocal is the exact quotient
  const float iT = 1.0f / static_cast<float>(tile);
  const float fx0 = fminf(fmaxf(floorf((px - r) * iT), 0.0f), static_cast<float>(v.tiles_x));
  const float fx1 = fminf(fmaxf(floorf((px + r) * iT) + 1.0f, 0.0f), static_cast<float>(v.tiles_x));
  const float fy0 = fminf(fmaxf(floorf((py - r) * iT), 0.0f), static_cast<float>(v.tiles_y));
  const float fy1 = fminf(fmaxf(floorf((py + r) * iT) + 1.0f, 0.0f), static_cast<float>(v.tiles_y));
  vis = vis && isfinite(px) && isfinite(py) && isfinite(r) && opacity >= 1.0f / 255.0f;
  o.x0 = vis ? static_cast<uint32_t>(fx0) : 0u;
  o.x1 = vis ? static_cast<uint32_t>(fx1) : 0u;
  o.y0 = vis ? static_cast<uint32_t>(fy0) : 0u;
  o.y1 = vis ? static_cast<uint32_t>(fy1) : 0u;
  o.visible = vis && (o.x1 > o.x0) && (o.y1 > o.y0);
  o.depth = Zc;
  o.px = px;
  o.py = py;
  o.ca = __fdiv_rn(c, det);
  o.cb = -__fdiv_rn(b, det);
  o.cc = __fdiv_rn(a, det);
  return o;
}

// grid: x over Gaussians of the view's scene, y over views.  Writes the per-item records and the
// visibility flag consumed by the compaction scan.  Each thread projects one item; the reached tiles
// are then counted block-wide so that the footprint tests do not diverge with the rectangle sizes:
// the tiles of all rectangles of at most 32 tiles are numbered consecutively (a block prefix sum of
// their areas, an LDS map from test number to item) and shared round-robin by the block's threads,
// which set the reached bits of the items' row-major masks; larger rectangles are tested by whole
// waves, 64 tiles per round.
__global__ __launch_bounds__(256) void k_project(const DevView* __restrict__ views, int tile, vbm_gaussians_c g,
                                                 float* __restrict__ depth, uint32_t* __restrict__ ntiles,
                                                 float4* __restrict__ rec, float4* __restrict__ coef,
                                                 float* __restrict__ blue, uint32_t* __restrict__ vis_flag,
                                                 uint4* __restrict__ bin, unsigned long long* __restrict__ word_count,
                                                 unsigned long long* __restrict__ words, uint32_t word_cap) {
  __shared__ float s_par[8][256];      // per thread: mean2d.xy, conic A B C, tau, nBA, nBC
  __shared__ uint32_t s_org[256];      // rectangle origin x0 | y0 << 16
  __shared__ uint32_t s_w[256];        // rectangle width
  __shared__ uint32_t s_h[256];        // rectangle height
  __shared__ float s_invw[256];        // 1 / width
  __shared__ uint32_t s_start[256];    // first test number of a small rectangle
  __shared__ uint32_t s_mask[256];     // reached-tile mask of a small rectangle
  __shared__ uint8_t s_map[256 * kSmallRect];   // test number -> thread of its rectangle
  __shared__ uint32_t s_q[256];        // threads with a large rectangle
  __shared__ uint32_t s_wofs[256];     // first ballot word of a large rectangle, within the block's
  __shared__ uint32_t s_band[256];     // band bits of a large rectangle (band_bits)
  __shared__ uint32_t s_n, s_words;
  __shared__ unsigned long long s_wbase;
  if (threadIdx.x == 0) {
    s_n = 0;
    s_words = 0;
  }
  s_mask[threadIdx.x] = 0u;
  __syncthreads();
  const DevView& v = views[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int64_t item = v.item_offset + i;
  uint32_t small_area = 0, rx = 0, ry = 0, band = 3u << 28;
  bool deferred = false;
  if (i < v.n_gauss) {
    const int64_t gi = v.gauss_offset + i;
    const int64_t S = g.stride;
    const float op = g.opacity[gi];
    const ProjResult p = project_one(v, tile, g.means[gi], g.means[S + gi], g.means[2 * S + gi], g.scales[gi],
                                     g.scales[S + gi], g.scales[2 * S + gi], g.quats[gi], g.quats[S + gi],
                                     g.quats[2 * S + gi], g.quats[3 * S + gi], op);
    if (p.visible) {
      const float par[8] = {p.px, p.py, p.ca, p.cb, p.cc, footprint_tau(op), -__fdiv_rn(p.cb, p.ca),
                            -__fdiv_rn(p.cb, p.cc)};
#pragma unroll
      for (int k = 0; k < 8; ++k) s_par[k][threadIdx.x] = par[k];
      s_org[threadIdx.x] = p.x0 | (p.y0 << 16);
      s_w[threadIdx.x] = p.x1 - p.x0;
      s_h[threadIdx.x] = p.y1 - p.y0;
      s_invw[threadIdx.x] = 1.0f / static_cast<float>(p.x1 - p.x0);
      const uint32_t area = (p.x1 - p.x0) * (p.y1 - p.y0);
      if (tile == 16) band = band_bits(p.py, p.ca, p.cb, p.cc, par[5], p.y0, p.y1);
      s_band[threadIdx.x] = band;
      if (area <= kSmallRect) {
        small_area = area;
      } else {
        deferred = true;
        s_q[atomicAdd(&s_n, 1u)] = threadIdx.x;
        s_wofs[threadIdx.x] = atomicAdd(&s_words, (area + 63u) >> 6);
      }
    }
    depth[item] = p.visible ? p.depth : 0.0f;
    rx = p.x0 | (p.x1 << 16);
    ry = p.y0 | (p.y1 << 16);
    rec[item] = make_float4(p.ca, p.cb, p.cc, op);
    // Compositing record: the exponent in base 2 with log2(opacity) folded in,
    // e2 = hA dx^2 + hB dx dy + hC dy^2 + log2(o) = log2(o) - (A dx^2 + 2 B dx dy + C dy^2) log2(e) / 2.
    constexpr float kLog2e = 1.44269504088896341f;
    coef[2 * item] = make_float4(p.px, p.py, (-0.5f * kLog2e) * p.ca, -kLog2e * p.cb);
    coef[2 * item + 1] =
        make_float4((-0.5f * kLog2e) * p.cc, p.visible ? __log2f(op) : 0.0f, g.rgb[gi], g.rgb[S + gi]);
    blue[item] = g.rgb[2 * S + gi];
  }
  uint32_t n_tests;
  const uint32_t start = block_excl_scan(small_area, &n_tests);
  s_start[threadIdx.x] = start;
  for (uint32_t k = 0; k < small_area; ++k) s_map[start + k] = static_cast<uint8_t>(threadIdx.x);
  __syncthreads();
  // One allocation per block for the ballot words of its large rectangles; its result is published
  // after this thread's tests, so that the round trip of the atomic overlaps them.
  unsigned long long wbase = 0;
  if (threadIdx.x == 0 && s_words) wbase = atomicAdd(word_count, static_cast<unsigned long long>(s_words));
  for (uint32_t t = threadIdx.x; t < n_tests; t += 256) {
    const uint32_t o = s_map[t];
    const uint32_t k = t - s_start[o];
    uint32_t tx, ty;
    rect_tile(k, s_w[o], s_invw[o], tx, ty);
    const uint32_t org = s_org[o];
    if (tile_reached(s_par[0][o], s_par[1][o], s_par[2][o], s_par[3][o], s_par[4][o], s_par[6][o], s_par[7][o],
                     s_par[5][o], static_cast<int>((org & 0xFFFFu) + tx), static_cast<int>((org >> 16) + ty), tile,
                     v.width, v.height))
      atomicOr(&s_mask[o], 1u << k);
  }
  if (threadIdx.x == 0) s_wbase = wbase;
  __syncthreads();
  if (i < v.n_gauss && !deferred) {
    // small or invisible rectangles here; a large one is completed below by the wave that tests it
    const uint32_t mask = small_area ? s_mask[threadIdx.x] : 0u;
    const uint32_t nt = static_cast<uint32_t>(__popc(mask));
    bin[item] = make_uint4(rx, ry | band, mask, nt);
    ntiles[item] = nt;
    vis_flag[item] = nt ? 1u : 0u;
  }
  const uint32_t n_def = s_n;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  for (uint32_t d = threadIdx.x >> 6; d < n_def; d += 4) {
    const uint32_t o = s_q[d];
    const uint32_t org = s_org[o];
    const uint32_t x0 = org & 0xFFFFu, y0 = org >> 16;
    const int64_t it = v.item_offset + static_cast<int64_t>(blockIdx.x) * 256 + o;
    const uint32_t w = s_w[o], h = s_h[o];
    const uint32_t area = w * h;
    const float inv_w = s_invw[o];
    const unsigned long long first = s_wbase + s_wofs[o];
    const bool keep = first + ((area + 63u) >> 6) <= word_cap;
    uint32_t nt = 0;
    for (uint32_t t0 = 0; t0 < area; t0 += 64) {
      const uint32_t t = t0 + static_cast<uint32_t>(lane);
      uint32_t tx, ty;
      rect_tile(t, w, inv_w, tx, ty);
      const bool hit = t < area && tile_reached(s_par[0][o], s_par[1][o], s_par[2][o], s_par[3][o], s_par[4][o],
                                                s_par[6][o], s_par[7][o], s_par[5][o], static_cast<int>(x0 + tx),
                                                static_cast<int>(y0 + ty), tile, v.width, v.height);
      const uint64_t m = __ballot(hit);
      nt += static_cast<uint32_t>(__popcll(m));
      if (keep && lane == 0) words[first + (t0 >> 6)] = m;
    }
    if (lane == 0) {
      ntiles[it] = nt;
      vis_flag[it] = nt ? 1u : 0u;
      bin[it] = make_uint4(x0 | ((x0 + w) << 16), (y0 | ((y0 + h) << 16)) | s_band[o],
                           keep ? static_cast<uint32_t>(first) : kNoWords, nt);
    }
  }
}

// Stable compaction of visible items into (view << 32 | depth bits, item) pairs.
__global__ __launch_bounds__(256) void k_compact_visible(const DevView* __restrict__ views,
                                                         const uint32_t* __restrict__ ntiles,
                                                         const float* __restrict__ depth,
                                                         const uint32_t* __restrict__ pos,
                                                         uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const DevView& v = views[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= v.n_gauss) return;
  const int64_t item = v.item_offset + i;
  if (ntiles[item] == 0) return;
  const uint32_t p = pos[item];
  keys[p] = __float_as_uint(depth[item]);   // depth > near plane > 0: sign bit 0
  vals[p] = static_cast<uint32_t>(item);
}

// The view an item belongs to: the last view whose first item is at or below it (views hold
// consecutive item ranges in view order; a view with no items shares its start with the next).
__device__ __forceinline__ int view_of_item(const DevView* __restrict__ views, int n_views, uint32_t item) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (static_cast<uint32_t>(views[mid].item_offset) <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The depth-sorted items' bin entries (rectangle, reach mask or first ballot word, tile count),
// gathered once into sorted order for the emission, and their tile counts for the pair offsets.
__global__ __launch_bounds__(256) void k_gather_bins(const uint32_t* __restrict__ vals,
                                                     const uint4* __restrict__ bin,
                                                     const uint32_t* __restrict__ counters, int64_t n_max,
                                                     uint32_t* __restrict__ out, uint4* __restrict__ sorted_bin) {
  const int64_t n = min(static_cast<int64_t>(counters[0]), n_max);
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * 256) {
    const uint4 b = bin[vals[p]];
    sorted_bin[p] = b;
    out[p] = b.w;
  }
}

// Writes each visible item's tiles in the items' depth order (views interleaved; the stable tile
// sort that follows yields (tile, depth, item)).  Pairs past the capacity are dropped and flagged.
// Rectangles of at most 32 tiles walk the projection's reach mask per thread; larger ones are
// queued in the block and emitted by whole waves afterwards (64 tiles per round, positions from
// the ballot of reached tiles).  Each pair value carries the lane groups (row bands) of its tile
// that the footprint can reach (band_mask).
__global__ __launch_bounds__(256) void k_emit(const DevView* __restrict__ views, int n_views,
                                              const uint32_t* __restrict__ vals, const uint32_t* __restrict__ offs,
                                              const uint4* __restrict__ sorted_bin, const float4* __restrict__ rec,
                                              const float4* __restrict__ coef,
                                              const unsigned long long* __restrict__ words,
                                              int tile, uint32_t* __restrict__ counters, int64_t n_max,
                                              int64_t capacity, uint32_t* __restrict__ pair_tile,
                                              uint32_t* __restrict__ pair_item) {
  __shared__ uint32_t s_q[256];
  __shared__ uint32_t s_n;
  const int64_t n = min(static_cast<int64_t>(counters[0]), n_max);
  const int lane = static_cast<int>(threadIdx.x) & 63;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * 256; base < n; base += static_cast<int64_t>(gridDim.x) * 256) {
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const int64_t p = base + threadIdx.x;
    if (p < n) {
      const uint32_t item = vals[p];
      const DevView& v = views[view_of_item(views, n_views, item)];
      const uint4 b = sorted_bin[p];
      const uint32_t x0 = b.x & 0xFFFFu, x1 = b.x >> 16, y0 = b.y & 0xFFFu, y1 = (b.y >> 16) & 0xFFFu;
      const uint32_t w = x1 - x0, h = y1 - y0;
      if (w * h <= kSmallRect) {
        // The mask lists the reached tiles in row-major order; it is walked row by row (w bits per
        // row), which needs no integer division.
        int64_t o = offs[p];
        bool over = false;
        uint32_t m = b.z;
        const uint32_t row_mask = w >= 32 ? 0xFFFFFFFFu : (1u << w) - 1u;
        uint32_t t_row = static_cast<uint32_t>(v.tile_offset) + y0 * static_cast<uint32_t>(v.tiles_x) + x0;
        for (uint32_t row = 0; m; m >>= w, t_row += static_cast<uint32_t>(v.tiles_x), ++row) {
          const uint32_t pv = item | band_mask(b.y, row, h);
          for (uint32_t r = m & row_mask; r; r &= r - 1) {
            if (o < capacity) {
              pair_tile[o] = t_row + static_cast<uint32_t>(__builtin_ctz(r));
              pair_item[o] = pv;
            } else {
              over = true;
            }
            ++o;
          }
          if (w >= 32) break;
        }
        if (over) counters[2] = 1u;
      } else {
        s_q[atomicAdd(&s_n, 1u)] = threadIdx.x;
      }
    }
    __syncthreads();
    const uint32_t n_q = s_n;
    for (uint32_t d = threadIdx.x >> 6; d < n_q; d += 4) {
      // Everything about a queued rectangle is the same for the whole wave: with its position and
      // item in scalar registers its bin entry, view and ballot words come through the scalar cache
      // instead of 64 lanes' copies through the texture units, which this loop would saturate.
      const int64_t q = base + __builtin_amdgcn_readfirstlane(s_q[d]);
      const uint32_t item = __builtin_amdgcn_readfirstlane(vals[q]);
      const DevView& v = views[__builtin_amdgcn_readfirstlane(view_of_item(views, n_views, item))];
      const uint4 b = sorted_bin[q];
      const uint32_t x0 = b.x & 0xFFFFu, x1 = b.x >> 16, y0 = b.y & 0xFFFu, y1 = (b.y >> 16) & 0xFFFu;
      const uint32_t h = y1 - y0, w = x1 - x0, area = w * h;
      const float inv_w = 1.0f / static_cast<float>(w);
      int64_t o = offs[q];
      bool over = false;
      if (b.z != kNoWords) {
        // the projection's ballots: bit l of word k is tile 64 k + l of the rectangle (row-major)
        const unsigned long long* wk = words + b.z;
        for (uint32_t t0 = 0; t0 < area; t0 += 64, ++wk) {
          const uint64_t m = *wk;
          if (m == 0) continue;
          if ((m >> lane) & 1u) {
            uint32_t tx, ty;
            rect_tile(t0 + static_cast<uint32_t>(lane), w, inv_w, tx, ty);
            const int64_t oo = o + lanes_below(m);
            if (oo < capacity) {
              pair_tile[oo] = static_cast<uint32_t>(v.tile_offset) + (y0 + ty) * static_cast<uint32_t>(v.tiles_x) +
                              x0 + tx;
              pair_item[oo] = item | band_mask(b.y, ty, h);
            } else {
              over = true;
            }
          }
          o += __popcll(m);
        }
        if (over) counters[2] = 1u;
        continue;
      }
      // the conic and opacity (binning record) and the mean (compositing record), as projected
      const float4 cr = rec[item];
      const float4 cm = coef[2 * static_cast<int64_t>(item)];
      const float tau = footprint_tau(cr.w);
      const float nBA = -__fdiv_rn(cr.y, cr.x), nBC = -__fdiv_rn(cr.y, cr.z);
      for (uint32_t t0 = 0; t0 < area; t0 += 64) {
        const uint32_t t = t0 + static_cast<uint32_t>(lane);
        uint32_t tx, ty;
        rect_tile(t, w, inv_w, tx, ty);
        const uint32_t pv = item | band_mask(b.y, ty, h);
        tx += x0;
        ty += y0;
        const bool hit = t < area && tile_reached(cm.x, cm.y, cr.x, cr.y, cr.z, nBA, nBC, tau, static_cast<int>(tx),
                                                  static_cast<int>(ty), tile, v.width, v.height);
        const uint64_t m = __ballot(hit);
        if (hit) {
          const int64_t oo = o + lanes_below(m);
          if (oo < capacity) {
            pair_tile[oo] = static_cast<uint32_t>(v.tile_offset) + ty * static_cast<uint32_t>(v.tiles_x) + tx;
            pair_item[oo] = pv;
          } else {
            over = true;
          }
        }
        o += __popcll(m);
      }
      if (over) counters[2] = 1u;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ pair_tile,
                                                const uint32_t* __restrict__ counters, int64_t capacity,
                                                uint2* __restrict__ ranges) {
  const int64_t P = min(static_cast<int64_t>(counters[1]), capacity);
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < P;
       i += static_cast<int64_t>(gridDim.x) * 256) {
    const uint32_t t = pair_tile[i];
    if (i == 0 || pair_tile[i - 1] != t) ranges[t].x = static_cast<uint32_t>(i);
    if (i == P - 1 || pair_tile[i + 1] != t) ranges[t].y = static_cast<uint32_t>(i + 1);
  }
}

// Sort keys that put the tiles with the longest lists first (one key step per 8 list entries,
// lists of 2040 or more share the first key); the values are the tile indices.
__global__ __launch_bounds__(256) void k_tile_keys(const uint2* __restrict__ ranges, int64_t n_tiles,
                                                   uint32_t* __restrict__ keys, uint32_t* __restrict__ tiles) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (t >= n_tiles) return;
  const uint2 r = ranges[t];
  keys[t] = 255u - min(255u, (r.y - r.x) >> 3);
  tiles[t] = static_cast<uint32_t>(t);
}

__global__ void k_status(const uint32_t* __restrict__ counters, int32_t* __restrict__ status) {
  if (threadIdx.x == 0) {
    status[0] = static_cast<int32_t>(counters[2]);
    status[1] = static_cast<int32_t>(counters[1]);
    status[2] = static_cast<int32_t>(counters[0]);
    status[3] += counters[2] ? 1 : 0;
  }
}

// ------------------------------------------------------------------ projection backward
// Chain rule from the per-item 2D gradients (mean2d, conic, opacity, rgb) to the activated 3D
// parameters, summed over the views that show the Gaussian's scene (deterministic: one thread per
// Gaussian walks its views in order).
__device__ __forceinline__ void project_bwd_one(const DevView& v, const float m[3], const float s[3], const float q[4],
                                                const float g2[5], float dm[3], float ds[3], float dq[4]) {
  const float* R = v.R;
  const float X = ((R[0] * m[0] + R[1] * m[1]) + R[2] * m[2]) + v.t[0];
  const float Y = ((R[3] * m[0] + R[4] * m[1]) + R[5] * m[2]) + v.t[1];
  const float Z = ((R[6] * m[0] + R[7] * m[1]) + R[8] * m[2]) + v.t[2];
  const float fx = v.fx, fy = v.fy;
  const float limx = v.lim_x, limy = v.lim_y;
  const float txz = X / Z, tyz = Y / Z;
  const bool clx = txz < -limx || txz > limx;
  const bool cly = tyz < -limy || tyz > limy;
  const float cx_ = fminf(limx, fmaxf(-limx, txz));
  const float cy_ = fminf(limy, fmaxf(-limy, tyz));
  const float z2 = Z * Z, z3 = z2 * Z;
  const float J00 = fx / Z, J02 = -fx * cx_ / Z, J11 = fy / Z, J12 = -fy * cy_ / Z;
  float A[2][3];
  for (int k = 0; k < 3; ++k) {
    A[0][k] = J00 * R[k] + J02 * R[6 + k];
    A[1][k] = J11 * R[3 + k] + J12 * R[6 + k];
  }
  float Rq[3][3], qn[4];
  rot_from_quat(q[0], q[1], q[2], q[3], Rq, qn);
  float M[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) M[i][k] = Rq[i][k] * s[k];
  float V[2][3];
  for (int a = 0; a < 2; ++a)
    for (int k = 0; k < 3; ++k) V[a][k] = A[a][0] * M[0][k] + A[a][1] * M[1][k] + A[a][2] * M[2][k];
  const float a = V[0][0] * V[0][0] + V[0][1] * V[0][1] + V[0][2] * V[0][2] + 0.3f;
  const float b = V[0][0] * V[1][0] + V[0][1] * V[1][1] + V[0][2] * V[1][2];
  const float c = V[1][0] * V[1][0] + V[1][1] * V[1][1] + V[1][2] * V[1][2] + 0.3f;
  const float det = a * c - b * b;
  const float id2 = 1.0f / (det * det);
  const float gA = g2[2], gB = g2[3], gC = g2[4];
  // conic = (c, -b, a) / det
  const float ga = (-c * c * gA + b * c * gB - b * b * gC) * id2;
  const float gb = (2.0f * b * c * gA - (a * c + b * b) * gB + 2.0f * a * b * gC) * id2;
  const float gc = (-b * b * gA + a * b * gB - a * a * gC) * id2;
  // Sigma2 = V V^T + 0.3 I
  float dV[2][3];
  for (int k = 0; k < 3; ++k) {
    dV[0][k] = 2.0f * ga * V[0][k] + gb * V[1][k];
    dV[1][k] = gb * V[0][k] + 2.0f * gc * V[1][k];
  }
  // V = A M
  float dM[3][3], dA[2][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) dM[i][k] = A[0][i] * dV[0][k] + A[1][i] * dV[1][k];
  for (int a2 = 0; a2 < 2; ++a2)
    for (int i = 0; i < 3; ++i) dA[a2][i] = dV[a2][0] * M[i][0] + dV[a2][1] * M[i][1] + dV[a2][2] * M[i][2];
  // A = J R_view
  const float dJ00 = dA[0][0] * R[0] + dA[0][1] * R[1] + dA[0][2] * R[2];
  const float dJ02 = dA[0][0] * R[6] + dA[0][1] * R[7] + dA[0][2] * R[8];
  const float dJ11 = dA[1][0] * R[3] + dA[1][1] * R[4] + dA[1][2] * R[5];
  const float dJ12 = dA[1][0] * R[6] + dA[1][1] * R[7] + dA[1][2] * R[8];
  float dX = 0.0f, dY = 0.0f, dZ = 0.0f;
  dZ += -fx / z2 * dJ00 - fy / z2 * dJ11;
  if (!clx) {
    dX += -fx / z2 * dJ02;
    dZ += 2.0f * fx * X / z3 * dJ02;
  } else {
    dZ += fx * cx_ / z2 * dJ02;
  }
  if (!cly) {
    dY += -fy / z2 * dJ12;
    dZ += 2.0f * fy * Y / z3 * dJ12;
  } else {
    dZ += fy * cy_ / z2 * dJ12;
  }
  // mean2d = (fx X/Z + cx, fy Y/Z + cy)
  dX += fx / Z * g2[0];
  dZ += -fx * X / z2 * g2[0];
  dY += fy / Z * g2[1];
  dZ += -fy * Y / z2 * g2[1];
  dm[0] = R[0] * dX + R[3] * dY + R[6] * dZ;
  dm[1] = R[1] * dX + R[4] * dY + R[7] * dZ;
  dm[2] = R[2] * dX + R[5] * dY + R[8] * dZ;
  // M = R_q diag(s)
  float dR[3][3];
  for (int k = 0; k < 3; ++k) {
    ds[k] = Rq[0][k] * dM[0][k] + Rq[1][k] * dM[1][k] + Rq[2][k] * dM[2][k];
    for (int i = 0; i < 3; ++i) dR[i][k] = dM[i][k] * s[k];
  }
  const float w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  float dqn[4];
  dqn[0] = 2.0f * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
  dqn[1] = 2.0f * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.0f * x * dR[1][1] - w * dR[1][2] + z * dR[2][0] +
                   w * dR[2][1] - 2.0f * x * dR[2][2]);
  dqn[2] = 2.0f * (-2.0f * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] - w * dR[2][0] +
                   z * dR[2][1] - 2.0f * y * dR[2][2]);
  dqn[3] = 2.0f * (-2.0f * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2.0f * z * dR[1][1] +
                   y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
  const float nq = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float dot = w * dqn[0] + x * dqn[1] + y * dqn[2] + z * dqn[3];
  for (int i = 0; i < 4; ++i) dq[i] = (dqn[i] - qn[i] * dot) / nq;
}

// The compositing backward leaves per item the moments of dL/dpower over the pixels it reached
// (sum dx dp, sum dp dy, sum dx^2 dp, sum dx dp dy, sum dp dy^2, sum dp; d = mean2d - pixel) and
// the colour gradient.  power = -(A dx^2 + 2 B dx dy + C dy^2) / 2 and alpha = o exp(power) make
// the 2D gradients linear in them:
//   dmean.x = -(A m0 + B m1), dmean.y = -(B m0 + C m1), dA = -m2 / 2, dB = -m3, dC = -m4 / 2,
//   dopacity = m5 / o.
__device__ __forceinline__ void moments_to_grad2d(const float4 cr, float g2[9]) {
  const float A = cr.x, B = cr.y, Cc = cr.z, o = cr.w;
  const float m0 = g2[0], m1 = g2[1];
  g2[0] = -(A * m0 + B * m1);
  g2[1] = -(B * m0 + Cc * m1);
  g2[2] = -0.5f * g2[2];
  g2[3] = -g2[3];
  g2[4] = -0.5f * g2[4];
  g2[5] = g2[5] / o;
}

// Adds one view's contribution of a Gaussian: the item's raw moments (accumulator row, nine
// columns) turned into 2D gradients with its conic and opacity (cr), then the chain rule to the 3D
// parameters.
__device__ __forceinline__ void project_bwd_view(const DevView& v, const float m[3], const float sc3[3],
                                                 const float q[4], float4 q0, float4 q1, float4 q2, float4 cr,
                                                 float am[3], float as[3], float aq[4], float& ao, float ac[3]) {
  float g2[9] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x};
  moments_to_grad2d(cr, g2);
  ao += g2[5];
  ac[0] += g2[6];
  ac[1] += g2[7];
  ac[2] += g2[8];
  if (g2[0] == 0.0f && g2[1] == 0.0f && g2[2] == 0.0f && g2[3] == 0.0f && g2[4] == 0.0f) return;
  float dm[3], ds[3], dq[4];
  project_bwd_one(v, m, sc3, q, g2, dm, ds, dq);
  for (int k = 0; k < 3; ++k) {
    am[k] += dm[k];
    as[k] += ds[k];
  }
  for (int k = 0; k < 4; ++k) aq[k] += dq[k];
}

// One thread per Gaussian, its views in order (deterministic).  When a wave's 64 Gaussians all
// belong to one scene, their items in a view are 64 consecutive accumulator rows (4 KB): the wave
// reads them as coalesced 16-byte vectors and hands each lane its own row through LDS, instead of
// 64 strided row reads, which keep the texture units busy far longer than the bytes need (the
// 16-byte records are coalesced as they are).  A wave that straddles a scene boundary or the end
// reads per lane.
__global__ __launch_bounds__(256) void k_project_bwd(const DevView* __restrict__ views, int n_views,
                                                     const DevScene* __restrict__ scenes, int n_scenes,
                                                     vbm_gaussians_c g, float* __restrict__ grad2d,
                                                     const float4* __restrict__ rec, int64_t n_items,
                                                     const uint32_t* __restrict__ ntiles, vbm_gaussians grads,
                                                     int accumulate, int64_t n_total) {
  constexpr int kRowPitch = 5;   // float4 per LDS row (padded: spreads the banks)
  __shared__ float4 s_row[4][64 * kRowPitch];
  const int64_t gi = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int lane = static_cast<int>(threadIdx.x) & 63, wv = static_cast<int>(threadIdx.x) >> 6;
  const bool valid = gi < n_total;
  int sc = 0;
  for (int s = 1; s < n_scenes; ++s)
    if (scenes[s].gauss_offset <= gi) sc = s;
  const int sc0 = __builtin_amdgcn_readfirstlane(sc);
  const bool uniform_wave = __ballot(valid && sc == sc0) == ~0ull;
  if (!valid) return;
  const int64_t S = g.stride;
  const float m[3] = {g.means[gi], g.means[S + gi], g.means[2 * S + gi]};
  const float sc3[3] = {g.scales[gi], g.scales[S + gi], g.scales[2 * S + gi]};
  const float q[4] = {g.quats[gi], g.quats[S + gi], g.quats[2 * S + gi], g.quats[3 * S + gi]};
  float am[3] = {0, 0, 0}, as[3] = {0, 0, 0}, aq[4] = {0, 0, 0, 0}, ao = 0.0f, ac[3] = {0, 0, 0};
  if (uniform_wave) {
    const int64_t g0 = gi - lane;
    for (int vi = 0; vi < n_views; ++vi) {
      const DevView& v = views[vi];
      if (v.scene != sc0) continue;   // uniform
      const int64_t item0 = v.item_offset + (g0 - v.gauss_offset);
      const float4* rsrc = reinterpret_cast<const float4*>(grad2d + 16 * item0);
      float4 t[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) t[k] = rsrc[lane + 64 * k];
      const float4 cr = rec[item0 + lane];
      const uint32_t nt = ntiles[item0 + lane];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int e = lane + 64 * k;   // float4 e of the wave's rows: row e / 4, quarter e % 4
        s_row[wv][kRowPitch * (e >> 2) + (e & 3)] = t[k];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (nt != 0) {
        const float4* my = &s_row[wv][kRowPitch * lane];
        project_bwd_view(v, m, sc3, q, my[0], my[1], my[2], cr, am, as, aq, ao, ac);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  } else {
    for (int vi = 0; vi < n_views; ++vi) {
      const DevView& v = views[vi];
      if (v.scene != sc) continue;
      const int64_t item = v.item_offset + (gi - v.gauss_offset);
      if (ntiles[item] == 0) continue;
      const float4* row = reinterpret_cast<const float4*>(grad2d + 16 * item);
      project_bwd_view(v, m, sc3, q, row[0], row[1], row[2], rec[item], am, as, aq, ao, ac);
    }
  }
  const int64_t GS = grads.stride;
  if (accumulate) {
    for (int k = 0; k < 3; ++k) {
      grads.means[k * GS + gi] += am[k];
      grads.scales[k * GS + gi] += as[k];
      grads.rgb[k * GS + gi] += ac[k];
    }
    for (int k = 0; k < 4; ++k) grads.quats[k * GS + gi] += aq[k];
    grads.opacity[gi] += ao;
  } else {
    for (int k = 0; k < 3; ++k) {
      grads.means[k * GS + gi] = am[k];
      grads.scales[k * GS + gi] = as[k];
      grads.rgb[k * GS + gi] = ac[k];
    }
    for (int k = 0; k < 4; ++k) grads.quats[k * GS + gi] = aq[k];
    grads.opacity[gi] = ao;
  }
}

}  // namespace vbm
