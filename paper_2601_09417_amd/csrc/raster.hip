// Front-to-back alpha compositing and its reverse-order backward (Sec. 3, the Gaussian mixture
// rendered by the 3DGS rasteriser cited in Sec. 4.4).
//
// Work decomposition: one wave64 per 256 pixels of a tile (a 16x16 tile is one wave, a 32x32 tile
// four independent waves, an 8x8 tile one wave with one pixel per lane), each lane owning
// PPL = 4 pixels of ONE pixel column (rows 64 / TILE apart), so the horizontal offset to a
// Gaussian's centre is shared by a lane's pixels.  The tile's depth-sorted list is walked by every
// wave in lockstep: a Gaussian's item id and its 36-byte record are wave-uniform, fetched with
// buffer loads at a uniform offset (records two list steps ahead of use, item ids four) -- no LDS
// staging, no barriers, and the per-Gaussian load cost is amortised over 256 pixels.
//
// The record holds the exponent in base 2 with the log-opacity folded in:
//   e2(d) = hA dx^2 + hB dx dy + hC dy^2 + log2(o) = log2(o) + power(d) log2(e),
// so alpha = min(0.99, 2^e2) costs one exponential and no multiply by the opacity.  Projection
// keeps only Gaussians with a positive-definite conic, for which power <= 0 at every pixel, so a
// "skip when power > 0" guard could only fire on float32 rounding near the centre and is left out.
//
// The backward walks the list in reverse from the wave's largest n_contrib, recomputes each
// pixel's transmittance from final_T by division and keeps the normalised colour behind the
// current Gaussian in one running value per channel.  The geometric gradient is accumulated as
// three per-lane moments of dL/dpower (sum, first and second moment in dy); the lane's column
// offset dx turns them into the five sums the 2D parameters need.  Nine per-wave sums are then
// formed with a DPP reduce-scatter inside 16-lane rows (27 VALU operations, one value per lane)
// plus two cross-row lane swaps, and nine lanes issue one float atomic each into the item's
// 64-byte accumulator row (one cache segment per pair instead of nine lines) -- only when some
// pixel contributed.  The atomics add those raw moments; the projection backward turns them into
// mean/conic/opacity gradients with the item's conic, since that map is linear.
#include <hip/hip_runtime.h>

#include "common.h"

namespace vbm {

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
// Item ids stay below 2^27 (the plan enforces it); the forward keeps per-pair lane-group marks in
// the bits above.
constexpr int kItemBits = 27;
constexpr uint32_t kItemMask = (1u << kItemBits) - 1u;

template <int TILE>
struct TileCfg {
  static constexpr int kPix = TILE * TILE;
  static constexpr int kWaves = kPix >= 256 ? kPix / 256 : 1;
  static constexpr int kPPL = kPix / (64 * kWaves);  // pixels per lane
  static constexpr int kThreads = 64 * kWaves;
  static_assert(64 % TILE == 0, "a lane's pixels must share one column");
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

// One Gaussian's compositing record (wave-uniform values).
struct Rec {
  float mx, my, hA, hB, hC, lo, r, g, b;
};

typedef int v4i __attribute__((ext_vector_type(4)));
constexpr int kRsrcWord3 = 0x00020000;  // raw (untyped) buffer access on the gfx9 family

// Buffer descriptors of the arrays the list walk reads.  Buffer loads are vector-memory
// operations (completed in issue order, so a prefetch is waited for exactly) with a
// uniform SGPR offset (no per-lane address arithmetic), and the hardware range check turns a read
// past num_records into a zero instead of an access fault.
struct ListSrc {
  __amdgpu_buffer_rsrc_t items, coef, blue;
};

__device__ __forceinline__ ListSrc make_list_src(const uint32_t* pair_item, int64_t n_pairs, const float* coef,
                                                 const float* blue, int64_t n_items) {
  // num_records is a 32-bit byte count: the plan bounds n_items by 2^27 and n_pairs by 2^30.
  ListSrc s;
  s.items = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(pair_item), (short)0,
                                              static_cast<int>(static_cast<uint32_t>(n_pairs * 4)), kRsrcWord3);
  s.coef = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(coef), (short)0,
                                             static_cast<int>(static_cast<uint32_t>(n_items * 32)), kRsrcWord3);
  s.blue = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(blue), (short)0,
                                             static_cast<int>(static_cast<uint32_t>(n_items * 4)), kRsrcWord3);
  return s;
}

__device__ __forceinline__ uint32_t load_item(const ListSrc& s, int j) {
  return static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b32(s.items, 0, 4 * j, 0));
}

// Rewrites the n <= 3 pair values j, j + 1, j + 2 (uniform v0, v1, v2) with one vector store from
// lanes 0 .. n - 1.
__device__ __forceinline__ void store_pair_values(const ListSrc& s, int lane, int j, int n, uint32_t v0, uint32_t v1,
                                                  uint32_t v2) {
  const uint32_t v = lane == 0 ? v0 : lane == 1 ? v1 : v2;
  if (lane < n) __builtin_amdgcn_raw_buffer_store_b32(v, s.items, 4 * lane, 4 * j, 0);
}

// The record of a pair value (the item id in its low kItemBits bits).
__device__ __forceinline__ Rec load_rec(const ListSrc& s, uint32_t pv) {
  const uint32_t it = pv & kItemMask;
  const int off = static_cast<int>(32u * it);
  const v4i a = __builtin_amdgcn_raw_buffer_load_b128(s.coef, 0, off, 0);
  const v4i b = __builtin_amdgcn_raw_buffer_load_b128(s.coef, 16, off, 0);
  Rec r;
  r.mx = __int_as_float(a.x);
  r.my = __int_as_float(a.y);
  r.hA = __int_as_float(a.z);
  r.hB = __int_as_float(a.w);
  r.hC = __int_as_float(b.x);
  r.lo = __int_as_float(b.y);
  r.r = __int_as_float(b.z);
  r.g = __int_as_float(b.w);
  r.b = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(s.blue, 0, static_cast<int>(4u * it), 0));
  return r;
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// True when the predicate holds on some active lane: one scalar test of the predicate's lane mask.
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

// Base-2 exponent of the Gaussian at a pixel whose per-lane terms u = hA dx^2 + log2(o) and
// v = hB dx are precomputed; one expression shared by the forward and the backward so that both
// take bit-identical skip / contribute decisions.
__device__ __forceinline__ float exponent2(const Rec& r, float u, float v, float dy) {
  return fmaf(fmaf(r.hC, dy, v), dy, u);
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// One step of a reduce-scatter inside 16-lane rows: lanes with `hi` clear keep value a, the others
// value b, each adding its DPP partner's copy (the partner always has the opposite `hi`).
template <int CTRL>
__device__ __forceinline__ float rs_pair(float a, float b, bool hi) {
  const float keep = hi ? b : a;
  const float send = hi ? a : b;
  return keep + dpp_move<CTRL>(send);
}
template <int CTRL>
__device__ __forceinline__ float rs_single(float v) {
  return v + dpp_move<CTRL>(v);
}

constexpr int kRowMirror = 0x140;
constexpr int kRowHalfMirror = 0x141;
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]

// Wave sums of nine values (every lane active).  Lane l < 16 ends with the sum of value
// rs_index(l): even lanes l hold value 4 b1 + 2 b2 + b3 (b_i = bit i of l), odd lanes value 8.
__device__ __forceinline__ float reduce_scatter9(const float g[9], int lane) {
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
  const float A = rs_pair<kRowMirror>(g[0], g[1], b3);
  const float B = rs_pair<kRowMirror>(g[2], g[3], b3);
  const float C = rs_pair<kRowMirror>(g[4], g[5], b3);
  const float D = rs_pair<kRowMirror>(g[6], g[7], b3);
  float E = rs_single<kRowMirror>(g[8]);
  const float F = rs_pair<kRowHalfMirror>(A, B, b2);
  const float G = rs_pair<kRowHalfMirror>(C, D, b2);
  E = rs_single<kRowHalfMirror>(E);
  const float H = rs_pair<kQuadXor2>(F, G, b1);
  E = rs_single<kQuadXor2>(E);
  const float K = rs_pair<kQuadXor1>(H, E, b0);
  // Cross-row sums for lanes 0..15 only: permlane32_swap hands lanes 0..31 of its second operand
  // the upper half of its first (which keeps its own lower half), permlane16_swap likewise hands
  // row 0 the contents of row 1.
  const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(K), 0u, false, false);
  const float K2 = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(K2), 0u, false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ int rs_index(int lane) {
  return (lane & 1) ? 8 : ((lane >> 1) & 1) * 4 + ((lane >> 2) & 1) * 2 + ((lane >> 3) & 1);
}

// a + b over the wave's halves: lanes 0..31 get a[l] + a[l + 32], lanes 32..63 b[l - 32] + b[l].
__device__ __forceinline__ float add_halves(float a, float b) {
  const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(h[0]) + __uint_as_float(h[1]);
}
// The same over 16-lane row pairs: rows 0 and 2 get a's rows (0 + 1) and (2 + 3), rows 1 and 3 b's.
__device__ __forceinline__ float add_row_pairs(float a, float b) {
  const auto h = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(h[0]) + __uint_as_float(h[1]);
}

// Wave sums of the nine gradient terms {dx s0, s1, dx^2 s0, dx s1, s2, s0, wr, wg, wb} when lanes
// l, l + 16, l + 32, l + 48 share a pixel column (so dx): the six per-lane sums are first added
// over those lanes (row k of 16 lanes then holds s0, s1, wr, wg column sums in P and s2, s2, wb, wb
// in Q), scaled by dx, dx^2, and the four values P, P dx, P dx^2, Q reduced inside each row.  The
// sums land in the lanes that col_index names.
__device__ __forceinline__ float reduce_cols9(float s0, float s1, float s2, float wr, float wg, float wb, float dx,
                                              float dx2, int lane) {
  const float P = add_row_pairs(add_halves(s0, wr), add_halves(s1, wg));
  const float Z = add_halves(s2, wb);
  const float Q = add_row_pairs(Z, Z);
  const bool b3 = lane & 8, b2 = lane & 4;
  const float V1 = rs_pair<kRowMirror>(P, P * dx, b3);       // lanes 0..7: P, 8..15: P dx
  const float V2 = rs_pair<kRowMirror>(P * dx2, Q, b3);      // lanes 0..7: P dx^2, 8..15: Q
  const float W = rs_pair<kRowHalfMirror>(V1, V2, b2);       // quads: P, P dx^2, P dx, Q
  return rs_single<kQuadXor1>(rs_single<kQuadXor2>(W));
}

// Gradient column (0..8) whose sum reduce_cols9 leaves in the lane, or -1.
__device__ __forceinline__ int col_index(int lane) {
  switch (lane) {
    case 0: return 5;    // s0
    case 4: return 2;    // dx^2 s0
    case 8: return 0;    // dx s0
    case 12: return 4;   // s2
    case 16: return 1;   // s1
    case 24: return 3;   // dx s1
    case 32: return 6;   // wr
    case 44: return 8;   // wb
    case 48: return 7;   // wg
    default: return -1;
  }
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

// A pixel that has terminated (or lies outside the image) gets this row coordinate: its exponent
// then overflows to -inf, alpha underflows to 0 and it never contributes again, so the step needs
// no separate liveness test.
constexpr float kDeadRow = 1e30f;
// log2(1/255) - 0.001: below it 2^e2 < 1/255 with a margin far above the exponential's error.
constexpr float kE2Skip = -7.9953534f;
constexpr float kLiveBound = 1e29f;

template <int PPL>
__device__ __forceinline__ bool any_live(const float (&fy)[PPL]) {
  float m = fy[0];
#pragma unroll
  for (int k = 1; k < PPL; ++k) m = fminf(m, fy[k]);
  return wave_any(m < kLiveBound);
}

// One list step of the forward for the lane's pixels: alpha = min(0.99, 2^e2); a pixel takes the
// Gaussian when alpha >= 1/255, unless the new transmittance would fall below 1e-4, in which case
// the pixel stops without it.  Returns the mask of lane groups k that were evaluated: every group
// with a pixel that took the Gaussian is among them.
template <int PPL, bool STATS>
__device__ __forceinline__ uint32_t fwd_step(const Rec& r, int pos, float fx, float (&fy)[PPL], float (&T)[PPL],
                                             float (&cr)[PPL], float (&cg)[PPL], float (&cb)[PPL], int (&last)[PPL],
                                             uint32_t& n_eval, uint32_t& n_used) {
  uint32_t groups = 0;
  const float dx = r.mx - fx;
  const float u = fmaf(r.hA, dx * dx, r.lo);
  const float vb = r.hB * dx;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const float dy = r.my - fy[k];
    const float e2 = exponent2(r, u, vb, dy);
    // A lane group where every pixel has 2^e2 clearly below 1/255 (or is terminated, e2 = -inf)
    // takes nothing from this Gaussian: skip the exponential and the update with one uniform branch.
    if (!wave_any(e2 >= kE2Skip)) {
      if (STATS) n_eval += fy[k] < kLiveBound ? 1u : 0u;
      continue;
    }
    groups |= 1u << k;
    const float alpha = fminf(kAlphaMax, __builtin_amdgcn_exp2f(e2));
    const bool ok = alpha >= kAlphaMin;
    // A pixel that fails the alpha test takes weight 0, which leaves T and its colour unchanged.
    float w = (ok ? alpha : 0.0f) * T[k];
    float Tn = T[k] - w;
    // A live pixel keeps T >= 1e-4, so only one that takes the Gaussian can fall below: it stops
    // without it (rare, so handled in a uniform branch).
    const bool stop = Tn < kTMin;
    if (wave_any(stop)) {
      __asm__ volatile("" ::: "memory");   // keeps this a branch: the compiler would select both ways
      w = stop ? 0.0f : w;
      Tn = stop ? T[k] : Tn;
      fy[k] = stop ? kDeadRow : fy[k];
    }
    const bool use = ok && !stop;
    if (STATS) {
      n_eval += fy[k] < kLiveBound || stop ? 1u : 0u;
      n_used += use ? 1u : 0u;
    }
    cr[k] = fmaf(r.r, w, cr[k]);
    cg[k] = fmaf(r.g, w, cg[k]);
    cb[k] = fmaf(r.b, w, cb[k]);
    T[k] = Tn;
    last[k] = use ? pos : last[k];
  }
  return groups;
}

template <int TILE, bool STATS>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_composite_fwd(
    const DevView* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ tile_order,
    uint32_t* __restrict__ pair_item, int64_t n_pairs, const float* __restrict__ coef,
    const float* __restrict__ blue, int64_t n_items, float* __restrict__ image, float* __restrict__ final_T,
    int32_t* __restrict__ n_contrib, unsigned long long* __restrict__ stats) {
  using C = TileCfg<TILE>;
  constexpr int PPL = C::kPPL;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int wave = static_cast<int>(threadIdx.x) >> 6;
  const int tile = static_cast<int>(tile_order[blockIdx.x]);
  const DevView& v = views[find_view(views, n_views, tile)];
  const int local = tile - v.tile_offset;
  const int tx = local % v.tiles_x, ty = local / v.tiles_x;
  float fy[PPL], T[PPL], cr[PPL], cg[PPL], cb[PPL];
  int last[PPL];
  bool inside[PPL];
  int py[PPL];
  const int q0 = wave * (C::kPix / C::kWaves) + lane;
  const int px = tx * TILE + q0 % TILE;
  const float fx = static_cast<float>(px) + 0.5f;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    py[k] = ty * TILE + (q0 + k * 64) / TILE;
    inside[k] = px < v.width && py[k] < v.height;
    fy[k] = inside[k] ? static_cast<float>(py[k]) + 0.5f : kDeadRow;
    T[k] = 1.0f;
    cr[k] = cg[k] = cb[k] = 0.0f;
    last[k] = 0;
  }
  const uint2 rg = ranges[tile];
  const int start = static_cast<int>(rg.x), end = static_cast<int>(rg.y);
  uint32_t n_eval = 0, n_used = 0;
  // Load pipeline, unrolled by three so that buffers rotate without copies: the record of list
  // step s is requested at step s - 2 and the item id that addresses it at step s - 4 (three
  // record buffers R, three item slots L).  All three steps of an iteration run (a branch between
  // them would let the compiler sink the prefetch below it); past the end of the list a record is
  // a clamped duplicate whose log-opacity is set to -inf, so alpha = 0 and it changes nothing.
  const ListSrc src = make_list_src(pair_item, n_pairs, coef, blue, n_items);
  const int lastj = end > start ? end - 1 : start;
  // With one wave per tile, each processed pair value is written back with the mask of the lane
  // groups that the step evaluated in bits kItemBits.. (see fwd_step): the backward visits only
  // those groups.
  constexpr bool kMark = C::kWaves == 1;
  uint32_t u0 = uniform(load_item(src, start)), u1 = uniform(load_item(src, min(start + 1, lastj))), u2;
  Rec R0 = load_rec(src, u0);
  Rec R1 = load_rec(src, u1);
  Rec R2;
  uint32_t L1, L2 = load_item(src, min(start + 2, lastj)), L0 = load_item(src, min(start + 3, lastj));
  for (int j = start; j < end; j += 3) {
    if (!any_live(fy)) break;
    u2 = uniform(L2);
    R2 = load_rec(src, u2);
    L1 = load_item(src, min(j + 4, lastj));
    const uint32_t m0 = (u0 & kItemMask) | (fwd_step<PPL, STATS>(R0, j - start + 1, fx, fy, T, cr, cg, cb, last,
                                                                  n_eval, n_used) << kItemBits);
    R1.lo = j + 1 < end ? R1.lo : -__builtin_inff();
    u0 = uniform(L0);
    R0 = load_rec(src, u0);
    L2 = load_item(src, min(j + 5, lastj));
    const uint32_t m1 = (u1 & kItemMask) | (fwd_step<PPL, STATS>(R1, j - start + 2, fx, fy, T, cr, cg, cb, last,
                                                                  n_eval, n_used) << kItemBits);
    R2.lo = j + 2 < end ? R2.lo : -__builtin_inff();
    u1 = uniform(L1);
    R1 = load_rec(src, u1);
    L0 = load_item(src, min(j + 6, lastj));
    const uint32_t m2 = (u2 & kItemMask) | (fwd_step<PPL, STATS>(R2, j - start + 3, fx, fy, T, cr, cg, cb, last,
                                                                  n_eval, n_used) << kItemBits);
    if (kMark) store_pair_values(src, lane, j, min(end - j, 3), m0, m1, m2);
  }
  if (STATS) add_stats(stats, n_eval, n_used);
  const int64_t HW = static_cast<int64_t>(v.width) * v.height;
  float* img = image + 3 * static_cast<int64_t>(v.pixel_offset);
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    if (!inside[k]) continue;
    const int64_t pix = static_cast<int64_t>(py[k]) * v.width + px;
    img[pix] = cr[k] + T[k] * v.bg[0];
    img[HW + pix] = cg[k] + T[k] * v.bg[1];
    img[2 * HW + pix] = cb[k] + T[k] * v.bg[2];
    final_T[v.pixel_offset + pix] = T[k];
    n_contrib[v.pixel_offset + pix] = last[k];
  }
}

// Per-wave gradient state of one list step of the backward (see bwd_step).
template <int PPL>
struct BwdPix {
  float fy[PPL], T[PPL], dr[PPL], dg[PPL], db[PPL], S[PPL];
  int nc[PPL];
};

// One list step (list position j, 0-based) of the backward for the lane's pixels.  A pixel takes
// part when j < n_contrib and the forward's alpha test holds; its transmittance before the
// Gaussian is T / (1 - alpha), dL/dalpha = T_before * sum_c dL/dC_c (c_c - acc_c) with acc the
// normalised colour behind the Gaussian (the background at first), which then becomes
// alpha c + (1 - alpha) acc.  Only the projection S = sum_c dL/dC_c acc_c enters, so that scalar is
// what the pixel carries: dL/dalpha = T_before (D_c - S) with D_c = sum_c dL/dC_c c_c, and S moves
// to S + alpha (D_c - S).  dL/dpower = alpha dL/dalpha unless alpha was clamped.
template <int PPL, bool MARKED, bool COLS, bool STATS>
__device__ __forceinline__ void bwd_step(const Rec& r, uint32_t pv, int j, float fx, BwdPix<PPL>& P, int lane,
                                         int out_k, bool out_lane, float* __restrict__ grad2d, uint32_t& n_eval,
                                         uint32_t& n_used) {
  if (STATS)
#pragma unroll
    for (int k = 0; k < PPL; ++k) n_eval += j < P.nc[k] ? 1u : 0u;
  // MARKED: the forward left in the pair value the lane groups it evaluated, a superset of those
  // with a contributing pixel; each is handled wholly inside its own uniform branch.
  const uint32_t groups = MARKED ? pv >> kItemBits : (1u << PPL) - 1u;
  if (groups == 0) return;
  const float dx = r.mx - fx;
  const float dx2 = dx * dx;
  const float u = fmaf(r.hA, dx2, r.lo);
  const float vb = r.hB * dx;
  // Per-lane sums: s0 = sum dp, s1 = sum dp dy, s2 = sum dp dy^2 (dp = dL/dpower), and the colour
  // weights alpha T_before dL/dC.
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, wr = 0.0f, wg = 0.0f, wb = 0.0f;
  bool anyc = false;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    if (!((groups >> k) & 1u)) continue;
    const float dy = r.my - P.fy[k];
    const float G2 = __builtin_amdgcn_exp2f(exponent2(r, u, vb, dy));
    const float alpha = fminf(kAlphaMax, G2);
    const bool c = j < P.nc[k] && alpha >= kAlphaMin;
    if (STATS) n_used += c ? 1u : 0u;
    anyc |= c;
    if (c) {
      const float Tk = P.T[k] * __builtin_amdgcn_rcpf(1.0f - alpha);
      P.T[k] = Tk;
      const float D = fmaf(P.dr[k], r.r, fmaf(P.dg[k], r.g, P.db[k] * r.b)) - P.S[k];
      P.S[k] = fmaf(alpha, D, P.S[k]);
      const float w = alpha * Tk;
      wr = fmaf(w, P.dr[k], wr);
      wg = fmaf(w, P.dg[k], wg);
      wb = fmaf(w, P.db[k], wb);
      const float dp = G2 <= kAlphaMax ? w * D : 0.0f;     // alpha dL/dalpha
      const float t = dp * dy;
      s0 += dp;
      s1 += t;
      s2 = fmaf(t, dy, s2);
    }
  }
  // (with marks the superset is tight enough that the test does not pay for itself)
  if (!MARKED && !wave_any(anyc)) return;
  float sum;
  if constexpr (COLS) {
    sum = reduce_cols9(s0, s1, s2, wr, wg, wb, dx, dx2, lane);
  } else {
    const float g[9] = {dx * s0, s1, dx2 * s0, dx * s1, s2, s0, wr, wg, wb};
    sum = reduce_scatter9(g, lane);
  }
  if (out_lane && sum != 0.0f) unsafeAtomicAdd(&grad2d[16 * static_cast<size_t>(pv & kItemMask) + out_k], sum);
}

template <int TILE, bool STATS>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_composite_bwd(
    const DevView* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ tile_order,
    const uint32_t* __restrict__ pair_item, int64_t n_pairs, const float* __restrict__ coef,
    const float* __restrict__ blue, const float* __restrict__ final_T, const int32_t* __restrict__ n_contrib,
    const float* __restrict__ dL_dimg, float* __restrict__ grad2d, int64_t n_items,
    unsigned long long* __restrict__ stats) {
  using C = TileCfg<TILE>;
  constexpr int PPL = C::kPPL;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int wave = static_cast<int>(threadIdx.x) >> 6;
  const int tile = static_cast<int>(tile_order[blockIdx.x]);
  const DevView& v = views[find_view(views, n_views, tile)];
  const int local = tile - v.tile_offset;
  const int tx = local % v.tiles_x, ty = local / v.tiles_x;
  const int64_t HW = static_cast<int64_t>(v.width) * v.height;
  BwdPix<PPL> P;
  int maxn = 0;
  const int q0 = wave * (C::kPix / C::kWaves) + lane;
  const int px = tx * TILE + q0 % TILE;
  const float fx = static_cast<float>(px) + 0.5f;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int py = ty * TILE + (q0 + k * 64) / TILE;
    const bool inside = px < v.width && py < v.height;
    P.fy[k] = static_cast<float>(py) + 0.5f;
    P.T[k] = 1.0f;
    P.nc[k] = 0;
    P.dr[k] = P.dg[k] = P.db[k] = 0.0f;
    if (inside) {
      const int64_t pix = static_cast<int64_t>(py) * v.width + px;
      P.T[k] = final_T[v.pixel_offset + pix];
      P.nc[k] = n_contrib[v.pixel_offset + pix];
      const float* g = dL_dimg + 3 * static_cast<int64_t>(v.pixel_offset);
      P.dr[k] = g[pix];
      P.dg[k] = g[HW + pix];
      P.db[k] = g[2 * HW + pix];
    }
    P.S[k] = fmaf(P.dr[k], v.bg[0], fmaf(P.dg[k], v.bg[1], P.db[k] * v.bg[2]));
    maxn = max(maxn, P.nc[k]);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) maxn = max(maxn, __shfl_xor(maxn, d, 64));
  maxn = __builtin_amdgcn_readfirstlane(maxn);
  const int start = static_cast<int>(ranges[tile].x);
  // Lanes l, l + 16, l + 32, l + 48 share a pixel column when the tile is at most 16 wide.
  constexpr bool kCols = 16 % TILE == 0;
  const int out_k = kCols ? col_index(lane) : rs_index(lane & 15);
  const bool out_lane = kCols ? out_k >= 0 : lane < 16 && ((lane & 1) == 0 || lane == 1);
  uint32_t n_eval = 0, n_used = 0;
  // The forward's load pipeline, walking list positions maxn - 1 .. 0 (a step's record is
  // requested two steps ahead, its item id four).  The distance also keeps every wait clear of
  // the atomics issued at the end of the previous step: vector-memory operations complete in issue
  // order, and the newest operation a step waits for was issued two steps earlier.  Positions
  // below 0 are clamped to 0 and their loads never used.
  const ListSrc src = make_list_src(pair_item, n_pairs, coef, blue, n_items);
  constexpr bool kMarked = C::kWaves == 1;   // the forward marked each pair's evaluated groups
  const int top = max(maxn - 1, 0);
  uint32_t u0 = uniform(load_item(src, start + top));
  uint32_t u1 = uniform(load_item(src, start + max(top - 1, 0)));
  uint32_t u2;
  Rec R0 = load_rec(src, u0);
  Rec R1 = load_rec(src, u1);
  Rec R2;
  uint32_t L1, L2 = load_item(src, start + max(top - 2, 0)), L0 = load_item(src, start + max(top - 3, 0));
  for (int j = maxn - 1; j >= 0; j -= 3) {
    u2 = uniform(L2);
    R2 = load_rec(src, u2);
    L1 = load_item(src, start + max(j - 4, 0));
    bwd_step<PPL, kMarked, kCols, STATS>(R0, u0, j, fx, P, lane, out_k, out_lane, grad2d, n_eval, n_used);
    if (j == 0) break;
    u0 = uniform(L0);
    R0 = load_rec(src, u0);
    L2 = load_item(src, start + max(j - 5, 0));
    bwd_step<PPL, kMarked, kCols, STATS>(R1, u1, j - 1, fx, P, lane, out_k, out_lane, grad2d, n_eval, n_used);
    if (j == 1) break;
    u1 = uniform(L1);
    R1 = load_rec(src, u1);
    L0 = load_item(src, start + max(j - 6, 0));
    bwd_step<PPL, kMarked, kCols, STATS>(R2, u2, j - 2, fx, P, lane, out_k, out_lane, grad2d, n_eval, n_used);
  }
  if (STATS) add_stats(stats, n_eval, n_used);
}

template <int TILE>
static vbm_status launch_fwd_t(const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges, const uint32_t* tile_order,
                               uint32_t* pair_item, int64_t n_pairs, const float* coef, const float* blue,
                               int64_t n_items, float* image, float* final_T, int32_t* n_contrib,
                               unsigned long long* stats, hipStream_t s) {
  const dim3 block(TileCfg<TILE>::kThreads);
  if (stats)
    hipLaunchKernelGGL((k_composite_fwd<TILE, true>), dim3(n_tiles), block, 0, s, views, n_views, ranges, tile_order, pair_item,
                       n_pairs, coef, blue, n_items, image, final_T, n_contrib, stats);
  else
    hipLaunchKernelGGL((k_composite_fwd<TILE, false>), dim3(n_tiles), block, 0, s, views, n_views, ranges, tile_order, pair_item,
                       n_pairs, coef, blue, n_items, image, final_T, n_contrib, stats);
  VBM_LAUNCH_CHECK("composite_fwd");
  return VBM_OK;
}

template <int TILE>
static vbm_status launch_bwd_t(const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges, const uint32_t* tile_order,
                               const uint32_t* pair_item, int64_t n_pairs, const float* coef, const float* blue,
                               const float* final_T,
                               const int32_t* n_contrib, const float* dL_dimg, float* grad2d, int64_t n_items,
                               unsigned long long* stats, hipStream_t s) {
  const dim3 block(TileCfg<TILE>::kThreads);
  if (stats)
    hipLaunchKernelGGL((k_composite_bwd<TILE, true>), dim3(n_tiles), block, 0, s, views, n_views, ranges, tile_order, pair_item,
                       n_pairs, coef, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats);
  else
    hipLaunchKernelGGL((k_composite_bwd<TILE, false>), dim3(n_tiles), block, 0, s, views, n_views, ranges, tile_order, pair_item,
                       n_pairs, coef, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats);
  VBM_LAUNCH_CHECK("composite_bwd");
  return VBM_OK;
}

vbm_status launch_composite_fwd(int tile, const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges, const uint32_t* tile_order,
                                uint32_t* pair_item, int64_t n_pairs, const float* coef, const float* blue,
                                int64_t n_items, float* image, float* final_T, int32_t* n_contrib,
                                unsigned long long* stats, hipStream_t s) {
  switch (tile) {
    case 8: return launch_fwd_t<8>(views, n_views, n_tiles, ranges, tile_order, pair_item, n_pairs, coef, blue, n_items, image, final_T, n_contrib, stats, s);
    case 16: return launch_fwd_t<16>(views, n_views, n_tiles, ranges, tile_order, pair_item, n_pairs, coef, blue, n_items, image, final_T, n_contrib, stats, s);
    case 32: return launch_fwd_t<32>(views, n_views, n_tiles, ranges, tile_order, pair_item, n_pairs, coef, blue, n_items, image, final_T, n_contrib, stats, s);
  }
  set_error("unsupported tile size %d", tile);
  return VBM_ERR_UNSUPPORTED;
}

vbm_status launch_composite_bwd(int tile, const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges, const uint32_t* tile_order,
                                const uint32_t* pair_item, int64_t n_pairs, const float* coef, const float* blue,
                                const float* final_T,
                                const int32_t* n_contrib, const float* dL_dimg, float* grad2d, int64_t n_items,
                                unsigned long long* stats, hipStream_t s) {
  switch (tile) {
    case 8: return launch_bwd_t<8>(views, n_views, n_tiles, ranges, tile_order, pair_item, n_pairs, coef, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats, s);
    case 16: return launch_bwd_t<16>(views, n_views, n_tiles, ranges, tile_order, pair_item, n_pairs, coef, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats, s);
    case 32: return launch_bwd_t<32>(views, n_views, n_tiles, ranges, tile_order, pair_item, n_pairs, coef, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats, s);
  }
  set_error("unsupported tile size %d", tile);
  return VBM_ERR_UNSUPPORTED;
}

}  // namespace vbm
