// Front-to-back alpha compositing and its reverse-order backward (Sec. 3, the Gaussian mixture
// rendered by the 3DGS rasteriser cited in Sec. 4.4).
//
// Work decomposition: one wave64 per 256 pixels of a tile (a 16x16 tile is one wave, a 32x32 tile
// four independent waves, an 8x8 tile one wave with one pixel per lane), each lane owning
// PPL = 4 pixels of ONE pixel column (rows 64 / TILE apart), so the horizontal offset to a
// Gaussian's centre is shared by a lane's pixels.  The tile's depth-sorted list is walked by every
// wave in lockstep, with each Gaussian's 36-byte record wave-uniform, in one of two ways chosen by
// the plan: through the scalar data cache into SGPRs, each record one list step ahead of its use
// (no LDS, no barriers, no per-lane copies of a uniform value); or staged in LDS, where the first
// LDSB lanes each gather one list entry's record with vector loads into a double-buffered batch
// that the wave then reads entry by entry.  Either way the per-Gaussian load cost is amortised over
// 256 pixels; a vector load of a uniform address instead would move 64 lanes' copies through the
// texture address and data units, which the list walk would saturate.
//
// The record holds the exponent in base 2 with the log-opacity folded in:
//   e2(d) = hA dx^2 + hB dx dy + hC dy^2 + log2(o) = log2(o) + power(d) log2(e),
// so alpha = min(0.99, 2^e2) costs one exponential and no multiply by the opacity.  Projection
// keeps only Gaussians with a positive-definite conic, for which power <= 0 at every pixel, so a
// "skip when power > 0" guard could only fire on float32 rounding near the centre and is left out.
// The forward keeps each pixel's transmittance in place; a pixel that stops records its list
// position as n_contrib and parks at a far row, where alpha underflows to zero.
//
// The backward walks the list in reverse from the wave's largest n_contrib, recomputes each
// pixel's transmittance from final_T by division and carries one scalar per pixel for the colour
// behind the current Gaussian (see bwd_step).  The geometric gradient is accumulated as three
// per-lane moments of dL/dpower (sum, first and second moment in dy); the lane's column offset dx
// turns them into the five sums the 2D parameters need.  Nine per-wave sums are then formed by
// cross-row lane swaps and a DPP reduction inside 16-lane rows (one value per lane), and nine lanes
// issue one float atomic each into the item's 64-byte accumulator row (one cache segment per pair
// instead of nine lines) -- only when some pixel contributed.  The atomics add those raw moments;
// the projection backward turns them into mean/conic/opacity gradients with the item's conic,
// since that map is linear.
#include <hip/hip_runtime.h>

#include "common.h"

namespace vbm {

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

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

// The forward reads pair values with vector buffer loads, three list steps ahead: they complete
// in issue order (so each is waited for exactly, without waiting for the next record's scalar
// loads) and a position past num_records reads zero instead of faulting.  num_records is a 32-bit
// byte count; the plan bounds the pair capacity by 2^30.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t item_rsrc(const uint32_t* pair_item, int64_t n_pairs) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(pair_item), (short)0,
                                           static_cast<int>(static_cast<uint32_t>(n_pairs * 4)), 0x00020000);
}
__device__ __forceinline__ uint32_t load_item(__amdgpu_buffer_rsrc_t items, int j) {
  return static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b32(items, 0, 4 * j, 0));
}

// Rewrites the n <= 3 pair values j, j + 1, j + 2 (uniform v0, v1, v2) of the marked copy with
// one vector store from lanes 0 .. n - 1.
__device__ __forceinline__ void store_pair_values(uint32_t* __restrict__ marked, int lane, int j, int n, uint32_t v0,
                                                  uint32_t v1, uint32_t v2) {
  const uint32_t v = lane == 0 ? v0 : lane == 1 ? v1 : v2;
  if (lane < n) marked[j + lane] = v;
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// The record of a (wave-uniform) pair value, fetched through the scalar data cache into SGPRs.
// The item id is clamped to the record arrays (a past-the-end or empty-list step reads a valid
// record that it then ignores).
__device__ __forceinline__ Rec load_rec_s(const float4* __restrict__ crec, const float* __restrict__ cblue,
                                          uint32_t pv, uint32_t imax) {
  const uint32_t it = min(pv & kItemMask, imax);
  const float4 a = crec[2 * it];
  const float4 b = crec[2 * it + 1];
  Rec r;
  r.mx = a.x;
  r.my = a.y;
  r.hA = a.z;
  r.hB = a.w;
  r.hC = b.x;
  r.lo = b.y;
  r.r = b.z;
  r.g = b.w;
  r.b = cblue[it];
  return r;
}

// Waits for every scalar load in flight (they may complete out of order, so only a full wait
// identifies one): the list walks call it where the next record's loads are about to be issued,
// so that the wait covers the record requested one step earlier and not the next one.
__device__ __forceinline__ void wait_scalar_loads() { __builtin_amdgcn_s_waitcnt(0xC07F); }

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

// One list step (0-based list position pos) of the forward for the lane's pixels:
// alpha = min(0.99, 2^e2); a pixel takes the Gaussian when alpha >= 1/255, unless the new
// transmittance would fall below 1e-4, in which case the pixel stops without it and records pos as
// the number of list entries its compositing took into account.  Only the lane groups in `reach`
// (the pair value's groups that the footprint can reach, uniform) are looked at.  Returns the mask
// of lane groups k that were evaluated: every group with a pixel that took the Gaussian is among
// them.
template <int PPL, bool STATS>
__device__ __forceinline__ uint32_t fwd_step(const Rec& r, uint32_t reach, int pos, float fx, float (&fy)[PPL],
                                             float (&T)[PPL], float (&cr)[PPL], float (&cg)[PPL], float (&cb)[PPL],
                                             int (&nvis)[PPL], uint32_t& n_eval, uint32_t& n_used) {
  uint32_t groups = 0;
  const float dx = r.mx - fx;
  const float u = fmaf(r.hA, dx * dx, r.lo);
  const float vb = r.hB * dx;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    // a group out of the footprint's rows: nothing to evaluate (a scalar bit test)
    if (!((reach >> k) & 1u)) {
      if (STATS) n_eval += fy[k] < kLiveBound ? 1u : 0u;
      continue;
    }
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
    T[k] -= w;
    // A live pixel keeps T >= 1e-4, so only one that takes the Gaussian can fall below: it stops
    // without it (rare, so handled in a uniform branch), its transmittance going back to the value
    // before the Gaussian (T + w, within a unit in the last place of it).
    if (wave_any(T[k] < kTMin)) {
      __asm__ volatile("" ::: "memory");   // keeps this a branch: the compiler would select both ways
      const bool stop = T[k] < kTMin;
      T[k] = stop ? T[k] + w : T[k];
      w = stop ? 0.0f : w;
      fy[k] = stop ? kDeadRow : fy[k];
      nvis[k] = stop ? pos : nvis[k];
      if (STATS) n_eval += stop ? 1u : 0u;
    }
    if (STATS) {
      n_eval += fy[k] < kLiveBound ? 1u : 0u;
      n_used += ok && fy[k] < kLiveBound ? 1u : 0u;
    }
    cr[k] = fmaf(r.r, w, cr[k]);
    cg[k] = fmaf(r.g, w, cg[k]);
    cb[k] = fmaf(r.b, w, cb[k]);
  }
  return groups;
}

// Records of an LDS batch (the optional staged list walk): B consecutive list entries, one per
// lane, loaded with per-lane vector loads and written to LDS, then read back at a uniform address
// by every list step of the batch.
template <int B>
struct LdsBatch {
  float4 a[2][B], b[2][B];
  float4 c[2][B];   // c.x: blue, c.y: the pair value's bits (a 16-byte slot, so that one address
                    // serves all the reads of an entry)
};

template <int B>
__device__ __forceinline__ void lds_put(LdsBatch<B>& L, int buf, int lane, const float4& ra, const float4& rb,
                                        float bl, uint32_t pv) {
  if (lane < B) {
    L.a[buf][lane] = ra;
    L.b[buf][lane] = rb;
    L.c[buf][lane].x = bl;
    L.c[buf][lane].y = __uint_as_float(pv);
  }
}

// The pair value of entry b, in a scalar register.
template <int B>
__device__ __forceinline__ uint32_t lds_pv(const LdsBatch<B>& L, int buf, int b) {
  return uniform(__float_as_uint(L.c[buf][b].y));
}

template <int B>
__device__ __forceinline__ Rec lds_get(const LdsBatch<B>& L, int buf, int b) {
  const float4 a = L.a[buf][b], c = L.b[buf][b];
  Rec r;
  r.mx = a.x;
  r.my = a.y;
  r.hA = a.z;
  r.hB = a.w;
  r.hC = c.x;
  r.lo = c.y;
  r.r = c.z;
  r.g = c.w;
  r.b = L.c[buf][b].x;
  return r;
}

// Lane-group marks of an LDS batch, one 4-bit nibble per list step, kept in wave-uniform 64-bit
// words (scalar registers, so collecting them costs the vector pipes nothing).  A step ORs its
// marks into the current word at bits 4 (b mod 16); every 16 steps the word is pushed onto a short
// queue of filled words (most recent first), so the per-step cost does not grow with the batch and
// no word is ever selected by a computed index (which would put them in scratch memory).
template <int B>
struct MarkWords {
  static_assert(B == 32 || B == 64, "16 list steps per word, two or four words");
  uint64_t cur = 0, w0 = 0, w1 = 0, w2 = 0, w3 = 0;
  int filled = 0;
  __device__ __forceinline__ void set(int b, uint32_t g) {
    cur |= static_cast<uint64_t>(g) << (4 * (b & 15));
    if ((b & 15) == 15) push();
  }
  // after the batch's n steps: pushes a partly filled last word
  __device__ __forceinline__ void finish(int n) {
    if (n & 15) push();
  }
  // The marks of step `lane` (lane < B).
  __device__ __forceinline__ uint32_t of_lane(int lane) const {
    const int q = filled - 1 - (lane >> 4);   // queue slot of the lane's word
    uint64_t x = q == 0 ? w0 : w1;
    if (B == 64) x = q == 2 ? w2 : (q == 3 ? w3 : x);
    return static_cast<uint32_t>(x >> (4 * (lane & 15))) & 15u;
  }

 private:
  __device__ __forceinline__ void push() {
    if (B == 64) {
      w3 = w2;
      w2 = w1;
    }
    w1 = w0;
    w0 = cur;
    cur = 0;
    ++filled;
  }
};

// Lane t's entry of the batch at list positions pos(t) (per-lane vector loads): its pair value and
// record (the record of a clamped item when the position lies outside [lo, hi], never read).
__device__ __forceinline__ void lds_fetch(const uint32_t* __restrict__ values, const float4* __restrict__ crec,
                                          const float* __restrict__ cblue, uint32_t imax, int pos, bool ok,
                                          uint32_t& pv, float4& ra, float4& rb, float& bl) {
  pv = ok ? values[pos] : 0u;
  const uint32_t it = min(pv & kItemMask, imax);
  ra = crec[2 * it];
  rb = crec[2 * it + 1];
  bl = cblue[it];
}

// LDSB = 0: records through the scalar cache (the default); LDSB = 32 or 64: the list is staged in
// LDS batches of that many entries (one wave per tile only), a tuning candidate.
template <int TILE, bool STATS, int LDSB>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_composite_fwd(
    const DevView* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ tile_order,
    const uint32_t* __restrict__ pair_item, int64_t n_pairs, uint32_t* __restrict__ pair_marked,
    const float* __restrict__ coef, const float* __restrict__ blue, int64_t n_items, float* __restrict__ image,
    float* __restrict__ final_T, int32_t* __restrict__ n_contrib, unsigned long long* __restrict__ stats) {
  using C = TileCfg<TILE>;
  constexpr int PPL = C::kPPL;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int wave = static_cast<int>(threadIdx.x) >> 6;
  const int tile = static_cast<int>(tile_order[blockIdx.x]);
  const DevView& v = views[find_view(views, n_views, tile)];
  const int local = tile - v.tile_offset;
  const int tx = local % v.tiles_x, ty = local / v.tiles_x;
  float fy[PPL], T[PPL], cr[PPL], cg[PPL], cb[PPL];
  int nvis[PPL];
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
  }
  const uint2 rg = ranges[tile];
  // the range is the same for every lane: keep it (and the list walk's counters) in scalar registers
  const int start = static_cast<int>(uniform(rg.x)), end = static_cast<int>(uniform(rg.y));
#pragma unroll
  for (int k = 0; k < PPL; ++k) nvis[k] = end - start;
  uint32_t n_eval = 0, n_used = 0;
  const int lastj = end > start ? end - 1 : start;
  // With one wave per tile, each processed pair value is copied to pair_marked with the mask of the
  // lane groups that the step evaluated in bits kItemBits.. (see fwd_step): the backward visits
  // only those, reading the copy through the scalar cache.
  constexpr bool kMark = C::kWaves == 1;
  const float4* __restrict__ crec = reinterpret_cast<const float4*>(coef);
  const uint32_t imax = n_items > 0 ? static_cast<uint32_t>(n_items - 1) : 0u;
  if constexpr (LDSB > 0) {
    static_assert(C::kWaves == 1, "LDS batches are wave-private");
    // Double-buffered batches: the next batch's entries are loaded into registers (one per lane)
    // while the current one is walked, then written to the other LDS buffer.  A single wave uses
    // the LDS, whose operations it issues in order, so no barrier separates the writes from the
    // reads.  The marks of a batch collect in uniform words and go out with one coalesced store
    // (lane b: step b).
    __shared__ LdsBatch<LDSB> L;
    uint32_t pv, pvc;
    float4 ra, rb;
    float bl;
    lds_fetch(pair_item, crec, blue, imax, start + lane, lane < LDSB && start + lane < end, pvc, ra, rb, bl);
    lds_put<LDSB>(L, 0, lane, ra, rb, bl, pvc);
    int buf = 0;
    for (int base = start; base < end; base += LDSB) {
      if (!any_live(fy)) break;
      const int nb = base + LDSB;
      lds_fetch(pair_item, crec, blue, imax, nb + lane, lane < LDSB && nb + lane < end, pv, ra, rb, bl);
      // batch length and first list position, kept scalar so that the step loop runs on the SALU
      const int n = static_cast<int>(uniform(static_cast<uint32_t>(min(LDSB, end - base))));
      const int pos0 = static_cast<int>(uniform(static_cast<uint32_t>(base - start)));
      MarkWords<LDSB> mw;
      for (int b = 0; b < n; ++b) {
        const Rec r = lds_get<LDSB>(L, buf, b);
        const uint32_t reach = lds_pv<LDSB>(L, buf, b) >> kItemBits;
        mw.set(b, fwd_step<PPL, STATS>(r, reach, pos0 + b, fx, fy, T, cr, cg, cb, nvis, n_eval, n_used));
      }
      mw.finish(n);
      if (lane < n) pair_marked[base + lane] = (pvc & kItemMask) | (mw.of_lane(lane) << kItemBits);
      buf ^= 1;
      pvc = pv;
      lds_put<LDSB>(L, buf, lane, ra, rb, bl, pv);
    }
  } else {
  // Records through the scalar cache one list step ahead of their use, pair values by vector loads
  // three steps ahead (measured faster here than scalar pair-value loads, which put a second
  // scalar round trip in front of every record), unrolled by three so that the item slots rotate
  // without copies.  All three steps of an iteration run; past the end of the list a record is a
  // duplicate whose log-opacity is set to -inf, so alpha = 0 and it changes nothing.
  const __amdgpu_buffer_rsrc_t irs = item_rsrc(pair_item, n_pairs);
  uint32_t u0 = uniform(load_item(irs, start)), u1, u2;
  Rec R0 = load_rec_s(crec, blue, u0, imax), R1, R2;
  uint32_t L1 = load_item(irs, min(start + 1, lastj)), L2 = load_item(irs, min(start + 2, lastj)),
           L0 = load_item(irs, min(start + 3, lastj));
  for (int j = start; j < end; j += 3) {
    if (!any_live(fy)) break;
    wait_scalar_loads();
    u1 = uniform(L1);
    R1 = load_rec_s(crec, blue, u1, imax);
    L1 = load_item(irs, min(j + 4, lastj));
    const uint32_t m0 = (u0 & kItemMask) | (fwd_step<PPL, STATS>(R0, u0 >> kItemBits, j - start, fx, fy, T, cr, cg, cb, nvis,
                                                                  n_eval, n_used) << kItemBits);
    wait_scalar_loads();
    R1.lo = j + 1 < end ? R1.lo : -__builtin_inff();
    u2 = uniform(L2);
    R2 = load_rec_s(crec, blue, u2, imax);
    L2 = load_item(irs, min(j + 5, lastj));
    const uint32_t un = uniform(L0);
    const uint32_t m1 = (u1 & kItemMask) | (fwd_step<PPL, STATS>(R1, u1 >> kItemBits, j - start + 1, fx, fy, T, cr, cg, cb, nvis,
                                                                  n_eval, n_used) << kItemBits);
    wait_scalar_loads();
    R2.lo = j + 2 < end ? R2.lo : -__builtin_inff();
    R0 = load_rec_s(crec, blue, un, imax);
    L0 = load_item(irs, min(j + 6, lastj));
    const uint32_t m2 = (u2 & kItemMask) | (fwd_step<PPL, STATS>(R2, u2 >> kItemBits, j - start + 2, fx, fy, T, cr, cg, cb, nvis,
                                                                  n_eval, n_used) << kItemBits);
    if (kMark) store_pair_values(pair_marked, lane, j, min(end - j, 3), m0, m1, m2);
    u0 = un;
  }
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
    n_contrib[v.pixel_offset + pix] = nvis[k];
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

template <int TILE, bool STATS, int LDSB>
__global__ __launch_bounds__(TileCfg<TILE>::kThreads) void k_composite_bwd(
    const DevView* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ tile_order,
    const uint32_t* __restrict__ pair_values, const float* __restrict__ coef,
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
  const int start = static_cast<int>(uniform(ranges[tile].x));
  // Lanes l, l + 16, l + 32, l + 48 share a pixel column when the tile is at most 16 wide.
  constexpr bool kCols = 16 % TILE == 0;
  const int out_k = kCols ? col_index(lane) : rs_index(lane & 15);
  const bool out_lane = kCols ? out_k >= 0 : lane < 16 && ((lane & 1) == 0 || lane == 1);
  uint32_t n_eval = 0, n_used = 0;
  // pair_values: the forward's marked copy with one wave per tile (marks of the groups it
  // evaluated), else the sorted pair values.
  constexpr bool kMarked = C::kWaves == 1;
  const float4* __restrict__ crec = reinterpret_cast<const float4*>(coef);
  const uint32_t imax = n_items > 0 ? static_cast<uint32_t>(n_items - 1) : 0u;
  if constexpr (LDSB > 0) {
    static_assert(C::kWaves == 1, "LDS batches are wave-private");
    // The forward's LDS batches walked in reverse: the batch ending at list position hi holds
    // positions hi, hi - 1, ... in lanes 0, 1, ...
    __shared__ LdsBatch<LDSB> L;
    uint32_t pv;
    float4 ra, rb;
    float bl;
    int hi = maxn - 1;
    lds_fetch(pair_values, crec, blue, imax, start + hi - lane, lane < LDSB && hi - lane >= 0, pv, ra, rb, bl);
    lds_put<LDSB>(L, 0, lane, ra, rb, bl, pv);
    int buf = 0;
    for (; hi >= 0; hi -= LDSB) {
      const int nh = hi - LDSB;
      lds_fetch(pair_values, crec, blue, imax, start + nh - lane, lane < LDSB && nh - lane >= 0, pv, ra, rb, bl);
      const int n = min(LDSB, hi + 1);
      for (int b = 0; b < n; ++b) {
        const Rec r = lds_get<LDSB>(L, buf, b);
        bwd_step<PPL, kMarked, kCols, STATS>(r, lds_pv<LDSB>(L, buf, b), hi - b, fx, P, lane, out_k, out_lane,
                                             grad2d, n_eval, n_used);
      }
      buf ^= 1;
      lds_put<LDSB>(L, buf, lane, ra, rb, bl, pv);
    }
  } else {
  // Records through the scalar cache one step ahead of their use, pair values through the scalar
  // cache one step before the record they address, walking positions maxn - 1 .. 0 (positions
  // below 0 are clamped to 0 and their loads never used).
  const int top = max(maxn - 1, 0);
  uint32_t u0 = pair_values[start + top];
  Rec R0 = load_rec_s(crec, blue, u0, imax), R1, R2;
  uint32_t u1 = pair_values[start + max(top - 1, 0)], u2;
  for (int j = maxn - 1; j >= 0; j -= 3) {
    wait_scalar_loads();
    R1 = load_rec_s(crec, blue, u1, imax);
    u2 = pair_values[start + max(j - 2, 0)];
    bwd_step<PPL, kMarked, kCols, STATS>(R0, u0, j, fx, P, lane, out_k, out_lane, grad2d, n_eval, n_used);
    if (j == 0) break;
    wait_scalar_loads();
    R2 = load_rec_s(crec, blue, u2, imax);
    u0 = pair_values[start + max(j - 3, 0)];
    bwd_step<PPL, kMarked, kCols, STATS>(R1, u1, j - 1, fx, P, lane, out_k, out_lane, grad2d, n_eval, n_used);
    if (j == 1) break;
    wait_scalar_loads();
    R0 = load_rec_s(crec, blue, u0, imax);
    u1 = pair_values[start + max(j - 4, 0)];
    bwd_step<PPL, kMarked, kCols, STATS>(R2, u2, j - 2, fx, P, lane, out_k, out_lane, grad2d, n_eval, n_used);
  }
  }
  if (STATS) add_stats(stats, n_eval, n_used);
}

template <int TILE, int LDSB>
static vbm_status launch_fwd_t(const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges,
                               const uint32_t* tile_order, const uint32_t* pair_item, int64_t n_pairs,
                               uint32_t* pair_marked, const float* coef, const float* blue, int64_t n_items,
                               float* image, float* final_T, int32_t* n_contrib, unsigned long long* stats,
                               hipStream_t s) {
  const dim3 block(TileCfg<TILE>::kThreads);
  if (stats)
    hipLaunchKernelGGL((k_composite_fwd<TILE, true, LDSB>), dim3(n_tiles), block, 0, s, views, n_views, ranges,
                       tile_order, pair_item, n_pairs, pair_marked, coef, blue, n_items, image, final_T, n_contrib,
                       stats);
  else
    hipLaunchKernelGGL((k_composite_fwd<TILE, false, LDSB>), dim3(n_tiles), block, 0, s, views, n_views, ranges,
                       tile_order, pair_item, n_pairs, pair_marked, coef, blue, n_items, image, final_T, n_contrib,
                       stats);
  VBM_LAUNCH_CHECK("composite_fwd");
  return VBM_OK;
}

template <int TILE, int LDSB>
static vbm_status launch_bwd_t(const DevView* views, int n_views, int64_t n_tiles, const uint2* ranges,
                               const uint32_t* tile_order, const uint32_t* pair_item, const uint32_t* pair_marked,
                               const float* coef, const float* blue, const float* final_T, const int32_t* n_contrib,
                               const float* dL_dimg, float* grad2d, int64_t n_items, unsigned long long* stats,
                               hipStream_t s) {
  const dim3 block(TileCfg<TILE>::kThreads);
  // one wave per tile: the forward's marked copy; otherwise the sorted pair values
  const uint32_t* values = TileCfg<TILE>::kWaves == 1 ? pair_marked : pair_item;
  if (stats)
    hipLaunchKernelGGL((k_composite_bwd<TILE, true, LDSB>), dim3(n_tiles), block, 0, s, views, n_views, ranges,
                       tile_order, values, coef, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats);
  else
    hipLaunchKernelGGL((k_composite_bwd<TILE, false, LDSB>), dim3(n_tiles), block, 0, s, views, n_views, ranges,
                       tile_order, values, coef, blue, final_T, n_contrib, dL_dimg, grad2d, n_items, stats);
  VBM_LAUNCH_CHECK("composite_bwd");
  return VBM_OK;
}

vbm_status launch_composite_fwd(int tile, int lds_batch, const DevView* views, int n_views, int64_t n_tiles,
                                const uint2* ranges, const uint32_t* tile_order, const uint32_t* pair_item,
                                int64_t n_pairs, uint32_t* pair_marked, const float* coef, const float* blue,
                                int64_t n_items, float* image, float* final_T, int32_t* n_contrib,
                                unsigned long long* stats, hipStream_t s) {
#define VBM_FWD(T, B)                                                                                              \
  return launch_fwd_t<T, B>(views, n_views, n_tiles, ranges, tile_order, pair_item, n_pairs, pair_marked, coef,   \
                            blue, n_items, image, final_T, n_contrib, stats, s)
  if (tile == 8 && lds_batch == 0) VBM_FWD(8, 0);
  if (tile == 8 && lds_batch == 32) VBM_FWD(8, 32);
  if (tile == 8 && lds_batch == 64) VBM_FWD(8, 64);
  if (tile == 16 && lds_batch == 0) VBM_FWD(16, 0);
  if (tile == 16 && lds_batch == 32) VBM_FWD(16, 32);
  if (tile == 16 && lds_batch == 64) VBM_FWD(16, 64);
  if (tile == 32 && lds_batch == 0) VBM_FWD(32, 0);
#undef VBM_FWD
  set_error("unsupported tile size %d with LDS batch %d", tile, lds_batch);
  return VBM_ERR_UNSUPPORTED;
}

vbm_status launch_composite_bwd(int tile, int lds_batch, const DevView* views, int n_views, int64_t n_tiles,
                                const uint2* ranges, const uint32_t* tile_order, const uint32_t* pair_item,
                                const uint32_t* pair_marked, const float* coef, const float* blue,
                                const float* final_T, const int32_t* n_contrib, const float* dL_dimg, float* grad2d,
                                int64_t n_items, unsigned long long* stats, hipStream_t s) {
#define VBM_BWD(T, B)                                                                                              \
  return launch_bwd_t<T, B>(views, n_views, n_tiles, ranges, tile_order, pair_item, pair_marked, coef, blue,       \
                            final_T, n_contrib, dL_dimg, grad2d, n_items, stats, s)
  if (tile == 8 && lds_batch == 0) VBM_BWD(8, 0);
  if (tile == 8 && lds_batch == 32) VBM_BWD(8, 32);
  if (tile == 8 && lds_batch == 64) VBM_BWD(8, 64);
  if (tile == 16 && lds_batch == 0) VBM_BWD(16, 0);
  if (tile == 16 && lds_batch == 32) VBM_BWD(16, 32);
  if (tile == 16 && lds_batch == 64) VBM_BWD(16, 64);
  if (tile == 32 && lds_batch == 0) VBM_BWD(32, 0);
#undef VBM_BWD
  set_error("unsupported tile size %d with LDS batch %d", tile, lds_batch);
  return VBM_ERR_UNSUPPORTED;
}

}  // namespace vbm
