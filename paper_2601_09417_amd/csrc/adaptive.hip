// vbm_adaptive_select: adaptive per-subband coefficient selection (Supp. A: global budget
// allocation across subbands, joint multi-channel sparsification, robust MAD-based thresholding,
// top-K selection under sparsity constraints).
//
// Every subband of the packed layout (the LLL block, then the seven detail blocks of each level
// from the coarsest) is cut into chunks of 16384 coefficients that never straddle a subband; one
// block per chunk.  The order statistics (the two medians and the K-th largest joint norm) come
// from four-pass 8-bit radix selects on float32 bit patterns (non-negative floats order like their
// bits), run for all subbands at once with per-subband histograms; the two middle ranks of a median
// are selected side by side, and the K_band-th largest joint norm alongside the median of the
// joint norms (it does not depend on the threshold: when fewer than K_band values pass T, the
// K-th largest is the smallest value >= T, which the count pass finds).  Every keep/drop decision
// uses float32 values computed in a fixed
// order; energies and budgets are float64.  Per-subband counts are summed from per-chunk counts
// (no same-address atomics across blocks).  Nothing is read back to the host.
#include <hip/hip_runtime.h>

#include <cmath>

#include "block_scan.h"
#include "common.h"

namespace vbm {
namespace {

constexpr int kT = 256;
constexpr int kChunk = 16384;
constexpr int kPer = kChunk / kT;
constexpr int kMaxBands = 7 * 10 + 1;

struct BandTable {
  int32_t nb;
  int64_t off[kMaxBands];
  int64_t n[kMaxBands];
  int64_t chunk0[kMaxBands + 1];   // first chunk of each subband; chunk0[nb] = number of chunks
};

// Select targets: 0 and 1 the two middle ranks (of v, then of |v - median|), 2 the K_band-th
// largest v (selected alongside the median; active when 1 <= K_band <= N).
constexpr int kTargets = 3;

struct BandState {
  uint32_t prefix[kTargets];   // key bits fixed so far, per select target
  uint32_t rank[kTargets];     // ascending 0-based rank still to find inside the prefix's bucket
  uint32_t use2;               // target 2 active
  uint32_t vmin;               // smallest v >= T (bit pattern; +inf when none)
  double E, quotient;   // reference energy, K_tot S / sum S
  int64_t K_band;       // max(min_band, floor(quotient))
  float med, mad, sigma, T, vK, thr;
  uint32_t C, K;        // #(v >= T), min(K_band, C)
  uint32_t kept, pad;
};

__device__ __forceinline__ int band_of(const BandTable& bt, int64_t chunk) {
  int b = 0;
  while (b + 1 < bt.nb && chunk >= bt.chunk0[b + 1]) ++b;
  return b;
}

// [begin, end) of chunk `chunk` inside subband b.
__device__ __forceinline__ void chunk_range(const BandTable& bt, int b, int64_t chunk, int64_t& begin, int64_t& end) {
  begin = bt.off[b] + (chunk - bt.chunk0[b]) * kChunk;
  end = min(begin + kChunk, bt.off[b] + bt.n[b]);
}

// Keys begin + (r0 + q) * 256 + thread, q < 16, with indices past `end` clamped to end - 1 (a chunk is
// never empty): the loads are unconditional so that all sixteen are in flight at once.
__device__ __forceinline__ void load16(const uint32_t* __restrict__ keys, int64_t begin, int64_t end, int r0,
                                       uint32_t (&k)[16]) {
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t i = begin + static_cast<int64_t>(r0 + q) * kT + threadIdx.x;
    k[q] = keys[i < end ? i : end - 1];
  }
}

__device__ __forceinline__ double block_sum_f64(double v, double* s_red) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  if (lane_id() == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kT / 64; ++w) t += s_red[w];
  __syncthreads();
  return t;
}

__device__ __forceinline__ uint32_t block_min_u32(uint32_t v, uint32_t* s_red) {
  for (int d = 32; d >= 1; d >>= 1) v = min(v, static_cast<uint32_t>(__shfl_xor(v, d, 64)));
  if (lane_id() == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t t = 0xFFFFFFFFu;
  for (int w = 0; w < kT / 64; ++w) t = min(t, s_red[w]);
  __syncthreads();
  return t;
}

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t* s_red) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  if (lane_id() == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t t = 0;
  for (int w = 0; w < kT / 64; ++w) t += s_red[w];
  __syncthreads();
  return t;
}

#pragma clang fp contract(off)
// Joint norm sqrt(((R^2 + G^2) + B^2) + A^2) in float32 (the order of the top-K key) as its bit
// pattern, and the chunk's reference-channel energy in float64 (fixed summation order).
__global__ __launch_bounds__(kT) void k_af_norm(const float* __restrict__ coeffs, int64_t M, BandTable bt, int ref,
                                               uint32_t* __restrict__ keys, double* __restrict__ epart) {
  __shared__ double s_red[kT / 64];
  const int b = band_of(bt, blockIdx.x);
  int64_t begin, end;
  chunk_range(bt, b, blockIdx.x, begin, end);
  double e = 0.0;
  for (int r0 = 0; r0 < kPer; r0 += 4) {
    // four coefficients (sixteen loads) in flight; indices past the chunk are clamped and unused
    float c[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = begin + static_cast<int64_t>(r0 + q) * kT + threadIdx.x;
      const int64_t j = i < end ? i : end - 1;
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) c[q][ch] = coeffs[ch * M + j];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = begin + static_cast<int64_t>(r0 + q) * kT + threadIdx.x;
      if (i >= end) continue;
      const float cr = c[q][0], cg = c[q][1], cb = c[q][2], ca = c[q][3];
      keys[i] = __float_as_uint(sqrt_rn_f32(((cr * cr + cg * cg) + cb * cb) + ca * ca));
      const double x = static_cast<double>(ref == 0 ? cr : ref == 1 ? cg : ref == 2 ? cb : ca);
      e += x * x;
    }
  }
  e = block_sum_f64(e, s_red);
  if (threadIdx.x == 0) epart[blockIdx.x] = e;
}

// E per subband (one block per subband, fixed order).
__global__ __launch_bounds__(kT) void k_af_energy(BandTable bt, const double* __restrict__ epart,
                                                 BandState* __restrict__ st) {
  __shared__ double s_red[kT / 64];
  const int b = blockIdx.x;
  double e = 0.0;
  for (int64_t c = bt.chunk0[b] + threadIdx.x; c < bt.chunk0[b + 1]; c += kT) e += epart[c];
  e = block_sum_f64(e, s_red);
  if (threadIdx.x == 0) st[b].E = e;
}

// Budgets K_{j,o} = max(min_band, floor(K_tot S / sum S)), S = E^alpha N^beta, and the first
// select: the two middle ranks of each subband's joint norms.
__global__ void k_af_budget(BandTable bt, BandState* __restrict__ st, int64_t K_tot, double alpha, double beta,
                            int64_t min_band) {
  __shared__ double s_S[kMaxBands];
  __shared__ double s_tot;
  const int b = threadIdx.x;
  if (b < bt.nb) s_S[b] = pow(st[b].E, alpha) * pow(static_cast<double>(bt.n[b]), beta);
  __syncthreads();
  if (b == 0) {
    double t = 0.0;
    for (int k = 0; k < bt.nb; ++k) t += s_S[k];
    s_tot = t;
  }
  __syncthreads();
  if (b < bt.nb) {
    const double q = s_tot == 0.0 ? 0.0 : static_cast<double>(K_tot) * s_S[b] / s_tot;
    const double f = floor(q);
    st[b].quotient = q;
    st[b].K_band = f > static_cast<double>(min_band) ? static_cast<int64_t>(f) : min_band;
    st[b].prefix[0] = st[b].prefix[1] = st[b].prefix[2] = 0u;
    st[b].rank[0] = static_cast<uint32_t>((bt.n[b] - 1) / 2);
    st[b].rank[1] = static_cast<uint32_t>(bt.n[b] / 2);
    const bool use2 = st[b].K_band >= 1 && st[b].K_band <= bt.n[b];
    st[b].use2 = use2 ? 1u : 0u;
    st[b].rank[2] = use2 ? static_cast<uint32_t>(bt.n[b] - st[b].K_band) : 0u;
  }
}

// Key of a coefficient for a select: the joint norm (mode 0) or its distance to the subband's
// median (mode 1), both non-negative float32 bit patterns.
__device__ __forceinline__ uint32_t select_key(uint32_t v, int mode, float med) {
  return mode == 0 ? v : __float_as_uint(fabsf(__uint_as_float(v) - med));
}

// Histogram of digit `shift` over the keys whose higher digits match each target's prefix (target 2
// only in the first select, mode 0).  Targets whose prefixes coincide share one histogram.
__global__ __launch_bounds__(kT) void k_af_hist(const uint32_t* __restrict__ keys, BandTable bt,
                                               const BandState* __restrict__ st, int mode, int shift,
                                               uint32_t* __restrict__ ghist) {
  __shared__ uint32_t h[kT / 64][kTargets][256];   // one set per wave: less contention
  const int b = band_of(bt, blockIdx.x);
  int64_t begin, end;
  chunk_range(bt, b, blockIdx.x, begin, end);
  for (int x = threadIdx.x; x < (kT / 64) * kTargets * 256; x += kT) (&h[0][0][0])[x] = 0;
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const uint32_t hi_mask = shift >= 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
  const uint32_t p0 = st[b].prefix[0] & hi_mask, p1 = st[b].prefix[1] & hi_mask, p2 = st[b].prefix[2] & hi_mask;
  const bool same01 = p0 == p1;
  const bool use2 = mode == 0 && st[b].use2 != 0u;
  const bool own2 = use2 && p2 != p0 && p2 != p1;   // target 2 needs its own histogram
  const float med = st[b].med;
  for (int r0 = 0; r0 < kPer; r0 += 16) {
    uint32_t kk[16];
    load16(keys, begin, end, r0, kk);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (begin + static_cast<int64_t>(r0 + q) * kT + threadIdx.x >= end) continue;
      const uint32_t k = select_key(kk[q], mode, med);
      const uint32_t d = (k >> shift) & 255u;
      const uint32_t hk = k & hi_mask;
      if (hk == p0) atomicAdd(&h[w][0][d], 1u);
      else if (!same01 && hk == p1) atomicAdd(&h[w][1][d], 1u);
      else if (own2 && hk == p2) atomicAdd(&h[w][2][d], 1u);
    }
  }
  __syncthreads();
  uint32_t c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
  for (int ww = 0; ww < kT / 64; ++ww) {
    c0 += h[ww][0][threadIdx.x];
    c1 += h[ww][1][threadIdx.x];
    c2 += h[ww][2][threadIdx.x];
  }
  if (same01) c1 = c0;
  if (use2 && !own2) c2 = p2 == p0 ? c0 : c1;
  uint32_t* g = ghist + static_cast<int64_t>(b) * (kTargets * 256);
  if (c0) atomicAdd(&g[threadIdx.x], c0);
  if (c1) atomicAdd(&g[256 + threadIdx.x], c1);
  if (c2) atomicAdd(&g[512 + threadIdx.x], c2);
}

// Picks, per subband and target, the digit whose bucket holds the target rank; clears the
// histograms for the next pass.
__global__ __launch_bounds__(kT) void k_af_pick(BandState* __restrict__ st, uint32_t* __restrict__ ghist, int shift) {
  const int b = blockIdx.x, d = threadIdx.x;
  uint32_t* g = ghist + static_cast<int64_t>(b) * (kTargets * 256);
  uint32_t hv[kTargets], below[kTargets], tot;
#pragma unroll
  for (int t = 0; t < kTargets; ++t) {
    hv[t] = g[256 * t + d];
    below[t] = block_excl_scan(hv[t], &tot);
  }
  uint32_t r[kTargets];
#pragma unroll
  for (int t = 0; t < kTargets; ++t) r[t] = st[b].rank[t];
  __syncthreads();
#pragma unroll
  for (int t = 0; t < kTargets; ++t) {
    if (below[t] <= r[t] && r[t] < below[t] + hv[t]) {
      st[b].prefix[t] |= static_cast<uint32_t>(d) << shift;
      st[b].rank[t] = r[t] - below[t];
    }
    g[256 * t + d] = 0;
  }
}

__device__ __forceinline__ float mid_mean(const BandState& s) {
  return (__uint_as_float(s.prefix[0]) + __uint_as_float(s.prefix[1])) * 0.5f;
}

// Median of the joint norms; the next select (the same two ranks) runs on |v - median|.
__global__ void k_af_median(BandTable bt, BandState* __restrict__ st) {
  const int b = threadIdx.x;
  if (b >= bt.nb) return;
  st[b].med = mid_mean(st[b]);
  st[b].prefix[0] = st[b].prefix[1] = 0u;
  st[b].rank[0] = static_cast<uint32_t>((bt.n[b] - 1) / 2);
  st[b].rank[1] = static_cast<uint32_t>(bt.n[b] / 2);
}

// MAD, sigma = MAD / 0.6745 and the threshold T = lambda sigma (float32).
__global__ void k_af_thresh(BandTable bt, BandState* __restrict__ st, float lambda) {
  const int b = threadIdx.x;
  if (b >= bt.nb) return;
  const float mad = mid_mean(st[b]);
  const float sigma = __fdiv_rn(mad, 0.6745f);
  st[b].mad = mad;
  st[b].sigma = sigma;
  st[b].T = lambda * sigma;
}

// #(v >= T) and the smallest such v per chunk (combined per subband by k_af_band_sum); keys are
// non-negative float bit patterns, so their unsigned order is the float order.
__global__ __launch_bounds__(kT) void k_af_count(const uint32_t* __restrict__ keys, BandTable bt,
                                                const BandState* __restrict__ st, uint32_t* __restrict__ cnt,
                                                uint32_t* __restrict__ cmin) {
  __shared__ uint32_t s_red[kT / 64];
  const int b = band_of(bt, blockIdx.x);
  int64_t begin, end;
  chunk_range(bt, b, blockIdx.x, begin, end);
  const float T = st[b].T;
  uint32_t c = 0, mn = 0xFFFFFFFFu;
  for (int r0 = 0; r0 < kPer; r0 += 16) {
    uint32_t kk[16];
    load16(keys, begin, end, r0, kk);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const bool in = begin + static_cast<int64_t>(r0 + q) * kT + threadIdx.x < end && __uint_as_float(kk[q]) >= T;
      c += in ? 1u : 0u;
      mn = in ? min(mn, kk[q]) : mn;
    }
  }
  c = block_sum_u32(c, s_red);
  mn = block_min_u32(mn, s_red);
  if (threadIdx.x == 0) {
    cnt[blockIdx.x] = c;
    cmin[blockIdx.x] = mn;
  }
}

// Sum of the per-chunk counts of each subband (one block per subband) into C and the smallest
// v >= T into vmin (which = 0, from k_af_count), or into the kept count (which = 1).
__global__ __launch_bounds__(kT) void k_af_band_sum(BandTable bt, const uint32_t* __restrict__ cnt,
                                                   const uint32_t* __restrict__ cmin, int which,
                                                   BandState* __restrict__ st) {
  __shared__ uint32_t s_red[kT / 64];
  const int b = blockIdx.x;
  uint32_t c = 0, mn = 0xFFFFFFFFu;
  for (int64_t k = bt.chunk0[b] + threadIdx.x; k < bt.chunk0[b + 1]; k += kT) {
    c += cnt[k];
    if (which == 0) mn = min(mn, cmin[k]);
  }
  c = block_sum_u32(c, s_red);
  if (which == 0) mn = block_min_u32(mn, s_red);
  if (threadIdx.x == 0) {
    if (which == 0) {
      st[b].C = c;
      st[b].vmin = mn;
    } else {
      st[b].kept = c;
    }
  }
}

// K = min(K_band, C) and v_(K), the K-th largest joint norm: when K_band <= C it is the K_band-th
// largest, found by target 2 of the first select; otherwise K = C and the C largest values are
// exactly those >= T, so v_(C) is the smallest v >= T.  Keep threshold max(T, v_(K)), or +inf when
// K = 0.
__global__ void k_af_thr(BandTable bt, BandState* __restrict__ st) {
  const int b = threadIdx.x;
  if (b >= bt.nb) return;
  const int64_t C = static_cast<int64_t>(st[b].C);
  const int64_t K = st[b].K_band < C ? st[b].K_band : C;
  st[b].K = static_cast<uint32_t>(K);
  const float vK = K < 1 ? __builtin_inff()
                         : __uint_as_float(st[b].K_band <= C ? st[b].prefix[2] : st[b].vmin);
  st[b].vK = vK;
  st[b].thr = K >= 1 ? fmaxf(st[b].T, vK) : __builtin_inff();
}

// Kept coefficients per chunk.
__global__ __launch_bounds__(kT) void k_af_flags(const uint32_t* __restrict__ keys, BandTable bt,
                                                const BandState* __restrict__ st, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t s_red[kT / 64];
  const int b = band_of(bt, blockIdx.x);
  int64_t begin, end;
  chunk_range(bt, b, blockIdx.x, begin, end);
  const float thr = st[b].thr;
  uint32_t c = 0;
  for (int r0 = 0; r0 < kPer; r0 += 16) {
    uint32_t kk[16];
    load16(keys, begin, end, r0, kk);
#pragma unroll
    for (int q = 0; q < 16; ++q)
      c += begin + static_cast<int64_t>(r0 + q) * kT + threadIdx.x < end && __uint_as_float(kk[q]) >= thr ? 1u : 0u;
  }
  c = block_sum_u32(c, s_red);
  if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

__global__ __launch_bounds__(kT) void k_af_write(const uint32_t* __restrict__ keys, BandTable bt,
                                                const BandState* __restrict__ st, const uint32_t* __restrict__ offs,
                                                const uint32_t* __restrict__ cnt, int64_t capacity,
                                                int64_t* __restrict__ kept) {
  if (cnt[blockIdx.x] == 0) return;   // nothing kept in this chunk (uniform for the block)
  const int b = band_of(bt, blockIdx.x);
  int64_t begin, end;
  chunk_range(bt, b, blockIdx.x, begin, end);
  // Sub-rounds of 4096 coefficients in which each thread owns 16 consecutive ones, so the block's
  // scan of the per-thread counts numbers the kept ones in ascending index order.  A full sub-round
  // that starts on a 16-byte boundary (subband sizes are cubes of even numbers except for an odd
  // coarsest side) is read as four 16-byte vectors per thread.
  constexpr int kSub = 16;
  const float thr = st[b].thr;
  int64_t pos0 = static_cast<int64_t>(offs[blockIdx.x]);
  for (int64_t base = begin; base < end; base += kSub * kT) {
    uint32_t f = 0;
    const int64_t first = base + static_cast<int64_t>(threadIdx.x) * kSub;
    if (base + kSub * kT <= end && (reinterpret_cast<uintptr_t>(keys + base) & 15u) == 0) {
      const uint4* src = reinterpret_cast<const uint4*>(keys + first);
#pragma unroll
      for (int q = 0; q < kSub / 4; ++q) {
        const uint4 k4 = src[q];
        f |= (__uint_as_float(k4.x) >= thr ? 1u : 0u) << (4 * q);
        f |= (__uint_as_float(k4.y) >= thr ? 1u : 0u) << (4 * q + 1);
        f |= (__uint_as_float(k4.z) >= thr ? 1u : 0u) << (4 * q + 2);
        f |= (__uint_as_float(k4.w) >= thr ? 1u : 0u) << (4 * q + 3);
      }
    } else {
      for (int r = 0; r < kSub; ++r) {
        const int64_t i = first + r;
        if (i < end && __uint_as_float(keys[i]) >= thr) f |= 1u << r;
      }
    }
    uint32_t tot;
    int64_t pos = pos0 + block_excl_scan(static_cast<uint32_t>(__popc(f)), &tot);
    for (int r = 0; r < kSub; ++r) {
      if (!((f >> r) & 1u)) continue;
      if (pos < capacity) kept[pos] = base + static_cast<int64_t>(threadIdx.x) * kSub + r;
      ++pos;
    }
    pos0 += tot;
  }
}

// Kept count and the per-subband statistics.
__global__ void k_af_final(BandTable bt, const BandState* __restrict__ st, const uint32_t* __restrict__ total,
                           int64_t* __restrict__ count_dev, double* __restrict__ stats) {
  const int b = threadIdx.x;
  if (b == 0) count_dev[0] = static_cast<int64_t>(total[0]);
  if (b >= bt.nb || !stats) return;
  const BandState& s = st[b];
  double* o = stats + static_cast<int64_t>(b) * VBM_ADAPTIVE_STATS;
  o[0] = s.E;
  o[1] = static_cast<double>(bt.n[b]);
  o[2] = s.quotient;
  o[3] = static_cast<double>(s.K_band);
  o[4] = s.med;
  o[5] = s.mad;
  o[6] = s.sigma;
  o[7] = s.T;
  o[8] = s.C;
  o[9] = s.K;
  o[10] = s.vK;
  o[11] = static_cast<double>(s.kept);
}

bool make_table(int G, int J, BandTable* bt) {
  if (7 * J + 1 > kMaxBands) return false;
  bt->nb = 7 * J + 1;
  int64_t off = 0, chunk = 0;
  for (int b = 0; b < bt->nb; ++b) {
    const int j = b == 0 ? J : J - (b - 1) / 7;
    const int64_t side = G >> j;
    bt->off[b] = off;
    bt->n[b] = side * side * side;
    bt->chunk0[b] = chunk;
    off += bt->n[b];
    chunk += ceil_div(bt->n[b], kChunk);
  }
  bt->chunk0[bt->nb] = chunk;
  return off == static_cast<int64_t>(G) * G * G;
}

struct AdaptiveWs {
  uint32_t* keys;
  double* epart;
  uint32_t* cnt;
  uint32_t* cmin;
  uint32_t* offs;
  uint32_t* total;
  BandState* st;
  uint32_t* ghist;
  void* scan;
};

AdaptiveWs carve(Carver& c, int64_t M, int64_t chunks) {
  AdaptiveWs w;
  w.keys = c.take<uint32_t>(M);
  w.epart = c.take<double>(chunks);
  w.cnt = c.take<uint32_t>(chunks);
  w.cmin = c.take<uint32_t>(chunks);
  w.offs = c.take<uint32_t>(chunks);
  w.total = c.take<uint32_t>(1);
  w.st = c.take<BandState>(kMaxBands);
  w.ghist = c.take<uint32_t>(static_cast<size_t>(kMaxBands) * kTargets * 256);
  w.scan = c.take<char>(scan_scratch_bytes(chunks));
  return w;
}

bool grid_ok(int G, int J) { return G >= 2 && G <= 1024 && J >= 1 && J <= 10 && (G % (1 << J)) == 0 && (G >> J) >= 2; }

}  // namespace
}  // namespace vbm

using namespace vbm;

extern "C" size_t vbm_adaptive_workspace_size(int32_t G, int32_t J) {
  BandTable bt;
  if (!grid_ok(G, J) || !make_table(G, J, &bt)) return 0;
  Carver c(nullptr);
  carve(c, static_cast<int64_t>(G) * G * G, bt.chunk0[bt.nb]);
  return align_up(c.off, 256);
}

extern "C" vbm_status vbm_adaptive_select(const float* coeffs, int32_t G, int32_t J, const vbm_adaptive_opts* opts,
                                          int64_t capacity, int64_t* kept_index, int64_t* count_dev,
                                          double* band_stats, void* ws, size_t ws_bytes, void* stream) {
  if (!coeffs || !opts || !kept_index || !count_dev || !ws) {
    set_error("vbm_adaptive_select: null pointer");
    return VBM_ERR_INVALID;
  }
  BandTable bt;
  if (!grid_ok(G, J) || !make_table(G, J, &bt)) {
    set_error("vbm_adaptive_select: bad G=%d J=%d", G, J);
    return VBM_ERR_INVALID;
  }
  const int64_t M = static_cast<int64_t>(G) * G * G;
  if (opts->K_tot < 1 || opts->K_tot > M || opts->min_band < 0 || opts->min_band > M ||
      !(opts->lambda >= 0.0f) || !std::isfinite(opts->lambda) || !(opts->alpha >= 0.0) || !(opts->beta >= 0.0) ||
      !std::isfinite(opts->alpha) || !std::isfinite(opts->beta) || opts->ref_channel < 0 || opts->ref_channel > 3) {
    set_error("vbm_adaptive_select: need 1 <= K_tot <= G^3, 0 <= min_band <= G^3, finite lambda, alpha, "
              "beta >= 0 and ref_channel in 0..3");
    return VBM_ERR_INVALID;
  }
  if (capacity < 0) {
    set_error("vbm_adaptive_select: negative capacity");
    return VBM_ERR_INVALID;
  }
  if (ws_bytes < vbm_adaptive_workspace_size(G, J)) {
    set_error("vbm_adaptive_select: workspace %zu < %zu", ws_bytes, vbm_adaptive_workspace_size(G, J));
    return VBM_ERR_WORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t chunks = bt.chunk0[bt.nb];
  Carver c(ws);
  const AdaptiveWs w = carve(c, M, chunks);
  const dim3 cg(static_cast<unsigned>(chunks)), blk(kT), nbg(static_cast<unsigned>(bt.nb));

  hipLaunchKernelGGL(k_af_norm, cg, blk, 0, s, coeffs, M, bt, opts->ref_channel, w.keys, w.epart);
  VBM_LAUNCH_CHECK("adaptive_norm");
  VBM_TRY(fill_u32(w.ghist, 0u, static_cast<int64_t>(kMaxBands) * kTargets * 256, s));
  hipLaunchKernelGGL(k_af_energy, nbg, blk, 0, s, bt, w.epart, w.st);
  VBM_LAUNCH_CHECK("adaptive_energy");
  hipLaunchKernelGGL(k_af_budget, dim3(1), dim3(128), 0, s, bt, w.st, opts->K_tot, opts->alpha, opts->beta,
                     static_cast<int64_t>(opts->min_band));
  VBM_LAUNCH_CHECK("adaptive_budget");
  // two radix selects: median(v) together with the K_band-th largest v, then median(|v - median|)
  for (int sel = 0; sel < 2; ++sel) {
    for (int shift = 24; shift >= 0; shift -= 8) {
      hipLaunchKernelGGL(k_af_hist, cg, blk, 0, s, w.keys, bt, w.st, sel, shift, w.ghist);
      VBM_LAUNCH_CHECK("adaptive_hist");
      hipLaunchKernelGGL(k_af_pick, nbg, blk, 0, s, w.st, w.ghist, shift);
      VBM_LAUNCH_CHECK("adaptive_pick");
    }
    if (sel == 0) {
      hipLaunchKernelGGL(k_af_median, dim3(1), dim3(128), 0, s, bt, w.st);
      VBM_LAUNCH_CHECK("adaptive_median");
    }
  }
  hipLaunchKernelGGL(k_af_thresh, dim3(1), dim3(128), 0, s, bt, w.st, opts->lambda);
  VBM_LAUNCH_CHECK("adaptive_thresh");
  hipLaunchKernelGGL(k_af_count, cg, blk, 0, s, w.keys, bt, w.st, w.cnt, w.cmin);
  VBM_LAUNCH_CHECK("adaptive_count");
  hipLaunchKernelGGL(k_af_band_sum, nbg, blk, 0, s, bt, w.cnt, w.cmin, 0, w.st);
  VBM_LAUNCH_CHECK("adaptive_band_sum");
  hipLaunchKernelGGL(k_af_thr, dim3(1), dim3(128), 0, s, bt, w.st);
  VBM_LAUNCH_CHECK("adaptive_thr");
  hipLaunchKernelGGL(k_af_flags, cg, blk, 0, s, w.keys, bt, w.st, w.cnt);
  VBM_LAUNCH_CHECK("adaptive_flags");
  hipLaunchKernelGGL(k_af_band_sum, nbg, blk, 0, s, bt, w.cnt, static_cast<const uint32_t*>(nullptr), 1, w.st);
  VBM_LAUNCH_CHECK("adaptive_band_sum");
  VBM_TRY(scan_exclusive_u32(w.cnt, w.offs, chunks, nullptr, w.total, w.scan, s));
  hipLaunchKernelGGL(k_af_write, cg, blk, 0, s, w.keys, bt, w.st, w.offs, w.cnt, capacity, kept_index);
  VBM_LAUNCH_CHECK("adaptive_write");
  hipLaunchKernelGGL(k_af_final, dim3(1), dim3(128), 0, s, bt, w.st, w.total, count_dev, band_stats);
  VBM_LAUNCH_CHECK("adaptive_final");
  return VBM_OK;
}
