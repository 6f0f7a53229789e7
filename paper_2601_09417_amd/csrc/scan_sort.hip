// Device-wide exclusive scan and stable LSD radix sort (gfx950, wave64, 256-thread blocks).
//
// Scan: reduce -> single-workgroup scan of the block sums -> per-block scan with the block
// offset added.  Sort: per pass a digit histogram per 4096-key tile, an exclusive scan of every
// digit's row of the digit-major histogram (one block per digit, which also yields the digit
// totals), then a stable scatter that ranks equal digits
// inside each wave with ballots (a lane's rank = set bits of its digit-match mask below it) and
// across a wave's rounds through per-wave LDS counters, partitions the tile in LDS, and writes it
// out in digit order (coalesced runs).
#include <hip/hip_runtime.h>

#include "block_scan.h"
#include "common.h"

namespace vbm {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kChunk = kThreads * kItems;  // elements per block
constexpr int kWaves = kThreads / 64;
static_assert(kThreads == 256, "one thread per 8-bit digit in the scatter's LDS bookkeeping");

__device__ __forceinline__ bool aligned16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

__device__ __forceinline__ int64_t active_count(int64_t n_max, const uint32_t* n_dev) {
  if (!n_dev) return n_max;
  int64_t n = static_cast<int64_t>(*n_dev);
  return n < n_max ? n : n_max;
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const T* __restrict__ in, T* __restrict__ block_sums,
                                                          int64_t n_max, const uint32_t* n_dev) {
  const int64_t n = active_count(n_max, n_dev);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kChunk;
  T acc = 0;
  if (sizeof(T) == 4 && base + kChunk <= n && aligned16(in)) {
    // a full block of 32-bit values: four 16-byte loads per thread, consecutive across the wave
    const uint4* src = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
    for (int r = 0; r < kItems / 4; ++r) {
      const uint4 q = src[r * kThreads + threadIdx.x];
      acc += static_cast<T>(q.x) + static_cast<T>(q.y) + static_cast<T>(q.z) + static_cast<T>(q.w);
    }
  } else if (base < n) {
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      int64_t i = base + r * kThreads + threadIdx.x;
      if (i < n) acc += in[i];
    }
  }
  T tot;
  block_excl_scan(acc, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// One workgroup scans all block sums in place (exclusive), carrying across 4096-entry chunks.
template <class T>
__global__ __launch_bounds__(kThreads) void k_scan_top(T* __restrict__ sums, int64_t nb, T* __restrict__ total) {
  T carry = 0;
  for (int64_t base = 0; base < nb; base += kChunk) {
    T items[kItems];
    T acc = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      int64_t i = base + static_cast<int64_t>(threadIdx.x) * kItems + r;
      items[r] = i < nb ? sums[i] : T(0);
      acc += items[r];
    }
    T tot;
    T ex = block_excl_scan(acc, &tot) + carry;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      int64_t i = base + static_cast<int64_t>(threadIdx.x) * kItems + r;
      if (i < nb) sums[i] = ex;
      ex += items[r];
    }
    carry += tot;
  }
  if (total && threadIdx.x == 0) *total = carry;
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_scan_down(const T* __restrict__ in, T* __restrict__ out,
                                                        const T* __restrict__ block_offsets, int64_t n_max,
                                                        const uint32_t* n_dev) {
  const int64_t n = active_count(n_max, n_dev);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kChunk;
  if (base >= n) return;  // uniform per block
  // A full block of 32-bit values moves as four 16-byte vectors per thread (thread t owns
  // elements [16 t, 16 t + 16) of the block, as in the general path).
  const bool vec = sizeof(T) == 4 && base + kChunk <= n && aligned16(in) && aligned16(out);
  T items[kItems];
  T acc = 0;
  if (vec) {
    const uint4* src = reinterpret_cast<const uint4*>(in + base) + threadIdx.x * (kItems / 4);
#pragma unroll
    for (int r = 0; r < kItems / 4; ++r) {
      const uint4 q = src[r];
      items[4 * r] = static_cast<T>(q.x);
      items[4 * r + 1] = static_cast<T>(q.y);
      items[4 * r + 2] = static_cast<T>(q.z);
      items[4 * r + 3] = static_cast<T>(q.w);
    }
  } else {
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      int64_t i = base + static_cast<int64_t>(threadIdx.x) * kItems + r;
      items[r] = i < n ? in[i] : T(0);
    }
  }
#pragma unroll
  for (int r = 0; r < kItems; ++r) acc += items[r];
  T tot;
  T ex = block_excl_scan(acc, &tot) + block_offsets[blockIdx.x];
  if (vec) {
    uint4* dst = reinterpret_cast<uint4*>(out + base) + threadIdx.x * (kItems / 4);
#pragma unroll
    for (int r = 0; r < kItems / 4; ++r) {
      uint4 q;
      q.x = static_cast<uint32_t>(ex);
      ex += items[4 * r];
      q.y = static_cast<uint32_t>(ex);
      ex += items[4 * r + 1];
      q.z = static_cast<uint32_t>(ex);
      ex += items[4 * r + 2];
      q.w = static_cast<uint32_t>(ex);
      ex += items[4 * r + 3];
      dst[r] = q;
    }
  } else {
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      int64_t i = base + static_cast<int64_t>(threadIdx.x) * kItems + r;
      if (i < n) out[i] = ex;
      ex += items[r];
    }
  }
}

// Fills n values; a 16-byte aligned buffer is written as 16-byte vectors plus a scalar tail.
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t first = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  if (aligned16(p)) {
    const int64_t n4 = n >> 2;
    uint4* q = reinterpret_cast<uint4*>(p);
    const uint4 vv = make_uint4(v, v, v, v);
    for (int64_t i = first; i < n4; i += stride) q[i] = vv;
    for (int64_t i = 4 * n4 + first; i < n; i += stride) p[i] = v;
  } else {
    for (int64_t i = first; i < n; i += stride) p[i] = v;
  }
}

// ------------------------------------------------------------------ radix sort
template <class K>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const K* __restrict__ keys, uint32_t* __restrict__ hist,
                                                         int64_t n_max, const uint32_t* n_dev, int shift,
                                                         int bits, int64_t n_blocks) {
  __shared__ uint32_t s_hist[256];
  const int radix = 1 << bits;
  for (int d = threadIdx.x; d < radix; d += kThreads) s_hist[d] = 0;
  __syncthreads();
  const int64_t n = active_count(n_max, n_dev);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kChunk;
  const uint32_t mask = static_cast<uint32_t>(radix - 1);
  if (base < n) {
#pragma unroll 4
    for (int r = 0; r < kItems; ++r) {
      int64_t i = base + r * kThreads + threadIdx.x;
      if (i < n) {
        uint32_t d = static_cast<uint32_t>(keys[i] >> shift) & mask;
        atomicAdd(&s_hist[d], 1u);
      }
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < radix; d += kThreads) hist[static_cast<int64_t>(d) * n_blocks + blockIdx.x] = s_hist[d];
}

// Exclusive scan of one digit's row of the digit-major histogram (the digit's count in every
// tile, in tile order), in place; block d handles digit d and writes the digit's total.  The
// scatter adds the exclusive scan of the totals, so one launch replaces a device-wide scan.
__global__ __launch_bounds__(kThreads) void k_radix_digit_scan(uint32_t* __restrict__ hist, int64_t n_blocks,
                                                               uint32_t* __restrict__ totals) {
  uint32_t* row = hist + static_cast<int64_t>(blockIdx.x) * n_blocks;
  uint32_t carry = 0;
  for (int64_t base = 0; base < n_blocks; base += kChunk) {
    uint32_t items[kItems];
    uint32_t acc = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const int64_t i = base + static_cast<int64_t>(threadIdx.x) * kItems + r;
      items[r] = i < n_blocks ? row[i] : 0u;
      acc += items[r];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(acc, &tot) + carry;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const int64_t i = base + static_cast<int64_t>(threadIdx.x) * kItems + r;
      if (i < n_blocks) row[i] = ex;
      ex += items[r];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Stable scatter of one 4096-key tile.  Wave w owns keys [1024 w, 1024 w + 1024) and ranks them
// in 16 rounds of 64 against its own LDS digit counters: a lane's rank among the round's equal
// digits comes from ballots, and the wave's LDS operations complete in issue order, so a round
// reads its digits' counters before its leaders advance them with no barrier in between.  After
// one barrier the per-wave counters become per-wave bases (digit start in the tile plus the counts
// of the lower waves), the tile is partitioned in LDS, and it is written out in digit order, so
// consecutive lanes store to consecutive addresses of a digit's output run.
template <class K>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                            K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                            const uint32_t* __restrict__ offsets,
                                                            const uint32_t* __restrict__ digit_totals, int64_t n_max,
                                                            const uint32_t* n_dev, int shift, int bits,
                                                            int64_t n_blocks) {
  constexpr int kPerWave = kChunk / kWaves;
  __shared__ K s_key[kChunk];
  __shared__ uint32_t s_val[kChunk];
  __shared__ uint32_t s_cnt[kWaves][256];   // per-wave digit counts, then per-wave digit bases
  __shared__ uint32_t s_start[256];         // start of each digit in the partitioned tile
  __shared__ uint32_t s_glob[256];          // global start of this tile's run of each digit
  const int64_t n = active_count(n_max, n_dev);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kChunk;
  if (base >= n) return;  // uniform per block
  const int count = static_cast<int>(min(static_cast<int64_t>(kChunk), n - base));
  const int radix = 1 << bits;
  const uint32_t mask = static_cast<uint32_t>(radix - 1);
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  for (int x = threadIdx.x; x < kWaves * 256; x += kThreads) (&s_cnt[0][0])[x] = 0;
  {
    // global start of digit d's run from this tile: all keys of lower digits, plus digit d's keys
    // in the lower tiles
    const bool has = static_cast<int>(threadIdx.x) < radix;
    uint32_t all;
    const uint32_t below = block_excl_scan(has ? digit_totals[threadIdx.x] : 0u, &all);
    if (has) s_glob[threadIdx.x] = below + offsets[static_cast<int64_t>(threadIdx.x) * n_blocks + blockIdx.x];
  }
  K keys[kItems];
  uint32_t vals[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int li = w * kPerWave + r * 64 + lane;
    keys[r] = li < count ? kin[base + li] : K(0);
    vals[r] = li < count ? vin[base + li] : 0u;
  }
  __syncthreads();
  uint32_t slot[kItems];   // rank among the wave's keys of the same digit
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const bool valid = w * kPerWave + r * 64 + lane < count;
    const uint32_t d = static_cast<uint32_t>(keys[r] >> shift) & mask;
    uint64_t m = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t rank = popc_below(m);
    const uint32_t before = s_cnt[w][d];
    if (valid && rank == 0) s_cnt[w][d] = before + static_cast<uint32_t>(__popcll(m));
    slot[r] = before + rank;
  }
  __syncthreads();
  {
    uint32_t c[kWaves], t = 0;
#pragma unroll
    for (int ww = 0; ww < kWaves; ++ww) {
      c[ww] = s_cnt[ww][threadIdx.x];
      t += c[ww];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(t, &tot);
    s_start[threadIdx.x] = run;
#pragma unroll
    for (int ww = 0; ww < kWaves; ++ww) {
      s_cnt[ww][threadIdx.x] = run;
      run += c[ww];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    if (w * kPerWave + r * 64 + lane < count) {
      const uint32_t pos = s_cnt[w][static_cast<uint32_t>(keys[r] >> shift) & mask] + slot[r];
      s_key[pos] = keys[r];
      s_val[pos] = vals[r];
    }
  }
  __syncthreads();
  // write out in digit order
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int lp = r * kThreads + threadIdx.x;
    if (lp < count) {
      const K key = s_key[lp];
      const uint32_t d = static_cast<uint32_t>(key >> shift) & mask;
      const uint32_t gp = s_glob[d] + (static_cast<uint32_t>(lp) - s_start[d]);
      kout[gp] = key;
      vout[gp] = s_val[lp];
    }
  }
}

}  // namespace

size_t scan_scratch_bytes(int64_t n_max) {
  int64_t nb = ceil_div(n_max > 0 ? n_max : 1, kChunk);
  return align_up(static_cast<size_t>(nb) * 8, 256) + 256;
}

template <class T>
static vbm_status scan_impl(const T* in, T* out, int64_t n_max, const uint32_t* n_dev, T* total_dev, void* scratch,
                            hipStream_t s) {
  if (n_max <= 0) return VBM_OK;
  const int64_t nb = ceil_div(n_max, kChunk);
  T* sums = static_cast<T*>(scratch);
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3(nb), dim3(kThreads), 0, s, in, sums, n_max, n_dev);
  VBM_LAUNCH_CHECK("scan_reduce");
  hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(kThreads), 0, s, sums, nb, total_dev);
  VBM_LAUNCH_CHECK("scan_top");
  hipLaunchKernelGGL(k_scan_down<T>, dim3(nb), dim3(kThreads), 0, s, in, out, sums, n_max, n_dev);
  VBM_LAUNCH_CHECK("scan_down");
  return VBM_OK;
}

vbm_status scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n_max, const uint32_t* n_dev,
                              uint32_t* total_dev, void* scratch, hipStream_t s) {
  return scan_impl<uint32_t>(in, out, n_max, n_dev, total_dev, scratch, s);
}

vbm_status scan_exclusive_u64(const uint64_t* in, uint64_t* out, int64_t n_max, const uint32_t* n_dev,
                              uint64_t* total_dev, void* scratch, hipStream_t s) {
  return scan_impl<uint64_t>(in, out, n_max, n_dev, total_dev, scratch, s);
}

vbm_status fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return VBM_OK;
  int64_t blocks = ceil_div(ceil_div(n, 4), 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, value, n);
  VBM_LAUNCH_CHECK("fill_u32");
  return VBM_OK;
}

size_t radix_scratch_bytes(int64_t n_max, int digit_bits) {
  const int64_t nb = ceil_div(n_max > 0 ? n_max : 1, kChunk);
  const int64_t hist = static_cast<int64_t>(1 << digit_bits) * nb;
  return align_up(static_cast<size_t>(hist) * 4, 256) + 256 * 4;
}

template <class K>
vbm_status radix_sort_pairs(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t n_max, const uint32_t* n_dev,
                            int end_bit, int digit_bits, void* scratch, hipStream_t s, bool* result_in_k1) {
  *result_in_k1 = false;
  if (n_max <= 0 || end_bit <= 0) return VBM_OK;
  if (digit_bits < 1 || digit_bits > 8) {
    set_error("radix digit width %d outside 1..8", digit_bits);
    return VBM_ERR_INVALID;
  }
  const int64_t nb = ceil_div(n_max, kChunk);
  const int64_t hist_n = static_cast<int64_t>(1 << digit_bits) * nb;
  uint32_t* hist = static_cast<uint32_t*>(scratch);
  uint32_t* totals = reinterpret_cast<uint32_t*>(static_cast<char*>(scratch) +
                                                 align_up(static_cast<size_t>(hist_n) * 4, 256));
  K* kin = k0;
  uint32_t* vin = v0;
  K* kout = k1;
  uint32_t* vout = v1;
  for (int shift = 0; shift < end_bit; shift += digit_bits) {
    const int bits = (end_bit - shift) < digit_bits ? (end_bit - shift) : digit_bits;
    hipLaunchKernelGGL(k_radix_hist<K>, dim3(nb), dim3(kThreads), 0, s, kin, hist, n_max, n_dev, shift, bits, nb);
    VBM_LAUNCH_CHECK("radix_hist");
    hipLaunchKernelGGL(k_radix_digit_scan, dim3(1 << bits), dim3(kThreads), 0, s, hist, nb, totals);
    VBM_LAUNCH_CHECK("radix_digit_scan");
    hipLaunchKernelGGL(k_radix_scatter<K>, dim3(nb), dim3(kThreads), 0, s, kin, vin, kout, vout, hist, totals, n_max,
                       n_dev, shift, bits, nb);
    VBM_LAUNCH_CHECK("radix_scatter");
    K* tk = kin;
    kin = kout;
    kout = tk;
    uint32_t* tv = vin;
    vin = vout;
    vout = tv;
    *result_in_k1 = !*result_in_k1;
  }
  return VBM_OK;
}

template vbm_status radix_sort_pairs<uint32_t>(uint32_t*, uint32_t*, uint32_t*, uint32_t*, int64_t, const uint32_t*,
                                               int, int, void*, hipStream_t, bool*);
template vbm_status radix_sort_pairs<uint64_t>(uint64_t*, uint32_t*, uint64_t*, uint32_t*, int64_t, const uint32_t*,
                                               int, int, void*, hipStream_t, bool*);

}  // namespace vbm
