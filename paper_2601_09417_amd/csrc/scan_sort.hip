// Device-wide exclusive scan and stable LSD radix sort (gfx950, wave64, 256-thread blocks).
//
// Scan: reduce -> single-workgroup scan of the block sums -> per-block scan with the block
// offset added.  Sort: one histogram kernel counts the digits of every pass in one read of the
// keys, then each pass is a single kernel over 8192-key tiles that ranks equal digits inside each
// wave with ballots (a lane's rank = set bits of its digit-match mask below it) and across a
// wave's rounds through per-wave LDS counters, learns the earlier tiles' digit counts by
// decoupled look-back, partitions the tile in LDS, and writes it out in digit order (coalesced
// runs).
#include <hip/hip_runtime.h>

#include "block_scan.h"
#include "common.h"

namespace vbm {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kChunk = kThreads * kItems;  // elements per block
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
// One-sweep LSD radix sort (after Adinets and Garland's Onesweep, built on Merrill and Garland's
// decoupled look-back): one histogram kernel counts the digits of every pass in a single read of
// the keys, a small kernel adds the per-block counts into digit totals, and then every pass is one
// kernel.  A pass block takes its key tile in acquisition order from a counter, ranks the tile's
// keys, publishes the tile's digit counts, and finds how many keys of each digit the earlier tiles
// hold by walking back over their published counts (a tile that has already found its own prefix
// publishes that, so the walk stops there).  No per-pass histogram or scan launch and no per-tile
// digit offsets in memory.
constexpr int kUpThreads = 512;       // histogram block
constexpr int kUpBlocksMax = 256;     // histogram grid: enough loads in flight to stream at the HBM rate
constexpr int kMaxPasses = 8;         // 32-bit keys with digits of at least 4 bits
constexpr int kTopThreads = 1024;     // digit-total block: 16 row groups x 64 columns
constexpr uint32_t kFlagAgg = 1u << 30;   // status word: the tile's own count of the digit
constexpr uint32_t kFlagInc = 2u << 30;   // status word: the count in this tile and every earlier one
constexpr uint32_t kCountMask = kFlagAgg - 1u;
constexpr int kFallbackRounds = 128;  // look-back rounds that find a tile unpublished before counting it directly
constexpr int kLookback = 8;          // earlier tiles' status words read per look-back round
// Threads of a one-sweep pass block (kItems keys each, so 8192-key tiles): at workload H the pass
// time per step was 0.435 ms with 4096-key tiles, 0.404 ms with 8192 and 0.461 ms with 16384 (one
// block per CU); fewer tiles shorten the look-back chain and lengthen each digit's output run.
constexpr int kSweepThreads = 512;

// Exclusive scan of one value per thread across a block of NT threads (NT a multiple of 64);
// block total in *total.  Every thread of the block must call it (it synchronises).
template <int NT, class T>
__device__ __forceinline__ T block_excl_scan_n(T v, T* total) {
  __shared__ T s_wave[NT / 64];
  const int w = threadIdx.x >> 6;
  T incl = wave_incl_scan(v);
  if (lane_id() == 63) s_wave[w] = incl;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    T x = s_wave[i];
    if (i < w) base += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

__device__ __forceinline__ uint32_t status_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Keys of digit d in the full tile j of CH keys (the look-back's fallback for a tile whose block has
// not published its counts).
template <int CH, class K>
__device__ uint32_t count_digit(const K* __restrict__ kin, int64_t j, int shift, uint32_t mask, uint32_t d) {
  const K* src = kin + j * CH;
  uint32_t c = 0;
  for (int i = 0; i < CH; ++i) c += (static_cast<uint32_t>(src[i] >> shift) & mask) == d ? 1u : 0u;
  return c;
}

// Digit counts of every pass in one read of the keys.  Block b takes 4096-key chunks b, b + G, ...
// and writes its counts as row b of part[G][passes * 256]; lane l adds into LDS copy l & 3, so
// equal digits within a wave (the top digits of clustered keys) contend four ways less.  The block
// also clears its share of the passes' look-back status words.
template <class K>
__global__ __launch_bounds__(kUpThreads) void k_radix_upsweep(const K* __restrict__ keys, int64_t n_max,
                                                              const uint32_t* n_dev, int end_bit, int digit_bits,
                                                              int passes, uint32_t* __restrict__ part,
                                                              uint32_t* __restrict__ clear, int64_t clear_n) {
  __shared__ uint32_t s_h[4][kMaxPasses * 256];
  const int R = passes * 256;
  for (int i = threadIdx.x; i < 4 * R; i += kUpThreads) s_h[i / R][i % R] = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kUpThreads + threadIdx.x; i < clear_n;
       i += static_cast<int64_t>(gridDim.x) * kUpThreads)
    clear[i] = 0u;
  __syncthreads();
  const int64_t n = active_count(n_max, n_dev);
  uint32_t* h = s_h[threadIdx.x & 3];
  constexpr int kPer = kChunk / kUpThreads;   // 8 keys per thread and chunk
  for (int64_t c = blockIdx.x; c * kChunk < n; c += gridDim.x) {
    const int64_t base = c * kChunk;
    K k[kPer];
    bool ok[kPer];
    if (sizeof(K) == 4 && base + kChunk <= n && aligned16(keys)) {
      // two 16-byte loads per thread, consecutive across the block
      const uint4* src = reinterpret_cast<const uint4*>(keys + base);
#pragma unroll
      for (int r = 0; r < kPer / 4; ++r) {
        const uint4 q = src[r * kUpThreads + threadIdx.x];
        k[4 * r] = static_cast<K>(q.x);
        k[4 * r + 1] = static_cast<K>(q.y);
        k[4 * r + 2] = static_cast<K>(q.z);
        k[4 * r + 3] = static_cast<K>(q.w);
        ok[4 * r] = ok[4 * r + 1] = ok[4 * r + 2] = ok[4 * r + 3] = true;
      }
    } else {
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        const int64_t i = base + r * kUpThreads + threadIdx.x;
        ok[r] = i < n;
        k[r] = ok[r] ? keys[i] : K(0);
      }
    }
    for (int p = 0; p < passes; ++p) {
      const int shift = p * digit_bits;
      const int bits = end_bit - shift < digit_bits ? end_bit - shift : digit_bits;
      const uint32_t mask = (1u << bits) - 1u;
#pragma unroll
      for (int r = 0; r < kPer; ++r)
        if (ok[r]) atomicAdd(&h[p * 256 + (static_cast<uint32_t>(k[r] >> shift) & mask)], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += kUpThreads)
    part[static_cast<int64_t>(blockIdx.x) * R + i] = (s_h[0][i] + s_h[1][i]) + (s_h[2][i] + s_h[3][i]);
}

// Digit totals: column sums of part[G][R].  Block c sums columns [64 c, 64 c + 64); its 16 row
// groups take every 16th row, so each thread has at most G / 16 independent loads.
__global__ __launch_bounds__(kTopThreads) void k_radix_totals(const uint32_t* __restrict__ part, int G, int R,
                                                             uint32_t* __restrict__ tot) {
  __shared__ uint32_t s[kTopThreads / 64][64];
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int rg = threadIdx.x >> 6;
  uint32_t acc = 0;
  if (col < R)
    for (int r = rg; r < G; r += kTopThreads / 64) acc += part[static_cast<int64_t>(r) * R + col];
  s[rg][threadIdx.x & 63] = acc;
  __syncthreads();
  if (threadIdx.x < 64 && col < R) {
    uint32_t t = 0;
#pragma unroll
    for (int g = 0; g < kTopThreads / 64; ++g) t += s[g][threadIdx.x];
    tot[col] = t;
  }
}

// One stable pass over tiles of NT x 16 keys.  Wave w of a tile owns keys [1024 w, 1024 w + 1024)
// and ranks them in 16 rounds of 64 against its own LDS digit counters: a lane's rank among the
// round's equal digits comes from ballots, and the wave's LDS operations complete in issue order,
// so a round reads its digits' counters before its leaders advance them with no barrier in
// between.  The per-wave counts give the tile's digit counts (published for the later tiles) and
// per-wave bases; the look-back gives the keys of each digit in the earlier tiles; the tile is
// partitioned in LDS and written out in digit order, so consecutive lanes store to consecutive
// addresses of a digit's output run.
template <int NT, class K>
__global__ __launch_bounds__(NT) void k_radix_onesweep(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                             K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                             const uint32_t* __restrict__ totals,
                                                             uint32_t* __restrict__ status, int64_t n_max,
                                                             const uint32_t* n_dev, int shift, int bits) {
  constexpr int CH = NT * kItems;          // keys per tile
  constexpr int NW = NT / 64;
  constexpr int kPerWave = CH / NW;
  __shared__ K s_key[CH];
  __shared__ uint32_t s_val[CH];
  __shared__ uint32_t s_cnt[NW][256];       // per-wave digit counts, then per-wave digit bases
  __shared__ uint32_t s_start[256];         // start of each digit in the partitioned tile
  __shared__ uint32_t s_glob[256];          // global start of this tile's run of each digit
  const int64_t n = active_count(n_max, n_dev);
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * CH;
  if (base >= n) return;  // uniform per block; no tile waits on a later one
  for (int x = threadIdx.x; x < NW * 256; x += NT) (&s_cnt[0][0])[x] = 0;
  const int count = static_cast<int>(min(static_cast<int64_t>(CH), n - base));
  const int radix = 1 << bits;
  const uint32_t mask = static_cast<uint32_t>(radix - 1);
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
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
  const bool has = static_cast<int>(threadIdx.x) < radix;
  const bool dig = threadIdx.x < 256;   // the threads that own a digit's bookkeeping
  {
    uint32_t c[NW], t = 0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      c[ww] = dig ? s_cnt[ww][threadIdx.x] : 0u;
      t += c[ww];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan_n<NT>(t, &tot);
    if (dig) {
      s_start[threadIdx.x] = run;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) {
        s_cnt[ww][threadIdx.x] = run;
        run += c[ww];
      }
    }
    // keys of lower digits in the whole input: the exclusive scan of the digit totals
    uint32_t all;
    const uint32_t below = block_excl_scan_n<NT>(has ? totals[threadIdx.x] : 0u, &all);
    if (has) {
      uint32_t* mine = status + tile * radix + threadIdx.x;
      uint32_t excl = 0;
      if (tile == 0) {
        status_store(mine, kFlagInc | t);
      } else {
        status_store(mine, kFlagAgg | t);
        // Walk back over windows of kLookback earlier tiles, their status words read together
        // (one memory round trip per window rather than per tile): add the counts nearest
        // first until a tile that holds its inclusive count; a window that meets a tile that has
        // published nothing yet is read again from that tile.  Nothing here assumes that the
        // earlier tiles' blocks are running: after kFallbackRounds such rounds the thread counts
        // its digit in that tile's keys itself and walks on, so every wait ends.
        int64_t j = tile - 1;
        int rounds = 0;
        for (;;) {
          uint32_t v[kLookback];
#pragma unroll
          for (int k = 0; k < kLookback; ++k)
            v[k] = j - k >= 0 ? status_load(status + (j - k) * radix + threadIdx.x) : kFlagInc;
          int k = 0;
          bool done = false;
#pragma unroll
          for (int q = 0; q < kLookback; ++q) {
            if (!done && k == q) {
              if ((v[q] & ~kCountMask) == 0u) continue;   // not published yet: stop here
              excl += v[q] & kCountMask;
              done = (v[q] & kFlagInc) != 0u;
              k = q + 1;
            }
          }
          if (done) break;
          j -= k;
          if (k < kLookback) {
            if (++rounds > kFallbackRounds) {
              excl += count_digit<CH>(kin, j, shift, mask, threadIdx.x);   // tile j < tile is full
              --j;
              rounds = 0;
            } else {
              __builtin_amdgcn_s_sleep(1);
            }
          }
        }
        status_store(mine, kFlagInc | (excl + t));
      }
      s_glob[threadIdx.x] = below + excl;
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
    const int lp = r * NT + threadIdx.x;
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

namespace {
// Scratch of one sort: per-block digit counts of the histogram kernel, digit totals, then the
// look-back status words of every pass, which the histogram kernel clears.
struct RadixLayout {
  int64_t nb;        // 4096-key tiles (status words are sized for them, twice what a pass uses)
  int passes_max;    // passes of a 32-bit key
  int radix;         // 1 << digit width
  int G;             // histogram blocks
  size_t off_tot, off_status, bytes;
};

RadixLayout radix_layout(int64_t n_max, int digit_bits) {
  RadixLayout L;
  L.nb = ceil_div(n_max > 0 ? n_max : 1, kChunk);
  L.passes_max = static_cast<int>(ceil_div(32, digit_bits));
  L.radix = 1 << digit_bits;
  L.G = static_cast<int>(L.nb < kUpBlocksMax ? L.nb : kUpBlocksMax);
  const size_t part = static_cast<size_t>(L.G) * L.passes_max * 256 * 4;
  L.off_tot = align_up(part, 256);
  L.off_status = align_up(L.off_tot + static_cast<size_t>(L.passes_max) * 256 * 4, 256);
  L.bytes = align_up(L.off_status + static_cast<size_t>(L.passes_max) * L.nb * L.radix * 4, 256);
  return L;
}
}  // namespace

size_t radix_scratch_bytes(int64_t n_max, int digit_bits) {
  if (digit_bits < 4) digit_bits = 4;
  return radix_layout(n_max, digit_bits).bytes;
}

template <class K>
vbm_status radix_sort_pairs(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t n_max, const uint32_t* n_dev,
                            int end_bit, int digit_bits, void* scratch, hipStream_t s, bool* result_in_k1) {
  *result_in_k1 = false;
  if (n_max <= 0 || end_bit <= 0) return VBM_OK;
  if (digit_bits < 4 || digit_bits > 8) {
    set_error("radix digit width %d outside 4..8", digit_bits);
    return VBM_ERR_INVALID;
  }
  if (end_bit > 32 || end_bit > static_cast<int>(8 * sizeof(K))) {
    set_error("radix sort over %d key bits (at most 32)", end_bit);
    return VBM_ERR_INVALID;
  }
  const RadixLayout L = radix_layout(n_max, digit_bits);
  const int passes = static_cast<int>(ceil_div(end_bit, digit_bits));
  char* base = static_cast<char*>(scratch);
  uint32_t* part = reinterpret_cast<uint32_t*>(base);
  uint32_t* tot = reinterpret_cast<uint32_t*>(base + L.off_tot);
  uint32_t* status = reinterpret_cast<uint32_t*>(base + L.off_status);
  const int64_t pass_words = L.nb * L.radix;
  const int64_t clear_n = static_cast<int64_t>(passes) * pass_words;
  hipLaunchKernelGGL(k_radix_upsweep<K>, dim3(L.G), dim3(kUpThreads), 0, s, k0, n_max, n_dev, end_bit, digit_bits,
                     passes, part, status, clear_n);
  VBM_LAUNCH_CHECK("radix_upsweep");
  const int R = passes * 256;
  hipLaunchKernelGGL(k_radix_totals, dim3(ceil_div(R, 64)), dim3(kTopThreads), 0, s, part, L.G, R, tot);
  VBM_LAUNCH_CHECK("radix_totals");
  K* kin = k0;
  uint32_t* vin = v0;
  K* kout = k1;
  uint32_t* vout = v1;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * digit_bits;
    const int bits = (end_bit - shift) < digit_bits ? (end_bit - shift) : digit_bits;
    hipLaunchKernelGGL((k_radix_onesweep<kSweepThreads, K>), dim3(ceil_div(n_max, kSweepThreads * kItems)),
                       dim3(kSweepThreads), 0, s, kin, vin, kout, vout, tot + p * 256, status + p * pass_words, n_max,
                       n_dev, shift, bits);
    VBM_LAUNCH_CHECK("radix_onesweep");
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

}  // namespace vbm
