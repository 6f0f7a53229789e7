// vbm_build_gaussians: joint-norm global top-K (Supp. A, joint magnitude) and analytical Gaussian
// construction by bank lookup (Sec. 4.3: eq. per_location_weight, eq. wavelet_gaussian_kernel,
// eq. translation_operator).
//
// Selection is exact and deterministic: a float32 key per location, four 8-bit radix-select
// passes (most significant digit first) find the K-th largest key t, then one stable compaction
// keeps every key > t plus the lowest-index keys == t until K are kept, in ascending index order.
#include <hip/hip_runtime.h>

#include "block_scan.h"
#include "common.h"

namespace vbm {
namespace {

constexpr int kT = 256;
constexpr int kPerThread = 16;
constexpr int kChunk = kT * kPerThread;

struct SelectState {
  uint32_t prefix;    // key bits fixed so far
  uint32_t k_rem;     // elements still to take from the bucket matching `prefix`
  uint32_t count_gt;  // elements strictly above the bucket
  uint32_t pad;
};

#pragma clang fp contract(off)
__global__ __launch_bounds__(kT) void k_joint_keys(const float* __restrict__ coeffs, int64_t M,
                                                  uint32_t* __restrict__ keys) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x; i < M;
       i += static_cast<int64_t>(gridDim.x) * kT) {
    const float r = coeffs[i], g = coeffs[M + i], b = coeffs[2 * M + i], a = coeffs[3 * M + i];
    const float s = ((r * r + g * g) + b * b) + a * a;
    keys[i] = __float_as_uint(sqrt_rn_f32(s));
  }
}

__global__ void k_select_init(SelectState* st, uint32_t K, uint32_t* hist) {
  if (threadIdx.x == 0) {
    st->prefix = 0;
    st->k_rem = K;
    st->count_gt = 0;
  }
  hist[threadIdx.x] = 0;
}

// Histogram of digit `shift` over keys whose higher digits equal the current prefix.
__global__ __launch_bounds__(kT) void k_select_hist(const uint32_t* __restrict__ keys, int64_t M, int shift,
                                                   const SelectState* __restrict__ st, uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_hist[256];
  s_hist[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t hi_mask = shift >= 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
  const uint32_t prefix = st->prefix & hi_mask;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x; i < M;
       i += static_cast<int64_t>(gridDim.x) * kT) {
    const uint32_t k = keys[i];
    if ((k & hi_mask) == prefix) atomicAdd(&s_hist[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  const uint32_t c = s_hist[threadIdx.x];
  if (c) atomicAdd(&hist[threadIdx.x], c);
}

// Picks the digit holding the k_rem-th largest key (one block of 256 threads); clears the histogram.
__global__ __launch_bounds__(kT) void k_select_pick(SelectState* st, uint32_t* hist, int shift) {
  __shared__ uint32_t s_h[256];
  const int d = threadIdx.x;
  s_h[d] = hist[d];
  __syncthreads();
  // count strictly above digit d (digits d+1..255)
  uint32_t above = 0;
  for (int e = d + 1; e < 256; ++e) above += s_h[e];
  const uint32_t k = st->k_rem;
  const uint32_t here = s_h[d];
  __syncthreads();
  if (above < k && k <= above + here) {
    st->prefix |= static_cast<uint32_t>(d) << shift;
    st->count_gt += above;
    st->k_rem = k - above;
  }
  hist[d] = 0;
}

__device__ __forceinline__ uint64_t select_flags(uint32_t key, uint32_t thr) {
  return (key > thr ? 1ull : 0ull) | (key == thr ? (1ull << 32) : 0ull);
}

__global__ __launch_bounds__(kT) void k_compact_count(const uint32_t* __restrict__ keys, int64_t M,
                                                     const SelectState* __restrict__ st, uint64_t* __restrict__ sums) {
  const uint32_t thr = st->prefix;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kChunk;
  uint64_t acc = 0;
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t i = base + r * kT + threadIdx.x;
    if (i < M) acc += select_flags(keys[i], thr);
  }
  uint64_t tot;
  block_excl_scan(acc, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kT) void k_compact_top(uint64_t* sums, int64_t nb) {
  uint64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kChunk) {
    uint64_t it[kPerThread];
    uint64_t acc = 0;
    for (int r = 0; r < kPerThread; ++r) {
      const int64_t i = base + static_cast<int64_t>(threadIdx.x) * kPerThread + r;
      it[r] = i < nb ? sums[i] : 0ull;
      acc += it[r];
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan(acc, &tot) + carry;
    for (int r = 0; r < kPerThread; ++r) {
      const int64_t i = base + static_cast<int64_t>(threadIdx.x) * kPerThread + r;
      if (i < nb) sums[i] = ex;
      ex += it[r];
    }
    carry += tot;
  }
}

__global__ __launch_bounds__(kT) void k_compact_write(const uint32_t* __restrict__ keys, int64_t M,
                                                     const SelectState* __restrict__ st,
                                                     const uint64_t* __restrict__ offs, uint32_t* __restrict__ kept) {
  const uint32_t thr = st->prefix;
  const uint32_t need = st->k_rem;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kChunk;
  uint64_t f[kPerThread];
  uint64_t acc = 0;
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t i = base + static_cast<int64_t>(threadIdx.x) * kPerThread + r;
    f[r] = i < M ? select_flags(keys[i], thr) : 0ull;
    acc += f[r];
  }
  uint64_t tot;
  uint64_t ex = block_excl_scan(acc, &tot) + offs[blockIdx.x];
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t i = base + static_cast<int64_t>(threadIdx.x) * kPerThread + r;
    const uint32_t gt_before = static_cast<uint32_t>(ex);
    const uint32_t eq_before = static_cast<uint32_t>(ex >> 32);
    const bool keep = (f[r] & 1ull) || ((f[r] >> 32) && eq_before < need);
    if (keep) kept[gt_before + (eq_before < need ? eq_before : need)] = static_cast<uint32_t>(i);
    ex += f[r];
  }
}

struct BuildParams {
  int G, J;
  float h;
  float delta;
  float op_min, op_max;
  int s_mode;
  int unit_weight;
  int64_t M;
};

template <class I>
__global__ __launch_bounds__(kT) void k_build(const float* __restrict__ coeffs, const I* __restrict__ kept,
                                             int64_t K, const float* __restrict__ bank, BuildParams p,
                                             vbm_gaussians out, int64_t* __restrict__ kept_out) {
  const int64_t n = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
  if (n >= K) return;
  const int64_t idx = static_cast<int64_t>(kept[n]);
  if (idx < 0 || idx >= p.M) return;   // a caller-given index outside the grid builds nothing
  // decode the packed index: [LLL_J][level J: o=1..7]...[level 1: o=1..7]
  int j = p.J, b = 0;
  int64_t off = idx;
  int64_t nJ = p.G >> p.J;
  int64_t sz = nJ * nJ * nJ;
  int o = 0;
  int64_t side = nJ;
  if (off < sz) {
    o = 0;
  } else {
    off -= sz;
    for (j = p.J; j >= 1; --j) {
      side = p.G >> j;
      const int64_t s3 = side * side * side;
      if (off < 7 * s3) {
        o = 1 + static_cast<int>(off / s3);
        off -= static_cast<int64_t>(o - 1) * s3;
        break;
      }
      off -= 7 * s3;
    }
  }
  b = (o == 0) ? 0 : 1 + 7 * (p.J - j) + (o - 1);
  const int kx = static_cast<int>(off % side);
  const int ky = static_cast<int>((off / side) % side);
  const int kz = static_cast<int>(off / (side * side));
  const float* e = bank + static_cast<int64_t>(b) * VBM_BANK_FLOATS;
  const float w = p.unit_weight ? 1.0f : e[0];
  const float step = static_cast<float>(1 << j);
  out.means[n] = -1.0f + p.h * (e[1] + step * kx + p.delta);
  out.means[out.stride + n] = -1.0f + p.h * (e[2] + step * ky + p.delta);
  out.means[2 * out.stride + n] = -1.0f + p.h * (e[3] + step * kz + p.delta);
  for (int c = 0; c < 3; ++c) out.scales[c * out.stride + n] = p.h * e[4 + c];
  for (int c = 0; c < 4; ++c) out.quats[c * out.stride + n] = e[7 + c];
  const float s = p.s_mode == 0 ? exp2f(-1.5f * static_cast<float>(j)) : 1.0f;
  for (int c = 0; c < 3; ++c) {
    const float amp = s * fabsf(coeffs[c * p.M + idx]) * w;
    out.rgb[c * out.stride + n] = fminf(fmaxf(amp, 0.0f), 1.0f);
  }
  const float amp_a = s * fabsf(coeffs[3 * p.M + idx]) * w;
  out.opacity[n] = fminf(fmaxf(amp_a, p.op_min), p.op_max);
  if (kept_out) kept_out[n] = idx;
}

// Ablation without the transition bank: sigma_iso = mean over the n built Gaussians of the mean of
// their three scales (float64, fixed order: thread-strided sums, then a fixed tree), then every
// Gaussian gets scales sigma_iso and the identity rotation.  One block.
__global__ __launch_bounds__(1024) void k_isotropize(vbm_gaussians out, int64_t n) {
  __shared__ double s_sum[1024];
  const int64_t S = out.stride;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024)
    acc += (static_cast<double>(out.scales[i]) + static_cast<double>(out.scales[S + i]) +
            static_cast<double>(out.scales[2 * S + i])) / 3.0;
  s_sum[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 512; st >= 1; st >>= 1) {
    if (static_cast<int>(threadIdx.x) < st) s_sum[threadIdx.x] += s_sum[threadIdx.x + st];
    __syncthreads();
  }
  const float sigma = static_cast<float>(s_sum[0] / static_cast<double>(n));
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    out.scales[i] = out.scales[S + i] = out.scales[2 * S + i] = sigma;
    out.quats[i] = 1.0f;
    out.quats[S + i] = out.quats[2 * S + i] = out.quats[3 * S + i] = 0.0f;
  }
}

int grid_cap(int64_t n, int cap) {
  int64_t b = ceil_div(n, kT);
  return static_cast<int>(b < cap ? b : cap);
}

}  // namespace
}  // namespace vbm

using namespace vbm;

extern "C" size_t vbm_build_workspace_size(int32_t G, int32_t J) {
  (void)J;
  if (G <= 0) return 0;
  const int64_t M = static_cast<int64_t>(G) * G * G;
  const int64_t nb = ceil_div(M, kChunk);
  size_t s = 0;
  s += align_up(M * 4, 256);           // keys
  s += align_up(M * 4, 256);           // kept indices (capacity M)
  s += align_up(nb * 8, 256);          // block sums
  s += align_up(256 * 4, 256);         // histogram
  s += align_up(sizeof(SelectState), 256);
  return s;
}

extern "C" vbm_status vbm_build_gaussians(const float* coeffs, int32_t G, int32_t J, const float* bank_dev, int64_t K,
                                          const vbm_build_opts* opts, vbm_gaussians out, int64_t* kept_index, void* ws,
                                          size_t ws_bytes, void* stream) {
  if (!coeffs || !bank_dev || !opts || !ws || !out.means || !out.scales || !out.quats || !out.opacity || !out.rgb) {
    set_error("vbm_build_gaussians: null pointer");
    return VBM_ERR_INVALID;
  }
  if (G < 2 || G > 1024 || J < 1 || J > 10 || (G % (1 << J)) != 0 || (G >> J) < 2) {
    set_error("vbm_build_gaussians: bad G=%d J=%d", G, J);
    return VBM_ERR_INVALID;
  }
  const int64_t M = static_cast<int64_t>(G) * G * G;
  if (K < 1 || K > M) {
    set_error("vbm_build_gaussians: K=%lld outside 1..G^3", static_cast<long long>(K));
    return VBM_ERR_INVALID;
  }
  if (out.stride < K) {
    set_error("vbm_build_gaussians: output stride %lld < K", static_cast<long long>(out.stride));
    return VBM_ERR_INVALID;
  }
  if (opts->s_mode != 0 && opts->s_mode != 1) {
    set_error("vbm_build_gaussians: s_mode must be 0 (paper) or 1 (none)");
    return VBM_ERR_INVALID;
  }
  if (!(opts->opacity_min >= 0.0f && opts->opacity_min <= opts->opacity_max && opts->opacity_max <= 1.0f)) {
    set_error("vbm_build_gaussians: need 0 <= opacity_min <= opacity_max <= 1");
    return VBM_ERR_INVALID;
  }
  if ((opts->isotropic != 0 && opts->isotropic != 1) || (opts->unit_weight != 0 && opts->unit_weight != 1)) {
    set_error("vbm_build_gaussians: isotropic and unit_weight must be 0 or 1");
    return VBM_ERR_INVALID;
  }
  if (ws_bytes < vbm_build_workspace_size(G, J)) {
    set_error("vbm_build_gaussians: workspace %zu < %zu", ws_bytes, vbm_build_workspace_size(G, J));
    return VBM_ERR_WORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws);
  const int64_t nb = ceil_div(M, kChunk);
  uint32_t* keys = c.take<uint32_t>(M);
  uint32_t* kept = c.take<uint32_t>(M);
  uint64_t* sums = c.take<uint64_t>(nb);
  uint32_t* hist = c.take<uint32_t>(256);
  SelectState* st = c.take<SelectState>(1);

  hipLaunchKernelGGL(k_joint_keys, dim3(grid_cap(M, 16384)), dim3(kT), 0, s, coeffs, M, keys);
  VBM_LAUNCH_CHECK("joint_keys");
  hipLaunchKernelGGL(k_select_init, dim3(1), dim3(256), 0, s, st, static_cast<uint32_t>(K), hist);
  VBM_LAUNCH_CHECK("select_init");
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(k_select_hist, dim3(grid_cap(M, 4096)), dim3(kT), 0, s, keys, M, shift, st, hist);
    VBM_LAUNCH_CHECK("select_hist");
    hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(256), 0, s, st, hist, shift);
    VBM_LAUNCH_CHECK("select_pick");
  }
  hipLaunchKernelGGL(k_compact_count, dim3(nb), dim3(kT), 0, s, keys, M, st, sums);
  VBM_LAUNCH_CHECK("compact_count");
  hipLaunchKernelGGL(k_compact_top, dim3(1), dim3(kT), 0, s, sums, nb);
  VBM_LAUNCH_CHECK("compact_top");
  hipLaunchKernelGGL(k_compact_write, dim3(nb), dim3(kT), 0, s, keys, M, st, sums, kept);
  VBM_LAUNCH_CHECK("compact_write");

  BuildParams p;
  p.G = G;
  p.J = J;
  p.h = 2.0f / static_cast<float>(G);
  p.delta = opts->delta;
  p.op_min = opts->opacity_min;
  p.op_max = opts->opacity_max;
  p.s_mode = opts->s_mode;
  p.unit_weight = opts->unit_weight;
  p.M = M;
  hipLaunchKernelGGL(k_build<uint32_t>, dim3(ceil_div(K, kT)), dim3(kT), 0, s, coeffs, kept, K, bank_dev, p, out,
                     kept_index);
  VBM_LAUNCH_CHECK("build");
  if (opts->isotropic) {
    hipLaunchKernelGGL(k_isotropize, dim3(1), dim3(1024), 0, s, out, K);
    VBM_LAUNCH_CHECK("isotropize");
  }
  return VBM_OK;
}

extern "C" vbm_status vbm_construct_gaussians(const float* coeffs, int32_t G, int32_t J, const float* bank_dev,
                                              const int64_t* kept_index, int64_t n, const vbm_build_opts* opts,
                                              vbm_gaussians out, void* stream) {
  if (!coeffs || !bank_dev || !opts || (n > 0 && !kept_index) || !out.means || !out.scales || !out.quats ||
      !out.opacity || !out.rgb) {
    set_error("vbm_construct_gaussians: null pointer");
    return VBM_ERR_INVALID;
  }
  if (G < 2 || G > 1024 || J < 1 || J > 10 || (G % (1 << J)) != 0 || (G >> J) < 2) {
    set_error("vbm_construct_gaussians: bad G=%d J=%d", G, J);
    return VBM_ERR_INVALID;
  }
  if (n < 0 || out.stride < n) {
    set_error("vbm_construct_gaussians: need 0 <= n <= out.stride");
    return VBM_ERR_INVALID;
  }
  if ((opts->s_mode != 0 && opts->s_mode != 1) ||
      !(opts->opacity_min >= 0.0f && opts->opacity_min <= opts->opacity_max && opts->opacity_max <= 1.0f) ||
      (opts->isotropic != 0 && opts->isotropic != 1) || (opts->unit_weight != 0 && opts->unit_weight != 1)) {
    set_error("vbm_construct_gaussians: bad opts");
    return VBM_ERR_INVALID;
  }
  if (n == 0) return VBM_OK;
  BuildParams p;
  p.G = G;
  p.J = J;
  p.h = 2.0f / static_cast<float>(G);
  p.delta = opts->delta;
  p.op_min = opts->opacity_min;
  p.op_max = opts->opacity_max;
  p.s_mode = opts->s_mode;
  p.unit_weight = opts->unit_weight;
  p.M = static_cast<int64_t>(G) * G * G;
  hipLaunchKernelGGL(k_build<int64_t>, dim3(ceil_div(n, kT)), dim3(kT), 0, static_cast<hipStream_t>(stream), coeffs,
                     kept_index, n, bank_dev, p, out, static_cast<int64_t*>(nullptr));
  VBM_LAUNCH_CHECK("construct");
  if (opts->isotropic) {
    hipLaunchKernelGGL(k_isotropize, dim3(1), dim3(1024), 0, static_cast<hipStream_t>(stream), out, n);
    VBM_LAUNCH_CHECK("isotropize");
  }
  return VBM_OK;
}
