// vbm_dwt3d: transfer function + periodised separable J-level 3D DWT (Sec. 3; Sec. 4.3,
// eq. mul_wavelet_coff).
//
// Each level runs three separable passes (x, y, z) over the current n^3 approximation of the four
// RGBA channels; every thread produces one low/high output pair along the pass axis, with threads
// laid out x-fastest so loads and stores coalesce.  The level-1 x pass reads the scalar field and
// applies the transfer function at each tap (RGBA is never materialised).  The z pass writes the
// seven detail octants straight into the packed subband layout and LLL into the next level's input.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstring>

#include "common.h"
#include "filters.h"
#include "tf.h"

namespace vbm {
namespace {

struct DevFilters {
  float lo[10];
  float hi[10];
  int lo_first, lo_len, hi_first, hi_len;
};

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// x pass.  in: scalar [n][n][n] (with_tf) or rgba [4][n^3]; out: rgba [4][n^3], x split low|high.
template <bool kWithTF>
__global__ __launch_bounds__(256) void k_dwt_x(const float* __restrict__ in, float* __restrict__ out, int n,
                                               DevFilters f, DevTF tf) {
  const int h = n >> 1;
  const int64_t total = static_cast<int64_t>(h) * n * n;
  const int64_t cs = static_cast<int64_t>(n) * n * n;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int k = static_cast<int>(t % h);
    const int64_t row = t / h;  // z * n + y
    const float* src = in + row * n;
    float lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
    for (int i = 0; i < f.lo_len; ++i) {
      const int x = wrap(2 * k + f.lo_first + i, n);
      float v[4];
      if (kWithTF) {
        float4 c = tf_eval(tf, src[x]);
        v[0] = c.x; v[1] = c.y; v[2] = c.z; v[3] = c.w;
      } else {
        for (int c = 0; c < 4; ++c) v[c] = src[c * cs + x];
      }
      for (int c = 0; c < 4; ++c) lo[c] += f.lo[i] * v[c];
    }
    for (int i = 0; i < f.hi_len; ++i) {
      const int x = wrap(2 * k + f.hi_first + i, n);
      float v[4];
      if (kWithTF) {
        float4 c = tf_eval(tf, src[x]);
        v[0] = c.x; v[1] = c.y; v[2] = c.z; v[3] = c.w;
      } else {
        for (int c = 0; c < 4; ++c) v[c] = src[c * cs + x];
      }
      for (int c = 0; c < 4; ++c) hi[c] += f.hi[i] * v[c];
    }
    for (int c = 0; c < 4; ++c) {
      out[c * cs + row * n + k] = lo[c];
      out[c * cs + row * n + h + k] = hi[c];
    }
  }
}

// y pass: in/out rgba [4][n^3], y split low|high.
__global__ __launch_bounds__(256) void k_dwt_y(const float* __restrict__ in, float* __restrict__ out, int n,
                                               DevFilters f) {
  const int h = n >> 1;
  const int64_t total = static_cast<int64_t>(n) * h * n;
  const int64_t cs = static_cast<int64_t>(n) * n * n;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int x = static_cast<int>(t % n);
    const int k = static_cast<int>((t / n) % h);
    const int z = static_cast<int>(t / (static_cast<int64_t>(n) * h));
    const int64_t plane = static_cast<int64_t>(z) * n * n;
    float lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
    for (int i = 0; i < f.lo_len; ++i) {
      const int y = wrap(2 * k + f.lo_first + i, n);
      for (int c = 0; c < 4; ++c) lo[c] += f.lo[i] * in[c * cs + plane + static_cast<int64_t>(y) * n + x];
    }
    for (int i = 0; i < f.hi_len; ++i) {
      const int y = wrap(2 * k + f.hi_first + i, n);
      for (int c = 0; c < 4; ++c) hi[c] += f.hi[i] * in[c * cs + plane + static_cast<int64_t>(y) * n + x];
    }
    for (int c = 0; c < 4; ++c) {
      out[c * cs + plane + static_cast<int64_t>(k) * n + x] = lo[c];
      out[c * cs + plane + static_cast<int64_t>(h + k) * n + x] = hi[c];
    }
  }
}

// z pass: writes the 7 detail octants of level j into the packed output and LLL to lll_out
// (per-channel stride h^3; for the last level lll_out is the packed LLL_J block itself).
__global__ __launch_bounds__(256) void k_dwt_z(const float* __restrict__ in, float* __restrict__ coeffs,
                                               float* __restrict__ lll_out, int64_t lll_cstride, int n,
                                               int64_t G3, int64_t level_base, DevFilters f) {
  const int h = n >> 1;
  const int64_t total = static_cast<int64_t>(h) * n * n;
  const int64_t cs = static_cast<int64_t>(n) * n * n;
  const int64_t h3 = static_cast<int64_t>(h) * h * h;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int x = static_cast<int>(t % n);
    const int y = static_cast<int>((t / n) % n);
    const int k = static_cast<int>(t / (static_cast<int64_t>(n) * n));
    const int64_t col = static_cast<int64_t>(y) * n + x;
    float lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
    for (int i = 0; i < f.lo_len; ++i) {
      const int z = wrap(2 * k + f.lo_first + i, n);
      for (int c = 0; c < 4; ++c) lo[c] += f.lo[i] * in[c * cs + static_cast<int64_t>(z) * n * n + col];
    }
    for (int i = 0; i < f.hi_len; ++i) {
      const int z = wrap(2 * k + f.hi_first + i, n);
      for (int c = 0; c < 4; ++c) hi[c] += f.hi[i] * in[c * cs + static_cast<int64_t>(z) * n * n + col];
    }
    const int ox = x >= h ? 1 : 0, oy = y >= h ? 1 : 0;
    const int xx = x - ox * h, yy = y - oy * h;
    const int64_t pos = (static_cast<int64_t>(k) * h + yy) * h + xx;
    const int o_lo = ox | (oy << 1);
    const int o_hi = o_lo | 4;
    for (int c = 0; c < 4; ++c) {
      if (o_lo == 0) {
        lll_out[c * lll_cstride + pos] = lo[c];
      } else {
        coeffs[c * G3 + level_base + (o_lo - 1) * h3 + pos] = lo[c];
      }
      coeffs[c * G3 + level_base + (o_hi - 1) * h3 + pos] = hi[c];
    }
  }
}

DevFilters to_dev(const Filter1D& lo, const Filter1D& hi) {
  DevFilters d;
  std::memset(&d, 0, sizeof(d));
  d.lo_len = static_cast<int>(lo.taps.size());
  d.hi_len = static_cast<int>(hi.taps.size());
  d.lo_first = lo.first;
  d.hi_first = hi.first;
  for (int i = 0; i < d.lo_len; ++i) d.lo[i] = static_cast<float>(lo.taps[i]);
  for (int i = 0; i < d.hi_len; ++i) d.hi[i] = static_cast<float>(hi.taps[i]);
  return d;
}

int grid_for(int64_t total) {
  int64_t b = ceil_div(total, 256);
  return static_cast<int>(b < 65536 ? b : 65536);
}

}  // namespace
}  // namespace vbm

using namespace vbm;

extern "C" size_t vbm_dwt3d_workspace_size(int32_t G, int32_t J) {
  (void)J;
  if (G <= 0) return 0;
  const size_t plane = static_cast<size_t>(G) * G * G;
  // two ping-pong buffers of 4 channels at level-1 size; later levels fit inside them
  return 2 * align_up(4 * plane * sizeof(float), 256);
}

extern "C" vbm_status vbm_dwt3d(const float* vol, int32_t G, int32_t J, int32_t wavelet, const vbm_tf* tf,
                                float* coeffs, void* ws, size_t ws_bytes, void* stream) {
  if (!vol || !coeffs || !ws) {
    set_error("vbm_dwt3d: null pointer");
    return VBM_ERR_INVALID;
  }
  if (G < 2 || G > 1024 || J < 1 || J > 10 || (G % (1 << J)) != 0 || (G >> J) < 2) {
    set_error("vbm_dwt3d: need G %% 2^J == 0, G/2^J >= 2, 1 <= J <= 10, G <= 1024 (G=%d J=%d)", G, J);
    return VBM_ERR_INVALID;
  }
  if (wavelet != VBM_WAVELET_HAAR && wavelet != VBM_WAVELET_BIOR44) {
    set_error("vbm_dwt3d: unknown wavelet %d", wavelet);
    return VBM_ERR_UNSUPPORTED;
  }
  DevTF dtf;
  std::memset(&dtf, 0, sizeof(dtf));
  if (tf) {
    if (tf->n_points < 2 || tf->n_points > VBM_TF_MAX_POINTS) {
      set_error("vbm_dwt3d: transfer function needs 2..%d points", VBM_TF_MAX_POINTS);
      return VBM_ERR_UNSUPPORTED;
    }
    for (int i = 1; i < tf->n_points; ++i)
      if (!(tf->x[i] >= tf->x[i - 1])) {
        set_error("vbm_dwt3d: transfer-function control points must ascend");
        return VBM_ERR_INVALID;
      }
    dtf.n = tf->n_points;
    for (int i = 0; i < tf->n_points; ++i) {
      dtf.x[i] = tf->x[i];
      for (int c = 0; c < 4; ++c) dtf.rgba[i][c] = tf->rgba[i][c];
    }
  }
  if (ws_bytes < vbm_dwt3d_workspace_size(G, J)) {
    set_error("vbm_dwt3d: workspace %zu < %zu bytes", ws_bytes, vbm_dwt3d_workspace_size(G, J));
    return VBM_ERR_WORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const FilterBankD fb = make_filter_bank(wavelet);
  const DevFilters f = to_dev(fb.lo_a, fb.hi_a);
  const int64_t G3 = static_cast<int64_t>(G) * G * G;
  float* bufA = static_cast<float*>(ws);
  float* bufB = reinterpret_cast<float*>(static_cast<char*>(ws) + align_up(4 * G3 * sizeof(float), 256));
  // Buffer roles per level: x pass cur -> p, y pass p -> q, z pass q -> details + LLL into p;
  // the next level reads p, so the roles swap (each pass only overwrites data already consumed).
  float* p = bufA;
  float* q = bufB;
  const float* cur = vol;
  bool cur_is_rgba = tf == nullptr;
  for (int j = 1; j <= J; ++j) {
    const int n = G >> (j - 1);
    const int h = n >> 1;
    // packed offset of block (j, 1): n_J^3 + sum_{j' > j} 7 n_{j'}^3
    int64_t level_base = static_cast<int64_t>(G >> J) * (G >> J) * (G >> J);
    for (int jj = J; jj > j; --jj) level_base += 7LL * (G >> jj) * (G >> jj) * (G >> jj);
    const int64_t hn2 = static_cast<int64_t>(h) * n * n;
    if (cur_is_rgba) {
      hipLaunchKernelGGL(k_dwt_x<false>, dim3(grid_for(hn2)), dim3(256), 0, s, cur, p, n, f, dtf);
    } else {
      hipLaunchKernelGGL(k_dwt_x<true>, dim3(grid_for(hn2)), dim3(256), 0, s, cur, p, n, f, dtf);
    }
    VBM_LAUNCH_CHECK("dwt_x");
    hipLaunchKernelGGL(k_dwt_y, dim3(grid_for(hn2)), dim3(256), 0, s, p, q, n, f);
    VBM_LAUNCH_CHECK("dwt_y");
    const int64_t h3 = static_cast<int64_t>(h) * h * h;
    float* lll = (j == J) ? coeffs : p;
    const int64_t lll_cs = (j == J) ? G3 : h3;
    hipLaunchKernelGGL(k_dwt_z, dim3(grid_for(hn2)), dim3(256), 0, s, q, coeffs, lll, lll_cs, n, G3, level_base,
                       f);
    VBM_LAUNCH_CHECK("dwt_z");
    cur = p;
    cur_is_rgba = true;
    float* t = p;
    p = q;
    q = t;
  }
  return VBM_OK;
}
