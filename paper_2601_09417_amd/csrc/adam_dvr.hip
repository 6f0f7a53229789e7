// vbm_adam_init / vbm_adam_step (Adam on the raw parameters, Sec. 5 Implementation Details) and vbm_dvr_render
// (ray-marched supervision images, Sec. 4.4).
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "tf.h"

namespace vbm {
namespace {

struct AdamParams {
  float lr[5];
  float beta1, beta2, eps;
  float bc1, bc2;  // 1 - beta^t when the step count is a host value
};

// Advances the device step counter; k_adam then reads it (keeps a captured graph replayable).
__global__ void k_step_inc(int32_t* step) {
  if (threadIdx.x == 0) step[0] += 1;
}

// One thread per Gaussian; rows 0-2 means, 3-5 log scales, 6-9 quats, 10 logit opacity, 11-13 rgb.
__global__ __launch_bounds__(256) void k_adam(int64_t n, int64_t stride, float* __restrict__ raw,
                                              float* __restrict__ m, float* __restrict__ v, vbm_gaussians_c g,
                                              vbm_gaussians act, AdamParams p, const int32_t* __restrict__ step_dev) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  if (step_dev) {
    const float t = static_cast<float>(step_dev[0]);
    p.bc1 = 1.0f - powf(p.beta1, t);
    p.bc2 = 1.0f - powf(p.beta2, t);
  }
  const int64_t GS = g.stride, AS = act.stride;
#pragma unroll
  for (int r = 0; r < 14; ++r) {
    const int grp = r < 3 ? 0 : (r < 6 ? 1 : (r < 10 ? 2 : (r == 10 ? 3 : 4)));
    const int64_t o = r * stride + i;
    float x = raw[o];
    float gr;
    if (grp == 0) gr = g.means[r * GS + i];
    else if (grp == 1) gr = g.scales[(r - 3) * GS + i] * expf(x);
    else if (grp == 2) gr = g.quats[(r - 6) * GS + i];
    else if (grp == 3) {
      const float sg = 1.0f / (1.0f + expf(-x));
      gr = g.opacity[i] * sg * (1.0f - sg);
    } else gr = g.rgb[(r - 11) * GS + i];
    const float mm = p.beta1 * m[o] + (1.0f - p.beta1) * gr;
    const float vv = p.beta2 * v[o] + (1.0f - p.beta2) * gr * gr;
    m[o] = mm;
    v[o] = vv;
    const float mhat = mm / p.bc1;
    const float vhat = vv / p.bc2;
    x -= p.lr[grp] * mhat / (sqrtf(vhat) + p.eps);
    raw[o] = x;
    if (grp == 0) act.means[r * AS + i] = x;
    else if (grp == 1) act.scales[(r - 3) * AS + i] = expf(x);
    else if (grp == 2) act.quats[(r - 6) * AS + i] = x;
    else if (grp == 3) act.opacity[i] = 1.0f / (1.0f + expf(-x));
    else act.rgb[(r - 11) * AS + i] = x;
  }
}

// One thread per Gaussian: raw rows from the activated ones (log of the scales, logit of the
// opacity, the other rows copied) and zeroed moments.
__global__ __launch_bounds__(256) void k_adam_init(int64_t n, int64_t stride, vbm_gaussians_c act,
                                                   float* __restrict__ raw, float* __restrict__ m,
                                                   float* __restrict__ v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t AS = act.stride;
#pragma unroll
  for (int r = 0; r < 14; ++r) {
    float x;
    if (r < 3) x = act.means[r * AS + i];
    else if (r < 6) x = logf(act.scales[(r - 3) * AS + i]);
    else if (r < 10) x = act.quats[(r - 6) * AS + i];
    else if (r == 10) {
      const float o = act.opacity[i];
      x = logf(o / (1.0f - o));
    } else x = act.rgb[(r - 11) * AS + i];
    const int64_t o = r * stride + i;
    raw[o] = x;
    m[o] = 0.0f;
    v[o] = 0.0f;
  }
}

// Transfer function in float64 at a float64 scalar (the control points are float32 values).
__device__ __forceinline__ void tf_eval_f64(const DevTF& tf, double f, double c[4]) {
  const int n = tf.n;
  int j0, j1;
  double t;
  if (!(f > static_cast<double>(tf.x[0]))) {
    j0 = j1 = 0;
    t = 0.0;
  } else if (f >= static_cast<double>(tf.x[n - 1])) {
    j0 = j1 = n - 1;
    t = 0.0;
  } else {
    int j = 0;
    for (int i = 1; i < n - 1; ++i)
      if (static_cast<double>(tf.x[i]) <= f) j = i;
    const double x0 = tf.x[j], x1 = tf.x[j + 1];
    j0 = j;
    j1 = j + 1;
    t = x1 > x0 ? (f - x0) / (x1 - x0) : 1.0;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double a = tf.rgba[j0][k], b = tf.rgba[j1][k];
    c[k] = a + t * (b - a);
  }
}

// One thread per pixel of one view.  The supervision images are made once per scene, off the
// fine-tuning loop, and every image the renderer is fitted to comes from here; so the ray, the
// sample positions, the trilinear weights, the transfer function and the compositing run in
// float64 (on CDNA the float64 vector rate equals the unpacked float32 rate), and only the volume
// and the control points are float32 values.  Over the thousand-odd samples of a 512^3 ray,
// float32 positions and products would drift by more than 1e-5 of the image.
__global__ __launch_bounds__(256) void k_dvr(const float* __restrict__ vol, int G, DevTF tf, vbm_view view,
                                             double step_vox, float* __restrict__ image) {
  const int64_t HW = static_cast<int64_t>(view.width) * view.height;
  const int64_t pix = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (pix >= HW) return;
  const int px = static_cast<int>(pix % view.width), py = static_cast<int>(pix / view.width);
  double V[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) V[i] = view.viewmat[i];
  // eye = -R^T t, direction = R^T d_cam (normalised)
  const double ex = -(V[0] * V[3] + V[4] * V[7] + V[8] * V[11]);
  const double ey = -(V[1] * V[3] + V[5] * V[7] + V[9] * V[11]);
  const double ez = -(V[2] * V[3] + V[6] * V[7] + V[10] * V[11]);
  const double u = (static_cast<double>(px) + 0.5 - static_cast<double>(view.cx)) / static_cast<double>(view.fx);
  const double w = (static_cast<double>(py) + 0.5 - static_cast<double>(view.cy)) / static_cast<double>(view.fy);
  double dx = V[0] * u + V[4] * w + V[8];
  double dy = V[1] * u + V[5] * w + V[9];
  double dz = V[2] * u + V[6] * w + V[10];
  const double nrm = sqrt(dx * dx + dy * dy + dz * dz);
  dx /= nrm;
  dy /= nrm;
  dz /= nrm;
  const double e[3] = {ex, ey, ez}, d[3] = {dx, dy, dz};
  double tn = -INFINITY, tf_ = INFINITY;
  for (int a = 0; a < 3; ++a) {
    const double inv = 1.0 / d[a];
    const double t1 = (-1.0 - e[a]) * inv, t2 = (1.0 - e[a]) * inv;
    tn = fmax(tn, fmin(t1, t2));
    tf_ = fmin(tf_, fmax(t1, t2));
  }
  tn = fmax(tn, 0.0);
  double T = 1.0, cr = 0.0, cg = 0.0, cb = 0.0;
  if (tf_ > tn) {
    const double h = 2.0 / static_cast<double>(G);
    const double dt = step_vox * h;
    const int64_t nsteps = static_cast<int64_t>(floor((tf_ - tn) / dt)) + 1;
    const int64_t G2 = static_cast<int64_t>(G) * G;
    const bool half_step = step_vox == 0.5;
    for (int64_t k = 0; k < nsteps && T >= 1e-4; ++k) {
      const double t = tn + static_cast<double>(k) * dt;
      const double p[3] = {ex + t * dx, ey + t * dy, ez + t * dz};
      int i0[3];
      double f[3];
      for (int a = 0; a < 3; ++a) {
        double q = (p[a] + 1.0) / h - 0.5;
        q = fmin(fmax(q, 0.0), static_cast<double>(G - 1));
        int i = static_cast<int>(floor(q));
        if (i > G - 2) i = G - 2;
        i0[a] = i;
        f[a] = q - static_cast<double>(i);
      }
      const float* b = vol + i0[2] * G2 + static_cast<int64_t>(i0[1]) * G + i0[0];
      const double c000 = b[0], c001 = b[1], c010 = b[G], c011 = b[G + 1];
      const double c100 = b[G2], c101 = b[G2 + 1], c110 = b[G2 + G], c111 = b[G2 + G + 1];
      const double c00 = c000 + f[0] * (c001 - c000), c01 = c010 + f[0] * (c011 - c010);
      const double c10 = c100 + f[0] * (c101 - c100), c11 = c110 + f[0] * (c111 - c110);
      const double c0 = c00 + f[1] * (c01 - c00), c1 = c10 + f[1] * (c11 - c10);
      const double val = c0 + f[2] * (c1 - c0);
      double rgba[4];
      tf_eval_f64(tf, val, rgba);
      const double keep = half_step ? sqrt(1.0 - rgba[3]) : pow(1.0 - rgba[3], step_vox);
      const double a = 1.0 - keep;
      const double wgt = T * a;
      cr += wgt * rgba[0];
      cg += wgt * rgba[1];
      cb += wgt * rgba[2];
      T *= 1.0 - a;
    }
  }
  image[pix] = static_cast<float>(cr + T * view.bg[0]);
  image[HW + pix] = static_cast<float>(cg + T * view.bg[1]);
  image[2 * HW + pix] = static_cast<float>(cb + T * view.bg[2]);
}

}  // namespace
}  // namespace vbm

using namespace vbm;

extern "C" vbm_status vbm_adam_step(int64_t n, int64_t stride, float* raw, float* m, float* v, vbm_gaussians_c g,
                                    vbm_gaussians act, const vbm_adam_opts* o, int32_t* step_dev, void* stream) {
  if (!raw || !m || !v || !o || !g.means || !g.scales || !g.quats || !g.opacity || !g.rgb || !act.means ||
      !act.scales || !act.quats || !act.opacity || !act.rgb) {
    set_error("vbm_adam_step: null argument");
    return VBM_ERR_INVALID;
  }
  if (n < 0 || stride < n || g.stride < n || act.stride < n || (!step_dev && o->step < 1) || !(o->beta1 >= 0.0f && o->beta1 < 1.0f) ||
      !(o->beta2 >= 0.0f && o->beta2 < 1.0f) || !(o->eps >= 0.0f)) {
    set_error("vbm_adam_step: bad sizes or hyper-parameters");
    return VBM_ERR_INVALID;
  }
  if (n == 0) return VBM_OK;
  AdamParams p;
  for (int k = 0; k < 5; ++k) p.lr[k] = o->lr[k];
  p.beta1 = o->beta1;
  p.beta2 = o->beta2;
  p.eps = o->eps;
  p.bc1 = p.bc2 = 1.0f;
  if (!step_dev) {
    p.bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(o->beta1), o->step));
    p.bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(o->beta2), o->step));
  } else {
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), step_dev);
    VBM_LAUNCH_CHECK("adam_step_inc");
  }
  hipLaunchKernelGGL(k_adam, dim3(ceil_div(n, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), n, stride, raw, m,
                     v, g, act, p, static_cast<const int32_t*>(step_dev));
  VBM_LAUNCH_CHECK("adam");
  return VBM_OK;
}

extern "C" vbm_status vbm_adam_init(int64_t n, int64_t stride, vbm_gaussians_c act, float* raw, float* m, float* v,
                                    void* stream) {
  if (!raw || !m || !v || !act.means || !act.scales || !act.quats || !act.opacity || !act.rgb) {
    set_error("vbm_adam_init: null argument");
    return VBM_ERR_INVALID;
  }
  if (n < 0 || stride < n || act.stride < n) {
    set_error("vbm_adam_init: bad sizes (n %lld, stride %lld, parameter stride %lld)", static_cast<long long>(n),
              static_cast<long long>(stride), static_cast<long long>(act.stride));
    return VBM_ERR_INVALID;
  }
  if (n == 0) return VBM_OK;
  hipLaunchKernelGGL(k_adam_init, dim3(ceil_div(n, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), n, stride,
                     act, raw, m, v);
  VBM_LAUNCH_CHECK("adam_init");
  return VBM_OK;
}

extern "C" vbm_status vbm_dvr_render(const float* vol, int32_t G, const vbm_tf* tf, const vbm_view* views,
                                     int32_t n_views, float step_vox, float* image, void* stream) {
  if (!vol || !tf || !views || !image) {
    set_error("vbm_dvr_render: null argument");
    return VBM_ERR_INVALID;
  }
  if (G < 2 || G > 2048 || n_views < 1 || !(step_vox > 0.0f) || !tf_valid(*tf)) {
    set_error("vbm_dvr_render: bad grid, view count, step or transfer function");
    return VBM_ERR_INVALID;
  }
  const DevTF dtf = make_dev_tf(*tf);
  int64_t off = 0;
  for (int v = 0; v < n_views; ++v) {
    if (views[v].width < 1 || views[v].height < 1 || !(views[v].fx > 0.0f) || !(views[v].fy > 0.0f)) {
      set_error("vbm_dvr_render: view %d is invalid", v);
      return VBM_ERR_INVALID;
    }
  }
  for (int v = 0; v < n_views; ++v) {
    const int64_t HW = static_cast<int64_t>(views[v].width) * views[v].height;
    hipLaunchKernelGGL(k_dvr, dim3(ceil_div(HW, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), vol, G, dtf,
                       views[v], static_cast<double>(step_vox), image + off);
    VBM_LAUNCH_CHECK("dvr");
    off += 3 * HW;
  }
  return VBM_OK;
}
