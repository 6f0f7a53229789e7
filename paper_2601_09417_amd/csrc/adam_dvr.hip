// vbm_adam_step (Adam on the raw parameters, Sec. 5 Implementation Details) and vbm_dvr_render
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

// One thread per pixel of one view.
__global__ __launch_bounds__(256) void k_dvr(const float* __restrict__ vol, int G, DevTF tf, vbm_view view,
                                             float step_vox, float* __restrict__ image) {
  const int64_t HW = static_cast<int64_t>(view.width) * view.height;
  const int64_t pix = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (pix >= HW) return;
  const int px = static_cast<int>(pix % view.width), py = static_cast<int>(pix / view.width);
  const float* V = view.viewmat;
  // eye = -R^T t, direction = R^T d_cam (normalised)
  const float ex = -(V[0] * V[3] + V[4] * V[7] + V[8] * V[11]);
  const float ey = -(V[1] * V[3] + V[5] * V[7] + V[9] * V[11]);
  const float ez = -(V[2] * V[3] + V[6] * V[7] + V[10] * V[11]);
  const float u = (static_cast<float>(px) + 0.5f - view.cx) / view.fx;
  const float w = (static_cast<float>(py) + 0.5f - view.cy) / view.fy;
  float dx = V[0] * u + V[4] * w + V[8];
  float dy = V[1] * u + V[5] * w + V[9];
  float dz = V[2] * u + V[6] * w + V[10];
  const float inv_n = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  dx *= inv_n;
  dy *= inv_n;
  dz *= inv_n;
  const float e[3] = {ex, ey, ez}, d[3] = {dx, dy, dz};
  float tn = -INFINITY, tf_ = INFINITY;
  for (int a = 0; a < 3; ++a) {
    const float inv = 1.0f / d[a];
    const float t1 = (-1.0f - e[a]) * inv, t2 = (1.0f - e[a]) * inv;
    tn = fmaxf(tn, fminf(t1, t2));
    tf_ = fminf(tf_, fmaxf(t1, t2));
  }
  tn = fmaxf(tn, 0.0f);
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  if (tf_ > tn) {
    const float h = 2.0f / static_cast<float>(G);
    const float dt = step_vox * h;
    const int nsteps = static_cast<int>(floorf((tf_ - tn) / dt)) + 1;
    const int64_t G2 = static_cast<int64_t>(G) * G;
    for (int k = 0; k < nsteps && T >= 1e-4f; ++k) {
      const float t = tn + static_cast<float>(k) * dt;
      const float p[3] = {ex + t * dx, ey + t * dy, ez + t * dz};
      int i0[3];
      float f[3];
      for (int a = 0; a < 3; ++a) {
        float q = (p[a] + 1.0f) / h - 0.5f;
        q = fminf(fmaxf(q, 0.0f), static_cast<float>(G - 1));
        int i = static_cast<int>(floorf(q));
        if (i > G - 2) i = G - 2;
        i0[a] = i;
        f[a] = q - static_cast<float>(i);
      }
      const float* b = vol + i0[2] * G2 + static_cast<int64_t>(i0[1]) * G + i0[0];
      const float c000 = b[0], c001 = b[1], c010 = b[G], c011 = b[G + 1];
      const float c100 = b[G2], c101 = b[G2 + 1], c110 = b[G2 + G], c111 = b[G2 + G + 1];
      const float c00 = c000 + f[0] * (c001 - c000), c01 = c010 + f[0] * (c011 - c010);
      const float c10 = c100 + f[0] * (c101 - c100), c11 = c110 + f[0] * (c111 - c110);
      const float c0 = c00 + f[1] * (c01 - c00), c1 = c10 + f[1] * (c11 - c10);
      const float val = c0 + f[2] * (c1 - c0);
      const float4 rgba = tf_eval(tf, val);
      const float a = 1.0f - powf(1.0f - rgba.w, step_vox);
      const float wgt = T * a;
      cr += wgt * rgba.x;
      cg += wgt * rgba.y;
      cb += wgt * rgba.z;
      T *= 1.0f - a;
    }
  }
  image[pix] = cr + T * view.bg[0];
  image[HW + pix] = cg + T * view.bg[1];
  image[2 * HW + pix] = cb + T * view.bg[2];
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
                       views[v], step_vox, image + off);
    VBM_LAUNCH_CHECK("dvr");
    off += 3 * HW;
  }
  return VBM_OK;
}
