// Piecewise-linear transfer function evaluated on the device (Sec. 3, Transfer Function):
// RGBA by linear interpolation between ascending control points, constant beyond the end points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>

#include "common.h"

namespace vbm {

struct DevTF {
  float x[VBM_TF_MAX_POINTS];
  float rgba[VBM_TF_MAX_POINTS][4];
  int n;
};

__device__ __forceinline__ float4 tf_eval(const DevTF& tf, float f) {
  if (!(f > tf.x[0])) return make_float4(tf.rgba[0][0], tf.rgba[0][1], tf.rgba[0][2], tf.rgba[0][3]);
  const int n = tf.n;
  if (f >= tf.x[n - 1])
    return make_float4(tf.rgba[n - 1][0], tf.rgba[n - 1][1], tf.rgba[n - 1][2], tf.rgba[n - 1][3]);
  int j = 0;
  for (int i = 1; i < n - 1; ++i)
    if (tf.x[i] <= f) j = i;
  const float x0 = tf.x[j], x1 = tf.x[j + 1];
  const float t = x1 > x0 ? (f - x0) / (x1 - x0) : 1.0f;
  return make_float4(tf.rgba[j][0] + t * (tf.rgba[j + 1][0] - tf.rgba[j][0]),
                     tf.rgba[j][1] + t * (tf.rgba[j + 1][1] - tf.rgba[j][1]),
                     tf.rgba[j][2] + t * (tf.rgba[j + 1][2] - tf.rgba[j][2]),
                     tf.rgba[j][3] + t * (tf.rgba[j + 1][3] - tf.rgba[j][3]));
}

inline DevTF make_dev_tf(const vbm_tf& tf) {
  DevTF d;
  std::memset(&d, 0, sizeof(d));
  d.n = tf.n_points;
  for (int i = 0; i < tf.n_points; ++i) {
    d.x[i] = tf.x[i];
    for (int c = 0; c < 4; ++c) d.rgba[i][c] = tf.rgba[i][c];
  }
  return d;
}

inline bool tf_valid(const vbm_tf& tf) {
  if (tf.n_points < 2 || tf.n_points > VBM_TF_MAX_POINTS) return false;
  for (int i = 1; i < tf.n_points; ++i)
    if (!(tf.x[i] >= tf.x[i - 1])) return false;
  return true;
}

}  // namespace vbm
