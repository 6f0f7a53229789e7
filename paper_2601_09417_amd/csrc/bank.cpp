// Wavelet-to-Gaussian Transition Bank (Sec. 4.2), computed once on the host in double precision.
//
// For each subband (j, o) in packed block order -- (J, LLL) first, then the seven detail
// orientations of levels J..1 -- the canonical wavelet is the inverse DWT of a unit impulse at
// k = 0 (eq. wavelet_impulse, eq. canonical_wavelet).  The 3D synthesis is a tensor product and
// levels below j only apply low-pass synthesis, so the canonical wavelet is the outer product of
// three 1D impulse responses, each synthesised here on a periodic line long enough not to wrap.
// Dominant-lobe estimation keeps the ROI |psi| > tau max|psi| (eq. roi, equivalently W > tau max W),
// takes the |psi|-weighted centroid and covariance over it (eq. moment, voxel-index units relative
// to the impulse origin), and fits the amplitude by ridge regression of |psi| on the Gaussian of
// eq. canonical_gaussian over the ROI (eq. ridge_regression).  The covariance is factored as
// R diag(scale^2) R^T: identity rotation when it is diagonal, else a Jacobi eigendecomposition.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "filters.h"

namespace vbm {
namespace {

std::vector<double> synth_periodic(const std::vector<double>& lo, const std::vector<double>& hi, const FilterBankD& fb) {
  const int n = static_cast<int>(lo.size());
  const int N = 2 * n;
  std::vector<double> x(N, 0.0);
  for (int k = 0; k < n; ++k) {
    if (lo[k] != 0.0)
      for (size_t i = 0; i < fb.lo_s.taps.size(); ++i) {
        int m = fb.lo_s.first + static_cast<int>(i);
        x[((2 * k + m) % N + N) % N] += lo[k] * fb.lo_s.taps[i];
      }
    if (hi[k] != 0.0)
      for (size_t i = 0; i < fb.hi_s.taps.size(); ++i) {
        int m = fb.hi_s.first + static_cast<int>(i);
        x[((2 * k + m) % N + N) % N] += hi[k] * fb.hi_s.taps[i];
      }
  }
  return x;
}

struct Response {
  std::vector<double> v;
  int first_rel;  // position of v[0] relative to the impulse origin 2^j k0
};

Response impulse_response(const FilterBankD& fb, int j, bool high) {
  const int n = 64;
  const int k0 = n / 2;
  std::vector<double> lo(n, 0.0), hi(n, 0.0);
  (high ? hi : lo)[k0] = 1.0;
  std::vector<double> cur = synth_periodic(lo, hi, fb);
  for (int l = 1; l < j; ++l) {
    std::vector<double> z(cur.size(), 0.0);
    cur = synth_periodic(cur, z, fb);
  }
  int a = -1, b = -1;
  for (int i = 0; i < static_cast<int>(cur.size()); ++i)
    if (cur[i] != 0.0) {
      if (a < 0) a = i;
      b = i;
    }
  Response r;
  r.v.assign(cur.begin() + a, cur.begin() + b + 1);
  r.first_rel = a - (1 << j) * k0;
  return r;
}

// Jacobi eigendecomposition of a symmetric 3x3 matrix: A = V diag(e) V^T, e ascending.
void jacobi3(const double S[3][3], double e[3], double V[3][3]) {
  double A[3][3];
  std::memcpy(A, S, sizeof(A));
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) V[i][k] = i == k ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = std::fabs(A[0][1]) + std::fabs(A[0][2]) + std::fabs(A[1][2]);
    if (off < 1e-300) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (std::fabs(A[p][q]) < 1e-300) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {  // A <- A G
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  // A <- G^T A
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  int idx[3] = {0, 1, 2};
  for (int a = 0; a < 3; ++a)
    for (int b = a + 1; b < 3; ++b)
      if (A[idx[b]][idx[b]] < A[idx[a]][idx[a]]) std::swap(idx[a], idx[b]);
  double Vs[3][3];
  for (int c = 0; c < 3; ++c) {
    e[c] = A[idx[c]][idx[c]];
    for (int r = 0; r < 3; ++r) Vs[r][c] = V[r][idx[c]];
  }
  std::memcpy(V, Vs, sizeof(Vs));
}

void rotation_to_quat(const double R[3][3], double q[4]) {
  const double tr = R[0][0] + R[1][1] + R[2][2];
  if (tr > 0) {
    const double s = std::sqrt(tr + 1.0) * 2;
    q[0] = 0.25 * s;
    q[1] = (R[2][1] - R[1][2]) / s;
    q[2] = (R[0][2] - R[2][0]) / s;
    q[3] = (R[1][0] - R[0][1]) / s;
  } else if (R[0][0] > R[1][1] && R[0][0] > R[2][2]) {
    const double s = std::sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]) * 2;
    q[0] = (R[2][1] - R[1][2]) / s;
    q[1] = 0.25 * s;
    q[2] = (R[0][1] + R[1][0]) / s;
    q[3] = (R[0][2] + R[2][0]) / s;
  } else if (R[1][1] > R[2][2]) {
    const double s = std::sqrt(1.0 + R[1][1] - R[0][0] - R[2][2]) * 2;
    q[0] = (R[0][2] - R[2][0]) / s;
    q[1] = (R[0][1] + R[1][0]) / s;
    q[2] = 0.25 * s;
    q[3] = (R[1][2] + R[2][1]) / s;
  } else {
    const double s = std::sqrt(1.0 + R[2][2] - R[0][0] - R[1][1]) * 2;
    q[0] = (R[1][0] - R[0][1]) / s;
    q[1] = (R[0][2] + R[2][0]) / s;
    q[2] = (R[1][2] + R[2][1]) / s;
    q[3] = 0.25 * s;
  }
  double nrm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double sg = q[0] < 0 ? -1.0 : 1.0;
  for (int i = 0; i < 4; ++i) q[i] = sg * q[i] / nrm;
}

void fit(const Response r[3], double tau, double lambda, vbm_bank_entry* e) {
  double mx[3];
  for (int d = 0; d < 3; ++d) {
    mx[d] = 0;
    for (double v : r[d].v) mx[d] = std::fmax(mx[d], std::fabs(v));
  }
  const double thr = tau * mx[0] * mx[1] * mx[2];
  const int nx = static_cast<int>(r[0].v.size()), ny = static_cast<int>(r[1].v.size()),
            nz = static_cast<int>(r[2].v.size());
  double sw = 0, s1[3] = {0, 0, 0};
  int roi = 0;
  for (int c = 0; c < nz; ++c)
    for (int b = 0; b < ny; ++b)
      for (int a = 0; a < nx; ++a) {
        const double w = std::fabs(r[0].v[a] * r[1].v[b] * r[2].v[c]);
        if (!(w > thr)) continue;
        sw += w;
        s1[0] += w * (r[0].first_rel + a);
        s1[1] += w * (r[1].first_rel + b);
        s1[2] += w * (r[2].first_rel + c);
        ++roi;
      }
  double u[3] = {s1[0] / sw, s1[1] / sw, s1[2] / sw};
  double S[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int c = 0; c < nz; ++c)
    for (int b = 0; b < ny; ++b)
      for (int a = 0; a < nx; ++a) {
        const double w = std::fabs(r[0].v[a] * r[1].v[b] * r[2].v[c]);
        if (!(w > thr)) continue;
        const double d[3] = {r[0].first_rel + a - u[0], r[1].first_rel + b - u[1], r[2].first_rel + c - u[2]};
        for (int i = 0; i < 3; ++i)
          for (int k = 0; k < 3; ++k) S[i][k] += w * d[i] * d[k];
      }
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) S[i][k] /= sw;
  // inverse of S for the Gaussian envelope
  const double det = S[0][0] * (S[1][1] * S[2][2] - S[1][2] * S[2][1]) - S[0][1] * (S[1][0] * S[2][2] - S[1][2] * S[2][0]) +
                     S[0][2] * (S[1][0] * S[2][1] - S[1][1] * S[2][0]);
  double Si[3][3];
  Si[0][0] = (S[1][1] * S[2][2] - S[1][2] * S[2][1]) / det;
  Si[0][1] = (S[0][2] * S[2][1] - S[0][1] * S[2][2]) / det;
  Si[0][2] = (S[0][1] * S[1][2] - S[0][2] * S[1][1]) / det;
  Si[1][0] = Si[0][1];
  Si[1][1] = (S[0][0] * S[2][2] - S[0][2] * S[2][0]) / det;
  Si[1][2] = (S[0][2] * S[1][0] - S[0][0] * S[1][2]) / det;
  Si[2][0] = Si[0][2];
  Si[2][1] = Si[1][2];
  Si[2][2] = (S[0][0] * S[1][1] - S[0][1] * S[1][0]) / det;
  double gy = 0, gg = 0;
  for (int c = 0; c < nz; ++c)
    for (int b = 0; b < ny; ++b)
      for (int a = 0; a < nx; ++a) {
        const double y = std::fabs(r[0].v[a] * r[1].v[b] * r[2].v[c]);
        if (!(y > thr)) continue;
        const double d[3] = {r[0].first_rel + a - u[0], r[1].first_rel + b - u[1], r[2].first_rel + c - u[2]};
        double q = 0;
        for (int i = 0; i < 3; ++i)
          for (int k = 0; k < 3; ++k) q += d[i] * Si[i][k] * d[k];
        const double g = std::exp(-0.5 * q);
        gy += g * y;
        gg += g * g;
      }
  e->w = gy / (gg + lambda);
  for (int i = 0; i < 3; ++i) e->u[i] = u[i];
  e->sigma[0] = S[0][0];
  e->sigma[1] = S[1][1];
  e->sigma[2] = S[2][2];
  e->sigma[3] = S[0][1];
  e->sigma[4] = S[0][2];
  e->sigma[5] = S[1][2];
  e->roi_size = roi;
  const double offd = std::fmax(std::fabs(S[0][1]), std::fmax(std::fabs(S[0][2]), std::fabs(S[1][2])));
  const double dmax = std::fmax(std::fabs(S[0][0]), std::fmax(std::fabs(S[1][1]), std::fabs(S[2][2])));
  if (offd <= 1e-12 * dmax) {
    for (int i = 0; i < 3; ++i) e->scale[i] = std::sqrt(S[i][i]);
    e->quat[0] = 1.0;
    e->quat[1] = e->quat[2] = e->quat[3] = 0.0;
  } else {
    double ev[3], V[3][3];
    jacobi3(S, ev, V);
    const double dV = V[0][0] * (V[1][1] * V[2][2] - V[1][2] * V[2][1]) - V[0][1] * (V[1][0] * V[2][2] - V[1][2] * V[2][0]) +
                      V[0][2] * (V[1][0] * V[2][1] - V[1][1] * V[2][0]);
    if (dV < 0)
      for (int i = 0; i < 3; ++i) V[i][0] = -V[i][0];
    for (int i = 0; i < 3; ++i) e->scale[i] = std::sqrt(ev[i]);
    rotation_to_quat(V, e->quat);
  }
}

}  // namespace
}  // namespace vbm

using namespace vbm;

extern "C" int32_t vbm_bank_size(int32_t J) { return J >= 1 ? 7 * J + 1 : 0; }

extern "C" vbm_status vbm_bank_build(int32_t wavelet, int32_t J, double tau, double lambda, vbm_bank_entry* out) {
  if (!out) {
    set_error("vbm_bank_build: null output");
    return VBM_ERR_INVALID;
  }
  if (J < 1 || J > 8 || !(tau >= 0.0 && tau < 1.0) || !(lambda >= 0.0)) {
    set_error("vbm_bank_build: need 1 <= J <= 8, 0 <= tau < 1, lambda >= 0");
    return VBM_ERR_INVALID;
  }
  if (wavelet != VBM_WAVELET_HAAR && wavelet != VBM_WAVELET_BIOR44) {
    set_error("vbm_bank_build: unknown wavelet %d", wavelet);
    return VBM_ERR_UNSUPPORTED;
  }
  const FilterBankD fb = make_filter_bank(wavelet);
  int idx = 0;
  auto one = [&](int j, int o) {
    Response r[3];
    for (int d = 0; d < 3; ++d) r[d] = impulse_response(fb, j, (o >> d) & 1);
    vbm_bank_entry& e = out[idx++];
    std::memset(&e, 0, sizeof(e));
    e.j = j;
    e.o = o;
    fit(r, tau, lambda, &e);
  };
  one(J, 0);
  for (int j = J; j >= 1; --j)
    for (int o = 1; o < 8; ++o) one(j, o);
  return VBM_OK;
}

extern "C" vbm_status vbm_bank_pack(const vbm_bank_entry* e, int32_t n, float* out) {
  if (!e || !out || n <= 0) {
    set_error("vbm_bank_pack: bad arguments");
    return VBM_ERR_INVALID;
  }
  for (int i = 0; i < n; ++i) {
    float* o = out + static_cast<size_t>(i) * VBM_BANK_FLOATS;
    o[0] = static_cast<float>(e[i].w);
    for (int k = 0; k < 3; ++k) o[1 + k] = static_cast<float>(e[i].u[k]);
    for (int k = 0; k < 3; ++k) o[4 + k] = static_cast<float>(e[i].scale[k]);
    for (int k = 0; k < 4; ++k) o[7 + k] = static_cast<float>(e[i].quat[k]);
    o[11] = 0.0f;
  }
  return VBM_OK;
}
