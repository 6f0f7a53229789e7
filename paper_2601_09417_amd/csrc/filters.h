// Wavelet filter banks derived on the host in double precision.
//
// Haar: h = (1, 1)/sqrt(2) at positions 0, 1.
// bior4.4 (= CDF 9/7, the paper's default basis, Sec. 4.2): both low-pass filters carry the factor
// cos^4(w/2) = ((2 + z + 1/z)/4)^2; the rest splits the Daubechies Bezout polynomial
// P(y) = 1 + 4y + 10y^2 + 20y^3, y = sin^2(w/2) = (2 - z - 1/z)/4: its real root r gives the 7-tap
// factor (1 - y/r), its complex pair c, conj(c) the 9-tap factor (1 - y/c)(1 - y/conj c).  The
// 9-tap filter is the analysis low-pass; both are normalised to sum sqrt(2).  High-pass filters by
// the alternating flip: hi_analysis[n] = (-1)^n lo_synthesis[1 - n], hi_synthesis[n] = (-1)^n lo_analysis[1 - n].
#pragma once

#include <cmath>
#include <vector>

namespace vbm {

struct Filter1D {
  std::vector<double> taps;
  int first = 0;  // position of taps[0]
};

struct FilterBankD {
  Filter1D lo_a, hi_a, lo_s, hi_s;
};

inline std::vector<double> poly_mul(const std::vector<double>& a, const std::vector<double>& b) {
  std::vector<double> r(a.size() + b.size() - 1, 0.0);
  for (size_t i = 0; i < a.size(); ++i)
    for (size_t j = 0; j < b.size(); ++j) r[i + j] += a[i] * b[j];
  return r;
}

inline Filter1D alternating_flip(const Filter1D& f) {
  const int last = f.first + static_cast<int>(f.taps.size()) - 1;
  Filter1D g;
  g.first = 1 - last;
  g.taps.resize(f.taps.size());
  for (size_t i = 0; i < f.taps.size(); ++i) {
    const int n = g.first + static_cast<int>(i);
    const double sign = ((n % 2) + 2) % 2 ? -1.0 : 1.0;
    g.taps[i] = sign * f.taps[(1 - n) - f.first];
  }
  return g;
}

inline FilterBankD make_filter_bank(int wavelet) {
  FilterBankD fb;
  if (wavelet == 0) {
    const double h = 1.0 / std::sqrt(2.0);
    fb.lo_a = {{h, h}, 0};
    fb.lo_s = {{h, h}, 0};
  } else {
    // real root of 20y^3 + 10y^2 + 4y + 1 by Newton iteration
    double r = -0.3;
    for (int it = 0; it < 100; ++it) {
      const double f = ((20.0 * r + 10.0) * r + 4.0) * r + 1.0;
      const double d = (60.0 * r + 20.0) * r + 4.0;
      const double step = f / d;
      r -= step;
      if (std::fabs(step) < 1e-17) break;
    }
    // deflate: 20y^3 + 10y^2 + 4y + 1 = (y - r)(20y^2 + q1 y + q2)
    const double q1 = 10.0 + 20.0 * r;
    const double q2 = 4.0 + r * q1;
    // (1 - y/c)(1 - y/conj c) = 1 - s y + p y^2 with s = 2 Re(c)/|c|^2 = -q1/q2, p = 1/|c|^2 = 20/q2
    const double s = -q1 / q2;
    const double p = 20.0 / q2;
    const std::vector<double> y = {-0.25, 0.5, -0.25};
    const std::vector<double> cos2 = {0.25, 0.5, 0.25};
    const std::vector<double> cos4 = poly_mul(cos2, cos2);
    std::vector<double> f7r = {y[0] * (-1.0 / r), 1.0 + y[1] * (-1.0 / r), y[2] * (-1.0 / r)};
    std::vector<double> y2 = poly_mul(y, y);
    std::vector<double> f9r(5, 0.0);
    for (int i = 0; i < 5; ++i) f9r[i] = p * y2[i];
    for (int i = 0; i < 3; ++i) f9r[i + 1] += -s * y[i];
    f9r[2] += 1.0;
    std::vector<double> lo7 = poly_mul(cos4, f7r);
    std::vector<double> lo9 = poly_mul(cos4, f9r);
    double s7 = 0, s9 = 0;
    for (double v : lo7) s7 += v;
    for (double v : lo9) s9 += v;
    for (double& v : lo7) v *= std::sqrt(2.0) / s7;
    for (double& v : lo9) v *= std::sqrt(2.0) / s9;
    fb.lo_a = {lo9, -4};
    fb.lo_s = {lo7, -3};
  }
  fb.hi_a = alternating_flip(fb.lo_s);
  fb.hi_s = alternating_flip(fb.lo_a);
  return fb;
}

}  // namespace vbm
