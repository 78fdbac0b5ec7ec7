// Largest eigenvalue of a symmetric tridiagonal matrix and the last
// component of its eigenvector (host code; the Ritz step of the Lanczos
// estimate of ||Theta_K||^2).
#pragma once

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

namespace wdb {

// Largest eigenvalue of the symmetric tridiagonal matrix (diagonal a, off
// diagonal b) by bisection on the Sturm count, and the last component of its
// unit eigenvector by inverse iteration (tridiagonal elimination with
// partial pivoting).
struct TopRitz {
  double theta, last;
  std::vector<double> vec;  // the unit eigenvector (sign arbitrary)
};

inline int sturm_below(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double bb = i ? b[i - 1] * b[i - 1] : 0.0;
    q = a[i] - x - (i ? bb / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

inline TopRitz top_ritz(const std::vector<double>& a, const std::vector<double>& b) {
  const size_t m = a.size();
  double lo = a[0], hi = a[0];
  for (size_t i = 0; i < m; ++i) {
    const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {   // the top eigenvalue lies in (lo, hi]
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_below(a, b, mid) == static_cast<int>(m)) hi = mid; else lo = mid;
  }
  const double theta = hi;
  if (m == 1) return TopRitz{theta, 1.0, std::vector<double>(1, 1.0)};
  // inverse iteration on (T - shift I), shift just above theta
  const double shift = theta + 4.0 * std::numeric_limits<double>::epsilon() * std::max(std::fabs(theta), 1e-300);
  std::vector<double> x(m, 1.0), dl(m), d(m), du(m), du2(m), rhs(m);
  for (int pass = 0; pass < 3; ++pass) {
    for (size_t i = 0; i < m; ++i) {
      d[i] = a[i] - shift;
      if (i + 1 < m) dl[i] = du[i] = b[i];
      du2[i] = 0.0;
      rhs[i] = x[i];
    }
    std::vector<int> piv(m, 0);
    for (size_t i = 0; i + 1 < m; ++i) {   // elimination with row interchanges
      if (std::fabs(d[i]) >= std::fabs(dl[i])) {
        const double f = d[i] != 0.0 ? dl[i] / d[i] : 0.0;
        d[i + 1] -= f * du[i];
        rhs[i + 1] -= f * rhs[i];
        if (i + 2 < m) du2[i] = 0.0;
      } else {
        const double f = d[i] / dl[i];
        d[i] = dl[i];
        const double t = d[i + 1];
        d[i + 1] = du[i] - f * t;
        du[i] = t;
        if (i + 2 < m) {
          du2[i] = du[i + 1];
          du[i + 1] = -f * du[i + 1];
        }
        std::swap(rhs[i], rhs[i + 1]);
        rhs[i + 1] -= f * rhs[i];
        piv[i] = 1;
      }
    }
    for (size_t k = m; k-- > 0;) {   // back substitution
      double t = rhs[k];
      if (k + 1 < m) t -= du[k] * x[k + 1];
      if (k + 2 < m) t -= du2[k] * x[k + 2];
      x[k] = d[k] != 0.0 ? t / d[k] : t / 1e-300;
    }
    double nrm = 0.0;
    for (double v : x) nrm += v * v;
    nrm = std::sqrt(nrm);
    for (double& v : x) v /= nrm;
  }
  return TopRitz{theta, x[m - 1], x};
}


}  // namespace wdb
