// Wavelet filters, geometry checks and the canonical coefficient layout.
//
// The Daubechies filter with p vanishing moments (the family named in
// Sec. 3.5; vanishing moments are defined in Sec. 2) is derived here by
// spectral factorisation rather than typed in: the squared modulus of the
// low-pass response is cos(w/2)^(2p) P(sin(w/2)^2) with
// P(y) = sum_{k<p} binom(p-1+k, k) y^k.  The roots of P are found with the
// Weierstrass (Durand-Kerner) simultaneous iteration in long double; each root
// y gives the reciprocal pair z + 1/z = 2 - 4y, of which the root inside the
// unit circle is kept (minimum phase).  Expanding (1 + w)^p prod (1 - z_i w)
// in w = 1/z and scaling the taps to sum sqrt(2) yields h.  The Symmlet of
// the experiments of Sec. 5 is another factor of the same polynomial (below).
#include <algorithm>
#include <cmath>
#include <complex>

#include "common.hpp"

namespace wdb {

namespace {

using cplx = std::complex<long double>;

long double binom(int n, int k) {
  long double r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// All roots of sum_k c[k] y^k (c ascending, c.back() != 0).
std::vector<cplx> poly_roots(const std::vector<long double>& c) {
  const int d = static_cast<int>(c.size()) - 1;
  std::vector<cplx> r(d);
  if (d == 0) return r;
  const cplx seed(0.4L, 0.9L);
  cplx s = 1;
  for (int i = 0; i < d; ++i) { r[i] = s; s *= seed; }
  auto eval = [&](cplx y) {
    cplx acc = 0;
    for (int k = d; k >= 0; --k) acc = acc * y + cplx(c[k] / c[d]);
    return acc;
  };
  for (int it = 0; it < 500; ++it) {
    long double delta = 0;
    for (int i = 0; i < d; ++i) {
      cplx den = 1;
      for (int j = 0; j < d; ++j)
        if (j != i) den *= (r[i] - r[j]);
      cplx step = eval(r[i]) / den;
      r[i] -= step;
      delta = std::max(delta, std::abs(step));
    }
    if (delta < 1e-30L) break;
  }
  return r;
}

std::vector<double> daubechies(int p) {
  std::vector<long double> P(p);
  for (int k = 0; k < p; ++k) P[k] = binom(p - 1 + k, k);
  std::vector<cplx> coeffs{cplx(1)};
  auto mul = [&](cplx a0, cplx a1) {  // coeffs *= (a0 + a1 w)
    std::vector<cplx> out(coeffs.size() + 1, cplx(0));
    for (size_t i = 0; i < coeffs.size(); ++i) {
      out[i] += coeffs[i] * a0;
      out[i + 1] += coeffs[i] * a1;
    }
    coeffs.swap(out);
  };
  for (int i = 0; i < p; ++i) mul(1, 1);
  if (p > 1) {
    for (const cplx& y : poly_roots(P)) {
      const cplx b = 2.0L - 4.0L * y;  // z^2 - b z + 1 = 0
      const cplx disc = std::sqrt(b * b - 4.0L);
      cplx z1 = (b + disc) / 2.0L, z2 = (b - disc) / 2.0L;
      const cplx z = std::abs(z1) < std::abs(z2) ? z1 : z2;
      mul(1, -z);
    }
  }
  long double sum = 0;
  for (auto& c : coeffs) sum += c.real();
  const long double scale = std::sqrt(2.0L) / sum;
  std::vector<double> h(coeffs.size());
  for (size_t i = 0; i < coeffs.size(); ++i) h[i] = static_cast<double>(coeffs[i].real() * scale);
  return h;
}

// Least-asymmetric ("Symmlet") filter with p vanishing moments: a spectral
// factor of the same |m0|^2 whose phase is closest to linear (Daubechies'
// Symmlets).  Every root y of P offers z or 1/z; complex-conjugate roots take
// the same choice so the taps stay real.  The phase of
// Q(w) = prod (1 - z_i e^{-iw}) (the rest of m0, (1 + e^{-iw})^p, has exactly
// linear phase) is unwrapped on 2049 points of [0, pi] and the largest distance
// to its chord scores a choice; the smallest score wins.  A choice and its
// mirror image (every zero inverted: the time-reversed filter) score the
// same; the one taking the inner zero of the root with the smallest real part
// (then imaginary part) is kept.
std::vector<double> symlet(int p) {
  std::vector<long double> P(p);
  for (int k = 0; k < p; ++k) P[k] = binom(p - 1 + k, k);
  std::vector<cplx> ys = poly_roots(P);
  std::sort(ys.begin(), ys.end(), [](const cplx& a, const cplx& b) {
    const long double ar = std::round(a.real() * 1e12L), br = std::round(b.real() * 1e12L);
    if (ar != br) return ar < br;
    return std::round(a.imag() * 1e12L) < std::round(b.imag() * 1e12L);
  });
  struct Pair { cplx in, out; };
  std::vector<Pair> pr;
  for (const cplx& y : ys) {
    const cplx b = 2.0L - 4.0L * y;
    const cplx disc = std::sqrt(b * b - 4.0L);
    cplx z1 = (b + disc) / 2.0L, z2 = (b - disc) / 2.0L;
    if (std::abs(z1) > std::abs(z2)) std::swap(z1, z2);
    pr.push_back({z1, z2});
  }
  std::vector<std::vector<int>> groups;
  std::vector<bool> used(ys.size(), false);
  for (size_t i = 0; i < ys.size(); ++i) {
    if (used[i]) continue;
    used[i] = true;
    std::vector<int> g{static_cast<int>(i)};
    if (std::fabs(ys[i].imag()) > 1e-12L)
      for (size_t j = i + 1; j < ys.size(); ++j)
        if (!used[j] && std::abs(ys[j] - std::conj(ys[i])) < 1e-9L) {
          used[j] = true;
          g.push_back(static_cast<int>(j));
          break;
        }
    groups.push_back(g);
  }
  const long double pi = 3.141592653589793238462643383279502884L;
  auto score = [&](const std::vector<cplx>& zs) {
    const int M = 2048;
    std::vector<long double> ph(M + 1);
    long double prev = 0, acc = 0;
    for (int t = 0; t <= M; ++t) {
      const long double w = pi * t / M;
      const cplx e(std::cos(w), -std::sin(w));
      cplx q = 1;
      for (const cplx& z : zs) q *= (1.0L - z * e);
      const long double a = std::arg(q);
      if (t == 0) acc = a;
      else {
        long double d = a - prev;
        while (d > pi) d -= 2 * pi;
        while (d < -pi) d += 2 * pi;
        acc += d;
      }
      prev = a;
      ph[t] = acc;
    }
    long double worst = 0;
    for (int t = 0; t <= M; ++t) {
      const long double chord = ph[0] + (ph[M] - ph[0]) * t / M;
      worst = std::max(worst, std::fabs(ph[t] - chord));
    }
    return worst;
  };
  std::vector<cplx> best;
  long double best_score = 0;
  for (unsigned mask = 0; mask < (1u << groups.size()); ++mask) {
    if (mask & 1u) continue;  // mirror images: the first group keeps its inner zero
    std::vector<cplx> zs;
    for (size_t gi = 0; gi < groups.size(); ++gi)
      for (int i : groups[gi]) zs.push_back(((mask >> gi) & 1u) ? pr[i].out : pr[i].in);
    const long double sc = score(zs);
    if (best.empty() || sc < best_score - 1e-12L) {
      best = zs;
      best_score = sc;
    }
  }
  std::vector<cplx> coeffs{cplx(1)};
  auto mul = [&](cplx a0, cplx a1) {
    std::vector<cplx> out(coeffs.size() + 1, cplx(0));
    for (size_t i = 0; i < coeffs.size(); ++i) {
      out[i] += coeffs[i] * a0;
      out[i + 1] += coeffs[i] * a1;
    }
    coeffs.swap(out);
  };
  for (int i = 0; i < p; ++i) mul(1, 1);
  for (const cplx& z : best) mul(1, -z);
  long double sum = 0;
  for (auto& c : coeffs) sum += c.real();
  const long double scale = std::sqrt(2.0L) / sum;
  std::vector<double> h(coeffs.size());
  for (size_t i = 0; i < coeffs.size(); ++i) h[i] = static_cast<double>(coeffs[i].real() * scale);
  return h;
}

}  // namespace

Filter make_filter(int wavelet) {
  Filter f;
  if (wavelet == WDB_HAAR) {
    const double s = 1.0 / std::sqrt(2.0);
    f.h = {s, s};
  } else if (wavelet == WDB_DB4) {
    static const std::vector<double> taps = daubechies(4);  // factorised once per process
    f.h = taps;
  } else if (wavelet == WDB_SYM6) {
    static const std::vector<double> taps = symlet(6);
    f.h = taps;
  } else {
    fail(WDB_ERR_ARG, "unknown wavelet %d", wavelet);
  }
  const size_t L = f.h.size();
  f.g.resize(L);
  for (size_t m = 0; m < L; ++m) f.g[m] = ((m & 1) ? -1.0 : 1.0) * f.h[L - 1 - m];
  return f;
}

void check_geometry(int32_t n, int32_t levels, int flen) {
  WDB_REQUIRE(n >= 2 && (n & (n - 1)) == 0, WDB_ERR_SIZE, "image side %d is not a power of two >= 2", n);
  WDB_REQUIRE(n <= (1 << 14), WDB_ERR_SIZE, "image side %d exceeds 16384", n);
  WDB_REQUIRE(levels >= 1 && levels < 31 && (n >> levels) >= 1 && (n >> (levels - 1)) >= flen,
              WDB_ERR_LEVELS, "%d levels do not fit n = %d with a %d-tap filter", levels, n, flen);
}

std::vector<Subband> layout(int32_t n, int32_t levels) {
  std::vector<Subband> out;
  const int side = n >> levels;
  out.push_back({levels, 0, 0, 0, side});
  int64_t off = int64_t(side) * side;
  static const int E[3][2] = {{0, 1}, {1, 0}, {1, 1}};
  for (int lev = levels; lev >= 1; --lev) {
    const int s = n >> lev;
    for (auto& e : E) {
      out.push_back({lev, e[0], e[1], off, s});
      off += int64_t(s) * s;
    }
  }
  return out;
}

}  // namespace wdb

extern "C" wdb_status wdb_wavelet_filter(int32_t wavelet, double* h_out, int32_t capacity,
                                         int32_t* len_out) {
  WDB_API_BEGIN
  WDB_REQUIRE(len_out, WDB_ERR_ARG, "null len_out");
  WDB_REQUIRE(capacity >= 0, WDB_ERR_ARG, "negative capacity");
  wdb::Filter f = wdb::make_filter(wavelet);
  const int32_t taps = static_cast<int32_t>(f.h.size());
  *len_out = taps;
  if (h_out == nullptr && capacity == 0) return WDB_OK;  // length query
  WDB_REQUIRE(h_out, WDB_ERR_ARG, "null h_out with non-zero capacity");
  WDB_REQUIRE(capacity >= taps, WDB_ERR_ARG, "h_out holds %d doubles, the filter has %d taps", capacity, taps);
  for (int32_t i = 0; i < taps; ++i) h_out[i] = f.h[i];
  WDB_API_END
}
