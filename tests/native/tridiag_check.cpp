// Prints, for seeded random symmetric tridiagonal matrices of several sizes
// and spectra (including clustered top eigenvalues), the largest eigenvalue
// and the last component of its unit eigenvector as computed by the
// library's tridiag.hpp (the Ritz step of its Lanczos estimate).  Compared
// with numpy's dense symmetric eigensolver by tests/test_native_tridiag.py.
#include "../../paper_1512_08401_amd/csrc/tridiag.hpp"

#include <cstdio>
#include <random>

int main() {
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  const int sizes[] = {1, 2, 3, 7, 40, 200, 800};
  for (int kind = 0; kind < 3; ++kind) {
    for (int m : sizes) {
      std::vector<double> a(m), b(m > 1 ? m - 1 : 0);
      for (int i = 0; i < m; ++i) a[i] = kind == 2 ? 1.0 + 1e-9 * U(rng) : U(rng);
      for (int i = 0; i + 1 < m; ++i) b[i] = kind == 1 ? 1e-6 * U(rng) : (kind == 2 ? 1e-7 * U(rng) : U(rng));
      const wdb::TopRitz t = wdb::top_ritz(a, b);
      std::printf("%d %d", kind, m);
      for (double v : a) std::printf(" %.17g", v);
      for (double v : b) std::printf(" %.17g", v);
      std::printf(" | %.17g %.17g\n", t.theta, t.last);
    }
  }
  return 0;
}
