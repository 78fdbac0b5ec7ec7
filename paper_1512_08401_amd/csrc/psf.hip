// Spatially varying Gaussian blur (Sec. 3.1, column convention) on the GPU.
//
// Column s of H is the PSF k_s of source pixel s.  For an integer offset
// d = (dy, dx) (rows, columns):
//   t1 = dx cos(a) + dy sin(a),  t2 = -dx sin(a) + dy cos(a),
//   q  = t1^2 / sig_major^2 + t2^2 / sig_minor^2,
//   k_s(d) = exp(-q/2) / Z_s  if q <= trunc^2, else 0,   Z_s = sum_d exp(-q/2) [q <= trunc^2].
// Arithmetic is float64 with contraction disabled in q, so the cut-off
// decision is the plain IEEE evaluation of the formula.
#include <cmath>

#include "common.hpp"
#include "psf.hpp"

namespace wdb {

namespace {

__global__ __launch_bounds__(256) void k_psf_norm(PsfDev P, double* __restrict__ Z) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t N = static_cast<int64_t>(P.n) * P.n;
  if (s >= N) return;
  const int R = static_cast<int>(floor(P.trunc * fmax(P.sM[s], P.sm[s])));
  double z = 0.0;
  for (int dy = -R; dy <= R; ++dy)
    for (int dx = -R; dx <= R; ++dx) z += psf_unnormalised(P, s, dy, dx);
  Z[s] = z;
}

// out[i] = sum_d k_{i-d}(d) u[i-d]  (gather form of H u).
__global__ __launch_bounds__(256) void k_blur(PsfDev P, const float* __restrict__ u, float* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int n = P.n;
  const int64_t N = static_cast<int64_t>(n) * n;
  if (i >= N) return;
  const int ir = static_cast<int>(i / n), ic = static_cast<int>(i % n);
  const int R = P.R;
  double acc = 0.0;
  for (int dy = -R; dy <= R; ++dy) {
    const int sr = (ir - dy + n) & (n - 1);
    for (int dx = -R; dx <= R; ++dx) {
      const int sc = (ic - dx + n) & (n - 1);
      const int64_t s = static_cast<int64_t>(sr) * n + sc;
      const double w = psf_unnormalised(P, s, dy, dx);
      if (w != 0.0) acc += (w / P.Z[s]) * static_cast<double>(u[s]);
    }
  }
  out[i] = static_cast<float>(acc);
}

}  // namespace

PsfField::~PsfField() {}

void PsfField::upload(const wdb_psf_field* f, hipStream_t s) {
  WDB_REQUIRE(f, WDB_ERR_ARG, "null PSF field");
  WDB_REQUIRE(f->sig_major && f->sig_minor && f->angle, WDB_ERR_ARG, "null PSF field array");
  const int n = f->n;
  WDB_REQUIRE(n >= 2 && (n & (n - 1)) == 0 && n <= (1 << 14), WDB_ERR_SIZE,
              "image side %d is not a power of two in [2, 16384]", n);
  WDB_REQUIRE(std::isfinite(f->trunc) && f->trunc > 0, WDB_ERR_ARG, "trunc must be positive and finite");
  const int64_t N = static_cast<int64_t>(n) * n;
  std::vector<double> c(N), sn(N);
  double smax = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    const double a = f->sig_major[i], b = f->sig_minor[i], ang = f->angle[i];
    WDB_REQUIRE(std::isfinite(a) && std::isfinite(b) && std::isfinite(ang), WDB_ERR_NONFINITE,
                "non-finite PSF parameter at source %lld", static_cast<long long>(i));
    WDB_REQUIRE(a > 0 && b > 0, WDB_ERR_ARG, "PSF sigmas must be positive (source %lld)",
                static_cast<long long>(i));
    c[i] = std::cos(ang);
    sn[i] = std::sin(ang);
    smax = std::max(smax, std::max(a, b));
  }
  const double Rd = std::floor(f->trunc * smax);
  WDB_REQUIRE(2.0 * Rd + 1.0 <= n, WDB_ERR_SIZE,
              "PSF support (radius %.0f) wraps around an image of side %d", Rd, n);
  R = static_cast<int>(Rd);
  this->n = n;
  trunc = f->trunc;
  sM.alloc(N); sm.alloc(N); cs.alloc(N); sn_.alloc(N); Z.alloc(N);
  WDB_HIP(hipMemcpyAsync(sM.p, f->sig_major, N * sizeof(double), hipMemcpyHostToDevice, s));
  WDB_HIP(hipMemcpyAsync(sm.p, f->sig_minor, N * sizeof(double), hipMemcpyHostToDevice, s));
  WDB_HIP(hipMemcpyAsync(cs.p, c.data(), N * sizeof(double), hipMemcpyHostToDevice, s));
  WDB_HIP(hipMemcpyAsync(sn_.p, sn.data(), N * sizeof(double), hipMemcpyHostToDevice, s));
  const PsfDev P = dev();
  hipLaunchKernelGGL(k_psf_norm, dim3((N + 255) / 256), dim3(256), 0, s, P, Z.p);
  WDB_HIP(hipGetLastError());
  // host vectors must outlive the async copies
  WDB_HIP(hipStreamSynchronize(s));
}

PsfDev PsfField::dev() const {
  PsfDev P;
  P.n = n;
  P.R = R;
  P.trunc = trunc;
  P.T2 = trunc * trunc;
  P.sM = sM.p;
  P.sm = sm.p;
  P.c = cs.p;
  P.s = sn_.p;
  P.Z = Z.p;
  return P;
}

}  // namespace wdb

extern "C" wdb_status wdb_blur(const wdb_psf_field* field, const float* u, float* out, void* stream) {
  WDB_API_BEGIN
  WDB_REQUIRE(u && out, WDB_ERR_ARG, "null buffer");
  WDB_REQUIRE(u != out, WDB_ERR_ARG, "u and out must not alias");
  hipStream_t s = static_cast<hipStream_t>(stream);
  wdb::PsfField F;
  F.upload(field, s);
  const int64_t N = static_cast<int64_t>(F.n) * F.n;
  hipLaunchKernelGGL(wdb::k_blur, dim3((N + 255) / 256), dim3(256), 0, s, F.dev(), u, out);
  WDB_HIP(hipGetLastError());
  WDB_HIP(hipStreamSynchronize(s));
  WDB_API_END
}
