// Device view of a Gaussian PSF field (see psf.hip for the formula).
#pragma once

#include "common.hpp"

namespace wdb {

struct PsfDev {
  int n = 0;
  int R = 0;            // largest integer offset reachable by any PSF of the field
  double trunc = 0.0;
  double T2 = 0.0;      // trunc * trunc
  const double* sM = nullptr;
  const double* sm = nullptr;
  const double* c = nullptr;   // cos(angle), from the host libm
  const double* s = nullptr;   // sin(angle)
  const double* Z = nullptr;   // per-source normalisation sum
};

// exp(-q/2) if q <= trunc^2 else 0, for source s and offset (dy, dx).
__device__ __forceinline__ double psf_unnormalised(const PsfDev& P, int64_t s, int dy, int dx) {
#pragma clang fp contract(off)
  const double c = P.c[s], sn = P.s[s], a = P.sM[s], b = P.sm[s];
  const double fx = static_cast<double>(dx), fy = static_cast<double>(dy);
  const double t1 = fx * c + fy * sn;
  const double t2 = -fx * sn + fy * c;
  const double q = t1 * t1 / (a * a) + t2 * t2 / (b * b);
  return q <= P.T2 ? exp(-0.5 * q) : 0.0;
}

// Owns the uploaded field.
struct PsfField {
  int n = 0, R = 0;
  double trunc = 0.0;
  DevBuf<double> sM, sm, cs, sn_, Z;
  ~PsfField();
  void upload(const wdb_psf_field* f, hipStream_t s);
  PsfDev dev() const;
};

}  // namespace wdb
