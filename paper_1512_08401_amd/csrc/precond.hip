// Diagonal preconditioners for Alg. 2 (Sec. 4.2 Jacobi, Sec. 4.3 SPAI).
//
// With M = Theta_K^T Theta_K (float32-stored values, float64 arithmetic):
//   M_ii   = ||Theta_K e_i||^2          (squared norm of row i of Theta_K^T)
//   M^2_ii = ||M e_i||^2 = sum_j (sum_a Theta[a,i] Theta[a,j])^2.
// Column i of M is accumulated in a dense float64 scratch vector owned by one
// workgroup: the rows a with Theta[a,i] != 0 are visited one after another
// (columns within a row are distinct, so the scatter has no conflicts), then
// the touched entries are squared, summed and reset.  The visit order is
// fixed, so the result is deterministic.
#include <cmath>

#include "common.hpp"

namespace wdb {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_hessian_diag(const int64_t* __restrict__ soffT,
                                                         const float* __restrict__ valT,
                                                         const int32_t* __restrict__ colT,
                                                         const int32_t* __restrict__ permT, int64_t nslots,
                                                         int C, int64_t N,
                                                         const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val,
                                                         double* __restrict__ scratch, double* __restrict__ m1,
                                                         double* __restrict__ m2) {
  __shared__ double red[kBlock];
  double* acc = scratch + static_cast<size_t>(blockIdx.x) * N;
  for (int64_t q = blockIdx.x; q < nslots; q += gridDim.x) {
    const int64_t i = permT ? static_cast<int64_t>(permT[q]) : (q < N ? q : -1);
    if (i < 0) continue;  // uniform across the block
    const int64_t sl = q / C;
    const int lane = static_cast<int>(q % C);
    const int64_t base = soffT[sl];
    const int64_t w = (soffT[sl + 1] - base) / C;
    double s1 = 0.0;
    // scatter: acc += Theta[a,i] * Theta[a,:] for every a in column i
    for (int64_t k = 0; k < w; ++k) {
      const int64_t idx = sell_index(base, C, lane, k);
      const double c = static_cast<double>(valT[idx]);
      if (c == 0.0) continue;  // padding
      s1 += c * c;
      const int32_t a = colT[idx];
      for (int64_t t = rowptr[a] + threadIdx.x; t < rowptr[a + 1]; t += kBlock)
        acc[col[t]] += c * static_cast<double>(static_cast<float>(val[t]));
      __syncthreads();
    }
    // gather: sum of squares of the touched entries, resetting them
    double s2 = 0.0;
    for (int64_t k = 0; k < w; ++k) {
      const int64_t idx = sell_index(base, C, lane, k);
      if (valT[idx] == 0.0f) continue;
      const int32_t a = colT[idx];
      for (int64_t t = rowptr[a] + threadIdx.x; t < rowptr[a + 1]; t += kBlock) {
        const double v = acc[col[t]];
        if (v != 0.0) {
          s2 += v * v;
          acc[col[t]] = 0.0;
        }
      }
      __syncthreads();
    }
    red[threadIdx.x] = s2;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
      if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      m1[i] = s1;
      m2[i] = red[0];
    }
    __syncthreads();
  }
}

__global__ void k_to_float_inv(const double* __restrict__ p, float* __restrict__ pinv, double* __restrict__ dsq,
                               int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= N) return;
  pinv[i] = static_cast<float>(1.0 / p[i]);
  dsq[i] = 1.0 / sqrt(p[i]);
}

}  // namespace

}  // namespace wdb

extern "C" wdb_status wdb_set_precond(wdb_theta* th, int32_t kind, double eps, const double* start, double tol,
                                      int32_t max_iters) {
  using namespace wdb;
  WDB_API_BEGIN
  WDB_REQUIRE(th, WDB_ERR_ARG, "null handle");
  wdb::drop_graph(th);  // the cached iteration graph may refer to what this call changes
  WDB_REQUIRE(kind >= WDB_PRECOND_NONE && kind <= WDB_PRECOND_JACOBI, WDB_ERR_ARG, "unknown preconditioner %d", kind);
  WDB_HIP(hipSetDevice(th->device));
  if (kind == WDB_PRECOND_NONE) {
    th->precond = 0;
    th->Lp = 0.0;
    refresh_threshold_weights(th);
    return WDB_OK;
  }
  WDB_REQUIRE(kind != WDB_PRECOND_JACOBI || (std::isfinite(eps) && eps > 0), WDB_ERR_ARG,
              "Jacobi needs eps > 0");
  const int64_t N = th->N;
  hipStream_t s = nullptr;
  ensure_workspace(th);
  DevBuf<double> m1(N), m2(N);
  {
    const int nwg = static_cast<int>(std::min<int64_t>(N, 256));
    DevBuf<double> scratch(static_cast<size_t>(nwg) * N);
    WDB_HIP(hipMemsetAsync(scratch.p, 0, scratch.bytes(), s));
    hipLaunchKernelGGL(k_hessian_diag, dim3(nwg), dim3(kBlock), 0, s, th->At.slice_off, th->At.val, th->At.col,
                       th->At.perm, th->At.nslices * th->At.C, th->At.C, N,
                       th->csr.rowptr, th->csr.col, th->csr.val, scratch.p, m1.p, m2.p);
    WDB_HIP(hipGetLastError());
    WDB_HIP(hipStreamSynchronize(s));
  }
  std::vector<double> h1(N), h2(N), p(N, 1.0);
  WDB_HIP(hipMemcpy(h1.data(), m1.p, N * sizeof(double), hipMemcpyDeviceToHost));
  WDB_HIP(hipMemcpy(h2.data(), m2.p, N * sizeof(double), hipMemcpyDeviceToHost));
  if (kind == WDB_PRECOND_SPAI) {
    for (int64_t i = 0; i < N; ++i)
      if (h1[i] != 0.0) p[i] = h2[i] / h1[i];
  } else if (kind == WDB_PRECOND_JACOBI) {
    for (int64_t i = 0; i < N; ++i) p[i] = std::max(h1[i], eps);
  } else {
    // one group per scale: A_J, then the three detail subbands of each level
    const std::vector<Subband> lay = layout(th->n, th->levels);
    std::vector<int> grp(lay.size());
    int ng = 0;
    for (size_t k = 0; k < lay.size(); ++k) {
      if (k == 0) grp[k] = ng++;
      else if (lay[k].erow == 0 && lay[k].ecol == 1) grp[k] = ng++;
      else grp[k] = ng - 1;
    }
    std::vector<double> s1(ng, 0.0), s2(ng, 0.0);
    for (size_t k = 0; k < lay.size(); ++k) {
      const int64_t beg = lay[k].offset, end = beg + int64_t(lay[k].side) * lay[k].side;
      for (int64_t i = beg; i < end; ++i) {
        s1[grp[k]] += h1[i];
        s2[grp[k]] += h2[i];
      }
    }
    for (size_t k = 0; k < lay.size(); ++k) {
      const double pv = s1[grp[k]] != 0.0 ? s2[grp[k]] / s1[grp[k]] : 1.0;
      const int64_t beg = lay[k].offset, end = beg + int64_t(lay[k].side) * lay[k].side;
      for (int64_t i = beg; i < end; ++i) p[i] = pv;
    }
  }
  if (!th->p64) WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->p64), N * sizeof(double)));
  if (!th->pinv) WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->pinv), N * sizeof(float)));
  DevBuf<double> dsq(N);
  WDB_HIP(hipMemcpy(th->p64, p.data(), N * sizeof(double), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_to_float_inv, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, th->p64, th->pinv, dsq.p, N);
  WDB_HIP(hipGetLastError());
  const LanczosResult r = lanczos_max(th, start, dsq.p, tol, max_iters, s);
  th->Lp = r.theta + r.resid;
  th->precond = kind;
  refresh_threshold_weights(th);
  WDB_API_END
}

extern "C" wdb_status wdb_get_precond(const wdb_theta* th, double* p_out) {
  WDB_API_BEGIN
  WDB_REQUIRE(th && p_out, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(th->precond != 0 && th->p64, WDB_ERR_ARG, "no preconditioner set");
  WDB_HIP(hipSetDevice(th->device));
  WDB_HIP(hipMemcpy(p_out, th->p64, th->N * sizeof(double), hipMemcpyDeviceToHost));
  WDB_API_END
}
