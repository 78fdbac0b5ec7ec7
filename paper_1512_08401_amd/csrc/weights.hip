// Weights w of the l1 term, G(x) = sum_i w[i] |x[i]| (Sec. 1.3).  The
// experiments of Sec. 5 use w[i] = j(i), the scale of the i-th wavelet
// coefficient (a subband of scale j has 2^j x 2^j coefficients, so j =
// log2(n) - level, the approximation taking the scale of level J).  The
// proximal kernels read w / P per row when a diagonal preconditioner is in
// use (the threshold of Alg. 2 in the P-metric), w otherwise.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace wdb {

namespace {

__global__ void k_div(const float* __restrict__ w, const float* __restrict__ pinv, float* __restrict__ out, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = w[i] * pinv[i];
}

}  // namespace

const float* threshold_weights(const wdb_theta* th, bool pre) {
  if (!th->l1w) return nullptr;
  return pre ? th->l1w_pre : th->l1w;
}

void refresh_threshold_weights(wdb_theta* th) {
  if (th->l1w_pre) (void)hipFree(th->l1w_pre);
  th->l1w_pre = nullptr;
  if (!th->l1w || !th->pinv || th->precond == 0) return;
  WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->l1w_pre), th->N * sizeof(float)));
  hipLaunchKernelGGL(k_div, dim3(static_cast<unsigned>((th->N + 255) / 256)), dim3(256), 0, nullptr, th->l1w,
                     th->pinv, th->l1w_pre, th->N);
  WDB_HIP(hipGetLastError());
  WDB_HIP(hipDeviceSynchronize());
}

}  // namespace wdb

extern "C" wdb_status wdb_set_l1_weights(wdb_theta* th, int32_t kind, const float* w) {
  using namespace wdb;
  WDB_API_BEGIN
  WDB_REQUIRE(th, WDB_ERR_ARG, "null handle");
  wdb::drop_graph(th);  // the cached iteration graph may refer to what this call changes
  WDB_REQUIRE(kind >= WDB_L1_UNIFORM && kind <= WDB_L1_GIVEN, WDB_ERR_ARG, "unknown weight kind %d", kind);
  WDB_REQUIRE(kind != WDB_L1_GIVEN || w, WDB_ERR_ARG, "weights array is null");
  WDB_HIP(hipSetDevice(th->device));
  const int64_t N = th->N;
  std::vector<float> hw;
  if (kind == WDB_L1_SCALE) {
    hw.resize(N);
    int logn = 0;
    while ((1 << logn) < th->n) ++logn;
    for (const Subband& b : layout(th->n, th->levels)) {
      const float j = static_cast<float>(logn - b.level);
      for (int64_t i = b.offset; i < b.offset + int64_t(b.side) * b.side; ++i) hw[i] = j;
    }
  } else if (kind == WDB_L1_GIVEN) {
    hw.assign(w, w + N);
  }
  for (float v : hw) WDB_REQUIRE(std::isfinite(v) && v > 0.0f, WDB_ERR_NONFINITE, "weights must be finite and > 0");
  if (th->l1w) (void)hipFree(th->l1w);
  th->l1w = nullptr;
  th->l1_kind = 0;
  if (kind != WDB_L1_UNIFORM) {
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->l1w), N * sizeof(float)));
    WDB_HIP(hipMemcpy(th->l1w, hw.data(), N * sizeof(float), hipMemcpyHostToDevice));
    th->l1_kind = kind;
  }
  refresh_threshold_weights(th);
  WDB_API_END
}
