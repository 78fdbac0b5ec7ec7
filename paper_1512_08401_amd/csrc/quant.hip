// 16-bit storage of Theta_K's values for the iteration (the mixed-precision
// form; the paper states no GPU precision).
//
// Each kept value v (already rounded to float32) is scaled by a power of two
// u_A that depends on its row subband A, u_A = 2^-floor(log2 max_{rows in A} |v|),
// and rounded to binary16 or bfloat16 (nearest, ties to even).  The block
// scale of block (A, B) is therefore u_A for every column subband B.  Because
// u_A is a power of two, dequantisation is exact: the residual kernel multiplies
// its row sum by w_A = 1/u_A, and writes the residual pre-multiplied by w_A so the
// transposed kernel's gathers see exactly (q / u_A) * r.  The same values are
// also stored in the packed CSR form (value and column code in one 32-bit
// word), which the iteration uses by default.
#include <cmath>
#include <cstring>

#include "common.hpp"

namespace wdb {

namespace {

constexpr int kMaxBands = 48;

struct BandTab {
  int nb;
  int64_t off[kMaxBands + 1];
};

__device__ __forceinline__ int band_of(const BandTab& T, int64_t i) {
  int k = 0;
  while (k + 1 < T.nb && i >= T.off[k + 1]) ++k;
  return k;
}

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(b >> 16);
}

__device__ __forceinline__ uint16_t to_f16(float f) {
  const _Float16 h = static_cast<_Float16>(f);
  return __builtin_bit_cast(uint16_t, h);
}

__global__ void k_band_max(const int64_t* __restrict__ soff, const float* __restrict__ val,
                           const int32_t* __restrict__ perm, int64_t nslices, int C, int64_t nrows, BandTab T,
                           unsigned* __restrict__ bmax) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nslices * C) return;
  const int64_t row = perm ? perm[q] : (q < nrows ? q : -1);
  if (row < 0) return;
  const int64_t sl = q / C;
  const int lane = static_cast<int>(q % C);
  const int64_t base = soff[sl], w = (soff[sl + 1] - base) / C;
  float m = 0.0f;
  for (int64_t k = 0; k < w; ++k) m = fmaxf(m, fabsf(val[sell_index(base, C, lane, k)]));
  if (m > 0.0f) atomicMax(&bmax[band_of(T, row)], __float_as_uint(m));
}

// by_col = 0: scale by the band of the slot's row (Theta_K); 1: of its column (Theta_K^T).
__global__ void k_quantize(const int64_t* __restrict__ soff, const float* __restrict__ val,
                           const int32_t* __restrict__ col, const int32_t* __restrict__ perm, int64_t nslices,
                           int C, int64_t nrows, BandTab T, const float* __restrict__ ub, int by_col, int fmt,
                           uint16_t* __restrict__ out) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nslices * C) return;
  const int64_t row = perm ? perm[q] : (q < nrows ? q : -1);
  const int64_t sl = q / C;
  const int lane = static_cast<int>(q % C);
  const int64_t base = soff[sl], w = (soff[sl + 1] - base) / C;
  const float urow = row >= 0 ? ub[band_of(T, row)] : 1.0f;
  for (int64_t k = 0; k < w; ++k) {
    const int64_t idx = sell_index(base, C, lane, k);
    const float u = by_col ? ub[band_of(T, col[idx])] : urow;
    const float s = val[idx] * u;  // exact: u is a power of two
    out[idx] = fmt == WDB_VAL_BF16 ? to_bf16(s) : to_f16(s);
  }
}

__global__ void k_row_factor(BandTab T, const float* __restrict__ ub, int64_t N, float* __restrict__ wrow) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < N) wrow[i] = 1.0f / ub[band_of(T, i)];
}

}  // namespace

}  // namespace wdb

extern "C" wdb_status wdb_set_precision(wdb_theta* th, int32_t valtype) {
  using namespace wdb;
  WDB_API_BEGIN
  WDB_REQUIRE(th, WDB_ERR_ARG, "null handle");
  wdb::drop_graph(th);  // the cached iteration graph may refer to what this call changes
  WDB_REQUIRE(valtype == WDB_VAL_F32 || valtype == WDB_VAL_BF16 || valtype == WDB_VAL_F16, WDB_ERR_ARG,
              "unknown value type %d", valtype);
  WDB_HIP(hipSetDevice(th->device));
  if (th->val16) (void)hipFree(th->val16);
  if (th->val16T) (void)hipFree(th->val16T);
  if (th->wrow) (void)hipFree(th->wrow);
  th->val16 = th->val16T = nullptr;
  th->wrow = nullptr;
  th->pA.free_all();
  th->pAt.free_all();
  th->qA.free_all();
  th->qAt.free_all();
  th->qscale.clear();
  th->valtype = WDB_VAL_F32;
  if (valtype == WDB_VAL_F32) return WDB_OK;
  const std::vector<Subband> lay = layout(th->n, th->levels);
  WDB_REQUIRE(static_cast<int>(lay.size()) <= kMaxBands, WDB_ERR_LEVELS, "too many subbands");
  BandTab T{};
  T.nb = static_cast<int>(lay.size());
  for (int k = 0; k < T.nb; ++k) T.off[k] = lay[k].offset;
  T.off[T.nb] = th->N;
  hipStream_t s = nullptr;
  const int64_t slotsA = th->A.nslices * th->A.C, slotsT = th->At.nslices * th->At.C;
  DevBuf<unsigned> bmax(T.nb);
  WDB_HIP(hipMemset(bmax.p, 0, T.nb * sizeof(unsigned)));
  hipLaunchKernelGGL(k_band_max, dim3((slotsA + 255) / 256), dim3(256), 0, s, th->A.slice_off, th->A.val, th->A.perm,
                     th->A.nslices, th->A.C, th->N, T, bmax.p);
  WDB_HIP(hipGetLastError());
  std::vector<unsigned> hb(T.nb);
  WDB_HIP(hipMemcpy(hb.data(), bmax.p, T.nb * sizeof(unsigned), hipMemcpyDeviceToHost));
  std::vector<float> ub(T.nb, 1.0f);
  for (int k = 0; k < T.nb; ++k) {
    float m;
    std::memcpy(&m, &hb[k], sizeof(float));
    if (m > 0.0f) {
      int e = 0;
      std::frexp(static_cast<double>(m), &e);  // m = f 2^e, f in [0.5, 1)
      ub[k] = static_cast<float>(std::ldexp(1.0, -(e - 1)));
    }
  }
  DevBuf<float> dub(T.nb);
  WDB_HIP(hipMemcpy(dub.p, ub.data(), T.nb * sizeof(float), hipMemcpyHostToDevice));
  DevBuf<uint16_t> v16(std::max<int64_t>(th->A.stored, 4)), v16T(std::max<int64_t>(th->At.stored, 4));
  DevBuf<float> wrow(th->N);
  hipLaunchKernelGGL(k_quantize, dim3((slotsA + 255) / 256), dim3(256), 0, s, th->A.slice_off, th->A.val, th->A.col,
                     th->A.perm, th->A.nslices, th->A.C, th->N, T, dub.p, 0, valtype, v16.p);
  hipLaunchKernelGGL(k_quantize, dim3((slotsT + 255) / 256), dim3(256), 0, s, th->At.slice_off, th->At.val,
                     th->At.col, th->At.perm, th->At.nslices, th->At.C, th->N, T, dub.p, 1, valtype, v16T.p);
  hipLaunchKernelGGL(k_row_factor, dim3((th->N + 255) / 256), dim3(256), 0, s, T, dub.p, th->N, wrow.p);
  WDB_HIP(hipGetLastError());
  if (packed_supported(th)) build_packed(th, dub.p, valtype, s);
  WDB_HIP(hipDeviceSynchronize());
  th->val16 = v16.release();
  th->val16T = v16T.release();
  th->wrow = wrow.release();
  th->valtype = valtype;
  th->qscale = ub;
  if (th->q_group == kTiled) build_tiled16(th);  // the 16-bit tiled layout in use: rebuild for the new values
  WDB_API_END
}
