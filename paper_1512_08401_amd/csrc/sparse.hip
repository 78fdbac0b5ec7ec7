// Sparse storage of Theta_K: device CSR (float64, for export and
// construction) and the sliced-ELL copies of Theta_K and Theta_K^T that the
// solver streams (see common.hpp for the layout).
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace wdb {

namespace {

int bits_for(uint64_t v) {
  int b = 1;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

__global__ void k_make_keys(const int32_t* __restrict__ row, const int32_t* __restrict__ col, int64_t nnz,
                            int64_t N, uint64_t* __restrict__ key) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < nnz) key[i] = static_cast<uint64_t>(row[i]) * static_cast<uint64_t>(N) + static_cast<uint64_t>(col[i]);
}

// rowptr[r] = first position whose key >= r * N (keys sorted ascending).
__global__ void k_rowptr(const uint64_t* __restrict__ key, int64_t nnz, int64_t N, int64_t* __restrict__ rowptr) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r > N) return;
  const uint64_t target = static_cast<uint64_t>(r) * static_cast<uint64_t>(N);
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  rowptr[r] = lo;
}

__global__ void k_split_keys(const uint64_t* __restrict__ key, int64_t nnz, int64_t N, int32_t* __restrict__ col,
                             int* __restrict__ dup) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  col[i] = static_cast<int32_t>(key[i] % static_cast<uint64_t>(N));
  if (i > 0 && key[i] == key[i - 1]) atomicOr(dup, 1);
}

__global__ void k_expand_rows(const int64_t* __restrict__ rowptr, int64_t N, int32_t* __restrict__ row) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= N) return;
  for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) row[k] = static_cast<int32_t>(r);
}

__global__ void k_slice_width(const int64_t* __restrict__ rowptr, int64_t N, int64_t nslices,
                              int64_t* __restrict__ width) {
  const int64_t sl = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (sl >= nslices) return;
  int64_t w = 0;
  for (int l = 0; l < kSlice; ++l) {
    const int64_t r = sl * kSlice + l;
    if (r < N) w = max(w, rowptr[r + 1] - rowptr[r]);
  }
  width[sl] = (w + 3) & ~int64_t(3);
}

__global__ void k_fill_sell(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ ccol,
                            const double* __restrict__ cval, int64_t N, int64_t nslices,
                            const int64_t* __restrict__ soff, float* __restrict__ val, int32_t* __restrict__ col) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nslices * kSlice) return;
  const int64_t sl = r / kSlice;
  const int lane = static_cast<int>(r % kSlice);
  const int64_t base = soff[sl];
  const int64_t w = (soff[sl + 1] - base) / kSlice;
  int64_t beg = 0, len = 0;
  if (r < N) {
    beg = rowptr[r];
    len = rowptr[r + 1] - beg;
  }
  const int32_t pad_col = len ? ccol[beg + len - 1] : static_cast<int32_t>(r < N ? r : 0);
  for (int64_t k = 0; k < w; ++k) {
    const int64_t idx = base + (k >> 2) * (4 * kSlice) + lane * 4 + (k & 3);
    if (k < len) {
      val[idx] = static_cast<float>(cval[beg + k]);
      col[idx] = ccol[beg + k];
    } else {
      val[idx] = 0.0f;
      col[idx] = pad_col;
    }
  }
}

inline dim3 blocks_for(int64_t n, int b = 256) { return dim3(static_cast<unsigned>((n + b - 1) / b)); }

}  // namespace

void coo_to_csr(int64_t nrows, int64_t nnz, const int32_t* row, const int32_t* col, const double* val, Csr* out,
                hipStream_t s) {
  Csr c;
  c.nrows = nrows;
  c.nnz = nnz;
  DevBuf<int64_t> rowptr(nrows + 1);
  DevBuf<int32_t> ocol(nnz);
  DevBuf<double> oval(nnz);
  if (nnz > 0) {
    DevBuf<uint64_t> k_in(nnz), k_out(nnz);
    hipLaunchKernelGGL(k_make_keys, blocks_for(nnz), dim3(256), 0, s, row, col, nnz, nrows, k_in.p);
    WDB_HIP(hipGetLastError());
    const int end_bit = bits_for(static_cast<uint64_t>(nrows) * static_cast<uint64_t>(nrows));
    size_t tmp_bytes = 0;
    WDB_HIP(rocprim::radix_sort_pairs(nullptr, tmp_bytes, k_in.p, k_out.p, val, oval.p,
                                      static_cast<size_t>(nnz), 0, end_bit, s));
    DevBuf<char> tmp(tmp_bytes);
    WDB_HIP(rocprim::radix_sort_pairs(tmp.p, tmp_bytes, k_in.p, k_out.p, val, oval.p,
                                      static_cast<size_t>(nnz), 0, end_bit, s));
    DevBuf<int> dup(1);
    WDB_HIP(hipMemsetAsync(dup.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_split_keys, blocks_for(nnz), dim3(256), 0, s, k_out.p, nnz, nrows, ocol.p, dup.p);
    hipLaunchKernelGGL(k_rowptr, blocks_for(nrows + 1), dim3(256), 0, s, k_out.p, nnz, nrows, rowptr.p);
    WDB_HIP(hipGetLastError());
    int d = 0;
    WDB_HIP(hipMemcpyAsync(&d, dup.p, sizeof(int), hipMemcpyDeviceToHost, s));
    WDB_HIP(hipStreamSynchronize(s));
    WDB_REQUIRE(d == 0, WDB_ERR_FORMAT, "duplicate (row, col) entries");
  } else {
    WDB_HIP(hipMemsetAsync(rowptr.p, 0, (nrows + 1) * sizeof(int64_t), s));
    WDB_HIP(hipStreamSynchronize(s));
  }
  out->free_all();
  c.rowptr = rowptr.release();
  c.col = ocol.release();
  c.val = oval.release();
  *out = c;
}

void csr_transpose(const Csr& a, Csr* out, hipStream_t s) {
  DevBuf<int32_t> rows(a.nnz);
  if (a.nnz) {
    hipLaunchKernelGGL(k_expand_rows, blocks_for(a.nrows), dim3(256), 0, s, a.rowptr, a.nrows, rows.p);
    WDB_HIP(hipGetLastError());
  }
  // transposed entry (col, row)
  coo_to_csr(a.nrows, a.nnz, a.col, rows.p, a.val, out, s);
}

void csr_to_sell(const Csr& a, Sell* out, hipStream_t s) {
  Sell m;
  m.nrows = a.nrows;
  m.nslices = (a.nrows + kSlice - 1) / kSlice;
  DevBuf<int64_t> width(m.nslices);
  hipLaunchKernelGGL(k_slice_width, blocks_for(m.nslices), dim3(256), 0, s, a.rowptr, a.nrows, m.nslices, width.p);
  WDB_HIP(hipGetLastError());
  std::vector<int64_t> w(m.nslices), off(m.nslices + 1, 0);
  WDB_HIP(hipMemcpyAsync(w.data(), width.p, m.nslices * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  WDB_HIP(hipStreamSynchronize(s));
  for (int64_t i = 0; i < m.nslices; ++i) off[i + 1] = off[i] + w[i] * kSlice;
  m.stored = off[m.nslices];
  DevBuf<int64_t> soff(m.nslices + 1);
  DevBuf<float> val(std::max<int64_t>(m.stored, 4));
  DevBuf<int32_t> col(std::max<int64_t>(m.stored, 4));
  WDB_HIP(hipMemcpyAsync(soff.p, off.data(), (m.nslices + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_fill_sell, blocks_for(m.nslices * kSlice), dim3(256), 0, s, a.rowptr, a.col, a.val, a.nrows,
                     m.nslices, soff.p, val.p, col.p);
  WDB_HIP(hipGetLastError());
  WDB_HIP(hipStreamSynchronize(s));
  out->free_all();
  m.slice_off = soff.release();
  m.val = val.release();
  m.col = col.release();
  *out = m;
}

void finish_theta(wdb_theta* th, hipStream_t s) {
  csr_to_sell(th->csr, &th->A, s);
  Csr t;
  try {
    csr_transpose(th->csr, &t, s);
    csr_to_sell(t, &th->At, s);
  } catch (...) {
    t.free_all();
    throw;
  }
  t.free_all();
}

}  // namespace wdb

extern "C" wdb_status wdb_theta_import(int32_t n, int32_t wavelet, int32_t levels, int64_t nnz,
                                       const int64_t* rowptr, const int32_t* col, const double* val, void* stream,
                                       wdb_theta** out) {
  using namespace wdb;
  WDB_API_BEGIN
  WDB_REQUIRE(out && rowptr && (nnz == 0 || (col && val)), WDB_ERR_ARG, "null argument");
  const Filter f = make_filter(wavelet);
  check_geometry(n, levels, static_cast<int>(f.h.size()));
  const int64_t N = static_cast<int64_t>(n) * n;
  WDB_REQUIRE(nnz >= 0 && nnz <= N * N, WDB_ERR_FORMAT, "nnz %lld out of range", static_cast<long long>(nnz));
  WDB_REQUIRE(rowptr[0] == 0 && rowptr[N] == nnz, WDB_ERR_FORMAT, "rowptr must start at 0 and end at nnz");
  for (int64_t r = 0; r < N; ++r)
    WDB_REQUIRE(rowptr[r + 1] >= rowptr[r], WDB_ERR_FORMAT, "rowptr decreases at row %lld",
                static_cast<long long>(r));
  for (int64_t r = 0; r < N; ++r) {
    for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
      WDB_REQUIRE(col[k] >= 0 && col[k] < N, WDB_ERR_FORMAT, "column index out of range in row %lld",
                  static_cast<long long>(r));
      WDB_REQUIRE(k == rowptr[r] || col[k] > col[k - 1], WDB_ERR_FORMAT,
                  "column indices not strictly increasing in row %lld", static_cast<long long>(r));
      WDB_REQUIRE(std::isfinite(val[k]), WDB_ERR_NONFINITE, "non-finite value in row %lld",
                  static_cast<long long>(r));
    }
  }
  int dev = 0;
  WDB_HIP(hipGetDevice(&dev));
  hipStream_t s = static_cast<hipStream_t>(stream);
  wdb_theta* th = new wdb_theta();
  try {
    th->device = dev;
    th->n = n;
    th->levels = levels;
    th->wavelet = wavelet;
    th->N = N;
    th->nnz = nnz;
    DevBuf<int64_t> rp(N + 1);
    DevBuf<int32_t> cc(std::max<int64_t>(nnz, 1));
    DevBuf<double> vv(std::max<int64_t>(nnz, 1));
    WDB_HIP(hipMemcpyAsync(rp.p, rowptr, (N + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (nnz) {
      WDB_HIP(hipMemcpyAsync(cc.p, col, nnz * sizeof(int32_t), hipMemcpyHostToDevice, s));
      WDB_HIP(hipMemcpyAsync(vv.p, val, nnz * sizeof(double), hipMemcpyHostToDevice, s));
    }
    WDB_HIP(hipStreamSynchronize(s));
    th->csr.nrows = N;
    th->csr.nnz = nnz;
    th->csr.rowptr = rp.release();
    th->csr.col = cc.release();
    th->csr.val = vv.release();
    finish_theta(th, s);
  } catch (...) {
    wdb_theta_free(th);
    throw;
  }
  *out = th;
  WDB_API_END
}
