// Sparse storage of Theta_K: device CSR (float64, for export and
// construction) and the sliced-ELL copies of Theta_K and Theta_K^T that the
// solver streams (see common.hpp for the layout).
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>
#include <cstdlib>

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

__global__ void k_row_lengths(const int64_t* __restrict__ rowptr, int64_t N, int32_t* __restrict__ len) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r < N) len[r] = static_cast<int32_t>(rowptr[r + 1] - rowptr[r]);
}

// One thread per slot row q: copies matrix row perm[q] (or q) into the slice.
__global__ void k_fill_sell(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ ccol,
                            const double* __restrict__ cval, int64_t N, int64_t nslices, int C,
                            const int64_t* __restrict__ soff, const int32_t* __restrict__ perm,
                            float* __restrict__ val, int32_t* __restrict__ col) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nslices * C) return;
  const int64_t sl = q / C;
  const int lane = static_cast<int>(q % C);
  const int64_t base = soff[sl];
  const int64_t w = (soff[sl + 1] - base) / C;
  const int64_t r = perm ? static_cast<int64_t>(perm[q]) : (q < N ? q : -1);
  int64_t beg = 0, len = 0;
  if (r >= 0) {
    beg = rowptr[r];
    len = rowptr[r + 1] - beg;
  }
  const int32_t pad_col = len ? ccol[beg + len - 1] : static_cast<int32_t>(r >= 0 ? r : 0);
  for (int64_t k = 0; k < w; ++k) {
    const int64_t idx = sell_index(base, C, lane, k);
    if (k < len) {
      val[idx] = static_cast<float>(cval[beg + k]);
      col[idx] = ccol[beg + k];
    } else {
      val[idx] = 0.0f;
      col[idx] = pad_col;
    }
  }
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = static_cast<float>(a[i]);
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

void csr_to_sell(const Csr& a, Sell* out, hipStream_t s, int64_t sort_window, int C) {
  WDB_REQUIRE(C >= 1 && C <= kSliceMax && (C & (C - 1)) == 0, WDB_ERR_ARG, "slice height %d is not a power of two <= %d",
              C, kSliceMax);
  Sell m;
  m.C = C;
  m.nrows = a.nrows;
  m.nslices = (a.nrows + C - 1) / C;
  const int64_t slots = m.nslices * C;
  std::vector<int32_t> len(a.nrows);
  if (a.nrows) {
    DevBuf<int32_t> dlen(a.nrows);
    hipLaunchKernelGGL(k_row_lengths, blocks_for(a.nrows), dim3(256), 0, s, a.rowptr, a.nrows, dlen.p);
    WDB_HIP(hipGetLastError());
    WDB_HIP(hipMemcpyAsync(len.data(), dlen.p, a.nrows * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    WDB_HIP(hipStreamSynchronize(s));
  }
  // slot row -> matrix row: identity, or sorted by decreasing length inside
  // windows of sort_window rows (stable, so equal lengths keep their order)
  std::vector<int32_t> perm;
  const bool sorted = sort_window > C;
  if (sorted) {
    const int64_t W = (sort_window + C - 1) / C * C;
    perm.assign(slots, -1);
    std::vector<int32_t> idx;
    for (int64_t w0 = 0; w0 < a.nrows; w0 += W) {
      const int64_t w1 = std::min(a.nrows, w0 + W);
      idx.resize(w1 - w0);
      for (int64_t r = w0; r < w1; ++r) idx[r - w0] = static_cast<int32_t>(r);
      std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return len[x] > len[y]; });
      for (int64_t t = 0; t < w1 - w0; ++t) perm[w0 + t] = idx[t];
    }
  }
  std::vector<int64_t> off(m.nslices + 1, 0);
  for (int64_t sl = 0; sl < m.nslices; ++sl) {
    int64_t w = 0;
    for (int l = 0; l < C; ++l) {
      const int64_t q = sl * C + l;
      const int64_t r = sorted ? perm[q] : (q < a.nrows ? q : -1);
      if (r >= 0) w = std::max<int64_t>(w, len[r]);
    }
    off[sl + 1] = off[sl] + ((w + 3) & ~int64_t(3)) * C;
  }
  m.stored = off[m.nslices];
  DevBuf<int64_t> soff(m.nslices + 1);
  DevBuf<int32_t> dperm(sorted ? slots : 0);
  DevBuf<float> val(std::max<int64_t>(m.stored, 4));
  DevBuf<int32_t> col(std::max<int64_t>(m.stored, 4));
  WDB_HIP(hipMemcpyAsync(soff.p, off.data(), (m.nslices + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  if (sorted) WDB_HIP(hipMemcpyAsync(dperm.p, perm.data(), slots * sizeof(int32_t), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_fill_sell, blocks_for(slots), dim3(256), 0, s, a.rowptr, a.col, a.val, a.nrows, m.nslices, C,
                     soff.p, sorted ? dperm.p : static_cast<const int32_t*>(nullptr), val.p, col.p);
  WDB_HIP(hipGetLastError());
  WDB_HIP(hipStreamSynchronize(s));
  out->free_all();
  m.slice_off = soff.release();
  m.val = val.release();
  m.col = col.release();
  m.perm = sorted ? dperm.release() : nullptr;
  *out = m;
}

// Row r's entries go to [rowptr[r], rowptr[r] + len) and the rest of its
// padded range (a multiple of 4) holds value 0 with column r.
__global__ void k_fill_padded(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                              const double* __restrict__ val, const int64_t* __restrict__ prp, int64_t nrows,
                              int32_t* __restrict__ pcol, float* __restrict__ pval) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (row >= nrows) return;
  const int64_t b = rp[row], len = rp[row + 1] - b, d = prp[row], plen = prp[row + 1] - d;
  for (int64_t k = 0; k < plen; ++k) {
    pcol[d + k] = k < len ? col[b + k] : static_cast<int32_t>(row);
    pval[d + k] = k < len ? static_cast<float>(val[b + k]) : 0.0f;
  }
}

void csr_to_csr32(const Csr& a, Csr32* out, hipStream_t s) {
  Csr32 c;
  c.nrows = a.nrows;
  c.nnz = a.nnz;
  std::vector<int64_t> rp(a.nrows + 1), prp(a.nrows + 1);
  WDB_HIP(hipMemcpyAsync(rp.data(), a.rowptr, (a.nrows + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  WDB_HIP(hipStreamSynchronize(s));
  prp[0] = 0;
  for (int64_t r = 0; r < a.nrows; ++r) prp[r + 1] = prp[r] + (rp[r + 1] - rp[r] + 3) / 4 * 4;
  c.stored = prp[a.nrows];
  WDB_REQUIRE(c.stored / 4 < (int64_t{1} << 31), WDB_ERR_ARG, "operator too large for the padded CSR copy");
  DevBuf<int64_t> drp(a.nrows + 1);
  DevBuf<int32_t> col(std::max<int64_t>(c.stored, 4));
  DevBuf<float> val(std::max<int64_t>(c.stored, 4));
  WDB_HIP(hipMemcpyAsync(drp.p, prp.data(), (a.nrows + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  if (a.nrows) {
    hipLaunchKernelGGL(k_fill_padded, blocks_for(a.nrows), dim3(256), 0, s, a.rowptr, a.col, a.val, drp.p, a.nrows,
                       col.p, val.p);
    WDB_HIP(hipGetLastError());
  }
  WDB_HIP(hipStreamSynchronize(s));
  out->free_all();
  c.rowptr = drp.release();
  c.col = col.release();
  c.val = val.release();
  *out = c;
}

int default_slice_height() {
  static const int c = [] {
    const char* e = std::getenv("WDB_SLICE");
    const int v = e ? std::atoi(e) : kSliceMax;
    return (v >= 1 && v <= kSliceMax && (v & (v - 1)) == 0) ? v : kSliceMax;
  }();
  return c;
}

void set_slice_height(wdb_theta* th, int C, hipStream_t s) {
  if (th->A.val && th->A.C == C && th->At.val && th->At.C == C) return;
  csr_to_sell(th->csr, &th->A, s, sell_sort_window(), C);
  Csr t;
  try {
    csr_transpose(th->csr, &t, s);
    csr_to_sell(t, &th->At, s, sell_sort_window(), C);
  } catch (...) {
    t.free_all();
    throw;
  }
  t.free_all();
}

void finish_theta(wdb_theta* th, hipStream_t s) {
  const int C = default_slice_height();
  csr_to_sell(th->csr, &th->A, s, sell_sort_window(), C);
  csr_to_csr32(th->csr, &th->cA, s);
  Csr t;
  try {
    csr_transpose(th->csr, &t, s);
    csr_to_sell(t, &th->At, s, sell_sort_window(), C);
    csr_to_csr32(t, &th->cAt, s);
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
