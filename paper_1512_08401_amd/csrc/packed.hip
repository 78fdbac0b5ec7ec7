// Packed 16-bit storage of Theta_K and Theta_K^T for the mixed-precision
// iteration: one 32-bit word per kept entry, the 16-bit value in the high
// half and a 16-bit band-relative column code in the low half (4 bytes per
// entry instead of 8 for float32 values and int32 columns).
//
// Values.  As in the slot form: the float32 value times the power of two u of
// its scale block (row subband for Theta_K, column subband for Theta_K^T),
// rounded to binary16 or bfloat16.
//
// Column code: the band-relative 16-bit code of codes.hpp.  The kernels keep
// the row's two centre numerators in registers and decode each word with
// integer shifts, adds and masks.  Entries whose column does not fit the code
// are kept per row in an escape list (16-bit value, int32 column) read after
// the packed words.
//
// Rows are padded to whole groups of 4 words (value 0).  Kernels: G lanes per
// row; each lane loads two 16-byte groups of 4 words per step before its
// gathers, float32 accumulation in a fixed order, butterfly reduction inside
// the group.
#include <algorithm>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "codes.hpp"
#include "common.hpp"

namespace wdb {

namespace {

constexpr int kBlock = 256;
__device__ __forceinline__ uint16_t q_bf16(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(b >> 16);
}

__device__ __forceinline__ uint16_t q_f16(float f) {
  const _Float16 h = static_cast<_Float16>(f);
  return __builtin_bit_cast(uint16_t, h);
}

template <int FMT>
__device__ __forceinline__ float dq(uint32_t h) {
  if constexpr (FMT == WDB_VAL_BF16) return __uint_as_float(h << 16);
  else return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(h)));
}

// ---------------------------------------------------------------------------
// Encoding (one thread per row) from the padded float32 CSR copy; entries
// whose value is 0 (the copy's padding) are dropped.
// ---------------------------------------------------------------------------
__global__ void k_count(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                        const float* __restrict__ val, int64_t nrows, Geo g, int32_t* __restrict__ npk,
                        int32_t* __restrict__ nesc) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (row >= nrows) return;
  const Pos p = pos_of(g, row);
  int a = 0, e = 0;
  for (int64_t k = rp[row]; k < rp[row + 1]; ++k) {
    if (val[k] == 0.0f) continue;
    if (encode_col(g, p, col[k]) >= 0) ++a;
    else ++e;
  }
  npk[row] = a;
  nesc[row] = e;
}

// by_col = 0: the scale block is the row's subband (Theta_K); 1: the column's (Theta_K^T).
__global__ void k_encode(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                         const float* __restrict__ val, int64_t nrows, Geo g, const int2* __restrict__ meta,
                         const float* __restrict__ ub, int by_col, int fmt, uint32_t* __restrict__ word,
                         uint16_t* __restrict__ ev, int32_t* __restrict__ ec) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (row >= nrows) return;
  const Pos p = pos_of(g, row);
  const float urow = ub[band_index(g, p.level, p.orient)];
  int64_t wk = meta[row].x, ek = meta[row].y;
  for (int64_t k = rp[row]; k < rp[row + 1]; ++k) {
    if (val[k] == 0.0f) continue;
    const int64_t c = col[k];
    float u = urow;
    if (by_col) {
      const Pos q = pos_of(g, c);
      u = ub[band_index(g, q.level, q.orient)];
    }
    const float sv = val[k] * u;  // exact: u is a power of two
    const uint16_t h = fmt == WDB_VAL_BF16 ? q_bf16(sv) : q_f16(sv);
    const int code = encode_col(g, p, c);
    if (code >= 0) {
      word[wk++] = (static_cast<uint32_t>(h) << 16) | static_cast<uint32_t>(code);
    } else {
      ev[ek] = h;
      ec[ek++] = static_cast<int32_t>(c);
    }
  }
  for (; wk < meta[row + 1].x; ++wk) word[wk] = kPadCode;  // row padding: value 0
}

// ---------------------------------------------------------------------------
// Products.
// ---------------------------------------------------------------------------
struct PackedView {
  const int2* __restrict__ meta;
  const uint32_t* __restrict__ word;
  const uint16_t* __restrict__ ev;
  const int32_t* __restrict__ ec;
  int64_t nrows;
};

PackedView pview(const Packed& m) { return PackedView{m.meta, m.word, m.ev, m.ec, m.nrows}; }

template <int G, int FMT>
__device__ __forceinline__ float packed_dot(const PackedView& P, const Geo& g, int64_t row, int gl,
                                            const float* __restrict__ x) {
  constexpr int U = 2;
  float acc = 0.f;
  if (row < P.nrows) {
    const RowCode rc = row_code(g, pos_of(g, row));
    const int2 m0 = P.meta[row], m1 = P.meta[row + 1];
    const uint4* __restrict__ w4 = reinterpret_cast<const uint4*>(P.word);
    const int end = m1.x >> 2;
    for (int k = (m0.x >> 2) + gl; k < end; k += G * U) {
      uint4 e[U];
#pragma unroll
      for (int t = 0; t < U; ++t) e[t] = k + t * G < end ? w4[k + t * G] : make_uint4(kPadCode, kPadCode, kPadCode, kPadCode);
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const uint32_t q[4] = {e[t].x, e[t].y, e[t].z, e[t].w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          acc = fmaf(dq<FMT>(q[u] >> 16), x[decode_col(g, rc, q[u])], acc);
        }
      }
    }
    for (int k = m0.y + gl; k < m1.y; k += G) acc = fmaf(dq<FMT>(P.ev[k]), x[P.ec[k]], acc);
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
  return acc;
}

// r = w * (Q y) - b; stores w * r when scale_out (the input of the transposed kernel).
template <int G, int FMT>
__global__ __launch_bounds__(kBlock) void k_res_pk(PackedView P, Geo g, const float* __restrict__ wrow,
                                                   const float* __restrict__ y, const float* __restrict__ b,
                                                   float* __restrict__ r, int* __restrict__ kdev, int scale_out) {
  if (kdev && blockIdx.x == 0 && threadIdx.x == 0) *kdev += 1;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / G) + threadIdx.x / G;
  const int gl = threadIdx.x % G;
  const float acc = packed_dot<G, FMT>(P, g, row, gl, y);
  if (gl != 0 || row >= P.nrows) return;
  const float w = wrow[row];
  const float rr = b ? w * acc - b[row] : w * acc;
  r[row] = scale_out ? rr * w : rr;
}

// g = Q^T (w r); x_k = S(y - tau g / P); y = x_k + beta_k (x_k - x_{k-1}).
template <int G, int FMT, bool PRE>
__global__ __launch_bounds__(kBlock) void k_prox_pk(PackedView P, Geo g, const float* __restrict__ rs,
                                                    float* __restrict__ x, float* __restrict__ y, float tau,
                                                    float thr, const int* __restrict__ kdev,
                                                    const float* __restrict__ pinv, const float* __restrict__ tw) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / G) + threadIdx.x / G;
  const int gl = threadIdx.x % G;
  const float gr = packed_dot<G, FMT>(P, g, row, gl, rs);
  if (gl != 0 || row >= P.nrows) return;
  float beta = 0.0f;  // no counter: no extrapolation (ISTA)
  if (kdev) {
    const int k = *kdev;
    beta = static_cast<float>((static_cast<double>(k) - 1.0) / (static_cast<double>(k) + 2.0));
  }
  const float pi = PRE ? pinv[row] : 1.0f;
  const float z = y[row] - (tau * pi) * gr;
  const float t = thr * (tw ? tw[row] : pi);
  const float xn = copysignf(fmaxf(fabsf(z) - t, 0.0f), z);
  const float xo = x[row];
  x[row] = xn;
  y[row] = xn + beta * (xn - xo);
}


dim3 row_grid(int64_t nrows, int G) { return dim3(static_cast<unsigned>((nrows + kBlock / G - 1) / (kBlock / G))); }

template <typename F>
void with_group16(int G, F&& f) {
  switch (G) {
    case 2: f(std::integral_constant<int, 2>{}); return;
    case 4: f(std::integral_constant<int, 4>{}); return;
    case 8: f(std::integral_constant<int, 8>{}); return;
    case 16: f(std::integral_constant<int, 16>{}); return;
    default: fail(WDB_ERR_ARG, "unsupported lanes per row %d for the packed 16-bit kernels", G);
  }
}

void encode_one(const wdb_theta* th, const Csr32& src, const float* ub, int by_col, int fmt, Packed* out,
                hipStream_t s) {
  const Geo g = geo_of(th);
  const int64_t nrows = src.nrows;
  DevBuf<int32_t> npk(std::max<int64_t>(nrows, 1)), nesc(std::max<int64_t>(nrows, 1));
  const dim3 grid(static_cast<unsigned>((nrows + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_count, grid, dim3(kBlock), 0, s, src.rowptr, src.col, src.val, nrows, g, npk.p, nesc.p);
  WDB_HIP(hipGetLastError());
  std::vector<int32_t> ha(nrows), he(nrows);
  WDB_HIP(hipMemcpyAsync(ha.data(), npk.p, nrows * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  WDB_HIP(hipMemcpyAsync(he.data(), nesc.p, nrows * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  WDB_HIP(hipStreamSynchronize(s));
  std::vector<int2> meta(nrows + 1);
  int64_t w = 0, e = 0;
  for (int64_t r = 0; r <= nrows; ++r) {
    WDB_REQUIRE(w < (int64_t{1} << 31) && e < (int64_t{1} << 31), WDB_ERR_ARG, "too many entries for the packed form");
    meta[r] = make_int2(static_cast<int>(w), static_cast<int>(e));
    if (r < nrows) {
      w += (ha[r] + 3) / 4 * 4;  // rows padded to whole 16-byte groups
      e += he[r];
    }
  }
  Packed p;
  p.nrows = nrows;
  p.nesc = e;
  p.npacked = w;
  try {
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&p.meta), (nrows + 1) * sizeof(int2)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&p.word), std::max<int64_t>(p.npacked, 4) * sizeof(uint32_t)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&p.ev), std::max<int64_t>(p.nesc, 1) * sizeof(uint16_t)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&p.ec), std::max<int64_t>(p.nesc, 1) * sizeof(int32_t)));
    WDB_HIP(hipMemcpyAsync(p.meta, meta.data(), (nrows + 1) * sizeof(int2), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_encode, grid, dim3(kBlock), 0, s, src.rowptr, src.col, src.val, nrows, g, p.meta, ub, by_col,
                       fmt, p.word, p.ev, p.ec);
    WDB_HIP(hipGetLastError());
    WDB_HIP(hipStreamSynchronize(s));
  } catch (...) {
    p.free_all();
    throw;
  }
  out->free_all();
  *out = p;
}

}  // namespace

void Packed::free_all() {
  if (meta) (void)hipFree(meta);
  if (word) (void)hipFree(word);
  if (ev) (void)hipFree(ev);
  if (ec) (void)hipFree(ec);
  meta = nullptr;
  word = nullptr;
  ev = nullptr;
  ec = nullptr;
  nrows = npacked = nesc = 0;
}

bool packed_supported(const wdb_theta* th) {
  return th->n >= 2 && (th->n & (th->n - 1)) == 0 && th->n <= (1 << 14);
}

void build_packed(wdb_theta* th, const float* ub, int fmt, hipStream_t s) {
  encode_one(th, th->cA, ub, 0, fmt, &th->pA, s);
  encode_one(th, th->cAt, ub, 1, fmt, &th->pAt, s);
}

// Lanes per row of the packed kernels: the handle's choice, else WDB_Q_GROUP
// (0 selects the slot-layout 16-bit kernels instead), else 4.
int packed_group(const wdb_theta* th) {
  if (th->q_group > 0) return th->q_group;
  if (const char* e = std::getenv("WDB_Q_GROUP")) {
    const int G = std::atoi(e);
    if (G == 0 || G == 2 || G == 4 || G == 8 || G == 16) return G;
  }
  return 4;
}

void launch_res_packed(const wdb_theta* th, int G, const float* y, const float* b, float* r, int* kdev, int scale_out,
                       hipStream_t s) {
  const PackedView P = pview(th->pA);
  const Geo g = geo_of(th);
  with_group16(G, [&](auto gg) {
    constexpr int GG = decltype(gg)::value;
    if (th->valtype == WDB_VAL_BF16)
      hipLaunchKernelGGL((k_res_pk<GG, WDB_VAL_BF16>), row_grid(P.nrows, GG), dim3(kBlock), 0, s, P, g, th->wrow, y,
                         b, r, kdev, scale_out);
    else
      hipLaunchKernelGGL((k_res_pk<GG, WDB_VAL_F16>), row_grid(P.nrows, GG), dim3(kBlock), 0, s, P, g, th->wrow, y,
                         b, r, kdev, scale_out);
  });
}

void launch_prox_packed(const wdb_theta* th, int G, const float* rs, float* x, float* y, float tau, float thr,
                        const int* kdev, const float* pinv, const float* tw, hipStream_t s) {
  const PackedView P = pview(th->pAt);
  const Geo g = geo_of(th);
  with_group16(G, [&](auto gg) {
    constexpr int GG = decltype(gg)::value;
    const dim3 grid = row_grid(P.nrows, GG);
    if (th->valtype == WDB_VAL_BF16) {
      if (pinv)
        hipLaunchKernelGGL((k_prox_pk<GG, WDB_VAL_BF16, true>), grid, dim3(kBlock), 0, s, P, g, rs, x, y, tau, thr,
                           kdev, pinv, tw);
      else
        hipLaunchKernelGGL((k_prox_pk<GG, WDB_VAL_BF16, false>), grid, dim3(kBlock), 0, s, P, g, rs, x, y, tau, thr,
                           kdev, pinv, tw);
    } else {
      if (pinv)
        hipLaunchKernelGGL((k_prox_pk<GG, WDB_VAL_F16, true>), grid, dim3(kBlock), 0, s, P, g, rs, x, y, tau, thr,
                           kdev, pinv, tw);
      else
        hipLaunchKernelGGL((k_prox_pk<GG, WDB_VAL_F16, false>), grid, dim3(kBlock), 0, s, P, g, rs, x, y, tau, thr,
                           kdev, pinv, tw);
    }
  });
}

}  // namespace wdb

extern "C" wdb_status wdb_set_packed_group(wdb_theta* th, int32_t group) {
  WDB_API_BEGIN
  WDB_REQUIRE(th, WDB_ERR_ARG, "null handle");
  wdb::drop_graph(th);  // the cached iteration graph may refer to what this call changes
  WDB_REQUIRE(group == 0 || group == 2 || group == 4 || group == 8 || group == 16 || group == wdb::kTiled, WDB_ERR_ARG,
              "lanes per row of the packed kernels must be 0, 2, 4, 8 or 16, or 3 (16-bit tiled layout)");
  if (group == wdb::kTiled) wdb::build_tiled16(th);
  th->q_group = group;
  WDB_API_END
}
