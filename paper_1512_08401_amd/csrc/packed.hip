// Packed 16-bit storage of Theta_K and Theta_K^T for the mixed-precision
// iteration: one 32-bit word per kept entry, the 16-bit value in the high
// half and a 16-bit band-relative column code in the low half (4 bytes per
// entry instead of 8 for float32 values and int32 columns).
//
// Values.  As in the slot form: the float32 value times the power of two u of
// its scale block (row subband for Theta_K, column subband for Theta_K^T),
// rounded to binary16 or bfloat16.
//
// Column code.  An entry theta[a, b] is only large when the supports of the
// two atoms are close in space and in scale (the decay bound of Sec. 3.2, in
// the distance between the atoms' supports and in |j - k|).  For a row
// coefficient a at level la, position (ia, ja), and a column coefficient b at
// level lb, orientation o, position (ib, jb), the code stores
//   dL = lb - la in [-3, 3], band slot q in {0 (approximation), 1, 2, 3
//   (details (0,1), (1,0), (1,1))}, and (di, dj) in [-16, 15]^2: b's position
//   minus the point of level lb whose atom is centred nearest to a's atom,
//   modulo the side s of b's subband,
// as bit fields ((dL + 3) << 13) | (q << 11) | ((di + 16) << 5) | (dj + 16).
// b's index is then q s^2 + ((ci + di) mod s) s + ((cj + dj) mod s), exact
// integer arithmetic on power-of-two sides, so the packed operator has
// exactly the columns of Theta_K.  The kernels tabulate (ci - 16, cj - 16,
// s - 1, log2 s) per row and level difference in LDS once, so a decode is one
// LDS read and a few masks and shifts.  Entries outside this range are kept
// per row in an escape list (16-bit value, int32 column) read after the
// packed words.
//
// Rows are padded to whole groups of 4 words (value 0).  Kernels: G lanes per
// row; each lane loads two 16-byte groups of 4 words per step before its
// gathers, float32 accumulation in a fixed order, butterfly reduction inside
// the group.
#include <algorithm>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace wdb {

namespace {

constexpr int kBlock = 256;
constexpr int kDOff = 16;  // displacements in [-16, 15]
constexpr int kLMax = 3;
// Padding word of a partial step: value 0, column = a valid coefficient (a
// detail subband of the row's own level, which every level has).
constexpr uint32_t kPadCode = (static_cast<uint32_t>(kLMax) << 13) | (1u << 11) | (kDOff << 5) | kDOff;

struct Geo {
  int logn, J, L1;  // log2 of the image side, levels, filter length - 1
};

struct Pos {
  int level, orient, i, j;  // orient 0..2: details (0,1), (1,0), (1,1); 3: approximation
};

__host__ __device__ inline int floor_log2(uint64_t v) { return 63 - __builtin_clzll(v); }

// Subband position of canonical index r.  Level l details of side s = n >> l
// sit at offsets s^2, 2 s^2, 3 s^2; the approximation of side n >> J at 0.
__host__ __device__ inline Pos pos_of(const Geo& g, int64_t r) {
  const int lsJ = g.logn - g.J;
  if (r < (int64_t{1} << (2 * lsJ)))
    return Pos{g.J, 3, static_cast<int>(r >> lsJ), static_cast<int>(r & ((int64_t{1} << lsJ) - 1))};
  const int ls = floor_log2(static_cast<uint64_t>(r)) >> 1;
  const int o = static_cast<int>(r >> (2 * ls)) - 1;
  const int64_t p = r - (static_cast<int64_t>(o) + 1) * (int64_t{1} << (2 * ls));
  return Pos{g.logn - ls, o, static_cast<int>(p >> ls), static_cast<int>(p & ((int64_t{1} << ls) - 1))};
}

// Index of the subband (canonical order: approximation, then per level J..1
// the three detail orientations).
__host__ __device__ inline int band_index(const Geo& g, int level, int orient) {
  return orient == 3 ? 0 : 1 + 3 * (g.J - level) + orient;
}

// Point of level lb whose atom is centred nearest to the atom at index i of
// level la (atoms of level l at index i are centred at 2^l i + L1 (2^l - 1) / 2),
// not yet reduced modulo the side.  With P = (i << (la + 1)) + L1 2^la this is
// (P + (1 - L1) 2^lb) >> (lb + 1).
__host__ __device__ inline int centre_at(const Geo& g, int i, int la, int lb) {
  return ((i << (la + 1)) + g.L1 * ((1 << la) - (1 << lb)) + (1 << lb)) >> (lb + 1);
}

// Decode table entry of a row for one level difference: (ci - 16, cj - 16,
// s - 1, log2 s) of the column level lb (all zero when lb is not a level).
__host__ __device__ inline int4 decode_entry(const Geo& g, const Pos& p, int dL) {
  const int lb = p.level + dL;
  if (lb < 1 || lb > g.J) return make_int4(0, 0, 0, 0);
  const int ls = g.logn - lb;
  return make_int4(centre_at(g, p.i, p.level, lb) - kDOff, centre_at(g, p.j, p.level, lb) - kDOff, (1 << ls) - 1, ls);
}

__host__ __device__ inline int decode_with(const int4& t, uint32_t code) {
  const int q = static_cast<int>((code >> 11) & 3u);
  const int ib = (t.x + static_cast<int>((code >> 5) & 31u)) & t.z;
  const int jb = (t.y + static_cast<int>(code & 31u)) & t.z;
  return (q << (2 * t.w)) + (ib << t.w) + jb;
}

__host__ __device__ inline int decode_col(const Geo& g, const Pos& p, uint32_t code) {
  return decode_with(decode_entry(g, p, static_cast<int>((code >> 13) & 7u) - kLMax), code);
}

// Code of column `col` for row position p, or -1 if it does not fit.
__host__ __device__ inline int encode_col(const Geo& g, const Pos& p, int64_t col) {
  const Pos q = pos_of(g, col);
  const int dL = q.level - p.level;
  if (dL < -kLMax || dL > kLMax) return -1;
  const int ls = g.logn - q.level;
  const int s = 1 << ls, m = s - 1, h = s >> 1;
  const int di = ((q.i - centre_at(g, p.i, p.level, q.level) + h) & m) - h;
  const int dj = ((q.j - centre_at(g, p.j, p.level, q.level) + h) & m) - h;
  if (di < -kDOff || di >= kDOff || dj < -kDOff || dj >= kDOff) return -1;
  const int slot = q.orient == 3 ? 0 : q.orient + 1;
  return ((dL + kLMax) << 13) | (slot << 11) | ((di + kDOff) << 5) | (dj + kDOff);
}

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

// The G lanes of each row first fill the row's decode table (7 level
// differences) in LDS; `tab` holds kBlock / G rows of 8 entries.
template <int G>
__device__ __forceinline__ void fill_table(const Geo& g, int64_t row, int64_t nrows, int gl, int4 (*tab)[8]) {
  const int lr = threadIdx.x / G;
  if (row < nrows) {
    const Pos p = pos_of(g, row);
    for (int d = gl; d < 2 * kLMax + 1; d += G) tab[lr][d] = decode_entry(g, p, d - kLMax);
  }
  __syncthreads();
}

template <int G, int FMT>
__device__ __forceinline__ float packed_dot(const PackedView& P, int64_t row, int gl, const int4 (*tab)[8],
                                            const float* __restrict__ x) {
  constexpr int U = 2;
  float acc = 0.f;
  if (row < P.nrows) {
    const int4* __restrict__ rt = tab[threadIdx.x / G];
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
          const int4 te = rt[(q[u] >> 13) & 7u];
          acc = fmaf(dq<FMT>(q[u] >> 16), x[decode_with(te, q[u])], acc);
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
  __shared__ int4 tab[kBlock / G][8];
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / G) + threadIdx.x / G;
  const int gl = threadIdx.x % G;
  fill_table<G>(g, row, P.nrows, gl, tab);
  const float acc = packed_dot<G, FMT>(P, row, gl, tab, y);
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
  __shared__ int4 tab[kBlock / G][8];
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / G) + threadIdx.x / G;
  const int gl = threadIdx.x % G;
  fill_table<G>(g, row, P.nrows, gl, tab);
  const float gr = packed_dot<G, FMT>(P, row, gl, tab, rs);
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

Geo geo_of(const wdb_theta* th) {
  return Geo{floor_log2(static_cast<uint64_t>(th->n)), th->levels,
             static_cast<int>(make_filter(th->wavelet).h.size()) - 1};
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
  WDB_REQUIRE(group == 0 || group == 2 || group == 4 || group == 8 || group == 16, WDB_ERR_ARG,
              "lanes per row of the packed kernels must be 0, 2, 4, 8 or 16");
  th->q_group = group;
  WDB_API_END
}
