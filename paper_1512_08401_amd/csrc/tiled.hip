// Tiled pattern storage of Theta_K and Theta_K^T for the iteration (float32
// values, or scaled 16-bit values for the mixed-precision iteration).
//
// Rows are grouped in tiles of up to 64 coefficients of one subband: an 8 x 8
// block of positions when the subband's side is at least 8, else the whole
// subband.  The blur field varies slowly in space, so neighbouring
// coefficients of one subband keep entries at nearly the same band-relative
// displacements (the codes of codes.hpp, with 8-bit displacement fields).  A
// tile stores the sorted union of its rows' codes once, and one value per
// (code, row): zero where that row did not keep the entry.  No column index
// is stored.
//
// One wavefront covers a tile's rows (lane t = row t).  For each code every
// lane decodes its own column with a few integer operations on the row's
// centre numerators, so the x loads of one instruction fall on 8 runs of 8
// consecutive coefficients (column level = row level), on repeated
// coefficients (coarser columns) or on a comb of stride 2^k (finer columns),
// instead of 64 unrelated addresses as in a row-wise CSR product.
//
// Layout per matrix: per tile an int4 {first code, end code (multiples of the
// group size), first row, log2 side | flags}; codes as uint32 in groups of 4
// (float32) or 8 (16-bit values), padded with a code of value 0; values as
// [group][lane][group size] so that a lane loads one 16-byte vector per
// group.  The float32 copies also hold the kept-value layout (codes.hpp,
// GroupRec): per group of 4 codes a record with the codes, a row mask per code
// and an offset, and only the kept values, which a lane reads from its offset
// and spreads over the 4 codes with selects on the masks; the kernels read one
// layout or the other (wdb_set_tile_values, or the autotuner's pick) and add
// the same products in the same order.  The groups of a tile are dealt
// round-robin to the W wavefronts of
// its block and the W partial sums are added in LDS in wavefront order
// (deterministic).  Entries whose code does not fit (displacement beyond 128
// or level gap beyond 3) go to per-row escape lists, whose entries are dealt
// round-robin to the wavefronts as well.  The tiles are stored and launched
// in an XCD-aware order (xcd_order): each XCD works on one horizontal stripe
// of every subband, so its L2 serves overlapping windows of the gathered
// vector.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include "codes.hpp"
#include "common.hpp"
#include "prox.hpp"

namespace wdb {

namespace {

struct TiledView {
  const int4* __restrict__ desc;
  const uint4* __restrict__ code;
  const float4* __restrict__ val;   // float32 values, groups of 4 codes (dense layout)
  const uint4* __restrict__ val16;  // 16-bit values, groups of 8 codes
  const int* __restrict__ erp;
  const int* __restrict__ ec;
  const float* __restrict__ ev;
  const GroupRec* __restrict__ grec;  // kept-value layout: group records
  const float* __restrict__ kval;     // and the kept values
  uint32_t kbytes;                    // bytes of kval readable by a buffer load
};

TiledView tview(const Tiled& t) {
  return TiledView{reinterpret_cast<const int4*>(t.desc), reinterpret_cast<const uint4*>(t.code),
                   reinterpret_cast<const float4*>(t.val), reinterpret_cast<const uint4*>(t.val16), t.erp, t.ec,
                   t.ev, static_cast<const GroupRec*>(t.grec), t.kval, static_cast<uint32_t>(4 * (t.nkval + 4))};
}

template <int FMT>
__device__ __forceinline__ float dq16(uint32_t h) {
  if constexpr (FMT == WDB_VAL_BF16) return __uint_as_float(h << 16);
  else return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(h)));
}

// The row's escape entries (wavefront w takes entries w, w + W, ...), then the
// partial sums of the W wavefronts added in wavefront order; the result is
// complete in wavefront 0.
template <int W, typename A, typename X>
__device__ __forceinline__ A tile_finish(const TiledView& T, const int4& d, int row, int lane, int wv, A acc,
                                         const X* __restrict__ x) {
  if (row >= 0 && (d.w & kHasEsc))  // the row's escape entries, dealt round-robin to the wavefronts
    for (int k = T.erp[row] + wv; k < T.erp[row + 1]; k += W)
      acc = fma(static_cast<A>(T.ev[k]), static_cast<A>(x[T.ec[k]]), acc);
  if constexpr (W > 1) {
    __shared__ A part[W][64];
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int w = 1; w < W; ++w) acc += part[w][lane];
    }
  }
  return acc;
}

// x[i] as the vector's base plus a 32-bit byte offset (i < 2^28 and elements
// of at most 8 bytes, so the offset fits): the gathers then take the form
// with the base in scalar registers and one offset register per lane.
template <typename X>
__device__ __forceinline__ X ld_at(const X* __restrict__ x, int i) {
  const uint32_t off = static_cast<uint32_t>(i) * static_cast<uint32_t>(sizeof(X));
  return *reinterpret_cast<const X*>(reinterpret_cast<const char*>(x) + off);
}

// x at the 4 columns of a group: one 16-byte load when the columns are
// consecutive in every lane of the wavefront (a quad of codes that differ
// only in dj, away from the subband's edge), two 8-byte loads when they are
// two such pairs, else four gathers.  The vector loads are buffer loads over
// x's n^2 floats (4-byte aligned; a buffer load also returns zeros rather
// than reading past the records).
__device__ __forceinline__ float4 ld_group(const float* __restrict__ x, const Geo& g, const int4& col) {
  const bool p1 = col.y == col.x + 1, p2 = col.w == col.z + 1;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(x), 0, 4 << (2 * g.logn), kBufWord3);
  if (__all(p1 && p2 && col.z == col.x + 2)) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, col.x * 4, 0, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
  }
  if (__all(p1 && p2)) {
    const auto a = __builtin_amdgcn_raw_buffer_load_b64(rs, col.x * 4, 0, 0);
    const auto b = __builtin_amdgcn_raw_buffer_load_b64(rs, col.z * 4, 0, 0);
    return make_float4(__uint_as_float(a[0]), __uint_as_float(a[1]), __uint_as_float(b[0]), __uint_as_float(b[1]));
  }
  return make_float4(ld_at(x, col.x), ld_at(x, col.y), ld_at(x, col.z), ld_at(x, col.w));
}

// Codes and values of the U groups k, k + W, ... of a float32 tile with the
// dense [group][lane][4] values (padding past g1).
template <int W, int U>
__device__ __forceinline__ void tile_load(const TiledView& T, int k, int g1, int lane, uint4 (&c)[U],
                                          float4 (&v)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const bool ok = k + u * W < g1;
    c[u] = ok ? T.code[k + u * W] : make_uint4(kPadCodeTile, kPadCodeTile, kPadCodeTile, kPadCodeTile);
    v[u] = ok ? T.val[static_cast<int64_t>(k + u * W) * 64 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// Group record k of the kept-value layout, or past g1 a record of padding
// codes with empty masks (whose values expand to zeros).
__device__ __forceinline__ GroupRec rec_at(const TiledView& T, int k, int g1) {
  const bool ok = k < g1;
  GroupRec r = T.grec[ok ? k : 0];
  if (!ok) {
    r.code = make_uint4(kPadCodeTile, kPadCodeTile, kPadCodeTile, kPadCodeTile);
    r.m[0] = r.m[1] = r.m[2] = r.m[3] = 0;
  }
  return r;
}

// Codes, value loads and row masks of the groups of records r (kept-value
// layout): the 4 floats at the lane's kept values, expanded with the masks
// when they are used.
template <int U>
__device__ __forceinline__ void rec_take(const TiledView& T, const GroupRec (&r)[U], uint4 (&c)[U], float4 (&v)[U],
                                         uint64_t (&mk)[U][4]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    c[u] = r[u].code;
#pragma unroll
    for (int j = 0; j < 4; ++j) mk[u][j] = r[u].m[j];
    v[u] = ld_kept(T.kval, T.kbytes, kept_offset(r[u]));
  }
}

// Dot product of the lane's row with x over float32 values (groups of 4
// codes, U groups per step).  A step decodes its columns, issues the
// gathers, then the loads of the next step's codes and values, and only
// then waits for the gathers: the latency of the next loads overlaps the
// wait for this step's gathers instead of following it.  Waits on scalar
// loads cover every scalar load in flight, so the next codes are requested
// only after this step's codes are used (the scheduling barriers keep that
// order).  With kept values (KEPT) a value load needs its group record
// first, so the records are requested one step ahead of the values: a step
// issues the next step's value loads from records that arrived during this
// one, then requests the records of the step after.
template <int W, int U, bool KEPT>
__device__ __forceinline__ float tile_dot(const TiledView& T, const Geo& g, const int4& d, int row, int lane,
                                          int wv, const float* __restrict__ x) {
  const RowCode rc = tile_row_code(g, d, row);
  float acc = 0.f;
  const int g1 = d.y >> 2;
  int k = (d.x >> 2) + wv;
  uint4 c[U];
  float4 v[U];
  uint64_t mk[U][4];
  GroupRec rn[U];
  if constexpr (KEPT) {
#pragma unroll
    for (int u = 0; u < U; ++u) rn[u] = rec_at(T, k + u * W, g1);
    rec_take<U>(T, rn, c, v, mk);
#pragma unroll
    for (int u = 0; u < U; ++u) rn[u] = rec_at(T, k + (U + u) * W, g1);
  } else {
    tile_load<W, U>(T, k, g1, lane, c, v);
  }
  for (; k < g1; k += W * U) {
    float4 xs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      xs[u] = ld_group(x, g, group_cols(g, rc, c[u]));
    }
    __builtin_amdgcn_sched_barrier(0);
    float4 vn[U];
    uint64_t mn[U][4];
    if constexpr (KEPT) {
      uint4 cn[U];
      rec_take<U>(T, rn, cn, vn, mn);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        rn[u] = rec_at(T, k + (2 * U + u) * W, g1);
        c[u] = cn[u];
      }
    } else {
      tile_load<W, U>(T, k + W * U, g1, lane, c, vn);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float4 e = KEPT ? expand_kept(mk[u], v[u]) : v[u];
      acc = fmaf(e.x, xs[u].x, acc);
      acc = fmaf(e.y, xs[u].y, acc);
      acc = fmaf(e.z, xs[u].z, acc);
      acc = fmaf(e.w, xs[u].w, acc);
      v[u] = vn[u];
      if constexpr (KEPT) {
#pragma unroll
        for (int j = 0; j < 4; ++j) mk[u][j] = mn[u][j];
      }
    }
  }
  return tile_finish<W, float>(T, d, row, lane, wv, acc, x);
}

// The 8 codes of a 16-bit group, read as one 32-byte unit.
struct Codes8 {
  uint4 a, b;
};

// Codes and values of the U groups of a 16-bit tile (8 codes per group).
template <int W, int U>
__device__ __forceinline__ void tile_load16(const TiledView& T, int k, int g1, int lane, uint4 (&c)[2 * U],
                                            uint4 (&v)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (k + u * W < g1) {
      const Codes8 cc = reinterpret_cast<const Codes8*>(T.code)[k + u * W];
      c[2 * u] = cc.a;
      c[2 * u + 1] = cc.b;
      v[u] = T.val16[static_cast<int64_t>(k + u * W) * 64 + lane];
    } else {
      c[2 * u] = c[2 * u + 1] = make_uint4(kPadCodeTile, kPadCodeTile, kPadCodeTile, kPadCodeTile);
      v[u] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
}

// The same over 16-bit values: groups of 8 codes, one 16-byte vector of 8
// values per lane and group, in the same step order as tile_dot (the columns
// of each half group of 4 codes from group_cols).
template <int W, int U, int FMT>
__device__ __forceinline__ float tile_dot16(const TiledView& T, const Geo& g, const int4& d, int row, int lane,
                                            int wv, const float* __restrict__ x) {
  const RowCode rc = tile_row_code(g, d, row);
  float acc = 0.f;
  const int g1 = d.y >> 3;
  int k = (d.x >> 3) + wv;
  uint4 c[2 * U], v[U];
  tile_load16<W, U>(T, k, g1, lane, c, v);
  for (; k < g1; k += W * U) {
    float xs[8 * U];
#pragma unroll
    for (int u = 0; u < 2 * U; ++u) {
      const float4 q = ld_group(x, g, group_cols(g, rc, c[u]));
      xs[4 * u] = q.x;
      xs[4 * u + 1] = q.y;
      xs[4 * u + 2] = q.z;
      xs[4 * u + 3] = q.w;
    }
    __builtin_amdgcn_sched_barrier(0);
    uint4 vn[U];
    tile_load16<W, U>(T, k + W * U, g1, lane, c, vn);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t vs[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
      for (int e = 0; e < 8; ++e)
        acc = fmaf(dq16<FMT>((vs[e >> 1] >> (16 * (e & 1))) & 0xFFFFu), xs[8 * u + e], acc);
      v[u] = vn[u];
    }
  }
  return tile_finish<W, float>(T, d, row, lane, wv, acc, x);
}

// Float64 accumulation over the float32 tiles (the stopping test): x is
// float32 (forward product) or float64 (the transposed product of the
// float64 residual).
template <int W, int U, bool KEPT, typename X>
__device__ __forceinline__ double tile_dot64(const TiledView& T, const Geo& g, const int4& d, int row, int lane,
                                             int wv, const X* __restrict__ x) {
  const RowCode rc = tile_row_code(g, d, row);
  double acc = 0.0;
  const int g1 = d.y >> 2;
  int k = (d.x >> 2) + wv;
  uint4 c[U];
  float4 v[U];
  uint64_t mk[U][4];
  GroupRec rn[U];
  if constexpr (KEPT) {
#pragma unroll
    for (int u = 0; u < U; ++u) rn[u] = rec_at(T, k + u * W, g1);
    rec_take<U>(T, rn, c, v, mk);
#pragma unroll
    for (int u = 0; u < U; ++u) rn[u] = rec_at(T, k + (U + u) * W, g1);
  } else {
    tile_load<W, U>(T, k, g1, lane, c, v);
  }
  // the same step order as tile_dot: gathers, then the next step's loads,
  // then the float64 sums of this step in code order
  for (; k < g1; k += W * U) {
    X xs[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int4 col = group_cols(g, rc, c[u]);
      xs[u][0] = ld_at(x, col.x);
      xs[u][1] = ld_at(x, col.y);
      xs[u][2] = ld_at(x, col.z);
      xs[u][3] = ld_at(x, col.w);
    }
    __builtin_amdgcn_sched_barrier(0);
    float4 vn[U];
    uint64_t mn[U][4];
    if constexpr (KEPT) {
      uint4 cn[U];
      rec_take<U>(T, rn, cn, vn, mn);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        rn[u] = rec_at(T, k + (2 * U + u) * W, g1);
        c[u] = cn[u];
      }
    } else {
      tile_load<W, U>(T, k + W * U, g1, lane, c, vn);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float4 e = KEPT ? expand_kept(mk[u], v[u]) : v[u];
      acc = fma(static_cast<double>(e.x), static_cast<double>(xs[u][0]), acc);
      acc = fma(static_cast<double>(e.y), static_cast<double>(xs[u][1]), acc);
      acc = fma(static_cast<double>(e.z), static_cast<double>(xs[u][2]), acc);
      acc = fma(static_cast<double>(e.w), static_cast<double>(xs[u][3]), acc);
      v[u] = vn[u];
      if constexpr (KEPT) {
#pragma unroll
        for (int j = 0; j < 4; ++j) mk[u][j] = mn[u][j];
      }
    }
  }
  return tile_finish<W, double>(T, d, row, lane, wv, acc, x);
}

// Sum (or max) of a float64 over the lanes of wavefront 0, written to
// partial[blockIdx.x] by lane 0.
template <bool MAX>
__device__ __forceinline__ void wave0_partial(double v, int lane, double* __restrict__ partial) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off);
    v = MAX ? fmax(v, o) : v + o;
  }
  if (lane == 0) partial[blockIdx.x] = v;
}

// Stopping test, forward half: r64 = Theta_K x - x0 in float64 and per-tile
// partials of ||r||^2, <r, x0> and sum_i w_i |x_i|.
template <int W, int U, bool KEPT, typename X>
__global__ __launch_bounds__(64 * W) void k_obj_fwd_tl(TiledView T, Geo g, const X* __restrict__ x,
                                                       const float* __restrict__ b, const float* __restrict__ w,
                                                       double* __restrict__ r64, double* __restrict__ partial,
                                                       int64_t nblocks, float* __restrict__ cneg) {
  const int4 d = T.desc[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row = tile_row(d, lane);
  const double acc = tile_dot64<W, U, KEPT>(T, g, d, row, lane, wv, x);
  if (wv != 0) return;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  if (row >= 0) {
    const double bb = static_cast<double>(b[row]);
    const double rr = acc - bb;
    r64[row] = rr;
    if (cneg) cneg[row] = static_cast<float>(-rr);  // the anchored iteration's next right-hand side
    v0 = rr * rr;
    v1 = rr * bb;
    v2 = fabs(static_cast<double>(x[row])) * (w ? static_cast<double>(w[row]) : 1.0);
  }
  wave0_partial<false>(v0, lane, partial);
  wave0_partial<false>(v1, lane, partial + nblocks);
  wave0_partial<false>(v2, lane, partial + 2 * nblocks);
}

// Backward half: per-tile max of |(Theta_K^T r64)_i| / w_i.
template <int W, int U, bool KEPT>
__global__ __launch_bounds__(64 * W) void k_obj_bwd_tl(TiledView T, Geo g, const double* __restrict__ r64,
                                                       const float* __restrict__ w, double* __restrict__ partial) {
  const int4 d = T.desc[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row = tile_row(d, lane);
  const double gr = tile_dot64<W, U, KEPT>(T, g, d, row, lane, wv, r64);
  if (wv != 0) return;
  const double v = row >= 0 ? fabs(gr) / (w ? static_cast<double>(w[row]) : 1.0) : 0.0;
  wave0_partial<true>(v, lane, partial);
}

template <int W, int U, bool KEPT>
__global__ __launch_bounds__(64 * W) void k_res_tl(TiledView T, Geo g, const float* __restrict__ y,
                                                   const float* __restrict__ b, float* __restrict__ r,
                                                   int* __restrict__ kdev) {
  const int4 d = T.desc[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row = tile_row(d, lane);
  const bool out = wv == 0 && row >= 0;
  const float bv = b && out ? b[row] : 0.0f;  // issued before the product so its latency overlaps
  const float acc = tile_dot<W, U, KEPT>(T, g, d, row, lane, wv, y);
  if (out) r[row] = acc - bv;
  // the iteration counter moves after the product: a global store ahead of
  // the loop would keep the code loads off the scalar path
  if (kdev && blockIdx.x == 0 && threadIdx.x == 0) *kdev += 1;
}

// Operands of the proximal epilogue, loaded before the product (a: the
// float64 anchor of the coefficient when the iterate is anchored).
struct ProxIn {
  double a;
  float y, x, pi, tw, beta;
};

template <bool PRE>
__device__ __forceinline__ ProxIn prox_load(int row, bool out, const float* __restrict__ x,
                                            const float* __restrict__ y, const int* __restrict__ kdev, float beta,
                                            const float* __restrict__ pinv, const float* __restrict__ tw,
                                            const double* __restrict__ anc) {
  ProxIn p{0.0, 0.f, 0.f, 1.f, 1.f, beta};
  if (out) {
    p.y = y[row];
    p.x = x[row];
    if (PRE) p.pi = pinv[row];
    p.tw = tw ? tw[row] : p.pi;
    if (anc) p.a = anc[row];
  }
  if (kdev) {
    const int k = *kdev;
    p.beta = static_cast<float>((static_cast<double>(k) - 1.0) / (static_cast<double>(k) + 2.0));
  }
  return p;
}

__device__ __forceinline__ void prox_store(const ProxIn& p, int row, float gr, float tau, float thr,
                                           float* __restrict__ x, float* __restrict__ y, bool anchored) {
  const float sg = (tau * p.pi) * gr;
  const float t = thr * p.tw;
  const float xn = anchored ? prox_anchored(p.a, p.y, sg, t) : prox_plain(p.y, sg, t);
  x[row] = xn;
  y[row] = xn + p.beta * (xn - p.x);
}

template <int W, int U, bool PRE, bool KEPT>
__global__ __launch_bounds__(64 * W) void k_prox_tl(TiledView T, Geo g, const float* __restrict__ r,
                                                    float* __restrict__ x, float* __restrict__ y, float tau,
                                                    float thr, float beta, const int* __restrict__ kdev,
                                                    const float* __restrict__ pinv, const float* __restrict__ tw,
                                                    const double* __restrict__ anc) {
  const int4 d = T.desc[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row = tile_row(d, lane);
  const bool out = wv == 0 && row >= 0;
  const ProxIn p = prox_load<PRE>(row, out, x, y, kdev, beta, pinv, tw, anc);
  const float gr = tile_dot<W, U, KEPT>(T, g, d, row, lane, wv, r);
  if (out) prox_store(p, row, gr, tau, thr, x, y, anc != nullptr);
}

// 16-bit values scaled by a power of two u per scale block (row subband for
// Theta_K, column subband for Theta_K^T): r = w (Q y) - b with w = 1 / u of
// the row, stored times w when scale_out (the input of the transposed kernel).
template <int W, int U, int FMT>
__global__ __launch_bounds__(64 * W) void k_res_tl16(TiledView T, Geo g, const float* __restrict__ wrow,
                                                     const float* __restrict__ y, const float* __restrict__ b,
                                                     float* __restrict__ r, int* __restrict__ kdev, int scale_out) {
  const int4 d = T.desc[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row = tile_row(d, lane);
  const bool out = wv == 0 && row >= 0;
  const float w = out ? wrow[row] : 0.0f;
  const float bv = b && out ? b[row] : 0.0f;
  const float acc = tile_dot16<W, U, FMT>(T, g, d, row, lane, wv, y);
  if (kdev && blockIdx.x == 0 && threadIdx.x == 0) *kdev += 1;
  if (!out) return;
  const float rr = b ? w * acc - bv : w * acc;
  r[row] = scale_out ? rr * w : rr;
}

// g = Q^T (w r); x_k = S(y - tau g / P); y = x_k + beta_k (x_k - x_{k-1}).
template <int W, int U, int FMT, bool PRE>
__global__ __launch_bounds__(64 * W) void k_prox_tl16(TiledView T, Geo g, const float* __restrict__ rs,
                                                      float* __restrict__ x, float* __restrict__ y, float tau,
                                                      float thr, const int* __restrict__ kdev,
                                                      const float* __restrict__ pinv, const float* __restrict__ tw) {
  const int4 d = T.desc[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row = tile_row(d, lane);
  const bool out = wv == 0 && row >= 0;
  const ProxIn p = prox_load<PRE>(row, out, x, y, kdev, 0.0f, pinv, tw, nullptr);  // no counter: beta = 0 (ISTA)
  const float gr = tile_dot16<W, U, FMT>(T, g, d, row, lane, wv, rs);
  if (out) prox_store(p, row, gr, tau, thr, x, y, false);
}

// Wavefronts per tile W and groups in flight per wavefront U.
template <typename F>
void with_shape(int W, int U, F&& f) {
  auto w = [&](auto Wc) {
    switch (U) {
      case 1: f(Wc, std::integral_constant<int, 1>{}); return;
      case 2: f(Wc, std::integral_constant<int, 2>{}); return;
      case 4: f(Wc, std::integral_constant<int, 4>{}); return;
      default: fail(WDB_ERR_ARG, "unsupported groups in flight %d (1, 2 or 4)", U);
    }
  };
  switch (W) {
    case 1: w(std::integral_constant<int, 1>{}); return;
    case 2: w(std::integral_constant<int, 2>{}); return;
    case 4: w(std::integral_constant<int, 4>{}); return;
    case 8: w(std::integral_constant<int, 8>{}); return;
    default: fail(WDB_ERR_ARG, "unsupported wavefronts per tile %d (1, 2, 4 or 8)", W);
  }
}

// Tiles in canonical band order: 8 x 8 position blocks of subbands of side
// >= 8 (row-major over blocks), one tile per smaller subband; desc.x and
// desc.y are filled by the encoder.
std::vector<int4> tile_list(const Geo& g) {
  std::vector<int4> tiles;
  for (int b = 0; b <= 3 * g.J; ++b) {
    const int level = b == 0 ? g.J : g.J - (b - 1) / 3;
    const int o = b == 0 ? 3 : (b - 1) % 3;
    const int ls = g.logn - level, s = 1 << ls;
    const int base = o == 3 ? 0 : (o + 1) << (2 * ls);
    if (s >= 8) {
      for (int bi = 0; bi < s / 8; ++bi)
        for (int bj = 0; bj < s / 8; ++bj) tiles.push_back(make_int4(0, 0, base + ((8 * bi) << ls) + 8 * bj, ls));
    } else {
      tiles.push_back(make_int4(0, 0, base, ls | kSmall | ((s * s) << 16)));
    }
  }
  return tiles;
}

struct TileOut {
  std::vector<int4> desc;
  std::vector<uint32_t> code;
  std::vector<float> val;
  std::vector<int32_t> erow, ecol;
  std::vector<float> eval;
  // float32 tiles only: row mask of each code (bit t: lane t keeps it), the
  // kept values and each group's offset into them
  std::vector<uint64_t> gmask;
  std::vector<float> kval;
  std::vector<int64_t> koff;
};

// Launch order of the tiles.  Workgroups are dealt round-robin to the 8
// XCDs (block b to XCD b mod 8), each with its own L2.  Band by band (the
// coarse bands first, as in the tile list), the band's tiles are cut into 8
// contiguous runs and position p of the launch takes the next tile of run
// p mod 8, so each XCD works on one spatial run of every band and the x
// windows of its tiles overlap; a run that is used up hands its positions to
// the others.  Returns the tile-list index of each launch position.
std::vector<int> xcd_order(const std::vector<int4>& tiles) {
  constexpr int kX = 8;
  std::vector<int> order;
  order.reserve(tiles.size());
  size_t b0 = 0;
  while (b0 < tiles.size()) {
    size_t b1 = b0 + 1;  // tiles of one band are adjacent in the list, with the same side and band base
    const int ls = tiles[b0].w & 0xFF;
    const int base = tiles[b0].z & ~((1 << (2 * ls)) - 1);
    while (b1 < tiles.size() && (tiles[b1].w & 0xFF) == ls && (tiles[b1].z & ~((1 << (2 * ls)) - 1)) == base &&
           !(tiles[b1].w & kSmall))
      ++b1;
    const size_t n = b1 - b0;
    size_t next[kX], end[kX];
    for (int k = 0; k < kX; ++k) {
      next[k] = b0 + n * k / kX;
      end[k] = b0 + n * (k + 1) / kX;
    }
    for (size_t done = 0; done < n; ++done) {
      int k = static_cast<int>(order.size() % kX);
      for (int tries = 0; tries < kX && next[k] == end[k]; ++tries) k = (k + 1) % kX;
      order.push_back(static_cast<int>(next[k]++));
    }
    b0 = b1;
  }
  return order;
}

// Order of a tile's codes in its value groups.  `u` holds the tile's distinct
// codes in ascending order, so codes that differ only in dj (the low field)
// and follow each other in dj form runs; every lane's columns for such a run
// are consecutive in x (unless they wrap around the subband's side).  Each
// run is cut into quads of 4 consecutive codes (with `extend`, a last part of
// 3 is completed by the next code, value 0 in every lane, when dj has room:
// more 16-byte loads for 7% more stored values on the workloads here, which
// pays for 16-bit values, whose kernels are bound by the gathers, but not for
// float32 ones, bound by the value stream), and what is left into pairs of 2
// consecutive codes and single codes.  Groups of 4 are
// then the quads, two pairs each, and the singles four at a time (the last
// group mixing what remains); a group of 8 (16-bit values) is two such
// groups.  The sequence is padded with kPadCodeTile to a multiple of grp.
std::vector<uint32_t> group_runs(const std::vector<uint32_t>& u, int grp, bool extend,
                                 const std::vector<uint64_t>* rows = nullptr) {
  using F = CodeTile;
  std::vector<uint32_t> quads, pairs, singles;
  for (size_t a = 0; a < u.size();) {
    size_t b = a + 1;
    while (b < u.size() && u[b] == u[b - 1] + 1 && (u[b] & F::kMask) != 0) ++b;   // same fields above dj
    size_t k = a;
    for (; k + 4 <= b; k += 4)
      for (int e = 0; e < 4; ++e) quads.push_back(u[k] + e);
    if (extend && b - k == 3 && (u[k] & F::kMask) + 3 <= F::kMask) {
      for (int e = 0; e < 4; ++e) quads.push_back(u[k] + e);
      k = b;
    }
    if (b - k >= 2) {
      pairs.push_back(u[k]);
      pairs.push_back(u[k + 1]);
      k += 2;
    }
    for (; k < b; ++k) singles.push_back(u[k]);
    a = b;
  }
  if (rows) {
    // pairs and singles (whose order does not change the column loads)
    // ordered by their row masks, fuller masks first, so that the codes of a
    // group tend to be kept by the same rows
    const auto mask_of = [&](uint32_t c) {
      return (*rows)[static_cast<size_t>(std::lower_bound(u.begin(), u.end(), c) - u.begin())];
    };
    const auto fuller = [](uint64_t a, uint64_t b) {
      const int pa = __builtin_popcountll(a), pb = __builtin_popcountll(b);
      return pa != pb ? pa > pb : a < b;
    };
    std::vector<std::pair<uint64_t, uint32_t>> pm;
    for (size_t k = 0; k < pairs.size(); k += 2) pm.emplace_back(mask_of(pairs[k]) | mask_of(pairs[k + 1]), pairs[k]);
    std::stable_sort(pm.begin(), pm.end(), [&](const auto& x, const auto& y) { return fuller(x.first, y.first); });
    for (size_t k = 0; k < pm.size(); ++k) {
      pairs[2 * k] = pm[k].second;
      pairs[2 * k + 1] = pm[k].second + 1;
    }
    std::stable_sort(singles.begin(), singles.end(),
                     [&](uint32_t x, uint32_t y) { return fuller(mask_of(x), mask_of(y)); });
  }
  std::vector<uint32_t> seq(quads);
  seq.insert(seq.end(), pairs.begin(), pairs.end());
  seq.insert(seq.end(), singles.begin(), singles.end());
  while (seq.size() % grp) seq.push_back(kPadCodeTile);
  return seq;
}

// Encode the tiles [t0, t1) of the tile list into `o` (pattern indices local
// to `o`; the caller rebases them).
// grp: codes per value group (4 for float32, 8 for 16-bit values); ub: the
// power-of-two scale of each subband (canonical order) that multiplies the
// values, taken from the row's subband (by_col false) or the column's, or
// null for no scaling.
void encode_tiles(const Geo& g, const std::vector<int4>& tiles, size_t t0, size_t t1,
                  const std::vector<int64_t>& rp, const std::vector<int32_t>& col, const std::vector<float>& val,
                  int grp, const std::vector<float>* ub, bool by_col, TileOut& o) {
  std::vector<std::pair<uint32_t, int>> ent;  // (code, lane) per kept entry of the tile
  std::vector<float> ent_v;
  std::vector<uint32_t> u;
  std::vector<uint64_t> umask;
  for (size_t ti = t0; ti < t1; ++ti) {
    int4 d = tiles[ti];
    ent.clear();
    ent_v.clear();
    bool esc = false;
    for (int t = 0; t < 64; ++t) {
      const int row = tile_row(d, t);
      if (row < 0) continue;
      const Pos p = pos_of(g, row);
      const float urow = ub ? (*ub)[band_index(g, p.level, p.orient)] : 1.0f;
      for (int64_t k = rp[row]; k < rp[row + 1]; ++k) {
        if (val[k] == 0.0f) continue;  // padding of the float32 copy
        float u = urow;
        if (ub && by_col) {
          const Pos q = pos_of(g, col[k]);
          u = (*ub)[band_index(g, q.level, q.orient)];
        }
        const float v = val[k] * u;  // exact: u is a power of two
        const int c = encode_col_tile(g, p, col[k]);
        if (c < 0) {
          o.erow.push_back(row);
          o.ecol.push_back(col[k]);
          o.eval.push_back(v);
          esc = true;
        } else {
          ent.emplace_back(static_cast<uint32_t>(c), t);
          ent_v.push_back(v);
        }
      }
    }
    u.clear();
    for (const auto& e : ent) u.push_back(e.first);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    if (grp == 4) {  // row mask of each distinct code
      umask.assign(u.size(), 0);
      for (const auto& e : ent)
        umask[static_cast<size_t>(std::lower_bound(u.begin(), u.end(), e.first) - u.begin())] |= uint64_t{1}
                                                                                                   << e.second;
    }
    const std::vector<uint32_t> seq = group_runs(u, grp, grp == 8, grp == 4 ? &umask : nullptr);
    // position of each kept code in the sequence (extension and padding codes carry value 0)
    std::vector<std::pair<uint32_t, int>> at;
    at.reserve(u.size());
    for (size_t q = 0; q < seq.size(); ++q)
      if (std::binary_search(u.begin(), u.end(), seq[q])) at.emplace_back(seq[q], static_cast<int>(q));
    std::sort(at.begin(), at.end());
    at.erase(std::unique(at.begin(), at.end(),
                         [](const auto& a, const auto& b) { return a.first == b.first; }),
             at.end());
    const int pb = static_cast<int>(o.code.size());
    o.code.insert(o.code.end(), seq.begin(), seq.end());
    o.val.resize(o.val.size() + seq.size() * 64, 0.0f);
    if (grp == 4) o.gmask.resize(o.code.size(), 0);
    for (size_t e = 0; e < ent.size(); ++e) {
      const auto it = std::lower_bound(at.begin(), at.end(), std::make_pair(ent[e].first, -1));
      const int64_t q = pb + it->second;
      o.val[((q / grp) * 64 + ent[e].second) * grp + (q % grp)] = ent_v[e];
      if (grp == 4) o.gmask[q] |= uint64_t{1} << ent[e].second;
    }
    if (grp == 4) {
      // the kept values of each group, lane by lane, each lane's in code order
      for (size_t gi = pb / 4; gi < o.code.size() / 4; ++gi) {
        const uint64_t* m = &o.gmask[4 * gi];
        o.koff.push_back(static_cast<int64_t>(o.kval.size()));
        for (int t = 0; t < 64; ++t)
          for (int j = 0; j < 4; ++j)
            if ((m[j] >> t) & 1) o.kval.push_back(o.val[(gi * 64 + t) * 4 + j]);
      }
    }
    d.x = pb;
    d.y = pb + static_cast<int>(seq.size());
    if (esc) d.w |= kHasEsc;
    o.desc.push_back(d);
  }
}

uint16_t round16(float f, int fmt) {
  if (fmt == WDB_VAL_BF16) {
    uint32_t b;
    std::memcpy(&b, &f, 4);
    b += 0x7FFFu + ((b >> 16) & 1u);  // round to nearest even
    return static_cast<uint16_t>(b >> 16);
  }
  const _Float16 h = static_cast<_Float16>(f);
  uint16_t r;
  std::memcpy(&r, &h, 2);
  return r;
}

float widen16(uint16_t h, int fmt) {
  if (fmt == WDB_VAL_BF16) {
    const uint32_t b = static_cast<uint32_t>(h) << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
  }
  _Float16 v;
  std::memcpy(&v, &h, 2);
  return static_cast<float>(v);
}

// fmt: WDB_VAL_F32 (values as float32, groups of 4 codes) or a 16-bit format
// (values times the scale of `ub`, rounded; groups of 8 codes).
void build_one(const wdb_theta* th, const Csr32& src, Tiled* out, int fmt = WDB_VAL_F32,
               const std::vector<float>* ub = nullptr, bool by_col = false) {
  const int grp = fmt == WDB_VAL_F32 ? 4 : 8;
  const Geo g = geo_of(th);
  const int64_t N = src.nrows;
  std::vector<int64_t> rp(N + 1);
  std::vector<int32_t> col(src.stored);
  std::vector<float> val(src.stored);
  WDB_HIP(hipMemcpy(rp.data(), src.rowptr, (N + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (src.stored) {
    WDB_HIP(hipMemcpy(col.data(), src.col, src.stored * sizeof(int32_t), hipMemcpyDeviceToHost));
    WDB_HIP(hipMemcpy(val.data(), src.val, src.stored * sizeof(float), hipMemcpyDeviceToHost));
  }
  std::vector<int4> tiles;
  {
    const std::vector<int4> listed = tile_list(g);
    for (int t : xcd_order(listed)) tiles.push_back(listed[t]);
  }
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const size_t nt = tiles.size(), parts = std::min<size_t>(hw, std::max<size_t>(1, nt / 64));
  std::vector<TileOut> res(parts);
  std::vector<std::thread> pool;
  std::vector<std::exception_ptr> errs(parts);
  for (size_t p = 0; p < parts; ++p)
    pool.emplace_back([&, p]() {
      try {
        encode_tiles(g, tiles, nt * p / parts, nt * (p + 1) / parts, rp, col, val, grp, ub, by_col, res[p]);
      } catch (...) {
        errs[p] = std::current_exception();
      }
    });
  for (auto& t : pool) t.join();
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
  std::vector<int4> desc;
  std::vector<uint32_t> code;
  int64_t nval = 0;
  for (auto& r : res) {
    const int off = static_cast<int>(code.size());
    WDB_REQUIRE(code.size() + r.code.size() < (size_t{1} << 31) / 64, WDB_ERR_ARG, "too many tile patterns");
    for (int4 d : r.desc) desc.push_back(make_int4(d.x + off, d.y + off, d.z, d.w));
    code.insert(code.end(), r.code.begin(), r.code.end());
    nval += static_cast<int64_t>(r.val.size());
  }
  // Escapes as a CSR over rows.
  std::vector<int32_t> erp(N + 1, 0);
  int64_t nesc = 0;
  for (auto& r : res) {
    for (int32_t row : r.erow) ++erp[row + 1];
    nesc += static_cast<int64_t>(r.erow.size());
  }
  for (int64_t i = 0; i < N; ++i) erp[i + 1] += erp[i];
  std::vector<int32_t> ec(nesc);
  std::vector<float> ev(nesc);
  {
    std::vector<int32_t> at(erp.begin(), erp.end() - 1);
    std::vector<std::tuple<int32_t, int32_t, float>> all;
    all.reserve(nesc);
    for (auto& r : res)
      for (size_t k = 0; k < r.erow.size(); ++k) all.emplace_back(r.erow[k], r.ecol[k], r.eval[k]);
    std::sort(all.begin(), all.end(), [](const auto& a, const auto& b) {
      return std::get<0>(a) != std::get<0>(b) ? std::get<0>(a) < std::get<0>(b) : std::get<1>(a) < std::get<1>(b);
    });
    for (const auto& e : all) {
      ec[at[std::get<0>(e)]] = std::get<1>(e);
      const float v = std::get<2>(e);
      ev[at[std::get<0>(e)]++] = fmt == WDB_VAL_F32 ? v : widen16(round16(v, fmt), fmt);
    }
  }
  Tiled t;
  try {
    t.ntiles = static_cast<int64_t>(desc.size());
    t.npat = static_cast<int64_t>(code.size());
    t.nesc = nesc;
    t.nkept = src.nnz;
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&t.desc), std::max<size_t>(desc.size(), 1) * sizeof(int4)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&t.code), std::max<size_t>(code.size(), 4) * sizeof(uint32_t)));
    WDB_HIP(hipMemcpy(t.desc, desc.data(), desc.size() * sizeof(int4), hipMemcpyHostToDevice));
    if (!code.empty()) WDB_HIP(hipMemcpy(t.code, code.data(), code.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    int64_t at = 0;
    if (fmt == WDB_VAL_F32) {
      WDB_HIP(hipMalloc(reinterpret_cast<void**>(&t.val), std::max<int64_t>(nval, 4) * sizeof(float)));
      for (auto& r : res) {
        if (!r.val.empty())
          WDB_HIP(hipMemcpy(t.val + at, r.val.data(), r.val.size() * sizeof(float), hipMemcpyHostToDevice));
        at += static_cast<int64_t>(r.val.size());
      }
      // the kept-value layout: group records and kept values
      const size_t ng = code.size() / 4;
      std::vector<GroupRec> rec(ng);
      int64_t kb = 0;
      size_t gb = 0;
      for (auto& r : res) {
        const size_t n = r.code.size() / 4;
        for (size_t gi = 0; gi < n; ++gi) {
          GroupRec& a = rec[gb + gi];
          a = GroupRec{};
          a.code = make_uint4(r.code[4 * gi], r.code[4 * gi + 1], r.code[4 * gi + 2], r.code[4 * gi + 3]);
          for (int j = 0; j < 4; ++j) a.m[j] = r.gmask[4 * gi + j];
          a.voff = static_cast<uint32_t>(kb + r.koff[gi]);
        }
        gb += n;
        kb += static_cast<int64_t>(r.kval.size());
      }
      // kept values are addressed by 32-bit byte offsets of buffer loads: an
      // operator with more than 2 GiB of them keeps only the dense layout
      if (4 * (kb + 4) < (int64_t{1} << 31)) {
        t.nkval = kb;
        WDB_HIP(hipMalloc(&t.grec, std::max<size_t>(ng, 1) * sizeof(GroupRec)));
        WDB_HIP(hipMalloc(reinterpret_cast<void**>(&t.kval), (kb + 4) * sizeof(float)));
        WDB_HIP(hipMemset(t.grec, 0, sizeof(GroupRec)));  // the record a kernel reads past a tile's end
        if (ng) WDB_HIP(hipMemcpy(t.grec, rec.data(), ng * sizeof(GroupRec), hipMemcpyHostToDevice));
        WDB_HIP(hipMemset(t.kval, 0, (kb + 4) * sizeof(float)));
        int64_t ka = 0;
        for (auto& r : res) {
          if (!r.kval.empty())
            WDB_HIP(hipMemcpy(t.kval + ka, r.kval.data(), r.kval.size() * sizeof(float), hipMemcpyHostToDevice));
          ka += static_cast<int64_t>(r.kval.size());
        }
      }
    } else {
      WDB_HIP(hipMalloc(reinterpret_cast<void**>(&t.val16), std::max<int64_t>(nval, 8) * sizeof(uint16_t)));
      std::vector<uint16_t> h;
      for (auto& r : res) {
        h.resize(r.val.size());
        for (size_t i = 0; i < r.val.size(); ++i) h[i] = round16(r.val[i], fmt);
        if (!h.empty()) WDB_HIP(hipMemcpy(t.val16 + at, h.data(), h.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
        at += static_cast<int64_t>(h.size());
      }
    }
    if (nesc) {
      WDB_HIP(hipMalloc(reinterpret_cast<void**>(&t.erp), (N + 1) * sizeof(int32_t)));
      WDB_HIP(hipMalloc(reinterpret_cast<void**>(&t.ec), nesc * sizeof(int32_t)));
      WDB_HIP(hipMalloc(reinterpret_cast<void**>(&t.ev), nesc * sizeof(float)));
      WDB_HIP(hipMemcpy(t.erp, erp.data(), (N + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
      WDB_HIP(hipMemcpy(t.ec, ec.data(), nesc * sizeof(int32_t), hipMemcpyHostToDevice));
      WDB_HIP(hipMemcpy(t.ev, ev.data(), nesc * sizeof(float), hipMemcpyHostToDevice));
    }
  } catch (...) {
    t.free_all();
    throw;
  }
  out->free_all();
  *out = t;
}

}  // namespace

void Tiled::free_all() {
  for (void* p : {static_cast<void*>(desc), static_cast<void*>(code), static_cast<void*>(val),
                  static_cast<void*>(val16), static_cast<void*>(erp), static_cast<void*>(ec), static_cast<void*>(ev),
                  grec, static_cast<void*>(kval)})
    if (p) (void)hipFree(p);
  grec = nullptr;
  kval = nullptr;
  nkval = 0;
  desc = nullptr;
  code = nullptr;
  val = nullptr;
  val16 = nullptr;
  erp = ec = nullptr;
  ev = nullptr;
  ntiles = npat = nesc = nkept = 0;
}

bool tiled_supported(const wdb_theta* th) { return packed_supported(th); }

void build_tiled(wdb_theta* th) {
  WDB_REQUIRE(tiled_supported(th), WDB_ERR_ARG, "tiled storage needs subbands of side >= 1 at every level");
  if (th->tA.desc && th->tAt.desc) return;
  build_one(th, th->cA, &th->tA);
  build_one(th, th->cAt, &th->tAt);
  if (!tiled_kept_available(th)) th->tile_kept = 0;
}

bool tiled_kept_available(const wdb_theta* th) { return th->tA.grec && th->tAt.grec; }

void build_tiled16(wdb_theta* th) {
  WDB_REQUIRE(tiled_supported(th), WDB_ERR_ARG, "tiled storage needs subbands of side >= 1 at every level");
  WDB_REQUIRE(th->valtype != WDB_VAL_F32 && !th->qscale.empty(), WDB_ERR_ARG,
              "the 16-bit tiled layout needs 16-bit values (wdb_set_precision)");
  if (th->qA.desc && th->qAt.desc) return;
  build_one(th, th->cA, &th->qA, th->valtype, &th->qscale, false);
  build_one(th, th->cAt, &th->qAt, th->valtype, &th->qscale, true);
}

void launch_res_tiled16(const wdb_theta* th, const float* y, const float* b, float* r, int* kdev, int scale_out,
                        hipStream_t s) {
  const Tiled& T = th->qA;
  WDB_REQUIRE(T.desc && T.val16, WDB_ERR_ARG, "16-bit tiled storage not built");
  const Geo g = geo_of(th);
  with_shape(th->tile_waves16, th->tile_unroll16, [&](auto Wc, auto Uc) {
    constexpr int W = decltype(Wc)::value, U = decltype(Uc)::value;
    const dim3 grid(static_cast<unsigned>(T.ntiles)), block(64 * W);
    if (th->valtype == WDB_VAL_BF16)
      hipLaunchKernelGGL((k_res_tl16<W, U, WDB_VAL_BF16>), grid, block, 0, s, tview(T), g, th->wrow, y, b, r, kdev,
                         scale_out);
    else
      hipLaunchKernelGGL((k_res_tl16<W, U, WDB_VAL_F16>), grid, block, 0, s, tview(T), g, th->wrow, y, b, r, kdev,
                         scale_out);
  });
}

void launch_prox_tiled16(const wdb_theta* th, const float* rs, float* x, float* y, float tau, float thr,
                         const int* kdev, const float* pinv, const float* tw, hipStream_t s) {
  const Tiled& T = th->qAt;
  WDB_REQUIRE(T.desc && T.val16, WDB_ERR_ARG, "16-bit tiled storage not built");
  const Geo g = geo_of(th);
  with_shape(th->tile_waves16, th->tile_unroll16, [&](auto Wc, auto Uc) {
    constexpr int W = decltype(Wc)::value, U = decltype(Uc)::value;
    const dim3 grid(static_cast<unsigned>(T.ntiles)), block(64 * W);
    if (th->valtype == WDB_VAL_BF16) {
      if (pinv)
        hipLaunchKernelGGL((k_prox_tl16<W, U, WDB_VAL_BF16, true>), grid, block, 0, s, tview(T), g, rs, x, y, tau,
                           thr, kdev, pinv, tw);
      else
        hipLaunchKernelGGL((k_prox_tl16<W, U, WDB_VAL_BF16, false>), grid, block, 0, s, tview(T), g, rs, x, y, tau,
                           thr, kdev, pinv, tw);
    } else {
      if (pinv)
        hipLaunchKernelGGL((k_prox_tl16<W, U, WDB_VAL_F16, true>), grid, block, 0, s, tview(T), g, rs, x, y, tau,
                           thr, kdev, pinv, tw);
      else
        hipLaunchKernelGGL((k_prox_tl16<W, U, WDB_VAL_F16, false>), grid, block, 0, s, tview(T), g, rs, x, y, tau,
                           thr, kdev, pinv, tw);
    }
  });
}

int64_t tiled_check_blocks(const wdb_theta* th) {
  WDB_REQUIRE(th->tA.desc && th->tAt.desc && th->tA.ntiles == th->tAt.ntiles, WDB_ERR_ARG,
              "tiled storage not built");
  return th->tA.ntiles;
}

namespace {
template <typename X>
void objective_tiled(const wdb_theta* th, const X* x, const float* x0, double* r64, double* part, int64_t nb,
                     hipStream_t s, float* cneg) {
  WDB_REQUIRE(nb == tiled_check_blocks(th), WDB_ERR_ARG, "partial count does not match the tiles");
  WDB_REQUIRE(!th->tile_kept || tiled_kept_available(th), WDB_ERR_ARG, "kept-value tiles not built");
  const Geo g = geo_of(th);
  with_shape(th->tile_waves, th->tile_unroll, [&](auto Wc, auto Uc) {
    constexpr int W = decltype(Wc)::value, U = decltype(Uc)::value;
    const dim3 grid(static_cast<unsigned>(nb)), block(64 * W);
    if (th->tile_kept) {
      hipLaunchKernelGGL((k_obj_fwd_tl<W, U, true, X>), grid, block, 0, s, tview(th->tA), g, x, x0, th->l1w, r64,
                         part, nb, cneg);
      hipLaunchKernelGGL((k_obj_bwd_tl<W, U, true>), grid, block, 0, s, tview(th->tAt), g, r64, th->l1w, part + 3 * nb);
    } else {
      hipLaunchKernelGGL((k_obj_fwd_tl<W, U, false, X>), grid, block, 0, s, tview(th->tA), g, x, x0, th->l1w, r64,
                         part, nb, cneg);
      hipLaunchKernelGGL((k_obj_bwd_tl<W, U, false>), grid, block, 0, s, tview(th->tAt), g, r64, th->l1w,
                         part + 3 * nb);
    }
  });
}
}  // namespace

void launch_objective_tiled(const wdb_theta* th, const float* x, const float* x0, double* r64, double* part,
                            int64_t nb, hipStream_t s, float* cneg) {
  objective_tiled(th, x, x0, r64, part, nb, s, cneg);
}

void launch_objective_tiled(const wdb_theta* th, const double* x, const float* x0, double* r64, double* part,
                            int64_t nb, hipStream_t s, float* cneg) {
  objective_tiled(th, x, x0, r64, part, nb, s, cneg);
}

void launch_res_tiled(const wdb_theta* th, bool transpose, const float* y, const float* b, float* r, int* kdev,
                      hipStream_t s) {
  const Tiled& T = transpose ? th->tAt : th->tA;
  WDB_REQUIRE(T.desc && (!th->tile_kept || T.grec), WDB_ERR_ARG, "tiled storage not built");
  const Geo g = geo_of(th);
  with_shape(th->tile_waves, th->tile_unroll, [&](auto Wc, auto Uc) {
    constexpr int W = decltype(Wc)::value, U = decltype(Uc)::value;
    const dim3 grid(static_cast<unsigned>(T.ntiles)), block(64 * W);
    if (th->tile_kept)
      hipLaunchKernelGGL((k_res_tl<W, U, true>), grid, block, 0, s, tview(T), g, y, b, r, kdev);
    else
      hipLaunchKernelGGL((k_res_tl<W, U, false>), grid, block, 0, s, tview(T), g, y, b, r, kdev);
  });
}

void launch_prox_tiled(const wdb_theta* th, const float* r, float* x, float* y, float tau, float thr, float beta,
                       const int* kdev, const float* pinv, const float* tw, const double* anc, hipStream_t s) {
  const Tiled& T = th->tAt;
  WDB_REQUIRE(T.desc && (!th->tile_kept || T.grec), WDB_ERR_ARG, "tiled storage not built");
  const Geo g = geo_of(th);
  with_shape(th->tile_waves, th->tile_unroll, [&](auto Wc, auto Uc) {
    constexpr int W = decltype(Wc)::value, U = decltype(Uc)::value;
    const dim3 grid(static_cast<unsigned>(T.ntiles)), block(64 * W);
    auto go = [&](auto Kc) {
      constexpr bool KEPT = decltype(Kc)::value;
      if (pinv)
        hipLaunchKernelGGL((k_prox_tl<W, U, true, KEPT>), grid, block, 0, s, tview(T), g, r, x, y, tau, thr, beta,
                           kdev, pinv, tw, anc);
      else
        hipLaunchKernelGGL((k_prox_tl<W, U, false, KEPT>), grid, block, 0, s, tview(T), g, r, x, y, tau, thr, beta,
                           kdev, pinv, tw, anc);
    };
    if (th->tile_kept) go(std::true_type{});
    else go(std::false_type{});
  });
}

}  // namespace wdb

extern "C" wdb_status wdb_set_tile_values(wdb_theta* th, int32_t kept) {
  WDB_API_BEGIN
  WDB_REQUIRE(th, WDB_ERR_ARG, "null handle");
  WDB_REQUIRE(kept == 0 || kept == 1, WDB_ERR_ARG, "tile value layout must be 0 (dense) or 1 (kept values)");
  WDB_REQUIRE(!kept || !th->tA.desc || wdb::tiled_kept_available(th), WDB_ERR_ARG,
              "this operator's tiles have no kept-value layout (more than 2 GiB of kept values)");
  wdb::drop_graph(th);  // the cached iteration graph may refer to what this call changes
  th->tile_kept = kept;
  WDB_API_END
}

extern "C" wdb_status wdb_set_tile_shape(wdb_theta* th, int32_t waves, int32_t unroll) {
  WDB_API_BEGIN
  WDB_REQUIRE(th, WDB_ERR_ARG, "null handle");
  wdb::drop_graph(th);  // the cached iteration graph may refer to what this call changes
  WDB_REQUIRE(waves == 1 || waves == 2 || waves == 4 || waves == 8, WDB_ERR_ARG,
              "wavefronts per tile must be 1, 2, 4 or 8");
  WDB_REQUIRE(unroll == 0 || unroll == 1 || unroll == 2 || unroll == 4, WDB_ERR_ARG,
              "groups in flight must be 0 (default), 1, 2 or 4");
  if (th->valtype == WDB_VAL_F32) {
    th->tile_waves = waves;
    th->tile_unroll = unroll ? unroll : 2;
  } else {
    th->tile_waves16 = waves;
    th->tile_unroll16 = unroll ? unroll : 1;
  }
  WDB_API_END
}
