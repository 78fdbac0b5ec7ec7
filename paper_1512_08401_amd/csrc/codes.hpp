// Band-relative column codes shared by the packed 16-bit form and the tiled
// pattern storage (with wider displacement fields in the latter's 32-bit
// codes), and the tile descriptors of the tiled storage.
//
// An entry theta[a, b] is only large when the supports of the two atoms are
// close in space and in scale (the decay bound of Sec. 3.2).  For a row
// coefficient a at level la, position (ia, ja), and a column coefficient b at
// level lb, orientation o, position (ib, jb), the 16-bit code stores
//   dL = lb - la in [-3, 3], band slot q in {0 (approximation), 1, 2, 3
//   (details (0,1), (1,0), (1,1))}, and (di, dj) in [-16, 15]^2: b's position
//   minus the point of level lb whose atom is centred nearest to a's atom,
//   modulo the side s of b's subband,
// as bit fields ((dL + 3) << 13) | (q << 11) | ((di + 16) << 5) | (dj + 16).
// b's index is then q s^2 + ((ci + di) mod s) s + ((cj + dj) mod s), exact
// integer arithmetic on power-of-two sides.
#pragma once

#include <cstdint>

#include "common.hpp"

namespace wdb {

constexpr int kLMax = 3;  // level differences in [-3, 3]

// Bit layout of a column code: DB bits per displacement (stored plus 2^(DB-1)),
// dj at bit 0, di at bit DB, the band slot at bit QS, the level difference
// plus 3 at bit QS + 2.  The packed 16-bit form uses 5-bit displacements
// ([-16, 15]); the tiles, whose codes are 32-bit words, 8-bit ones ([-128, 127]).
template <int DB, int QS>
struct CodeLayout {
  static constexpr int kDB = DB, kQS = QS, kOff = 1 << (DB - 1);
  static constexpr uint32_t kMask = (1u << DB) - 1u;
  // Padding code: value 0, column = a valid coefficient (a detail subband of
  // the row's own level, which every level has).
  static constexpr uint32_t kPad = (static_cast<uint32_t>(kLMax) << (QS + 2)) | (1u << QS) |
                                   (static_cast<uint32_t>(kOff) << DB) | static_cast<uint32_t>(kOff);
};
using Code16 = CodeLayout<5, 11>;
using CodeTile = CodeLayout<8, 16>;
constexpr int kDOff = Code16::kOff;
constexpr uint32_t kPadCode = Code16::kPad;
constexpr uint32_t kPadCodeTile = CodeTile::kPad;

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

// Per-row constants of the decode: the numerators of the row atom's centre,
// (i << (la + 1)) + L1 2^la and the same in j, and la - 3.
struct RowCode {
  int pi, pj, lb0;
};

__host__ __device__ inline RowCode row_code(const Geo& g, const Pos& p) {
  return RowCode{(p.i << (p.level + 1)) + g.L1 * (1 << p.level), (p.j << (p.level + 1)) + g.L1 * (1 << p.level),
                 p.level - kLMax};
}

// Column of a code for the row of `rc`: the centre of the column level
// lb = la + dL is (num + (1 - L1) 2^lb) >> (lb + 1) (centre_at), then the
// displacement is added modulo the side.  lb is clamped to [1, J] so that
// any code decodes to an index below n^2 (the encoder only emits levels in
// range, where the clamp is the identity).
// Terms that depend on the code and the row level only (lb, the side, t, the
// mask, the displacements, the band offset) are grouped apart from the
// row's centre numerators, so that where the level is the same for all
// lanes (tile_row_code) they are computed once per wavefront.
template <class F>
__host__ __device__ inline int decode_col_as(const Geo& g, const RowCode& rc, uint32_t code) {
  const int lb = min(max(rc.lb0 + static_cast<int>((code >> (F::kQS + 2)) & 7u), 1), g.J);
  const int ls = g.logn - lb;
  const int t = (1 - g.L1) * (1 << lb);
  const int m = (1 << ls) - 1;
  const int di = static_cast<int>((code >> F::kDB) & F::kMask) - F::kOff;
  const int dj = static_cast<int>(code & F::kMask) - F::kOff;
  const int ib = (((rc.pi + t) >> (lb + 1)) + di) & m;
  const int jb = (((rc.pj + t) >> (lb + 1)) + dj) & m;
  return (static_cast<int>((code >> F::kQS) & 3u) << (2 * ls)) + (ib << ls) + jb;
}

// Code of column `col` for row position p, or -1 if it does not fit.
template <class F>
__host__ __device__ inline int encode_col_as(const Geo& g, const Pos& p, int64_t col) {
  const Pos q = pos_of(g, col);
  const int dL = q.level - p.level;
  if (dL < -kLMax || dL > kLMax) return -1;
  const int ls = g.logn - q.level;
  const int s = 1 << ls, m = s - 1, h = s >> 1;
  const int di = ((q.i - centre_at(g, p.i, p.level, q.level) + h) & m) - h;
  const int dj = ((q.j - centre_at(g, p.j, p.level, q.level) + h) & m) - h;
  if (di < -F::kOff || di >= F::kOff || dj < -F::kOff || dj >= F::kOff) return -1;
  const int slot = q.orient == 3 ? 0 : q.orient + 1;
  return ((dL + kLMax) << (F::kQS + 2)) | (slot << F::kQS) | ((di + F::kOff) << F::kDB) | (dj + F::kOff);
}

__host__ __device__ inline int decode_col(const Geo& g, const RowCode& rc, uint32_t code) {
  return decode_col_as<Code16>(g, rc, code);
}
__host__ __device__ inline int encode_col(const Geo& g, const Pos& p, int64_t col) {
  return encode_col_as<Code16>(g, p, col);
}
__host__ __device__ inline int decode_col_tile(const Geo& g, const RowCode& rc, uint32_t code) {
  return decode_col_as<CodeTile>(g, rc, code);
}
__host__ __device__ inline int encode_col_tile(const Geo& g, const Pos& p, int64_t col) {
  return encode_col_as<CodeTile>(g, p, col);
}

// Tile descriptors of the tiled pattern storage: int4 {first code, end code,
// first row, log2 side | flags}.
constexpr int kSmall = 1 << 8;   // flag: tile = a whole subband of side < 8, rows first + t for t < count
constexpr int kHasEsc = 1 << 30; // flag: some row of the tile has escape entries

// Row of lane t of a tile (8 x 8 positions, lane t at (t / 8, t mod 8)), or
// -1 for an idle lane of a small subband.
__host__ __device__ inline int tile_row(const int4& d, int t) {
  if (d.w & kSmall) return t < ((d.w >> 16) & 0x7F) ? d.z + t : -1;
  const int ls = d.w & 0xFF;
  return d.z + ((t >> 3) << ls) + (t & 7);
}

// Decode constants of `row` in tile d (an idle lane takes the tile's first
// row).  Every row of a tile lies in the tile's subband, so the row level is
// read from the descriptor: the same value as pos_of gives, but visibly
// uniform across the wavefront.
__host__ __device__ inline RowCode tile_row_code(const Geo& g, const int4& d, int row) {
  RowCode rc = row_code(g, pos_of(g, row >= 0 ? row : d.z));
  rc.lb0 = g.logn - (d.w & 0xFF) - kLMax;
  return rc;
}

// Columns of 4 codes.  When the 4 share the level and band fields (the
// common case: a tile's codes are sorted, so codes come in runs with the
// same level and band), the lane shifts its centre once for the group and
// each code only adds its displacements; otherwise each code is decoded in
// full.  Both give decode_col_tile's columns.
__host__ __device__ inline int4 group_cols(const Geo& g, const RowCode& rc, const uint4& c) {
  using F = CodeTile;
  if ((((c.x ^ c.y) | (c.x ^ c.z) | (c.x ^ c.w)) >> F::kQS) == 0) {
    const int lb = min(max(rc.lb0 + static_cast<int>((c.x >> (F::kQS + 2)) & 7u), 1), g.J);
    const int ls = g.logn - lb;
    const int t = (1 - g.L1) * (1 << lb);
    const int m = (1 << ls) - 1;
    const int ci = (rc.pi + t) >> (lb + 1);
    const int cj = (rc.pj + t) >> (lb + 1);
    const int qoff = static_cast<int>((c.x >> F::kQS) & 3u) << (2 * ls);
    const auto at = [&](uint32_t code) {
      const int di = static_cast<int>((code >> F::kDB) & F::kMask) - F::kOff;
      const int dj = static_cast<int>(code & F::kMask) - F::kOff;
      return qoff + (((ci + di) & m) << ls) + ((cj + dj) & m);
    };
    return make_int4(at(c.x), at(c.y), at(c.z), at(c.w));
  }
  return make_int4(decode_col_tile(g, rc, c.x), decode_col_tile(g, rc, c.y), decode_col_tile(g, rc, c.z),
                   decode_col_tile(g, rc, c.w));
}

// Kept-value layout of the float32 tiles.  A group of 4 codes stores, instead
// of 64 rows x 4 values with zeros where a row did not keep a code, only the
// kept values: lane by lane, each lane's values in code order.  Its record
// holds the codes, one row mask per code (bit t: row t of the tile keeps
// it) and the offset of the group's values; lane t finds its values at that
// offset plus the number of kept entries of the rows below t.
struct alignas(64) GroupRec {
  uint4 code;
  uint64_t m[4];
  uint32_t voff;
  uint32_t pad[3];
};
static_assert(sizeof(GroupRec) == 64, "one 64-byte record per group");

// A wavefront-uniform 64-bit value in scalar registers (the value of the
// first active lane; free when the compiler already holds it there).
__device__ __forceinline__ uint64_t wave_uniform(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// b if this lane's bit of the wavefront-uniform mask m is set, else a: one
// select with m itself as the lane condition (m must be uniform: the select
// reads it from scalar registers).
__device__ __forceinline__ float sel_lane(uint64_t m, float a, float b) {
  float r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(wave_uniform(m)));
  return r;
}

// acc plus the number of set bits of m below this lane.
__device__ __forceinline__ uint32_t rows_below(uint64_t m, uint32_t acc) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), acc));
}

// Word 3 of a raw buffer resource on gfx9-family chips: data format 32-bit,
// no swizzle, no index stride.
constexpr int kBufWord3 = 0x00020000;

// Byte offset of this lane's kept values of group r.
__device__ __forceinline__ uint32_t kept_offset(const GroupRec& r) {
  uint32_t o = r.voff;
#pragma unroll
  for (int j = 0; j < 4; ++j) o = rows_below(r.m[j], o);
  return 4 * o;
}

// 4 floats at byte offset `off` of the kept values (a buffer load over
// `bytes`: reads past the end return zeros).
__device__ __forceinline__ float4 ld_kept(const float* __restrict__ kval, uint32_t bytes, uint32_t off) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(kval), 0, static_cast<int>(bytes), kBufWord3);
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
  return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
}

// The lane's values of the group's 4 codes from its kept values packed in
// code order at v.x, v.y, ...: code j takes the next packed value if the
// lane's bit of m[j] is set, else 0.
__device__ __forceinline__ float4 expand_kept(const uint64_t (&m)[4], const float4& v) {
  const float z = 0.f;
  const float e0 = sel_lane(m[0], z, v.x);
  const float a0 = sel_lane(m[0], v.x, v.y), a1 = sel_lane(m[0], v.y, v.z), a2 = sel_lane(m[0], v.z, v.w);
  const float e1 = sel_lane(m[1], z, a0);
  const float b0 = sel_lane(m[1], a0, a1), b1 = sel_lane(m[1], a1, a2);
  const float e2 = sel_lane(m[2], z, b0);
  const float c0 = sel_lane(m[2], b0, b1);
  const float e3 = sel_lane(m[3], z, c0);
  return make_float4(e0, e1, e2, e3);
}

// The lane's 4 values of group r (record already loaded).
__device__ __forceinline__ float4 kept_values(const GroupRec& r, const float* __restrict__ kval, uint32_t bytes) {
  return expand_kept(r.m, ld_kept(kval, bytes, kept_offset(r)));
}

inline Geo geo_of(const wdb_theta* th) {
  return Geo{floor_log2(static_cast<uint64_t>(th->n)), th->levels,
             static_cast<int>(make_filter(th->wavelet).h.size()) - 1};
}

}  // namespace wdb
