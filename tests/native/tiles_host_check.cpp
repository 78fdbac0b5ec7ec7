// Host-side checks of the tiled pattern storage (no GPU needed): the tile
// list covers every coefficient once, the XCD launch order is a permutation
// of it, the shared group decode gives the same column as the per-code
// decode for every lane of every group, the kept-value layout of the float32
// tiles reads the same values as their dense layout, and the product over the
// encoded tiles (codes, values, escapes), for both value groupings, equals the
// row-wise product of the same sparse matrix exactly: values are multiples
// of 2^-8 and x of 2^-7, small enough that every float64 sum is exact in any
// order.
//
// Built by tests/test_native_tiles.py from the library's own sources: it
// includes tiled.hip and filters.cpp and stubs the few symbols that live in
// other translation units.
#include "../../paper_1512_08401_amd/csrc/tiled.hip"
#include "../../paper_1512_08401_amd/csrc/filters.cpp"

#include <cstdarg>
#include <cstdio>
#include <random>
#include <set>
#include <stdexcept>

namespace wdb {
[[noreturn]] void fail(wdb_status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw std::runtime_error(buf);
}
void set_last_error(const std::string&) {}
void clear_last_error() {}
int kernel_group(const wdb_theta*) { return 0; }
void Stencil::free_all() {}
bool packed_supported(const wdb_theta*) { return true; }
int packed_group(const wdb_theta*) { return 4; }
void Packed::free_all() {}
void drop_graph(wdb_theta*) {}
}  // namespace wdb

using namespace wdb;

namespace {

int failures = 0;

void expect(bool ok, const char* what, int logn, int J) {
  if (!ok) {
    ++failures;
    std::printf("FAIL %s (logn %d, J %d)\n", what, logn, J);
  }
}

// A random operator with the locality of a thresholded wavelet-domain blur:
// per row up to 24 columns at level gaps within [-3, 3] and displacements
// within [-4, 4] of the row's centre, plus now and then an arbitrary column
// (an escape when it does not fit a code) and an explicit zero.
void random_operator(const Geo& g, std::mt19937_64& rng, std::vector<int64_t>& rp, std::vector<int32_t>& col,
                     std::vector<float>& val) {
  const int N = 1 << (2 * g.logn);
  rp.assign(N + 1, 0);
  col.clear();
  val.clear();
  for (int r = 0; r < N; ++r) {
    const Pos p = pos_of(g, r);
    std::set<int> cols;
    for (int t = 0; t < 24; ++t) {
      const int lb = p.level + static_cast<int>(rng() % 7) - 3;
      if (lb < 1 || lb > g.J) continue;
      const int ls = g.logn - lb, s = 1 << ls;
      const int q = lb == g.J ? static_cast<int>(rng() % 4) : 1 + static_cast<int>(rng() % 3);
      const int ci = centre_at(g, p.i, p.level, lb), cj = centre_at(g, p.j, p.level, lb);
      const int ib = (ci + static_cast<int>(rng() % 9) - 4) & (s - 1);
      const int jb = (cj + static_cast<int>(rng() % 9) - 4) & (s - 1);
      cols.insert((q << (2 * ls)) + ib * s + jb);
    }
    if (rng() % 10 == 0) cols.insert(static_cast<int>(rng() % N));
    for (int c : cols) {
      col.push_back(c);
      val.push_back(static_cast<float>(static_cast<int>(rng() % 2001) - 1000) / 256.0f);
    }
    if (rng() % 3 == 0) {
      col.push_back(r);
      val.push_back(0.0f);
    }
    rp[r + 1] = static_cast<int64_t>(col.size());
  }
}

void check(int logn, int J, int L1, std::mt19937_64& rng) {
  const Geo g{logn, J, L1};
  const int N = 1 << (2 * logn);
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  std::vector<float> val;
  random_operator(g, rng, rp, col, val);

  const std::vector<int4> listed = tile_list(g);
  std::vector<int> cover(N, 0);
  for (const int4& d : listed)
    for (int t = 0; t < 64; ++t) {
      const int r = tile_row(d, t);
      if (r >= 0 && r < N) ++cover[r];
      expect(r < N, "tile row in range", logn, J);
    }
  bool once = true;
  for (int c : cover) once = once && c == 1;
  expect(once, "every coefficient in exactly one tile", logn, J);

  const std::vector<int> order = xcd_order(listed);
  std::vector<int> sorted(order);
  std::sort(sorted.begin(), sorted.end());
  bool perm = sorted.size() == listed.size();
  for (size_t i = 0; perm && i < sorted.size(); ++i) perm = sorted[i] == static_cast<int>(i);
  expect(perm, "launch order is a permutation of the tile list", logn, J);
  std::vector<int4> tiles;
  for (int t : order) tiles.push_back(listed[t]);

  std::vector<double> x(N);
  for (double& v : x) v = static_cast<double>(static_cast<int>(rng() % 1001) - 500) / 128.0;
  std::vector<double> ref(N, 0.0);
  for (int r = 0; r < N; ++r)
    for (int64_t k = rp[r]; k < rp[r + 1]; ++k) ref[r] += static_cast<double>(val[k]) * x[col[k]];

  // both value groupings: 4 codes (float32 values) and 8 codes (16-bit values,
  // whose grouping also completes runs of 3 with zero-valued codes)
  TileOut o;
  for (int grp : {8, 4}) {
    o = TileOut{};
    encode_tiles(g, tiles, 0, tiles.size(), rp, col, val, grp, nullptr, false, o);
    std::vector<double> got(N, 0.0);
    bool same_cols = true, in_range = true, whole = true;
    for (const int4& d : o.desc) {
      whole = whole && (d.y - d.x) % grp == 0;
      for (int t = 0; t < 64; ++t) {
        const int row = tile_row(d, t);
        const RowCode rc = tile_row_code(g, d, row);
        double acc = 0.0;
        for (int p = d.x; p < d.y; p += 4) {
          const uint4 c = make_uint4(o.code[p], o.code[p + 1], o.code[p + 2], o.code[p + 3]);
          const int4 gc = group_cols(g, rc, c);
          const int ref_cols[4] = {decode_col_tile(g, rc, c.x), decode_col_tile(g, rc, c.y),
                                   decode_col_tile(g, rc, c.z), decode_col_tile(g, rc, c.w)};
          const int got_cols[4] = {gc.x, gc.y, gc.z, gc.w};
          for (int e = 0; e < 4; ++e) {
            same_cols = same_cols && got_cols[e] == ref_cols[e];
            in_range = in_range && ref_cols[e] >= 0 && ref_cols[e] < N;
            const int64_t q = p + e;
            const float v = o.val[((q / grp) * 64 + t) * grp + q % grp];
            if (in_range) acc += static_cast<double>(v) * x[ref_cols[e]];
          }
        }
        if (row >= 0) got[row] += acc;
      }
    }
    for (size_t k = 0; k < o.erow.size(); ++k) got[o.erow[k]] += static_cast<double>(o.eval[k]) * x[o.ecol[k]];
    if (grp == 4) {
      // the kept-value layout, read as a lane reads it: its values start at the
      // group's offset plus the kept entries of the lanes below, and code j
      // takes the next one if the lane's bit of mask j is set; every slot must
      // equal the dense value (zero where the lane lacks the code)
      bool same_vals = o.gmask.size() == o.code.size() && o.koff.size() == o.code.size() / 4;
      int64_t kept = 0;
      for (size_t gi = 0; same_vals && gi < o.koff.size(); ++gi) {
        const uint64_t* m = &o.gmask[4 * gi];
        for (int t = 0; t < 64; ++t) {
          const uint64_t below = (uint64_t{1} << t) - 1;
          int64_t at = o.koff[gi];
          for (int j = 0; j < 4; ++j) at += __builtin_popcountll(m[j] & below);
          for (int j = 0; j < 4; ++j) {
            const bool has = (m[j] >> t) & 1;
            const float v = has ? o.kval[at++] : 0.0f;
            same_vals = same_vals && v == o.val[(gi * 64 + t) * 4 + j];
            kept += has;
          }
        }
      }
      int64_t nonzero = 0;
      for (float v : val) nonzero += v != 0.0f;
      expect(same_vals, "kept-value layout reads the dense values", logn, J);
      expect(kept == static_cast<int64_t>(o.kval.size()) &&
                 kept + static_cast<int64_t>(o.erow.size()) == nonzero,
             "kept values hold each non-escaped entry once", logn, J);
    }
    expect(whole, "tile code ranges are whole groups", logn, J);
    expect(same_cols, "group decode equals per-code decode", logn, J);
    expect(in_range, "decoded columns in range", logn, J);
    double err = 0.0;
    for (int r = 0; r < N; ++r) err = std::max(err, std::fabs(ref[r] - got[r]));
    expect(err == 0.0, "tile product equals row-wise product", logn, J);
  }
  std::printf("logn %d J %d L1 %d: %zu tiles, %zu codes, %zu escapes\n", logn, J, L1, o.desc.size(),
              o.code.size(), o.erow.size());
}

}  // namespace

int main() {
  std::mt19937_64 rng(20151208);
  const int cfg[][3] = {{5, 4, 1}, {6, 3, 7}, {6, 5, 1}, {7, 4, 7}, {8, 3, 11}, {8, 5, 7}};
  for (const auto& c : cfg) check(c[0], c[1], c[2], rng);
  std::printf("%s\n", failures ? "FAILED" : "all checks passed");
  return failures ? 1 : 0;
}
