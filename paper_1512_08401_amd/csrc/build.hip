// Theta_K = K largest-magnitude entries of Theta = Psi^* H Psi (Sec. 3.4,
// Sec. 3.7 naive rule), computed on the GPU in float64.
//
// Column b of Theta is Psi^*(H psi_b).  The paper notes that applying H to
// all N atoms and transforming them is O(N^3) for a spatially varying blur
// (Sec. 3.4).  Here each column is computed on its support only:
//
//  * psi_b is separable: f_erow,l(r - 2^l p) * f_ecol,l(c - 2^l q), with the
//    level-l equivalent filters f_0,l / f_1,l (the cascade of h and g that
//    maps pixels to level-l coefficients, periodised to n).
//  * H psi_b is non-zero only on the atom's window dilated by the PSF radius
//    R; it is gathered pixel by pixel in float64 from the source PSFs.
//  * Psi^* of that window is a local pyramid: at each level only the
//    coefficients whose footprint meets the current window are formed, with
//    periodic index arithmetic, so every non-zero <psi_a, H psi_b> of the
//    column is produced exactly once.
//
// One workgroup owns one column at a time (float64 window buffers in a
// per-workgroup slab of global memory).  The K largest magnitudes are found
// by a radix select on the IEEE bit pattern of |theta|: each histogram pass
// recomputes every column and counts 12-bit digits of the keys that match
// the prefix fixed so far; once the boundary digit holds few enough entries,
// an emit pass writes the entries above the boundary and collects the
// boundary digit, whose ties are ordered by (|theta| descending, a*N + b
// ascending).  The kept triples are then sorted into CSR.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <numeric>

#include "common.hpp"
#include "psf.hpp"

namespace wdb {

namespace {

constexpr int kMaxSub = 48;
constexpr int kMaxLev = 16;
constexpr int kDigits = 4096;
constexpr unsigned long long kBoundaryCap = 1ull << 22;

struct Geom {
  int n, J, L, R, nsub;
  int sub_level[kMaxSub], sub_er[kMaxSub], sub_ec[kMaxSub], sub_side[kMaxSub];
  int64_t sub_off[kMaxSub + 1];
  int flen[kMaxLev];
  int64_t foff[kMaxLev];
  double h[kMaxTaps], g[kMaxTaps];
};

struct Select {
  int mode;   // 0: histogram, 1: emit above prefix + collect prefix, 2: emit every non-zero
  int scaled; // 1: rank by sigma_b |theta| with sigma_b = 2^-k = 1 / (side of b's subband) (Sec. 3.7)
  int pbits;  // bits of the key already fixed
  int shift;  // histogram digit position
  unsigned long long prefix;
  unsigned long long dmask;
};

struct Emit {
  int32_t* row;
  int32_t* col;
  double* val;
  unsigned long long* count;
  unsigned long long cap;
};

struct Win {
  int s, len, M;  // positions (s + t) mod M for t < len
};

__host__ __device__ inline int floordiv2(int a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); }

// Window of level-(l+1) positions whose footprint [2i, 2i + L - 1] meets w.
__host__ __device__ inline Win next_win(Win w, int L) {
  const int Mh = w.M >> 1;
  if (w.len >= w.M) return Win{0, Mh, Mh};
  const int lo = floordiv2(w.s - L + 2);
  const int hi = floordiv2(w.s + w.len - 1);
  const int len = hi - lo + 1;
  if (len >= Mh) return Win{0, Mh, Mh};
  return Win{lo & (Mh - 1), len, Mh};
}

__device__ inline void emit_one(bool want, int a, int b, double v, const Emit& E, int* err) {
  const unsigned long long mask = __ballot(want);
  if (mask == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll(static_cast<long long>(mask)) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(E.count, static_cast<unsigned long long>(__popcll(mask)));
  const unsigned lo = __shfl(static_cast<unsigned>(base & 0xffffffffull), leader);
  const unsigned hi = __shfl(static_cast<unsigned>(base >> 32), leader);
  base = (static_cast<unsigned long long>(hi) << 32) | lo;
  if (want) {
    const unsigned long long idx = base + __popcll(mask & ((1ull << lane) - 1ull));
    if (idx < E.cap) {
      E.row[idx] = a;
      E.col[idx] = b;
      E.val[idx] = v;
    } else {
      atomicOr(err, 2);
    }
  }
}

// sb: the column's ranking weight (1, or sigma_b; a power of two, so the
// scaled magnitude is exact).
__device__ inline void handle(const Select& S, double v, double sb, int a, int b, unsigned* lhist, const Emit& out,
                              const Emit& bnd, int* err) {
  const bool nz = v != 0.0;
  const unsigned long long key = static_cast<unsigned long long>(__double_as_longlong(fabs(v) * sb));
  if (S.mode == 0) {
    if (nz && (S.pbits == 0 || (key >> (64 - S.pbits)) == S.prefix))
      atomicAdd(&lhist[(key >> S.shift) & S.dmask], 1u);
  } else if (S.mode == 2) {
    emit_one(nz, a, b, v, out, err);
  } else {
    const unsigned long long top = key >> (64 - S.pbits);
    emit_one(nz && top > S.prefix, a, b, v, out, err);
    emit_one(nz && top == S.prefix, a, b, v, bnd, err);
  }
}

__global__ __launch_bounds__(256) void k_theta_columns(Geom G, PsfDev P, const double* __restrict__ ftab,
                                                       double* __restrict__ scratch, int64_t cap,
                                                       int64_t b_begin, int64_t b_end, Select S,
                                                       unsigned long long* __restrict__ ghist, Emit out,
                                                       Emit bnd, int* err) {
  __shared__ unsigned lhist[kDigits];
  const int tid = threadIdx.x, nt = blockDim.x;
  if (S.mode == 0)
    for (int i = tid; i < kDigits; i += nt) lhist[i] = 0u;
  __syncthreads();
  double* bufA = scratch + static_cast<size_t>(blockIdx.x) * 2 * cap;
  double* bufB = bufA + cap;
  const int n = G.n, R = G.R, L = G.L;
  for (int64_t b = b_begin + blockIdx.x; b < b_end; b += gridDim.x) {
    int k = 0;
    while (k + 1 < G.nsub && b >= G.sub_off[k + 1]) ++k;
    const int lev = G.sub_level[k], side = G.sub_side[k];
    const double sb = S.scaled ? 1.0 / static_cast<double>(side) : 1.0;
    const int64_t pos = b - G.sub_off[k];
    const int p = static_cast<int>(pos / side), q = static_cast<int>(pos % side);
    const int wl = G.flen[lev];
    const double* fr = ftab + G.foff[lev] + (G.sub_er[k] ? wl : 0);
    const double* fc = ftab + G.foff[lev] + (G.sub_ec[k] ? wl : 0);
    const int r0 = (p << lev) & (n - 1), c0 = (q << lev) & (n - 1);
    // H psi_b on the atom window dilated by R (whole torus if that is wider).
    const int hl = min(wl + 2 * R, n);
    const int hr0 = (r0 - R) & (n - 1), hc0 = (c0 - R) & (n - 1);
    for (int o = tid; o < hl * hl; o += nt) {
      const int orow = o / hl, ocol = o - orow * hl;
      const int ir = (hr0 + orow) & (n - 1), ic = (hc0 + ocol) & (n - 1);
      double acc = 0.0;
      for (int dy = -R; dy <= R; ++dy) {
        const int tr = (ir - dy - r0) & (n - 1);
        if (tr >= wl) continue;
        const double vr = fr[tr];
        const int sr = (r0 + tr) & (n - 1);
        for (int dx = -R; dx <= R; ++dx) {
          const int tc = (ic - dx - c0) & (n - 1);
          if (tc >= wl) continue;
          const int64_t s = static_cast<int64_t>(sr) * n + ((c0 + tc) & (n - 1));
          const double w = psf_unnormalised(P, s, dy, dx);
          if (w != 0.0) acc += (vr * fc[tc]) * (w / P.Z[s]);
        }
      }
      bufA[o] = acc;
    }
    __syncthreads();
    // Local analysis pyramid of the window.
    Win inr{hr0, hl, n}, inc{hc0, hl, n};
    double* in = bufA;
    double* ob = bufB;
    for (int lv = 1; lv <= G.J; ++lv) {
      const int M = n >> (lv - 1), Mh = M >> 1;
      const Win onr = next_win(inr, L), onc = next_win(inc, L);
      const int cnt = onr.len * onc.len;
      if (cnt > cap) {
        if (tid == 0) atomicOr(err, 1);
        break;
      }
      const int ks = 1 + (G.J - lv) * 3;
      for (int o = tid; o < cnt; o += nt) {
        const int oi = o / onc.len, oj = o - oi * onc.len;
        const int I = (onr.s + oi) & (Mh - 1), Jc = (onc.s + oj) & (Mh - 1);
        double a00 = 0.0, a01 = 0.0, a10 = 0.0, a11 = 0.0;
        for (int m = 0; m < L; ++m) {
          const int rr = (2 * I + m - inr.s) & (M - 1);
          if (rr >= inr.len) continue;
          const double* rowp = in + static_cast<size_t>(rr) * inc.len;
          double lo = 0.0, hi = 0.0;
          for (int m2 = 0; m2 < L; ++m2) {
            const int cc = (2 * Jc + m2 - inc.s) & (M - 1);
            if (cc >= inc.len) continue;
            const double v = rowp[cc];
            lo += G.h[m2] * v;
            hi += G.g[m2] * v;
          }
          a00 += G.h[m] * lo;
          a01 += G.h[m] * hi;
          a10 += G.g[m] * lo;
          a11 += G.g[m] * hi;
        }
        ob[o] = a00;
        const int64_t loc = static_cast<int64_t>(I) * Mh + Jc;
        handle(S, a01, sb, static_cast<int>(G.sub_off[ks] + loc), static_cast<int>(b), lhist, out, bnd, err);
        handle(S, a10, sb, static_cast<int>(G.sub_off[ks + 1] + loc), static_cast<int>(b), lhist, out, bnd, err);
        handle(S, a11, sb, static_cast<int>(G.sub_off[ks + 2] + loc), static_cast<int>(b), lhist, out, bnd, err);
        if (lv == G.J) handle(S, a00, sb, static_cast<int>(G.sub_off[0] + loc), static_cast<int>(b), lhist, out, bnd, err);
      }
      __syncthreads();
      double* t = in;
      in = ob;
      ob = t;
      inr = onr;
      inc = onc;
    }
  }
  if (S.mode == 0) {
    __syncthreads();
    for (int i = tid; i < kDigits; i += nt)
      if (lhist[i]) atomicAdd(&ghist[i], static_cast<unsigned long long>(lhist[i]));
  }
}

// Level-l equivalent filters (index l = 1..J): phi_l = cascade of h,
// psi_l = g applied after l-1 low-pass steps, periodised to length <= n.
void level_filters(const Filter& f, int n, int J, std::vector<double>& tab, Geom& G) {
  const int L = static_cast<int>(f.h.size());
  std::vector<double> phi{1.0};
  tab.clear();
  for (int l = 1; l <= J; ++l) {
    const int up = 1 << (l - 1);
    const int len = static_cast<int>(phi.size()) + up * (L - 1);
    std::vector<double> nphi(len, 0.0), npsi(len, 0.0);
    for (size_t t = 0; t < phi.size(); ++t)
      for (int m = 0; m < L; ++m) {
        nphi[t + up * m] += f.h[m] * phi[t];
        npsi[t + up * m] += f.g[m] * phi[t];
      }
    const int plen = std::min(len, n);
    std::vector<double> pphi(plen, 0.0), ppsi(plen, 0.0);
    for (int t = 0; t < len; ++t) {
      pphi[t % n] += nphi[t];
      ppsi[t % n] += npsi[t];
    }
    G.flen[l] = plen;
    G.foff[l] = static_cast<int64_t>(tab.size());
    tab.insert(tab.end(), pphi.begin(), pphi.end());
    tab.insert(tab.end(), ppsi.begin(), ppsi.end());
    phi.swap(nphi);
  }
}

// Largest window side reached anywhere in a column's pyramid.
int max_window_side(const Geom& G) {
  int best = 0;
  for (int l = 1; l <= G.J; ++l) {
    const int hl = std::min(G.flen[l] + 2 * G.R, G.n);
    best = std::max(best, hl);
    int cur_len = hl, M = G.n;
    for (int lv = 1; lv <= G.J; ++lv) {
      int worst = 0;
      for (int s = 0; s < 2; ++s) worst = std::max(worst, next_win(Win{s, cur_len, M}, G.L).len);
      cur_len = worst;
      M >>= 1;
      best = std::max(best, cur_len);
    }
  }
  return best;
}

struct Builder {
  Geom G{};
  PsfField psf;
  DevBuf<double> ftab, scratch;
  DevBuf<unsigned long long> hist, counters;
  DevBuf<int> err;
  int64_t cap = 0;
  int nwg = 0;
  hipStream_t s = nullptr;
  bool log = false;

  void run(const Select& S, Emit out, Emit bnd) {
    const int64_t N = static_cast<int64_t>(G.n) * G.n;
    const int64_t chunk = 32768;
    for (int64_t b0 = 0; b0 < N; b0 += chunk) {
      const int64_t b1 = std::min(N, b0 + chunk);
      hipLaunchKernelGGL(k_theta_columns, dim3(nwg), dim3(256), 0, s, G, psf.dev(), ftab.p, scratch.p, cap, b0,
                         b1, S, hist.p, out, bnd, err.p);
      WDB_HIP(hipGetLastError());
    }
    WDB_HIP(hipStreamSynchronize(s));
    int e = 0;
    WDB_HIP(hipMemcpy(&e, err.p, sizeof(int), hipMemcpyDeviceToHost));
    WDB_REQUIRE(e == 0, WDB_ERR_HIP, "theta build consistency check failed (code %d)", e);
  }
};

// ---------------------------------------------------------------------------
// Convolution fast path (Alg. 3; circulant subband blocks, Sec. 3.6).
//
// With the same PSF at every pixel, H is a circular convolution with a kernel
// symmetric under x -> -x (the Gaussian of psf.hip), so H = H^* and Theta is
// symmetric.  Every block (R, C) of Theta is then a rectangular circulant
// matrix generated by the column gamma_k = Psi^*(H psi_k0) of one atom per
// subband k:
//   * C coarser than R:  Theta[(R, p + r q), (C, q)] = gamma_C[(R, p)],
//   * C as fine as R or finer: Theta[(R, m), (C, p + r m)] = gamma_R[(C, p)]
// (r the ratio of the two sides, positions taken modulo the finer side).  So
// the 3J + 1 representative columns are computed exactly as the general
// build computes any column, each non-zero becomes a generator with a known
// number of copies, the K largest magnitudes are selected on the generators
// (equal magnitudes at the cut ordered by a * N + b like the general build)
// and the kept copies are written out in parallel.
// ---------------------------------------------------------------------------
bool field_is_stationary(const wdb_psf_field* f) {
  const int64_t N = static_cast<int64_t>(f->n) * f->n;
  for (int64_t i = 1; i < N; ++i)
    if (f->sig_major[i] != f->sig_major[0] || f->sig_minor[i] != f->sig_minor[0] || f->angle[i] != f->angle[0])
      return false;
  return true;
}

struct GenDev {
  int64_t off_k, off_b;  // subband offsets: k enumerates the copies, b holds the moving position
  int side_k, side_b;
  int p1, p2, r, form;   // form 0: row in k, column in b; 1: row in b, column in k
  double v;
};

__device__ __host__ inline void gen_entry(const GenDev& g, int64_t idx, int32_t* row, int32_t* col) {
  const int i1 = static_cast<int>(idx / g.side_k), i2 = static_cast<int>(idx % g.side_k);
  const int q1 = (g.p1 + g.r * i1) & (g.side_b - 1), q2 = (g.p2 + g.r * i2) & (g.side_b - 1);
  const int64_t ak = g.off_k + static_cast<int64_t>(i1) * g.side_k + i2;
  const int64_t ab = g.off_b + static_cast<int64_t>(q1) * g.side_b + q2;
  *row = static_cast<int32_t>(g.form == 0 ? ak : ab);
  *col = static_cast<int32_t>(g.form == 0 ? ab : ak);
}

__global__ void k_expand(const GenDev* __restrict__ gens, const int64_t* __restrict__ first, int ngen,
                         int64_t total, int32_t* __restrict__ row, int32_t* __restrict__ col,
                         double* __restrict__ val) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  int lo = 0, hi = ngen - 1;  // last generator with first[g] <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (first[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  gen_entry(gens[lo], t - first[lo], row + t, col + t);
  val[t] = gens[lo].v;
}

// Builds Theta_K of a stationary field; returns the handle's CSR pieces.
void build_stationary(Builder& B, int64_t nnz_budget, int scaled, unsigned long long* K_out, double* thr_out,
                      DevBuf<int32_t>& orow, DevBuf<int32_t>& ocol, DevBuf<double>& oval,
                      std::vector<CircGen>& kept, std::vector<int32_t>& tie_r, std::vector<int32_t>& tie_c,
                      std::vector<double>& tie_v) {
  const Geom& G = B.G;
  const int64_t N = static_cast<int64_t>(G.n) * G.n;
  hipStream_t s = B.s;
  // 1. representative columns gamma_k (every non-zero, float64)
  DevBuf<int32_t> er(N), ec(N);
  DevBuf<double> ev(N);
  std::vector<GenDev> gens;
  std::vector<int32_t> hr;
  std::vector<double> hv;
  auto band_of = [&](int64_t a) {
    int k = 0;
    while (k + 1 < G.nsub && a >= G.sub_off[k + 1]) ++k;
    return k;
  };
  for (int k = 0; k < G.nsub; ++k) {
    WDB_HIP(hipMemsetAsync(B.counters.p, 0, sizeof(unsigned long long), s));
    Emit out{er.p, ec.p, ev.p, B.counters.p, static_cast<unsigned long long>(N)};
    Emit none{nullptr, nullptr, nullptr, B.counters.p + 1, 0};
    Select S{2, 0, 0, 0, 0, 0};
    hipLaunchKernelGGL(k_theta_columns, dim3(1), dim3(256), 0, s, G, B.psf.dev(), B.ftab.p, B.scratch.p, B.cap,
                       G.sub_off[k], G.sub_off[k] + 1, S, B.hist.p, out, none, B.err.p);
    WDB_HIP(hipGetLastError());
    unsigned long long cnt = 0;
    WDB_HIP(hipMemcpyAsync(&cnt, B.counters.p, sizeof(cnt), hipMemcpyDeviceToHost, s));
    WDB_HIP(hipStreamSynchronize(s));
    int e = 0;
    WDB_HIP(hipMemcpy(&e, B.err.p, sizeof(int), hipMemcpyDeviceToHost));
    WDB_REQUIRE(e == 0 && cnt <= static_cast<unsigned long long>(N), WDB_ERR_HIP,
                "representative column %d failed (code %d)", k, e);
    hr.resize(cnt);
    hv.resize(cnt);
    WDB_HIP(hipMemcpy(hr.data(), er.p, cnt * sizeof(int32_t), hipMemcpyDeviceToHost));
    WDB_HIP(hipMemcpy(hv.data(), ev.p, cnt * sizeof(double), hipMemcpyDeviceToHost));
    const int sk = G.sub_side[k];
    for (unsigned long long i = 0; i < cnt; ++i) {
      const int b = band_of(hr[i]);
      const int sb = G.sub_side[b];
      const int64_t pos = hr[i] - G.sub_off[b];
      GenDev g{G.sub_off[k], G.sub_off[b], sk, sb, static_cast<int>(pos / sb), static_cast<int>(pos % sb),
               sb / sk, 0, hv[i]};
      if (sb > sk) {  // block (R = b, C = k), C coarser: copies over the columns of k
        g.form = 1;
        gens.push_back(g);
      }
      if (sb >= sk) {  // block (R = k, C = b), C as fine or finer: copies over the rows of k
        g.form = 0;
        gens.push_back(g);
      }
    }
  }
  // 2. the K largest (weighted) magnitudes over the generators and their copies
  auto mag = [scaled](const GenDev& g) {
    const int side_col = g.form == 0 ? g.side_b : g.side_k;
    return scaled ? std::fabs(g.v) / side_col : std::fabs(g.v);
  };
  std::sort(gens.begin(), gens.end(), [&](const GenDev& x, const GenDev& y) { return mag(x) > mag(y); });
  const unsigned long long budget = static_cast<unsigned long long>(nnz_budget);
  unsigned long long cum = 0;
  size_t full = 0;
  std::vector<std::pair<int64_t, std::pair<int32_t, int32_t>>> tie;  // (a*N + b, (a, b))
  double threshold = 0.0;
  std::vector<double> tie_val;
  while (full < gens.size()) {
    size_t e = full;
    unsigned long long grp = 0;
    while (e < gens.size() && mag(gens[e]) == mag(gens[full])) {
      grp += static_cast<unsigned long long>(gens[e].side_k) * gens[e].side_k;
      ++e;
    }
    if (cum + grp <= budget) {
      cum += grp;
      threshold = mag(gens[full]);
      full = e;
      continue;
    }
    // equal magnitudes straddle the cut: keep the smallest linear indices
    const unsigned long long need = budget - cum;
    if (need == 0) break;
    std::vector<std::pair<int64_t, size_t>> cand;  // (a*N + b, generator * 2^32 + copy)
    cand.reserve(grp);
    for (size_t g = full; g < e; ++g) {
      const int64_t m = static_cast<int64_t>(gens[g].side_k) * gens[g].side_k;
      for (int64_t i = 0; i < m; ++i) {
        int32_t a, b;
        gen_entry(gens[g], i, &a, &b);
        cand.push_back({static_cast<int64_t>(a) * N + b, ((g - full) << 32) | static_cast<size_t>(i)});
      }
    }
    std::nth_element(cand.begin(), cand.begin() + (need - 1), cand.end());
    for (unsigned long long i = 0; i < need; ++i) {
      const size_t g = full + (cand[i].second >> 32);
      tie.push_back({cand[i].first, {static_cast<int32_t>(cand[i].first / N), static_cast<int32_t>(cand[i].first % N)}});
      tie_val.push_back(gens[g].v);
    }
    threshold = mag(gens[full]);
    cum += need;
    break;
  }
  // 3. write the kept copies
  const unsigned long long K = cum;
  const int ngen = static_cast<int>(full);
  std::vector<int64_t> first(ngen + 1, 0);
  for (int g = 0; g < ngen; ++g) first[g + 1] = first[g] + static_cast<int64_t>(gens[g].side_k) * gens[g].side_k;
  orow.alloc(std::max<unsigned long long>(K, 1));
  ocol.alloc(std::max<unsigned long long>(K, 1));
  oval.alloc(std::max<unsigned long long>(K, 1));
  if (ngen > 0) {
    DevBuf<GenDev> dg(ngen);
    DevBuf<int64_t> df(ngen + 1);
    WDB_HIP(hipMemcpy(dg.p, gens.data(), ngen * sizeof(GenDev), hipMemcpyHostToDevice));
    WDB_HIP(hipMemcpy(df.p, first.data(), (ngen + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    const int64_t tot = first[ngen];
    hipLaunchKernelGGL(k_expand, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s, dg.p, df.p, ngen,
                       tot, orow.p, ocol.p, oval.p);
    WDB_HIP(hipGetLastError());
    WDB_HIP(hipStreamSynchronize(s));
  }
  if (!tie.empty()) {
    std::vector<int32_t> tr(tie.size()), tc(tie.size());
    for (size_t i = 0; i < tie.size(); ++i) {
      tr[i] = tie[i].second.first;
      tc[i] = tie[i].second.second;
    }
    const int64_t at = first[ngen];
    WDB_HIP(hipMemcpy(orow.p + at, tr.data(), tie.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    WDB_HIP(hipMemcpy(ocol.p + at, tc.data(), tie.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    WDB_HIP(hipMemcpy(oval.p + at, tie_val.data(), tie.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  kept.clear();
  for (int g = 0; g < ngen; ++g) {
    const GenDev& d = gens[g];
    kept.push_back(CircGen{d.off_k, d.off_b, d.side_k, d.side_b, d.p1, d.p2, d.r, d.form, d.v});
  }
  tie_r.clear();
  tie_c.clear();
  tie_v.clear();
  for (size_t i = 0; i < tie.size(); ++i) {
    tie_r.push_back(tie[i].second.first);
    tie_c.push_back(tie[i].second.second);
    tie_v.push_back(tie_val[i]);
  }
  *K_out = K;
  *thr_out = threshold;
}

}  // namespace

}  // namespace wdb

extern "C" wdb_status wdb_build_theta(const wdb_psf_field* field, int32_t wavelet, int32_t levels,
                                      int64_t nnz_budget, void* stream, wdb_theta** out) {
  return wdb_build_theta_rule(field, wavelet, levels, nnz_budget, WDB_THRESH_NAIVE, stream, out);
}

extern "C" wdb_status wdb_build_theta_rule(const wdb_psf_field* field, int32_t wavelet, int32_t levels,
                                           int64_t nnz_budget, int32_t rule, void* stream, wdb_theta** out) {
  using namespace wdb;
  WDB_API_BEGIN
  WDB_REQUIRE(field && out, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(rule == WDB_THRESH_NAIVE || rule == WDB_THRESH_SCALE, WDB_ERR_ARG, "unknown thresholding rule %d", rule);
  const int scaled = rule == WDB_THRESH_SCALE ? 1 : 0;
  const Filter f = make_filter(wavelet);
  const int n = field->n;
  check_geometry(n, levels, static_cast<int>(f.h.size()));
  WDB_REQUIRE(levels < kMaxLev && 3 * levels + 1 <= kMaxSub, WDB_ERR_LEVELS, "too many levels");
  const int64_t N = static_cast<int64_t>(n) * n;
  WDB_REQUIRE(nnz_budget >= 1 && nnz_budget <= N * N, WDB_ERR_ARG, "nnz_budget %lld outside [1, N^2]",
              static_cast<long long>(nnz_budget));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Builder B;
  B.s = s;
  B.log = std::getenv("WDB_LOG") != nullptr;
  B.psf.upload(field, s);  // validates the field before any device call
  int dev = 0;
  WDB_HIP(hipGetDevice(&dev));
  Geom& G = B.G;
  G.n = n;
  G.J = levels;
  G.L = static_cast<int>(f.h.size());
  G.R = B.psf.R;
  const std::vector<Subband> lay = layout(n, levels);
  G.nsub = static_cast<int>(lay.size());
  for (int k = 0; k < G.nsub; ++k) {
    G.sub_level[k] = lay[k].level;
    G.sub_er[k] = lay[k].erow;
    G.sub_ec[k] = lay[k].ecol;
    G.sub_side[k] = lay[k].side;
    G.sub_off[k] = lay[k].offset;
  }
  G.sub_off[G.nsub] = N;
  for (int m = 0; m < G.L; ++m) {
    G.h[m] = f.h[m];
    G.g[m] = f.g[m];
  }
  std::vector<double> tab;
  level_filters(f, n, levels, tab, G);
  B.ftab.alloc(tab.size());
  WDB_HIP(hipMemcpy(B.ftab.p, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
  const int side = max_window_side(G);
  B.cap = static_cast<int64_t>(side) * side;
  B.nwg = static_cast<int>(std::min<int64_t>(1024, N));
  B.scratch.alloc(static_cast<size_t>(B.nwg) * 2 * B.cap);
  B.hist.alloc(kDigits);
  B.counters.alloc(2);
  B.err.alloc(1);
  WDB_HIP(hipMemset(B.err.p, 0, sizeof(int)));

  const char* force_general = std::getenv("WDB_BUILD_GENERAL");
  if (field_is_stationary(field) && !(force_general && *force_general == '1')) {
    unsigned long long K = 0;
    double threshold = 0.0;
    DevBuf<int32_t> orow, ocol;
    DevBuf<double> oval;
    std::vector<CircGen> kept;
    std::vector<int32_t> tie_r, tie_c;
    std::vector<double> tie_v;
    build_stationary(B, nnz_budget, scaled, &K, &threshold, orow, ocol, oval, kept, tie_r, tie_c, tie_v);
    B.scratch.reset();
    wdb_theta* th = new wdb_theta();
    try {
      th->device = dev;
      th->n = n;
      th->levels = levels;
      th->wavelet = wavelet;
      th->N = N;
      th->nnz = static_cast<int64_t>(K);
      th->threshold = threshold;
      th->conv_build = 1;
      th->rule = rule;
      coo_to_csr(N, th->nnz, orow.p, ocol.p, oval.p, &th->csr, s);
      finish_theta(th, s);
      build_stencils(th, kept, tie_r, tie_c, tie_v);
    } catch (...) {
      wdb_theta_free(th);
      throw;
    }
    *out = th;
    return WDB_OK;
  }

  Emit none{nullptr, nullptr, nullptr, B.counters.p, 0};
  // Radix select of the nnz_budget-th largest |theta|.
  unsigned long long need = static_cast<unsigned long long>(nnz_budget);
  unsigned long long prefix = 0, bcount = 0, total = 0;
  int pbits = 0;
  bool keep_all = false;
  std::vector<unsigned long long> h(kDigits);
  while (true) {
    const int w = std::min(12, 64 - pbits);
    Select S{0, scaled, pbits, 64 - pbits - w, prefix, (1ull << w) - 1ull};
    WDB_HIP(hipMemsetAsync(B.hist.p, 0, kDigits * sizeof(unsigned long long), s));
    B.run(S, none, none);
    WDB_HIP(hipMemcpy(h.data(), B.hist.p, kDigits * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    if (pbits == 0) {
      total = std::accumulate(h.begin(), h.end(), 0ull);
      if (total <= need) {
        keep_all = true;
        break;
      }
    }
    unsigned long long cum = 0;
    int digit = -1;
    for (int d = (1 << w) - 1; d >= 0; --d) {
      if (cum + h[d] >= need) {
        digit = d;
        break;
      }
      cum += h[d];
    }
    WDB_REQUIRE(digit >= 0, WDB_ERR_HIP, "radix select lost entries");
    need -= cum;
    prefix = (prefix << w) | static_cast<unsigned long long>(digit);
    pbits += w;
    bcount = h[digit];
    if (B.log)
      std::fprintf(stderr, "[wdb] build: digit pass %d bits, boundary %llu, need %llu\n", pbits, bcount, need);
    if (bcount <= kBoundaryCap || pbits >= 64) break;
  }
  const unsigned long long K = keep_all ? total : static_cast<unsigned long long>(nnz_budget);
  const unsigned long long above = keep_all ? total : K - need;
  DevBuf<int32_t> orow(K), ocol(K);
  DevBuf<double> oval(K);
  DevBuf<int32_t> brow(keep_all ? 0 : bcount), bcol(keep_all ? 0 : bcount);
  DevBuf<double> bval(keep_all ? 0 : bcount);
  WDB_HIP(hipMemsetAsync(B.counters.p, 0, 2 * sizeof(unsigned long long), s));
  Emit eo{orow.p, ocol.p, oval.p, B.counters.p, above};
  Emit eb{brow.p, bcol.p, bval.p, B.counters.p + 1, keep_all ? 0 : bcount};
  Select S{keep_all ? 2 : 1, scaled, pbits, 0, prefix, 0};
  B.run(S, eo, eb);
  unsigned long long cnt[2];
  WDB_HIP(hipMemcpy(cnt, B.counters.p, sizeof(cnt), hipMemcpyDeviceToHost));
  WDB_REQUIRE(cnt[0] == above && (keep_all || cnt[1] == bcount), WDB_ERR_HIP,
              "theta emit pass produced %llu/%llu entries, expected %llu/%llu", cnt[0], cnt[1], above, bcount);
  double threshold = 0.0;
  if (!keep_all) {
    // Order the boundary digit: |theta| descending, then linear index ascending.
    std::vector<int32_t> hr(bcount), hc(bcount);
    std::vector<double> hv(bcount);
    WDB_HIP(hipMemcpy(hr.data(), brow.p, bcount * sizeof(int32_t), hipMemcpyDeviceToHost));
    WDB_HIP(hipMemcpy(hc.data(), bcol.p, bcount * sizeof(int32_t), hipMemcpyDeviceToHost));
    WDB_HIP(hipMemcpy(hv.data(), bval.p, bcount * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<size_t> idx(bcount);
    std::iota(idx.begin(), idx.end(), size_t(0));
    const std::vector<Subband> lay = layout(n, levels);
    auto rank = [&](size_t x) {  // the ranked magnitude (times sigma_b of the column when scaled)
      if (!scaled) return std::fabs(hv[x]);
      int k = 0;
      while (k + 1 < static_cast<int>(lay.size()) && hc[x] >= lay[k + 1].offset) ++k;
      return std::fabs(hv[x]) / lay[k].side;
    };
    std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
      const double ax = rank(x), ay = rank(y);
      if (ax != ay) return ax > ay;
      return static_cast<int64_t>(hr[x]) * N + hc[x] < static_cast<int64_t>(hr[y]) * N + hc[y];
    });
    std::vector<int32_t> sr(need), sc(need);
    std::vector<double> sv(need);
    for (unsigned long long i = 0; i < need; ++i) {
      sr[i] = hr[idx[i]];
      sc[i] = hc[idx[i]];
      sv[i] = hv[idx[i]];
    }
    threshold = rank(idx[need - 1]);
    WDB_HIP(hipMemcpy(orow.p + above, sr.data(), need * sizeof(int32_t), hipMemcpyHostToDevice));
    WDB_HIP(hipMemcpy(ocol.p + above, sc.data(), need * sizeof(int32_t), hipMemcpyHostToDevice));
    WDB_HIP(hipMemcpy(oval.p + above, sv.data(), need * sizeof(double), hipMemcpyHostToDevice));
  }
  B.scratch.reset();

  wdb_theta* th = new wdb_theta();
  try {
    th->device = dev;
    th->n = n;
    th->levels = levels;
    th->wavelet = wavelet;
    th->N = N;
    th->nnz = static_cast<int64_t>(K);
    th->threshold = threshold;
    th->rule = rule;
    coo_to_csr(N, th->nnz, orow.p, ocol.p, oval.p, &th->csr, s);
    finish_theta(th, s);
  } catch (...) {
    wdb_theta_free(th);
    throw;
  }
  *out = th;
  WDB_API_END
}
