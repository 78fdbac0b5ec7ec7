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
  double h[8], g[8];
};

struct Select {
  int mode;   // 0: histogram, 1: emit above prefix + collect prefix, 2: emit every non-zero
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

__device__ inline void handle(const Select& S, double v, int a, int b, unsigned* lhist, const Emit& out,
                              const Emit& bnd, int* err) {
  const bool nz = v != 0.0;
  const unsigned long long key = static_cast<unsigned long long>(__double_as_longlong(fabs(v)));
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
        handle(S, a01, static_cast<int>(G.sub_off[ks] + loc), static_cast<int>(b), lhist, out, bnd, err);
        handle(S, a10, static_cast<int>(G.sub_off[ks + 1] + loc), static_cast<int>(b), lhist, out, bnd, err);
        handle(S, a11, static_cast<int>(G.sub_off[ks + 2] + loc), static_cast<int>(b), lhist, out, bnd, err);
        if (lv == G.J) handle(S, a00, static_cast<int>(G.sub_off[0] + loc), static_cast<int>(b), lhist, out, bnd, err);
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

}  // namespace

}  // namespace wdb

extern "C" wdb_status wdb_build_theta(const wdb_psf_field* field, int32_t wavelet, int32_t levels,
                                      int64_t nnz_budget, void* stream, wdb_theta** out) {
  using namespace wdb;
  WDB_API_BEGIN
  WDB_REQUIRE(field && out, WDB_ERR_ARG, "null argument");
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

  Emit none{nullptr, nullptr, nullptr, B.counters.p, 0};
  // Radix select of the nnz_budget-th largest |theta|.
  unsigned long long need = static_cast<unsigned long long>(nnz_budget);
  unsigned long long prefix = 0, bcount = 0, total = 0;
  int pbits = 0;
  bool keep_all = false;
  std::vector<unsigned long long> h(kDigits);
  while (true) {
    const int w = std::min(12, 64 - pbits);
    Select S{0, pbits, 64 - pbits - w, prefix, (1ull << w) - 1ull};
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
  Select S{keep_all ? 2 : 1, pbits, 0, prefix, 0};
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
    std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
      const double ax = std::fabs(hv[x]), ay = std::fabs(hv[y]);
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
    threshold = std::fabs(sv[need - 1]);
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
    coo_to_csr(N, th->nnz, orow.p, ocol.p, oval.p, &th->csr, s);
    finish_theta(th, s);
  } catch (...) {
    wdb_theta_free(th);
    throw;
  }
  *out = th;
  WDB_API_END
}
