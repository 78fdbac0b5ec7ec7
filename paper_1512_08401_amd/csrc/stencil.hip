// Circulant storage of Theta_K for a convolution (the second half of the
// fast path of Alg. 3; circulant subband blocks, Sec. 3.6).
//
// The fast build keeps whole circulant copies of generators: an entry of the
// representative column of subband k at position p of subband b stands for
// every entry of one block at the same relative offset.  For a row subband R
// and a column subband C (side s_R, s_C) these are
//   form 0 (C as fine or finer, r = s_C / s_R): row (R, m) -> column
//          (C, (p + r m) mod s_C), present in every row of R;
//   form 1 (C coarser, r = s_R / s_C): rows (R, p + r q) -> column (C, q), so a
//          row m of R holds it iff m = p (mod r) on both axes, with
//          q = ((m - p) mod s_R) / r.
// So the product needs no per-entry index or value stream: per row subband, a
// list of segments (one per column subband and form), each a list of
// (offset, value) generators shared by all rows (form 1: bucketed by the
// residue class of p mod r).  Entries of the cut's partial tie group, which
// break the circulant pattern, are kept per row in a short explicit list.
// Generators are (offset, value) pairs in lists padded to groups of 4; G
// lanes per row take turns on the groups (two 16-byte loads each), float32
// accumulation in a fixed order, butterfly reduction.
#include <algorithm>
#include <cstring>
#include <map>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "prox.hpp"

namespace wdb {

namespace {

constexpr int kBlock = 256;

struct SegDev {
  int form;      // 0 or 1 (see above)
  int off;       // offset of the column subband
  int sc_log2;   // log2 side of the column subband
  int r_log2;    // log2 of the side ratio
  int start;     // form 0: first generator; form 1: first entry of the residue table
  int count;     // form 0: number of generators; form 1: unused
};

struct StencilView {
  const int* __restrict__ seg_ptr;  // per row subband
  const SegDev* __restrict__ seg;
  const int4* __restrict__ g4;      // generators, two per int4: ((p1 << 16) | p2, value bits)
  const int* __restrict__ res;      // residue tables (absolute generator indices, multiples of 4)
  const int* __restrict__ xrp;      // explicit entries per row (null if none)
  const int* __restrict__ xc;
  const float* __restrict__ xv;
  int64_t nrows;
  int logn, J;
};

StencilView sview(const Stencil& s, const wdb_theta* th) {
  int logn = 0;
  while ((1 << logn) < th->n) ++logn;
  return StencilView{s.seg_ptr, reinterpret_cast<const SegDev*>(s.seg), reinterpret_cast<const int4*>(s.gp), s.res,
                     s.xrp, s.xc, s.xv, th->N, logn, th->levels};
}

// Subband index, level and position of canonical index r (power-of-two side).
__device__ __forceinline__ void locate(const StencilView& S, int64_t r, int* band, int* ls, int* m1, int* m2) {
  const int lsJ = S.logn - S.J;
  if (r < (int64_t{1} << (2 * lsJ))) {
    *band = 0;
    *ls = lsJ;
    *m1 = static_cast<int>(r >> lsJ);
    *m2 = static_cast<int>(r & ((int64_t{1} << lsJ) - 1));
    return;
  }
  const int l2 = (63 - __builtin_clzll(static_cast<unsigned long long>(r))) >> 1;
  const int o = static_cast<int>(r >> (2 * l2)) - 1;
  const int64_t p = r - (static_cast<int64_t>(o) + 1) * (int64_t{1} << (2 * l2));
  *band = 1 + 3 * (l2 - lsJ) + o;  // 1 + 3 (J - level) + o with level = logn - l2
  *ls = l2;
  *m1 = static_cast<int>(p >> l2);
  *m2 = static_cast<int>(p & ((int64_t{1} << l2) - 1));
}

// Generator lists are padded to groups of 4 (value 0, offset 0, which maps to
// a valid column); a lane loads a group as two 16-byte words.
__device__ __forceinline__ int col0(const SegDev& sg, int p, int b1, int b2, int mc) {
  return sg.off + ((((p >> 16) + b1) & mc) << sg.sc_log2) + (((p & 0xFFFF) + b2) & mc);
}

__device__ __forceinline__ int col1(const SegDev& sg, int p, int m1, int m2, int mR) {
  const int q1 = ((m1 - (p >> 16)) & mR) >> sg.r_log2, q2 = ((m2 - (p & 0xFFFF)) & mR) >> sg.r_log2;
  return sg.off + (q1 << sg.sc_log2) + q2;
}

template <int G>
__device__ __forceinline__ float stencil_dot(const StencilView& S, int64_t row, int gl, const float* __restrict__ x) {
  float acc = 0.f;
  if (row < S.nrows) {
    int band, lsR, m1, m2;
    locate(S, row, &band, &lsR, &m1, &m2);
    const int mR = (1 << lsR) - 1;
    for (int s = S.seg_ptr[band]; s < S.seg_ptr[band + 1]; ++s) {
      const SegDev sg = S.seg[s];
      int lo, hi;
      if (sg.form == 0) {
        lo = sg.start;
        hi = sg.start + sg.count;
      } else {
        const int rm = (1 << sg.r_log2) - 1;
        const int cls = ((m1 & rm) << sg.r_log2) | (m2 & rm);
        lo = S.res[sg.start + cls];
        hi = S.res[sg.start + cls + 1];
      }
      const int mc = (1 << sg.sc_log2) - 1;
      const int b1 = m1 << sg.r_log2, b2 = m2 << sg.r_log2;
      for (int t = (lo >> 2) + gl; t < (hi >> 2); t += G) {
        const int4 a = S.g4[2 * t], b = S.g4[2 * t + 1];
        const int ps[4] = {a.x, a.z, b.x, b.z};
        const int vs[4] = {a.y, a.w, b.y, b.w};
        int c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = sg.form == 0 ? col0(sg, ps[u], b1, b2, mc) : col1(sg, ps[u], m1, m2, mR);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = fmaf(__int_as_float(vs[u]), x[c[u]], acc);
      }
    }
    if (S.xrp)
      for (int t = S.xrp[row] + gl; t < S.xrp[row + 1]; t += G) acc = fmaf(S.xv[t], x[S.xc[t]], acc);
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
  return acc;
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_res_st(StencilView S, const float* __restrict__ y,
                                                   const float* __restrict__ b, float* __restrict__ r,
                                                   int* __restrict__ kdev) {
  if (kdev && blockIdx.x == 0 && threadIdx.x == 0) *kdev += 1;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / G) + threadIdx.x / G;
  const int gl = threadIdx.x % G;
  const float acc = stencil_dot<G>(S, row, gl, y);
  if (gl == 0 && row < S.nrows) r[row] = b ? acc - b[row] : acc;
}

template <int G, bool PRE>
__global__ __launch_bounds__(kBlock) void k_prox_st(StencilView S, const float* __restrict__ r,
                                                    float* __restrict__ x, float* __restrict__ y, float tau,
                                                    float thr, float beta, const int* __restrict__ kdev,
                                                    const float* __restrict__ pinv, const float* __restrict__ tw,
                                                    const double* __restrict__ anc) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / G) + threadIdx.x / G;
  const int gl = threadIdx.x % G;
  const float g = stencil_dot<G>(S, row, gl, r);
  if (gl != 0 || row >= S.nrows) return;
  if (kdev) {
    const int k = *kdev;
    beta = static_cast<float>((static_cast<double>(k) - 1.0) / (static_cast<double>(k) + 2.0));
  }
  const float pi = PRE ? pinv[row] : 1.0f;
  const float sg = (tau * pi) * g;
  const float t = thr * (tw ? tw[row] : pi);
  const float xn = anc ? prox_anchored(anc[row], y[row], sg, t) : prox_plain(y[row], sg, t);
  const float xo = x[row];
  x[row] = xn;
  y[row] = xn + beta * (xn - xo);
}

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Tables of one matrix.  gens: generators with (row band, column band) roles
// already resolved: form, row band R, column band C, sides, p, r, value.
struct Gen {
  int R, C, form, p1, p2, r_log2, sc_log2;
  float v;
};

void upload_stencil(const std::vector<Gen>& gens, int nsub, int64_t N, const std::vector<int32_t>& xr,
                    const std::vector<int32_t>& xcol, const std::vector<float>& xval, const std::vector<int64_t>& off,
                    Stencil* out) {
  // group: row band, then (column band, form); form 1 gens bucketed by residue class
  std::map<std::pair<int, std::pair<int, int>>, std::vector<const Gen*>> groups;
  for (const Gen& g : gens) groups[{g.R, {g.C, g.form}}].push_back(&g);
  std::vector<int> seg_ptr(nsub + 1, 0);
  std::vector<SegDev> segs;
  std::vector<int> gp, res;  // gp: (offset, value bits) pairs, lists padded to groups of 4
  auto push = [&](const Gen* g) {
    gp.push_back((g->p1 << 16) | g->p2);
    int vb;
    std::memcpy(&vb, &g->v, sizeof(vb));
    gp.push_back(vb);
  };
  auto pad4 = [&]() {
    while ((gp.size() / 2) % 4 != 0) {
      gp.push_back(0);
      gp.push_back(0);  // value 0.0f
    }
  };
  for (int R = 0; R < nsub; ++R) {
    seg_ptr[R] = static_cast<int>(segs.size());
    for (auto it = groups.lower_bound({R, {-1, -1}}); it != groups.end() && it->first.first == R; ++it) {
      const int C = it->first.second.first, form = it->first.second.second;
      const auto& lst = it->second;
      SegDev sd{form, static_cast<int>(off[C]), lst[0]->sc_log2, lst[0]->r_log2, 0, 0};
      if (form == 0) {
        sd.start = static_cast<int>(gp.size() / 2);
        for (const Gen* g : lst) push(g);
        pad4();
        sd.count = static_cast<int>(gp.size() / 2) - sd.start;
      } else {
        const int r = 1 << sd.r_log2;
        std::vector<std::vector<const Gen*>> cls(static_cast<size_t>(r) * r);
        for (const Gen* g : lst) cls[static_cast<size_t>((g->p1 & (r - 1)) * r + (g->p2 & (r - 1)))].push_back(g);
        sd.start = static_cast<int>(res.size());
        for (auto& c : cls) {
          res.push_back(static_cast<int>(gp.size() / 2));
          for (const Gen* g : c) push(g);
          pad4();
        }
        res.push_back(static_cast<int>(gp.size() / 2));
      }
      segs.push_back(sd);
    }
  }
  seg_ptr[nsub] = static_cast<int>(segs.size());
  Stencil s;
  s.nseg = static_cast<int64_t>(segs.size());
  s.ngen = static_cast<int64_t>(gp.size() / 2);
  try {
    auto up = [](auto** dst, const auto& v) {
      using T = std::remove_reference_t<decltype(v[0])>;
      const size_t n = std::max<size_t>(v.size(), 1);
      WDB_HIP(hipMalloc(reinterpret_cast<void**>(dst), n * sizeof(T)));
      if (!v.empty()) WDB_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    };
    up(&s.seg_ptr, seg_ptr);
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&s.seg), std::max<size_t>(segs.size(), 1) * sizeof(SegDev)));
    if (!segs.empty()) WDB_HIP(hipMemcpy(s.seg, segs.data(), segs.size() * sizeof(SegDev), hipMemcpyHostToDevice));
    up(&s.gp, gp);
    up(&s.res, res);
    if (!xr.empty()) {
      // explicit entries: CSR over all rows
      std::vector<int> order(xr.size());
      for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
      std::sort(order.begin(), order.end(), [&](int a, int b) {
        return xr[a] != xr[b] ? xr[a] < xr[b] : xcol[a] < xcol[b];
      });
      std::vector<int> xrp(N + 1, 0), xc(xr.size());
      std::vector<float> xv(xr.size());
      for (size_t i = 0; i < order.size(); ++i) {
        xrp[xr[order[i]] + 1]++;
        xc[i] = xcol[order[i]];
        xv[i] = xval[order[i]];
      }
      for (int64_t i = 0; i < N; ++i) xrp[i + 1] += xrp[i];
      up(&s.xrp, xrp);
      up(&s.xc, xc);
      up(&s.xv, xv);
      s.nextra = static_cast<int64_t>(xr.size());
    }
  } catch (...) {
    s.free_all();
    throw;
  }
  out->free_all();
  *out = s;
}

}  // namespace

void Stencil::free_all() {
  void* ps[] = {seg_ptr, seg, gp, res, xrp, xc, xv};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  seg_ptr = nullptr;
  seg = nullptr;
  gp = nullptr;
  res = nullptr;
  xrp = nullptr;
  xc = nullptr;
  xv = nullptr;
  nseg = ngen = nextra = 0;
}

void build_stencils(wdb_theta* th, const std::vector<CircGen>& gens, const std::vector<int32_t>& tr,
                    const std::vector<int32_t>& tc, const std::vector<double>& tv) {
  const std::vector<Subband> lay = layout(th->n, th->levels);
  const int nsub = static_cast<int>(lay.size());
  std::vector<int64_t> off(nsub);
  std::map<int64_t, int> band_at;
  for (int k = 0; k < nsub; ++k) {
    off[k] = lay[k].offset;
    band_at[lay[k].offset] = k;
  }
  std::vector<Gen> a, at;
  a.reserve(gens.size());
  at.reserve(gens.size());
  for (const CircGen& g : gens) {
    const int k = band_at.at(g.off_k), b = band_at.at(g.off_b);
    const int rl = ilog2(g.r);
    const float v = static_cast<float>(g.v);
    // in Theta_K: form 0 = rows in k, columns in b; form 1 = rows in b, columns in k
    if (g.form == 0) {
      a.push_back(Gen{k, b, 0, g.p1, g.p2, rl, ilog2(g.side_b), v});
      at.push_back(Gen{b, k, 1, g.p1, g.p2, rl, ilog2(g.side_k), v});
    } else {
      a.push_back(Gen{b, k, 1, g.p1, g.p2, rl, ilog2(g.side_k), v});
      at.push_back(Gen{k, b, 0, g.p1, g.p2, rl, ilog2(g.side_b), v});
    }
  }
  std::vector<float> fv(tv.size());
  for (size_t i = 0; i < tv.size(); ++i) fv[i] = static_cast<float>(tv[i]);
  upload_stencil(a, nsub, th->N, tr, tc, fv, off, &th->st);
  upload_stencil(at, nsub, th->N, tc, tr, fv, off, &th->stT);
}

void launch_res_stencil(const wdb_theta* th, bool transpose, const float* y, const float* b, float* r, int* kdev,
                        hipStream_t s) {
  const StencilView S = sview(transpose ? th->stT : th->st, th);
  constexpr int G = 4;
  const dim3 grid(static_cast<unsigned>((S.nrows + kBlock / G - 1) / (kBlock / G)));
  hipLaunchKernelGGL(k_res_st<G>, grid, dim3(kBlock), 0, s, S, y, b, r, kdev);
}

void launch_prox_stencil(const wdb_theta* th, const float* r, float* x, float* y, float tau, float thr, float beta,
                         const int* kdev, const float* pinv, const float* tw, const double* anc, hipStream_t s) {
  const StencilView S = sview(th->stT, th);
  constexpr int G = 4;
  const dim3 grid(static_cast<unsigned>((S.nrows + kBlock / G - 1) / (kBlock / G)));
  if (pinv)
    hipLaunchKernelGGL((k_prox_st<G, true>), grid, dim3(kBlock), 0, s, S, r, x, y, tau, thr, beta, kdev, pinv, tw,
                       anc);
  else
    hipLaunchKernelGGL((k_prox_st<G, false>), grid, dim3(kBlock), 0, s, S, r, x, y, tau, thr, beta, kdev, pinv, tw,
                       anc);
}

}  // namespace wdb
