// Exact-operator baseline (Sec. 1.2; the "Exact" columns of the experiments
// of Sec. 5): Alg. 1 on the wavelet coefficients with the gradient of
// 1/2 ||H Psi x - u0||^2 computed from the blur itself rather than from the
// thresholded Theta_K:
//
//   g = Psi^* H^* (H Psi y - u0)    (synthesis, blur, adjoint blur, analysis)
//
// For a spatially varying PSF there is no fast exact H (the paper's FFT
// applies to convolutions only), so both products evaluate the truncated
// PSFs on the fly from the field: H u gathers, for each target pixel, the
// sources whose ellipse can reach it (a box bounded per 16 x 16 tile); H^* r
// sums, for each source, r over its own ellipse's bounding box.  The PSF
// weights are computed in float64 with the formula of psf.hpp (the same
// cut-off decisions as the field's blur), accumulated in float64; images
// and coefficients are float32.  Because Psi is orthogonal, Psi^* H Psi is
// the untruncated Theta, so this solves the problem before thresholding.
#include <algorithm>
#include <cmath>
#include <functional>
#include <vector>

#include "common.hpp"
#include "prox.hpp"
#include "psf.hpp"

struct wdb_exact {
  int device = 0;
  int32_t n = 0, levels = 0, wavelet = 0;
  int64_t N = 0;
  wdb::PsfField F;
  wdb::DevBuf<int2> box;      // per source: half-widths (hx, hy) of its ellipse's bounding box
  wdb::DevBuf<int2> tbox;     // per 16 x 16 tile of sources: the largest half-widths
  int ntile = 0;              // tiles per side
  bool has_L = false;
  double L = 0.0;
  // workspace
  wdb::DevBuf<float> u0, y, img, r, gimg, g, sa, sb;
  wdb::DevBuf<double> part, scal;
  double* host = nullptr;     // pinned, 4 doubles
};

namespace wdb {
namespace {

constexpr int kT = 16;        // tile side of the products
constexpr int kThreads = kT * kT;

// Bounding box of source s's truncated ellipse: |dx| <= trunc sqrt(a^2 c^2 + b^2 s^2),
// |dy| <= trunc sqrt(a^2 s^2 + b^2 c^2); one more pixel of margin (the
// weight test itself decides), at most the field radius.
__global__ __launch_bounds__(256) void k_exact_box(PsfDev P, int2* __restrict__ box) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t N = static_cast<int64_t>(P.n) * P.n;
  if (s >= N) return;
  const double a = P.sM[s], b = P.sm[s], c = P.c[s], sn = P.s[s];
  const int hx = static_cast<int>(floor(P.trunc * sqrt(a * a * c * c + b * b * sn * sn))) + 1;
  const int hy = static_cast<int>(floor(P.trunc * sqrt(a * a * sn * sn + b * b * c * c))) + 1;
  box[s] = make_int2(min(hx, P.R), min(hy, P.R));
}

// Largest half-widths over each tile of sources.
__global__ __launch_bounds__(256) void k_exact_tbox(const int2* __restrict__ box, int n, int ntile,
                                                    int2* __restrict__ tbox) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntile * ntile) return;
  const int tr = t / ntile, tc = t % ntile;
  int hx = 0, hy = 0;
  for (int r = tr * kT; r < min(n, (tr + 1) * kT); ++r)
    for (int c = tc * kT; c < min(n, (tc + 1) * kT); ++c) {
      const int2 b = box[static_cast<int64_t>(r) * n + c];
      hx = max(hx, b.x);
      hy = max(hy, b.y);
    }
  tbox[t] = make_int2(hx, hy);
}

// out[i] = sum over sources s of k_s(i - s) in[s]  (- sub[i]): for the target
// tile of this block, the offsets searched are bounded by the largest boxes
// of the source tiles within the field radius.
template <typename TI, typename TO>
__global__ __launch_bounds__(kThreads) void k_exact_fwd(PsfDev P, const int2* __restrict__ tbox, int ntile,
                                                        const TI* __restrict__ in, const float* __restrict__ sub,
                                                        TO* __restrict__ out) {
  __shared__ int2 hb;
  const int n = P.n;
  const int tr = blockIdx.y, tc = blockIdx.x;
  if (threadIdx.x == 0) {
    const int reach = P.R / kT + 1;
    int hx = 0, hy = 0;
    for (int dr = -reach; dr <= reach; ++dr)
      for (int dc = -reach; dc <= reach; ++dc) {
        const int2 b = tbox[((tr + dr + ntile) % ntile) * ntile + (tc + dc + ntile) % ntile];
        hx = max(hx, b.x);
        hy = max(hy, b.y);
      }
    hb = make_int2(hx, hy);
  }
  __syncthreads();
  const int ir = tr * kT + static_cast<int>(threadIdx.x) / kT;
  const int ic = tc * kT + static_cast<int>(threadIdx.x) % kT;
  if (ir >= n || ic >= n) return;
  const int hx = hb.x, hy = hb.y;
  double acc = 0.0;
  for (int dy = -hy; dy <= hy; ++dy) {
    const int sr = (ir - dy + n) & (n - 1);
    for (int dx = -hx; dx <= hx; ++dx) {
      const int sc = (ic - dx + n) & (n - 1);
      const int64_t s = static_cast<int64_t>(sr) * n + sc;
      const double w = psf_unnormalised(P, s, dy, dx);
      if (w != 0.0) acc += (w / P.Z[s]) * static_cast<double>(in[s]);
    }
  }
  const int64_t i = static_cast<int64_t>(ir) * n + ic;
  out[i] = static_cast<TO>(sub ? acc - static_cast<double>(sub[i]) : acc);
}

// out[s] = sum_d k_s(d) in[s + d]  (H^*), over the source's own box.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_exact_adj(PsfDev P, const int2* __restrict__ box,
                                                   const TI* __restrict__ in, TO* __restrict__ out) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int n = P.n;
  const int64_t N = static_cast<int64_t>(n) * n;
  if (s >= N) return;
  const int sr = static_cast<int>(s / n), sc = static_cast<int>(s % n);
  const int2 b = box[s];
  const double iz = 1.0 / P.Z[s];
  double acc = 0.0;
  for (int dy = -b.y; dy <= b.y; ++dy) {
    const int64_t row = static_cast<int64_t>((sr + dy + n) & (n - 1)) * n;
    for (int dx = -b.x; dx <= b.x; ++dx) {
      const double w = psf_unnormalised(P, s, dy, dx);
      if (w != 0.0) acc += w * static_cast<double>(in[row + ((sc + dx + n) & (n - 1))]);
    }
  }
  out[s] = static_cast<TO>(acc * iz);
}

// Proximal step and momentum of Alg. 1 (beta from the host: the iteration
// index is known there).
__global__ __launch_bounds__(256) void k_exact_prox(const float* __restrict__ g, float* __restrict__ x,
                                                    float* __restrict__ y, float tau, float thr, float beta,
                                                    int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const float xn = prox_plain(y[i], tau * g[i], thr);
  const float xo = x[i];
  x[i] = xn;
  y[i] = xn + beta * (xn - xo);
}

// Per-block partials: sum r^2, sum r u0, sum |x|, max |g| (4 * nblocks).
__global__ __launch_bounds__(256) void k_exact_obj(const float* __restrict__ r, const float* __restrict__ u0,
                                                   const float* __restrict__ x, const float* __restrict__ g,
                                                   int64_t N, double* __restrict__ part, int64_t nblocks) {
  __shared__ double sh[4][256];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < N) {
    const double rr = r[i];
    v[0] = rr * rr;
    v[1] = rr * static_cast<double>(u0[i]);
    v[2] = fabs(static_cast<double>(x[i]));
    v[3] = fabs(static_cast<double>(g[i]));
  }
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 4; ++k)
        sh[k][threadIdx.x] = k == 3 ? fmax(sh[k][threadIdx.x], sh[k][threadIdx.x + w])
                                    : sh[k][threadIdx.x] + sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[threadIdx.x * nblocks + blockIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_exact_fin(const double* __restrict__ part, int64_t nblocks,
                                                   double* __restrict__ out) {
  __shared__ double sh[4][256];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t b = threadIdx.x; b < nblocks; b += 256)
    for (int k = 0; k < 4; ++k) v[k] = k == 3 ? fmax(v[k], part[k * nblocks + b]) : v[k] + part[k * nblocks + b];
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 4; ++k)
        sh[k][threadIdx.x] = k == 3 ? fmax(sh[k][threadIdx.x], sh[k][threadIdx.x + w])
                                    : sh[k][threadIdx.x] + sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_exact_init(const float* __restrict__ src, float* __restrict__ x, float* __restrict__ y, int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const float v = src ? src[i] : 0.0f;
  x[i] = v;
  y[i] = v;
}

dim3 tile_grid(const wdb_exact* ex) { return dim3(ex->ntile, ex->ntile); }
dim3 pix_grid(int64_t N) { return dim3(static_cast<unsigned>((N + 255) / 256)); }

template <typename TI, typename TO>
void apply_H(const wdb_exact* ex, const TI* in, const float* sub, TO* out, hipStream_t s) {
  hipLaunchKernelGGL((k_exact_fwd<TI, TO>), tile_grid(ex), dim3(kThreads), 0, s, ex->F.dev(), ex->tbox.p,
                     ex->ntile, in, sub, out);
}

template <typename TI, typename TO>
void apply_Ht(const wdb_exact* ex, const TI* in, TO* out, hipStream_t s) {
  hipLaunchKernelGGL((k_exact_adj<TI, TO>), pix_grid(ex->N), dim3(256), 0, s, ex->F.dev(), ex->box.p, in, out);
}

// g = Psi^* H^* (H Psi v - u0); leaves H Psi v - u0 in ex->r.
void gradient(wdb_exact* ex, const Filter& f, const float* v, float* g, hipStream_t s) {
  dwt_inverse(ex->n, ex->levels, f, v, ex->img.p, ex->sa.p, ex->sb.p, s);
  apply_H(ex, ex->img.p, ex->u0.p, ex->r.p, s);
  apply_Ht(ex, ex->r.p, ex->gimg.p, s);
  dwt_forward(ex->n, ex->levels, f, ex->gimg.p, g, ex->sa.p, ex->sb.p, s);
}

struct ExCheck {
  double E, rel_gap;
};

// E(x) = 1/2 ||H Psi x - u0||^2 + lambda ||x||_1 and the relative gap with the
// dual point s r, s = min(1, lambda / ||Psi^* H^* r||_inf) (float32 products,
// float64 sums).
ExCheck check(wdb_exact* ex, const Filter& f, const float* x, double lambda, hipStream_t s) {
  gradient(ex, f, x, ex->g.p, s);
  const int64_t nb = pix_grid(ex->N).x;
  hipLaunchKernelGGL(k_exact_obj, pix_grid(ex->N), dim3(256), 0, s, ex->r.p, ex->u0.p, x, ex->g.p, ex->N, ex->part.p,
                     nb);
  hipLaunchKernelGGL(k_exact_fin, dim3(1), dim3(256), 0, s, ex->part.p, nb, ex->scal.p);
  WDB_HIP(hipGetLastError());
  WDB_HIP(hipMemcpyAsync(ex->host, ex->scal.p, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  WDB_HIP(hipStreamSynchronize(s));
  const double rr = ex->host[0], ru = ex->host[1], l1 = ex->host[2], gm = ex->host[3];
  const double E = 0.5 * rr + lambda * l1;
  const double sc = gm <= lambda ? 1.0 : lambda / gm;
  const double D = -0.5 * sc * sc * rr - sc * ru;
  return ExCheck{E, E > 0 ? (E - D) / E : 0.0};
}

LanczosResult exact_lanczos(wdb_exact* ex, const double* start, double tol, int max_steps, hipStream_t s) {
  DevBuf<double> t(ex->N);
  auto apply = [&](const double* v, double* u) {   // u = H^* H v (pixel domain; Psi is orthogonal)
    apply_H(ex, v, static_cast<const float*>(nullptr), t.p, s);
    apply_Ht(ex, static_cast<const double*>(t.p), u, s);
  };
  return lanczos_core(ex->N, apply, start, tol, max_steps, s);
}

}  // namespace
}  // namespace wdb

extern "C" {

wdb_status wdb_exact_create(const wdb_psf_field* field, int32_t wavelet, int32_t levels, void* stream,
                            wdb_exact** out) {
  WDB_API_BEGIN
  WDB_REQUIRE(field && out, WDB_ERR_ARG, "null argument");
  const wdb::Filter f = wdb::make_filter(wavelet);
  wdb::check_geometry(field->n, levels, static_cast<int>(f.h.size()));
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* ex = new wdb_exact;
  try {
    WDB_HIP(hipGetDevice(&ex->device));
    ex->n = field->n;
    ex->levels = levels;
    ex->wavelet = wavelet;
    ex->N = static_cast<int64_t>(field->n) * field->n;
    ex->F.upload(field, s);
    const int64_t N = ex->N;
    ex->box.alloc(N);
    ex->ntile = (ex->n + wdb::kT - 1) / wdb::kT;
    ex->tbox.alloc(static_cast<size_t>(ex->ntile) * ex->ntile);
    hipLaunchKernelGGL(wdb::k_exact_box, wdb::pix_grid(N), dim3(256), 0, s, ex->F.dev(), ex->box.p);
    hipLaunchKernelGGL(wdb::k_exact_tbox, dim3((ex->ntile * ex->ntile + 255) / 256), dim3(256), 0, s, ex->box.p,
                       ex->n, ex->ntile, ex->tbox.p);
    for (auto* b : {&ex->u0, &ex->y, &ex->img, &ex->r, &ex->gimg, &ex->g}) b->alloc(N);
    ex->sa.alloc(N / 4 + 1);
    ex->sb.alloc(N / 4 + 1);
    const int64_t nb = wdb::pix_grid(N).x;
    ex->part.alloc(4 * nb);
    ex->scal.alloc(4);
    WDB_HIP(hipHostMalloc(reinterpret_cast<void**>(&ex->host), 4 * sizeof(double), hipHostMallocDefault));
    WDB_HIP(hipGetLastError());
    WDB_HIP(hipStreamSynchronize(s));
  } catch (...) {
    if (ex->host) (void)hipHostFree(ex->host);
    delete ex;
    throw;
  }
  *out = ex;
  WDB_API_END
}

void wdb_exact_free(wdb_exact* ex) {
  if (!ex) return;
  (void)hipSetDevice(ex->device);
  (void)hipDeviceSynchronize();
  if (ex->host) (void)hipHostFree(ex->host);
  delete ex;
}

wdb_status wdb_exact_apply(wdb_exact* ex, int32_t adjoint, const float* in, float* out, void* stream) {
  WDB_API_BEGIN
  WDB_REQUIRE(ex && in && out, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(in != out, WDB_ERR_ARG, "in and out must not alias");
  WDB_HIP(hipSetDevice(ex->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (adjoint)
    wdb::apply_Ht(ex, in, out, s);
  else
    wdb::apply_H(ex, in, static_cast<const float*>(nullptr), out, s);
  WDB_HIP(hipGetLastError());
  WDB_API_END
}

wdb_status wdb_exact_lipschitz(wdb_exact* ex, const double* start, double tol, int32_t max_steps, double* L_out,
                               int32_t* steps_out, double* resid_out) {
  WDB_API_BEGIN
  WDB_REQUIRE(ex, WDB_ERR_ARG, "null handle");
  WDB_HIP(hipSetDevice(ex->device));
  const wdb::LanczosResult r = wdb::exact_lanczos(ex, start, tol, max_steps, nullptr);
  ex->L = r.theta + r.resid;
  ex->has_L = true;
  if (L_out) *L_out = ex->L;
  if (steps_out) *steps_out = r.steps;
  if (resid_out) *resid_out = r.resid;
  if (!r.converged)
    wdb::fail(WDB_ERR_NOT_CONVERGED, "Lanczos reached max_steps = %d with residual %.3e > tol * theta", max_steps,
              r.resid);
  WDB_API_END
}

wdb_status wdb_exact_solve(wdb_exact* ex, const float* u, float lambda, const wdb_solve_opts* opts, float* x_out,
                           wdb_solve_info* info) {
  WDB_API_BEGIN
  WDB_REQUIRE(ex && u && opts && x_out, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(std::isfinite(lambda) && lambda >= 0.0f, WDB_ERR_NONFINITE, "lambda must be finite and >= 0");
  WDB_REQUIRE(opts->max_iters >= 0 && opts->check_every >= 0 && opts->k0 >= 0, WDB_ERR_ARG, "bad iteration counts");
  WDB_REQUIRE(!opts->use_precond, WDB_ERR_ARG, "the exact-operator solver has no preconditioner");
  WDB_HIP(hipSetDevice(ex->device));
  hipStream_t s = static_cast<hipStream_t>(opts->stream);
  if (!ex->has_L) {
    const wdb::LanczosResult r = wdb::exact_lanczos(ex, nullptr, 1e-12, 2000, s);
    ex->L = r.theta + r.resid;
    ex->has_L = true;
  }
  WDB_REQUIRE(ex->L > 0.0 && std::isfinite(ex->L), WDB_ERR_ARG, "operator has no positive Lipschitz constant");
  const double tau = 1.0 / ex->L;
  const float tau_f = static_cast<float>(tau), thr_f = static_cast<float>(tau * static_cast<double>(lambda));
  const wdb::Filter f = wdb::make_filter(ex->wavelet);
  const int64_t N = ex->N;
  WDB_HIP(hipMemcpyAsync(ex->u0.p, u, N * sizeof(float), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(wdb::k_exact_init, wdb::pix_grid(N), dim3(256), 0, s, opts->x_init, x_out, ex->y.p, N);
  const int k0 = opts->k0 > 0 ? opts->k0 : 1;
  const int c = opts->check_every, total = opts->max_iters;
  int done = 0, checks = 0;
  bool converged = false;
  wdb::ExCheck last{0.0, 0.0};
  while (done < total || (total == 0 && checks == 0)) {
    if (done < total) {
      const int k = k0 + done;
      const float beta = opts->ista ? 0.0f : static_cast<float>((k - 1.0) / (k + 2.0));
      wdb::gradient(ex, f, ex->y.p, ex->g.p, s);
      hipLaunchKernelGGL(wdb::k_exact_prox, wdb::pix_grid(N), dim3(256), 0, s, ex->g.p, x_out, ex->y.p, tau_f, thr_f,
                         beta, N);
      WDB_HIP(hipGetLastError());
      ++done;
    }
    if ((c > 0 && done % c == 0) || done == total) {
      last = wdb::check(ex, f, x_out, lambda, s);
      ++checks;
      if (opts->trace && checks <= opts->trace_cap) {
        opts->trace[3 * (checks - 1) + 0] = static_cast<double>(k0 - 1 + done);
        opts->trace[3 * (checks - 1) + 1] = last.E;
        opts->trace[3 * (checks - 1) + 2] = last.rel_gap;
      }
      WDB_REQUIRE(std::isfinite(last.E), WDB_ERR_DIVERGED, "objective became non-finite at iteration %d", done);
      if ((opts->tol_rel_gap > 0 && last.rel_gap <= opts->tol_rel_gap) ||
          (opts->target_objective > 0 && last.E <= opts->target_objective)) {
        converged = true;
        break;
      }
      if (total == 0) break;
    }
  }
  WDB_HIP(hipStreamSynchronize(s));
  if (info) {
    info->iters = done;
    info->checks = checks;
    info->objective = last.E;
    info->rel_gap = last.rel_gap;
    info->lipschitz = ex->L;
    info->tau = tau;
  }
  if ((opts->tol_rel_gap > 0 || opts->target_objective > 0) && !converged)
    wdb::fail(WDB_ERR_NOT_CONVERGED, "stopping test not met after %d iterations (relative gap %.3e)", done,
              last.rel_gap);
  WDB_API_END
}

}  // extern "C"
