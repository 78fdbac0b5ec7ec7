// Accelerated proximal gradient (Alg. 1; Alg. 2 with a diagonal P) on the
// wavelet-domain problem of Sec. 1.3, plus its float64 companions: the power
// iteration for the step 1/||Theta_K||^2 and the objective / duality-gap test.
//
// One FISTA iteration is two kernels over copies of Theta_K and Theta_K^T:
//   k_res  : r = Theta_K y - x0                      (first half of the gradient)
//   k_prox : g = Theta_K^T r; z = y - tau g / P;
//            x_k = S_{tau lambda / P}(z);
//            y = x_k + (k-1)/(k+2) (x_k - x_{k-1})   (rest of Alg. 1, fused)
// in one of two layouts chosen per operator: sliced ELL (one thread per row
// of a C-row slice, C = 8..64, streaming 16-byte value and index vectors) or
// padded CSR (G lanes per row, 16-byte loads of 4 values and 4 indices).
// Gathers go through the caches and every row is accumulated in float32 in a
// fixed order, so results are bitwise reproducible (no atomics on values).
// The 16-bit form uses the packed kernels of packed.hip instead.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <functional>
#include <limits>
#include <type_traits>

#include "common.hpp"
#include "prox.hpp"
#include "tridiag.hpp"

namespace wdb {

namespace {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;
constexpr int kRhoChunk = 64;

inline dim3 vec_grid(int64_t n) { return dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)); }

struct SellView {
  const int64_t* __restrict__ soff;
  const float4* __restrict__ val;
  const int4* __restrict__ col;
  const int32_t* __restrict__ perm;
  int64_t nslices, nrows;
  int C, cshift;  // slice height (power of two) and its log2
};

SellView view(const Sell& m) {
  return SellView{m.slice_off, reinterpret_cast<const float4*>(m.val), reinterpret_cast<const int4*>(m.col),
                  m.perm, m.nslices, m.nrows, m.C, __builtin_ctz(static_cast<unsigned>(m.C))};
}

__host__ __device__ inline int64_t slots(const SellView& A) { return A.nslices << A.cshift; }
inline dim3 slot_grid(const SellView& A) { return vec_grid(slots(A)); }

// Blocks of the reduction kernels over A and A^T (both copies share the slice
// height, so every partial-sum slot below this count is written).
int64_t partial_blocks(const SellView& A, const SellView& At) {
  const int64_t nb = slot_grid(A).x;
  WDB_REQUIRE(nb == static_cast<int64_t>(slot_grid(At).x), WDB_ERR_HIP, "mismatched slice heights");
  return nb;
}

// Matrix row held by slot row q (-1 for an empty slot row).
__device__ __forceinline__ int64_t slot_row(const SellView& A, int64_t q) {
  if (A.perm) return A.perm[q];
  return q < A.nrows ? q : -1;
}

// Padding slots hold value 0 and a valid column of the same row, so they
// are processed like real entries (a branch per entry serialises the gathers).
__device__ __forceinline__ float gather_fma(float v, int c, const float* __restrict__ x, float acc) {
  return fmaf(v, x[c], acc);
}

// Row sum of one lane's row in float32, storage order.
template <typename T>
__device__ __forceinline__ float row_dot_f32(const SellView& A, int64_t sl, int lane, const T* __restrict__ x) {
  const int64_t beg = A.soff[sl] >> 2, end = A.soff[sl + 1] >> 2;
  float acc = 0.f;
#pragma unroll 2
  for (int64_t j = beg + lane; j < end; j += A.C) {
    const float4 v = A.val[j];
    const int4 c = A.col[j];
    acc = gather_fma(v.x, c.x, x, acc);
    acc = gather_fma(v.y, c.y, x, acc);
    acc = gather_fma(v.z, c.z, x, acc);
    acc = gather_fma(v.w, c.w, x, acc);
  }
  return acc;
}

// Row sum in float64 (values promoted), storage order.
template <typename T>
__device__ __forceinline__ double row_dot_f64(const SellView& A, int64_t sl, int lane, const T* __restrict__ x) {
  const int64_t beg = A.soff[sl] >> 2, end = A.soff[sl + 1] >> 2;
  double acc = 0.0;
  for (int64_t j = beg + lane; j < end; j += A.C) {
    const float4 v = A.val[j];
    const int4 c = A.col[j];
    acc = fma(static_cast<double>(v.x), static_cast<double>(x[c.x]), acc);
    acc = fma(static_cast<double>(v.y), static_cast<double>(x[c.y]), acc);
    acc = fma(static_cast<double>(v.z), static_cast<double>(x[c.z]), acc);
    acc = fma(static_cast<double>(v.w), static_cast<double>(x[c.w]), acc);
  }
  return acc;
}

// Deterministic block reduction of NV values; bit k of MAXMASK selects max
// instead of sum.  Writes partial[k * nblocks + blockIdx.x].
template <int NV, unsigned MAXMASK>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* __restrict__ partial, int64_t nblocks) {
  __shared__ double sh[kWaves][NV];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = v[k];
    for (int off = kWave / 2; off > 0; off >>= 1) {
      const double y = __shfl_xor(x, off);
      x = ((MAXMASK >> k) & 1u) ? fmax(x, y) : x + y;
    }
    if (lane == 0) sh[wid][k] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double acc = sh[0][k];
      for (int w = 1; w < kWaves; ++w) acc = ((MAXMASK >> k) & 1u) ? fmax(acc, sh[w][k]) : acc + sh[w][k];
      partial[k * nblocks + blockIdx.x] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// FISTA kernels (float32).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_res(SellView A, const float* __restrict__ y, const float* __restrict__ b,
                                                float* __restrict__ r, int* __restrict__ kdev) {
  if (kdev && blockIdx.x == 0 && threadIdx.x == 0) *kdev += 1;
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= slots(A)) return;
  const int64_t sl = q >> A.cshift;
  const int lane = static_cast<int>(q & (A.C - 1));
  const float acc = row_dot_f32(A, sl, lane, y);
  const int64_t row = slot_row(A, q);
  if (row >= 0) r[row] = b ? acc - b[row] : acc;
}

// beta from the device counter (kdev) or, if kdev is null, from `beta`.  The
// threshold of row i is thr * tw[i] (tw = w / P, the l1 weights over the
// preconditioner), or thr / P_i when tw is null (uniform weights).
template <bool PRE>
__global__ __launch_bounds__(kBlock) void k_prox(SellView At, const float* __restrict__ r, float* __restrict__ x,
                                                 float* __restrict__ y, float tau, float thr, float beta,
                                                 const int* __restrict__ kdev, const float* __restrict__ pinv,
                                                 const float* __restrict__ tw, const double* __restrict__ anc) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t sl = q >> At.cshift;
  const int lane = static_cast<int>(q & (At.C - 1));
  if (sl >= At.nslices) return;
  const float g = row_dot_f32(At, sl, lane, r);
  const int64_t row = slot_row(At, q);
  if (row < 0) return;
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

// ---------------------------------------------------------------------------
// 16-bit value variants (mixed precision): the same slots and indices, values
// as binary16 / bfloat16 (four per 8-byte lane load), float32 accumulation.
// Row sums are multiplied by the row's power-of-two factor w (exact).
// ---------------------------------------------------------------------------
template <int FMT>
__device__ __forceinline__ float dq16(uint32_t h) {
  if constexpr (FMT == WDB_VAL_BF16) return __uint_as_float(h << 16);
  else return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(h)));
}

template <int FMT>
__device__ __forceinline__ float row_dot_q(const SellView& A, const uint2* __restrict__ v16, int64_t sl, int lane,
                                           const float* __restrict__ x) {
  const int64_t beg = A.soff[sl] >> 2, end = A.soff[sl + 1] >> 2;
  float acc = 0.f;
#pragma unroll 2
  for (int64_t j = beg + lane; j < end; j += A.C) {
    const uint2 v = v16[j];
    const int4 c = A.col[j];
    acc = fmaf(dq16<FMT>(v.x & 0xFFFFu), x[c.x], acc);
    acc = fmaf(dq16<FMT>(v.x >> 16), x[c.y], acc);
    acc = fmaf(dq16<FMT>(v.y & 0xFFFFu), x[c.z], acc);
    acc = fmaf(dq16<FMT>(v.y >> 16), x[c.w], acc);
  }
  return acc;
}

// r = w * (Q y) - b; stores w * r when scale_out (input of the transposed kernel).
template <int FMT>
__global__ __launch_bounds__(kBlock) void k_res_q(SellView A, const uint2* __restrict__ v16,
                                                  const float* __restrict__ wrow, const float* __restrict__ y,
                                                  const float* __restrict__ b, float* __restrict__ r,
                                                  int* __restrict__ kdev, int scale_out) {
  if (kdev && blockIdx.x == 0 && threadIdx.x == 0) *kdev += 1;
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= slots(A)) return;
  const int64_t sl = q >> A.cshift;
  const int lane = static_cast<int>(q & (A.C - 1));
  const float acc = row_dot_q<FMT>(A, v16, sl, lane, y);
  const int64_t row = slot_row(A, q);
  if (row < 0) return;
  const float w = wrow[row];
  const float rr = b ? w * acc - b[row] : w * acc;
  r[row] = scale_out ? rr * w : rr;
}

template <int FMT, bool PRE>
__global__ __launch_bounds__(kBlock) void k_prox_q(SellView At, const uint2* __restrict__ v16T,
                                                   const float* __restrict__ rs, float* __restrict__ x,
                                                   float* __restrict__ y, float tau, float thr,
                                                   const int* __restrict__ kdev, const float* __restrict__ pinv,
                                                   const float* __restrict__ tw) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t sl = q >> At.cshift;
  const int lane = static_cast<int>(q & (At.C - 1));
  if (sl >= At.nslices) return;
  const float g = row_dot_q<FMT>(At, v16T, sl, lane, rs);
  const int64_t row = slot_row(At, q);
  if (row < 0) return;
  float beta = 0.0f;  // no counter: no extrapolation (ISTA)
  if (kdev) {
    const int k = *kdev;
    beta = static_cast<float>((static_cast<double>(k) - 1.0) / (static_cast<double>(k) + 2.0));
  }
  const float pi = PRE ? pinv[row] : 1.0f;
  const float z = y[row] - (tau * pi) * g;
  const float t = thr * (tw ? tw[row] : pi);
  const float xn = copysignf(fmaxf(fabsf(z) - t, 0.0f), z);
  const float xo = x[row];
  x[row] = xn;
  y[row] = xn + beta * (xn - xo);
}

template <int FMT>
void launch_iteration_q(wdb_theta* th, float* x, bool pre, const int* kp, float tau, float thr, hipStream_t s) {
  const SellView A = view(th->A), At = view(th->At);
  const uint2* v16 = reinterpret_cast<const uint2*>(th->val16);
  const uint2* v16T = reinterpret_cast<const uint2*>(th->val16T);
  hipLaunchKernelGGL(k_res_q<FMT>, slot_grid(A), dim3(kBlock), 0, s, A, v16, th->wrow, th->ws_y,
                     th->ws_x0, th->ws_r, th->ws_k, 1);
  if (pre)
    hipLaunchKernelGGL((k_prox_q<FMT, true>), slot_grid(At), dim3(kBlock), 0, s, At, v16T, th->ws_r, x,
                       th->ws_y, tau, thr, kp, th->pinv, threshold_weights(th, true));
  else
    hipLaunchKernelGGL((k_prox_q<FMT, false>), slot_grid(At), dim3(kBlock), 0, s, At, v16T, th->ws_r, x,
                       th->ws_y, tau, thr, kp, static_cast<const float*>(nullptr),
                       threshold_weights(th, false));
}

// ---------------------------------------------------------------------------
// Vector-CSR variants over the padded CSR copy: G consecutive lanes share one
// row; each lane loads two 16-byte groups of 4 values and 4 columns (chunks
// c and c + G of the row) before its gathers, so a lane has 8 entries in
// flight per step and a row of 4k entries takes k / (2G) steps.  Partial sums
// are reduced with a fixed butterfly inside the group.
// ---------------------------------------------------------------------------
struct CsrView {
  const int64_t* __restrict__ rp;
  const int32_t* __restrict__ col;
  const float* __restrict__ val;
  int64_t nrows;
};

CsrView cview(const Csr32& m) { return CsrView{m.rowptr, m.col, m.val, m.nrows}; }

template <int G>
__device__ __forceinline__ float group_dot(const CsrView& A, int64_t row, int gl, const float* __restrict__ x) {
  constexpr int U = 2;
  float acc = 0.f;
  if (row < A.nrows) {
    const float4* __restrict__ v4 = reinterpret_cast<const float4*>(A.val);
    const int4* __restrict__ c4 = reinterpret_cast<const int4*>(A.col);
    const int64_t end = A.rp[row + 1] >> 2;
    for (int64_t k = (A.rp[row] >> 2) + gl; k < end; k += G * U) {
      float4 v[U];
      int4 c[U];
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const bool ok = k + t * G < end;
        v[t] = ok ? v4[k + t * G] : make_float4(0.f, 0.f, 0.f, 0.f);
        c[t] = ok ? c4[k + t * G] : make_int4(0, 0, 0, 0);
      }
#pragma unroll
      for (int t = 0; t < U; ++t) {
        acc = fmaf(v[t].x, x[c[t].x], acc);
        acc = fmaf(v[t].y, x[c[t].y], acc);
        acc = fmaf(v[t].z, x[c[t].z], acc);
        acc = fmaf(v[t].w, x[c[t].w], acc);
      }
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
  return acc;
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_res_csr(CsrView A, const float* __restrict__ y,
                                                    const float* __restrict__ b, float* __restrict__ r,
                                                    int* __restrict__ kdev) {
  if (kdev && blockIdx.x == 0 && threadIdx.x == 0) *kdev += 1;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / G) + threadIdx.x / G;
  const int gl = threadIdx.x % G;
  const float acc = group_dot<G>(A, row, gl, y);
  if (gl == 0 && row < A.nrows) r[row] = b ? acc - b[row] : acc;
}

template <int G, bool PRE>
__global__ __launch_bounds__(kBlock) void k_prox_csr(CsrView At, const float* __restrict__ r,
                                                     float* __restrict__ x, float* __restrict__ y, float tau,
                                                     float thr, float beta, const int* __restrict__ kdev,
                                                     const float* __restrict__ pinv, const float* __restrict__ tw,
                                                     const double* __restrict__ anc) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / G) + threadIdx.x / G;
  const int gl = threadIdx.x % G;
  const float g = group_dot<G>(At, row, gl, r);
  if (gl != 0 || row >= At.nrows) return;
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

template <int G>
void launch_res_csr(const CsrView& A, const float* y, const float* b, float* r, int* kdev, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((A.nrows + kBlock / G - 1) / (kBlock / G)));
  hipLaunchKernelGGL(k_res_csr<G>, grid, dim3(kBlock), 0, s, A, y, b, r, kdev);
}

template <int G>
void launch_prox_csr(const CsrView& At, const float* r, float* x, float* y, float tau, float thr, float beta,
                     const int* kdev, const float* pinv, const float* tw, const double* anc, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((At.nrows + kBlock / G - 1) / (kBlock / G)));
  if (pinv)
    hipLaunchKernelGGL((k_prox_csr<G, true>), grid, dim3(kBlock), 0, s, At, r, x, y, tau, thr, beta, kdev, pinv, tw,
                       anc);
  else
    hipLaunchKernelGGL((k_prox_csr<G, false>), grid, dim3(kBlock), 0, s, At, r, x, y, tau, thr, beta, kdev, pinv,
                       tw, anc);
}

}  // namespace

int kernel_group(const wdb_theta* th) {
  const int G = th->spmv_group >= 0 ? th->spmv_group : spmv_group();
  if (G == kStencil && !th->st.seg) return 0;
  if (G == kTiled && !th->tA.desc) return 0;
  return G;
}

// Lanes per row of the float64 CSR passes (the stencil layout checks on CSR).
int check_group(const wdb_theta* th) {
  const int G = kernel_group(th);
  return (G == kStencil || G == kTiled) ? 4 : G;
}

// r = A y - b with the kernel family G (0: sliced ELL; else vector CSR, G lanes per row).
void launch_res(int G, const Sell& sell, const Csr32& csr, const float* y, const float* b, float* r, int* kdev,
                hipStream_t s) {
  switch (G) {
    case 2: launch_res_csr<2>(cview(csr), y, b, r, kdev, s); return;
    case 4: launch_res_csr<4>(cview(csr), y, b, r, kdev, s); return;
    case 8: launch_res_csr<8>(cview(csr), y, b, r, kdev, s); return;
    case 16: launch_res_csr<16>(cview(csr), y, b, r, kdev, s); return;
    case 32: launch_res_csr<32>(cview(csr), y, b, r, kdev, s); return;
    case 64: launch_res_csr<64>(cview(csr), y, b, r, kdev, s); return;
    default: {
      const SellView A = view(sell);
      hipLaunchKernelGGL(k_res, slot_grid(A), dim3(kBlock), 0, s, A, y, b, r, kdev);
    }
  }
}

void launch_prox(int G, const Sell& sell, const Csr32& csr, const float* r, float* x, float* y, float tau, float thr,
                 float beta, const int* kdev, const float* pinv, const float* tw, const double* anc, hipStream_t s) {
  switch (G) {
    case 2: launch_prox_csr<2>(cview(csr), r, x, y, tau, thr, beta, kdev, pinv, tw, anc, s); return;
    case 4: launch_prox_csr<4>(cview(csr), r, x, y, tau, thr, beta, kdev, pinv, tw, anc, s); return;
    case 8: launch_prox_csr<8>(cview(csr), r, x, y, tau, thr, beta, kdev, pinv, tw, anc, s); return;
    case 16: launch_prox_csr<16>(cview(csr), r, x, y, tau, thr, beta, kdev, pinv, tw, anc, s); return;
    case 32: launch_prox_csr<32>(cview(csr), r, x, y, tau, thr, beta, kdev, pinv, tw, anc, s); return;
    case 64: launch_prox_csr<64>(cview(csr), r, x, y, tau, thr, beta, kdev, pinv, tw, anc, s); return;
    default: {
      const SellView At = view(sell);
      if (pinv)
        hipLaunchKernelGGL(k_prox<true>, slot_grid(At), dim3(kBlock), 0, s, At, r, x, y, tau, thr, beta,
                           kdev, pinv, tw, anc);
      else
        hipLaunchKernelGGL(k_prox<false>, slot_grid(At), dim3(kBlock), 0, s, At, r, x, y, tau, thr,
                           beta, kdev, pinv, tw, anc);
    }
  }
}

namespace {

// ---------------------------------------------------------------------------
// Float64 objective and duality gap.
// ---------------------------------------------------------------------------
// With l1 weights w (null = uniform): the l1 sum is sum_i w_i |x_i| and the
// dual scaling uses max_i |g_i| / w_i.
template <typename X>
__global__ __launch_bounds__(kBlock) void k_obj_fwd(SellView A, const X* __restrict__ x, const float* __restrict__ b,
                                                    const float* __restrict__ w, double* __restrict__ r64,
                                                    double* __restrict__ partial, int64_t nblocks) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t sl = q >> A.cshift;
  const int lane = static_cast<int>(q & (A.C - 1));
  double v[3] = {0.0, 0.0, 0.0};
  if (q < slots(A)) {
    const double acc = row_dot_f64(A, sl, lane, x);
    const int64_t row = slot_row(A, q);
    if (row >= 0) {
      const double bb = static_cast<double>(b[row]);
      const double rr = acc - bb;
      r64[row] = rr;
      v[0] = rr * rr;
      v[1] = rr * bb;
      v[2] = fabs(static_cast<double>(x[row])) * (w ? static_cast<double>(w[row]) : 1.0);
    }
  }
  block_partials<3, 0u>(v, partial, nblocks);
}

__global__ __launch_bounds__(kBlock) void k_obj_bwd(SellView At, const double* __restrict__ r64,
                                                    const float* __restrict__ w, double* __restrict__ partial,
                                                    int64_t nblocks) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t sl = q >> At.cshift;
  const int lane = static_cast<int>(q & (At.C - 1));
  double v[1] = {0.0};
  if (q < slots(At)) {
    const int64_t row = slot_row(At, q);
    const double g = row_dot_f64(At, sl, lane, r64);
    if (row >= 0) v[0] = fabs(g) / (w ? static_cast<double>(w[row]) : 1.0);
  }
  block_partials<1, 1u>(v, partial, nblocks);
}

// Final reduction of the stopping test's per-block partials in two passes
// with a fixed order: out[k] = sum (or max, bit k of maxmask) of
// partial[k * nblocks + i] over i, for k < 4.  Pass 1: block b folds the
// contiguous range b of kReduceParts ranges (thread t takes i = t, t + T, ...
// of the range), then a fixed tree, into tmp[k * kReduceParts + b]; pass 2: one
// block folds the kReduceParts values of each row with a fixed tree.  The max
// rows hold non-negative values, so 0 is their neutral element.
constexpr int kReduceParts = 64;
constexpr int kReduceThreads = 256;
__device__ __forceinline__ double fold4(unsigned maxmask, int k, double a, double b) {
  return ((maxmask >> k) & 1u) ? fmax(a, b) : a + b;
}
__global__ __launch_bounds__(kReduceThreads) void k_reduce4_part(const double* __restrict__ partial, int64_t nblocks,
                                                                 unsigned maxmask, double* __restrict__ tmp) {
  __shared__ double sh[4][kReduceThreads];
  const int64_t len = (nblocks + kReduceParts - 1) / kReduceParts;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * len;
  const int64_t i1 = i0 + len < nblocks ? i0 + len : nblocks;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kReduceThreads) {
    double p[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = partial[k * nblocks + i];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = fold4(maxmask, k, acc[k], p[k]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = fold4(maxmask, k, sh[k][threadIdx.x], sh[k][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) tmp[threadIdx.x * kReduceParts + blockIdx.x] = sh[threadIdx.x][0];
}
__global__ __launch_bounds__(kReduceParts) void k_reduce4_final(const double* __restrict__ tmp, unsigned maxmask,
                                                                double* __restrict__ out) {
  __shared__ double sh[4][kReduceParts];
#pragma unroll
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = tmp[k * kReduceParts + threadIdx.x];
  __syncthreads();
  for (int w = kReduceParts / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = fold4(maxmask, k, sh[k][threadIdx.x], sh[k][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = sh[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Power iteration (float64): w = A vd; u = d .* (A^T w); vd = d .* u / ||u||.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_pi_fwd(SellView A, const double* __restrict__ vd, double* __restrict__ w,
                                                   double* __restrict__ partial, int64_t nblocks) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t sl = q >> A.cshift;
  const int lane = static_cast<int>(q & (A.C - 1));
  double v[1] = {0.0};
  if (q < slots(A)) {
    const int64_t row = slot_row(A, q);
    const double acc = row_dot_f64(A, sl, lane, vd);
    if (row >= 0) {
      w[row] = acc;
      v[0] = acc * acc;
    }
  }
  block_partials<1, 0u>(v, partial, nblocks);
}

__global__ __launch_bounds__(kBlock) void k_pi_bwd(SellView At, const double* __restrict__ w,
                                                   const double* __restrict__ d, double* __restrict__ u,
                                                   double* __restrict__ partial, int64_t nblocks) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t sl = q >> At.cshift;
  const int lane = static_cast<int>(q & (At.C - 1));
  double v[1] = {0.0};
  if (q < slots(At)) {
    const int64_t row = slot_row(At, q);
    double acc = row_dot_f64(At, sl, lane, w);
    if (row >= 0) {
      if (d) acc *= d[row];
      u[row] = acc;
      v[0] = acc * acc;
    }
  }
  block_partials<1, 0u>(v, partial, nblocks);
}

__global__ __launch_bounds__(kBlock) void k_pi_finish(const double* __restrict__ partial, int64_t nblocks,
                                                      double* __restrict__ rho_hist, int slot,
                                                      double* __restrict__ scal) {
  __shared__ double sh[2][kBlock];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < nblocks; i += kBlock) {
    a += partial[i];
    b += partial[nblocks + i];
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    rho_hist[slot] = sh[0][0];
    scal[0] = sh[1][0] > 0.0 ? 1.0 / sqrt(sh[1][0]) : 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_pi_scale(const double* __restrict__ u, const double* __restrict__ d,
                                                     const double* __restrict__ scal, double* __restrict__ vd,
                                                     int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= N) return;
  const double v = u[i] * scal[0];
  vd[i] = d ? v * d[i] : v;
}

__global__ __launch_bounds__(kBlock) void k_mul(double* __restrict__ v, const double* __restrict__ d, int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < N) v[i] *= d[i];
}

__global__ __launch_bounds__(kBlock) void k_copy_or_zero(const float* __restrict__ src, float* __restrict__ a,
                                                         float* __restrict__ b, int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= N) return;
  const float v = src ? src[i] : 0.0f;
  a[i] = v;
  b[i] = v;
}

// ---------------------------------------------------------------------------
// The same float64 passes over the vector-CSR copies (G lanes per row).  Each
// block walks row tiles with a grid stride so the partial-sum count stays
// within the workspace; the result depends only on the grid, not on timing.
// ---------------------------------------------------------------------------
template <int G, typename T>
__device__ __forceinline__ double group_dot64(const CsrView& A, int64_t row, int gl, const T* __restrict__ x) {
  constexpr int U = 2;
  double acc = 0.0;
  if (row < A.nrows) {
    const float4* __restrict__ v4 = reinterpret_cast<const float4*>(A.val);
    const int4* __restrict__ c4 = reinterpret_cast<const int4*>(A.col);
    const int64_t end = A.rp[row + 1] >> 2;
    for (int64_t k = (A.rp[row] >> 2) + gl; k < end; k += G * U) {
      float4 v[U];
      int4 c[U];
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const bool ok = k + t * G < end;
        v[t] = ok ? v4[k + t * G] : make_float4(0.f, 0.f, 0.f, 0.f);
        c[t] = ok ? c4[k + t * G] : make_int4(0, 0, 0, 0);
      }
#pragma unroll
      for (int t = 0; t < U; ++t) {
        acc = fma(static_cast<double>(v[t].x), static_cast<double>(x[c[t].x]), acc);
        acc = fma(static_cast<double>(v[t].y), static_cast<double>(x[c[t].y]), acc);
        acc = fma(static_cast<double>(v[t].z), static_cast<double>(x[c[t].z]), acc);
        acc = fma(static_cast<double>(v[t].w), static_cast<double>(x[c[t].w]), acc);
      }
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
  return acc;
}

template <int G>
__device__ __forceinline__ int64_t csr_tiles(const CsrView& A) {
  return (A.nrows + kBlock / G - 1) / (kBlock / G);
}

template <int G, typename X>
__global__ __launch_bounds__(kBlock) void k_obj_fwd_csr(CsrView A, const X* __restrict__ x,
                                                        const float* __restrict__ b, const float* __restrict__ w,
                                                        double* __restrict__ r64, double* __restrict__ partial,
                                                        int64_t nblocks) {
  double v[3] = {0.0, 0.0, 0.0};
  const int gl = threadIdx.x % G;
  for (int64_t t = blockIdx.x; t < csr_tiles<G>(A); t += gridDim.x) {
    const int64_t row = t * (kBlock / G) + threadIdx.x / G;
    const double acc = group_dot64<G>(A, row, gl, x);
    if (gl == 0 && row < A.nrows) {
      const double bb = static_cast<double>(b[row]);
      const double rr = acc - bb;
      r64[row] = rr;
      v[0] += rr * rr;
      v[1] += rr * bb;
      v[2] += fabs(static_cast<double>(x[row])) * (w ? static_cast<double>(w[row]) : 1.0);
    }
  }
  block_partials<3, 0u>(v, partial, nblocks);
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_obj_bwd_csr(CsrView At, const double* __restrict__ r64,
                                                        const float* __restrict__ w, double* __restrict__ partial,
                                                        int64_t nblocks) {
  double v[1] = {0.0};
  const int gl = threadIdx.x % G;
  for (int64_t t = blockIdx.x; t < csr_tiles<G>(At); t += gridDim.x) {
    const int64_t row = t * (kBlock / G) + threadIdx.x / G;
    const double g = group_dot64<G>(At, row, gl, r64);
    if (gl == 0 && row < At.nrows) v[0] = fmax(v[0], fabs(g) / (w ? static_cast<double>(w[row]) : 1.0));
  }
  block_partials<1, 1u>(v, partial, nblocks);
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_pi_fwd_csr(CsrView A, const double* __restrict__ vd,
                                                       double* __restrict__ w, double* __restrict__ partial,
                                                       int64_t nblocks) {
  double v[1] = {0.0};
  const int gl = threadIdx.x % G;
  for (int64_t t = blockIdx.x; t < csr_tiles<G>(A); t += gridDim.x) {
    const int64_t row = t * (kBlock / G) + threadIdx.x / G;
    const double acc = group_dot64<G>(A, row, gl, vd);
    if (gl == 0 && row < A.nrows) {
      w[row] = acc;
      v[0] += acc * acc;
    }
  }
  block_partials<1, 0u>(v, partial, nblocks);
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_pi_bwd_csr(CsrView At, const double* __restrict__ w,
                                                       const double* __restrict__ d, double* __restrict__ u,
                                                       double* __restrict__ partial, int64_t nblocks) {
  double v[1] = {0.0};
  const int gl = threadIdx.x % G;
  for (int64_t t = blockIdx.x; t < csr_tiles<G>(At); t += gridDim.x) {
    const int64_t row = t * (kBlock / G) + threadIdx.x / G;
    double acc = group_dot64<G>(At, row, gl, w);
    if (gl == 0 && row < At.nrows) {
      if (d) acc *= d[row];
      u[row] = acc;
      v[0] += acc * acc;
    }
  }
  block_partials<1, 0u>(v, partial, nblocks);
}

// Calls f(std::integral_constant<int, G>) for a vector-CSR group size G.
template <typename F>
void with_group(int G, F&& f) {
  switch (G) {
    case 2: f(std::integral_constant<int, 2>{}); return;
    case 4: f(std::integral_constant<int, 4>{}); return;
    case 8: f(std::integral_constant<int, 8>{}); return;
    case 16: f(std::integral_constant<int, 16>{}); return;
    case 32: f(std::integral_constant<int, 32>{}); return;
    case 64: f(std::integral_constant<int, 64>{}); return;
    default: fail(WDB_ERR_ARG, "unsupported lanes per row %d", G);
  }
}

// Grid of the float64 vector-CSR passes: one block per row tile, at most the
// workspace's partial-sum capacity.
int64_t csr_check_blocks(const wdb_theta* th, int G) {
  const int64_t tiles = (th->N + kBlock / G - 1) / (kBlock / G);
  return std::max<int64_t>(1, std::min(tiles, th->ws_nblocks));
}

__global__ void k_set_int(int* p, int v) { *p = v; }

// Anchored iterate (x = a + d, a float64, d float32; see prox.hpp).
// Start: a = 0 and c = x0, so the displacement iteration is the plain one.
__global__ __launch_bounds__(kBlock) void k_anchor_init(double* __restrict__ a, float* __restrict__ c,
                                                        const float* __restrict__ x0, int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= N) return;
  a[i] = 0.0;
  c[i] = x0[i];
}

// Moves the displacement into the anchor: a += d, y -= d, d = 0 (x and the
// extrapolated point y keep their values as sums).
__global__ __launch_bounds__(kBlock) void k_reanchor(double* __restrict__ a, float* __restrict__ d,
                                                     float* __restrict__ y, int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= N) return;
  const float di = d[i];
  a[i] += static_cast<double>(di);
  y[i] -= di;
  d[i] = 0.0f;
}

// Right-hand side of the displacement iteration after a check on the anchor:
// r64 = Theta_K a - x0 (float64), so r = Theta_K d - c with c = -r64.
__global__ __launch_bounds__(kBlock) void k_anchor_rhs(const double* __restrict__ r64, float* __restrict__ c,
                                                       int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < N) c[i] = static_cast<float>(-r64[i]);
}

__global__ __launch_bounds__(kBlock) void k_widen(const float* __restrict__ x, double* __restrict__ x64, int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < N) x64[i] = static_cast<double>(x[i]);
}

// x = a rounded to float32 (the displacement is zero after a re-anchor).
__global__ __launch_bounds__(kBlock) void k_anchor_out(const double* __restrict__ a, float* __restrict__ x,
                                                       int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < N) x[i] = static_cast<float>(a[i]);
}

uint64_t splitmix64(uint64_t& state) {
  uint64_t z = (state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

}  // namespace

void drop_graph(wdb_theta* th) {
  if (th->g_exec) (void)hipGraphExecDestroy(th->g_exec);
  if (th->g_graph) (void)hipGraphDestroy(th->g_graph);
  th->g_exec = nullptr;
  th->g_graph = nullptr;
  th->g_x = nullptr;
  th->g_c = 0;
}

void ensure_workspace(wdb_theta* th) {
  if (th->ws_x0) return;
  const int64_t N = th->N;
  // enough partial-sum blocks for any slice height up to 64, and one per tile
  // of the tiled storage (N / 64 full tiles plus one per small subband)
  const int64_t nb = std::max<int64_t>((N + 64 + kBlock - 1) / kBlock, (N + 63) / 64 + 3 * th->levels + 1);
  th->ws_nblocks = std::max<int64_t>(nb, 1);
  try {
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_x0), N * sizeof(float)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_r), N * sizeof(float)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_y), N * sizeof(float)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_img), N * sizeof(float)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_img2), N * sizeof(float)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_r64), N * sizeof(double)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_a64), N * sizeof(double)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_c), N * sizeof(float)));
    WDB_HIP(hipMemset(th->ws_a64, 0, N * sizeof(double)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_v64), 3 * N * sizeof(double)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_partial), 4 * th->ws_nblocks * sizeof(double)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_scalar), (16 + 4 * kReduceParts) * sizeof(double)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_rho), kRhoChunk * sizeof(double)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_k), sizeof(int)));
    WDB_HIP(hipHostMalloc(reinterpret_cast<void**>(&th->host_scalar), 16 * sizeof(double), hipHostMallocDefault));
  } catch (...) {
    free_workspace(th);
    throw;
  }
}

double power_iteration(wdb_theta* th, const double* start_host, const double* dinv_sqrt, double tol, int max_iters,
                       int* iters_out, hipStream_t s, bool* converged_out) {
  if (converged_out) *converged_out = false;
  ensure_workspace(th);
  const int64_t N = th->N;
  WDB_REQUIRE(max_iters >= 1, WDB_ERR_ARG, "max_iters must be >= 1");
  WDB_REQUIRE(tol >= 0 && std::isfinite(tol), WDB_ERR_ARG, "tol must be finite and >= 0");
  std::vector<double> v(N);
  if (start_host) {
    for (int64_t i = 0; i < N; ++i) {
      WDB_REQUIRE(std::isfinite(start_host[i]), WDB_ERR_NONFINITE, "non-finite start vector");
      v[i] = start_host[i];
    }
  } else {
    uint64_t st = 0x5eedull;
    for (int64_t i = 0; i < N; ++i) v[i] = static_cast<double>(splitmix64(st) >> 11) * 0x1.0p-52 - 1.0;
  }
  double nrm = 0.0;
  for (double x : v) nrm += x * x;
  nrm = std::sqrt(nrm);
  WDB_REQUIRE(nrm > 0.0, WDB_ERR_ARG, "power-iteration start vector is zero");
  for (double& x : v) x /= nrm;
  double* vd = th->ws_v64;
  double* w = vd + N;
  double* u = w + N;
  WDB_HIP(hipMemcpyAsync(vd, v.data(), N * sizeof(double), hipMemcpyHostToDevice, s));
  if (dinv_sqrt) hipLaunchKernelGGL(k_mul, vec_grid(N), dim3(kBlock), 0, s, vd, dinv_sqrt, N);
  const SellView A = view(th->A), At = view(th->At);
  const int G = check_group(th);
  const int64_t nb = G > 0 ? csr_check_blocks(th, G) : partial_blocks(A, At);
  double* part = th->ws_partial;
  std::vector<double> hist(kRhoChunk);
  double prev = 0.0, rho = 0.0;
  int k = 0;
  while (k < max_iters) {
    const int m = std::min(kRhoChunk, max_iters - k);
    for (int j = 0; j < m; ++j) {
      if (G > 0) {
        with_group(G, [&](auto g) {
          constexpr int GG = decltype(g)::value;
          hipLaunchKernelGGL(k_pi_fwd_csr<GG>, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, cview(th->cA),
                             vd, w, part, nb);
          hipLaunchKernelGGL(k_pi_bwd_csr<GG>, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, cview(th->cAt),
                             w, dinv_sqrt, u, part + nb, nb);
        });
      } else {
        hipLaunchKernelGGL(k_pi_fwd, slot_grid(A), dim3(kBlock), 0, s, A, vd, w, part, nb);
        hipLaunchKernelGGL(k_pi_bwd, slot_grid(At), dim3(kBlock), 0, s, At, w, dinv_sqrt, u, part + nb, nb);
      }
      hipLaunchKernelGGL(k_pi_finish, dim3(1), dim3(kBlock), 0, s, part, nb, th->ws_rho, j, th->ws_scalar);
      hipLaunchKernelGGL(k_pi_scale, vec_grid(N), dim3(kBlock), 0, s, u, dinv_sqrt, th->ws_scalar, vd, N);
    }
    WDB_HIP(hipGetLastError());
    WDB_HIP(hipMemcpyAsync(hist.data(), th->ws_rho, m * sizeof(double), hipMemcpyDeviceToHost, s));
    WDB_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < m; ++j) {
      const int kk = k + j + 1;
      rho = hist[j];
      WDB_REQUIRE(std::isfinite(rho), WDB_ERR_DIVERGED, "power iteration produced a non-finite value");
      if (kk >= 2 && std::fabs(rho - prev) <= tol * rho) {
        if (iters_out) *iters_out = kk;
        if (converged_out) *converged_out = true;
        return rho;
      }
      prev = rho;
    }
    k += m;
  }
  if (iters_out) *iters_out = max_iters;
  return rho;
}

namespace {

// ---------------------------------------------------------------------------
// Lanczos for lambda_max of M = D Theta_K^T Theta_K D (float64, full
// reorthogonalisation), the largest Ritz value of the tridiagonal projection.
// ---------------------------------------------------------------------------
constexpr int kDotChunk = 8192;  // elements per block of the basis dot products

// partial[i * nchunk + c] = sum over chunk c of V_i . u, for basis vectors i < m.
__global__ __launch_bounds__(kBlock) void k_basis_dots(const double* __restrict__ V, int64_t N,
                                                       const double* __restrict__ u, double* __restrict__ partial,
                                                       int64_t nchunk) {
  const int i = blockIdx.y;
  const double* __restrict__ v = V + static_cast<int64_t>(i) * N;
  const int64_t beg = static_cast<int64_t>(blockIdx.x) * kDotChunk;
  const int64_t end = min(beg + kDotChunk, N);
  double acc = 0.0;
  for (int64_t k = beg + threadIdx.x; k < end; k += kBlock) acc = fma(v[k], u[k], acc);
  double vv[1] = {acc};
  __shared__ double sh[kWaves];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int off = kWave / 2; off > 0; off >>= 1) vv[0] += __shfl_xor(vv[0], off);
  if (lane == 0) sh[wid] = vv[0];
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
    for (int w = 1; w < kWaves; ++w) t += sh[w];
    partial[static_cast<int64_t>(i) * nchunk + blockIdx.x] = t;
  }
}

// h[i] = sum_c partial[i * nchunk + c], one block per basis vector (fixed order).
__global__ __launch_bounds__(kBlock) void k_basis_dots_fin(const double* __restrict__ partial, int64_t nchunk,
                                                           double* __restrict__ h) {
  __shared__ double sh[kBlock];
  double acc = 0.0;
  for (int64_t c = threadIdx.x; c < nchunk; c += kBlock) acc += partial[static_cast<int64_t>(blockIdx.x) * nchunk + c];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) h[blockIdx.x] = sh[0];
}

// u -= sum_{i < m} h[i] V_i, and the block partials of ||u||^2 after the update.
__global__ __launch_bounds__(kBlock) void k_basis_orth(const double* __restrict__ V, int64_t N, int m,
                                                       const double* __restrict__ h, double* __restrict__ u,
                                                       double* __restrict__ partial, int64_t nblocks) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  double v[1] = {0.0};
  if (k < N) {
    double acc = u[k];
    for (int i = 0; i < m; ++i) acc = fma(-h[i], V[static_cast<int64_t>(i) * N + k], acc);
    u[k] = acc;
    v[0] = acc * acc;
  }
  block_partials<1, 0u>(v, partial, nblocks);
}

// dst = src * scal[0]; vd = d .* dst (or dst; vd may alias src).
__global__ __launch_bounds__(kBlock) void k_basis_next(const double* src, const double* __restrict__ scal,
                                                       double* __restrict__ dst, const double* __restrict__ d,
                                                       double* vd, int64_t N) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= N) return;
  const double v = src[k] * scal[0];
  dst[k] = v;
  vd[k] = d ? v * d[k] : v;
}

// out = sum_{i < m} s[i] V_i (the Ritz vector of the restart).
__global__ __launch_bounds__(kBlock) void k_ritz_vector(const double* __restrict__ V, int64_t N, int m,
                                                        const double* __restrict__ sv, double* __restrict__ out) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= N) return;
  double acc = 0.0;
  for (int i = 0; i < m; ++i) acc = fma(sv[i], V[static_cast<int64_t>(i) * N + k], acc);
  out[k] = acc;
}

// Block partials of ||u||^2.
__global__ __launch_bounds__(kBlock) void k_sq_partials(const double* __restrict__ u, int64_t N,
                                                        double* __restrict__ partial, int64_t nblocks) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  double v[1] = {k < N ? u[k] * u[k] : 0.0};
  block_partials<1, 0u>(v, partial, nblocks);
}

// scal[0] = 1 / sqrt(sum of partials) (0 for a zero vector), scal[1] = the norm.
__global__ __launch_bounds__(kBlock) void k_inv_norm(const double* __restrict__ partial, int64_t nblocks,
                                                     double* __restrict__ scal) {
  __shared__ double sh[kBlock];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < nblocks; i += kBlock) a += partial[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nrm = sqrt(sh[0]);
    scal[0] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    scal[1] = nrm;
  }
}

}  // namespace

LanczosResult lanczos_core(int64_t N, const std::function<void(const double*, double*)>& apply,
                           const double* start_host, double tol, int max_steps, hipStream_t s, int cycle) {
  WDB_REQUIRE(max_steps >= 1, WDB_ERR_ARG, "max_steps must be >= 1");
  WDB_REQUIRE(tol >= 0 && std::isfinite(tol), WDB_ERR_ARG, "tol must be finite and >= 0");
  std::vector<double> v(N);
  if (start_host) {
    for (int64_t i = 0; i < N; ++i) {
      WDB_REQUIRE(std::isfinite(start_host[i]), WDB_ERR_NONFINITE, "non-finite start vector");
      v[i] = start_host[i];
    }
  } else {
    uint64_t st = 0x5eedull;
    for (int64_t i = 0; i < N; ++i) v[i] = static_cast<double>(splitmix64(st) >> 11) * 0x1.0p-52 - 1.0;
  }
  double nrm = 0.0;
  for (double x : v) nrm += x * x;
  nrm = std::sqrt(nrm);
  WDB_REQUIRE(nrm > 0.0, WDB_ERR_ARG, "Lanczos start vector is zero");
  for (double& x : v) x /= nrm;
  // a cycle builds at most k steps from its start vector, then restarts from
  // the top Ritz vector: the basis holds k + 1 vectors of N doubles
  const int k = static_cast<int>(std::min<int64_t>(std::max(cycle, 2), N));
  DevBuf<double> V(static_cast<size_t>(k + 1) * N);
  DevBuf<double> ub(N);
  double* u = ub.p;
  const int64_t nchunk = (N + kDotChunk - 1) / kDotChunk;
  DevBuf<double> dpart(static_cast<size_t>(k + 1) * nchunk);
  DevBuf<double> hh(2 * static_cast<size_t>(k + 1));
  DevBuf<double> sv(static_cast<size_t>(k + 1));
  const int64_t nbv = vec_grid(N).x;
  DevBuf<double> npart(nbv);
  DevBuf<double> scal(2);
  WDB_HIP(hipMemcpyAsync(V.p, v.data(), N * sizeof(double), hipMemcpyHostToDevice, s));
  LanczosResult res{0.0, 0.0, 0, false};
  double hstep[2], bn[2];
  while (res.steps < max_steps) {
    std::vector<double> alpha, beta;
    TopRitz tr{0.0, 1.0, {}};
    bool done = false;
    for (int j = 0; j < k && res.steps < max_steps; ++j) {
      apply(V.p + static_cast<int64_t>(j) * N, u);   // u = M v_j
      // two passes of classical Gram-Schmidt against v_0..v_j; the
      // coefficients of v_j add up to alpha_j
      const int m = j + 1;
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_basis_dots, dim3(static_cast<unsigned>(nchunk), static_cast<unsigned>(m)), dim3(kBlock),
                           0, s, V.p, N, u, dpart.p, nchunk);
        hipLaunchKernelGGL(k_basis_dots_fin, dim3(static_cast<unsigned>(m)), dim3(kBlock), 0, s, dpart.p, nchunk,
                           hh.p + pass * (k + 1));
        hipLaunchKernelGGL(k_basis_orth, vec_grid(N), dim3(kBlock), 0, s, V.p, N, m, hh.p + pass * (k + 1), u,
                           npart.p, nbv);
      }
      hipLaunchKernelGGL(k_inv_norm, dim3(1), dim3(kBlock), 0, s, npart.p, nbv, scal.p);
      WDB_HIP(hipGetLastError());
      WDB_HIP(hipMemcpyAsync(&hstep[0], hh.p + j, sizeof(double), hipMemcpyDeviceToHost, s));
      WDB_HIP(hipMemcpyAsync(&hstep[1], hh.p + (k + 1) + j, sizeof(double), hipMemcpyDeviceToHost, s));
      WDB_HIP(hipMemcpyAsync(bn, scal.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      WDB_HIP(hipStreamSynchronize(s));
      ++res.steps;
      alpha.push_back(hstep[0] + hstep[1]);
      WDB_REQUIRE(std::isfinite(alpha.back()) && std::isfinite(bn[1]), WDB_ERR_DIVERGED,
                  "Lanczos produced a non-finite value");
      const double bj = bn[1];
      tr = top_ritz(alpha, beta);
      res.theta = tr.theta;
      res.resid = bj * std::fabs(tr.last);
      if (res.resid <= tol * std::fabs(tr.theta) || bj == 0.0) {
        res.converged = true;
        done = true;
        break;
      }
      beta.push_back(bj);
      if (j + 1 < k)   // v_{j+1} = u / beta_j
        hipLaunchKernelGGL(k_basis_next, vec_grid(N), dim3(kBlock), 0, s, u, scal.p,
                           V.p + static_cast<int64_t>(j + 1) * N, static_cast<const double*>(nullptr),
                           V.p + static_cast<int64_t>(j + 1) * N, N);
    }
    if (done || res.steps >= max_steps) break;
    // restart from the top Ritz vector V s (normalised)
    const int m = static_cast<int>(tr.vec.size());
    WDB_HIP(hipMemcpyAsync(sv.p, tr.vec.data(), m * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ritz_vector, vec_grid(N), dim3(kBlock), 0, s, V.p, N, m, sv.p, u);
    hipLaunchKernelGGL(k_sq_partials, vec_grid(N), dim3(kBlock), 0, s, u, N, npart.p, nbv);
    hipLaunchKernelGGL(k_inv_norm, dim3(1), dim3(kBlock), 0, s, npart.p, nbv, scal.p);
    hipLaunchKernelGGL(k_basis_next, vec_grid(N), dim3(kBlock), 0, s, u, scal.p, V.p, static_cast<const double*>(nullptr),
                       V.p, N);
    WDB_HIP(hipGetLastError());
  }
  WDB_HIP(hipStreamSynchronize(s));
  return res;
}

LanczosResult lanczos_max(wdb_theta* th, const double* start_host, const double* dinv_sqrt, double tol, int max_steps,
                          hipStream_t s, int cycle) {
  ensure_workspace(th);
  const int64_t N = th->N;
  double* vd = th->ws_v64;
  double* w = vd + N;
  const SellView A = view(th->A), At = view(th->At);
  const int G = check_group(th);
  const int64_t nb = G > 0 ? csr_check_blocks(th, G) : partial_blocks(A, At);
  double* part = th->ws_partial;
  // u = D A^T A D v
  auto apply = [&](const double* v, double* u) {
    WDB_HIP(hipMemcpyAsync(vd, v, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (dinv_sqrt) hipLaunchKernelGGL(k_mul, vec_grid(N), dim3(kBlock), 0, s, vd, dinv_sqrt, N);
    if (G > 0) {
      with_group(G, [&](auto g) {
        constexpr int GG = decltype(g)::value;
        hipLaunchKernelGGL(k_pi_fwd_csr<GG>, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, cview(th->cA), vd,
                           w, part, nb);
        hipLaunchKernelGGL(k_pi_bwd_csr<GG>, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, cview(th->cAt), w,
                           dinv_sqrt, u, part + nb, nb);
      });
    } else {
      hipLaunchKernelGGL(k_pi_fwd, slot_grid(A), dim3(kBlock), 0, s, A, vd, w, part, nb);
      hipLaunchKernelGGL(k_pi_bwd, slot_grid(At), dim3(kBlock), 0, s, At, w, dinv_sqrt, u, part + nb, nb);
    }
  };
  return lanczos_core(N, apply, start_host, tol, max_steps, s, cycle);
}

namespace {

struct Check {
  double E, rel_gap;
};

// Enqueue the float64 stopping-test products and their reduction into four
// device doubles at `dst`: ||r||^2, <r, x0>, sum w|x|, max |g_i| / w_i.
// With `cneg` (tiled layouts only) the forward product also writes -r64 as
// float32 there; returns whether it did.
template <typename X>
bool enqueue_check(wdb_theta* th, const X* x, const float* x0, double* dst, hipStream_t s, float* cneg = nullptr) {
  const SellView A = view(th->A), At = view(th->At);
  const bool tiled = kernel_group(th) == kTiled;
  const int G = check_group(th);
  const int64_t nb = tiled ? tiled_check_blocks(th) : G > 0 ? csr_check_blocks(th, G) : partial_blocks(A, At);
  WDB_REQUIRE(nb <= th->ws_nblocks, WDB_ERR_ARG, "partial-sum workspace too small");
  double* part = th->ws_partial;
  if (tiled) {
    launch_objective_tiled(th, x, x0, th->ws_r64, part, nb, s, cneg);
  } else if (G > 0) {
    with_group(G, [&](auto g) {
      constexpr int GG = decltype(g)::value;
      hipLaunchKernelGGL((k_obj_fwd_csr<GG, X>), dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, cview(th->cA),
                         x, x0, th->l1w, th->ws_r64, part, nb);
      hipLaunchKernelGGL(k_obj_bwd_csr<GG>, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, cview(th->cAt),
                         th->ws_r64, th->l1w, part + 3 * nb, nb);
    });
  } else {
    hipLaunchKernelGGL(k_obj_fwd<X>, slot_grid(A), dim3(kBlock), 0, s, A, x, x0, th->l1w, th->ws_r64, part, nb);
    hipLaunchKernelGGL(k_obj_bwd, slot_grid(At), dim3(kBlock), 0, s, At, th->ws_r64, th->l1w, part + 3 * nb, nb);
  }
  double* tmp = th->ws_scalar + 16;  // 4 x kReduceParts doubles after the 16 scalars
  hipLaunchKernelGGL(k_reduce4_part, dim3(kReduceParts), dim3(kReduceThreads), 0, s, part, nb, 0x8u, tmp);
  hipLaunchKernelGGL(k_reduce4_final, dim3(1), dim3(kReduceParts), 0, s, tmp, 0x8u, dst);
  WDB_HIP(hipGetLastError());
  return tiled && cneg;
}

// E and the relative duality gap from the four reduced scalars.
Check check_from(const double* q, double lambda) {
  const double rr = q[0], rb = q[1], l1 = q[2], gmax = q[3];
  const double E = 0.5 * rr + lambda * l1;
  const double sc = gmax <= lambda ? 1.0 : lambda / gmax;
  const double D = -0.5 * sc * sc * rr - sc * rb;
  const double gap = E - D;
  return Check{E, E > 0 ? gap / E : 0.0};
}

template <typename X>
Check objective_check(wdb_theta* th, const X* x, const float* x0, double lambda, hipStream_t s) {
  enqueue_check(th, x, x0, th->ws_scalar, s);
  WDB_HIP(hipMemcpyAsync(th->host_scalar, th->ws_scalar, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  WDB_HIP(hipStreamSynchronize(s));
  return check_from(th->host_scalar, lambda);
}

// One iteration of Alg. 1 (Alg. 2 with `pre`); with `ista` the proximal kernel
// gets no counter and extrapolates with beta = 0 (plain proximal gradient).
// With `anchored` (float32 values only) x and y hold displacements from the
// float64 anchor ws_a64 and the residual subtracts c = x0 - Theta_K a.
void launch_iteration(wdb_theta* th, float* x, bool pre, bool ista, float tau, float thr, hipStream_t s,
                      bool anchored = false) {
  const int* kp = ista ? nullptr : th->ws_k;
  if (th->valtype != WDB_VAL_F32 && th->pA.word && packed_group(th) == kTiled) {
    launch_res_tiled16(th, th->ws_y, th->ws_x0, th->ws_r, th->ws_k, 1, s);
    launch_prox_tiled16(th, th->ws_r, x, th->ws_y, tau, thr, kp, pre ? th->pinv : nullptr,
                        threshold_weights(th, pre), s);
    return;
  }
  if (th->valtype != WDB_VAL_F32 && th->pA.word && packed_group(th) > 0) {
    const int G = packed_group(th);
    launch_res_packed(th, G, th->ws_y, th->ws_x0, th->ws_r, th->ws_k, 1, s);
    launch_prox_packed(th, G, th->ws_r, x, th->ws_y, tau, thr, kp, pre ? th->pinv : nullptr,
                       threshold_weights(th, pre), s);
    return;
  }
  if (th->valtype == WDB_VAL_BF16) return launch_iteration_q<WDB_VAL_BF16>(th, x, pre, kp, tau, thr, s);
  if (th->valtype == WDB_VAL_F16) return launch_iteration_q<WDB_VAL_F16>(th, x, pre, kp, tau, thr, s);
  const int G = kernel_group(th);
  const float* b = anchored ? th->ws_c : th->ws_x0;
  const double* anc = anchored ? th->ws_a64 : nullptr;
  if (G == kTiled) {
    launch_res_tiled(th, false, th->ws_y, b, th->ws_r, th->ws_k, s);
    launch_prox_tiled(th, th->ws_r, x, th->ws_y, tau, thr, 0.0f, kp, pre ? th->pinv : nullptr,
                      threshold_weights(th, pre), anc, s);
    return;
  }
  if (G == kStencil) {
    launch_res_stencil(th, false, th->ws_y, b, th->ws_r, th->ws_k, s);
    launch_prox_stencil(th, th->ws_r, x, th->ws_y, tau, thr, 0.0f, kp, pre ? th->pinv : nullptr,
                        threshold_weights(th, pre), anc, s);
    return;
  }
  launch_res(G, th->A, th->cA, th->ws_y, b, th->ws_r, th->ws_k, s);
  launch_prox(G, th->At, th->cAt, th->ws_r, x, th->ws_y, tau, thr, 0.0f, kp, pre ? th->pinv : nullptr,
              threshold_weights(th, pre), anc, s);
}

// Default step: the Lanczos bound theta + resid (an upper bound of
// lambda_max once the top Ritz pair has converged; larger than needed, never
// smaller, if it has not).
void ensure_lipschitz(wdb_theta* th, hipStream_t s) {
  if (th->has_L) return;
  const LanczosResult r = lanczos_max(th, nullptr, nullptr, 1e-12, 2000, s);
  th->L = r.theta + r.resid;
  th->has_L = true;
}

wdb_status solve_impl(wdb_theta* th, const float* x0_src, bool from_image, float lambda, const wdb_solve_opts* opts,
                      float* x_out, wdb_solve_info* info) {
  WDB_REQUIRE(th && x0_src && opts && x_out, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(std::isfinite(lambda) && lambda >= 0.0f, WDB_ERR_NONFINITE, "lambda must be finite and >= 0");
  WDB_REQUIRE(opts->max_iters >= 0, WDB_ERR_ARG, "max_iters must be >= 0");
  WDB_REQUIRE(opts->check_every >= 0, WDB_ERR_ARG, "check_every must be >= 0");
  WDB_REQUIRE(opts->k0 >= 0, WDB_ERR_ARG, "k0 must be >= 0");
  const bool pre = opts->use_precond != 0;
  WDB_REQUIRE(!pre || th->precond != 0, WDB_ERR_ARG, "no preconditioner set on this operator");
  WDB_HIP(hipSetDevice(th->device));
  hipStream_t s = static_cast<hipStream_t>(opts->stream);
  ensure_workspace(th);
  ensure_lipschitz(th, s);
  const double Luse = pre ? th->Lp : th->L;
  WDB_REQUIRE(Luse > 0.0 && std::isfinite(Luse), WDB_ERR_ARG, "operator has no positive Lipschitz constant");
  const double tau = 1.0 / Luse;
  const float tau_f = static_cast<float>(tau);
  const float thr_f = static_cast<float>(tau * static_cast<double>(lambda));
  const int64_t N = th->N;
  if (from_image) {
    const Filter f = make_filter(th->wavelet);
    const size_t q = static_cast<size_t>(th->n / 2) * (th->n / 2);
    dwt_forward(th->n, th->levels, f, x0_src, th->ws_x0, th->ws_img, th->ws_img + q, s);
  } else {
    WDB_HIP(hipMemcpyAsync(th->ws_x0, x0_src, N * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  hipLaunchKernelGGL(k_copy_or_zero, vec_grid(N), dim3(kBlock), 0, s, opts->x_init, x_out, th->ws_y, N);
  // Float32 values keep the iterate anchored (float64 anchor + float32
  // displacement, re-centred at every check) unless the caller asks for the
  // plain float32 iterate; the 16-bit forms always iterate plainly.
  const bool anchored = th->valtype == WDB_VAL_F32 && opts->plain_iterate == 0;
  if (anchored) hipLaunchKernelGGL(k_anchor_init, vec_grid(N), dim3(kBlock), 0, s, th->ws_a64, th->ws_c, th->ws_x0, N);
  // A check: with the anchored iterate the displacement first moves into the
  // anchor, the float64 products run on the anchor, and their residual gives
  // the next right-hand side.
  auto enqueue_point = [&](double* dst) {
    if (!anchored) {
      enqueue_check(th, static_cast<const float*>(x_out), th->ws_x0, dst, s);
      return;
    }
    hipLaunchKernelGGL(k_reanchor, vec_grid(N), dim3(kBlock), 0, s, th->ws_a64, x_out, th->ws_y, N);
    if (!enqueue_check(th, static_cast<const double*>(th->ws_a64), th->ws_x0, dst, s, th->ws_c))
      hipLaunchKernelGGL(k_anchor_rhs, vec_grid(N), dim3(kBlock), 0, s, th->ws_r64, th->ws_c, N);
    WDB_HIP(hipGetLastError());
  };
  auto check_point = [&]() {
    enqueue_point(th->ws_scalar);
    WDB_HIP(hipMemcpyAsync(th->host_scalar, th->ws_scalar, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    WDB_HIP(hipStreamSynchronize(s));
    return check_from(th->host_scalar, lambda);
  };
  const int k0 = opts->k0 > 0 ? opts->k0 : 1;
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, th->ws_k, k0 - 1);
  WDB_HIP(hipGetLastError());

  const int c = opts->check_every;
  const int total = opts->max_iters;
  int done = 0, checks = 0;
  Check last{0.0, 0.0};
  bool converged = false;
  hipGraphExec_t exec = nullptr;
  try {
    const bool use_graph = opts->use_graph && c > 1;
    if (use_graph && total >= c) {
      const int ista = opts->ista != 0 ? 1 : 0;
      if (!(th->g_exec && th->g_x == x_out && th->g_c == c && th->g_pre == (pre ? 1 : 0) && th->g_ista == ista &&
            th->g_anchor == (anchored ? 1 : 0) && th->g_tau == tau_f && th->g_thr == thr_f)) {
        drop_graph(th);
        if (!th->capture_stream) WDB_HIP(hipStreamCreateWithFlags(&th->capture_stream, hipStreamNonBlocking));
        WDB_HIP(hipStreamBeginCapture(th->capture_stream, hipStreamCaptureModeThreadLocal));
        try {
          for (int i = 0; i < c; ++i)
            launch_iteration(th, x_out, pre, ista != 0, tau_f, thr_f, th->capture_stream, anchored);
        } catch (...) {  // end the capture so the stream stays usable
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(th->capture_stream, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        hipGraph_t graph = nullptr;
        WDB_HIP(hipStreamEndCapture(th->capture_stream, &graph));
        th->g_graph = graph;
        WDB_HIP(hipGraphInstantiate(&th->g_exec, graph, nullptr, nullptr, 0));
        th->g_x = x_out;
        th->g_c = c;
        th->g_pre = pre ? 1 : 0;
        th->g_ista = ista;
        th->g_anchor = anchored ? 1 : 0;
        th->g_tau = tau_f;
        th->g_thr = thr_f;
      }
      exec = th->g_exec;
    }
    // Without a stopping test the checks are only recorded: their scalars go to
    // a device array and are read once at the end, so the host never waits
    // between the graph launches.
    const bool stop_test = opts->tol_rel_gap > 0 || opts->target_objective > 0;
    std::vector<int> at_iter;
    if (!stop_test) {
      const int64_t ncheck = (c > 0 ? total / c : 0) + 1;
      if (ncheck > th->ws_ncheck) {
        if (th->ws_checks) (void)hipFree(th->ws_checks);
        th->ws_checks = nullptr;
        th->ws_ncheck = 0;
        WDB_HIP(hipMalloc(reinterpret_cast<void**>(&th->ws_checks), 4 * ncheck * sizeof(double)));
        th->ws_ncheck = ncheck;
      }
    }
    // With the anchored iterate the next block of iterations is enqueued before
    // the host reads a check: the iterations only change the displacement, so
    // the anchor still holds the checked iterate if the check stops the solve
    // (the final output is taken from the anchor), and the GPU does not idle
    // while the host waits for the check's scalars.
    bool ahead = false;  // the block after the last check is already enqueued
    while (done < total) {
      int step = total - done;
      if (c > 0) step = std::min(step, c - (done % c));
      if (ahead) {
        ahead = false;
      } else if (exec && step == c) {
        WDB_HIP(hipGraphLaunch(exec, s));
      } else {
        for (int i = 0; i < step; ++i) launch_iteration(th, x_out, pre, opts->ista != 0, tau_f, thr_f, s, anchored);
        WDB_HIP(hipGetLastError());
      }
      done += step;
      const bool at_check = (c > 0 && done % c == 0) || done == total;
      if (at_check && !stop_test) {
        enqueue_point(th->ws_checks + 4 * at_iter.size());
        at_iter.push_back(done);
      } else if (at_check && anchored && exec && total - done >= c) {
        if (!th->check_event) WDB_HIP(hipEventCreateWithFlags(&th->check_event, hipEventDisableTiming));
        enqueue_point(th->ws_scalar);
        WDB_HIP(hipMemcpyAsync(th->host_scalar, th->ws_scalar, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        WDB_HIP(hipEventRecord(th->check_event, s));
        WDB_HIP(hipGraphLaunch(exec, s));
        ahead = true;
        WDB_HIP(hipEventSynchronize(th->check_event));
        last = check_from(th->host_scalar, lambda);
      } else if (at_check) {
        last = check_point();
      }
      if (at_check && stop_test) {
        ++checks;
        if (opts->trace && checks <= opts->trace_cap) {
          opts->trace[3 * (checks - 1) + 0] = static_cast<double>(k0 - 1 + done);
          opts->trace[3 * (checks - 1) + 1] = last.E;
          opts->trace[3 * (checks - 1) + 2] = last.rel_gap;
        }
        WDB_REQUIRE(std::isfinite(last.E), WDB_ERR_DIVERGED, "objective became non-finite at iteration %d",
                    k0 - 1 + done);
        if ((opts->tol_rel_gap > 0 && last.rel_gap <= opts->tol_rel_gap) ||
            (opts->target_objective > 0 && last.E <= opts->target_objective)) {
          converged = true;
          break;
        }
      }
    }
    if (!at_iter.empty()) {
      std::vector<double> q(4 * at_iter.size());
      WDB_HIP(hipMemcpyAsync(q.data(), th->ws_checks, q.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      WDB_HIP(hipStreamSynchronize(s));
      for (size_t j = 0; j < at_iter.size(); ++j) {
        last = check_from(&q[4 * j], lambda);
        ++checks;
        if (opts->trace && checks <= opts->trace_cap) {
          opts->trace[3 * (checks - 1) + 0] = static_cast<double>(k0 - 1 + at_iter[j]);
          opts->trace[3 * (checks - 1) + 1] = last.E;
          opts->trace[3 * (checks - 1) + 2] = last.rel_gap;
        }
        WDB_REQUIRE(std::isfinite(last.E), WDB_ERR_DIVERGED, "objective became non-finite at iteration %d",
                    k0 - 1 + at_iter[j]);
      }
    }
    if (total == 0) {
      last = check_point();
      ++checks;
    }
    if (anchored) {  // every solve ends on a check, which leaves a zero displacement
      hipLaunchKernelGGL(k_anchor_out, vec_grid(N), dim3(kBlock), 0, s, th->ws_a64, x_out, N);
      if (opts->x64_out)
        WDB_HIP(hipMemcpyAsync(opts->x64_out, th->ws_a64, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else if (opts->x64_out) {
      hipLaunchKernelGGL(k_widen, vec_grid(N), dim3(kBlock), 0, s, x_out, opts->x64_out, N);
    }
    WDB_HIP(hipGetLastError());
  } catch (...) {
    (void)hipStreamSynchronize(s);  // no replay in flight when the graph goes
    drop_graph(th);                 // a failed capture or replay leaves no graph behind
    throw;
  }
  if (info) {
    info->iters = done;
    info->checks = checks;
    info->objective = last.E;
    info->rel_gap = last.rel_gap;
    info->lipschitz = Luse;
    info->tau = tau;
  }
  if ((opts->tol_rel_gap > 0 || opts->target_objective > 0) && !converged)
    fail(WDB_ERR_NOT_CONVERGED, "stopping test not met after %d iterations (relative gap %.3e, objective %.9e)",
         done, last.rel_gap, last.E);
  return WDB_OK;
}

}  // namespace

}  // namespace wdb

extern "C" {

wdb_status wdb_theta_lipschitz(wdb_theta* th, const double* start, double tol, int32_t max_iters, double* L_out,
                               int32_t* iters_out) {
  WDB_API_BEGIN
  WDB_REQUIRE(th, WDB_ERR_ARG, "null handle");
  wdb::drop_graph(th);  // the cached iteration graph may refer to what this call changes
  WDB_HIP(hipSetDevice(th->device));
  int it = 0;
  bool converged = false;
  const double L = wdb::power_iteration(th, start, nullptr, tol, max_iters, &it, nullptr, &converged);
  th->L = L;
  th->has_L = true;
  if (L_out) *L_out = L;
  if (iters_out) *iters_out = it;
  if (!converged)
    wdb::fail(WDB_ERR_NOT_CONVERGED, "power iteration reached max_iters = %d without a relative change <= %.3g "
              "(L = %.17g is a lower bound of ||Theta_K||^2)", max_iters, tol, L);
  WDB_API_END
}

wdb_status wdb_theta_lipschitz_lanczos(wdb_theta* th, const double* start, double tol, int32_t max_steps,
                                       double* L_out, int32_t* steps_out, double* resid_out) {
  WDB_API_BEGIN
  WDB_REQUIRE(th, WDB_ERR_ARG, "null handle");
  wdb::drop_graph(th);  // the cached iteration graph may refer to what this call changes
  WDB_HIP(hipSetDevice(th->device));
  const wdb::LanczosResult r = wdb::lanczos_max(th, start, nullptr, tol, max_steps, nullptr);
  th->L = r.theta + r.resid;
  th->has_L = true;
  if (L_out) *L_out = th->L;
  if (steps_out) *steps_out = r.steps;
  if (resid_out) *resid_out = r.resid;
  if (!r.converged)
    wdb::fail(WDB_ERR_NOT_CONVERGED, "Lanczos reached max_steps = %d with residual %.3e > tol * theta "
              "(theta = %.17g; L = theta + residual stored)", max_steps, r.resid, r.theta);
  WDB_API_END
}

wdb_status wdb_solve(wdb_theta* th, const float* u, float lambda, const wdb_solve_opts* opts, float* x_out,
                     wdb_solve_info* info) {
  WDB_API_BEGIN
  return wdb::solve_impl(th, u, true, lambda, opts, x_out, info);
  WDB_API_END
}

wdb_status wdb_solve_coeffs(wdb_theta* th, const float* x0, float lambda, const wdb_solve_opts* opts, float* x_out,
                            wdb_solve_info* info) {
  WDB_API_BEGIN
  return wdb::solve_impl(th, x0, false, lambda, opts, x_out, info);
  WDB_API_END
}

wdb_status wdb_objective(wdb_theta* th, const float* x, const float* x0, float lambda, void* stream, double* E_out,
                         double* rel_gap_out) {
  WDB_API_BEGIN
  WDB_REQUIRE(th && x && x0, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(std::isfinite(lambda) && lambda >= 0.0f, WDB_ERR_NONFINITE, "lambda must be finite and >= 0");
  WDB_HIP(hipSetDevice(th->device));
  wdb::ensure_workspace(th);
  const auto c = wdb::objective_check(th, x, x0, lambda, static_cast<hipStream_t>(stream));
  if (E_out) *E_out = c.E;
  if (rel_gap_out) *rel_gap_out = c.rel_gap;
  WDB_API_END
}

wdb_status wdb_theta_apply(wdb_theta* th, int32_t transpose, const float* x, const float* b, float* y,
                           int32_t repeat, void* stream) {
  WDB_API_BEGIN
  WDB_REQUIRE(th && x && y, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(x != y, WDB_ERR_ARG, "x and y must not alias");
  WDB_REQUIRE(repeat >= 1, WDB_ERR_ARG, "repeat must be >= 1");
  WDB_HIP(hipSetDevice(th->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (th->valtype != WDB_VAL_F32) {
    WDB_REQUIRE(!transpose, WDB_ERR_ARG, "transposed apply is not available with 16-bit values");
    if (th->pA.word && wdb::packed_group(th) == wdb::kTiled) {
      for (int i = 0; i < repeat; ++i) wdb::launch_res_tiled16(th, x, b, y, nullptr, 0, s);
      WDB_HIP(hipGetLastError());
      return WDB_OK;
    }
    if (th->pA.word && wdb::packed_group(th) > 0) {
      for (int i = 0; i < repeat; ++i) wdb::launch_res_packed(th, wdb::packed_group(th), x, b, y, nullptr, 0, s);
      WDB_HIP(hipGetLastError());
      return WDB_OK;
    }
    const wdb::SellView A = wdb::view(th->A);
    const uint2* v16 = reinterpret_cast<const uint2*>(th->val16);
    for (int i = 0; i < repeat; ++i) {
      if (th->valtype == WDB_VAL_BF16)
        hipLaunchKernelGGL(wdb::k_res_q<WDB_VAL_BF16>, wdb::slot_grid(A), dim3(wdb::kBlock), 0, s, A, v16,
                           th->wrow, x, b, y, static_cast<int*>(nullptr), 0);
      else
        hipLaunchKernelGGL(wdb::k_res_q<WDB_VAL_F16>, wdb::slot_grid(A), dim3(wdb::kBlock), 0, s, A, v16,
                           th->wrow, x, b, y, static_cast<int*>(nullptr), 0);
    }
    WDB_HIP(hipGetLastError());
    return WDB_OK;
  }
  const int G = wdb::kernel_group(th);
  for (int i = 0; i < repeat; ++i) {
    if (G == wdb::kTiled)
      wdb::launch_res_tiled(th, transpose != 0, x, b, y, nullptr, s);
    else if (G == wdb::kStencil)
      wdb::launch_res_stencil(th, transpose != 0, x, b, y, nullptr, s);
    else
      wdb::launch_res(G, transpose ? th->At : th->A, transpose ? th->cAt : th->cA, x, b, y, nullptr, s);
  }
  WDB_HIP(hipGetLastError());
  WDB_API_END
}

wdb_status wdb_prox_step(wdb_theta* th, const float* r, float* x, float* y, float tau, float lambda, float beta,
                         int32_t use_precond, void* stream) {
  WDB_API_BEGIN
  WDB_REQUIRE(th && r && x && y, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(!use_precond || th->pinv, WDB_ERR_ARG, "no preconditioner set on this operator");
  WDB_REQUIRE(th->valtype == WDB_VAL_F32, WDB_ERR_ARG, "prox_step needs float32 values");
  WDB_HIP(hipSetDevice(th->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float thr = tau * lambda;
  if (wdb::kernel_group(th) == wdb::kTiled)
    wdb::launch_prox_tiled(th, r, x, y, tau, thr, beta, nullptr, use_precond ? th->pinv : nullptr,
                           wdb::threshold_weights(th, use_precond != 0), nullptr, s);
  else if (wdb::kernel_group(th) == wdb::kStencil)
    wdb::launch_prox_stencil(th, r, x, y, tau, thr, beta, nullptr, use_precond ? th->pinv : nullptr,
                             wdb::threshold_weights(th, use_precond != 0), nullptr, s);
  else
    wdb::launch_prox(wdb::kernel_group(th), th->At, th->cAt, r, x, y, tau, thr, beta, nullptr,
                     use_precond ? th->pinv : nullptr, wdb::threshold_weights(th, use_precond != 0), nullptr, s);
  WDB_HIP(hipGetLastError());
  WDB_API_END
}

}  // extern "C"
