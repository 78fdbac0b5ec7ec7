// Periodic separable 2D orthogonal wavelet transform on the GPU (Sec. 2:
// tensor-product wavelets at one scale, circular boundaries), float32.
//
// One launch per level.  Forward: each block owns an 8 x 32 tile of output
// positions (i, j) of the level's four subbands,
//   c_e[i][j] = sum_{m, m'} f_erow[m] f_ecol[m'] A[(2i+m) mod M][(2j+m') mod M]
// with f_0 = h (low-pass) and f_1 = g (high-pass): it stages the tile's input
// footprint (16 + L - 2 rows of 64 + L - 2 columns, periodic) in LDS with
// coalesced loads, filters the rows (low and high pass, every input row of
// the footprint once) into LDS, then the columns, and writes the four
// subbands row-contiguously.  Inverse (the transpose of the forward map):
// each block owns an 8 x 32 tile of output pixels, stages the four subbands'
// half-resolution footprint (4 + 6 rows of 16 + 6 columns, periodic) in LDS,
// and every thread sums the (L/2)^2 coefficients of each subband that cover
// its pixel from there.
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace wdb {
namespace {

struct Taps {
  float h[kMaxTaps];
  float g[kMaxTaps];
  int L;
};

Taps to_taps(const Filter& f) {
  Taps t{};
  t.L = static_cast<int>(f.h.size());
  for (int i = 0; i < t.L; ++i) {
    t.h[i] = static_cast<float>(f.h[i]);
    t.g[i] = static_cast<float>(f.g[i]);
  }
  return t;
}

constexpr int kTI = 8, kTJ = 32;                    // output tile of a forward block
constexpr int kRI = 2 * kTI + kMaxTaps - 2;          // input rows of its footprint (at most)
constexpr int kCI = 2 * kTJ + kMaxTaps - 2;          // input columns of its footprint (at most)

// Up to kBatch images per launch (blockIdx.z): per image the level's input,
// its approximation output and the coefficient vector holding its details.
constexpr int kBatch = 8;
struct FwdPtrs {
  const float* src[kBatch];
  float* ll[kBatch];
  float* out[kBatch];
};
struct InvPtrs {
  const float* ll[kBatch];
  const float* in[kBatch];
  float* dst[kBatch];
};

__global__ __launch_bounds__(256) void k_dwt_fwd_level(FwdPtrs P, int M, int64_t o01, int64_t o10, int64_t o11,
                                                       Taps t) {
  const float* __restrict__ A = P.src[blockIdx.z];
  float* __restrict__ LL = P.ll[blockIdx.z];
  float* __restrict__ d01 = P.out[blockIdx.z] + o01;
  float* __restrict__ d10 = P.out[blockIdx.z] + o10;
  float* __restrict__ d11 = P.out[blockIdx.z] + o11;
  __shared__ float in[kRI][kCI];
  __shared__ float lo[kRI][kTJ], hi[kRI][kTJ];
  const int Mh = M >> 1;
  const int i0 = blockIdx.y * kTI, j0 = blockIdx.x * kTJ;
  const int rows = 2 * kTI + t.L - 2, cols = 2 * kTJ + t.L - 2;
  for (int idx = threadIdx.x; idx < rows * cols; idx += blockDim.x) {
    const int r = idx / cols, c = idx - r * cols;
    in[r][c] = A[static_cast<size_t>((2 * i0 + r) & (M - 1)) * M + ((2 * j0 + c) & (M - 1))];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < rows * kTJ; idx += blockDim.x) {
    const int r = idx / kTJ, j = idx - r * kTJ;
    float l = 0.f, h = 0.f;
    for (int m2 = 0; m2 < t.L; ++m2) {
      const float v = in[r][2 * j + m2];
      l = fmaf(t.h[m2], v, l);
      h = fmaf(t.g[m2], v, h);
    }
    lo[r][j] = l;
    hi[r][j] = h;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kTI * kTJ; idx += blockDim.x) {
    const int i = idx / kTJ, j = idx - i * kTJ;
    if (i0 + i >= Mh || j0 + j >= Mh) continue;
    float a00 = 0.f, a01 = 0.f, a10 = 0.f, a11 = 0.f;
    for (int m = 0; m < t.L; ++m) {
      const float l = lo[2 * i + m][j], h = hi[2 * i + m][j];
      a00 = fmaf(t.h[m], l, a00);
      a01 = fmaf(t.h[m], h, a01);
      a10 = fmaf(t.g[m], l, a10);
      a11 = fmaf(t.g[m], h, a11);
    }
    const size_t o = static_cast<size_t>(i0 + i) * Mh + j0 + j;
    LL[o] = a00;
    d01[o] = a01;
    d10[o] = a10;
    d11[o] = a11;
  }
}

constexpr int kTP = 8, kTQ = 32;                   // output tile of an inverse block (full resolution)
constexpr int kHalo = kMaxTaps / 2;                  // half-resolution rows / columns below the tile
constexpr int kRP = kTP / 2 + kHalo, kCQ = kTQ / 2 + kHalo;

__global__ __launch_bounds__(256) void k_dwt_inv_level(InvPtrs P, int64_t o01, int64_t o10, int64_t o11, int Mh,
                                                       Taps t) {
  const float* __restrict__ LL = P.ll[blockIdx.z];
  const float* __restrict__ d01 = P.in[blockIdx.z] + o01;
  const float* __restrict__ d10 = P.in[blockIdx.z] + o10;
  const float* __restrict__ d11 = P.in[blockIdx.z] + o11;
  float* __restrict__ out = P.dst[blockIdx.z];
  __shared__ float sb[4][kRP][kCQ];
  const int M = Mh << 1;
  const int p0 = blockIdx.y * kTP, q0 = blockIdx.x * kTQ;
  const int ib = (p0 >> 1) - kHalo, jb = (q0 >> 1) - kHalo;  // half-resolution origin of the footprint
  for (int idx = threadIdx.x; idx < kRP * kCQ; idx += blockDim.x) {
    const int r = idx / kCQ, c = idx - r * kCQ;
    const size_t g = static_cast<size_t>((ib + r) & (Mh - 1)) * Mh + ((jb + c) & (Mh - 1));
    sb[0][r][c] = LL[g];
    sb[1][r][c] = d01[g];
    sb[2][r][c] = d10[g];
    sb[3][r][c] = d11[g];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kTP * kTQ; idx += blockDim.x) {
    const int pp = idx / kTQ, qq = idx - pp * kTQ;
    const int p = p0 + pp, q = q0 + qq;
    if (p >= M || q >= M) continue;
    float acc = 0.f;
    for (int m = p & 1; m < t.L; m += 2) {
      const int r = ((p - m) >> 1) - ib;
      const float hr = t.h[m], gr = t.g[m];
      for (int m2 = q & 1; m2 < t.L; m2 += 2) {
        const int c = ((q - m2) >> 1) - jb;
        acc = fmaf(hr * t.h[m2], sb[0][r][c], acc);
        acc = fmaf(hr * t.g[m2], sb[1][r][c], acc);
        acc = fmaf(gr * t.h[m2], sb[2][r][c], acc);
        acc = fmaf(gr * t.g[m2], sb[3][r][c], acc);
      }
    }
    out[static_cast<size_t>(p) * M + q] = acc;
  }
}

}  // namespace

// Detail subband offsets of level `lev` in the canonical layout.
static void level_offsets(int n, int levels, int lev, int64_t off[3]) {
  for (const Subband& sb : layout(n, levels))
    if (sb.level == lev && !(sb.erow == 0 && sb.ecol == 0)) {
      const int k = sb.erow * 2 + sb.ecol - 1;  // (0,1)->0, (1,0)->1, (1,1)->2
      off[k] = sb.offset;
    }
}

void dwt_forward_many(int n, int levels, const Filter& f, int count, const float* const* in, float* const* out,
                      float* const* scratch_a, float* const* scratch_b, hipStream_t s) {
  const Taps t = to_taps(f);
  for (int b0 = 0; b0 < count; b0 += kBatch) {
    const int nb = std::min(kBatch, count - b0);
    FwdPtrs P{};
    for (int z = 0; z < nb; ++z) P.src[z] = in[b0 + z];
    for (int lev = 1; lev <= levels; ++lev) {
      const int M = n >> (lev - 1);
      const int Mh = M >> 1;
      int64_t off[3];
      level_offsets(n, levels, lev, off);
      for (int z = 0; z < nb; ++z) {
        P.out[z] = out[b0 + z];
        P.ll[z] = (lev == levels) ? out[b0 + z] : ((lev & 1) ? scratch_b : scratch_a)[b0 + z];
      }
      const dim3 grid((Mh + kTJ - 1) / kTJ, (Mh + kTI - 1) / kTI, nb);
      hipLaunchKernelGGL(k_dwt_fwd_level, grid, dim3(256), 0, s, P, M, off[0], off[1], off[2], t);
      WDB_HIP(hipGetLastError());
      for (int z = 0; z < nb; ++z) P.src[z] = P.ll[z];
    }
  }
}

void dwt_inverse_many(int n, int levels, const Filter& f, int count, const float* const* in, float* const* out,
                      float* const* scratch_a, float* const* scratch_b, hipStream_t s) {
  const Taps t = to_taps(f);
  for (int b0 = 0; b0 < count; b0 += kBatch) {
    const int nb = std::min(kBatch, count - b0);
    InvPtrs P{};
    for (int z = 0; z < nb; ++z) {
      P.ll[z] = in[b0 + z];  // A_J sits at offset 0
      P.in[z] = in[b0 + z];
    }
    for (int lev = levels; lev >= 1; --lev) {
      const int Mh = n >> lev;
      const int M = Mh << 1;
      int64_t off[3];
      level_offsets(n, levels, lev, off);
      for (int z = 0; z < nb; ++z) P.dst[z] = (lev == 1) ? out[b0 + z] : ((lev & 1) ? scratch_b : scratch_a)[b0 + z];
      const dim3 grid((M + kTQ - 1) / kTQ, (M + kTP - 1) / kTP, nb);
      hipLaunchKernelGGL(k_dwt_inv_level, grid, dim3(256), 0, s, P, off[0], off[1], off[2], Mh, t);
      WDB_HIP(hipGetLastError());
      for (int z = 0; z < nb; ++z) P.ll[z] = P.dst[z];
    }
  }
}

void dwt_forward(int n, int levels, const Filter& f, const float* in, float* out, float* scratch_a,
                 float* scratch_b, hipStream_t s) {
  dwt_forward_many(n, levels, f, 1, &in, &out, &scratch_a, &scratch_b, s);
}

void dwt_inverse(int n, int levels, const Filter& f, const float* in, float* out, float* scratch_a,
                 float* scratch_b, hipStream_t s) {
  dwt_inverse_many(n, levels, f, 1, &in, &out, &scratch_a, &scratch_b, s);
}

}  // namespace wdb

extern "C" wdb_status wdb_dwt(int32_t n, int32_t wavelet, int32_t levels, const float* in, float* out,
                              int32_t inverse, void* stream) {
  WDB_API_BEGIN
  WDB_REQUIRE(in && out, WDB_ERR_ARG, "null buffer");
  WDB_REQUIRE(in != out, WDB_ERR_ARG, "in and out must not alias");
  wdb::Filter f = wdb::make_filter(wavelet);
  wdb::check_geometry(n, levels, static_cast<int>(f.h.size()));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t q = static_cast<size_t>(n / 2) * (n / 2);
  wdb::DevBuf<float> scratch(2 * q);
  if (inverse)
    wdb::dwt_inverse(n, levels, f, in, out, scratch.p, scratch.p + q, s);
  else
    wdb::dwt_forward(n, levels, f, in, out, scratch.p, scratch.p + q, s);
  WDB_HIP(hipStreamSynchronize(s));
  WDB_API_END
}

extern "C" wdb_status wdb_dwt_batched(int32_t n, int32_t wavelet, int32_t levels, int32_t count, const float* in,
                                      float* out, int32_t inverse, void* stream) {
  WDB_API_BEGIN
  WDB_REQUIRE(in && out, WDB_ERR_ARG, "null buffer");
  WDB_REQUIRE(count >= 1, WDB_ERR_ARG, "count %d must be >= 1", count);
  wdb::Filter f = wdb::make_filter(wavelet);
  wdb::check_geometry(n, levels, static_cast<int>(f.h.size()));
  const int64_t N = static_cast<int64_t>(n) * n;
  const char* ib = reinterpret_cast<const char*>(in);
  const char* ie = reinterpret_cast<const char*>(in + N * count);
  const char* ob = reinterpret_cast<const char*>(out);
  const char* oe = reinterpret_cast<const char*>(out + N * count);
  WDB_REQUIRE(ie <= ob || oe <= ib, WDB_ERR_ARG, "in and out must not overlap");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t q = static_cast<size_t>(n / 2) * (n / 2);
  const int nsc = std::min(count, 8);
  wdb::DevBuf<float> scratch(2 * q * nsc);
  std::vector<const float*> ip(count);
  std::vector<float*> op(count), sa(count), sb(count);
  for (int i = 0; i < count; ++i) {
    ip[i] = in + N * i;
    op[i] = out + N * i;
    sa[i] = scratch.p + 2 * q * (i % nsc);   // images of one launch use distinct scratch; launches are in order
    sb[i] = sa[i] + q;
  }
  if (inverse)
    wdb::dwt_inverse_many(n, levels, f, count, ip.data(), op.data(), sa.data(), sb.data(), s);
  else
    wdb::dwt_forward_many(n, levels, f, count, ip.data(), op.data(), sa.data(), sb.data(), s);
  WDB_HIP(hipStreamSynchronize(s));
  WDB_API_END
}

extern "C" wdb_status wdb_synthesize(const wdb_theta* th, const float* x, float* u_hat, void* stream) {
  WDB_API_BEGIN
  WDB_REQUIRE(th && x && u_hat, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(static_cast<const void*>(x) != static_cast<const void*>(u_hat), WDB_ERR_ARG,
              "x and u_hat must not alias");
  WDB_HIP(hipSetDevice(th->device));
  wdb_theta* t = const_cast<wdb_theta*>(th);
  wdb::ensure_workspace(t);
  wdb::Filter f = wdb::make_filter(th->wavelet);
  const size_t q = static_cast<size_t>(th->n / 2) * (th->n / 2);
  wdb::dwt_inverse(th->n, th->levels, f, x, u_hat, t->ws_img, t->ws_img + q,
                   static_cast<hipStream_t>(stream));
  WDB_API_END
}

// ---------------------------------------------------------------------------
// Transform without allocation.  The level-to-level intermediates live in a
// fixed device array instead of a per-call allocation: each GPU the library
// runs on holds its own copy (kNoAllocScratch floats, 8 MiB, enough for
// n <= 2048) until the process ends.  Host code never passes the array's name
// to a kernel: its device address is looked up once per device with
// hipGetSymbolAddress and only that address is used.  Every level writes the
// intermediate it later reads, so the array needs no clearing; calls that
// overlap on one GPU (different streams or threads) share it and race.
// ---------------------------------------------------------------------------
namespace {
constexpr int kNoAllocMaxN = 2048;
constexpr size_t kNoAllocScratch = 2 * static_cast<size_t>(kNoAllocMaxN / 2) * (kNoAllocMaxN / 2);
constexpr int kMaxDevices = 64;
static __device__ __align__(256) float scratch[kNoAllocScratch];

std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
float* scratch_address() {
  int dev = 0;
  WDB_HIP(hipGetDevice(&dev));
  WDB_REQUIRE(dev >= 0 && dev < kMaxDevices, WDB_ERR_ARG, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    WDB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    WDB_REQUIRE(ptr != nullptr, WDB_ERR_HIP, "no device address for the transform scratch array");
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" wdb_status wdb_dwt_noalloc(int32_t n, int32_t wavelet, int32_t levels, const float* in, float* out,
                                      int32_t inverse, void* stream) {
  WDB_API_BEGIN
  WDB_REQUIRE(in && out, WDB_ERR_ARG, "null buffer");
  WDB_REQUIRE(in != out, WDB_ERR_ARG, "in and out must not alias");
  wdb::Filter f = wdb::make_filter(wavelet);
  wdb::check_geometry(n, levels, static_cast<int>(f.h.size()));
  WDB_REQUIRE(n <= kNoAllocMaxN, WDB_ERR_SIZE,
              "wdb_dwt_noalloc: image side %d exceeds the fixed scratch limit of %d (use wdb_dwt)", n, kNoAllocMaxN);
  float* sc = scratch_address();
  const size_t q = static_cast<size_t>(n / 2) * (n / 2);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (inverse)
    wdb::dwt_inverse(n, levels, f, in, out, sc, sc + q, s);
  else
    wdb::dwt_forward(n, levels, f, in, out, sc, sc + q, s);
  WDB_API_END
}
