// Warm-start network on wavelet coefficients (not in the paper): one stack of
// three circular 3x3 convolutions per wavelet level (A_J with 1 channel, the
// detail levels with their 3 subbands as channels), ReLU after the first two,
// a residual connection, MSE loss and Adam with float32 master weights.
// Compute uses bfloat16 copies of the parameters and float32 accumulation.
//
//   h1 = relu(conv(z; W1, b1)), h2 = relu(conv(h1; W2, b2)), out = z + conv(h2; W3, b3),
//   conv(z; W, b)[o, i, j] = b[o] + sum_{c, di, dj} W[o, c, di, dj] z[c, (i+di-1) mod s, (j+dj-1) mod s].
//
// Activations are stored pre-ReLU (a1, a2); consumers apply the ReLU on load
// and the backward pass masks with a > 0.  Weight gradients are reduced in two
// deterministic stages (fixed per-block partial sums, then a fixed-order sum).
// Parameters are flattened stack by stack: W1, b1, W2, b2, W3, b3.
#include <cmath>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <map>
#include <type_traits>

#include "common.hpp"

namespace {
constexpr int kF = 32;       // hidden channels
constexpr int kBlk = 256;
constexpr int kP = 32;       // positions per weight-gradient chunk
constexpr int kWGridMax = 1024;   // partial rows of a weight gradient (blocks of its kernel)

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

uint16_t f2bf_host(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(b >> 16);
}

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(b >> 16);
}

// out[b, o] = bias[o] + conv(in[b]) (+ resid[b, o]); input ReLU applied on load if in_relu.
template <int CI, int CO>
__global__ __launch_bounds__(kBlk) void k_conv_fwd(const float* __restrict__ in, int64_t in_bs, int in_relu, int s,
                                                   int B, const uint16_t* __restrict__ w,
                                                   const uint16_t* __restrict__ bias, float* __restrict__ out,
                                                   int64_t out_bs, const float* __restrict__ resid, int64_t res_bs) {
  __shared__ float sw[CO * CI * 9];
  __shared__ float sb[CO];
  for (int t = threadIdx.x; t < CO * CI * 9; t += kBlk) sw[t] = bf2f(w[t]);
  for (int t = threadIdx.x; t < CO; t += kBlk) sb[t] = bf2f(bias[t]);
  __syncthreads();
  const int64_t per = static_cast<int64_t>(s) * s;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlk + threadIdx.x;
  if (p >= B * per) return;
  const int64_t b = p / per, ij = p % per;
  const int i = static_cast<int>(ij / s), j = static_cast<int>(ij % s);
  float acc[CO];
#pragma unroll
  for (int o = 0; o < CO; ++o) acc[o] = sb[o];
  const float* inb = in + b * in_bs;
  for (int c = 0; c < CI; ++c) {
    const float* ch = inb + c * per;
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      const float* row = ch + static_cast<int64_t>((i + di - 1) & (s - 1)) * s;
#pragma unroll
      for (int dj = 0; dj < 3; ++dj) {
        float v = row[(j + dj - 1) & (s - 1)];
        if (in_relu) v = fmaxf(v, 0.0f);
#pragma unroll
        for (int o = 0; o < CO; ++o) acc[o] = fmaf(sw[(o * CI + c) * 9 + di * 3 + dj], v, acc[o]);
      }
    }
  }
  float* ob = out + b * out_bs + ij;
  const float* rb = resid ? resid + b * res_bs + ij : nullptr;
#pragma unroll
  for (int o = 0; o < CO; ++o) ob[o * per] = acc[o] + (rb ? rb[o * per] : 0.0f);
}

// Convolutions into the 32 hidden channels on the matrix cores (f32 32x32x2
// MFMA: the float32 products and float32 sums of the vector kernels, in
// another order), for CI = 1, 3 or 32 input channels.  A block of 4
// wavefronts takes TR x TC positions of one image (TC = min(s, 32), TR = 128 /
// TC, s >= 16); the input tile with a one-pixel circular halo (ReLU applied on
// load if in_relu) and the weights as [k = d * CI + c][o] (tap d, channel c;
// K = 9 CI rows, padded to an even count with a zero row) are staged in LDS;
// a wavefront accumulates the 32 outputs of its 32 positions over k, two k a
// step: D[o][p] += W[o][k] X[k][p], lane l giving W[l mod 32][k] and
// X[k][p = l mod 32] for k = 2 step + l / 32, and holding
// D[8 (j / 4) + 4 (l / 32) + j mod 4][l mod 32] in its accumulator j.
// FLIP: the data gradient of a layer with 32 input channels and CI outputs,
// which is the convolution of g with W'[c][o][d] = W[c][o][8 - d] (W in the
// layer's own [out][in][tap] layout), masked by a > 0.  `w` holds the weights
// already in the kernel's [k][o] order (packed_weight), KP rows of 32.
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kMP = 33;                    // LDS floats per staged position (32 channels; odd stride)
constexpr int kMaxTilePos = 6 * 34;        // (TR + 2) (TC + 2) for TC = 32 (204 >= 10 * 18 for TC = 16)
constexpr int kTileMax = 128;              // positions per block tile

// Block tiles: TC x TR positions, TC = 16 for a side of 16 and 32 above (a
// compile-time width, so the staging loops divide by constants).
template <int TC>
struct TileG {
  static constexpr int TR = kTileMax / TC, W2 = TC + 2, P2 = (TC + 2) * (kTileMax / TC + 2);
};

// Image and origin of tile t of the batch (tiles of an image in row-major order).
template <int TC>
__device__ __forceinline__ void tile_origin(int t, int s, int& b, int& ty0, int& tx0) {
  const int tiles_x = s / TC, per_img = (s / TileG<TC>::TR) * tiles_x;
  b = t / per_img;
  const int ti = t - b * per_img;
  ty0 = (ti / tiles_x) * TileG<TC>::TR;
  tx0 = (ti % tiles_x) * TC;
}

// Staging of a tile in two halves, so that the loads of the next tile can be
// in flight while the matrix cores work on the current one: load_* fills a
// thread's registers, store_* writes them to LDS (ReLU applied there).
//
// Halo: channels [0, CH) of the tile at (ty0, tx0) with its circular halo as
// dst[q * stride + c], q = halo row * W2 + halo column; NT threads.
template <int CH, int TC, int NT = 256>
struct Halo {
  static constexpr int NE = CH * TileG<TC>::P2, NIT = (NE + NT - 1) / NT;
};

template <int CH, int TC, int NT = 256>
__device__ __forceinline__ void load_halo(const float* __restrict__ src, int64_t per, int s, int ty0, int tx0,
                                          float (&v)[Halo<CH, TC, NT>::NIT]) {
  using G = TileG<TC>;
  using H = Halo<CH, TC, NT>;
#pragma unroll
  for (int i = 0; i < H::NIT; ++i) {
    const int e = static_cast<int>(threadIdx.x) + i * NT;
    if (e < H::NE) {
      const int c = e / G::P2, q = e - c * G::P2;
      const int yy = q / G::W2, xx = q - yy * G::W2;
      const int gy = (ty0 + yy - 1) & (s - 1), gx = (tx0 + xx - 1) & (s - 1);
      v[i] = src[c * per + static_cast<int64_t>(gy) * s + gx];
    }
  }
}

template <int CH, int TC, int NT = 256>
__device__ __forceinline__ void store_halo(const float (&v)[Halo<CH, TC, NT>::NIT], int relu, float* __restrict__ dst,
                                           int stride) {
  using G = TileG<TC>;
  using H = Halo<CH, TC, NT>;
#pragma unroll
  for (int i = 0; i < H::NIT; ++i) {
    const int e = static_cast<int>(threadIdx.x) + i * NT;
    if (e < H::NE) {
      const int c = e / G::P2, q = e - c * G::P2;
      dst[q * stride + c] = relu ? fmaxf(v[i], 0.0f) : v[i];
    }
  }
}

// Tile32: the 32 channels of the tile's own 128 positions as dst[p * kMP + c].
template <int NT = 256>
struct Tile32 {
  static constexpr int NE = kF * kTileMax, NIT = (NE + NT - 1) / NT;
};

template <int TC, int NT = 256>
__device__ __forceinline__ void load_tile32(const float* __restrict__ src, int64_t per, int s, int ty0, int tx0,
                                            float (&v)[Tile32<NT>::NIT]) {
#pragma unroll
  for (int i = 0; i < Tile32<NT>::NIT; ++i) {
    const int e = static_cast<int>(threadIdx.x) + i * NT;
    if (e < Tile32<NT>::NE) {
      const int c = e / kTileMax, q = e % kTileMax;
      const int yy = q / TC, xx = q - yy * TC;
      v[i] = src[c * per + static_cast<int64_t>(ty0 + yy) * s + tx0 + xx];
    }
  }
}

template <int NT = 256>
__device__ __forceinline__ void store_tile32(const float (&v)[Tile32<NT>::NIT], int relu, float* __restrict__ dst) {
#pragma unroll
  for (int i = 0; i < Tile32<NT>::NIT; ++i) {
    const int e = static_cast<int>(threadIdx.x) + i * NT;
    if (e < Tile32<NT>::NE) dst[(e % kTileMax) * kMP + e / kTileMax] = relu ? fmaxf(v[i], 0.0f) : v[i];
  }
}

// Blocks of the convolution kernels: each takes tiles t = blockIdx.x,
// + gridDim.x, ... of the batch, its weights staged once.  The grid is as
// many blocks as the device holds at once (so every compute unit gets the
// same number of tiles, within one), at most kWGridMax.

template <int CI, bool FLIP, int TC>
__global__ __launch_bounds__(256) void k_conv_mfma_in(const float* __restrict__ in, int64_t in_bs, int in_relu, int s,
                                                      int ntiles, const uint16_t* __restrict__ w,
                                                      const uint16_t* __restrict__ bias, float* __restrict__ out,
                                                      int64_t out_bs, const float* __restrict__ resid,
                                                      int64_t res_bs, const float* __restrict__ mask, int64_t m_bs) {
  using G = TileG<TC>;
  constexpr int K = 9 * CI, KP = K + (K & 1);
  constexpr int XS = CI == kF ? kMP : CI;   // LDS floats per staged position
  __shared__ float sx[G::P2 * XS];
  __shared__ __align__(16) uint16_t swt[KP * kF];   // bfloat16 weights, [k][o]
  const int64_t per = static_cast<int64_t>(s) * s;
  static_assert((KP * kF) % 8 == 0, "the packed weights copy in 16-byte pieces");
  for (int e = threadIdx.x; e < KP * kF / 8; e += 256)
    reinterpret_cast<uint4*>(swt)[e] = reinterpret_cast<const uint4*>(w)[e];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int pl = wv * 32 + (lane & 31);
  const int ty = pl / TC, tx = pl - ty * TC;
  const int kh = lane >> 5;
  float v[Halo<CI, TC>::NIT];
  int b, ty0, tx0;
  if (static_cast<int>(blockIdx.x) < ntiles) {
    tile_origin<TC>(blockIdx.x, s, b, ty0, tx0);
    load_halo<CI, TC>(in + b * in_bs, per, s, ty0, tx0, v);
  }
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    tile_origin<TC>(t, s, b, ty0, tx0);
    store_halo<CI, TC>(v, in_relu, sx, XS);
    __syncthreads();
    if (t + static_cast<int>(gridDim.x) < ntiles) {   // the next tile's loads overlap this tile's products
      int bn, yn, xn;
      tile_origin<TC>(t + gridDim.x, s, bn, yn, xn);
      load_halo<CI, TC>(in + bn * in_bs, per, s, yn, xn, v);
    }
    f32x16 acc = {};
    if constexpr (CI == kF) {
#pragma unroll
      for (int d = 0; d < 9; ++d) {
        const float* xr = sx + ((ty + d / 3) * G::W2 + tx + d % 3) * XS + kh;
        const uint16_t* wr = swt + (d * kF + kh) * kF + (lane & 31);
#pragma unroll
        for (int cb = 0; cb < kF / 2; ++cb)
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(bf2f(wr[2 * cb * kF]), xr[2 * cb], acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int st = 0; st < KP / 2; ++st) {
        const int k = 2 * st + kh;
        const int dk = k / CI, c = k - dk * CI;   // k = K (the zero row) reads tap 8, channel 0
        const int d = min(dk, 8);
        const float xv = sx[((ty + d / 3) * G::W2 + tx + d % 3) * XS + c];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(bf2f(swt[k * kF + (lane & 31)]), xv, acc, 0, 0, 0);
      }
    }
    __syncthreads();   // every wavefront is done with sx before the next tile is staged
    const int64_t gpos = static_cast<int64_t>(ty0 + ty) * s + tx0 + tx;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int o = 8 * (j >> 2) + 4 * kh + (j & 3);
      float v = acc[j];
      if (FLIP) {
        if (mask && !(mask[b * m_bs + o * per + gpos] > 0.0f)) v = 0.0f;
      } else {
        v += bf2f(bias[o]);
        if (resid) v += resid[b * res_bs + o * per + gpos];
      }
      out[b * out_bs + o * per + gpos] = v;
    }
  }
}

// Weight (k, o) of the matrix-core kernel for CI input channels, k = d CI + c
// (zero for the padding row k >= 9 CI), from a layer's [out][in][tap] weights;
// flip: the data-gradient form W'[c][o][d] = W[c][o][8 - d] of a layer with
// 32 inputs.
__device__ __forceinline__ uint16_t packed_weight(const uint16_t* __restrict__ w, int CI, bool flip, int k, int o) {
  if (k >= 9 * CI) return 0;
  const int d = k / CI, c = k - d * CI;
  return flip ? w[(c * kF + o) * 9 + (8 - d)] : w[(o * CI + c) * 9 + d];
}

// The four packed matrices of one stack (blockIdx.y): W1 (CI = C), W2, W2
// flipped (CI = 32), W3 flipped (CI = C).
__global__ void k_pack_stack(const uint16_t* __restrict__ w1, const uint16_t* __restrict__ w2,
                             const uint16_t* __restrict__ w3, int C, uint16_t* __restrict__ o1,
                             uint16_t* __restrict__ o2, uint16_t* __restrict__ o2f, uint16_t* __restrict__ o3f) {
  const int seg = blockIdx.y;
  const int CI = (seg == 1 || seg == 2) ? kF : C;
  const int KP = 9 * CI + ((9 * CI) & 1);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= KP * kF) return;
  const int k = e >> 5, o = e & 31;
  const uint16_t* w = seg == 0 ? w1 : (seg == 3 ? w3 : w2);
  uint16_t* out = seg == 0 ? o1 : (seg == 1 ? o2 : (seg == 2 ? o2f : o3f));
  out[e] = packed_weight(w, CI, seg >= 2, k, o);
}

// The last convolution of a stack (32 -> CO channels, CO = 1 or 3) on the
// matrix cores: first the per-tap products T[m = 9 o + d][q] = sum_c W[o][c][d]
// x[q][c] at every position q of the tile and its halo (an MFMA over the 32
// channels, rows m >= 9 CO zero), then out[o][p] = b[o] + resid[o][p] +
// sum_d T[9 o + d][p + off(d)] on the vector units.
template <int CO, int TC>
__global__ __launch_bounds__(256) void k_conv_mfma_out(const float* __restrict__ in, int64_t in_bs, int in_relu,
                                                       int s, int ntiles, const uint16_t* __restrict__ w,
                                                       const uint16_t* __restrict__ bias, float* __restrict__ out,
                                                       int64_t out_bs, const float* __restrict__ resid,
                                                       int64_t res_bs) {
  using G = TileG<TC>;
  constexpr int M = 9 * CO;   // rows used of the 32 (and the LDS stride of T: odd)
  constexpr int NG = (G::P2 + 31) / 32;   // groups of 32 halo positions
  __shared__ float sx[G::P2 * kMP];
  __shared__ float sT[NG * 32 * M];
  __shared__ float swt[kF * kF];
  const int64_t per = static_cast<int64_t>(s) * s;
  for (int e = threadIdx.x; e < kF * kF; e += 256) {
    const int c = e >> 5, m = e & 31;
    swt[e] = m < M ? bf2f(w[((m / 9) * kF + c) * 9 + m % 9]) : 0.0f;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, kh = lane >> 5, l32 = lane & 31;
  float v[Halo<kF, TC>::NIT];
  int b, ty0, tx0;
  if (static_cast<int>(blockIdx.x) < ntiles) {
    tile_origin<TC>(blockIdx.x, s, b, ty0, tx0);
    load_halo<kF, TC>(in + b * in_bs, per, s, ty0, tx0, v);
  }
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    tile_origin<TC>(t, s, b, ty0, tx0);
    store_halo<kF, TC>(v, in_relu, sx, kMP);
    __syncthreads();
    if (t + static_cast<int>(gridDim.x) < ntiles) {   // the next tile's loads overlap this tile's products
      int bn, yn, xn;
      tile_origin<TC>(t + gridDim.x, s, bn, yn, xn);
      load_halo<kF, TC>(in + bn * in_bs, per, s, yn, xn, v);
    }
    for (int gq = wv; gq < NG; gq += 4) {   // wave-uniform
      const int q = gq * 32 + l32;
      const int qr = min(q, G::P2 - 1);
      f32x16 acc = {};
#pragma unroll
      for (int cb = 0; cb < kF / 2; ++cb)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(swt[(2 * cb + kh) * kF + l32], sx[qr * kMP + 2 * cb + kh], acc,
                                                   0, 0, 0);
      if (q < G::P2) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int m = 8 * (j >> 2) + 4 * kh + (j & 3);
          if (m < M) sT[q * M + m] = acc[j];
        }
      }
    }
    __syncthreads();   // T complete; sx is free for the next tile (the sums below read only T)
    for (int e = threadIdx.x; e < kTileMax * CO; e += 256) {
      const int p = e & (kTileMax - 1), o = e / kTileMax;
      const int ty = p / TC, tx = p - ty * TC;
      float v = 0.0f;
#pragma unroll
      for (int d = 0; d < 9; ++d) v += sT[((ty + d / 3) * G::W2 + tx + d % 3) * M + o * 9 + d];
      v += bf2f(bias[o]);
      const int64_t gpos = static_cast<int64_t>(ty0 + ty) * s + tx0 + tx;
      if (resid) v += resid[b * res_bs + o * per + gpos];
      out[b * out_bs + o * per + gpos] = v;
    }
  }
}

// gin[b, c] = sum_{o, d} W[o, c, d] g[b, o, shifted]  (times [a_in > 0] if mask given).
template <int CO, int CI>
__global__ __launch_bounds__(kBlk) void k_conv_bwd_data(const float* __restrict__ g, int64_t g_bs, int s, int B,
                                                        const uint16_t* __restrict__ w, const float* __restrict__ mask,
                                                        int64_t m_bs, float* __restrict__ gin, int64_t gin_bs) {
  __shared__ float sw[CO * CI * 9];
  for (int t = threadIdx.x; t < CO * CI * 9; t += kBlk) sw[t] = bf2f(w[t]);
  __syncthreads();
  const int64_t per = static_cast<int64_t>(s) * s;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlk + threadIdx.x;
  if (p >= B * per) return;
  const int64_t b = p / per, ij = p % per;
  const int i = static_cast<int>(ij / s), j = static_cast<int>(ij % s);
  float acc[CI];
#pragma unroll
  for (int c = 0; c < CI; ++c) acc[c] = 0.0f;
  const float* gb = g + b * g_bs;
  for (int o = 0; o < CO; ++o) {
    const float* ch = gb + o * per;
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      const float* row = ch + static_cast<int64_t>((i - di + 1) & (s - 1)) * s;
#pragma unroll
      for (int dj = 0; dj < 3; ++dj) {
        const float v = row[(j - dj + 1) & (s - 1)];
#pragma unroll
        for (int c = 0; c < CI; ++c) acc[c] = fmaf(sw[(o * CI + c) * 9 + di * 3 + dj], v, acc[c]);
      }
    }
  }
  float* ob = gin + b * gin_bs + ij;
  const float* mb = mask ? mask + b * m_bs + ij : nullptr;
#pragma unroll
  for (int c = 0; c < CI; ++c) ob[c * per] = (mb && !(mb[c * per] > 0.0f)) ? 0.0f : acc[c];
}

// Per-block partial sums of dW[o, c, d] = sum_p g[p, o] act[p, c, d] and db[o] = sum_p g[p, o].
template <int CI, int CO>
__global__ __launch_bounds__(kBlk) void k_conv_bwd_w(const float* __restrict__ act, int64_t a_bs, int act_relu,
                                                     const float* __restrict__ g, int64_t g_bs, int s, int B,
                                                     float* __restrict__ partial) {
  constexpr int NW = CO * CI * 9;
  constexpr int NT = NW + CO;
  constexpr int NPT = (NT + kBlk - 1) / kBlk;
  __shared__ float sg[CO][kP];
  __shared__ float sa[CI * 9][kP];
  float acc[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) acc[k] = 0.0f;
  const int64_t per = static_cast<int64_t>(s) * s;
  const int64_t T = B * per;
  const int64_t nchunks = (T + kP - 1) / kP;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const int64_t p0 = ch * kP;
    for (int t = threadIdx.x; t < CO * kP; t += kBlk) {
      const int o = t / kP, q = t % kP;
      const int64_t p = p0 + q;
      float v = 0.0f;
      if (p < T) v = g[(p / per) * g_bs + o * per + (p % per)];
      sg[o][q] = v;
    }
    for (int t = threadIdx.x; t < CI * 9 * kP; t += kBlk) {
      const int cd = t / kP, q = t % kP;
      const int c = cd / 9, d = cd % 9;
      const int64_t p = p0 + q;
      float v = 0.0f;
      if (p < T) {
        const int64_t b = p / per, ij = p % per;
        const int i = static_cast<int>(ij / s), j = static_cast<int>(ij % s);
        const int ii = (i + d / 3 - 1) & (s - 1), jj = (j + d % 3 - 1) & (s - 1);
        v = act[b * a_bs + c * per + static_cast<int64_t>(ii) * s + jj];
        if (act_relu) v = fmaxf(v, 0.0f);
      }
      sa[cd][q] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int idx = threadIdx.x + k * kBlk;
      if (idx < NW) {
        const int o = idx / (CI * 9), cd = idx % (CI * 9);
        float a = acc[k];
#pragma unroll 8
        for (int q = 0; q < kP; ++q) a = fmaf(sg[o][q], sa[cd][q], a);
        acc[k] = a;
      } else if (idx < NT) {
        const int o = idx - NW;
        float a = acc[k];
        for (int q = 0; q < kP; ++q) a += sg[o][q];
        acc[k] = a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int idx = threadIdx.x + k * kBlk;
    if (idx < NT) partial[static_cast<int64_t>(blockIdx.x) * NT + idx] = acc[k];
  }
}

// Weight gradient of the hidden 32 -> 32 layer on the matrix cores: per block
// the partial sums over the 128-position tiles it takes (tile t = blockIdx.x,
// + gridDim.x, ...), in the partial layout of k_conv_bwd_w.  A block has one
// wavefront per tap d (9 wavefronts); wavefront d contracts the tile's 128
// positions two at a time, D_d[o][c] += G[o][p] A_d[p][c], lane l giving
// G[l mod 32][p] = g[p][o] and A_d[p][l mod 32] = act[p + off(d)][c] for
// p = 2 step + l / 32.  Each wavefront owns its tap's outputs (wavefront 0
// also the bias sums), so no sum crosses wavefronts and the result does not
// depend on scheduling.
constexpr int kRedFloats = 9 * kF * kF + kF;
constexpr int kBwdWaves = 9;
constexpr int kBwdThreads = 64 * kBwdWaves;

template <int TC>
__global__ __launch_bounds__(kBwdThreads) void k_conv32_bwd_w_mfma(const float* __restrict__ act, int64_t a_bs,
                                                                   int act_relu, const float* __restrict__ g,
                                                                   int64_t g_bs, int s, int ntiles,
                                                                   float* __restrict__ partial) {
  constexpr int W2 = TileG<TC>::W2, P2 = TileG<TC>::P2;
  __shared__ float sx[P2 * kMP];            // act tile with halo, [pos][c]
  __shared__ float sg[kTileMax * kMP];      // g tile, [pos][o]
  const int64_t per = static_cast<int64_t>(s) * s;
  const int lane = threadIdx.x & 63, d = threadIdx.x >> 6, kh = lane >> 5, l32 = lane & 31;
  f32x16 acc = {};
  float bsum = 0.0f;
  float va[Halo<kF, TC, kBwdThreads>::NIT], vg[Tile32<kBwdThreads>::NIT];
  if (static_cast<int>(blockIdx.x) < ntiles) {
    int b, ty0, tx0;
    tile_origin<TC>(blockIdx.x, s, b, ty0, tx0);
    load_halo<kF, TC, kBwdThreads>(act + b * a_bs, per, s, ty0, tx0, va);
    load_tile32<TC, kBwdThreads>(g + b * g_bs, per, s, ty0, tx0, vg);
  }
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    store_halo<kF, TC, kBwdThreads>(va, act_relu, sx, kMP);
    store_tile32<kBwdThreads>(vg, 0, sg);
    __syncthreads();
    if (t + static_cast<int>(gridDim.x) < ntiles) {   // the next tile's loads overlap this tile's products
      int bn, yn, xn;
      tile_origin<TC>(t + gridDim.x, s, bn, yn, xn);
      load_halo<kF, TC, kBwdThreads>(act + bn * a_bs, per, s, yn, xn, va);
      load_tile32<TC, kBwdThreads>(g + bn * g_bs, per, s, yn, xn, vg);
    }
    const int dy = d / 3, dx = d % 3;
#pragma unroll 8
    for (int st = 0; st < kTileMax / 2; ++st) {
      const int q = 2 * st + kh;
      const int ty = q / TC, tx = q - ty * TC;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(sg[q * kMP + l32], sx[((ty + dy) * W2 + tx + dx) * kMP + l32], acc,
                                                 0, 0, 0);
    }
    if (d == 0 && kh == 0)
      for (int p = 0; p < kTileMax; ++p) bsum += sg[p * kMP + l32];
    __syncthreads();
  }
  float* pr = partial + static_cast<int64_t>(blockIdx.x) * kRedFloats;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int o = 8 * (j >> 2) + 4 * kh + (j & 3);
    pr[o * (kF * 9) + l32 * 9 + d] = acc[j];
  }
  if (d == 0 && kh == 0) pr[9 * kF * kF + l32] = bsum;
}

// Weight gradients of a stack's thin convolutions (C = 1 or 3 channels on one
// side, 32 on the other) on the matrix cores, per block the partial sums over
// its tiles in the partial layout of k_conv_bwd_w.  A wavefront contracts its
// 32 positions p two at a time, D[m][n] += A[m][p] B[p][n], with A the
// 32-channel operand at p and B the C-channel operand at p shifted by tap d:
//   first convolution (C -> 32): m = o, n = 9 c + d,
//     D = sum_p g[p][o] z[p + off(d)][c], bias sum_p g[p][o];
//   last convolution (32 -> C, L3): m = c, n = 9 o + d,
//     D = sum_p relu(a)[p][c] g[p - off(d)][o] (the same sum over p + off(d)), bias sum_p g[p][o].
// Columns n >= 9 C are zero.  The four wavefronts' sums are added in a fixed order.
template <int C, bool L3, int TC>
__global__ __launch_bounds__(256) void k_bwd_w_thin(const float* __restrict__ act, int64_t a_bs, int act_relu,
                                                    const float* __restrict__ g, int64_t g_bs, int s, int ntiles,
                                                    float* __restrict__ partial) {
  constexpr int NN = 9 * C;
  constexpr int NT = NN * kF + (L3 ? C : kF);
  __shared__ float sw[kTileMax * kMP];     // the 32-channel operand, [p][ch]
  __shared__ float sn[kMaxTilePos * C];    // the C-channel operand with halo, [q][ch]
  __shared__ float red[NT];
  const float* __restrict__ wide = L3 ? act : g;
  const float* __restrict__ thin = L3 ? g : act;
  const int64_t wide_bs = L3 ? a_bs : g_bs, thin_bs = L3 ? g_bs : a_bs;
  const int wide_relu = L3 ? act_relu : 0, thin_relu = L3 ? 0 : act_relu;
  using G = TileG<TC>;
  const int64_t per = static_cast<int64_t>(s) * s;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, kh = lane >> 5, l32 = lane & 31;
  const bool nv = l32 < NN;
  const int nc = nv ? l32 / 9 : 0;                               // c (first) or o (last)
  const int nd = nv ? (L3 ? 8 - l32 % 9 : l32 % 9) : 4;          // tap of the shift
  f32x16 acc = {};
  float bsum = 0.0f;
  float vw[Tile32<>::NIT], vn[Halo<C, TC>::NIT];
  if (static_cast<int>(blockIdx.x) < ntiles) {
    int b, ty0, tx0;
    tile_origin<TC>(blockIdx.x, s, b, ty0, tx0);
    load_tile32<TC>(wide + b * wide_bs, per, s, ty0, tx0, vw);
    load_halo<C, TC>(thin + b * thin_bs, per, s, ty0, tx0, vn);
  }
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    store_tile32(vw, wide_relu, sw);
    store_halo<C, TC>(vn, thin_relu, sn, C);
    __syncthreads();
    if (t + static_cast<int>(gridDim.x) < ntiles) {   // the next tile's loads overlap this tile's products
      int bn, yn, xn;
      tile_origin<TC>(t + gridDim.x, s, bn, yn, xn);
      load_tile32<TC>(wide + bn * wide_bs, per, s, yn, xn, vw);
      load_halo<C, TC>(thin + bn * thin_bs, per, s, yn, xn, vn);
    }
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int p = wv * 32 + 2 * st + kh;
      const int ty = p / TC, tx = p - ty * TC;
      const float bv = nv ? sn[((ty + nd / 3) * G::W2 + tx + nd % 3) * C + nc] : 0.0f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(sw[p * kMP + l32], bv, acc, 0, 0, 0);
    }
    if (kh == 0) {
      if (!L3) {
        for (int p = 0; p < 32; ++p) bsum += sw[(wv * 32 + p) * kMP + l32];
      } else if (l32 < C) {
        for (int p = 0; p < 32; ++p) {
          const int q = wv * 32 + p, ty = q / TC, tx = q - ty * TC;
          bsum += sn[((ty + 1) * G::W2 + tx + 1) * C + l32];
        }
      }
    }
    __syncthreads();
  }
  for (int w = 0; w < 4; ++w) {
    if (wv == w) {
      if (nv) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int m = 8 * (j >> 2) + 4 * kh + (j & 3);
          const int idx = L3 ? (l32 / 9) * (kF * 9) + m * 9 + l32 % 9 : m * NN + l32;
          red[idx] = (w == 0 ? 0.0f : red[idx]) + acc[j];
        }
      }
      if (kh == 0 && l32 < (L3 ? C : kF)) red[NN * kF + l32] = (w == 0 ? 0.0f : red[NN * kF + l32]) + bsum;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < NT; e += 256) partial[static_cast<int64_t>(blockIdx.x) * NT + e] = red[e];
}

// out[i] = sum over the partial rows b of partial[b][i]: a block of 16
// wavefronts takes 64 consecutive i, wavefront w the rows b = w, w + 16, ...
// (eight loads in flight per step), and the 16 sums are added in a fixed order.
constexpr int kSumWaves = 16;
__global__ __launch_bounds__(64 * kSumWaves) void k_sum_partials(const float* __restrict__ partial, int nblocks,
                                                                 int NT, float* __restrict__ out) {
  __shared__ float red[kSumWaves][64];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + l;
  float a = 0.0f;
  if (i < NT) {
    int b = w;
    for (; b + 7 * kSumWaves < nblocks; b += 8 * kSumWaves) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partial[static_cast<int64_t>(b + u * kSumWaves) * NT + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) a += v[u];
    }
    for (; b < nblocks; b += kSumWaves) a += partial[static_cast<int64_t>(b) * NT + i];
  }
  red[w][l] = a;
  __syncthreads();
  if (w == 0 && i < NT) {
    float t = 0.0f;
    for (int k = 0; k < kSumWaves; ++k) t += red[k][l];
    out[i] = t;
  }
}

// g = 2 (pred - target) / (B N); per-block partial sums of (pred - target)^2 in float64.
__global__ __launch_bounds__(kBlk) void k_mse(const float* __restrict__ pred, const float* __restrict__ tgt, int64_t n,
                                              float scale, float* __restrict__ g, double* __restrict__ part) {
  __shared__ double sh[kBlk];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlk + threadIdx.x;
  double d2 = 0.0;
  if (i < n) {
    const float d = pred[i] - tgt[i];
    g[i] = scale * d;
    d2 = static_cast<double>(d) * d;
  }
  sh[threadIdx.x] = d2;
  __syncthreads();
  for (int w = kBlk / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_adam(float* __restrict__ master, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float c1, float c2,
                       float eps, uint16_t* __restrict__ wbf) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = master[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  master[i] = w;
  wbf[i] = f2bf(w);
}

__global__ void k_round_bf16(const float* __restrict__ master, uint16_t* __restrict__ wbf, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) wbf[i] = f2bf(master[i]);
}

inline dim3 grid_for(int64_t n) { return dim3(static_cast<unsigned>((n + kBlk - 1) / kBlk)); }

}  // namespace

struct wdb_cnn {
  int device = 0;
  int n = 0, levels = 0, F = kF;
  int64_t N = 0;
  struct Stack {
    int64_t off;
    int C, s;
    int64_t p[6];  // offsets of W1, b1, W2, b2, W3, b3
    int64_t pk[4]; // offsets in wpk of the [k][o] weights: W1, W2, W2 flipped, W3 flipped
  };
  std::vector<Stack> stacks;
  int64_t nparam = 0;
  float* master = nullptr;
  uint16_t* wbf = nullptr;
  uint16_t* wpk = nullptr;   // the matrix-core kernels' weights, [k][o] per stack (see pack_weights)
  int64_t npk = 0;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  int64_t t = 0;
  int bcap = 0;
  float* a1 = nullptr;   // per batch capacity: largest stack's B*F*s*s
  float* a2 = nullptr;
  float* ga = nullptr;
  float* gb = nullptr;
  float* pred = nullptr; // B*N
  float* gout = nullptr; // B*N
  float* partial = nullptr;
  double* dpart = nullptr;
  double* hpart = nullptr;
};

namespace {

void cnn_free_ws(wdb_cnn* c) {
  float* fs[] = {c->a1, c->a2, c->ga, c->gb, c->pred, c->gout, c->partial};
  for (float* p : fs)
    if (p) (void)hipFree(p);
  if (c->dpart) (void)hipFree(c->dpart);
  if (c->hpart) (void)hipHostFree(c->hpart);
  c->a1 = c->a2 = c->ga = c->gb = c->pred = c->gout = c->partial = nullptr;
  c->dpart = nullptr;
  c->hpart = nullptr;
  c->bcap = 0;
}

void cnn_ensure(wdb_cnn* c, int B) {
  if (B <= c->bcap) return;
  cnn_free_ws(c);
  int64_t big = 0;
  for (auto& st : c->stacks) big = std::max<int64_t>(big, static_cast<int64_t>(st.s) * st.s);
  const int64_t act = static_cast<int64_t>(B) * c->F * big;
  const int64_t vec = static_cast<int64_t>(B) * c->N;
  WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->a1), act * sizeof(float)));
  WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->a2), act * sizeof(float)));
  WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->ga), act * sizeof(float)));
  WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->gb), act * sizeof(float)));
  WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->pred), vec * sizeof(float)));
  WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->gout), vec * sizeof(float)));
  WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->partial),
                    static_cast<size_t>(kWGridMax) * (kF * kF * 9 + kF) * sizeof(float)));
  const int64_t nb = (vec + kBlk - 1) / kBlk;
  WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->dpart), nb * sizeof(double)));
  WDB_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->hpart), nb * sizeof(double), hipHostMallocDefault));
  c->bcap = B;
}

// Blocks of `kernel` (threads per block) resident on the current device at
// once, looked up once per kernel.
int resident_blocks(const void* kernel, int threads) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
  int dev = 0;
  WDB_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find({kernel, dev});
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  WDB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
  WDB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int n = std::max(1, std::min(kWGridMax, std::max(per_cu, 1) * std::max(cus, 1)));
  cache[{kernel, dev}] = n;
  return n;
}

template <class K>
dim3 conv_grid(K kernel, int threads, int ntiles) {
  return dim3(static_cast<unsigned>(std::min(ntiles, resident_blocks(reinterpret_cast<const void*>(kernel), threads))));
}

// The matrix-core kernels take 128-position tiles of 16 x 8 (side 16) or
// 32 x 4 (larger sides) positions; with_tc calls f with that width.
template <class F>
void with_tc(int s, F&& f) {
  if (s == 16)
    f(std::integral_constant<int, 16>{});
  else
    f(std::integral_constant<int, 32>{});
}

// w: the layer's [out][in][tap] weights; wpk: the same packed for the
// matrix-core kernel (layers with 32 outputs; unused otherwise).
template <int CI, int CO>
void conv_fwd(const float* in, int64_t in_bs, int in_relu, int s, int B, const uint16_t* w, const uint16_t* b,
              const uint16_t* wpk, float* out, int64_t out_bs, const float* resid, int64_t res_bs, hipStream_t st) {
  if (s >= 16) {   // on the matrix cores
    const int ntiles = static_cast<int>(static_cast<int64_t>(B) * s * s / kTileMax);
    if constexpr (CO == kF) {
      with_tc(s, [&](auto tc) {
        auto* k = k_conv_mfma_in<CI, false, decltype(tc)::value>;
        hipLaunchKernelGGL(k, conv_grid(k, 256, ntiles), dim3(256), 0, st, in, in_bs, in_relu, s, ntiles, wpk, b, out,
                           out_bs, resid, res_bs, static_cast<const float*>(nullptr), int64_t{0});
      });
      return;
    } else if constexpr (CI == kF) {
      with_tc(s, [&](auto tc) {
        auto* k = k_conv_mfma_out<CO, decltype(tc)::value>;
        hipLaunchKernelGGL(k, conv_grid(k, 256, ntiles), dim3(256), 0, st, in, in_bs, in_relu, s, ntiles, w, b, out,
                           out_bs, resid, res_bs);
      });
      return;
    }
  }
  hipLaunchKernelGGL((k_conv_fwd<CI, CO>), grid_for(static_cast<int64_t>(B) * s * s), dim3(kBlk), 0, st, in, in_bs,
                     in_relu, s, B, w, b, out, out_bs, resid, res_bs);
}

// Data gradient of a layer with CI inputs and CO outputs: a convolution of the
// CO-channel gradient into CI channels.
template <int CO, int CI>
void conv_bwd_data(const float* g, int64_t g_bs, int s, int B, const uint16_t* w, const uint16_t* wpk,
                   const float* mask, int64_t m_bs, float* gin, int64_t gin_bs, hipStream_t st) {
  if constexpr (CI == kF) {
    if (s >= 16) {
      const int ntiles = static_cast<int>(static_cast<int64_t>(B) * s * s / kTileMax);
      with_tc(s, [&](auto tc) {
        auto* k = k_conv_mfma_in<CO, true, decltype(tc)::value>;
        hipLaunchKernelGGL(k, conv_grid(k, 256, ntiles), dim3(256), 0, st, g, g_bs, 0, s, ntiles, wpk,
                           static_cast<const uint16_t*>(nullptr), gin, gin_bs, static_cast<const float*>(nullptr),
                           int64_t{0}, mask, m_bs);
      });
      return;
    }
  }
  hipLaunchKernelGGL((k_conv_bwd_data<CO, CI>), grid_for(static_cast<int64_t>(B) * s * s), dim3(kBlk), 0, st, g,
                     g_bs, s, B, w, mask, m_bs, gin, gin_bs);
}

template <int CI, int CO>
void conv_bwd_w(const float* act, int64_t a_bs, int act_relu, const float* g, int64_t g_bs, int s, int B,
                float* partial, float* out, hipStream_t st) {
  const int64_t T = static_cast<int64_t>(B) * s * s;
  const int NT = CO * CI * 9 + CO;
  if (s >= 16) {   // on the matrix cores
    const int ntiles = static_cast<int>(T / kTileMax);
    int nb = 0;
    with_tc(s, [&](auto tc) {
      constexpr int TC = decltype(tc)::value;
      if constexpr (CI == kF && CO == kF) {
        auto* k = k_conv32_bwd_w_mfma<TC>;
        const dim3 grid = conv_grid(k, kBwdThreads, ntiles);
        nb = static_cast<int>(grid.x);
        hipLaunchKernelGGL(k, grid, dim3(kBwdThreads), 0, st, act, a_bs, act_relu, g, g_bs, s, ntiles, partial);
      } else {
        auto* k = k_bwd_w_thin<CI == kF ? CO : CI, CI == kF, TC>;
        const dim3 grid = conv_grid(k, 256, ntiles);
        nb = static_cast<int>(grid.x);
        hipLaunchKernelGGL(k, grid, dim3(256), 0, st, act, a_bs, act_relu, g, g_bs, s, ntiles, partial);
      }
    });
    hipLaunchKernelGGL(k_sum_partials, dim3((NT + 63) / 64), dim3(64 * kSumWaves), 0, st, partial, nb, NT, out);
    return;
  }
  const int nb = static_cast<int>(std::min<int64_t>(kWGridMax, (T + kP - 1) / kP));
  hipLaunchKernelGGL((k_conv_bwd_w<CI, CO>), dim3(nb), dim3(kBlk), 0, st, act, a_bs, act_relu, g, g_bs, s, B,
                     partial);
  hipLaunchKernelGGL(k_sum_partials, dim3((NT + 63) / 64), dim3(64 * kSumWaves), 0, st, partial, nb, NT, out);
}

// Refresh the packed [k][o] weights of the matrix-core kernels from the
// bfloat16 parameters (after every change of wbf).
void pack_weights(wdb_cnn* c, hipStream_t st) {
  for (auto& S : c->stacks) {
    uint16_t* pk = c->wpk;
    const dim3 grid((9 * kF * kF + 255) / 256, 4);
    hipLaunchKernelGGL(k_pack_stack, grid, dim3(256), 0, st, c->wbf + S.p[0], c->wbf + S.p[2], c->wbf + S.p[4], S.C,
                       pk + S.pk[0], pk + S.pk[1], pk + S.pk[2], pk + S.pk[3]);
  }
  WDB_HIP(hipGetLastError());
}

void forward(wdb_cnn* c, const float* x0, int B, float* pred, hipStream_t st) {
  const int64_t N = c->N;
  for (auto& S : c->stacks) {
    const int64_t per = static_cast<int64_t>(S.s) * S.s;
    const float* z = x0 + S.off;
    const uint16_t* w = c->wbf;
    const uint16_t* pk = c->wpk;
    const int64_t hb = static_cast<int64_t>(kF) * per;
    if (S.C == 1) conv_fwd<1, kF>(z, N, 0, S.s, B, w + S.p[0], w + S.p[1], pk + S.pk[0], c->a1, hb, nullptr, 0, st);
    else conv_fwd<3, kF>(z, N, 0, S.s, B, w + S.p[0], w + S.p[1], pk + S.pk[0], c->a1, hb, nullptr, 0, st);
    conv_fwd<kF, kF>(c->a1, hb, 1, S.s, B, w + S.p[2], w + S.p[3], pk + S.pk[1], c->a2, hb, nullptr, 0, st);
    if (S.C == 1) conv_fwd<kF, 1>(c->a2, hb, 1, S.s, B, w + S.p[4], w + S.p[5], nullptr, pred + S.off, N, z, N, st);
    else conv_fwd<kF, 3>(c->a2, hb, 1, S.s, B, w + S.p[4], w + S.p[5], nullptr, pred + S.off, N, z, N, st);
  }
  WDB_HIP(hipGetLastError());
}

// Loss and gradient into c->grad (float32).  Recomputes the forward pass per
// stack so only one stack's activations are held at a time.
double loss_grad(wdb_cnn* c, const float* x0, const float* tgt, int B, hipStream_t st) {
  const int64_t N = c->N;
  const int64_t tot = static_cast<int64_t>(B) * N;
  forward(c, x0, B, c->pred, st);
  const int64_t nb = (tot + kBlk - 1) / kBlk;
  hipLaunchKernelGGL(k_mse, dim3(static_cast<unsigned>(nb)), dim3(kBlk), 0, st, c->pred, tgt, tot,
                     static_cast<float>(2.0 / static_cast<double>(tot)), c->gout, c->dpart);
  WDB_HIP(hipMemcpyAsync(c->hpart, c->dpart, nb * sizeof(double), hipMemcpyDeviceToHost, st));
  for (auto& S : c->stacks) {
    const int64_t per = static_cast<int64_t>(S.s) * S.s;
    const int64_t hb = static_cast<int64_t>(kF) * per;
    const float* z = x0 + S.off;
    const uint16_t* w = c->wbf;
    const uint16_t* pk = c->wpk;
    // recompute this stack's activations
    if (S.C == 1) conv_fwd<1, kF>(z, N, 0, S.s, B, w + S.p[0], w + S.p[1], pk + S.pk[0], c->a1, hb, nullptr, 0, st);
    else conv_fwd<3, kF>(z, N, 0, S.s, B, w + S.p[0], w + S.p[1], pk + S.pk[0], c->a1, hb, nullptr, 0, st);
    conv_fwd<kF, kF>(c->a1, hb, 1, S.s, B, w + S.p[2], w + S.p[3], pk + S.pk[1], c->a2, hb, nullptr, 0, st);
    const float* g = c->gout + S.off;
    float* gr = c->grad;
    // layer 3: out = z + conv(h2; W3, b3)
    if (S.C == 1) {
      conv_bwd_w<kF, 1>(c->a2, hb, 1, g, N, S.s, B, c->partial, gr + S.p[4], st);
      conv_bwd_data<1, kF>(g, N, S.s, B, w + S.p[4], pk + S.pk[3], c->a2, hb, c->ga, hb, st);
    } else {
      conv_bwd_w<kF, 3>(c->a2, hb, 1, g, N, S.s, B, c->partial, gr + S.p[4], st);
      conv_bwd_data<3, kF>(g, N, S.s, B, w + S.p[4], pk + S.pk[3], c->a2, hb, c->ga, hb, st);
    }
    // layer 2
    conv_bwd_w<kF, kF>(c->a1, hb, 1, c->ga, hb, S.s, B, c->partial, gr + S.p[2], st);
    conv_bwd_data<kF, kF>(c->ga, hb, S.s, B, w + S.p[2], pk + S.pk[2], c->a1, hb, c->gb, hb, st);
    // layer 1
    if (S.C == 1) conv_bwd_w<1, kF>(z, N, 0, c->gb, hb, S.s, B, c->partial, gr + S.p[0], st);
    else conv_bwd_w<3, kF>(z, N, 0, c->gb, hb, S.s, B, c->partial, gr + S.p[0], st);
  }
  WDB_HIP(hipGetLastError());
  WDB_HIP(hipStreamSynchronize(st));
  double sum = 0.0;
  for (int64_t i = 0; i < nb; ++i) sum += c->hpart[i];
  return sum / static_cast<double>(tot);
}

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

wdb_status wdb_cnn_create(int32_t n, int32_t levels, int32_t features, uint64_t seed, wdb_cnn** out) {
  using namespace wdb;
  WDB_API_BEGIN
  WDB_REQUIRE(out, WDB_ERR_ARG, "null output");
  WDB_REQUIRE(features == kF, WDB_ERR_ARG, "only %d hidden channels are built", kF);
  check_geometry(n, levels, 2);
  WDB_REQUIRE((n >> levels) >= 2, WDB_ERR_LEVELS, "coarsest level too small for 3x3 convolutions");
  wdb_cnn* c = new wdb_cnn();
  try {
    WDB_HIP(hipGetDevice(&c->device));
    c->n = n;
    c->levels = levels;
    c->N = static_cast<int64_t>(n) * n;
    const std::vector<Subband> lay = layout(n, levels);
    int64_t pos = 0;
    int64_t pkpos = 0;
    auto add = [&](int64_t off, int C, int s) {
      wdb_cnn::Stack S{off, C, s, {0, 0, 0, 0, 0, 0}, {0, 0, 0, 0}};
      const int64_t sizes[6] = {int64_t(kF) * C * 9, kF, int64_t(kF) * kF * 9, kF, int64_t(C) * kF * 9, C};
      for (int k = 0; k < 6; ++k) {
        S.p[k] = pos;
        pos += sizes[k];
      }
      const int kpc = 9 * C + ((9 * C) & 1);
      const int64_t pks[4] = {int64_t(kpc) * kF, int64_t(9) * kF * kF, int64_t(9) * kF * kF, int64_t(kpc) * kF};
      for (int k = 0; k < 4; ++k) {
        S.pk[k] = pkpos;
        pkpos += pks[k];   // multiples of 32 entries: every matrix starts 64-byte aligned
      }
      c->stacks.push_back(S);
    };
    add(lay[0].offset, 1, lay[0].side);
    for (size_t k = 1; k < lay.size(); k += 3) add(lay[k].offset, 3, lay[k].side);
    c->nparam = pos;
    // He-normal convolution weights (SplitMix64 + Box-Muller), zero biases; the
    // last convolution of each stack starts 10x smaller so the network starts
    // close to the identity map.
    std::vector<float> h(pos, 0.0f);
    uint64_t st = seed;
    auto normal = [&]() {
      const double u1 = (static_cast<double>(splitmix(st) >> 11) + 0.5) * 0x1.0p-53;
      const double u2 = static_cast<double>(splitmix(st) >> 11) * 0x1.0p-53;
      return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    };
    for (auto& S : c->stacks) {
      const int fan[3] = {S.C * 9, kF * 9, kF * 9};
      const int64_t len[3] = {int64_t(kF) * S.C * 9, int64_t(kF) * kF * 9, int64_t(S.C) * kF * 9};
      for (int l = 0; l < 3; ++l) {
        const double sd = std::sqrt(2.0 / fan[l]) * (l == 2 ? 0.1 : 1.0);
        for (int64_t i = 0; i < len[l]; ++i) h[S.p[2 * l] + i] = static_cast<float>(sd * normal());
      }
    }
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->master), pos * sizeof(float)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->wbf), pos * sizeof(uint16_t)));
    c->npk = pkpos;
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->wpk), pkpos * sizeof(uint16_t)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->m), pos * sizeof(float)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->v), pos * sizeof(float)));
    WDB_HIP(hipMalloc(reinterpret_cast<void**>(&c->grad), pos * sizeof(float)));
    WDB_HIP(hipMemcpy(c->master, h.data(), pos * sizeof(float), hipMemcpyHostToDevice));
    WDB_HIP(hipMemset(c->m, 0, pos * sizeof(float)));
    WDB_HIP(hipMemset(c->v, 0, pos * sizeof(float)));
    hipLaunchKernelGGL(k_round_bf16, grid_for(pos), dim3(kBlk), 0, nullptr, c->master, c->wbf, pos);
    pack_weights(c, nullptr);
    WDB_HIP(hipGetLastError());
    WDB_HIP(hipDeviceSynchronize());
  } catch (...) {
    wdb_cnn_free(c);
    throw;
  }
  *out = c;
  WDB_API_END
}

wdb_status wdb_cnn_param_count(const wdb_cnn* c, int64_t* count) {
  WDB_API_BEGIN
  WDB_REQUIRE(c && count, WDB_ERR_ARG, "null argument");
  *count = c->nparam;
  WDB_API_END
}

wdb_status wdb_cnn_set_params(wdb_cnn* c, const float* host, int64_t count) {
  WDB_API_BEGIN
  WDB_REQUIRE(c && host, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(count == c->nparam, WDB_ERR_ARG, "expected %lld parameters", static_cast<long long>(c->nparam));
  for (int64_t i = 0; i < count; ++i)
    WDB_REQUIRE(std::isfinite(host[i]), WDB_ERR_NONFINITE, "non-finite parameter %lld", static_cast<long long>(i));
  WDB_HIP(hipSetDevice(c->device));
  WDB_HIP(hipMemcpy(c->master, host, count * sizeof(float), hipMemcpyHostToDevice));
  WDB_HIP(hipMemset(c->m, 0, count * sizeof(float)));
  WDB_HIP(hipMemset(c->v, 0, count * sizeof(float)));
  c->t = 0;
  hipLaunchKernelGGL(k_round_bf16, grid_for(count), dim3(kBlk), 0, nullptr, c->master, c->wbf, count);
  pack_weights(c, nullptr);
  WDB_HIP(hipGetLastError());
  WDB_HIP(hipDeviceSynchronize());
  WDB_API_END
}

wdb_status wdb_cnn_get_params(const wdb_cnn* c, float* host, int32_t rounded) {
  WDB_API_BEGIN
  WDB_REQUIRE(c && host, WDB_ERR_ARG, "null argument");
  WDB_HIP(hipSetDevice(c->device));
  if (!rounded) {
    WDB_HIP(hipMemcpy(host, c->master, c->nparam * sizeof(float), hipMemcpyDeviceToHost));
  } else {
    std::vector<uint16_t> b(c->nparam);
    WDB_HIP(hipMemcpy(b.data(), c->wbf, c->nparam * sizeof(uint16_t), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < c->nparam; ++i) {
      const uint32_t u = static_cast<uint32_t>(b[i]) << 16;
      std::memcpy(&host[i], &u, 4);
    }
  }
  WDB_API_END
}

wdb_status wdb_cnn_predict(wdb_cnn* c, const float* x0, int32_t batch, float* out, void* stream) {
  WDB_API_BEGIN
  WDB_REQUIRE(c && x0 && out, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(batch >= 1, WDB_ERR_ARG, "batch must be >= 1");
  WDB_REQUIRE(x0 != out, WDB_ERR_ARG, "x0 and out must not alias");
  WDB_HIP(hipSetDevice(c->device));
  cnn_ensure(c, batch);
  forward(c, x0, batch, out, static_cast<hipStream_t>(stream));
  WDB_API_END
}

wdb_status wdb_cnn_loss_grad(wdb_cnn* c, const float* x0, const float* target, int32_t batch, double* loss,
                             float* grad_host, void* stream) {
  WDB_API_BEGIN
  WDB_REQUIRE(c && x0 && target, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(batch >= 1, WDB_ERR_ARG, "batch must be >= 1");
  WDB_HIP(hipSetDevice(c->device));
  cnn_ensure(c, batch);
  const double L = loss_grad(c, x0, target, batch, static_cast<hipStream_t>(stream));
  if (loss) *loss = L;
  if (grad_host) WDB_HIP(hipMemcpy(grad_host, c->grad, c->nparam * sizeof(float), hipMemcpyDeviceToHost));
  WDB_API_END
}

wdb_status wdb_cnn_train_step(wdb_cnn* c, const float* x0, const float* target, int32_t batch, float lr,
                              double* loss, void* stream) {
  WDB_API_BEGIN
  WDB_REQUIRE(c && x0 && target, WDB_ERR_ARG, "null argument");
  WDB_REQUIRE(batch >= 1 && std::isfinite(lr) && lr > 0, WDB_ERR_ARG, "bad batch or learning rate");
  WDB_HIP(hipSetDevice(c->device));
  cnn_ensure(c, batch);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double L = loss_grad(c, x0, target, batch, st);
  WDB_REQUIRE(std::isfinite(L), WDB_ERR_DIVERGED, "training loss became non-finite");
  c->t += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = static_cast<float>(1.0 - std::pow(b1, static_cast<double>(c->t)));
  const float c2 = static_cast<float>(1.0 - std::pow(b2, static_cast<double>(c->t)));
  hipLaunchKernelGGL(k_adam, grid_for(c->nparam), dim3(kBlk), 0, st, c->master, c->m, c->v, c->grad, c->nparam, lr,
                     static_cast<float>(b1), static_cast<float>(b2), c1, c2, 1e-8f, c->wbf);
  pack_weights(c, st);
  WDB_HIP(hipGetLastError());
  if (loss) *loss = L;
  WDB_API_END
}

void wdb_cnn_free(wdb_cnn* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  cnn_free_ws(c);
  float* fs[] = {c->master, c->m, c->v, c->grad};
  for (float* p : fs)
    if (p) (void)hipFree(p);
  if (c->wbf) (void)hipFree(c->wbf);
  if (c->wpk) (void)hipFree(c->wpk);
  delete c;
}

}  // extern "C"
