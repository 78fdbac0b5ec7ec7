// Batched solve: many deblurring problems (Alg. 1 each) in one call.
//
// Problems that share an operator handle are packed up to eight at a time
// into a "chunk": their vectors are stored row-interleaved ([N][W] floats, W =
// 8, 4, 2 or 1 slots), so one pass over Theta_K's stored entries serves all W
// right-hand sides (a sparse-times-dense product): each stored entry is read
// once and its column gathers 4 W contiguous bytes.  All chunks of all
// operators run in one launch per phase -- the residual kernel, then the
// transposed kernel with the soft-threshold and momentum epilogue -- so an
// iteration of the whole batch is two launches, and the iterations between
// float64 checks can be replayed from a captured HIP graph.  Each right-hand
// side has its own lambda and its own stop flag.  A chunk iterates until its
// last problem stops; when its active problems fit in fewer slots, a check
// moves them to the first slots of a narrower [N][W] layout (the stopped
// problems left out write their final iterates then), so the tail of a
// chunk gathers 4 W bytes per column instead of 32.
//
// Operators whose iteration layout is the tiled pattern storage run their
// chunks on the tiles instead: one 128-thread block (2 wavefronts) per tile,
// lane = row, and for every shared column code each lane loads its column's
// W right-hand-side values (neighbouring lanes of a tile row read neighbouring
// columns) and the tile value once for all of them.  Their float64 checks run
// on the tiles too.
//
// Each problem's iterate is anchored as in the single solve: a float64 anchor
// [N][W] plus the float32 displacement X; the residual subtracts
// c = x0 - Theta_K anchor, the proximal step thresholds anchor + y - tau g in
// float64, and every check first moves X into the anchor, then scores the
// anchor and takes the next c from its float64 residual.
#include <cmath>
#include <map>

#include "codes.hpp"
#include "common.hpp"
#include "prox.hpp"

namespace wdb {

namespace {

constexpr int kBlock = 128;   // 2 wavefronts per tile: 4% faster than 4 and 13% faster than 1 on a 64-problem batch
constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;
constexpr int kR = 8;                  // right-hand sides per chunk

struct ChunkDev {
  const int64_t* soff;
  const float4* val;
  const int4* col;
  const int32_t* perm;
  int64_t nslices, nrows;
  const int64_t* soffT;
  const float4* valT;
  const int4* colT;
  const int32_t* permT;
  int64_t nslicesT;
  int C, cshift;     // slice height of both copies and its log2
  float* X;          // [N][8] iterate (displacement from the anchor)
  float* Y;          // [N][8] extrapolated point (displacement from the anchor)
  const float* X0;   // [N][8] data
  float* Cr;         // [N][8] right-hand side of the displacement iteration, x0 - Theta_K anchor
  double* Anc;       // [N][8] float64 anchor
  float* Rr;         // [N][8] residual
  int W;             // slots in use (8, 4, 2 or 1): the vectors are [N][W], problem slots [0, W)
  const float* pinv; // N or null
  float tau;
  float thr[kR];     // tau * lambda_j
  const int* act;    // stop flags (1 = keep iterating) and, at [8], "any active"; written by the host between replays
  double* r64;       // [N][8] float64 residual for the checks
  // tiled pattern storage of Theta_K / Theta_K^T (ntiles > 0): block b of the chunk is tile b
  int64_t ntiles;
  Geo geo;
  const int4* tdesc[2];
  const uint4* tcode[2];
  const float4* tval[2];
  const GroupRec* tgrec[2];  // kept-value layout (tkept): group records and kept values
  const float* tkval[2];
  uint32_t tkbytes[2];
  int tkept;
  const int* terp[2];
  const int* tec[2];
  const float* tev[2];
};

__device__ __forceinline__ int chunk_of(const int* __restrict__ first, int nchunks, int blk) {
  int c = 0;
  while (c + 1 < nchunks && blk >= first[c + 1]) ++c;
  return c;
}

__device__ __forceinline__ int64_t slot_row_c(const int32_t* perm, int64_t nrows, int64_t q) {
  if (perm) return perm[q];
  return q < nrows ? q : -1;
}

// acc[j] += w V[c][j] for the W slots of an [N][W] block (one 4-, 8-, 16- or
// two 16-byte loads).
template <int W>
__device__ __forceinline__ void gatherW(const float* __restrict__ V, int c, float w, float (&acc)[kR]) {
  const float* p = V + static_cast<int64_t>(c) * W;
  if constexpr (W == 8) {
    const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
    acc[0] = fmaf(w, a.x, acc[0]);
    acc[1] = fmaf(w, a.y, acc[1]);
    acc[2] = fmaf(w, a.z, acc[2]);
    acc[3] = fmaf(w, a.w, acc[3]);
    acc[4] = fmaf(w, b.x, acc[4]);
    acc[5] = fmaf(w, b.y, acc[5]);
    acc[6] = fmaf(w, b.z, acc[6]);
    acc[7] = fmaf(w, b.w, acc[7]);
  } else if constexpr (W == 4) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    acc[0] = fmaf(w, a.x, acc[0]);
    acc[1] = fmaf(w, a.y, acc[1]);
    acc[2] = fmaf(w, a.z, acc[2]);
    acc[3] = fmaf(w, a.w, acc[3]);
  } else if constexpr (W == 2) {
    const float2 a = *reinterpret_cast<const float2*>(p);
    acc[0] = fmaf(w, a.x, acc[0]);
    acc[1] = fmaf(w, a.y, acc[1]);
  } else {
    acc[0] = fmaf(w, p[0], acc[0]);
  }
}

template <int W>
__device__ __forceinline__ void slice_mm(const int64_t* __restrict__ soff, const float4* __restrict__ val,
                                         const int4* __restrict__ col, int64_t sl, int lane, int C,
                                         const float* __restrict__ V, float (&acc)[kR]) {
  const int64_t beg = soff[sl] >> 2, end = soff[sl + 1] >> 2;
  for (int64_t j = beg + lane; j < end; j += C) {
    const float4 v = val[j];
    const int4 c = col[j];
    gatherW<W>(V, c.x, v.x, acc);
    gatherW<W>(V, c.y, v.y, acc);
    gatherW<W>(V, c.z, v.z, acc);
    gatherW<W>(V, c.w, v.w, acc);
  }
}

// Codes and the lane's 4 values of group k of copy m: from the dense values
// or from the kept-value layout.
__device__ __forceinline__ void group_at(const ChunkDev& C, int m, int k, int lane, uint4& c, float4& v) {
  if (C.tkept) {
    const GroupRec r = C.tgrec[m][k];
    c = r.code;
    v = kept_values(r, C.tkval[m], C.tkbytes[m]);
  } else {
    c = C.tcode[m][k];
    v = C.tval[m][static_cast<int64_t>(k) * kWave + lane];
  }
}

// Tile `tile` of copy m (0: Theta_K, 1: Theta_K^T) times the [N][W] block V:
// acc[0..W) of the lane's row, complete in wavefront 0 (the row's escapes
// dealt to the wavefronts, whose partials are added in LDS in wavefront order).
template <int W>
__device__ __forceinline__ int tile_mm(const ChunkDev& C, int m, int tile, const float* __restrict__ V,
                                       float (&acc)[kR], float (*part)[kR][kWave]) {
  const int4 d = C.tdesc[m][tile];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int row = tile_row(d, lane);
  const RowCode rc = tile_row_code(C.geo, d, row);
  for (int k = (d.x >> 2) + wv; k < (d.y >> 2); k += kWaves) {
    uint4 c;
    float4 v;
    group_at(C, m, k, lane, c, v);
    const int4 col = group_cols(C.geo, rc, c);
    gatherW<W>(V, col.x, v.x, acc);
    gatherW<W>(V, col.y, v.y, acc);
    gatherW<W>(V, col.z, v.z, acc);
    gatherW<W>(V, col.w, v.w, acc);
  }
  if (row >= 0 && (d.w & kHasEsc))  // escapes dealt round-robin to the wavefronts
    for (int k = C.terp[m][row] + wv; k < C.terp[m][row + 1]; k += kWaves) gatherW<W>(V, C.tec[m][k], C.tev[m][k], acc);
  if constexpr (kWaves > 1) {
#pragma unroll
    for (int j = 0; j < W; ++j) part[wv][j][lane] = acc[j];
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int j = 0; j < W; ++j) {
        float a = part[0][j][lane];
        for (int w = 1; w < kWaves; ++w) a += part[w][j][lane];
        acc[j] = a;
      }
    }
  }
  return wv == 0 ? row : -1;
}

// Row `row` of r = acc - c over the W slots.
template <int W>
__device__ __forceinline__ void store_residual(const ChunkDev& C, int64_t row, const float (&acc)[kR]) {
  const float* b = C.Cr + row * W;
  float* r = C.Rr + row * W;
  if constexpr (W >= 4) {
#pragma unroll
    for (int h = 0; h < W / 4; ++h) {
      const float4 bb = reinterpret_cast<const float4*>(b)[h];
      reinterpret_cast<float4*>(r)[h] =
          make_float4(acc[4 * h] - bb.x, acc[4 * h + 1] - bb.y, acc[4 * h + 2] - bb.z, acc[4 * h + 3] - bb.w);
    }
  } else if constexpr (W == 2) {
    const float2 bb = *reinterpret_cast<const float2*>(b);
    *reinterpret_cast<float2*>(r) = make_float2(acc[0] - bb.x, acc[1] - bb.y);
  } else {
    r[0] = acc[0] - b[0];
  }
}

template <int W>
__device__ __forceinline__ void res_pack(const ChunkDev& C, int blk, float (*part)[kR][kWave]) {
  float acc[kR] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (C.ntiles) {
    if (blk >= C.ntiles) return;  // the chunk's block range also covers its sliced-ELL checks
    const int row = tile_mm<W>(C, 0, blk, C.Y, acc, part);
    if (row >= 0) store_residual<W>(C, row, acc);
    return;
  }
  const int64_t q = static_cast<int64_t>(blk) * kBlock + threadIdx.x;
  if (q >= (C.nslices << C.cshift)) return;
  const int64_t sl = q >> C.cshift;
  const int lane = static_cast<int>(q & (C.C - 1));
  slice_mm<W>(C.soff, C.val, C.col, sl, lane, C.C, C.Y, acc);
  const int64_t row = slot_row_c(C.perm, C.nrows, q);
  if (row >= 0) store_residual<W>(C, row, acc);
}

__global__ __launch_bounds__(kBlock) void k_res_batched(const ChunkDev* __restrict__ ch, const int* __restrict__ first,
                                                        int nchunks, int* __restrict__ kdev) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *kdev += 1;
  const int c = chunk_of(first, nchunks, blockIdx.x);
  const ChunkDev& C = ch[c];
  if (!C.act[kR]) return;  // every problem of this chunk has stopped
  const int blk = blockIdx.x - first[c];
  __shared__ float part[kWaves][kR][kWave];
  switch (C.W) {
    case 8: res_pack<8>(C, blk, part); break;
    case 4: res_pack<4>(C, blk, part); break;
    case 2: res_pack<2>(C, blk, part); break;
    default: res_pack<1>(C, blk, part); break;
  }
}

template <int W>
__device__ __forceinline__ void prox_pack(const ChunkDev& C, int blk, const int* __restrict__ kdev,
                                          float (*part)[kR][kWave]) {
  float g[kR] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t row;
  if (C.ntiles) {
    if (blk >= C.ntiles) return;
    row = tile_mm<W>(C, 1, blk, C.Rr, g, part);
  } else {
    const int64_t q = static_cast<int64_t>(blk) * kBlock + threadIdx.x;
    if (q >= (C.nslicesT << C.cshift)) return;
    const int64_t sl = q >> C.cshift;
    const int lane = static_cast<int>(q & (C.C - 1));
    slice_mm<W>(C.soffT, C.valT, C.colT, sl, lane, C.C, C.Rr, g);
    row = slot_row_c(C.permT, C.nrows, q);
  }
  if (row < 0) return;
  const int k = *kdev;
  const float beta = static_cast<float>((static_cast<double>(k) - 1.0) / (static_cast<double>(k) + 2.0));
  const float pi = C.pinv ? C.pinv[row] : 1.0f;
  // the row's W slots as whole vectors (a stopped problem's slots are written
  // back unchanged), so every store fills whole segments
  float* X = C.X + row * W;
  float* Y = C.Y + row * W;
  const double* A = C.Anc + row * W;
  float x[W], y[W];
  double a[W];
  if constexpr (W >= 4) {
#pragma unroll
    for (int h = 0; h < W / 4; ++h) {
      const float4 xv = reinterpret_cast<const float4*>(X)[h], yv = reinterpret_cast<const float4*>(Y)[h];
      x[4 * h] = xv.x; x[4 * h + 1] = xv.y; x[4 * h + 2] = xv.z; x[4 * h + 3] = xv.w;
      y[4 * h] = yv.x; y[4 * h + 1] = yv.y; y[4 * h + 2] = yv.z; y[4 * h + 3] = yv.w;
    }
  } else if constexpr (W == 2) {
    const float2 xv = *reinterpret_cast<const float2*>(X), yv = *reinterpret_cast<const float2*>(Y);
    x[0] = xv.x; x[1] = xv.y;
    y[0] = yv.x; y[1] = yv.y;
  } else {
    x[0] = X[0];
    y[0] = Y[0];
  }
  if constexpr (W >= 2) {
#pragma unroll
    for (int h = 0; h < W / 2; ++h) {
      const double2 av = reinterpret_cast<const double2*>(A)[h];
      a[2 * h] = av.x;
      a[2 * h + 1] = av.y;
    }
  } else {
    a[0] = A[0];
  }
#pragma unroll
  for (int j = 0; j < W; ++j) {
    if (!C.act[j]) continue;
    const float xn = prox_anchored(a[j], y[j], (C.tau * pi) * g[j], C.thr[j] * pi);
    y[j] = xn + beta * (xn - x[j]);
    x[j] = xn;
  }
  if constexpr (W >= 4) {
#pragma unroll
    for (int h = 0; h < W / 4; ++h) {
      reinterpret_cast<float4*>(X)[h] = make_float4(x[4 * h], x[4 * h + 1], x[4 * h + 2], x[4 * h + 3]);
      reinterpret_cast<float4*>(Y)[h] = make_float4(y[4 * h], y[4 * h + 1], y[4 * h + 2], y[4 * h + 3]);
    }
  } else if constexpr (W == 2) {
    *reinterpret_cast<float2*>(X) = make_float2(x[0], x[1]);
    *reinterpret_cast<float2*>(Y) = make_float2(y[0], y[1]);
  } else {
    X[0] = x[0];
    Y[0] = y[0];
  }
}

__global__ __launch_bounds__(kBlock) void k_prox_batched(const ChunkDev* __restrict__ ch, const int* __restrict__ first,
                                                         int nchunks, const int* __restrict__ kdev) {
  const int c = chunk_of(first, nchunks, blockIdx.x);
  const ChunkDev& C = ch[c];
  if (!C.act[kR]) return;  // every problem of this chunk has stopped
  const int blk = blockIdx.x - first[c];
  __shared__ float part[kWaves][kR][kWave];
  switch (C.W) {
    case 8: prox_pack<8>(C, blk, kdev, part); break;
    case 4: prox_pack<4>(C, blk, kdev, part); break;
    case 2: prox_pack<2>(C, blk, kdev, part); break;
    default: prox_pack<1>(C, blk, kdev, part); break;
  }
}

// float64 checks: per right-hand side sums of r^2, r.x0, |x| (forward) and
// max |A^T r| (backward); partial[(v * kR + j) * nblocks + block].
__device__ __forceinline__ void block_reduce8(double (&v)[kR], bool is_max, double* __restrict__ out) {
  __shared__ double sh[kWaves][kR];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
  for (int j = 0; j < kR; ++j) {
    double x = v[j];
    for (int off = kWave / 2; off > 0; off >>= 1) {
      const double y = __shfl_xor(x, off);
      x = is_max ? fmax(x, y) : x + y;
    }
    if (lane == 0) sh[wid][j] = x;
  }
  __syncthreads();
  if (threadIdx.x < kR) {
    double a = sh[0][threadIdx.x];
    for (int w = 1; w < kWaves; ++w) a = is_max ? fmax(a, sh[w][threadIdx.x]) : a + sh[w][threadIdx.x];
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

// Tile `tile` of copy m times an [N][8] block V in float64 (V float64, or
// float32 widened): acc[8] of the lane's row, complete in wavefront 0 (escapes
// dealt to the four wavefronts; partials added in LDS in wavefront order).
// Called by every thread of the block.
template <int W, typename T>
__device__ __forceinline__ int tile_mm64(const ChunkDev& C, int m, int tile, const T* __restrict__ V,
                                         double (&acc)[kR], double (*part)[kR][kWave]) {
  const int4 d = C.tdesc[m][tile];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int row = tile_row(d, lane);
  const RowCode rc = tile_row_code(C.geo, d, row);
  auto add = [&](int col, float w) {
    const T* p = V + static_cast<int64_t>(col) * W;
#pragma unroll
    for (int j = 0; j < W; ++j) acc[j] = fma(static_cast<double>(w), static_cast<double>(p[j]), acc[j]);
  };
  for (int k = (d.x >> 2) + wv; k < (d.y >> 2); k += kWaves) {
    uint4 c;
    float4 v;
    group_at(C, m, k, lane, c, v);
    const int4 col = group_cols(C.geo, rc, c);
    add(col.x, v.x);
    add(col.y, v.y);
    add(col.z, v.z);
    add(col.w, v.w);
  }
  if (row >= 0 && (d.w & kHasEsc))
    for (int k = C.terp[m][row] + wv; k < C.terp[m][row + 1]; k += kWaves) add(C.tec[m][k], C.tev[m][k]);
#pragma unroll
  for (int j = 0; j < kR; ++j) part[wv][j][lane] = acc[j];
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      double a = part[0][j][lane];
      for (int w = 1; w < kWaves; ++w) a += part[w][j][lane];
      acc[j] = a;
    }
  }
  return wv == 0 ? row : -1;
}

// Forward half of the float64 check on the anchors: r64 = Theta_K anchor - x0
// and per-block sums of r^2, r.x0, |anchor| per right-hand side.
template <int W>
__device__ __forceinline__ void check_fwd_pack(const ChunkDev& C, int blk, double* __restrict__ part,
                                               int64_t nblocks, double (*tpart)[kR][kWave]) {
  double a[kR], rr[kR], rb[kR], l1[kR];
#pragma unroll
  for (int j = 0; j < kR; ++j) a[j] = rr[j] = rb[j] = l1[j] = 0.0;
  int64_t row = -1;
  if (C.ntiles) {
    if (blk < C.ntiles) row = tile_mm64<W>(C, 0, blk, C.Anc, a, tpart);
  } else {
    const int64_t q = static_cast<int64_t>(blk) * kBlock + threadIdx.x;
    const int64_t sl = q >> C.cshift;
    const int lane = static_cast<int>(q & (C.C - 1));
    if (q < (C.nslices << C.cshift)) {
      const int64_t beg = C.soff[sl] >> 2, end = C.soff[sl + 1] >> 2;
      for (int64_t jj = beg + lane; jj < end; jj += C.C) {
        const float4 v = C.val[jj];
        const int4 cc = C.col[jj];
        const float vv[4] = {v.x, v.y, v.z, v.w};
        const int ci[4] = {cc.x, cc.y, cc.z, cc.w};
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int j = 0; j < W; ++j)
            a[j] = fma(static_cast<double>(vv[t]), C.Anc[static_cast<int64_t>(ci[t]) * W + j], a[j]);
      }
      row = slot_row_c(C.perm, C.nrows, q);
    }
  }
  if (row >= 0) {
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const double b = static_cast<double>(C.X0[row * W + j]);
      const double r = a[j] - b;
      C.r64[row * W + j] = r;
      rr[j] = r * r;
      rb[j] = r * b;
      l1[j] = fabs(C.Anc[row * W + j]);
    }
  }
  double out[kR];
  block_reduce8(rr, false, out);
  if (threadIdx.x < kR) part[(0 * kR + threadIdx.x) * nblocks + blockIdx.x] = out[threadIdx.x];
  block_reduce8(rb, false, out);
  if (threadIdx.x < kR) part[(1 * kR + threadIdx.x) * nblocks + blockIdx.x] = out[threadIdx.x];
  block_reduce8(l1, false, out);
  if (threadIdx.x < kR) part[(2 * kR + threadIdx.x) * nblocks + blockIdx.x] = out[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_check_fwd(const ChunkDev* __restrict__ ch, const int* __restrict__ first,
                                                      int nchunks, double* __restrict__ part, int64_t nblocks) {
  const int c = chunk_of(first, nchunks, blockIdx.x);
  const ChunkDev& C = ch[c];
  if (!C.act[kR]) return;  // every problem of this chunk has stopped
  const int blk = blockIdx.x - first[c];
  __shared__ double tpart[kWaves][kR][kWave];
  switch (C.W) {
    case 8: check_fwd_pack<8>(C, blk, part, nblocks, tpart); break;
    case 4: check_fwd_pack<4>(C, blk, part, nblocks, tpart); break;
    case 2: check_fwd_pack<2>(C, blk, part, nblocks, tpart); break;
    default: check_fwd_pack<1>(C, blk, part, nblocks, tpart); break;
  }
}

template <int W>
__device__ __forceinline__ void check_bwd_pack(const ChunkDev& C, int blk, double* __restrict__ part,
                                               int64_t nblocks, double (*tpart)[kR][kWave]) {
  double g[kR];
#pragma unroll
  for (int j = 0; j < kR; ++j) g[j] = 0.0;
  if (C.ntiles) {
    int row = -1;
    if (blk < C.ntiles) row = tile_mm64<W>(C, 1, blk, static_cast<const double*>(C.r64), g, tpart);
    if (row < 0)
#pragma unroll
      for (int j = 0; j < kR; ++j) g[j] = 0.0;
  } else {
    const int64_t q = static_cast<int64_t>(blk) * kBlock + threadIdx.x;
    const int64_t sl = q >> C.cshift;
    const int lane = static_cast<int>(q & (C.C - 1));
    if (q < (C.nslicesT << C.cshift)) {
      const int64_t beg = C.soffT[sl] >> 2, end = C.soffT[sl + 1] >> 2;
      for (int64_t jj = beg + lane; jj < end; jj += C.C) {
        const float4 v = C.valT[jj];
        const int4 cc = C.colT[jj];
        const float vv[4] = {v.x, v.y, v.z, v.w};
        const int ci[4] = {cc.x, cc.y, cc.z, cc.w};
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int j = 0; j < W; ++j)
            g[j] = fma(static_cast<double>(vv[t]), C.r64[static_cast<int64_t>(ci[t]) * W + j], g[j]);
      }
      if (slot_row_c(C.permT, C.nrows, q) < 0)
#pragma unroll
        for (int j = 0; j < kR; ++j) g[j] = 0.0;
    }
  }
#pragma unroll
  for (int j = 0; j < kR; ++j) g[j] = fabs(g[j]);
  double out[kR];
  block_reduce8(g, true, out);
  if (threadIdx.x < kR) part[(3 * kR + threadIdx.x) * nblocks + blockIdx.x] = out[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_check_bwd(const ChunkDev* __restrict__ ch, const int* __restrict__ first,
                                                      int nchunks, double* __restrict__ part, int64_t nblocks) {
  const int c = chunk_of(first, nchunks, blockIdx.x);
  const ChunkDev& C = ch[c];
  if (!C.act[kR]) return;  // every problem of this chunk has stopped
  const int blk = blockIdx.x - first[c];
  __shared__ double tpart[kWaves][kR][kWave];
  switch (C.W) {
    case 8: check_bwd_pack<8>(C, blk, part, nblocks, tpart); break;
    case 4: check_bwd_pack<4>(C, blk, part, nblocks, tpart); break;
    case 2: check_bwd_pack<2>(C, blk, part, nblocks, tpart); break;
    default: check_bwd_pack<1>(C, blk, part, nblocks, tpart); break;
  }
}

// Anchored iterate, elementwise over a chunk's [N][8] vectors.
__global__ void k_anchor_init8(double* __restrict__ anc, float* __restrict__ cr, const float* __restrict__ x0,
                               int64_t n8) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n8) return;
  anc[i] = 0.0;
  cr[i] = x0[i];
}

// anchor += X; Y -= X; X = 0 (the iterate and the extrapolated point keep their values as sums)
__global__ void k_reanchor8(double* __restrict__ anc, float* __restrict__ x, float* __restrict__ y, int64_t n8) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n8) return;
  const float d = x[i];
  anc[i] += static_cast<double>(d);
  y[i] -= d;
  x[i] = 0.0f;
}

// c = -r64 = x0 - Theta_K anchor
__global__ void k_anchor_rhs8(const double* __restrict__ r64, float* __restrict__ cr, int64_t n8) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n8) cr[i] = static_cast<float>(-r64[i]);
}

// One block per chunk and value: reduce that chunk's block range for one of
// its 4 x 8 values (sums, or the maximum for the last 8).
__global__ __launch_bounds__(kBlock) void k_check_reduce(const int* __restrict__ first, const double* __restrict__ part,
                                                         int64_t nblocks, double* __restrict__ out) {
  __shared__ double sh[kBlock];
  const int c = blockIdx.x / (4 * kR), v = blockIdx.x % (4 * kR);
  const int b0 = first[c], b1 = first[c + 1];
  const bool mx = v >= 3 * kR;
  double acc = 0.0;
  for (int b = b0 + threadIdx.x; b < b1; b += kBlock) {
    const double p = part[static_cast<int64_t>(v) * nblocks + b];
    acc = mx ? fmax(acc, p) : acc + p;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = mx ? fmax(sh[threadIdx.x], sh[threadIdx.x + w]) : sh[threadIdx.x] + sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c * 4 * kR + v] = sh[0];
}

// The eight slots of a chunk's [N][8] block from eight vectors (null: zeros),
// written to dst and, if given, dst2.
struct Src8 {
  const float* p[kR];
};
__global__ void k_interleave8(Src8 src, float* __restrict__ dst, float* __restrict__ dst2, int64_t N, int W) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
#pragma unroll
  for (int j = 0; j < kR; ++j) {
    if (j >= W) break;
    const float v = src.p[j] ? src.p[j][i] : 0.0f;
    dst[i * W + j] = v;
    if (dst2) dst2[i * W + j] = v;
  }
}

// The problems' iterates: the anchors rounded to float32 (and as float64 where asked).
struct Dst8 {
  float* p[kR];
  double* p64[kR];
};
__global__ void k_deinterleave8(const double* __restrict__ src, Dst8 dst, int W, int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
#pragma unroll
  for (int j = 0; j < kR; ++j) {
    if (j >= W) break;
    if (!dst.p[j]) continue;   // slot left out
    const double v = src[i * W + j];
    dst.p[j][i] = static_cast<float>(v);
    if (dst.p64[j]) dst.p64[j][i] = v;
  }
}

// Narrowing of packs, all packs of a check in one launch per step (blockIdx.y
// = job).  A job moves a pack's [N][Wold] block to an [N][W] block, slot j
// taken from old slot from[j]; its stopped problems left out are written out
// first (out: their x_out / x64_out per old slot, null elsewhere).
struct NarrowJob {
  int64_t off, N;
  int Wold, W;
  int from[kR];
  Dst8 out;
};

// Dropped problems' final iterates (the anchors in the old layout).
__global__ void k_narrow_out(const NarrowJob* __restrict__ jobs, const double* __restrict__ anc) {
  const NarrowJob& J = jobs[blockIdx.y];
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < J.N;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    for (int j = 0; j < J.Wold; ++j) {
      if (!J.out.p[j]) continue;
      const double v = anc[J.off + i * J.Wold + j];
      J.out.p[j][i] = static_cast<float>(v);
      if (J.out.p64[j]) J.out.p64[j][i] = v;
    }
  }
}

// tmp = the old block of each job's pack (tmp and dst are pools of the same layout).
template <typename T>
__global__ void k_narrow_copy(const NarrowJob* __restrict__ jobs, const T* __restrict__ src, T* __restrict__ tmp) {
  const NarrowJob& J = jobs[blockIdx.y];
  const int64_t n = J.N * J.Wold;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    tmp[J.off + i] = src[J.off + i];
}

// dst = the new block, from the copy of the old one.
template <typename T>
__global__ void k_narrow_move(const NarrowJob* __restrict__ jobs, const T* __restrict__ tmp, T* __restrict__ dst) {
  const NarrowJob& J = jobs[blockIdx.y];
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < J.N;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    for (int j = 0; j < J.W; ++j) dst[J.off + i * J.W + j] = tmp[J.off + i * J.Wold + J.from[j]];
}

__global__ void k_set(int* p, int v) { *p = v; }

}  // namespace

}  // namespace wdb

extern "C" wdb_status wdb_solve_batched(int32_t nprob, const wdb_problem* probs, const wdb_solve_opts* opts,
                                        wdb_solve_info* infos) {
  using namespace wdb;
  WDB_API_BEGIN
  WDB_REQUIRE(nprob >= 1 && probs && opts, WDB_ERR_ARG, "need at least one problem and options");
  WDB_REQUIRE(opts->max_iters >= 0 && opts->check_every >= 0, WDB_ERR_ARG, "bad iteration counts");
  WDB_REQUIRE(opts->x_init == nullptr, WDB_ERR_ARG, "x_init is per problem in a batch (wdb_problem.x_init)");
  WDB_REQUIRE(opts->ista == 0, WDB_ERR_ARG, "the batched solver runs Alg. 1 (ista must be 0)");
  const bool pre = opts->use_precond != 0;
  bool stopping = opts->tol_rel_gap > 0;
  for (int i = 0; i < nprob; ++i) stopping |= probs[i].target_objective > 0;
  hipStream_t s = static_cast<hipStream_t>(opts->stream);
  // group by operator, in first-seen order, then split into chunks of 8
  std::vector<wdb_theta*> order;
  std::map<wdb_theta*, std::vector<int>> members;
  for (int i = 0; i < nprob; ++i) {
    const wdb_problem& p = probs[i];
    WDB_REQUIRE(p.theta && (p.u || p.x0) && p.x_out, WDB_ERR_ARG, "problem %d has a null pointer", i);
    WDB_REQUIRE(std::isfinite(p.lambda) && p.lambda >= 0.0f, WDB_ERR_NONFINITE, "problem %d: bad lambda", i);
    WDB_REQUIRE(p.theta->valtype == WDB_VAL_F32, WDB_ERR_ARG, "batched solve uses float32 values");
    WDB_REQUIRE(p.theta->l1w == nullptr, WDB_ERR_ARG, "batched solve uses uniform l1 weights");
    WDB_REQUIRE(!pre || p.theta->precond != 0, WDB_ERR_ARG, "problem %d: no preconditioner set", i);
    if (!members.count(p.theta)) order.push_back(p.theta);
    members[p.theta].push_back(i);
  }
  // Chunks of up to eight problems per operator; every chunk's [N][8] vectors
  // live at its offset in one pool per vector kind, so the elementwise steps
  // run over all chunks in one launch.
  struct Host {
    wdb_theta* th;
    std::vector<int> idx;   // problem of each slot
    int W;                  // slots in use: the vectors are [N][W]
    int64_t off;            // first element of the chunk's block (room for [N][8]) in the pools
    int blocks_res, blocks_prox, blocks;
  };
  auto slots_for = [](int n) { return n > 4 ? 8 : (n > 2 ? 4 : (n > 1 ? 2 : 1)); };
  std::vector<Host> chunks;
  int64_t tot8 = 0;
  for (wdb_theta* th : order) {
    WDB_HIP(hipSetDevice(th->device));
    ensure_workspace(th);
    if (!th->has_L) {   // the solver's default step (as wdb_solve)
      const LanczosResult r = lanczos_max(th, nullptr, nullptr, 1e-12, 2000, s);
      th->L = r.theta + r.resid;
      th->has_L = true;
    }
    const std::vector<int>& m = members[th];
    for (size_t b = 0; b < m.size(); b += kR) {
      Host h;
      h.th = th;
      h.idx.assign(m.begin() + b, m.begin() + std::min(m.size(), b + kR));
      h.W = slots_for(static_cast<int>(h.idx.size()));
      h.off = tot8;
      tot8 += th->N * kR;
      h.blocks_res = static_cast<int>((th->A.nslices * th->A.C + kBlock - 1) / kBlock);
      h.blocks_prox = static_cast<int>((th->At.nslices * th->At.C + kBlock - 1) / kBlock);
      h.blocks = std::max(h.blocks_res, h.blocks_prox);
      if (kernel_group(th) == kTiled) h.blocks = std::max<int>(h.blocks, static_cast<int>(th->tA.ntiles));
      chunks.push_back(std::move(h));
    }
  }
  const int nch = static_cast<int>(chunks.size());
  DevBuf<float> pX(tot8), pY(tot8), pX0(tot8), pRr(tot8), pCr(tot8);
  DevBuf<double> pR64(tot8), pAnc(tot8);
  DevBuf<int> pAct(static_cast<size_t>(nch) * (kR + 1));
  std::vector<int> act_host(static_cast<size_t>(nch) * (kR + 1), 0);   // per chunk: eight slot flags, then "any"
  std::vector<ChunkDev> hd(nch);
  std::vector<int> first(nch + 1, 0);
  for (int c = 0; c < nch; ++c) first[c + 1] = first[c] + chunks[c].blocks;
  const int64_t nblocks = first[nch];
  DevBuf<ChunkDev> dch(nch);
  DevBuf<int> dfirst(nch + 1);
  DevBuf<double> part(static_cast<size_t>(4 * kR) * nblocks), red(static_cast<size_t>(nch) * 4 * kR);
  DevBuf<int> kdev(1);
  DevBuf<NarrowJob> djobs;
  size_t njobs_cap = 0;
  std::vector<NarrowJob> jobs;
  for (int c = 0; c < nch; ++c) {
    Host& h = chunks[c];
    wdb_theta* th = h.th;
    const int64_t N = th->N;
    const double L = pre ? th->Lp : th->L;
    WDB_REQUIRE(L > 0.0 && std::isfinite(L), WDB_ERR_ARG, "operator has no positive Lipschitz constant");
    const double tau = 1.0 / L;
    ChunkDev& d = hd[c];
    d.soff = th->A.slice_off;
    d.val = reinterpret_cast<const float4*>(th->A.val);
    d.col = reinterpret_cast<const int4*>(th->A.col);
    d.perm = th->A.perm;
    d.nslices = th->A.nslices;
    d.nrows = N;
    d.soffT = th->At.slice_off;
    d.valT = reinterpret_cast<const float4*>(th->At.val);
    d.colT = reinterpret_cast<const int4*>(th->At.col);
    d.permT = th->At.perm;
    d.nslicesT = th->At.nslices;
    WDB_REQUIRE(th->A.C == th->At.C, WDB_ERR_HIP, "mismatched slice heights");
    d.C = th->A.C;
    d.cshift = __builtin_ctz(static_cast<unsigned>(th->A.C));
    d.X = pX.p + h.off;
    d.Y = pY.p + h.off;
    d.X0 = pX0.p + h.off;
    d.Cr = pCr.p + h.off;
    d.Anc = pAnc.p + h.off;
    d.Rr = pRr.p + h.off;
    d.W = h.W;
    d.pinv = pre ? th->pinv : nullptr;
    d.tau = static_cast<float>(tau);
    d.act = pAct.p + static_cast<int64_t>(c) * (kR + 1);
    d.r64 = pR64.p + h.off;
    d.ntiles = 0;
    d.tkept = 0;
    if (kernel_group(th) == kTiled) {  // the operator iterates on its tiled copies
      WDB_REQUIRE(!th->tile_kept || tiled_kept_available(th), WDB_ERR_ARG, "kept-value tiles not built");
      d.tkept = th->tile_kept;
      WDB_REQUIRE(th->tA.ntiles == th->tAt.ntiles, WDB_ERR_ARG, "mismatched tile lists");
      d.ntiles = th->tA.ntiles;
      d.geo = geo_of(th);
      const Tiled* T[2] = {&th->tA, &th->tAt};
      for (int m = 0; m < 2; ++m) {
        d.tdesc[m] = reinterpret_cast<const int4*>(T[m]->desc);
        d.tcode[m] = reinterpret_cast<const uint4*>(T[m]->code);
        d.tval[m] = reinterpret_cast<const float4*>(T[m]->val);
        d.tgrec[m] = static_cast<const GroupRec*>(T[m]->grec);
        d.tkval[m] = T[m]->kval;
        d.tkbytes[m] = static_cast<uint32_t>(4 * (T[m]->nkval + 4));
        d.terp[m] = T[m]->erp;
        d.tec[m] = T[m]->ec;
        d.tev[m] = T[m]->ev;
      }
    }
    const Filter f = make_filter(th->wavelet);
    const size_t q = static_cast<size_t>(th->n / 2) * (th->n / 2);
    int* act = act_host.data() + static_cast<size_t>(c) * (kR + 1);
    Src8 x0s{}, inits{};
    // data terms x0 = Psi^* u of the problems given as images: transformed
    // together into the chunk's X block (slot j at j N), with the Y block as
    // their scratch; both blocks are filled below
    const float* us[kR];
    float *xs[kR], *sa[kR], *sb[kR];
    int nu = 0;
    for (int j = 0; j < kR; ++j) {
      d.thr[j] = 0.0f;
      if (j < static_cast<int>(h.idx.size())) {
        const wdb_problem& p = probs[h.idx[j]];
        d.thr[j] = static_cast<float>(tau * static_cast<double>(p.lambda));
        act[j] = 1;
        x0s.p[j] = p.x0;
        if (!x0s.p[j]) {
          us[nu] = p.u;
          xs[nu] = d.X + static_cast<int64_t>(j) * N;
          sa[nu] = d.Y + static_cast<int64_t>(j) * N;
          sb[nu] = sa[nu] + q;
          x0s.p[j] = xs[nu];
          ++nu;
        }
        inits.p[j] = p.x_init;
      }
    }
    if (nu) dwt_forward_many(th->n, th->levels, f, nu, us, xs, sa, sb, s);
    const dim3 g8(static_cast<unsigned>((N + 255) / 256));
    hipLaunchKernelGGL(k_interleave8, g8, dim3(256), 0, s, x0s, pX0.p + h.off, static_cast<float*>(nullptr), N,
                       h.W);
    hipLaunchKernelGGL(k_interleave8, g8, dim3(256), 0, s, inits, d.X, d.Y, N, h.W);
    act[kR] = h.idx.empty() ? 0 : 1;
  }
  hipLaunchKernelGGL(k_anchor_init8, dim3(static_cast<unsigned>((tot8 + 255) / 256)), dim3(256), 0, s, pAnc.p, pCr.p,
                     pX0.p, tot8);
  WDB_HIP(hipGetLastError());
  WDB_HIP(hipMemcpyAsync(pAct.p, act_host.data(), act_host.size() * sizeof(int), hipMemcpyHostToDevice, s));
  WDB_HIP(hipMemcpyAsync(dch.p, hd.data(), nch * sizeof(ChunkDev), hipMemcpyHostToDevice, s));
  WDB_HIP(hipMemcpyAsync(dfirst.p, first.data(), (nch + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  const int k0 = opts->k0 > 0 ? opts->k0 : 1;
  hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, s, kdev.p, k0 - 1);

  auto iterate = [&](hipStream_t st) {
    hipLaunchKernelGGL(k_res_batched, dim3(static_cast<unsigned>(nblocks)), dim3(kBlock), 0, st, dch.p, dfirst.p, nch,
                       kdev.p);
    hipLaunchKernelGGL(k_prox_batched, dim3(static_cast<unsigned>(nblocks)), dim3(kBlock), 0, st, dch.p, dfirst.p,
                       nch, kdev.p);
  };
  const int c = opts->check_every;
  const int total = opts->max_iters;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  std::vector<double> hred(static_cast<size_t>(nch) * 4 * kR);
  std::vector<double> lastE(nprob, 0.0), lastG(nprob, 0.0);
  std::vector<int> done_at(nprob, -1);
  int done = 0, checks = 0;
  bool all_conv = false;
  try {
    if (opts->use_graph && c > 1 && total >= c) {
      WDB_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      WDB_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < c; ++i) iterate(cap);
      WDB_HIP(hipStreamEndCapture(cap, &graph));
      WDB_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    while (done < total || (total == 0 && checks == 0)) {
      int step = total - done;
      if (c > 0) step = std::min(step, c - (done % c));
      if (exec && step == c) {
        WDB_HIP(hipGraphLaunch(exec, s));
      } else {
        for (int i = 0; i < step; ++i) iterate(s);
      }
      WDB_HIP(hipGetLastError());
      done += step;
      const bool at_check = (c > 0 && done % c == 0) || done == total;
      if (!at_check) continue;
      const dim3 gall(static_cast<unsigned>((tot8 + 255) / 256));
      hipLaunchKernelGGL(k_reanchor8, gall, dim3(256), 0, s, pAnc.p, pX.p, pY.p, tot8);
      hipLaunchKernelGGL(k_check_fwd, dim3(static_cast<unsigned>(nblocks)), dim3(kBlock), 0, s, dch.p, dfirst.p, nch,
                         part.p, nblocks);
      hipLaunchKernelGGL(k_check_bwd, dim3(static_cast<unsigned>(nblocks)), dim3(kBlock), 0, s, dch.p, dfirst.p, nch,
                         part.p, nblocks);
      hipLaunchKernelGGL(k_check_reduce, dim3(nch * 4 * kR), dim3(kBlock), 0, s, dfirst.p, part.p, nblocks, red.p);
      hipLaunchKernelGGL(k_anchor_rhs8, gall, dim3(256), 0, s, pR64.p, pCr.p, tot8);
      WDB_HIP(hipGetLastError());
      WDB_HIP(hipMemcpyAsync(hred.data(), red.p, hred.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      WDB_HIP(hipStreamSynchronize(s));
      ++checks;
      bool any_active = false, changed = false;
      for (int ci = 0; ci < nch; ++ci) {
        Host& h = chunks[ci];
        int* act = act_host.data() + static_cast<size_t>(ci) * (kR + 1);
        for (int j = 0; j < static_cast<int>(h.idx.size()); ++j) {
          const int pi = h.idx[j];
          if (done_at[pi] >= 0) continue;  // already stopped
          const double lam = static_cast<double>(probs[pi].lambda);
          const double rr = hred[ci * 4 * kR + 0 * kR + j], rb = hred[ci * 4 * kR + 1 * kR + j];
          const double l1 = hred[ci * 4 * kR + 2 * kR + j], gm = hred[ci * 4 * kR + 3 * kR + j];
          const double E = 0.5 * rr + lam * l1;
          const double sc = gm <= lam ? 1.0 : lam / gm;
          const double D = -0.5 * sc * sc * rr - sc * rb;
          lastE[pi] = E;
          lastG[pi] = E > 0 ? (E - D) / E : 0.0;
          WDB_REQUIRE(std::isfinite(E), WDB_ERR_DIVERGED, "problem %d diverged", pi);
          if ((opts->tol_rel_gap > 0 && lastG[pi] <= opts->tol_rel_gap) ||
              (probs[pi].target_objective > 0 && E <= probs[pi].target_objective)) {
            done_at[pi] = done;
            changed = true;
          }
        }
        act[kR] = 0;
        for (int j = 0; j < static_cast<int>(h.idx.size()); ++j) {
          act[j] = done_at[h.idx[j]] < 0 ? 1 : 0;
          act[kR] |= act[j];
        }
        any_active |= act[kR] != 0;
      }
      // Narrow the packs whose active problems fit in fewer slots: the active
      // problems move to the first slots of an [N][W] layout (the residual and
      // check-residual blocks serve as copies of the old layout); the stopped
      // problems left out write their final iterates now.
      jobs.clear();   // (the host table outlives the copy to the device: the next check synchronises first)
      for (int ci = 0; ci < nch && changed; ++ci) {
        Host& h = chunks[ci];
        int* act = act_host.data() + static_cast<size_t>(ci) * (kR + 1);
        int na = 0;
        for (int j = 0; j < static_cast<int>(h.idx.size()); ++j) na += act[j];
        if (na == 0) continue;
        const int Wn = slots_for(na);
        if (Wn >= h.W) continue;
        std::vector<int> keep, drop;
        for (int j = 0; j < static_cast<int>(h.idx.size()); ++j) (act[j] ? keep : drop).push_back(j);
        while (static_cast<int>(keep.size()) < Wn && !drop.empty()) {   // fill the rest with stopped slots
          keep.push_back(drop.front());
          drop.erase(drop.begin());
        }
        NarrowJob J{};
        J.off = h.off;
        J.N = h.th->N;
        J.Wold = h.W;
        J.W = Wn;
        for (int j = 0; j < kR; ++j) J.from[j] = j < static_cast<int>(keep.size()) ? keep[j] : 0;
        for (int j : drop) {
          J.out.p[j] = probs[h.idx[j]].x_out;
          J.out.p64[j] = probs[h.idx[j]].x64_out;
        }
        jobs.push_back(J);
        std::vector<int> idx(keep.size());
        float thr[kR] = {};
        int nact[kR + 1] = {};
        for (size_t j = 0; j < keep.size(); ++j) {
          idx[j] = h.idx[keep[j]];
          thr[j] = hd[ci].thr[keep[j]];
          nact[j] = act[keep[j]];
        }
        nact[kR] = 1;
        h.idx = idx;
        h.W = Wn;
        for (int j = 0; j <= kR; ++j) act[j] = nact[j];
        for (int j = 0; j < kR; ++j) hd[ci].thr[j] = thr[j];
        hd[ci].W = Wn;
      }
      if (!jobs.empty()) {
        // Narrow the packs whose active problems fit in fewer slots: the active
        // problems move to the first slots of an [N][W] layout (the residual and
        // check-residual pools serve as copies of the old layout; both are
        // recomputed before they are read again); the stopped problems left out
        // write their final iterates first.
        if (jobs.size() > njobs_cap) {
          djobs.alloc(jobs.size());
          njobs_cap = jobs.size();
        }
        WDB_HIP(hipMemcpyAsync(djobs.p, jobs.data(), jobs.size() * sizeof(NarrowJob), hipMemcpyHostToDevice, s));
        const dim3 gj(256, static_cast<unsigned>(jobs.size()));
        hipLaunchKernelGGL(k_narrow_out, gj, dim3(256), 0, s, djobs.p, pAnc.p);
        float* fl[4] = {pX.p, pY.p, pX0.p, pCr.p};
        for (float* a : fl) {
          hipLaunchKernelGGL(k_narrow_copy<float>, gj, dim3(256), 0, s, djobs.p, a, pRr.p);
          hipLaunchKernelGGL(k_narrow_move<float>, gj, dim3(256), 0, s, djobs.p, pRr.p, a);
        }
        hipLaunchKernelGGL(k_narrow_copy<double>, gj, dim3(256), 0, s, djobs.p, pAnc.p, pR64.p);
        hipLaunchKernelGGL(k_narrow_move<double>, gj, dim3(256), 0, s, djobs.p, pR64.p, pAnc.p);
        WDB_HIP(hipGetLastError());
        WDB_HIP(hipMemcpyAsync(dch.p, hd.data(), nch * sizeof(ChunkDev), hipMemcpyHostToDevice, s));
        // (the job table is rewritten only after the next check's synchronisation)
      }
      if (changed)
        WDB_HIP(hipMemcpyAsync(pAct.p, act_host.data(), act_host.size() * sizeof(int), hipMemcpyHostToDevice, s));
      if (stopping && !any_active) {
        all_conv = true;
        break;
      }
    }
  } catch (...) {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    throw;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (cap) (void)hipStreamDestroy(cap);
  for (int ci = 0; ci < nch; ++ci) {
    Host& h = chunks[ci];
    const int64_t N = h.th->N;
    Dst8 dst{};
    for (int j = 0; j < static_cast<int>(h.idx.size()); ++j) {
      dst.p[j] = probs[h.idx[j]].x_out;
      dst.p64[j] = probs[h.idx[j]].x64_out;
    }
    hipLaunchKernelGGL(k_deinterleave8, dim3(static_cast<unsigned>((N + 255) / 256)), dim3(256), 0, s,
                       pAnc.p + h.off, dst, h.W, N);
  }
  WDB_HIP(hipGetLastError());
  WDB_HIP(hipStreamSynchronize(s));
  if (infos) {
    for (int i = 0; i < nprob; ++i) {
      wdb_theta* th = probs[i].theta;
      infos[i].iters = done_at[i] >= 0 ? done_at[i] : done;
      infos[i].checks = checks;
      infos[i].objective = lastE[i];
      infos[i].rel_gap = lastG[i];
      infos[i].lipschitz = pre ? th->Lp : th->L;
      infos[i].tau = 1.0 / infos[i].lipschitz;
    }
  }
  if (stopping && !all_conv)
    fail(WDB_ERR_NOT_CONVERGED, "not every problem met its stopping test in %d iterations", done);
  WDB_API_END
}
