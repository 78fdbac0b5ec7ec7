// Internal declarations shared by the wdb library sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <functional>
#include <string>
#include <vector>

#include "../../include/wdb.h"

namespace wdb {

// ---------------------------------------------------------------------------
// Errors: internal code throws wdb::Error; every extern "C" entry point
// catches it, records the message for wdb_last_error() and returns the code.
// ---------------------------------------------------------------------------
struct Error {
  wdb_status code;
  std::string msg;
};

[[noreturn]] void fail(wdb_status code, const char* fmt, ...);
void set_last_error(const std::string& msg);
void clear_last_error();

#define WDB_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      ::wdb::fail(e_ == hipErrorOutOfMemory ? WDB_ERR_OOM : WDB_ERR_HIP, "%s: %s (%s:%d)", \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                    \
  } while (0)

#define WDB_REQUIRE(cond, code, ...) \
  do {                               \
    if (!(cond)) ::wdb::fail(code, __VA_ARGS__); \
  } while (0)

#define WDB_API_BEGIN try { ::wdb::clear_last_error();
#define WDB_API_END                                        \
  }                                                        \
  catch (const ::wdb::Error& e_) {                         \
    ::wdb::set_last_error(e_.msg);                         \
    return e_.code;                                        \
  }                                                        \
  catch (const std::bad_alloc&) {                          \
    ::wdb::set_last_error("host allocation failed");       \
    return WDB_ERR_OOM;                                    \
  }                                                        \
  catch (...) {                                            \
    ::wdb::set_last_error("unexpected internal exception"); \
    return WDB_ERR_HIP;                                    \
  }                                                        \
  return WDB_OK;

// Device allocation owned by RAII (frees on scope exit unless released).
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    reset();
    p = o.p; n = o.n; o.p = nullptr; o.n = 0;
    return *this;
  }
  ~DevBuf() { reset(); }
  void alloc(size_t count) {
    reset();
    n = count;
    if (count) WDB_HIP(hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)));
  }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  T* release() { T* q = p; p = nullptr; n = 0; return q; }
  size_t bytes() const { return n * sizeof(T); }
};

// ---------------------------------------------------------------------------
// Filters (host, float64).
// ---------------------------------------------------------------------------
constexpr int kMaxTaps = 12;  // longest filter (Symmlet 6)

struct Filter {
  std::vector<double> h;  // low-pass analysis taps
  std::vector<double> g;  // high-pass g[m] = (-1)^m h[L-1-m]
};
Filter make_filter(int wavelet);  // throws WDB_ERR_ARG for unknown wavelets

// Validate n (power of two >= 2) and levels against the filter length.
void check_geometry(int32_t n, int32_t levels, int flen);

// Canonical coefficient layout: subband k has (level, e_row, e_col, offset, side).
struct Subband {
  int level, erow, ecol;
  int64_t offset;
  int side;
};
std::vector<Subband> layout(int32_t n, int32_t levels);

// ---------------------------------------------------------------------------
// Sliced-ELL storage of one sparse N x N matrix (rows = output index).
// Rows are grouped in slices of C (a power of two, 8..64; one thread per row).
// Slice s holds width w_s (a multiple of 4) entries per row, laid out as
// [w_s/4][C rows][4], so each thread reads one 16-byte vector of values and
// one of column indices per step and a slice step is 16*C contiguous bytes.
// Padding slots have value 0 and repeat a valid column of the same row.
// Rows may be reordered inside windows of `sort_window` rows by decreasing
// length (sliced ELL with local sorting), so that the rows sharing a slice
// have similar lengths; `perm` then maps each slot row to its matrix row.
// ---------------------------------------------------------------------------
constexpr int kSliceMax = 64;

struct Sell {
  int C = kSliceMax;             // slice height
  int64_t nrows = 0, nslices = 0, stored = 0;
  int64_t* slice_off = nullptr;  // device, nslices + 1 (element offsets)
  float* val = nullptr;          // device, stored
  int32_t* col = nullptr;        // device, stored
  int32_t* perm = nullptr;       // device, nslices * C (-1: empty slot row), or null = identity
  void free_all();
};

// Rows per sorting window of the sliced-ELL layout (0 or 64: no reordering).
int64_t sell_sort_window();

// Device CSR (sorted columns) of one matrix.
struct Csr {
  int64_t nrows = 0, nnz = 0;
  int64_t* rowptr = nullptr;  // device, nrows + 1
  int32_t* col = nullptr;     // device, nnz
  double* val = nullptr;      // device, nnz
  void free_all();
};

// Float32 CSR copy used by the row-group ("vector CSR") kernels, with every
// row padded to a multiple of 4 entries (value 0, column = the row index) so
// row starts are 16-byte aligned and a lane can load 4 values and 4 columns at
// once.  rowptr holds the padded offsets (multiples of 4).
struct Csr32 {
  int64_t nrows = 0, nnz = 0, stored = 0;
  int64_t* rowptr = nullptr;  // device, nrows + 1
  int32_t* col = nullptr;     // device, stored
  float* val = nullptr;       // device, stored
  void free_all();
};
void csr_to_csr32(const Csr& a, Csr32* out, hipStream_t s);

// Circulant (stencil) storage of a convolution's Theta_K, built by the fast
// path: per row subband, segments of (offset, value) generators shared by all
// rows, plus explicit entries of the cut's partial tie group.
struct Stencil {
  int* seg_ptr = nullptr;  // device, nsub + 1
  void* seg = nullptr;     // device, nseg segment records
  int* gp = nullptr;       // device, ngen (offset, value bits) pairs
  int* res = nullptr;      // device, residue tables
  int* xrp = nullptr;      // device, N + 1 (null: no explicit entries)
  int* xc = nullptr;
  float* xv = nullptr;
  int64_t nseg = 0, ngen = 0, nextra = 0;
  void free_all();
};
// One kept generator of the fast build: `form` 0 = rows in subband k (at
// offset off_k), columns in b; 1 = rows in b, columns in k; p the offset in
// b, r the side ratio.
struct CircGen {
  int64_t off_k, off_b;
  int side_k, side_b, p1, p2, r, form;
  double v;
};


// Packed 16-bit form of one matrix (CSR order): per entry a 32-bit word holding
// the scaled 16-bit value (high half) and a band-relative column code (low
// half); entries whose column does not fit the code go to a per-row escape
// list.  Row r owns words [meta[r].x, meta[r+1].x) (a multiple of 4, padded
// with value-0 words) and escapes [meta[r].y, meta[r+1].y).
struct Packed {
  int64_t nrows = 0, npacked = 0, nesc = 0;
  int2* meta = nullptr;      // device, nrows + 1
  uint32_t* word = nullptr;  // device, npacked
  uint16_t* ev = nullptr;    // device, nesc: escape values
  int32_t* ec = nullptr;     // device, nesc: escape columns
  void free_all();
};
// Tiled pattern storage of one matrix: tiles of up to 64 rows of one subband
// share a sorted list of band-relative column codes; values are stored per
// (code, row) with zeros where a row lacks the entry.  Tile t owns codes
// [desc[t].x, desc[t].y) and values [desc[t].x * 64, desc[t].y * 64) laid out
// [group of 4 codes][lane][4]; rows with entries that have no code keep them
// in a per-row escape list (erp null when there are none).
struct Tiled {
  int64_t ntiles = 0, npat = 0, nesc = 0, nkept = 0;
  int* desc = nullptr;       // device, 4 * ntiles (int4 per tile)
  uint32_t* code = nullptr;  // device, npat
  float* val = nullptr;      // device, 64 * npat (float32 copies)
  uint16_t* val16 = nullptr; // device, 64 * npat (16-bit copies: groups of 8 codes, scaled values)
  int* erp = nullptr;        // device, nrows + 1
  int* ec = nullptr;         // device, nesc
  float* ev = nullptr;       // device, nesc
  // Kept-value layout of the float32 copies (groups of 4 codes): per group a
  // record with the codes, a row mask per code and the offset of its kept
  // values, which are stored without the zeros of the dense values.
  void* grec = nullptr;      // device, one 64-byte record per group
  float* kval = nullptr;     // device, nkval (+ 4 zeros)
  int64_t nkval = 0;
  void free_all();
};
// Lanes per row of the vector-CSR kernels (0: sliced-ELL kernels).
int spmv_group();

// Build a SELL copy of a device CSR (float64 values rounded to float32).
void csr_to_sell(const Csr& a, Sell* out, hipStream_t s, int64_t sort_window, int C);
// Element index of entry k of slot row `lane` in the slice starting at `base`.
__host__ __device__ inline int64_t sell_index(int64_t base, int C, int lane, int64_t k) {
  return base + (k >> 2) * (4 * static_cast<int64_t>(C)) + lane * 4 + (k & 3);
}
// Transpose a device CSR (sorted output).
void csr_transpose(const Csr& a, Csr* out, hipStream_t s);
// Sort device COO triples by (row, col) into a CSR; consumes nothing.
void coo_to_csr(int64_t nrows, int64_t nnz, const int32_t* row, const int32_t* col,
                const double* val, Csr* out, hipStream_t s);

}  // namespace wdb

// Operator handle.
struct wdb_theta {
  int device = 0;
  int32_t n = 0, levels = 0, wavelet = 0;
  int64_t N = 0, nnz = 0;
  double threshold = 0.0;
  int conv_build = 0;  // 1 when built by the convolution fast path
  int rule = 0;        // thresholding rule of the build (wdb_threshold_rule)
  wdb::Csr csr;        // Theta_K, float64 values (export)
  wdb::Sell A;         // Theta_K   (rows = output coefficient)
  wdb::Sell At;        // Theta_K^T (rows = input coefficient)
  wdb::Csr32 cA, cAt;  // float32 CSR of Theta_K and Theta_K^T
  int spmv_group = -1; // iteration kernels: 0 sliced ELL, G > 0 vector CSR with G lanes per row,
                       // -1 not chosen yet (process default)
  // 16-bit iteration values (same slots as A / At) and per-row dequantisation
  // factors (a power of two per row subband); valtype 0 = float32 iteration.
  int valtype = 0;
  uint16_t* val16 = nullptr;
  uint16_t* val16T = nullptr;
  float* wrow = nullptr;
  wdb::Packed pA, pAt;  // packed 16-bit forms (CSR order), when valtype != 0
  wdb::Stencil st, stT; // circulant storage of Theta_K and Theta_K^T (convolution fast path only)
  wdb::Tiled tA, tAt;   // tiled pattern storage of Theta_K and Theta_K^T (built on demand)
  int tile_waves = 4;   // wavefronts per tile of the tiled kernels
  int tile_unroll = 2;  // groups of 4 codes in flight per wavefront
  int tile_kept = 0;    // float32 tiles read: 1 the kept-value layout, 0 the dense values
  wdb::Tiled qA, qAt;   // the same with 16-bit values (built on demand when valtype != 0)
  int tile_waves16 = 4;
  int tile_unroll16 = 1;  // groups of 8 codes in flight per wavefront
  std::vector<float> qscale;  // host copy of the per-subband scales of the 16-bit values
  int q_group = 0;      // lanes per row of the packed kernels (0: default)
  bool has_L = false;
  double L = 0.0;
  int precond = 0;
  double Lp = 0.0;
  double* p64 = nullptr;    // device, N: diagonal P
  float* pinv = nullptr;    // device, N: 1/P as float32
  int l1_kind = 0;          // l1 weights: 0 uniform, 1 scale index j(i), 2 caller's
  float* l1w = nullptr;     // device, N: w (null when uniform)
  float* l1w_pre = nullptr; // device, N: w / P (null when uniform or no P)
  // Solver workspace (allocated on first solve).
  float* ws_x0 = nullptr;
  float* ws_r = nullptr;
  float* ws_y = nullptr;
  double* ws_r64 = nullptr;
  double* ws_a64 = nullptr;      // float64 anchor of the iterate (x = anchor + float32 displacement)
  float* ws_c = nullptr;         // x0 - Theta_K anchor (right-hand side of the displacement iteration)
  double* ws_v64 = nullptr;
  double* ws_partial = nullptr;  // per-block partial reductions (4 per block)
  double* ws_scalar = nullptr;   // device scalars
  double* host_scalar = nullptr; // pinned host mirror
  float* ws_img = nullptr;       // n*n scratch for transforms
  float* ws_img2 = nullptr;
  int* ws_k = nullptr;           // device iteration counter
  double* ws_checks = nullptr;   // device, 4 scalars per recorded check of a solve without a stopping test
  int64_t ws_ncheck = 0;
  double* ws_rho = nullptr;      // power-iteration history (64 entries)
  int64_t ws_nblocks = 0;
  hipStream_t capture_stream = nullptr;
  hipEvent_t check_event = nullptr;  // marks a check's scalars on the host while the next block runs
  // Instantiated graph of `g_c` iterations of the last graph-replayed solve and
  // the parameters it was captured with; dropped by every call that changes the
  // handle (layout, precision, preconditioner, weights, L), so a replay only
  // ever sees the storage it was captured on.
  hipGraph_t g_graph = nullptr;
  hipGraphExec_t g_exec = nullptr;
  const float* g_x = nullptr;
  int g_c = 0, g_pre = 0, g_ista = 0, g_anchor = 0;
  float g_tau = 0.0f, g_thr = 0.0f;
};

namespace wdb {
void ensure_workspace(wdb_theta* th);
void drop_graph(wdb_theta* th);  // destroys the cached iteration graph (if any)
void free_workspace(wdb_theta* th);
void finish_theta(wdb_theta* th, hipStream_t s);   // builds A/At from csr
void set_slice_height(wdb_theta* th, int C, hipStream_t s);  // rebuilds A/At with slices of C rows
// Packed 16-bit forms: build from cA / cAt with per-subband scales ub (device,
// canonical subband order) and value format fmt; launchers of the packed
// residual (Theta_K) and proximal (Theta_K^T) kernels with G lanes per row.
bool packed_supported(const wdb_theta* th);
void build_packed(wdb_theta* th, const float* ub, int fmt, hipStream_t s);
int packed_group(const wdb_theta* th);
void launch_res_packed(const wdb_theta* th, int G, const float* y, const float* b, float* r, int* kdev,
                       int scale_out, hipStream_t s);
void launch_prox_packed(const wdb_theta* th, int G, const float* rs, float* x, float* y, float tau, float thr,
                        const int* kdev, const float* pinv, const float* tw, hipStream_t s);
void build_stencils(wdb_theta* th, const std::vector<CircGen>& gens, const std::vector<int32_t>& tie_rows,
                    const std::vector<int32_t>& tie_cols, const std::vector<double>& tie_vals);
constexpr int kStencil = 1;  // kernel "group" value selecting the stencil kernels
constexpr int kTiled = 3;    // kernel "group" value selecting the tiled pattern kernels
bool tiled_supported(const wdb_theta* th);
void build_tiled(wdb_theta* th);    // builds tA / tAt from cA / cAt if not built yet
bool tiled_kept_available(const wdb_theta* th);  // both tiled copies hold the kept-value layout
void build_tiled16(wdb_theta* th);  // builds qA / qAt (16-bit values, scales qscale) if not built yet
// Float64 stopping-test products over the tiles: partials of ||r||^2, <r, x0>,
// sum w|x| at part[0..3 nb) and of max |g_i| / w_i at part[3 nb, 4 nb), one
// per tile (nb = tiled_check_blocks).
int64_t tiled_check_blocks(const wdb_theta* th);
void launch_objective_tiled(const wdb_theta* th, const float* x, const float* x0, double* r64, double* part,
                            int64_t nb, hipStream_t s, float* cneg = nullptr);
void launch_objective_tiled(const wdb_theta* th, const double* x, const float* x0, double* r64, double* part,
                            int64_t nb, hipStream_t s, float* cneg = nullptr);
void launch_res_tiled16(const wdb_theta* th, const float* y, const float* b, float* r, int* kdev, int scale_out,
                        hipStream_t s);
void launch_prox_tiled16(const wdb_theta* th, const float* rs, float* x, float* y, float tau, float thr,
                         const int* kdev, const float* pinv, const float* tw, hipStream_t s);
void launch_res_tiled(const wdb_theta* th, bool transpose, const float* y, const float* b, float* r, int* kdev,
                      hipStream_t s);
void launch_prox_tiled(const wdb_theta* th, const float* r, float* x, float* y, float tau, float thr, float beta,
                       const int* kdev, const float* pinv, const float* tw, const double* anc, hipStream_t s);
void launch_res_stencil(const wdb_theta* th, bool transpose, const float* y, const float* b, float* r, int* kdev,
                        hipStream_t s);
void launch_prox_stencil(const wdb_theta* th, const float* r, float* x, float* y, float tau, float thr, float beta,
                         const int* kdev, const float* pinv, const float* tw, const double* anc, hipStream_t s);

// Per-row threshold multipliers of the proximal step: w (l1 weights) or w / P
// (with the preconditioner), or null for uniform weights.
const float* threshold_weights(const wdb_theta* th, bool pre);
// Recompute w / P after the weights or the preconditioner changed.
void refresh_threshold_weights(wdb_theta* th);
int default_slice_height();
int kernel_group(const wdb_theta* th);  // lanes per row in use (0: sliced ELL)
// Lanczos on D A^T A D (d = nullptr: identity), float64, full
// reorthogonalisation within a cycle: the largest Ritz value theta, the residual bound
// resid = beta_m |s_m| of its Ritz pair (some eigenvalue lies within resid of
// theta), the steps taken, and whether resid <= tol * theta was met.
struct LanczosResult {
  double theta, resid;
  int steps;
  bool converged;
};
// Restarted every `cycle` steps from the top Ritz vector (the basis then
// holds cycle + 1 vectors of N doubles).
LanczosResult lanczos_max(wdb_theta* th, const double* start_host, const double* dinv_sqrt, double tol, int max_steps,
                          hipStream_t s, int cycle = 48);
// The same for any symmetric positive semidefinite M of size N given by
// apply(v, u): u = M v (device float64 vectors; the basis vector v must not be
// written).
LanczosResult lanczos_core(int64_t N, const std::function<void(const double*, double*)>& apply,
                           const double* start_host, double tol, int max_steps, hipStream_t s, int cycle = 48);
// Power iteration on D^-1/2 A^T A D^-1/2 (d = nullptr: identity), float64.
double power_iteration(wdb_theta* th, const double* start_host, const double* dinv_sqrt,
                       double tol, int max_iters, int* iters_out, hipStream_t s, bool* converged_out = nullptr);
// Forward/inverse float32 transform on device (scratch of n*n/4 * 2 floats).
void dwt_forward(int n, int levels, const Filter& f, const float* in, float* out,
                 float* scratch_a, float* scratch_b, hipStream_t s);
void dwt_inverse(int n, int levels, const Filter& f, const float* in, float* out,
                 float* scratch_a, float* scratch_b, hipStream_t s);
// The same for `count` images, up to 8 per launch (one launch per level and
// group of 8); scratch_a[i], scratch_b[i]: n*n/4 floats each for image i, and
// images in one group of 8 must not share scratch.
void dwt_forward_many(int n, int levels, const Filter& f, int count, const float* const* in, float* const* out,
                      float* const* scratch_a, float* const* scratch_b, hipStream_t s);
void dwt_inverse_many(int n, int levels, const Filter& f, int count, const float* const* in, float* const* out,
                      float* const* scratch_a, float* const* scratch_b, hipStream_t s);
}  // namespace wdb
