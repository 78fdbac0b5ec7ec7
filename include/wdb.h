/*
 * wdb — wavelet-domain l1-l2 deblurring on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the hot path of Escande & Weiss, "Real-time l1-l2 deblurring
 * using wavelet expansions of operators".  The method solves
 *
 *     min_x  1/2 || Theta_K x - Psi^* u ||_2^2 + lambda || x ||_1        (Sec. 1.3)
 *
 * where Theta = Psi^* H Psi is the blur H written in an orthogonal wavelet
 * basis (Sec. 3.4) and Theta_K keeps its K largest-magnitude entries
 * (Sec. 3.7), by the accelerated proximal gradient of Alg. 1 (Alg. 2 with a
 * diagonal preconditioner, Sec. 4).  The deblurred image is Psi x.
 *
 * Conventions
 *  - Images are n x n, n a power of two, row-major (index row * n + col),
 *    float32, on the torus (circular boundaries, Sec. 2).
 *  - Wavelet coefficient vectors have N = n*n float32 entries in this
 *    order: the coarsest approximation A_J, then for level l = J..1 the three
 *    detail subbands e = (0,1), (1,0), (1,1) (e_row, e_col: 1 = high-pass
 *    along that axis), each row-major with side n / 2^l.  Level l = 1 is
 *    the finest; the paper's scale index is j = log2(n) - l.
 *  - Theta[a, b] = <psi_a, H psi_b>: row a is the output coefficient, column
 *    b the input coefficient, so (Theta x)_a = sum_b Theta[a,b] x_b.
 *  - The blur is H[i, s] = k_s(i - s): column s is the point spread function
 *    of source pixel s (Sec. 3.1, kernel K(., y) is the PSF at y).  Each k_s
 *    is a Gaussian with axes sig_major, sig_minor, the major axis turned by
 *    `angle` from the column (x) axis toward the row (y) axis, cut where the
 *    Mahalanobis distance exceeds `trunc`, normalised to unit sum.
 *  - Pointers documented "device" must be HIP device memory of the current
 *    device (e.g. from torch tensors); "host" pointers are ordinary memory.
 *    The caller owns every buffer it passes; handles are owned by the
 *    library until freed with wdb_theta_free.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Work is ordered on that stream; calls return once their work is queued
 *    unless documented to synchronise.
 *  - Every call returns a wdb_status; on failure it is negative, outputs are
 *    left untouched where possible, and wdb_last_error() describes it.
 *  - One handle must not be used by two calls at the same time.
 */
#ifndef WDB_H
#define WDB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WDB_OK = 0,
  WDB_ERR_ARG = -1,          /* null pointer or invalid enum/parameter       */
  WDB_ERR_SIZE = -2,         /* n not a power of two, PSF wider than image   */
  WDB_ERR_LEVELS = -3,       /* too many levels for n and the filter length  */
  WDB_ERR_NONFINITE = -4,    /* NaN/Inf in an input                           */
  WDB_ERR_OOM = -5,          /* device or host allocation failed             */
  WDB_ERR_HIP = -6,          /* a HIP runtime call failed                    */
  WDB_ERR_DIVERGED = -7,     /* non-finite objective during a solve          */
  WDB_ERR_NOT_CONVERGED = -8,/* tolerance not met within max_iters           */
  WDB_ERR_FORMAT = -9        /* malformed sparse input                       */
} wdb_status;

typedef enum {
  WDB_HAAR = 0,   /* Haar, 2 taps                                      */
  WDB_DB4 = 1,    /* Daubechies, 4 vanishing moments, 8 taps (Sec. 3.5) */
  WDB_SYM6 = 2    /* Symmlet, 6 vanishing moments, 12 taps: the least-asymmetric
                     factor of the Daubechies response (the wavelet of Sec. 5) */
} wdb_wavelet;

/* Spatially varying Gaussian PSF field (Sec. 3.1).  Host arrays of n*n
 * doubles indexed by SOURCE pixel (row * n + col).  Requirements: every
 * sigma > 0 and finite, trunc > 0, and 2 * floor(trunc * max sig_major) + 1
 * <= n (a PSF may not wrap onto itself). */
typedef struct {
  int32_t n;
  const double* sig_major;
  const double* sig_minor;
  const double* angle;
  double trunc;
} wdb_psf_field;

typedef struct wdb_theta wdb_theta;   /* opaque operator handle */

/* Storage of Theta_K's values for the iteration (not in the paper, which
 * states no GPU precision): float32, or 16 bits with per-block power-of-two
 * scales and float32 accumulation. */
typedef enum {
  WDB_VAL_F32 = 0,
  WDB_VAL_BF16 = 1,
  WDB_VAL_F16 = 2
} wdb_valtype;

/* Description of an operator handle. */
typedef struct {
  int32_t n;           /* image side                                   */
  int32_t levels;      /* decomposition levels J                        */
  int32_t wavelet;     /* wdb_wavelet                                   */
  int32_t has_lipschitz;
  int64_t nnz;         /* K, kept entries                               */
  int64_t stored;      /* stored slots per copy including padding       */
  double lipschitz;    /* L = ||Theta_K||_2^2 (valid if has_lipschitz)  */
  double threshold;    /* smallest kept |Theta| (0 for imported)        */
  double lipschitz_p;  /* lambda_max(P^-1/2 Theta_K^T Theta_K P^-1/2)    */
  int32_t precond;     /* 0 none, else the wdb_precond kind in use      */
  int32_t valtype;     /* wdb_valtype of the iteration values            */
  int32_t slice;       /* sliced-ELL slice height of the iteration copies */
  int32_t group;       /* lanes per row of the vector-CSR kernels (0: sliced ELL; 1: circulant,
                          3: tiled pattern storage) */
  int32_t group16;     /* lanes per row of the packed 16-bit kernels (0: not in use; 3: 16-bit
                          tiled pattern storage) */
  int64_t escapes;     /* entries of Theta_K and Theta_K^T outside the packed column code */
  int32_t conv_build;  /* 1 if wdb_build_theta took the convolution fast path */
  int32_t l1_weights;  /* wdb_l1_weights kind in use */
  int32_t rule;        /* wdb_threshold_rule of the build (threshold is then the ranked value) */
  int64_t circulant;   /* -1: no circulant storage; else the explicit entries beside it (the
                          part of the cut's tie group that breaks the circulant pattern) */
  int32_t tile_waves;  /* wavefronts per tile of the tiled layout (group 3) */
  int64_t tile_slots;  /* stored values of the tiled copies of Theta_K and Theta_K^T (0: not built) */
  int32_t tile_waves16; /* wavefronts per tile of the 16-bit tiled layout (group16 3) */
  int32_t tile_unroll;  /* groups of 4 codes in flight per wavefront, tiled layout */
  int32_t tile_unroll16; /* groups of 8 codes in flight per wavefront, 16-bit tiled layout */
  int64_t tile_escapes; /* entries of the tiled copies kept in per-row escape lists */
  int32_t tile_kept;    /* 1: the float32 tiled kernels read the kept-value layout, 0: the dense values */
  int32_t reserved;
  int64_t tile_kept_values; /* values stored by the kept-value layout of both tiled copies (0: not built) */
} wdb_theta_desc;

/* ---------------------------------------------------------------------------
 * Operator construction.
 * ------------------------------------------------------------------------- */

/* Theta = Psi^* H Psi (Sec. 3.4) for the PSF field, thresholded to the
 * nnz_budget entries of largest magnitude (Sec. 3.7, naive rule; equal
 * magnitudes at the cut keep the smaller linear index a*N + b; fewer
 * non-zeros than the budget keeps them all).  Every entry is computed in
 * float64 from its definition <psi_a, H psi_b> on the GPU; the kept values
 * are stored as float32 for the solver and as float64 for export.
 * When every pixel carries the same PSF (H is a convolution) the build takes
 * the fast path of Alg. 3: the subband blocks of Theta are circulant (Sec.
 * 3.6), so only one column per subband (3J + 1 columns) is computed and the
 * kept entries are copied out of them; set the environment variable
 * WDB_BUILD_GENERAL=1 to force the general build.  The result is the same
 * Theta_K up to rounding of the values (and the order of near-equal
 * magnitudes at the cut).
 * `field` and its arrays are host memory, read during the call.
 * Synchronises `stream`.  Errors: WDB_ERR_ARG, _SIZE, _LEVELS, _NONFINITE,
 * _OOM, _HIP. */
wdb_status wdb_build_theta(const wdb_psf_field* field, int32_t wavelet, int32_t levels,
                           int64_t nnz_budget, void* stream, wdb_theta** out);

/* Thresholding rules of Sec. 3.7: WDB_THRESH_NAIVE keeps the K largest
 * |Theta[a, b]|; WDB_THRESH_SCALE keeps the K largest sigma_b |Theta[a, b]|
 * with sigma_b = 2^-k for a column b of scale k (the weights the paper
 * recommends; sigma weighs the input coefficient the operator acts on, which
 * is the closed form of the paper's minimax problem with the input measured
 * in the norm sum_b |x_b| / sigma_b).  Equal ranked values at the cut keep
 * the smaller a*N + b; the kept values are Theta's own.  wdb_build_theta is
 * this call with WDB_THRESH_NAIVE. */
typedef enum { WDB_THRESH_NAIVE = 0, WDB_THRESH_SCALE = 1 } wdb_threshold_rule;
wdb_status wdb_build_theta_rule(const wdb_psf_field* field, int32_t wavelet, int32_t levels,
                                int64_t nnz_budget, int32_t rule, void* stream, wdb_theta** out);

/* Operator from a host CSR matrix (N = n*n rows, strictly increasing column
 * indices within each row, values float64 rounded to float32 for the
 * solver).  rowptr has N+1 entries with rowptr[0] = 0, rowptr[N] = nnz.
 * Synchronises `stream`.  Errors: WDB_ERR_ARG, _SIZE, _LEVELS, _FORMAT,
 * _NONFINITE, _OOM, _HIP. */
wdb_status wdb_theta_import(int32_t n, int32_t wavelet, int32_t levels, int64_t nnz,
                            const int64_t* rowptr, const int32_t* col, const double* val,
                            void* stream, wdb_theta** out);

/* Copy the kept entries to host CSR arrays sized from wdb_theta_info
 * (rowptr: N+1, col/val: nnz).  val receives the float64 values (for a
 * built operator, the values before rounding to float32).  Any of the three
 * pointers may be NULL to skip it.  Synchronises. */
wdb_status wdb_theta_export(const wdb_theta* th, int64_t* rowptr, int32_t* col, double* val);

wdb_status wdb_theta_info(const wdb_theta* th, wdb_theta_desc* out);

/* L = lambda_max(Theta_K^T Theta_K) = ||Theta_K||_2^2, the step 1/L of
 * Alg. 1, by power iteration in float64 on the float32-stored operator:
 * v_0 = start/||start||; w = Theta_K v, rho_k = ||w||^2, v = Theta_K^T w /
 * ||Theta_K^T w||; stops at the first k >= 2 with |rho_k - rho_{k-1}| <=
 * tol * rho_k, or at max_iters.  `start` is a host array of N doubles (NULL:
 * a fixed SplitMix64-derived vector).  Stores L in the handle and returns it.
 * When max_iters is reached without meeting tol the call returns
 * WDB_ERR_NOT_CONVERGED, still storing and returning the last quotient (a
 * lower bound of ||Theta_K||^2: a step 1/L from it may be too long; prefer
 * wdb_theta_lipschitz_lanczos).  Synchronises. */
wdb_status wdb_theta_lipschitz(wdb_theta* th, const double* start, double tol,
                               int32_t max_iters, double* L_out, int32_t* iters_out);

/* The same constant by restarted Lanczos in float64 (the solver's default
 * when a handle has no L): cycles of up to 48 steps on Theta_K^T Theta_K
 * from v_0 = start/||start|| (NULL: as above), each step one product pair
 * and two passes of Gram-Schmidt against the cycle's basis; after each step
 * the largest eigenvalue theta of the tridiagonal projection and the residual
 * bound resid = beta_m |s_m| of its Ritz pair (some eigenvalue of
 * Theta_K^T Theta_K lies within resid of theta); a cycle restarts from the
 * top Ritz vector.  Stops when resid <= tol * theta or after max_steps steps
 * in all.  Stores L = theta + resid in the handle (an upper bound of
 * lambda_max when the Ritz pair approximates the top eigenvector, which a
 * random start gives with probability one) and returns it in L_out, with the
 * steps taken and resid.  WDB_ERR_NOT_CONVERGED (outputs still written, L
 * stored) when max_steps ends the run first.  Device memory: 49 vectors of N
 * doubles for the basis.  Synchronises. */
wdb_status wdb_theta_lipschitz_lanczos(wdb_theta* th, const double* start, double tol, int32_t max_steps,
                                       double* L_out, int32_t* steps_out, double* resid_out);

/* Diagonal preconditioner P for Alg. 2 (Sec. 4), from M = Theta_K^T Theta_K:
 *   WDB_PRECOND_NONE      remove it;
 *   WDB_PRECOND_SPAI      P_ii = M^2_ii / M_ii (Sec. 4.3 lemma; 1 where M_ii = 0);
 *   WDB_PRECOND_SPAI_SCALE one value per scale (A_J its own group),
 *                         p_s = sum_s M^2_ii / sum_s M_ii, the minimiser of the
 *                         same Frobenius objective under that constraint;
 *   WDB_PRECOND_JACOBI    P = max(M_ii, eps) (Sec. 4.2).
 * Also computes L_P = lambda_max(P^-1/2 M P^-1/2) by the restarted Lanczos
 * of wdb_theta_lipschitz_lanczos (start as there; tol and max_iters are its
 * tolerance and step cap), storing theta + resid.  Synchronises. */
typedef enum {
  WDB_PRECOND_NONE = 0,
  WDB_PRECOND_SPAI = 1,
  WDB_PRECOND_SPAI_SCALE = 2,
  WDB_PRECOND_JACOBI = 3
} wdb_precond;
wdb_status wdb_set_precond(wdb_theta* th, int32_t kind, double eps, const double* start,
                           double tol, int32_t max_iters);

/* Mixed precision.  valtype = WDB_VAL_F16 / WDB_VAL_BF16 makes the solver's
 * iteration stream 16-bit copies of Theta_K's values (same slots and column
 * indices as the float32 copy), accumulating in float32; WDB_VAL_F32 goes back
 * to float32 values.  Rule: each value v (the float32-stored value) of a row in
 * subband A is stored as q = round16(v * u_A), u_A = 2^-floor(log2 m_A), m_A the
 * largest |v| among the rows of subband A (1 if none), rounding to nearest-even;
 * the iteration then uses q / u_A exactly.  The block scale of block (A, B) is
 * u_A for every column subband B.  The iteration reads a packed copy: one
 * 32-bit word per entry, q in the high half and a band-relative column code in
 * the low half (column level minus row level in [-3, 3], orientation, and the
 * 2-D displacement in [-16, 15]^2 from the point of that level nearest to the
 * row's atom, modulo the subband side), so 4 bytes per entry; entries outside
 * the code (counted in wdb_theta_desc.escapes) are read from a per-row list
 * with int32 columns.  The columns decode exactly, so the product is that of
 * the dequantised matrix.  The float64 objective and duality-gap checks keep
 * using the float32 values, so they score iterates against the unquantised
 * Theta_K.  Synchronises.  Errors: WDB_ERR_ARG, _OOM, _HIP. */
wdb_status wdb_set_precision(wdb_theta* th, int32_t valtype);

/* Weights w of the l1 term, G(x) = sum_i w[i] |x[i]| (Sec. 1.3), used by the
 * single-problem solver (proximal threshold tau lambda w_i / P_i) and by its
 * float64 checks (E = 1/2 ||r||^2 + lambda sum_i w_i |x_i|; the dual point is
 * scaled by s = min(1, lambda / max_i |(Theta_K^T r)_i| / w_i)).
 * kind WDB_L1_UNIFORM: w = 1 (default); WDB_L1_SCALE: w[i] = j(i), the scale
 * of coefficient i (log2 n - level; the weights of the experiments of Sec. 5);
 * WDB_L1_GIVEN: w = the N floats at `w` (host, finite, > 0).  The batched
 * solver refuses handles with non-uniform weights.  Synchronises.  Errors:
 * WDB_ERR_ARG, _NONFINITE, _OOM, _HIP. */
typedef enum { WDB_L1_UNIFORM = 0, WDB_L1_SCALE = 1, WDB_L1_GIVEN = 2 } wdb_l1_weights;
wdb_status wdb_set_l1_weights(wdb_theta* th, int32_t kind, const float* w);

/* Lanes per row of the packed 16-bit kernels: 2, 4, 8 or 16, or 0 for the
 * default (4, or the environment variable WDB_Q_GROUP, where 0 selects the
 * slot-layout 16-bit kernels).  Changes only the summation order.  Errors:
 * WDB_ERR_ARG. */
wdb_status wdb_set_packed_group(wdb_theta* th, int32_t group);

/* Kernel layout of the iteration: sliced ELL with `slice` rows per slice
 * (8, 16, 32 or 64; rows in coefficient order) and group = 0, vector CSR
 * with `group` lanes per row (2..64), group = 1: the circulant storage of
 * a convolution build (Alg. 3 fast path; per subband block one list of
 * offsets and values shared by all rows, no per-entry indices), or
 * group = 3: the tiled pattern storage (tiles of 64 coefficients of one
 * subband -- 8 x 8 positions, or a whole subband of side < 8 -- share one
 * sorted list of band-relative column codes; one wavefront per tile, lane =
 * row; built on first use).  The float32 tiles hold two value layouts: dense
 * (values stored per code and row with zeros where a row lacks the entry,
 * about 1.6 x K values per matrix for the smoothly varying fields of Sec. 5)
 * and kept (only the kept values, with a 64-bit row mask per code;
 * wdb_set_tile_values).  The float64 checks and the power
 * iteration use vector CSR under layouts 1 and 3, else the same choice; the
 * batched solver runs an operator's packs on its tiled copies under layout 3
 * and on the sliced-ELL copies otherwise; the 16-bit iteration reads its
 * packed copy or its 16-bit tiles (wdb_set_precision).  Synchronises.
 * Errors: WDB_ERR_ARG, _OOM, _HIP. */
wdb_status wdb_set_kernel_layout(wdb_theta* th, int32_t slice, int32_t group);

/* Shape of the tiled kernels of the current value type (float32: layout 3;
 * 16-bit: packed group 3): `waves` wavefronts per tile (1, 2, 4 or 8) share
 * the tile's code groups round-robin and add their partial sums in
 * wavefront order; each wavefront keeps `unroll` groups (1, 2 or 4; 0 = the
 * default, 2 for float32 and 1 for 16-bit values) of loads in flight.
 * Changes only the summation order.  Errors: WDB_ERR_ARG. */
wdb_status wdb_set_tile_shape(wdb_theta* th, int32_t waves, int32_t unroll);

/* Value layout the float32 tiled kernels read (iteration, float64 checks and
 * the batched solver): kept = 0 the dense values (per group of 4 codes, 4
 * values for each of the tile's 64 rows, zeros where a row lacks a code);
 * kept = 1 only the kept values, lane by lane in code order, with a record
 * per group of 4 codes holding the codes, a 64-bit row mask per code and the
 * offset of the group's values (a lane's values start at that offset plus
 * the kept entries of the rows below it).  Same products, same summation
 * order; the kept layout streams fewer bytes and spends more instructions per
 * group.  Both layouts are built with the tiles (the kept one when its
 * values fit in 2 GiB, the reach of its 32-bit offsets); the autotuner also
 * picks between them.  Errors: WDB_ERR_ARG (kept not 0 or 1, or kept = 1 on
 * tiles built without the kept layout). */
wdb_status wdb_set_tile_values(wdb_theta* th, int32_t kept);

/* Project autotuner: times the iteration kernel pair `reps` times (two
 * alternating passes, the better pass counted) for every candidate layout on
 * this operator -- sliced ELL with 64/32/16/8 rows per slice; vector CSR with
 * 2/4/8/16 lanes per row; the circulant storage when the operator came from
 * the convolution fast path; the tiled pattern storage with dense or kept
 * values, 1/2/4/8 wavefronts per tile and 1/2/4 code groups in flight -- and
 * keeps the first
 * candidate in that order within 2% of the fastest.  With 16-bit values set
 * it instead picks among the packed kernels (2/4/8/16 lanes per row) and the
 * 16-bit tiles (1/2/4/8 wavefronts, 1/2 groups in flight).  If cache_path is not NULL the
 * decision is looked up in / appended to that text file, keyed by the
 * operator's shape and a hash of its row pointer.  Outputs (optional): the
 * chosen slice height and lanes per row, and the time of one iteration pair in
 * microseconds.  Synchronises. */
wdb_status wdb_autotune(wdb_theta* th, const char* cache_path, int32_t reps, int32_t* slice_out,
                        int32_t* group_out, double* us_out);

/* Copy the diagonal P (N doubles, host) of the active preconditioner. */
wdb_status wdb_get_precond(const wdb_theta* th, double* p_out);

void wdb_theta_free(wdb_theta* th);

/* ---------------------------------------------------------------------------
 * Solver (Alg. 1 / Alg. 2).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t max_iters;     /* iterations to run (upper bound when tol > 0)           */
  int32_t check_every;   /* float64 objective + duality gap every c iterations;
                            0 = only once after the last iteration               */
  double tol_rel_gap;    /* stop at the first check with gap/E <= tol (0: never)  */
  const float* x_init;   /* device, N coefficients, or NULL for x = 0             */
  int32_t k0;            /* index of the first iteration (>= 1; resume), 0 = 1     */
  int32_t use_precond;   /* 1: Alg. 2 with the handle's preconditioner            */
  void* stream;
  double* trace;         /* host, optional: (k, E, rel_gap) per check             */
  int32_t trace_cap;     /* number of triples `trace` can hold                    */
  int32_t use_graph;     /* 1: replay the iterations between checks as a HIP graph */
  double target_objective; /* > 0: also stop at the first check with E <= target     */
  int32_t ista;          /* 1: no extrapolation, x_k = prox(x_{k-1} - tau grad) (ISTA, the
                            un-accelerated baseline of the paper's comparison)     */
  int32_t plain_iterate; /* 0 (default): with float32 values the iterate is held as a
                            float64 anchor plus a float32 displacement, moved into the
                            anchor at every check, so the float64 stopping test can
                            certify gaps far below what a float32 iterate's rounding
                            allows (one extra 8-byte read per coefficient and
                            iteration); 1: float32 iterate only.  16-bit values
                            always use the float32 iterate; the batched solver
                            always anchors.                                       */
  double* x64_out;       /* device, N doubles, or NULL: receives the float64 iterate the
                            last check scored (the anchor; x_out is its float32
                            rounding, whose own gap can be larger); with a plain
                            float32 iterate, x_out widened to float64             */
} wdb_solve_opts;

typedef struct {
  int32_t iters;         /* iterations run                                         */
  int32_t checks;        /* float64 checks done                                     */
  double objective;      /* E(x) = 1/2||Theta_K x - x0||^2 + lambda||x||_1 (float64) */
  double rel_gap;        /* duality gap / E at the last check                       */
  double lipschitz;      /* L (or L_P) used                                         */
  double tau;            /* step 1/L                                                */
} wdb_solve_info;

/* Stopping: with tol_rel_gap > 0 or target_objective > 0 the solve ends at the
 * first check meeting either; WDB_ERR_NOT_CONVERGED if neither was met within
 * max_iters (x_out is still written). */

/* Solve from a blurred image: x0 = Psi^* u (forward transform on the GPU),
 * then FISTA iterations from x_init, x_out receives x^(k).  u: device n*n
 * image; x_out: device N coefficients.  Computes L on first use if the
 * handle has none (default start).  Every iteration is one fused
 * r = Theta_K y - x0 kernel and one fused Theta_K^T r + soft-threshold +
 * momentum kernel; the float64 check adds one product pair per check.
 * Synchronises at each check.  Errors: WDB_ERR_ARG, _NONFINITE (lambda),
 * _DIVERGED, _NOT_CONVERGED (tol > 0 not reached; x_out still written), _HIP. */
wdb_status wdb_solve(wdb_theta* th, const float* u, float lambda, const wdb_solve_opts* opts,
                     float* x_out, wdb_solve_info* info);

/* Same as wdb_solve with the wavelet-domain data x0 (device, N) given directly. */
wdb_status wdb_solve_coeffs(wdb_theta* th, const float* x0, float lambda,
                            const wdb_solve_opts* opts, float* x_out, wdb_solve_info* info);

/* One problem of a batched solve. */
typedef struct {
  wdb_theta* theta;      /* operator; problems may share one                 */
  const float* u;        /* device, n*n blurred image; may be NULL when x0 is set */
  float lambda;
  const float* x_init;   /* device, N coefficients, or NULL for x = 0         */
  float* x_out;          /* device, N coefficients (written at the end)      */
  double target_objective; /* > 0: this problem stops at the first check with E <= target */
  const float* x0;       /* device, N coefficients Psi^* u given directly (u is then
                            not read), or NULL to transform u on the device   */
  double* x64_out;       /* device, N doubles, or NULL: the float64 iterate the
                            problem's last check scored (x_out is its float32
                            rounding)                                         */
} wdb_problem;

/* Solve many problems in one call (Alg. 1 for each).  Problems sharing a
 * handle are packed up to eight at a time so each iteration reads every
 * stored entry of Theta_K once for all right-hand sides of a pack; all packs
 * of all operators run in one launch per phase (two launches per iteration
 * for the whole batch), replayed from a HIP graph between float64 checks
 * when opts->use_graph is set.  opts is shared (its x_init must be NULL; use
 * the per-problem x_init), each problem has its own lambda, step 1/L of its
 * handle (computed on first use if absent), and its own stop flag: with
 * tol_rel_gap > 0 a problem stops updating at the first check where its gap
 * is below tolerance (or, with its target_objective > 0, where E <= target).
 * A pack whose remaining problems fit in fewer slots continues on a narrower
 * layout; this changes the cost per iteration, not the iterates.  infos
 * (optional) receives nprob entries.  Handles must hold float32 values.
 * Allocates its working vectors (room for eight slots per pack) for the call
 * and synchronises at each check.  Errors: as wdb_solve;
 * WDB_ERR_NOT_CONVERGED if any problem missed the tolerance (all outputs are
 * still written). */
wdb_status wdb_solve_batched(int32_t nprob, const wdb_problem* probs, const wdb_solve_opts* opts,
                             wdb_solve_info* infos);

/* Float64 objective E(x) and relative duality gap for coefficients x and data
 * x0 (device arrays of N float32).  With r = Theta_K x - x0,
 * s = min(1, lambda / ||Theta_K^T r||_inf): D = -s^2||r||^2/2 - s<r, x0>,
 * gap = E - D.  Synchronises `stream`. */
wdb_status wdb_objective(wdb_theta* th, const float* x, const float* x0, float lambda,
                         void* stream, double* E_out, double* rel_gap_out);

/* y = Theta_K x - b (transpose = 0) or y = Theta_K^T x - b (transpose = 1),
 * float32, one kernel launch per repetition (repeat >= 1 launches the same
 * product `repeat` times, for timing).  b may be NULL (treated as 0).
 * x, b, y: device, N floats; y must not alias x. */
wdb_status wdb_theta_apply(wdb_theta* th, int32_t transpose, const float* x, const float* b,
                           float* y, int32_t repeat, void* stream);

/* With 16-bit values set (wdb_set_precision), transpose = 0 uses them
 * (y = Theta~_K x - b with the dequantised values); transpose = 1 is refused
 * (WDB_ERR_ARG) in that mode. */

/* One fused proximal-gradient step (Alg. 1, steps 3-4) given the residual r
 * (float32 values only: WDB_ERR_ARG when 16-bit values are set):
 * g = Theta_K^T r; z = y - tau * g / P; x_new = S_{tau*lambda/P}(z);
 * y = x_new + beta (x_new - x); x = x_new  (P = 1 unless use_precond). */
wdb_status wdb_prox_step(wdb_theta* th, const float* r, float* x, float* y, float tau,
                         float lambda, float beta, int32_t use_precond, void* stream);

/* ---------------------------------------------------------------------------
 * Transforms.
 * ------------------------------------------------------------------------- */

/* Psi x: inverse transform of N coefficients to an n x n image (Sec. 2). */
wdb_status wdb_synthesize(const wdb_theta* th, const float* x, float* u_hat, void* stream);

/* Forward (inverse = 0: out = Psi^* in) or inverse (inverse = 1: out = Psi in)
 * periodic orthogonal 2D transform with `levels` levels; in/out: device, n*n
 * floats, must not alias.  Errors: WDB_ERR_ARG, _SIZE, _LEVELS, _HIP. */
wdb_status wdb_dwt(int32_t n, int32_t wavelet, int32_t levels, const float* in, float* out,
                   int32_t inverse, void* stream);

/* The same transform for `count` images at once (Sec. 2, applied image by
 * image): in/out are device arrays of count * n * n floats, image i at i n^2,
 * and must not overlap.  Up to 8 images share each level's launch, so a
 * batch costs a few launches per level instead of one per image and level.
 * Results equal wdb_dwt's for each image, bit for bit.  Allocates 2 n^2 / 4
 * floats of scratch per image of a launch (at most 8) and synchronises
 * `stream` before returning.  Errors: as wdb_dwt, and WDB_ERR_ARG for
 * count < 1. */
wdb_status wdb_dwt_batched(int32_t n, int32_t wavelet, int32_t levels, int32_t count, const float* in,
                           float* out, int32_t inverse, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * transform as wdb_dwt, bit for bit, with its level-to-level intermediates
 * in a fixed device array of the library (8 MiB per GPU, held until the
 * process ends) instead of a per-call allocation.  n <= 2048 (WDB_ERR_SIZE
 * otherwise, before any GPU work).  No allocation, no synchronisation: the
 * work is only enqueued on `stream`.  Calls that overlap on one GPU share the
 * array and race; serialise them.  Errors: as wdb_dwt. */
wdb_status wdb_dwt_noalloc(int32_t n, int32_t wavelet, int32_t levels, const float* in, float* out,
                           int32_t inverse, void* stream);

/* out = H u for the PSF field (Sec. 3.1, column convention), float64
 * arithmetic, float32 storage; u, out: device n*n floats, must not alias.
 * Synchronises `stream` (uploads the field).  Errors: as wdb_build_theta. */
wdb_status wdb_blur(const wdb_psf_field* field, const float* u, float* out, void* stream);

/* ---------------------------------------------------------------------------
 * Exact-operator baseline (Sec. 1.2; the "Exact" columns of the experiments
 * of Sec. 5): Alg. 1 on the wavelet coefficients with the gradient of
 * 1/2 ||H Psi x - u0||^2 computed from the blur itself,
 * g = Psi^* H^* (H Psi y - u0), instead of from Theta_K.  Psi is orthogonal,
 * so this is the problem before thresholding (Theta = Psi^* H Psi, all of
 * it).  H and H^* evaluate the truncated PSFs of the field on the fly in
 * float64 (the formula and cut-off of wdb_blur), accumulating in float64;
 * images and coefficients are float32.  Device memory: about 40 N bytes.
 * ------------------------------------------------------------------------- */
typedef struct wdb_exact wdb_exact;

/* Handle for the PSF field (host arrays, read during the call) with the
 * given wavelet and levels.  Synchronises `stream`.  Errors: as
 * wdb_build_theta. */
wdb_status wdb_exact_create(const wdb_psf_field* field, int32_t wavelet, int32_t levels, void* stream,
                            wdb_exact** out);
/* out = H in (adjoint = 0) or H^* in (adjoint = 1) on n*n images (device
 * float32, must not alias); no synchronisation. */
wdb_status wdb_exact_apply(wdb_exact* ex, int32_t adjoint, const float* in, float* out, void* stream);
/* L = ||H||^2 (= ||Psi^* H Psi||^2) by the restarted Lanczos of
 * wdb_theta_lipschitz_lanczos on H^* H in float64; stores L = theta + resid.
 * WDB_ERR_NOT_CONVERGED (outputs written) when max_steps ends the run first. */
wdb_status wdb_exact_lipschitz(wdb_exact* ex, const double* start, double tol, int32_t max_steps, double* L_out,
                               int32_t* steps_out, double* resid_out);
/* Alg. 1 with the exact gradient from the blurred image u (device n*n) into
 * x_out (device N coefficients).  opts: max_iters, check_every (objective
 * E = 1/2 ||H Psi x - u0||^2 + lambda ||x||_1 and relative duality gap, from
 * float32 products with float64 sums, one gradient evaluation per check; the
 * float32 residual puts the gap's accuracy near 1e-3 relative at the
 * workloads' lambda, the objective's near 1e-7),
 * tol_rel_gap, target_objective, x_init, k0, ista, trace/trace_cap, stream;
 * use_precond is refused, use_graph and plain_iterate are ignored (float32
 * iterate, launches issued per iteration).  Computes L on first use.
 * Synchronises at each check.  Errors: as wdb_solve. */
wdb_status wdb_exact_solve(wdb_exact* ex, const float* u, float lambda, const wdb_solve_opts* opts, float* x_out,
                           wdb_solve_info* info);
void wdb_exact_free(wdb_exact* ex);

/* ---------------------------------------------------------------------------
 * Warm start (not in the paper): a small network on wavelet coefficients that
 * predicts an initial iterate from x0 = Psi^* u.  One stack per level (the
 * coarsest approximation, 1 channel; each detail level, its 3 subbands as
 * channels): h1 = relu(conv(z)), h2 = relu(conv(h1)), out = z + conv(h2), with
 * circular 3x3 convolutions, `features` hidden channels (32), bfloat16 compute
 * copies of the parameters, float32 accumulation and float32 master weights
 * updated by Adam (beta 0.9 / 0.999, eps 1e-8) on the mean squared error.
 * Batches are device arrays [batch][N] in the canonical coefficient layout.
 * Parameters are flattened stack by stack (A_J first, then levels J..1), each
 * as W1 [F][C][3][3], b1 [F], W2 [F][F][3][3], b2 [F], W3 [C][F][3][3], b3 [C].
 * The solver remains the judge: a prediction is only ever used as x_init.
 * ------------------------------------------------------------------------- */
typedef struct wdb_cnn wdb_cnn;

/* Network for n x n images with `levels` levels; weights He-normal from a
 * SplitMix64 stream seeded with `seed` (last convolution of each stack 10x
 * smaller), biases zero.  Errors: WDB_ERR_ARG, _SIZE, _LEVELS, _OOM, _HIP. */
wdb_status wdb_cnn_create(int32_t n, int32_t levels, int32_t features, uint64_t seed, wdb_cnn** out);
wdb_status wdb_cnn_param_count(const wdb_cnn* net, int64_t* count);
/* Set the float32 master parameters (host array of param_count floats);
 * resets the Adam state. */
wdb_status wdb_cnn_set_params(wdb_cnn* net, const float* host, int64_t count);
/* Copy the parameters to host: masters (rounded = 0) or the bfloat16 values
 * the kernels compute with (rounded = 1). */
wdb_status wdb_cnn_get_params(const wdb_cnn* net, float* host, int32_t rounded);
/* out = network(x0) for a batch (device arrays, must not alias). */
wdb_status wdb_cnn_predict(wdb_cnn* net, const float* x0, int32_t batch, float* out, void* stream);
/* Mean squared error against target and its gradient (float32, copied to
 * grad_host if not NULL).  Synchronises. */
wdb_status wdb_cnn_loss_grad(wdb_cnn* net, const float* x0, const float* target, int32_t batch, double* loss,
                             float* grad_host, void* stream);
/* One Adam step with learning rate lr on the batch; *loss gets the loss
 * before the step.  Synchronises (to return the loss). */
wdb_status wdb_cnn_train_step(wdb_cnn* net, const float* x0, const float* target, int32_t batch, float lr,
                              double* loss, void* stream);
void wdb_cnn_free(wdb_cnn* net);

/* ---------------------------------------------------------------------------
 * Misc.
 * ------------------------------------------------------------------------- */

/* Message for the last failed call on this thread ("" if none). */
const char* wdb_last_error(void);

/* Library version string. */
const char* wdb_version(void);

/* Low-pass analysis filter the library uses for `wavelet` (derived in
 * float64; Daubechies and Symmlet by spectral factorisation).  h_out is a
 * host array of `capacity` doubles (taps: 2 for Haar, 8 for db4, 12 for
 * sym6; 12 covers every wavelet); *len_out always receives the number of
 * taps.  h_out = NULL with capacity = 0 only queries the length.  Errors:
 * WDB_ERR_ARG for an unknown wavelet, a null len_out, or capacity below the
 * number of taps (h_out is then not written).  Host only: no device is
 * touched. */
wdb_status wdb_wavelet_filter(int32_t wavelet, double* h_out, int32_t capacity, int32_t* len_out);

#ifdef __cplusplus
}
#endif

#endif /* WDB_H */
