// Error reporting, version and handle-level entry points of the wdb C ABI.
#include <cstdlib>
#include <cstring>

#include "common.hpp"

namespace wdb {

namespace {
thread_local std::string g_last_error;
}

void fail(wdb_status code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Error{code, std::string(buf)};
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

int64_t sell_sort_window() {
  static const int64_t w = [] {
    const char* e = std::getenv("WDB_SELL_SORT");
    const long long v = e ? std::atoll(e) : 0;
    return static_cast<int64_t>(v < 0 ? 0 : v);
  }();
  return w;
}
void clear_last_error() { g_last_error.clear(); }

void Sell::free_all() {
  if (perm) (void)hipFree(perm);
  perm = nullptr;
  if (slice_off) (void)hipFree(slice_off);
  if (val) (void)hipFree(val);
  if (col) (void)hipFree(col);
  slice_off = nullptr;
  val = nullptr;
  col = nullptr;
  nrows = nslices = stored = 0;
}

void Csr32::free_all() {
  if (rowptr) (void)hipFree(rowptr);
  if (col) (void)hipFree(col);
  if (val) (void)hipFree(val);
  rowptr = nullptr;
  col = nullptr;
  val = nullptr;
  nrows = nnz = 0;
}

int spmv_group() {
  static const int g = [] {
    const char* e = std::getenv("WDB_SPMV_GROUP");
    const int v = e ? std::atoi(e) : 0;
    return (v == 2 || v == 4 || v == 8 || v == 16 || v == 32 || v == 64) ? v : 0;
  }();
  return g;
}

void Csr::free_all() {
  if (rowptr) (void)hipFree(rowptr);
  if (col) (void)hipFree(col);
  if (val) (void)hipFree(val);
  rowptr = nullptr;
  col = nullptr;
  val = nullptr;
  nrows = nnz = 0;
}

void free_workspace(wdb_theta* th) {
  drop_graph(th);
  float* fs[] = {th->ws_x0, th->ws_r, th->ws_y, th->ws_img, th->ws_img2, th->pinv, th->ws_c};
  for (float* p : fs)
    if (p) (void)hipFree(p);
  double* ds[] = {th->ws_r64, th->ws_v64, th->ws_partial, th->ws_scalar, th->p64, th->ws_checks, th->ws_a64};
  for (double* p : ds)
    if (p) (void)hipFree(p);
  if (th->host_scalar) (void)hipHostFree(th->host_scalar);
  if (th->ws_k) (void)hipFree(th->ws_k);
  if (th->ws_rho) (void)hipFree(th->ws_rho);
  if (th->capture_stream) (void)hipStreamDestroy(th->capture_stream);
  if (th->check_event) (void)hipEventDestroy(th->check_event);
  th->check_event = nullptr;
  th->ws_k = nullptr;
  th->ws_rho = nullptr;
  th->capture_stream = nullptr;
  th->ws_x0 = th->ws_r = th->ws_y = th->ws_img = th->ws_img2 = th->pinv = th->ws_c = nullptr;
  th->ws_r64 = th->ws_v64 = th->ws_partial = th->ws_scalar = th->p64 = th->ws_checks = th->ws_a64 = nullptr;
  th->ws_ncheck = 0;
  th->host_scalar = nullptr;
}

}  // namespace wdb

extern "C" {

const char* wdb_last_error(void) { return wdb::g_last_error.c_str(); }

const char* wdb_version(void) { return "wdb 0.1 (gfx950)"; }

wdb_status wdb_theta_info(const wdb_theta* th, wdb_theta_desc* out) {
  WDB_API_BEGIN
  WDB_REQUIRE(th && out, WDB_ERR_ARG, "null handle or output");
  std::memset(out, 0, sizeof(*out));
  out->n = th->n;
  out->levels = th->levels;
  out->wavelet = th->wavelet;
  out->has_lipschitz = th->has_L ? 1 : 0;
  out->nnz = th->nnz;
  out->stored = th->A.stored;
  out->lipschitz = th->L;
  out->threshold = th->threshold;
  out->lipschitz_p = th->Lp;
  out->precond = th->precond;
  out->valtype = th->valtype;
  out->slice = th->A.C;
  out->group = wdb::kernel_group(th);
  out->group16 = th->valtype != WDB_VAL_F32 && th->pA.word ? wdb::packed_group(th) : 0;
  out->escapes = th->pA.nesc + th->pAt.nesc;
  out->conv_build = th->conv_build;
  out->l1_weights = th->l1_kind;
  out->rule = th->rule;
  out->circulant = th->st.seg ? th->st.nextra : -1;
  out->tile_waves = th->tile_waves;
  out->tile_waves16 = th->tile_waves16;
  out->tile_unroll = th->tile_unroll;
  out->tile_unroll16 = th->tile_unroll16;
  out->tile_escapes = th->tA.nesc + th->tAt.nesc;
  out->tile_slots = 64 * (th->tA.npat + th->tAt.npat);
  out->tile_kept = th->tile_kept;
  out->tile_kept_values = th->tA.nkval + th->tAt.nkval;
  WDB_API_END
}

wdb_status wdb_theta_export(const wdb_theta* th, int64_t* rowptr, int32_t* col, double* val) {
  WDB_API_BEGIN
  WDB_REQUIRE(th, WDB_ERR_ARG, "null handle");
  WDB_HIP(hipSetDevice(th->device));
  WDB_HIP(hipDeviceSynchronize());
  if (rowptr)
    WDB_HIP(hipMemcpy(rowptr, th->csr.rowptr, (th->N + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (col && th->nnz)
    WDB_HIP(hipMemcpy(col, th->csr.col, th->nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (val && th->nnz)
    WDB_HIP(hipMemcpy(val, th->csr.val, th->nnz * sizeof(double), hipMemcpyDeviceToHost));
  WDB_API_END
}

void wdb_theta_free(wdb_theta* th) {
  if (!th) return;
  (void)hipSetDevice(th->device);
  (void)hipDeviceSynchronize();
  th->csr.free_all();
  th->A.free_all();
  th->At.free_all();
  th->cA.free_all();
  th->cAt.free_all();
  if (th->val16) (void)hipFree(th->val16);
  if (th->val16T) (void)hipFree(th->val16T);
  if (th->wrow) (void)hipFree(th->wrow);
  th->pA.free_all();
  th->pAt.free_all();
  th->st.free_all();
  th->stT.free_all();
  th->tA.free_all();
  th->tAt.free_all();
  th->qA.free_all();
  th->qAt.free_all();
  if (th->l1w) (void)hipFree(th->l1w);
  if (th->l1w_pre) (void)hipFree(th->l1w_pre);
  wdb::free_workspace(th);
  delete th;
}

}  // extern "C"
