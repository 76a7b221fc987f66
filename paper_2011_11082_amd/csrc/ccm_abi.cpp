// C ABI of the CCM hot path: argument checks, workspace layout and kernel launches.
// Every entry point is asynchronous on the caller's stream and never synchronises.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <string>

#include "../../include/ccm.h"

extern "C" {
hipError_t ccm_launch_knn(const float* ts, int64_t ld, int L, const int* lib_ids, const int* lib_E,
                          int n_lib, int tau, int Tp, int k_max, const uint8_t* cand_mask,
                          int* nbr_idx, float* nbr_w, float* nbr_d2, hipStream_t stream);
hipError_t ccm_launch_simplex(const float* ts, int64_t ld, int L, const int* ids, int n, int E_min,
                              int E_max, int tau, int Tp, int mode, int* optE, float* rho_E,
                              double* rho64, hipStream_t stream);
hipError_t ccm_launch_embed(const float* ts, int64_t ld, int L, const int* ids, int n, int E,
                            int tau, float* emb, hipStream_t stream);
size_t ccm_gather_lds_bytes(int L);
int ccm_gather_tile_in_lds(int L);
int ccm_gather_tile_targets(int L);
void ccm_gather_force_tile(int tj);
hipError_t ccm_launch_crossmap_fp32(const float* ts, int64_t ld, int L, int tau, int tgt0,
                                    int n_tgt, const int* nbr_idx, const float* nbr_w,
                                    const int* lib_E, int n_lib, int k_max, float* rho,
                                    double* moments, uint32_t* poff, float* pw, int* lib_k,
                                    int* order, float* gtile, double* gsum, hipStream_t stream);
int ccm_target_E_max_tiles(int n_tgt, int tj);
hipError_t ccm_launch_crossmap_fp32_target_E(
    const float* ts, int64_t ld, int L, int tau, int tgt0, int n_tgt, const int* nbr_idx,
    const float* nbr_w, int n_lib, int E_lo, int n_E, int k_max, const int* tgt_E, float* rho,
    double* moments, uint32_t* poff, float* pw, int* lib_k, int* table_E, int* perm, int* tiles,
    int* ntiles, float* gtile, double* gsum, hipStream_t stream);
size_t ccm_bf16_lds_bytes();
hipError_t ccm_launch_crossmap_bf16(const float* ts, int64_t ld, int L, int tau, int tgt0, int n_tgt,
                                    const int* nbr_idx, const float* nbr_w, const int* lib_E,
                                    int n_lib, int k_max, float* rho, double* moments, uint16_t* yt,
                                    float* cref, uint32_t* ent, int* stage_off, int* lib_k,
                                    int* order, hipStream_t stream);
size_t ccm_backward_ws_bytes(int L, int n_lib, int n_pairs, int k_max);
int ccm_noalloc_max_series();
hipError_t ccm_noalloc_scratch(double** out);
hipError_t ccm_launch_backward(const float* ts, int64_t ld, int L, const float* lib_ts,
                               const int* nbr_idx, const float* nbr_w, const int* lib_E, int n_lib,
                               int k_max, int tau, const int* pair_lib, const int* pair_tgt,
                               const float* grad_rho, int n_pairs, float* grad_ts, float* grad_lib,
                               void* ws, hipStream_t stream);
}

namespace {

thread_local std::string g_last_error;

ccm_status fail(ccm_status s, const char* fn, const char* msg) {
  g_last_error = std::string(fn) + ": " + msg;
  return s;
}

ccm_status device_status(const char* fn, hipError_t e) {
  if (e == hipSuccess) return CCM_OK;
  g_last_error = std::string(fn) + ": HIP error: " + hipGetErrorString(e);
  return CCM_EDEVICE;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace of the FP32 cross-map: blocked tables (byte offsets, weights), lib_k, order, and
// for series too long for the LDS tile a global copy of every target tile ([n_tiles][L][tj]
// floats, tj targets per tile) with its FP64 column sums ([n_tiles][2][21][tj]).
struct CrossmapWs {
  size_t off_poff, off_pw, off_libk, off_order, off_gtile, off_gsum, total;
};

CrossmapWs crossmap_ws(int L, int n_lib, int k_max, int n_tiles, int tj) {
  CrossmapWs w;
  const size_t KSM = (size_t)(k_max + 3) / 4;
  // tables blocked by RB = 64 / (tj / 4) query rows (4 entries per row and slot), with spare
  // blocks after the last library: the gather prefetches block b + 1 unguarded; sized for
  // every tile width
  size_t ent = 0;
  for (int w = 4; w <= 32; w *= 2) {
    const size_t rb = 64 / (size_t)(w / 4);
    const size_t e = ((size_t)n_lib * ((L + rb - 1) / rb) + 3) * KSM * 4 * rb;
    if (e > ent) ent = e;
  }
  w.off_poff = 0;
  w.off_pw = align_up(w.off_poff + ent * 4);
  w.off_libk = align_up(w.off_pw + ent * 4);
  w.off_order = align_up(w.off_libk + (size_t)n_lib * 4);
  w.off_gtile = align_up(w.off_order + (size_t)n_lib * 4);
  const bool global_tile = !ccm_gather_tile_in_lds(L);
  w.off_gsum = align_up(w.off_gtile + (global_tile ? (size_t)n_tiles * L * tj * 4 : 0));
  w.total = align_up(w.off_gsum + (global_tile ? (size_t)n_tiles * 2 * (CCM_E_MAX + 1) * tj * 8 : 0));
  return w;
}

// The library-E cross-map: 16-, 8- or 4-target tiles in LDS, or 32-target tiles from the
// global copy.
CrossmapWs fp32_ws(int L, int n_lib, int k_max, int n_tgt) {
  const int tj = ccm_gather_tile_targets(L);
  return crossmap_ws(L, n_lib, k_max, (n_tgt + tj - 1) / tj, tj);
}

// Workspace of the per-target-E cross-map: the FP32 workspace over n_tab = n_E * n_lib
// tables, their E, the targets sorted by E, the tile list and its length.
struct TargetEWs {
  CrossmapWs tab;
  size_t off_tabE, off_perm, off_tiles, off_ntiles, total;
};

TargetEWs target_E_ws(int L, int n_tab, int n_tgt, int k_max) {
  TargetEWs w;
  const int tj = ccm_gather_tile_targets(L);
  w.tab = crossmap_ws(L, n_tab, k_max, ccm_target_E_max_tiles(n_tgt, tj), tj);
  w.off_tabE = w.tab.total;
  w.off_perm = align_up(w.off_tabE + (size_t)n_tab * 4);
  w.off_tiles = align_up(w.off_perm + (size_t)n_tgt * 4);
  w.off_ntiles = align_up(w.off_tiles + (size_t)ccm_target_E_max_tiles(n_tgt, tj) * 3 * 4);
  w.total = align_up(w.off_ntiles + 4);
  return w;
}

// Workspace of the BF16 cross-map: BF16 target panel (target-major), the targets' centring
// values, table entries sorted by (stage, row quarter), their bucket offsets, lib_k, order.
struct Bf16Ws {
  size_t off_yt, off_cref, off_ent, off_so, off_libk, off_order, total;
};

Bf16Ws bf16_ws(int L, int n_lib, int n_tgt) {
  Bf16Ws w;
  const size_t nst = (size_t)(L + 63) / 64;
  const size_t nch = (size_t)(L + 127) / 128;
  w.off_yt = 0;
  w.off_cref = align_up(w.off_yt + (size_t)n_tgt * nst * 64 * 2);
  w.off_ent = align_up(w.off_cref + (size_t)n_tgt * 4);
  w.off_so = align_up(w.off_ent + (size_t)n_lib * nch * 128 * CCM_K_MAX * 4);
  w.off_libk = align_up(w.off_so + (size_t)n_lib * nch * (4 * nst + 1) * 4);
  w.off_order = align_up(w.off_libk + (size_t)n_lib * 4);
  w.total = align_up(w.off_order + (size_t)n_lib * 4);
  return w;
}

// ---- debug mode: finiteness of the inputs (off by default) ------------------------------
std::atomic<int> g_check_finite{0};

// Sets *bad when a value of the listed series (columns `cols`, or col0 .. col0 + n_cols - 1
// when cols is NULL; ids outside [0, ld) are skipped) is not finite.
__global__ void finite_cols_kernel(const float* ts, int64_t ld, int L, const int* cols, int col0,
                                   int n_cols, int* bad) {
  const int64_t total = (int64_t)L * n_cols;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int ci = (int)(g % n_cols);
    const int64_t t = g / n_cols;
    const int c = cols ? cols[ci] : col0 + ci;
    if (c >= 0 && c < ld && !isfinite(ts[t * ld + c])) *bad = 1;
  }
}

__global__ void finite_flat_kernel(const float* a, int64_t n, int* bad) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(a[g])) *bad = 1;
}

struct FiniteSpec {
  const float* ts = nullptr;   // series columns of the panel
  int64_t ld = 0;
  int L = 0;
  const int* cols = nullptr;
  int col0 = 0, n_cols = 0;
  const float* flat[3] = {nullptr, nullptr, nullptr};   // whole arrays
  int64_t flat_n[3] = {0, 0, 0};
};

unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// In debug mode, runs the checks on `stream`, waits for them and returns EINVAL if a value
// is not finite (CCM_OK otherwise, and at once when debug mode is off).
ccm_status check_finite(const char* fn, const FiniteSpec& f, hipStream_t stream) {
  if (!g_check_finite.load(std::memory_order_relaxed)) return CCM_OK;
  int* bad = nullptr;
  hipError_t e = hipMalloc((void**)&bad, sizeof(int));
  if (e != hipSuccess) return device_status(fn, e);
  int h = 0;
  e = hipMemcpyAsync(bad, &h, sizeof(int), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && f.ts && f.n_cols > 0 && f.L > 0) {
    hipLaunchKernelGGL(finite_cols_kernel, dim3(grid_for((int64_t)f.L * f.n_cols)), dim3(256), 0,
                       stream, f.ts, f.ld, f.L, f.cols, f.col0, f.n_cols, bad);
    e = hipGetLastError();
  }
  for (int a = 0; a < 3 && e == hipSuccess; ++a)
    if (f.flat[a] && f.flat_n[a] > 0) {
      hipLaunchKernelGGL(finite_flat_kernel, dim3(grid_for(f.flat_n[a])), dim3(256), 0, stream,
                         f.flat[a], f.flat_n[a], bad);
      e = hipGetLastError();
    }
  if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  const hipError_t ef = hipFree(bad);
  if (e == hipSuccess) e = ef;
  if (e != hipSuccess) return device_status(fn, e);
  return h ? fail(CCM_EINVAL, fn, "non-finite input value (debug check)") : CCM_OK;
}

FiniteSpec targets_and_weights(const float* ts, int64_t ld, int L, int tgt0, int n_tgt,
                               const float* nbr_w, int64_t n_w) {
  FiniteSpec f;
  f.ts = ts; f.ld = ld; f.L = L; f.col0 = tgt0; f.n_cols = n_tgt;
  f.flat[0] = nbr_w; f.flat_n[0] = n_w;
  return f;
}

bool check_series(const char* fn, ccm_status* st, const float* ts, int64_t ld, int32_t L,
                  int32_t tau) {
  if (!ts) { *st = fail(CCM_EINVAL, fn, "ts is NULL"); return false; }
  if (ld < 1) { *st = fail(CCM_EINVAL, fn, "ld must be >= 1"); return false; }
  if (L < 2 || L > CCM_L_MAX) { *st = fail(CCM_ERANGE, fn, "L outside [2, CCM_L_MAX]"); return false; }
  if (tau < 1) { *st = fail(CCM_ERANGE, fn, "tau must be >= 1"); return false; }
  return true;
}

}  // namespace

extern "C" {

const char* ccm_version(void) { return "ccm-gfx950 0.1"; }

ccm_status ccm_set_check_finite(int32_t on) {
  g_check_finite.store(on ? 1 : 0, std::memory_order_relaxed);
  return CCM_OK;
}

ccm_status ccm_set_gather_tile(int32_t targets) {
  if (targets != 0 && targets != 4 && targets != 8 && targets != 16 && targets != 32)
    return fail(CCM_EINVAL, "ccm_set_gather_tile", "targets must be 0, 4, 8, 16 or 32");
  ccm_gather_force_tile(targets);
  return CCM_OK;
}

const char* ccm_last_error(void) { return g_last_error.c_str(); }

const char* ccm_status_string(ccm_status s) {
  switch (s) {
    case CCM_OK: return "CCM_OK";
    case CCM_EINVAL: return "CCM_EINVAL: invalid argument";
    case CCM_ERANGE: return "CCM_ERANGE: value out of range";
    case CCM_EDEVICE: return "CCM_EDEVICE: HIP runtime error";
    case CCM_ENOTSUP: return "CCM_ENOTSUP: not supported";
    case CCM_EWORKSPACE: return "CCM_EWORKSPACE: workspace too small";
    default: return "unknown ccm_status";
  }
}

ccm_status ccm_workspace_size(int32_t op, int32_t L, int32_t n_lib, int32_t n_tgt, int32_t k_max,
                              size_t* bytes) {
  if (!bytes) return fail(CCM_EINVAL, "ccm_workspace_size", "bytes is NULL");
  if (L < 0 || n_lib < 0 || n_tgt < 0 || k_max < 0)
    return fail(CCM_EINVAL, "ccm_workspace_size", "negative size");
  switch (op) {
    case CCM_OP_EMBED:
    case CCM_OP_KNN:
      *bytes = 0;
      return CCM_OK;
    case CCM_OP_SIMPLEX:  // FP64 skill per (series, E); n_lib = number of series
      *bytes = align_up((size_t)n_lib * CCM_E_MAX * sizeof(double));
      return CCM_OK;
    case CCM_OP_CROSSMAP_FP32:
      *bytes = fp32_ws(L, n_lib, k_max, n_tgt).total;
      return CCM_OK;
    case CCM_OP_CROSSMAP_BF16:
      *bytes = bf16_ws(L, n_lib, n_tgt).total;
      return CCM_OK;
    case CCM_OP_CROSSMAP_TARGET_E:  // n_lib = number of (E, library) tables
      *bytes = target_E_ws(L, n_lib, n_tgt, k_max).total;
      return CCM_OK;
    case CCM_OP_CROSSMAP_BACKWARD:  // n_tgt = number of pairs
      *bytes = ccm_backward_ws_bytes(L, n_lib, n_tgt, k_max);
      return CCM_OK;
    default:
      return fail(CCM_EINVAL, "ccm_workspace_size", "unknown op");
  }
}

ccm_status ccm_embed(const float* ts, int64_t ld, int32_t L, const int32_t* ids, int32_t n,
                     int32_t E, int32_t tau, float* emb, void* stream) {
  const char* fn = "ccm_embed";
  ccm_status st = CCM_OK;
  if (!check_series(fn, &st, ts, ld, L, tau)) return st;
  if (n < 0) return fail(CCM_EINVAL, fn, "n < 0");
  if (E < 1 || E > CCM_E_MAX) return fail(CCM_ERANGE, fn, "E outside [1, CCM_E_MAX]");
  if ((int64_t)(E - 1) * tau >= L) return fail(CCM_ERANGE, fn, "(E-1)*tau >= L");
  if (n > 0 && (!ids || !emb)) return fail(CCM_EINVAL, fn, "ids or emb is NULL");
  FiniteSpec f;
  f.ts = ts; f.ld = ld; f.L = L; f.cols = ids; f.n_cols = n;
  if ((st = check_finite(fn, f, (hipStream_t)stream)) != CCM_OK) return st;
  return device_status(fn, ccm_launch_embed(ts, ld, L, ids, n, E, tau, emb, (hipStream_t)stream));
}

namespace {
ccm_status knn_common(const char* fn, const float* ts, int64_t ld, int32_t L,
                      const int32_t* lib_ids, const int32_t* lib_E, int32_t n_lib, int32_t tau,
                      int32_t Tp, int32_t k_max, const uint8_t* cand_mask, int32_t* nbr_idx,
                      float* nbr_w, float* nbr_d2, void* stream) {
  ccm_status st = CCM_OK;
  if (!check_series(fn, &st, ts, ld, L, tau)) return st;
  if (n_lib < 0) return fail(CCM_EINVAL, fn, "n_lib < 0");
  if (n_lib > 0 && (!lib_ids || !lib_E || !nbr_idx || !nbr_w))
    return fail(CCM_EINVAL, fn, "NULL array argument");
  if (k_max < 2 || k_max > CCM_K_MAX) return fail(CCM_EINVAL, fn, "k_max outside [2, CCM_K_MAX]");
  if (Tp < 0 || Tp >= L) return fail(CCM_EINVAL, fn, "Tp outside [0, L)");
  FiniteSpec f;
  f.ts = ts; f.ld = ld; f.L = L; f.cols = lib_ids; f.n_cols = n_lib;
  if ((st = check_finite(fn, f, (hipStream_t)stream)) != CCM_OK) return st;
  return device_status(fn, ccm_launch_knn(ts, ld, L, lib_ids, lib_E, n_lib, tau, Tp, k_max,
                                          cand_mask, nbr_idx, nbr_w, nbr_d2, (hipStream_t)stream));
}
}  // namespace

ccm_status ccm_knn(const float* ts, int64_t ld, int32_t L, const int32_t* lib_ids,
                   const int32_t* lib_E, int32_t n_lib, int32_t tau, int32_t Tp, int32_t k_max,
                   int32_t* nbr_idx, float* nbr_w, float* nbr_d2, void* ws, size_t ws_bytes,
                   void* stream) {
  (void)ws;
  (void)ws_bytes;
  return knn_common("ccm_knn", ts, ld, L, lib_ids, lib_E, n_lib, tau, Tp, k_max, nullptr, nbr_idx,
                    nbr_w, nbr_d2, stream);
}

ccm_status ccm_knn_subset(const float* ts, int64_t ld, int32_t L, const int32_t* lib_ids,
                          const int32_t* lib_E, int32_t n_lib, int32_t tau, int32_t Tp,
                          int32_t k_max, const uint8_t* cand_mask, int32_t* nbr_idx,
                          float* nbr_w, float* nbr_d2, void* ws, size_t ws_bytes, void* stream) {
  (void)ws;
  (void)ws_bytes;
  if (n_lib > 0 && !cand_mask) return fail(CCM_EINVAL, "ccm_knn_subset", "cand_mask is NULL");
  return knn_common("ccm_knn_subset", ts, ld, L, lib_ids, lib_E, n_lib, tau, Tp, k_max, cand_mask,
                    nbr_idx, nbr_w, nbr_d2, stream);
}

}  // extern "C"

namespace {
// Argument checks shared by both optE entry points.
bool check_simplex(const char* fn, ccm_status* st, const float* ts, int64_t ld, int32_t L,
                   const int32_t* ids, int32_t n, int32_t E_min, int32_t E_max, int32_t tau,
                   int32_t Tp, int32_t mode, const int32_t* optE) {
  if (!check_series(fn, st, ts, ld, L, tau)) return false;
  if (n < 0) { *st = fail(CCM_EINVAL, fn, "n < 0"); return false; }
  if (n > 0 && (!ids || !optE)) { *st = fail(CCM_EINVAL, fn, "ids or optE is NULL"); return false; }
  if (mode != CCM_MODE_LOO && mode != CCM_MODE_HALF) {
    *st = fail(CCM_EINVAL, fn, "unknown mode");
    return false;
  }
  if (Tp < 0) { *st = fail(CCM_EINVAL, fn, "Tp < 0"); return false; }
  if (E_min < 1 || E_max > CCM_E_MAX || E_min > E_max) {
    *st = fail(CCM_ERANGE, fn, "need 1 <= E_min <= E_max <= CCM_E_MAX");
    return false;
  }
  // admissible candidates at the largest E must cover k = E_max + 1
  const int64_t lo = (int64_t)(E_max - 1) * tau;
  int64_t ncand;
  if (mode == CCM_MODE_LOO)
    ncand = (L - 1 - Tp) - lo + 1 - 1;  // query excluded
  else
    ncand = (L / 2 - 1 - Tp) - lo + 1;
  if (ncand < E_max + 1) {
    *st = fail(CCM_ERANGE, fn, "too few points for k = E_max + 1 neighbours");
    return false;
  }
  return true;
}
}  // namespace

extern "C" {

ccm_status ccm_simplex_optE(const float* ts, int64_t ld, int32_t L, const int32_t* ids, int32_t n,
                            int32_t E_min, int32_t E_max, int32_t tau, int32_t Tp, int32_t mode,
                            int32_t* optE, float* rho_E, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "ccm_simplex_optE";
  ccm_status st = CCM_OK;
  if (!check_simplex(fn, &st, ts, ld, L, ids, n, E_min, E_max, tau, Tp, mode, optE)) return st;
  if (n == 0) return CCM_OK;
  const size_t need = align_up((size_t)n * CCM_E_MAX * sizeof(double));
  if (!ws || ws_bytes < need) return fail(CCM_EWORKSPACE, fn, "workspace too small");
  FiniteSpec f;
  f.ts = ts; f.ld = ld; f.L = L; f.cols = ids; f.n_cols = n;
  if ((st = check_finite(fn, f, (hipStream_t)stream)) != CCM_OK) return st;
  return device_status(fn, ccm_launch_simplex(ts, ld, L, ids, n, E_min, E_max, tau, Tp, mode, optE,
                                              rho_E, (double*)ws, (hipStream_t)stream));
}

ccm_status ccm_simplex_optE_noalloc(const float* ts, int64_t ld, int32_t L, const int32_t* ids,
                                    int32_t n, int32_t E_min, int32_t E_max, int32_t tau,
                                    int32_t Tp, int32_t mode, int32_t* optE, float* rho_E,
                                    void* stream) {
  const char* fn = "ccm_simplex_optE_noalloc";
  ccm_status st = CCM_OK;
  if (!check_simplex(fn, &st, ts, ld, L, ids, n, E_min, E_max, tau, Tp, mode, optE)) return st;
  if (n > ccm_noalloc_max_series())
    return fail(CCM_ERANGE, fn, "n exceeds CCM_NOALLOC_MAX_SERIES (the static scratch)");
  if (n == 0) return CCM_OK;
  // every skill the finalize step reads is written earlier in the same call, so the shared
  // scratch needs no clearing
  double* scratch = nullptr;
  hipError_t e = ccm_noalloc_scratch(&scratch);
  if (e != hipSuccess) return device_status(fn, e);
  return device_status(fn, ccm_launch_simplex(ts, ld, L, ids, n, E_min, E_max, tau, Tp, mode, optE,
                                              rho_E, scratch, (hipStream_t)stream));
}

ccm_status ccm_crossmap_rho(const float* ts, int64_t ld, int32_t L, const int32_t* nbr_idx,
                            const float* nbr_w, const int32_t* lib_E, int32_t n_lib, int32_t k_max,
                            int32_t tau, int32_t tgt0, int32_t n_tgt, int32_t precision, float* rho,
                            double* moments, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "ccm_crossmap_rho";
  ccm_status st = CCM_OK;
  if (!check_series(fn, &st, ts, ld, L, tau)) return st;
  if (n_lib < 0 || n_tgt < 0 || tgt0 < 0) return fail(CCM_EINVAL, fn, "negative size or offset");
  if ((int64_t)tgt0 + n_tgt > ld) return fail(CCM_EINVAL, fn, "targets exceed the panel width ld");
  if (n_lib > 0 && n_tgt > 0 && (!nbr_idx || !nbr_w || !lib_E || !rho))
    return fail(CCM_EINVAL, fn, "NULL array argument");
  if (k_max < 2 || k_max > CCM_K_MAX) return fail(CCM_EINVAL, fn, "k_max outside [2, CCM_K_MAX]");
  if (L < 4) return fail(CCM_ERANGE, fn, "L < 4");
  if (precision == CCM_PRECISION_FP32) {
    CrossmapWs w = fp32_ws(L, n_lib, k_max, n_tgt);
    if (n_lib == 0 || n_tgt == 0) return CCM_OK;
    if (!ws || ws_bytes < w.total) return fail(CCM_EWORKSPACE, fn, "workspace too small");
    if ((st = check_finite(fn, targets_and_weights(ts, ld, L, tgt0, n_tgt, nbr_w,
                                                   (int64_t)n_lib * L * k_max),
                           (hipStream_t)stream)) != CCM_OK)
      return st;
    char* base = (char*)ws;
    return device_status(
        fn, ccm_launch_crossmap_fp32(ts, ld, L, tau, tgt0, n_tgt, nbr_idx, nbr_w, lib_E, n_lib, k_max,
                                     rho, moments, (uint32_t*)(base + w.off_poff),
                                     (float*)(base + w.off_pw), (int*)(base + w.off_libk),
                                     (int*)(base + w.off_order), (float*)(base + w.off_gtile),
                                     (double*)(base + w.off_gsum), (hipStream_t)stream));
  }
  if (precision == CCM_PRECISION_BF16) {
    Bf16Ws w = bf16_ws(L, n_lib, n_tgt);
    if (n_lib == 0 || n_tgt == 0) return CCM_OK;
    if (!ws || ws_bytes < w.total) return fail(CCM_EWORKSPACE, fn, "workspace too small");
    if ((st = check_finite(fn, targets_and_weights(ts, ld, L, tgt0, n_tgt, nbr_w,
                                                   (int64_t)n_lib * L * k_max),
                           (hipStream_t)stream)) != CCM_OK)
      return st;
    char* base = (char*)ws;
    return device_status(
        fn, ccm_launch_crossmap_bf16(ts, ld, L, tau, tgt0, n_tgt, nbr_idx, nbr_w, lib_E, n_lib, k_max,
                                     rho, moments, (uint16_t*)(base + w.off_yt),
                                     (float*)(base + w.off_cref),
                                     (uint32_t*)(base + w.off_ent), (int*)(base + w.off_so),
                                     (int*)(base + w.off_libk), (int*)(base + w.off_order),
                                     (hipStream_t)stream));
  }
  return fail(CCM_EINVAL, fn, "unknown precision");
}

ccm_status ccm_crossmap_rho_target_E(const float* ts, int64_t ld, int32_t L,
                                     const int32_t* nbr_idx, const float* nbr_w, int32_t n_lib,
                                     int32_t E_lo, int32_t n_E, int32_t k_max, int32_t tau,
                                     const int32_t* tgt_E, int32_t tgt0, int32_t n_tgt,
                                     float* rho, double* moments, void* ws, size_t ws_bytes,
                                     void* stream) {
  const char* fn = "ccm_crossmap_rho_target_E";
  ccm_status st = CCM_OK;
  if (!check_series(fn, &st, ts, ld, L, tau)) return st;
  if (n_lib < 0 || n_tgt < 0 || tgt0 < 0) return fail(CCM_EINVAL, fn, "negative size or offset");
  if ((int64_t)tgt0 + n_tgt > ld) return fail(CCM_EINVAL, fn, "targets exceed the panel width ld");
  if (k_max < 2 || k_max > CCM_K_MAX) return fail(CCM_EINVAL, fn, "k_max outside [2, CCM_K_MAX]");
  if (E_lo < 1 || n_E < 1 || E_lo + n_E - 1 > CCM_E_MAX)
    return fail(CCM_ERANGE, fn, "E_lo .. E_lo + n_E - 1 outside [1, CCM_E_MAX]");
  if (E_lo + n_E > k_max) return fail(CCM_ERANGE, fn, "k_max < largest E + 1");
  if ((int64_t)n_E * n_lib > INT32_MAX / 2) return fail(CCM_EINVAL, fn, "too many tables");
  if (n_lib > 0 && n_tgt > 0 && (!nbr_idx || !nbr_w || !tgt_E || !rho))
    return fail(CCM_EINVAL, fn, "NULL array argument");
  if (L < 4) return fail(CCM_ERANGE, fn, "L < 4");
  const TargetEWs w = target_E_ws(L, n_E * n_lib, n_tgt, k_max);
  if (n_lib == 0 || n_tgt == 0) return CCM_OK;
  if (!ws || ws_bytes < w.total) return fail(CCM_EWORKSPACE, fn, "workspace too small");
  if ((st = check_finite(fn, targets_and_weights(ts, ld, L, tgt0, n_tgt, nbr_w,
                                                 (int64_t)n_E * n_lib * L * k_max),
                         (hipStream_t)stream)) != CCM_OK)
    return st;
  char* base = (char*)ws;
  return device_status(
      fn, ccm_launch_crossmap_fp32_target_E(
              ts, ld, L, tau, tgt0, n_tgt, nbr_idx, nbr_w, n_lib, E_lo, n_E, k_max, tgt_E, rho,
              moments, (uint32_t*)(base + w.tab.off_poff), (float*)(base + w.tab.off_pw),
              (int*)(base + w.tab.off_libk), (int*)(base + w.off_tabE), (int*)(base + w.off_perm),
              (int*)(base + w.off_tiles), (int*)(base + w.off_ntiles),
              (float*)(base + w.tab.off_gtile), (double*)(base + w.tab.off_gsum),
              (hipStream_t)stream));
}

ccm_status ccm_crossmap_rho_backward(const float* ts, int64_t ld, int32_t L, const float* lib_ts,
                                     const int32_t* nbr_idx, const float* nbr_w,
                                     const int32_t* lib_E, int32_t n_lib, int32_t k_max,
                                     int32_t tau, const int32_t* pair_lib, const int32_t* pair_tgt,
                                     const float* grad_rho, int32_t n_pairs, float* grad_ts,
                                     float* grad_lib, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "ccm_crossmap_rho_backward";
  ccm_status st = CCM_OK;
  if (!check_series(fn, &st, ts, ld, L, tau)) return st;
  if (n_lib < 0 || n_pairs < 0) return fail(CCM_EINVAL, fn, "negative size");
  if (k_max < 2 || k_max > CCM_K_MAX) return fail(CCM_EINVAL, fn, "k_max outside [2, CCM_K_MAX]");
  if (n_pairs == 0) return CCM_OK;
  if (!lib_ts || !nbr_idx || !nbr_w || !lib_E || !pair_lib || !pair_tgt || !grad_rho)
    return fail(CCM_EINVAL, fn, "NULL array argument");
  if (!grad_ts && !grad_lib) return fail(CCM_EINVAL, fn, "both gradients are NULL");
  const size_t need = ccm_backward_ws_bytes(L, n_lib, n_pairs, k_max);
  if (!ws || ws_bytes < need) return fail(CCM_EWORKSPACE, fn, "workspace too small");
  FiniteSpec f;
  f.ts = ts; f.ld = ld; f.L = L; f.cols = pair_tgt; f.n_cols = n_pairs;
  f.flat[0] = lib_ts; f.flat_n[0] = (int64_t)n_lib * L;
  f.flat[1] = nbr_w; f.flat_n[1] = (int64_t)n_lib * L * k_max;
  f.flat[2] = grad_rho; f.flat_n[2] = n_pairs;
  if ((st = check_finite(fn, f, (hipStream_t)stream)) != CCM_OK) return st;
  return device_status(fn, ccm_launch_backward(ts, ld, L, lib_ts, nbr_idx, nbr_w, lib_E, n_lib,
                                               k_max, tau, pair_lib, pair_tgt, grad_rho, n_pairs,
                                               grad_ts, grad_lib, ws, (hipStream_t)stream));
}

}  // extern "C"
