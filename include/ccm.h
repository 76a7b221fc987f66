/*
 * ccm.h -- C ABI of the MI355X (gfx950) all-pairs Convergent Cross Mapping hot path.
 *
 * The method is the one of Watanakeesuntorn et al., "Massively Parallel Causal Inference
 * of Whole Brain Dynamics at Single Neuron Resolution" (IEEE eScience 2020):
 *   - delay embedding of each series (Sec. II-B);
 *   - an exact k-nearest-neighbour table per library series, k = E + 1 (Sec. III-B,
 *     Alg. 3 / Alg. 4), turned into exponential weights normalised per row
 *     (Sec. III-A, "normalize");
 *   - optimal E per series by simplex projection (Sec. II-B; Alg. 1 phase 1);
 *   - one table per library reused to cross-map every target series (Sec. III-B, Alg. 2)
 *     through the lookup of Alg. 5 and a Pearson correlation (corrcoef).
 *
 * Conventions shared by every entry point
 *   - Every function returns a ccm_status.  No C++ exception crosses this boundary.
 *   - Array arguments are DEVICE pointers owned by the caller, unless stated otherwise.
 *     The library keeps no allocation between calls; scratch space is the caller's
 *     workspace (size from ccm_workspace_size).  The one exception is the static device
 *     array behind ccm_simplex_optE_noalloc.
 *   - Every call is asynchronous on `stream` (a hipStream_t passed as void*, NULL = the
 *     default stream) and never synchronises the host.  Device-side problems that cannot
 *     be seen without a synchronisation (a library E out of range) are reported in the
 *     outputs, as described per function, never by blocking.
 *   - The series panel `ts` is time-major: value x_c(t) of series c is ts[t * ld + c],
 *     t = 0 .. L-1.  Series indices (ids) are columns of that panel.
 *   - Time indices are int32; values are float32; correlation moments are float64.
 *   - A point of an E-dimensional embedding is labelled by its newest coordinate:
 *     point t = (x(t), x(t - tau), ..., x(t - (E-1) tau)), t >= (E-1) tau.
 *   - Inputs must be finite.  ccm_set_check_finite(1) turns on a debug mode in which each
 *     entry point first checks the floating-point inputs it reads and returns CCM_EINVAL
 *     for a non-finite value (that mode synchronises the stream).
 *   - 1 <= E <= CCM_E_MAX, tau >= 1, L <= CCM_L_MAX.
 */
#ifndef CCM_H
#define CCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ccm_status;

#define CCM_OK 0
#define CCM_EINVAL 1     /* null pointer, negative size, bad enum                      */
#define CCM_ERANGE 2     /* E outside [1, CCM_E_MAX], k > admissible candidates, L too big */
#define CCM_EDEVICE 3    /* a HIP runtime error; text in ccm_last_error()              */
#define CCM_ENOTSUP 4    /* valid request this build does not implement                */
#define CCM_EWORKSPACE 5 /* workspace missing or smaller than ccm_workspace_size says  */

#define CCM_E_MAX 20
#define CCM_K_MAX (CCM_E_MAX + 1)
#define CCM_L_MAX 16384

/* selection protocol of ccm_simplex_optE */
#define CCM_MODE_LOO 0   /* leave-one-out over the whole series (query excluded)         */
#define CCM_MODE_HALF 1  /* the paper's split: first half = library, second half = target */

/* arithmetic form of ccm_crossmap_rho */
#define CCM_PRECISION_FP32 0 /* FP32 gather of the k neighbour rows, FP64 moments       */
#define CCM_PRECISION_BF16 1 /* tables densified to BF16, MFMA contraction, FP32 accum.  */

/* operation codes of ccm_workspace_size */
#define CCM_OP_EMBED 0
#define CCM_OP_KNN 1
#define CCM_OP_SIMPLEX 2
#define CCM_OP_CROSSMAP_FP32 3
#define CCM_OP_CROSSMAP_BF16 4
#define CCM_OP_CROSSMAP_BACKWARD 5
#define CCM_OP_CROSSMAP_TARGET_E 6   /* n_lib argument = number of (E, library) tables */

/*
 * ccm_embed -- delay embedding (Sec. II-B; the explicit blocks of Alg. 4).
 *   ts [L][ld]       input panel.
 *   ids [n]          series (columns of ts) to embed.
 *   emb [n][L-(E-1)tau][E]  output; emb[i][r][e] = ts[(r + (E-1)tau - e tau) * ld + ids[i]].
 * Errors: EINVAL for null pointers or n < 0; ERANGE if E outside [1, CCM_E_MAX], tau < 1
 * or (E-1) tau >= L.  A series id outside [0, ld) gets NaN in every element of its block.
 */
ccm_status ccm_embed(const float* ts, int64_t ld, int32_t L, const int32_t* ids, int32_t n,
                     int32_t E, int32_t tau, float* emb, void* stream);

/*
 * ccm_knn -- neighbour tables, one per library, at the library's own E (Sec. III-B,
 * Alg. 2 lines computing indices/distances, Alg. 3 / Alg. 4; weights per Sec. III-A).
 *   lib_ids [n_lib]  library series (columns of ts).
 *   lib_E   [n_lib]  embedding dimension of each library (device array).
 *   Tp               prediction horizon; candidates s need s + Tp <= L-1.  The cross-map
 *                    uses Tp = 0.
 *   Query set = candidate set = {t : (E-1) tau <= t <= L-1-Tp}; a query is excluded from
 *   its own candidates; k = E + 1 smallest by (d^2, time index) where
 *   d^2 = canonical FP32 sum over lags e = 0..E-1 of (x(t-e tau) - x(s-e tau))^2, each
 *   subtraction, product and sum rounded once, lag 0 first.
 *   Outputs, row-major [n_lib][L][k_max]:
 *     nbr_idx  neighbour time indices, nearest first;
 *     nbr_w    weights u_k / sum(u), u_k = exp(-d_k / d_1), with each selected neighbour's
 *              distance d recomputed in FP64 from the series; when d_1 = 0, u_k = 1
 *              where d_k = 0 and 0 elsewhere;
 *     nbr_d2   (nullable) the FP32 d^2 of each neighbour.
 *   Rows t outside the query set and slots beyond E + 1 are padding: idx = -1, w = 0,
 *   d2 = +inf.  A library whose E is out of [1, CCM_E_MAX], has E + 1 > k_max, or has
 *   fewer than E + 2 points, or whose series id is outside [0, ld), gets padding in every row
 *   (and NaN rho downstream).
 * Errors: EINVAL (nulls, n_lib < 0, k_max < 2 or > CCM_K_MAX, Tp < 0); ERANGE (L or tau).
 * Workspace: none (ws may be NULL).
 */
ccm_status ccm_knn(const float* ts, int64_t ld, int32_t L, const int32_t* lib_ids,
                   const int32_t* lib_E, int32_t n_lib, int32_t tau, int32_t Tp, int32_t k_max,
                   int32_t* nbr_idx, float* nbr_w, float* nbr_d2, void* ws, size_t ws_bytes,
                   void* stream);

/*
 * ccm_knn_subset -- ccm_knn over a library subsample, for the CCM convergence test (the
 * original CCM definition recalled in Sec. III-A: predictions repeated with random
 * library subsets of growing size).
 *   cand_mask [n_lib][L]  (device, uint8) nonzero at the time indices library row i may
 *                         take as neighbours; every point of the query set is still a
 *                         query, and excluded from its own candidates.
 *   Everything else as ccm_knn.  A library with fewer than E + 2 marked points in its
 *   candidate set gets padding in every row.
 * Errors: as ccm_knn, and EINVAL if cand_mask is NULL.  Workspace: none.
 */
ccm_status ccm_knn_subset(const float* ts, int64_t ld, int32_t L, const int32_t* lib_ids,
                          const int32_t* lib_E, int32_t n_lib, int32_t tau, int32_t Tp,
                          int32_t k_max, const uint8_t* cand_mask, int32_t* nbr_idx,
                          float* nbr_w, float* nbr_d2, void* ws, size_t ws_bytes, void* stream);

/*
 * ccm_simplex_optE -- optimal embedding dimension per series by simplex projection
 * (Sec. II-B; Alg. 1 lines "for E = 1..E_max ... optE = argmax").
 *   For every E in [E_min, E_max]: neighbours as in ccm_knn with horizon Tp, prediction
 *   xhat(t+Tp) = sum_k w_k x(n_k + Tp), skill rho_E = Pearson(x(t+Tp), xhat(t+Tp)) over the
 *   query set (FP64 sums).  mode CCM_MODE_LOO: query = candidate set over the whole series,
 *   query excluded.  mode CCM_MODE_HALF: candidates from the first half [0, L/2) and queries
 *   from the second half, each half embedded on its own, no exclusion.
 *   optE [n]                 smallest E reaching the largest non-NaN rho_E (E_min if all NaN).
 *   rho_E [n][E_max-E_min+1] (nullable) the skills; NaN where a variance vanishes, and in
 *                            every E for a series id outside [0, ld) (whose optE is E_min).
 * Errors: EINVAL (nulls, bad mode, Tp < 0); ERANGE (E range, or too few points for
 * k = E_max + 1 candidates).  Workspace: ccm_workspace_size(CCM_OP_SIMPLEX, ...).
 */
ccm_status ccm_simplex_optE(const float* ts, int64_t ld, int32_t L, const int32_t* ids,
                            int32_t n, int32_t E_min, int32_t E_max, int32_t tau, int32_t Tp,
                            int32_t mode, int32_t* optE, float* rho_E, void* ws,
                            size_t ws_bytes, void* stream);

/*
 * ccm_simplex_optE_noalloc -- ccm_simplex_optE for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, outputs, kernels and results as ccm_simplex_optE, without the
 * workspace: the per-(series, E) FP64 skills live in a static device array of the library
 * (16 MiB, CCM_NOALLOC_MAX_SERIES x CCM_E_MAX doubles), one per GPU, held from the first
 * call on that GPU until the process ends.  The call makes no hipMalloc, hipFree or other
 * allocating call; its first call on a device looks up the array's device address once.
 *   n                 at most CCM_NOALLOC_MAX_SERIES (ERANGE beyond it).
 * Calls on one GPU share its array: calls that overlap in time on that GPU (on different
 * streams, or from different host threads without ordering) race and give undefined
 * outputs; calls ordered on one stream are safe.  The debug finiteness check
 * (ccm_set_check_finite) is not applied here (it allocates).
 * Errors: as ccm_simplex_optE, plus ERANGE for n > CCM_NOALLOC_MAX_SERIES.
 */
#define CCM_NOALLOC_MAX_SERIES 104857
ccm_status ccm_simplex_optE_noalloc(const float* ts, int64_t ld, int32_t L, const int32_t* ids,
                                    int32_t n, int32_t E_min, int32_t E_max, int32_t tau,
                                    int32_t Tp, int32_t mode, int32_t* optE, float* rho_E,
                                    void* stream);

/*
 * ccm_crossmap_rho -- cross-map every target with every library table and reduce each
 * prediction to Pearson rho (Sec. III-B, Alg. 2 inner loop, Alg. 5, corrcoef).
 *   nbr_idx, nbr_w [n_lib][L][k_max]  tables from ccm_knn (Tp = 0).
 *   lib_E [n_lib]                    E of each library (device); rows t >= (E-1) tau used.
 *   targets: series tgt0 .. tgt0 + n_tgt - 1 of ts.
 *   yhat_ij(t) = sum_k w_i[t,k] * ts[n_ik(t) * ld + j];  rho[i][j - tgt0] = Pearson over
 *   t = (E_i-1) tau .. L-1 of (ts[t * ld + j], yhat_ij(t)); NaN where a variance vanishes.
 *   precision CCM_PRECISION_FP32: FP32 products and sums per prediction, FP64 moments.
 *     The target tile sits in LDS: 16 targets up to L = 2475, 8 up to L = 5035; longer
 *     series (to CCM_L_MAX) read 32-target tiles from a global copy through L2, which the
 *     workspace then holds (n_tgt x L x 4 bytes plus 10.8 KB per 32 targets).
 *     ccm_set_gather_tile can force a tile width for testing.
 *   precision CCM_PRECISION_BF16: target values and weights rounded to BF16, contracted on
 *   MFMA with FP32 accumulation; observed values FP32; FP64 moments.
 *   Both forms first centre each target column on c_j, its mean over t = 0..L-1 rounded to
 *   FP32, and work on y - c_j (rho is unchanged by a common shift of y and yhat, and the
 *   weights of a row sum to 1), so a large offset of a series costs the FP32 and BF16
 *   arithmetic no digits; the zero-variance test and the moments refer to the uncentred y.
 *   rho [n_lib][n_tgt]               output (row = library, column = target).
 *   moments [n_lib][n_tgt][3]        (nullable) FP64 sum(yhat), sum(yhat^2), sum(y*yhat).
 * Errors: EINVAL (nulls, sizes, precision), ERANGE (k_max, L), EWORKSPACE.
 * Workspace: ccm_workspace_size(CCM_OP_CROSSMAP_FP32 or _BF16, L, n_lib, n_tgt, k_max).
 */
ccm_status ccm_crossmap_rho(const float* ts, int64_t ld, int32_t L, const int32_t* nbr_idx,
                            const float* nbr_w, const int32_t* lib_E, int32_t n_lib,
                            int32_t k_max, int32_t tau, int32_t tgt0, int32_t n_tgt,
                            int32_t precision, float* rho, double* moments, void* ws,
                            size_t ws_bytes, void* stream);

/*
 * ccm_crossmap_rho_target_E -- the paper's own form of Alg. 2 (Sec. III-B): target j is
 * cross-mapped with every library's table at the TARGET's E, E_j = tgt_E[j] (its optimal E
 * from phase 1), so one table per (library, E) is shared by all targets of that E.
 *   nbr_idx, nbr_w [n_E][n_lib][L][k_max]  tables from ccm_knn (Tp = 0), E-major: table
 *                    e * n_lib + i is library i at E = E_lo + e (E_lo + n_E - 1 < k_max).
 *   tgt_E [n_tgt]    E of each target (device); a target whose E is outside
 *                    [E_lo, E_lo + n_E) gets rho = NaN in every row.
 *   targets: series tgt0 .. tgt0 + n_tgt - 1 of ts.
 *   rho[i][j] = Pearson over t = (E_j-1) tau .. L-1 of (ts[t * ld + tgt0 + j], yhat_ij(t)),
 *   yhat_ij(t) = sum_k w[t,k] * ts[n_k(t) * ld + tgt0 + j] over library i's table at E_j;
 *   FP32 products and sums per prediction (targets centred as in ccm_crossmap_rho), FP64
 *   moments; NaN where a variance vanishes.
 *   rho [n_lib][n_tgt], moments [n_lib][n_tgt][3] (nullable) as in ccm_crossmap_rho.
 *   Targets are grouped by E on the device (no host synchronisation).
 *   Tile widths (LDS or the global copy) follow L as in ccm_crossmap_rho.
 * Errors: EINVAL (nulls, sizes), ERANGE (E_lo, n_E, k_max, L), EWORKSPACE.  Workspace:
 * ccm_workspace_size(CCM_OP_CROSSMAP_TARGET_E, L, n_E * n_lib, n_tgt, k_max).
 */
ccm_status ccm_crossmap_rho_target_E(const float* ts, int64_t ld, int32_t L,
                                     const int32_t* nbr_idx, const float* nbr_w, int32_t n_lib,
                                     int32_t E_lo, int32_t n_E, int32_t k_max, int32_t tau,
                                     const int32_t* tgt_E, int32_t tgt0, int32_t n_tgt,
                                     float* rho, double* moments, void* ws, size_t ws_bytes,
                                     void* stream);

/*
 * ccm_crossmap_rho_backward -- adjoint of loss = sum_p grad_rho[p] * rho[pair_lib[p]][pair_tgt[p]]
 * with every neighbour set held fixed.
 *   lib_ts [n_lib][L]   the library series (contiguous rows) the tables were built from.
 *   nbr_idx, nbr_w, lib_E, k_max, tau as in ccm_crossmap_rho (Tp = 0 tables).
 *   pair_lib [n_pairs], pair_tgt [n_pairs]  library row and target COLUMN of ts of each pair.
 *   grad_rho [n_pairs]  upstream gradient of each pair's rho.
 *   grad_ts [L][ld]     (nullable) += d loss / d ts through the targets (observed values and
 *                       the looked-up neighbour values).
 *   grad_lib [n_lib][L] (nullable) += d loss / d library series through the weights
 *                       (distances -> exp -> normalisation, including the d_1 path).
 *   The gradient through a zero distance (d_k = 0 or d_1 = 0) is taken as 0.  Pairs whose
 *   rho is NaN contribute nothing.  Accumulation order is fixed (no atomics), so results
 *   are deterministic.
 *   The tables' rows must hold distinct neighbours (as ccm_knn writes them).  Padding entries
 *   (index -1, as in rows of a subsampled table) count as absent: no weight, no distance.
 *   Any n_pairs >= 0 is accepted: pairs run in chunks (at most 65,535 pairs and at most
 *   4 GiB of per-pair buffers each, 6 L + 2 L k_max floats and 21 L doubles per pair), one
 *   after another in pair order, so the result does not depend on the chunk size and the
 *   workspace stays bounded (about 4 GiB plus 16 n_lib L k_max bytes for the per-library
 *   lists).
 * Errors: EINVAL, ERANGE, EWORKSPACE.  Workspace: ccm_workspace_size(CCM_OP_CROSSMAP_BACKWARD,
 * L, n_lib, n_pairs, k_max).
 */
ccm_status ccm_crossmap_rho_backward(const float* ts, int64_t ld, int32_t L, const float* lib_ts,
                                     const int32_t* nbr_idx, const float* nbr_w,
                                     const int32_t* lib_E, int32_t n_lib, int32_t k_max,
                                     int32_t tau, const int32_t* pair_lib,
                                     const int32_t* pair_tgt, const float* grad_rho,
                                     int32_t n_pairs, float* grad_ts, float* grad_lib, void* ws,
                                     size_t ws_bytes, void* stream);

/*
 * ccm_workspace_size -- bytes of workspace the operation `op` needs (host call, no device
 * work).  n_tgt is the number of targets (crossmap) or of pairs (backward).
 */
ccm_status ccm_workspace_size(int32_t op, int32_t L, int32_t n_lib, int32_t n_tgt,
                              int32_t k_max, size_t* bytes);

/*
 * ccm_set_check_finite -- debug mode for the convention that inputs are finite (host call,
 * process-wide, off by default).  With on != 0, every later call first checks, on its
 * stream, the series columns it reads (ids, library ids, targets, or the pairs' target
 * columns), the tables' weights, and the backward's library series and upstream gradients,
 * waits for that check (a host synchronisation, which the calls otherwise never make),
 * and returns CCM_EINVAL ("non-finite input value") without launching the operation if a
 * value is NaN or infinite.  With on = 0 nothing is checked: non-finite inputs then give
 * unspecified (typically NaN) outputs, never a fault.  Always returns CCM_OK.
 */
ccm_status ccm_set_check_finite(int32_t on);

/*
 * ccm_set_gather_tile -- testing switch (process-wide) for the FP32 cross-map's target tile
 * (ccm_crossmap_rho and ccm_crossmap_rho_target_E).
 *   targets  0 (the default): chosen from L -- 16 targets per tile in LDS while that tile
 *            fits (L <= 2475), then 8 (L <= 5035), beyond that 32 targets read from a
 *            global copy of the tile kept in the workspace;
 *            4, 8 or 16: that LDS tile wherever it fits (4 targets: L <= 10155), else the
 *            default choice;
 *            32: the global copy at every L.
 * Every tile width computes the same products; only the order of a row's FP32 products can
 * differ, so rho agrees within FP32 rounding.  Workspace sizes follow the switch: set it
 * before ccm_workspace_size and keep it until the call has been enqueued.
 * Errors: EINVAL for any other value.
 */
ccm_status ccm_set_gather_tile(int32_t targets);

/* Static text of a status code. */
const char* ccm_status_string(ccm_status s);
/* Text of the last error raised on the calling thread ("" if none). */
const char* ccm_last_error(void);
/* Library version string. */
const char* ccm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CCM_H */
