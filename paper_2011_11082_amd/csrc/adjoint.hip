// Adjoint of the cross-map: gradient of loss = sum_p g_p * rho[lib_p][tgt_p] with every
// neighbour set held fixed (not in the paper; the forward is Sec. III-B, Alg. 2 / Alg. 5
// with corrcoef, and the weights of Sec. III-A).
//
// For one pair (library i, target column j) with rows t in Q = [(E-1)tau, L-1]:
//   yhat(t) = sum_m w[t,m] y(n_m(t));  rho = c / sqrt(a b) with centred sums
//   a = sum (y-ybar)^2, b = sum (yhat-pbar)^2, c = sum (y-ybar)(yhat-pbar)
//   H(t)  = g drho/dyhat(t) = g [ (y(t)-ybar)/sqrt(ab) - rho (yhat(t)-pbar)/b ]
//   Gy(t) = g drho/dy(t)|obs = g [ (yhat(t)-pbar)/sqrt(ab) - rho (y(t)-ybar)/a ]
//   target:  dL/dy(s) = Gy(s) [s in Q] + sum_{(t,m): n_m(t) = s} w[t,m] H(t)
//   weights: wbar[t,m] = H(t) y(n_m(t));  w = u / S, u_m = exp(-d_m / d_1)
//            ubar_m = (wbar_m - sum_l wbar_l w_l) / S
//            dbar_m = -ubar_m u_m / d_1 (m >= 2);  dbar_1 = sum_{m>=2} ubar_m u_m d_m / d_1^2
//            (u_1 = e^-1 does not depend on x; zero distances contribute nothing)
//   library: d_m = ||v(t) - v(n_m)||, so coef = dbar_m / d_m gives
//            dL/dx(t - e tau) += coef (x(t-e tau) - x(n_m - e tau))
//            dL/dx(n_m - e tau) -= coef (x(t-e tau) - x(n_m - e tau))
//
// gfx950 design: no atomics on values, fixed summation order (deterministic results).
//   Kernel 3 (first): one workgroup per library builds the transposed neighbour relation
//   (for each time s, the table entries whose neighbour is s, in table order), the position
//   of every entry in it and an m-major copy of the table (both [m][t]), and the weights in
//   list order.
//   Kernel 1: one workgroup per pair reads its target column once (into LDS, and a
//   contiguous copy for kernel 2), recomputes yhat and the FP64 Pearson pieces and stores
//   H, Gy.  Kernel 2: one thread per (pair, t) turns wbar into distance coefficients
//   (distances recomputed in FP64 from the library series, staged in LDS with the target
//   column), written m-major and in the transposed order.  Kernel 4, in two steps: one thread per (pair, u) reads table row u
//   (m-major, consecutive u in consecutive lanes) and u's transposed list (coefficients
//   and weights contiguous) once and keeps E partial sums, one per lag; one thread per
//   (pair, s) then combines the E partial sums and the target term that land on time s.
//   Kernel 5: one wave per (64 times, column hash) adds the pairs' contributions in pair
//   order into the target and library gradients.
//   The per-pair kernels run on XCD-aware grids (xcd_pair_block), pairs grouped by library.
// Padding entries (-1) count as absent everywhere.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "wave.h"

namespace ccm {

constexpr int kBwThreads = 256;
constexpr int kXcdA = 8;   // XCDs: workgroup b of a launch runs on XCD b mod 8

// XCD-aware placement of a chunk's pairs: XCD x takes the x-th eighth of the pairs in
// processing order (pairs of one library are adjacent there), and the nb workgroups of one
// pair (its blocks of time indices) all land on that XCD, so a pair's buffers and its
// library's table and lists are read through one L2.  Grid = 8 * ceil(np / 8) * nb
// workgroups; returns false for the spare ones.
__device__ __forceinline__ bool xcd_pair_block(int b, int np, int nb, int& slot, int& tb) {
  const int per = (np + kXcdA - 1) / kXcdA;
  const int x = b % kXcdA, q = b / kXcdA;
  const int r = q / nb;
  tb = q % nb;
  slot = x * per + r;
  return r < per && slot < np;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) s += red[w];
  return s;
}

__global__ __launch_bounds__(kBwThreads) void bw_pair_kernel(
    const float* __restrict__ ts, int64_t ld, int L, const int* __restrict__ nbr_idx,
    const float* __restrict__ nbr_w, const int* __restrict__ lib_E, int n_lib, int k_max, int tau,
    const int* __restrict__ pair_lib, const int* __restrict__ pair_tgt,
    const float* __restrict__ grad_rho, float* __restrict__ yhat, float* __restrict__ H,
    float* __restrict__ Gy, int* __restrict__ pair_ok, float* __restrict__ ycol,
    const int* __restrict__ perm, int n_pairs) {
  __shared__ double red[kBwThreads / kWave];
  extern __shared__ float yl[];   // the pair's target column, [L]
  int slot, tb;
  if (!xcd_pair_block(blockIdx.x, n_pairs, 1, slot, tb)) return;   // whole workgroup
  const int p = perm ? perm[slot] : slot;
  const int i = pair_lib[p];
  const int j = pair_tgt[p];
  const int E = (i >= 0 && i < n_lib) ? lib_E[i] : 0;
  const int k = E + 1;
  const int lo = (E - 1) * tau;
  bool ok = i >= 0 && i < n_lib && j >= 0 && j < ld && E >= 1 && E <= kEMax && k <= k_max &&
            L - lo >= k + 1;
  if (ok) ok = nbr_idx[((size_t)i * L + lo) * k_max] >= 0;
  float* yh = yhat + (size_t)p * L;
  float* hp = H + (size_t)p * L;
  float* gp = Gy + (size_t)p * L;
  if (!ok) {
    for (int t = threadIdx.x; t < L; t += blockDim.x) hp[t] = gp[t] = yh[t] = 0.0f;
    if (threadIdx.x == 0) pair_ok[p] = 0;
    return;
  }
  // the target column, read once from the panel: LDS for this kernel, a contiguous copy
  // in the workspace for the coefficient kernel
  float* yc = ycol + (size_t)p * L;
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    const float v = ts[(int64_t)t * ld + j];
    yl[t] = v;
    yc[t] = v;
  }
  __syncthreads();
  double sy = 0.0, sp = 0.0;
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    float v = 0.0f;
    if (t >= lo) {
      const int* ri = nbr_idx + ((size_t)i * L + t) * k_max;
      const float* rw = nbr_w + ((size_t)i * L + t) * k_max;
      for (int m = 0; m < k; ++m)
        if (ri[m] >= 0) v = fmaf(rw[m], yl[ri[m]], v);   // -1: padding
      sy += yl[t];
      sp += v;
    }
    yh[t] = v;
  }
  const double n = (double)(L - lo);
  const double ybar = block_sum(sy, red) / n;
  const double pbar = block_sum(sp, red) / n;
  double a = 0.0, b = 0.0, c = 0.0, ay = 0.0, bp = 0.0;
  for (int t = lo + threadIdx.x; t < L; t += blockDim.x) {
    const double y = yl[t];
    const double q = yh[t];
    a += (y - ybar) * (y - ybar);
    b += (q - pbar) * (q - pbar);
    c += (y - ybar) * (q - pbar);
    ay += y * y;
    bp += q * q;
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  c = block_sum(c, red);
  ay = block_sum(ay, red);
  bp = block_sum(bp, red);
  const bool good = a > 1e-10 * ay && b > 1e-10 * bp;
  const double g = grad_rho[p];
  const double sab = sqrt(a * b);
  const double rho = good ? c / sab : 0.0;
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    double h = 0.0, gy = 0.0;
    if (good && t >= lo) {
      const double dy = (double)yl[t] - ybar;
      const double dq = (double)yh[t] - pbar;
      h = g * (dy / sab - rho * dq / b);
      gy = g * (dq / sab - rho * dy / a);
    }
    hp[t] = (float)h;
    gp[t] = (float)gy;
  }
  if (threadIdx.x == 0) pair_ok[p] = good ? 1 : 0;
}

// coef = dbar_m / d_m (0 for zero distances), one thread per (pair, t), written twice: m-major
// (com[p][m][t], read by the query side) and in the library's transposed order (coT[p][q] at
// q = pos[m][t], read by the neighbour side).  Only entries that step reads are written: rows
// t >= (E-1) tau, m < E + 1, pairs with a finite rho.
// One row's coefficients at a compile-time k = E + 1, so the per-neighbour FP64 distances
// and kernel values stay in registers (the weighted target h y(n_m) is re-read).  The table
// row and its list positions are read m-major (stride L), so consecutive t in consecutive
// lanes read contiguous runs; the library series and the target column sit in LDS.
__device__ __forceinline__ double coef_wb(const float* yc, int nb, double h) {
  return nb < 0 ? 0.0 : h * (double)yc[nb];
}
template <int K>
__device__ __forceinline__ void coef_row(const float* x, const float* yc, const int* im,
                                         const int* pm, int t, int tau, double h, int L,
                                         float* cm_out, float* cT) {
  constexpr int E = K - 1;
  int ri[K];
  double d[K], u[K];
#pragma unroll
  for (int m = 0; m < K; ++m) ri[m] = im[(size_t)m * L];
  // the K distances advance one lag at a time, so the K reads of a lag are independent
  // (each sum still runs over the lags in order)
#pragma unroll
  for (int m = 0; m < K; ++m) d[m] = 0.0;
#pragma unroll 1
  for (int e = 0; e < E; ++e) {
    const double xt = x[t - e * tau];
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const double df = xt - (double)x[(ri[m] < 0 ? t : ri[m]) - e * tau];
      d[m] += df * df;
    }
  }
#pragma unroll
  for (int m = 0; m < K; ++m) d[m] = ri[m] < 0 ? INFINITY : sqrt(d[m]);   // padding: no distance
  const double d1 = d[0];
  double S = 0.0;
#pragma unroll
  for (int m = 0; m < K; ++m) {
    u[m] = ri[m] < 0 ? 0.0 : d1 > 0.0 ? exp(-d[m] / d1) : (d[m] == 0.0 ? 1.0 : 0.0);
    S += u[m];
  }
  double sw = 0.0;
#pragma unroll
  for (int m = 0; m < K; ++m) sw += coef_wb(yc, ri[m], h) * (u[m] / S);
  double dbar1 = 0.0;
#pragma unroll
  for (int m = 1; m < K; ++m) {
    double cm = 0.0;
    if (ri[m] >= 0 && d1 > 0.0 && d[m] > 0.0) {
      const double ub = (coef_wb(yc, ri[m], h) - sw) / S;
      const double db = -ub * u[m] / d1;
      dbar1 += ub * u[m] * d[m] / (d1 * d1);
      cm = db / d[m];
    }
    cm_out[(size_t)m * L] = (float)cm;
    if (ri[m] >= 0 && ri[m] < L) cT[pm[(size_t)m * L]] = (float)cm;
  }
  const float c0 = d1 > 0.0 ? (float)(dbar1 / d1) : 0.0f;
  cm_out[0] = c0;
  if (ri[0] >= 0 && ri[0] < L) cT[pm[0]] = c0;
}

__global__ __launch_bounds__(256) void bw_coef_kernel(
    int L, const float* __restrict__ lib_ts, const int* __restrict__ lib_E, int k_max, int tau,
    const int* __restrict__ pair_lib, int n_pairs, const float* __restrict__ H,
    const int* __restrict__ pair_ok, const int* __restrict__ pos_m, const int* __restrict__ idx_m,
    const float* __restrict__ ycol, float* __restrict__ com, float* __restrict__ coT,
    const int* __restrict__ perm) {
  extern __shared__ float sm[];   // the library series [L], then the target column [L]
  int slot, tb;
  if (!xcd_pair_block(blockIdx.x, n_pairs, (L + 255) / 256, slot, tb)) return;   // whole workgroup
  const int p = perm ? perm[slot] : slot;
  if (!pair_ok[p]) return;   // whole workgroup: the rows step skips the pair
  const int i = pair_lib[p];
  const int E = lib_E[i];   // pair_ok guarantees 1 <= E <= 20 and E + 1 <= k_max
  const int K = E + 1;
  const int lo = (E - 1) * tau;
  if (tb * 256 + 255 < lo) return;   // whole workgroup: no query row in this block
  float* x = sm;
  float* yc = sm + L;
  for (int q = threadIdx.x; q < L; q += blockDim.x) {
    x[q] = lib_ts[(size_t)i * L + q];
    yc[q] = ycol[(size_t)p * L + q];
  }
  __syncthreads();
  const int t = tb * 256 + threadIdx.x;
  if (t >= L || t < lo) return;
  const int* im = idx_m + (size_t)i * k_max * L + t;   // [m][t]
  const int* pm = pos_m + (size_t)i * k_max * L + t;   // [m][t]
  float* cm_out = com + (size_t)p * k_max * L + t;     // [m][t]
  float* cT = coT + (size_t)p * L * k_max;             // transposed order
  const double h = H[(size_t)p * L + t];
  if (im[0] < 0) {   // a row of padding (a subsampled table): no contribution
    for (int m = 0; m < K; ++m) {
      cm_out[(size_t)m * L] = 0.0f;
      const int nb = im[(size_t)m * L];
      if (nb >= 0 && nb < L) cT[pm[(size_t)m * L]] = 0.0f;
    }
    return;
  }
  switch (E) {
#define CCM_K(EE) \
  case EE: coef_row<EE + 1>(x, yc, im, pm, t, tau, h, L, cm_out, cT); break;
    CCM_K(1) CCM_K(2) CCM_K(3) CCM_K(4) CCM_K(5) CCM_K(6) CCM_K(7) CCM_K(8) CCM_K(9) CCM_K(10)
    CCM_K(11) CCM_K(12) CCM_K(13) CCM_K(14) CCM_K(15) CCM_K(16) CCM_K(17) CCM_K(18) CCM_K(19)
    CCM_K(20)
#undef CCM_K
    default: break;
  }
}

// Transposed neighbour relation of each library's table: for every time s, the entries
// (t, m) with n_m(t) = s, in increasing (t, m) order, packed as t * 32 + m.  Counts and
// offsets in LDS; one wave then walks the rows in order (the k neighbours of a row are
// distinct, so its lanes never write the same list), which keeps the order deterministic.
// The walk loads kTrRows rows at a time before placing them, so one load latency is paid
// per group of rows rather than per row.  Also written: each entry's list position and an
// m-major copy of the table ([m][t] each, rows t >= (E-1) tau, m < k), and the weights in
// list order.
constexpr int kTrThreads = 256;
constexpr int kTrRows = 16;

__global__ __launch_bounds__(kTrThreads) void bw_transpose_kernel(
    const int* __restrict__ nbr_idx, const float* __restrict__ nbr_w, const int* __restrict__ lib_E,
    int L, int k_max, int tau, int* __restrict__ csr_off, int* __restrict__ csr_ent,
    int* __restrict__ pos_m, float* __restrict__ csr_w, int* __restrict__ idx_m) {
  extern __shared__ int cnt[];          // [L + 1], then chunk sums [kTrThreads]
  int* csum = cnt + L + 1;
  const int i = blockIdx.x;
  const int E = lib_E[i];
  const int k = E + 1;
  const bool ok = E >= 1 && E <= kEMax && k <= k_max;
  const int lo = ok ? (E - 1) * tau : L;
  for (int q = threadIdx.x; q <= L; q += blockDim.x) cnt[q] = 0;
  __syncthreads();
  const int* tab = nbr_idx + (size_t)i * L * k_max;
  int* im = idx_m + (size_t)i * k_max * L;
  for (int q = threadIdx.x; q < (L - lo) * k; q += blockDim.x) {
    const int t = lo + q / k, m = q % k;
    const int s = tab[(size_t)t * k_max + m];
    im[(size_t)m * L + t] = s;
    if (s >= 0 && s < L) atomicAdd(&cnt[s], 1);
  }
  __syncthreads();
  // exclusive scan of cnt[0..L): per-thread chunks, then the chunk sums
  const int chunk = (L + kTrThreads - 1) / kTrThreads;
  const int c0 = min((int)threadIdx.x * chunk, L), c1 = min(c0 + chunk, L);
  int acc = 0;
  for (int q = c0; q < c1; ++q) {
    const int c = cnt[q];
    cnt[q] = acc;
    acc += c;
  }
  csum[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int th = 0; th < kTrThreads; ++th) {
      const int c = csum[th];
      csum[th] = run;
      run += c;
    }
    cnt[L] = run;
  }
  __syncthreads();
  for (int q = c0; q < c1; ++q) cnt[q] += csum[threadIdx.x];
  __syncthreads();
  int* off = csr_off + (size_t)i * (L + 1);
  for (int q = threadIdx.x; q <= L; q += blockDim.x) off[q] = cnt[q];
  __syncthreads();
  int* ent = csr_ent + (size_t)i * L * k_max;
  int* pos = pos_m + (size_t)i * k_max * L;
  float* cw = csr_w + (size_t)i * L * k_max;
  const float* wtab = nbr_w + (size_t)i * L * k_max;
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    for (int t0 = lo; t0 < L; t0 += kTrRows) {
      int sv[kTrRows];
      float wv[kTrRows];
#pragma unroll
      for (int r = 0; r < kTrRows; ++r) {
        const bool in = lane < k && t0 + r < L;
        sv[r] = in ? tab[(size_t)(t0 + r) * k_max + lane] : -1;
        wv[r] = in ? wtab[(size_t)(t0 + r) * k_max + lane] : 0.0f;
      }
#pragma unroll
      for (int r = 0; r < kTrRows; ++r) {
        const int s = sv[r];
        if (s >= 0 && s < L) {
          const int q = cnt[s]++;
          ent[q] = (t0 + r) * 32 + lane;
          pos[(size_t)lane * L + t0 + r] = q;
          cw[q] = wv[r];
        }
      }
    }
  }
}

// Everything that lands on time s, in two steps.  For time u, lag e and s = u - e tau:
//   R(u, e) = sum_m c[u][m] (x(s) - x(n_m(u) - e tau))              (u as a query row, u >= lo)
//           - sum_q c(q) (x(t_q - e tau) - x(s))                     (u as a neighbour: the
//                                                                     entries q = (t_q, m) of
//                                                                     u's transposed list)
//   TT(u)   = sum_q w(q) H(t_q)
// The library gradient at s is sum_e R(s + e tau, e) and the target gradient is
// Gy(s) + TT(s): the same terms as summing over the rows and lists that reach s, each
// difference formed before its product as there.  Step one (bw_rows_kernel) reads table row
// u and u's list once and keeps the E partial sums in FP64 registers; step two
// (bw_sum_kernel) adds the E of them that land on s.  Every row and list was read E times
// (once per s that needs it) when each s gathered for itself.
template <int E>
__device__ __forceinline__ void rows_at(const float* x, const float* hp, int u, int L, int lo,
                                        int tau, const float* cm, const int* im, const int* off,
                                        const int* ent, const float* cw, const float* cT,
                                        double* sr) {
  constexpr int K = E + 1;
  double TT = 0.0, R[E], xs[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    R[e] = 0.0;
    const int s = u - e * tau;   // the time this lag of u lands on (none if negative)
    xs[e] = s >= 0 ? (double)x[s] : 0.0;
  }
  if (u >= lo) {   // u as a query row (then u - e tau >= 0 for every e < E)
#pragma unroll 1
    for (int m = 0; m < K; ++m) {
      const int n = im[(size_t)m * L + u];
      if (n < 0) continue;   // padding
      const double c = cm[(size_t)m * L + u];
#pragma unroll
      for (int e = 0; e < E; ++e) R[e] += c * (xs[e] - (double)x[n - e * tau]);
    }
  }
  for (int q = off[u]; q < off[u + 1]; ++q) {   // u as a neighbour
    const int v = ent[q];
    const int t = v >> 5, m = v & 31;
    if (t < lo || t >= L || m >= K) continue;   // only a malformed table (repeated neighbours)
    const double c = cT[q];
    TT += (double)cw[q] * (double)hp[t];
#pragma unroll
    for (int e = 0; e < E; ++e) R[e] -= c * ((double)x[t - e * tau] - xs[e]);
  }
  sr[0] = TT;
#pragma unroll
  for (int e = 0; e < E; ++e) sr[(size_t)(1 + e) * L] = R[e];
}

// Step one: one thread per (pair, u); writes TT(u), R(u, e) to sr[p][0 | 1 + e][u] (FP64).
__global__ __launch_bounds__(256) void bw_rows_kernel(
    int L, const float* __restrict__ lib_ts, const int* __restrict__ lib_E, int k_max, int tau,
    const int* __restrict__ pair_lib, int n_pairs, const float* __restrict__ H,
    const int* __restrict__ pair_ok, const float* __restrict__ com, const float* __restrict__ coT,
    const int* __restrict__ csr_off, const int* __restrict__ csr_ent, const float* __restrict__ csr_w,
    const int* __restrict__ idx_m, double* __restrict__ srb, const int* __restrict__ perm) {
  extern __shared__ float sm[];   // the library series [L], then the pair's H [L]
  int slot, tb;
  if (!xcd_pair_block(blockIdx.x, n_pairs, (L + 255) / 256, slot, tb)) return;   // whole workgroup
  const int p = perm ? perm[slot] : slot;
  if (!pair_ok[p]) return;   // the whole workgroup: the second step writes zeros
  const int i = pair_lib[p];
  const int E = lib_E[i];
  const int lo = (E - 1) * tau;
  // the series and H are read at scattered times: from LDS
  float* x = sm;
  float* hp = sm + L;
  for (int q = threadIdx.x; q < L; q += blockDim.x) {
    x[q] = lib_ts[(size_t)i * L + q];
    hp[q] = H[(size_t)p * L + q];
  }
  __syncthreads();
  const int u = tb * blockDim.x + threadIdx.x;
  if (u >= L) return;
  const float* cm = com + (size_t)p * k_max * L;       // [m][t]
  const float* cT = coT + (size_t)p * L * k_max;       // transposed order
  const int* im = idx_m + (size_t)i * k_max * L;       // [m][t]
  const int* off = csr_off + (size_t)i * (L + 1);
  const int* ent = csr_ent + (size_t)i * L * k_max;
  const float* cw = csr_w + (size_t)i * L * k_max;
  double* sr = srb + (size_t)p * (kEMax + 1) * L + u;
  switch (E) {   // pair_ok guarantees 1 <= E <= 20
#define CCM_E(EE) \
  case EE: rows_at<EE>(x, hp, u, L, lo, tau, cm, im, off, ent, cw, cT, sr); break;
    CCM_E(1) CCM_E(2) CCM_E(3) CCM_E(4) CCM_E(5) CCM_E(6) CCM_E(7) CCM_E(8) CCM_E(9) CCM_E(10)
    CCM_E(11) CCM_E(12) CCM_E(13) CCM_E(14) CCM_E(15) CCM_E(16) CCM_E(17) CCM_E(18) CCM_E(19)
    CCM_E(20)
#undef CCM_E
    default: break;
  }
}

// Step two: one thread per (pair, s): tc[p][s] = Gy(s) + TT(s) (target), lc[p][s] =
// sum_e R(s + e tau, e) (library); zeros for a pair whose rho is NaN.
__global__ __launch_bounds__(256) void bw_sum_kernel(
    int L, const int* __restrict__ lib_E, int tau, const int* __restrict__ pair_lib, int n_pairs,
    const float* __restrict__ Gy, const int* __restrict__ pair_ok, const double* __restrict__ srb,
    float* __restrict__ tc, float* __restrict__ lc, const int* __restrict__ perm) {
  int slot, tb;
  if (!xcd_pair_block(blockIdx.x, n_pairs, (L + 255) / 256, slot, tb)) return;
  const int p = perm ? perm[slot] : slot;
  const int s = tb * blockDim.x + threadIdx.x;
  if (s >= L) return;
  float* tco = tc + (size_t)p * L;
  float* lco = lc + (size_t)p * L;
  if (!pair_ok[p]) {
    tco[s] = 0.0f;
    lco[s] = 0.0f;
    return;
  }
  const int E = lib_E[pair_lib[p]];
  const int lo = (E - 1) * tau;
  const double* sr = srb + (size_t)p * (kEMax + 1) * L;
  double Lb = 0.0;
  for (int e = 0; e < E; ++e) {
    const int u = s + e * tau;
    if (u >= L) break;
    Lb += sr[(size_t)(1 + e) * L + u];
  }
  const double T = (s >= lo ? (double)Gy[(size_t)p * L + s] : 0.0) + sr[s];
  tco[s] = (float)T;
  lco[s] = (float)Lb;
}

// Pairs of a chunk grouped by library (a counting sort in LDS, for up to kOrderMaxLib
// libraries): the per-pair kernels take pair perm[b] at position b, so pairs of one library
// run together and share its table, lists and series in L2.  Only the processing order
// changes: every pair writes its own buffers, and the contributions are added in pair order
// afterwards.
constexpr int kOrderThreads = 1024;
constexpr int kOrderMaxLib = 16384;

__global__ __launch_bounds__(kOrderThreads) void bw_pair_order_kernel(
    const int* __restrict__ pair_lib, int np, int n_lib, int* __restrict__ perm) {
  extern __shared__ int cnt[];   // [n_lib + 1] (bucket n_lib: library ids out of range)
  int* csum = cnt + n_lib + 1;   // [kOrderThreads]
  const int nb = n_lib + 1;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    const int i = pair_lib[p];
    atomicAdd(&cnt[(i >= 0 && i < n_lib) ? i : n_lib], 1);
  }
  __syncthreads();
  const int chunk = (nb + kOrderThreads - 1) / kOrderThreads;
  const int c0 = min((int)threadIdx.x * chunk, nb), c1 = min(c0 + chunk, nb);
  int acc = 0;
  for (int q = c0; q < c1; ++q) {
    const int c = cnt[q];
    cnt[q] = acc;
    acc += c;
  }
  csum[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int th = 0; th < kOrderThreads; ++th) {
      const int c = csum[th];
      csum[th] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int q = c0; q < c1; ++q) cnt[q] += csum[threadIdx.x];
  __syncthreads();
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    const int i = pair_lib[p];
    perm[atomicAdd(&cnt[(i >= 0 && i < n_lib) ? i : n_lib], 1)] = p;
  }
}

// grad_ts[s][tgt_p] += tc[p][s], grad_lib[lib_p][s] += lc[p][s], pairs in order.  One wave
// per (64 consecutive s, hash h): it takes the pairs whose target (for grad_ts) or library
// (for grad_lib) is congruent to h modulo kRedHash, in pair order, so every output element
// is summed by one lane in pair order.  The pair list is read 64 entries at a time.
constexpr int kRedHash = 64;

__global__ __launch_bounds__(kWave) void bw_reduce_kernel(
    int64_t ld, int L, const int* __restrict__ pair_lib, const int* __restrict__ pair_tgt,
    int n_pairs, const int* __restrict__ pair_ok, const float* __restrict__ tc,
    const float* __restrict__ lc, float* __restrict__ grad_ts, float* __restrict__ grad_lib) {
  const int lane = lane_id();
  const int s = blockIdx.x * kWave + lane;
  const int h = blockIdx.y;
  const bool in = s < L;
  for (int p0 = 0; p0 < n_pairs; p0 += kWave) {
    const int pc = p0 + lane;
    const bool okp = pc < n_pairs && pair_ok[pc] != 0;
    const int tg = okp ? pair_tgt[pc] : -1;
    const int lb = okp ? pair_lib[pc] : -1;
    uint64_t mt = grad_ts ? ballot(okp && tg % kRedHash == h) : 0;
    uint64_t ml = grad_lib ? ballot(okp && lb % kRedHash == h) : 0;
    uint64_t mall = mt | ml;
    while (mall) {
      const int b = __builtin_ctzll(mall);
      mall &= mall - 1;
      const int p = p0 + b;
      if ((mt >> b) & 1) {
        const int j = readlane(tg, b);
        if (in) grad_ts[(int64_t)s * ld + j] += tc[(size_t)p * L + s];
      }
      if ((ml >> b) & 1) {
        const int i = readlane(lb, b);
        if (in) grad_lib[(size_t)i * L + s] += lc[(size_t)p * L + s];
      }
    }
  }
}

}  // namespace ccm

static size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

// Pairs are processed in chunks whose per-pair buffers fit in 4 GiB (and of at most 65,535
// pairs).  Chunks run in pair order and each adds its pairs into the
// gradients in pair order, so the result does not depend on the chunk size.
static constexpr size_t kBwChunkBytes = (size_t)4 << 30;

static size_t bw_pair_bytes(int L, int k_max) {
  return 6 * (size_t)L * 4 + 2 * (size_t)L * k_max * 4 + (size_t)(ccm::kEMax + 1) * L * 8 + 8;
}

extern "C" int ccm_backward_chunk_pairs(int L, int k_max) {
  size_t c = kBwChunkBytes / bw_pair_bytes(L, k_max);
  if (c < 1) c = 1;
  if (c > 65535) c = 65535;
  return (int)c;
}

extern "C" size_t ccm_backward_ws_bytes(int L, int n_lib, int n_pairs, int k_max) {
  // per pair of a chunk: yhat, H, Gy, tc, lc, the target column ([P][L] floats each), the
  // coefficients twice ([P][k_max][L] and [P][L k_max] floats), pair_ok and the processing
  // order ([P] ints each), the per-time partial sums ([P][21][L] doubles); per library: CSR
  // offsets [L + 1], entries, positions, weights and the m-major table copy, [L k_max] each
  const int chunk = ccm_backward_chunk_pairs(L, k_max);
  const size_t P = (size_t)(n_pairs < chunk ? n_pairs : chunk);
  const size_t a = up256(P * L * 4);
  const size_t c = up256(P * L * k_max * 4);
  const size_t t = up256((size_t)n_lib * L * k_max * 4);
  return 6 * a + 2 * c + up256(P * 4) + up256((size_t)n_lib * (L + 1) * 4) + 4 * t +
         up256(P * 4) +                                  // the pairs' processing order
         up256(P * (ccm::kEMax + 1) * L * 8);            // per-time partial sums (FP64)
}

extern "C" hipError_t ccm_launch_backward(const float* ts, int64_t ld, int L, const float* lib_ts,
                                          const int* nbr_idx, const float* nbr_w, const int* lib_E,
                                          int n_lib, int k_max, int tau, const int* pair_lib,
                                          const int* pair_tgt, const float* grad_rho, int n_pairs,
                                          float* grad_ts, float* grad_lib, void* ws,
                                          hipStream_t stream) {
  if (n_pairs == 0) return hipSuccess;
  const int chunk = ccm_backward_chunk_pairs(L, k_max);
  const size_t P = (size_t)(n_pairs < chunk ? n_pairs : chunk);
  const size_t a = up256(P * L * 4);
  char* base = (char*)ws;
  float* yhat = (float*)base;
  float* H = (float*)(base + a);
  float* Gy = (float*)(base + 2 * a);
  float* tc = (float*)(base + 3 * a);
  float* lc = (float*)(base + 4 * a);
  const size_t c = up256(P * L * k_max * 4);
  const size_t tb = up256((size_t)n_lib * L * k_max * 4);
  float* ycol = (float*)(base + 5 * a);
  float* com = (float*)(base + 6 * a);
  float* coT = (float*)(base + 6 * a + c);
  char* after_coef = base + 6 * a + 2 * c;
  int* pair_ok = (int*)after_coef;
  int* csr_off = (int*)(after_coef + up256(P * 4));
  int* csr_ent = (int*)((char*)csr_off + up256((size_t)n_lib * (L + 1) * 4));
  int* pos_m = (int*)((char*)csr_ent + tb);
  float* csr_w = (float*)((char*)pos_m + tb);
  int* idx_m = (int*)((char*)csr_w + tb);
  int* perm = (int*)((char*)idx_m + tb);
  double* srb = (double*)((char*)perm + up256(P * 4));
  static std::atomic<uint64_t> attr{0};
  hipError_t e = ccm::allow_lds_once((const void*)ccm::bw_transpose_kernel, attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ccm::bw_transpose_kernel, dim3(n_lib), dim3(ccm::kTrThreads),
                     (size_t)(L + 1 + ccm::kTrThreads) * sizeof(int), stream, nbr_idx, nbr_w, lib_E,
                     L, k_max, tau, csr_off, csr_ent, pos_m, csr_w, idx_m);
  static std::atomic<uint64_t> attr_pair{0};
  e = ccm::allow_lds_once((const void*)ccm::bw_pair_kernel, attr_pair);
  if (e != hipSuccess) return e;
  static std::atomic<uint64_t> attr_coef{0};
  e = ccm::allow_lds_once((const void*)ccm::bw_coef_kernel, attr_coef);
  if (e != hipSuccess) return e;
  static std::atomic<uint64_t> attr_rows{0};
  e = ccm::allow_lds_once((const void*)ccm::bw_rows_kernel, attr_rows);
  if (e != hipSuccess) return e;
  static std::atomic<uint64_t> attr_order{0};
  e = ccm::allow_lds_once((const void*)ccm::bw_pair_order_kernel, attr_order);
  if (e != hipSuccess) return e;
  const bool sorted = n_lib <= ccm::kOrderMaxLib;
  const int* pord = sorted ? (const int*)perm : nullptr;
  for (int p0 = 0; p0 < n_pairs; p0 += chunk) {
    const int np = n_pairs - p0 < chunk ? n_pairs - p0 : chunk;
    const int* pl = pair_lib + p0;
    const int* pt = pair_tgt + p0;
    if (sorted)
      hipLaunchKernelGGL(ccm::bw_pair_order_kernel, dim3(1), dim3(ccm::kOrderThreads),
                         (size_t)(n_lib + 1 + ccm::kOrderThreads) * sizeof(int), stream, pl, np,
                         n_lib, perm);
    // XCD-aware grids (xcd_pair_block): 8 * ceil(np / 8) slots, times the time blocks
    const unsigned slots = (unsigned)((np + ccm::kXcdA - 1) / ccm::kXcdA * ccm::kXcdA);
    const unsigned tblocks = (unsigned)((L + 255) / 256);
    hipLaunchKernelGGL(ccm::bw_pair_kernel, dim3(slots), dim3(ccm::kBwThreads), (size_t)L * sizeof(float),
                       stream, ts, ld, L, nbr_idx, nbr_w, lib_E, n_lib, k_max, tau, pl, pt,
                       grad_rho + p0, yhat, H, Gy, pair_ok, ycol, pord, np);
    hipLaunchKernelGGL(ccm::bw_coef_kernel, dim3(slots * tblocks), dim3(256),
                       (size_t)2 * L * sizeof(float), stream, L, lib_ts, lib_E, k_max, tau, pl, np,
                       H, pair_ok, pos_m, idx_m, ycol, com, coT, pord);
    hipLaunchKernelGGL(ccm::bw_rows_kernel, dim3(slots * tblocks), dim3(256),
                       (size_t)2 * L * sizeof(float), stream, L, lib_ts, lib_E, k_max, tau, pl, np,
                       H, pair_ok, com, coT, csr_off, csr_ent, csr_w, idx_m, srb, pord);
    hipLaunchKernelGGL(ccm::bw_sum_kernel, dim3(slots * tblocks), dim3(256), 0, stream, L, lib_E,
                       tau, pl, np, Gy, pair_ok, srb, tc, lc, pord);
    hipLaunchKernelGGL(ccm::bw_reduce_kernel, dim3((L + ccm::kWave - 1) / ccm::kWave, ccm::kRedHash),
                       dim3(ccm::kWave), 0, stream, ld, L, pl, pt, np, pair_ok, tc, lc, grad_ts,
                       grad_lib);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
