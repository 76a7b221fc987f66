// Exact k-nearest-neighbour search on delay embeddings, and simplex-projection optE.
//
// Method: Sec. III-B of the paper (Alg. 3 / Alg. 4: all-pairs distances between embedded
// points, then the E+1 smallest per query), the weights of Sec. III-A ("normalize":
// exponential scale, each row normalised) and the simplex projection of Sec. II-B scored
// per E as in Alg. 1 phase 1.
//
// gfx950 design (not the paper's): one wavefront owns one query point.  Its 64 lanes
// evaluate 64 candidate points at a time straight from an LDS copy of the series (the
// embedding is never materialised), and the k best so far live in a sorted list spread
// across lanes 0..k-1 (lane j holds the j-th nearest).  A candidate enters only if its d^2
// beats the current k-th (one compare per lane, one ballot per chunk); the rare winners are
// inserted one at a time, in ascending time order, by a DPP wave shift.  Because
// candidates arrive in ascending time order, "strictly smaller d^2" is exactly the
// (d^2, time index) order, so ties go to the lower index with no extra work.
//
// Selection distances follow one canonical FP32 operation sequence (lag 0 first; one rounding per
// subtraction, product and sum; no fused multiply-add: this file is compiled with
// -ffp-contract=off), so the selected indices are bit-identical to any implementation
// that follows the same sequence.  For the E scan of optE the squared distance of E is
// the E-1 value plus one term, so one pass over the lags serves all E at once, each E
// with its own list.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "wave.h"

#pragma clang fp contract(off)

namespace ccm {

// Insert candidate (v, sv) into the wave-distributed ascending list (ld, li).  Entries
// equal to v stay ahead of it (they carry lower time indices).
__device__ __forceinline__ void list_insert(float& ld, int& li, float v, int sv) {
  float pd = wave_shr1(ld, -INFINITY);
  int pi = wave_shr1(li, -1);
  bool gt = ld > v;
  bool gtp = pd > v;
  float nd = gtp ? pd : v;
  int ni = gtp ? pi : sv;
  ld = gt ? nd : ld;
  li = gt ? ni : li;
}

// Offer this chunk's candidates (cand = +inf where not admissible) to one list.
// `k1` is k - 1, the lane holding the current k-th smallest.
__device__ __forceinline__ void offer_chunk(float cand, int base, float& ld, int& li, float& thr,
                                            int k1) {
  uint64_t m = ballot(cand < thr);
  while (m) {
    int src = __ffsll((unsigned long long)m) - 1;
    float v = readlane(cand, src);
    list_insert(ld, li, v, base + src);
    thr = readlane(ld, k1);
    m &= (~0ull << src) << 1;
    m &= ballot(cand < thr);
  }
}

// Simplex weights of a finished list (lanes 0..k-1 hold neighbour n_j of query t).  The
// distance of each selected neighbour is recomputed in FP64 from the series (k x E terms,
// negligible next to the scan), so the weights do not depend on FP32 rounding or
// underflow of d^2: u = exp(-d/d1); when d1 = 0, u = 1 on zero distances, 0 elsewhere.
// Returns u (lanes >= k: 0) and the wave-wide sum of u in `usum`.
__device__ __forceinline__ double list_weight64(const float* x, int t, int nb, int E, int tau,
                                                int k, double& usum) {
  const int lane = lane_id();
  const bool in = lane < k && nb >= 0;
  double dd = 0.0;
  if (in)
    for (int e = 0; e < E; ++e) {
      double df = (double)x[t - e * tau] - (double)x[nb - e * tau];
      dd += df * df;
    }
  const double d = sqrt(dd);
  const double d1 = __hiloint2double(readlane(__double2hiint(d), 0), readlane(__double2loint(d), 0));
  double u = 0.0;
  if (in) u = d1 > 0.0 ? exp(-d / d1) : (d == 0.0 ? 1.0 : 0.0);
  usum = wave_sum(u);
  return u;
}

// ---------------------------------------------------------------------------------------
// Neighbour tables at each library's own E (one launch for every E).
// grid.x = n_lib, block = 256 (4 waves); LDS: the library series.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void knn_table_kernel(const float* __restrict__ ts, int64_t ld,
                                                        int L, const int* __restrict__ lib_ids,
                                                        const int* __restrict__ lib_E, int tau,
                                                        int Tp, int k_max, int* __restrict__ nbr_idx,
                                                        float* __restrict__ nbr_w,
                                                        float* __restrict__ nbr_d2) {
  extern __shared__ float x[];
  const int lib = blockIdx.x;
  const int sid = lib_ids[lib];
  for (int t = threadIdx.x; t < L; t += blockDim.x) x[t] = ts[(int64_t)t * ld + sid];
  __syncthreads();

  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int E = lib_E[lib];
  const int k = E + 1;
  const int lo = (E - 1) * tau;           // first point
  const int hi = L - 1 - Tp;              // last point with a future
  const bool ok = E >= 1 && E <= kEMax && k <= k_max && (hi - lo + 1) - 1 >= k;
  const size_t rowbase = (size_t)lib * L;

  for (int t = wave; t < L; t += nw) {
    int* oi = nbr_idx + (rowbase + t) * k_max;
    float* ow = nbr_w + (rowbase + t) * k_max;
    float* od = nbr_d2 ? nbr_d2 + (rowbase + t) * k_max : nullptr;
    if (!ok || t < lo || t > hi) {
      if (lane < k_max) {
        oi[lane] = -1;
        ow[lane] = 0.0f;
        if (od) od[lane] = INFINITY;
      }
      continue;
    }
    float xq[kEMax];
#pragma unroll
    for (int e = 0; e < kEMax; ++e) xq[e] = (e < E) ? x[t - e * tau] : 0.0f;

    float ldist = INFINITY;
    int lidx = -1;
    float thr = INFINITY;
    for (int base = lo; base <= hi; base += kWave) {
      const int s = base + lane;
      const bool inr = s <= hi;
      const int sc = inr ? s : hi;
      float acc = 0.0f;
#pragma unroll
      for (int e = 0; e < kEMax; ++e) {
        if (e < E) {
          float df = xq[e] - x[sc - e * tau];
          acc = acc + df * df;
        }
      }
      float cand = (inr && s != t) ? acc : INFINITY;
      offer_chunk(cand, base, ldist, lidx, thr, k - 1);
    }
    double usum;
    double u = list_weight64(x, t, lidx, E, tau, k, usum);
    if (lane < k_max) {
      bool in = lane < k;
      oi[lane] = in ? lidx : -1;
      ow[lane] = in ? (float)(u / usum) : 0.0f;
      if (od) od[lane] = in ? ldist : INFINITY;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Simplex projection skill for E = E_min..E_max and optE, one workgroup per series.
// LOO: Q_E = C_E = [(E-1)tau, L-1-Tp], query excluded.  HALF: C_E = [(E-1)tau, h-1-Tp],
// Q_E = [h+(E-1)tau, L-1-Tp], h = L/2, no exclusion.
// ---------------------------------------------------------------------------------------
constexpr int kSimplexThreads = 512;

__global__ __launch_bounds__(kSimplexThreads) void simplex_kernel(
    const float* __restrict__ ts, int64_t ld, int L, const int* __restrict__ ids, int E_min,
    int E_max, int tau, int Tp, int mode, int* __restrict__ optE, float* __restrict__ rho_E) {
  extern __shared__ float x[];
  __shared__ double wsum[kSimplexThreads / kWave][kEMax][5];
  const int sid = ids[blockIdx.x];
  for (int t = threadIdx.x; t < L; t += blockDim.x) x[t] = ts[(int64_t)t * ld + sid];
  __syncthreads();

  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const bool half = mode == 1;
  const int h = L / 2;
  const int qbase = half ? h : 0;
  const int chi = half ? h - 1 - Tp : L - 1 - Tp;     // last candidate
  const int clo = (E_min - 1) * tau;                   // first candidate over all E
  const int qlo = qbase + (E_min - 1) * tau;
  const int qhi = L - 1 - Tp;

  // lane e holds the five FP64 moment sums of E = e + 1
  double m_o = 0.0, m_oo = 0.0, m_p = 0.0, m_pp = 0.0, m_op = 0.0;

  for (int t = qlo + wave; t <= qhi; t += nw) {
    float xq[kEMax];
#pragma unroll
    for (int e = 0; e < kEMax; ++e) xq[e] = (e < E_max && t - e * tau >= 0) ? x[t - e * tau] : 0.0f;
    float ldist[kEMax];
    int lidx[kEMax];
    float thr[kEMax];
#pragma unroll
    for (int e = 0; e < kEMax; ++e) {
      ldist[e] = INFINITY;
      lidx[e] = -1;
      thr[e] = INFINITY;
    }
    for (int base = clo; base <= chi; base += kWave) {
      const int s = base + lane;
      const bool inr = s <= chi;
      const int sc = inr ? s : chi;
      float acc = 0.0f;
#pragma unroll
      for (int e = 0; e < kEMax; ++e) {
        if (e < E_max) {
          const int xi = sc - e * tau;
          float df = xq[e] - x[xi > 0 ? xi : 0];
          acc = acc + df * df;
          const int E = e + 1;
          if (E >= E_min && t >= qbase + (E - 1) * tau) {
            const bool adm = inr && sc >= (E - 1) * tau && (half || s != t);
            float cand = adm ? acc : INFINITY;
            offer_chunk(cand, base, ldist[e], lidx[e], thr[e], E);
          }
        }
      }
    }
    const float obs = x[t + Tp];
#pragma unroll
    for (int e = 0; e < kEMax; ++e) {
      const int E = e + 1;
      if (e < E_max && E >= E_min && t >= qbase + (E - 1) * tau) {
        double usum;
        double u = list_weight64(x, t, lidx[e], E, tau, E + 1, usum);
        double f = (lane <= E && lidx[e] >= 0) ? (double)x[lidx[e] + Tp] : 0.0;
        double pred = wave_sum(u * f) / usum;
        if (lane == e) {
          double o = obs, p = pred;
          m_o += o;
          m_oo += o * o;
          m_p += p;
          m_pp += p * p;
          m_op += o * p;
        }
      }
    }
  }
  if (lane < kEMax) {
    wsum[wave][lane][0] = m_o;
    wsum[wave][lane][1] = m_oo;
    wsum[wave][lane][2] = m_p;
    wsum[wave][lane][3] = m_pp;
    wsum[wave][lane][4] = m_op;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nE = E_max - E_min + 1;
    double best = 0.0;
    int bestE = E_min;
    bool have = false;
    for (int E = E_min; E <= E_max; ++E) {
      double s[5] = {0, 0, 0, 0, 0};
      for (int w = 0; w < nw; ++w)
        for (int c = 0; c < 5; ++c) s[c] += wsum[w][E - 1][c];
      const int qfirst = qbase + (E - 1) * tau;
      const double n = (double)(qhi - qfirst + 1);
      double r = n > 0 ? pearson_from_moments(n, s[0], s[1], s[2], s[3], s[4]) : __builtin_nan("");
      if (rho_E) rho_E[(size_t)blockIdx.x * nE + (E - E_min)] = (float)r;
      if (r == r && (!have || r > best)) {
        best = r;
        bestE = E;
        have = true;
      }
    }
    optE[blockIdx.x] = bestE;
  }
}

// ---------------------------------------------------------------------------------------
// Explicit delay embedding: emb[i][r][e] = x_i(r + (E-1)tau - e tau).
// ---------------------------------------------------------------------------------------
__global__ void embed_kernel(const float* __restrict__ ts, int64_t ld, int L,
                             const int* __restrict__ ids, int n, int E, int tau,
                             float* __restrict__ emb) {
  const int nr = L - (E - 1) * tau;
  const int64_t total = (int64_t)n * nr * E;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(g % E);
    const int64_t re = g / E;
    const int r = (int)(re % nr);
    const int i = (int)(re / nr);
    const int t = r + (E - 1) * tau - e * tau;
    emb[g] = ts[(int64_t)t * ld + ids[i]];
  }
}

}  // namespace ccm

// ---- launchers (called from the C ABI) ----------------------------------------------
extern "C" hipError_t ccm_launch_knn(const float* ts, int64_t ld, int L, const int* lib_ids,
                                     const int* lib_E, int n_lib, int tau, int Tp, int k_max,
                                     int* nbr_idx, float* nbr_w, float* nbr_d2,
                                     hipStream_t stream) {
  if (n_lib == 0) return hipSuccess;
  size_t lds = (size_t)L * sizeof(float);
  hipLaunchKernelGGL(ccm::knn_table_kernel, dim3(n_lib), dim3(256), lds, stream, ts, ld, L, lib_ids,
                     lib_E, tau, Tp, k_max, nbr_idx, nbr_w, nbr_d2);
  return hipGetLastError();
}

extern "C" hipError_t ccm_launch_simplex(const float* ts, int64_t ld, int L, const int* ids, int n,
                                         int E_min, int E_max, int tau, int Tp, int mode,
                                         int* optE, float* rho_E, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  size_t lds = (size_t)L * sizeof(float);
  hipLaunchKernelGGL(ccm::simplex_kernel, dim3(n), dim3(ccm::kSimplexThreads), lds, stream, ts, ld,
                     L, ids, E_min, E_max, tau, Tp, mode, optE, rho_E);
  return hipGetLastError();
}

extern "C" hipError_t ccm_launch_embed(const float* ts, int64_t ld, int L, const int* ids, int n,
                                       int E, int tau, float* emb, hipStream_t stream) {
  int64_t total = (int64_t)n * (L - (E - 1) * tau) * E;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(ccm::embed_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, ts, ld, L, ids,
                     n, E, tau, emb);
  return hipGetLastError();
}
