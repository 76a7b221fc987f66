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
// across lanes 0..k-1 (lane j holds the j-th nearest by (d^2, time index)).  A candidate
// can enter only if its d^2 does not exceed the current k-th (one compare per lane, one
// ballot per chunk); the few survivors are inserted one at a time by a DPP wave shift.
// A wave walks consecutive queries and seeds each list from the previous query's
// neighbours shifted one step (the optE scan pools the shifted lists of E - 1, E and
// E + 1); the first query of a range scans the chunk around its own time first instead.
// Either way the k-th distance is tight early and later chunks rarely insert.  The list
// order is lexicographic in (d^2, time index), so the scan order does not change the
// result and ties go to the lower index.
//
// Selection distances follow one canonical FP32 operation sequence (lag 0 first; one rounding per
// subtraction, product and sum; no fused multiply-add: this file is compiled with
// -ffp-contract=off), so the selected indices are bit-identical to any implementation
// that follows the same sequence.  For the E scan of optE the squared distance of E is
// the E-1 value plus one term, so one pass over the lags serves every E of a group of
// four, each E with its own list.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "wave.h"

#pragma clang fp contract(off)

namespace ccm {

// A list entry is the 64-bit key (bits of d^2) << 32 | time index: d^2 >= 0, so its IEEE
// bits order like the value, and comparing keys as unsigned integers is exactly the
// (d^2, time index) order.  Empty slots and inadmissible candidates hold ~0.
__device__ __forceinline__ uint64_t nkey(float d2, int s) {
  return ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)s;
}
__device__ __forceinline__ float key_d2(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ int key_idx(uint64_t k) { return (int)(uint32_t)k; }

__device__ __forceinline__ uint64_t readlane(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// Insert key kv into the wave-distributed ascending list (lane j = j-th smallest).  A key
// larger than the k-th entry lands at lane k or beyond, outside the list.
__device__ __forceinline__ void list_insert(uint64_t& key, uint64_t kv) {
  const uint32_t plo = (uint32_t)wave_shr1((int)(uint32_t)key, 0);
  const uint32_t phi = (uint32_t)wave_shr1((int)(uint32_t)(key >> 32), 0);
  const uint64_t prev = ((uint64_t)phi << 32) | plo;  // lane 0: 0, below every key
  const bool gt = key > kv;
  const bool gtp = prev > kv;
  const uint64_t nk = gtp ? prev : kv;
  key = gt ? nk : key;
}

// Offer this chunk's candidate keys (~0 where not admissible) to one list whose k-th entry
// sits in lane k1; `thr` is that entry's key.  Survivors are inserted one at a time; a key
// already in the list (a seed met again by the scan) is skipped.
__device__ __forceinline__ void offer_chunk(uint64_t cand, uint64_t& key, uint64_t& thr, int k1) {
  uint64_t m = ballot(cand < thr);
  while (m) {
    const int src = __ffsll((unsigned long long)m) - 1;
    const uint64_t kv = readlane(cand, src);
    m &= (~0ull << src) << 1;
    if (ballot(key == kv) == 0) {   // a key met again leaves the list and its k-th as they are
      list_insert(key, kv);
      thr = readlane(key, k1);
      m &= ballot(cand < thr);
    }
  }
}

// First chunk base of the scan: the 64 points centred on the query, inside [clo, chi].
__device__ __forceinline__ int window_base(int t, int clo, int chi) {
  int b = t - 32;
  if (b > chi - (kWave - 1)) b = chi - (kWave - 1);
  if (b < clo) b = clo;
  return b;
}

// The series sits in LDS after kPad zeros, so x[-kPad .. -1] reads 0 and lag reads at
// tau = 1 need no clamp, and before kWave zeros, so the lanes of a last chunk that lie past
// the final candidate read zeros (they are never admitted) without clamping their index.
constexpr int kPad = 32;

// Lag values x[sc - e tau], e = 0..NL-1, of the candidate at sc; all NL reads are issued
// before the arithmetic.  With tau = 1 they are one base address plus immediate offsets.
template <int NL, bool TAU1>
__device__ __forceinline__ void lag_values(const float* x, int sc, int tau, float (&xs)[NL]) {
  if constexpr (TAU1) {
    // one unsigned byte address (never negative: x is preceded by kPad >= NL zeros) plus
    // immediate offsets
    const char* lds0 = (const char*)(x - kPad);
    const uint32_t a = (uint32_t)(sc + kPad - (NL - 1)) * 4u;
#pragma unroll
    for (int e = 0; e < NL; ++e) xs[e] = *(const float*)(lds0 + a + 4u * (NL - 1 - e));
  } else {
#pragma unroll
    for (int e = 0; e < NL; ++e) {
      const int xi = sc - e * tau;
      xs[e] = x[xi > 0 ? xi : 0];
    }
  }
}

// Lag values x[sc - e tau] for e = A..NL-1 only (the addressing of lag_values<NL>).
template <int A, int NL, bool TAU1>
__device__ __forceinline__ void lag_range(const float* x, int sc, int tau, float (&xs)[NL]) {
  if constexpr (TAU1) {
    const char* lds0 = (const char*)(x - kPad);
    const uint32_t a = (uint32_t)(sc + kPad - (NL - 1)) * 4u;
#pragma unroll
    for (int e = A; e < NL; ++e) xs[e] = *(const float*)(lds0 + a + 4u * (NL - 1 - e));
  } else {
#pragma unroll
    for (int e = A; e < NL; ++e) {
      const int xi = sc - e * tau;
      xs[e] = x[xi > 0 ? xi : 0];
    }
  }
}

// Build a sorted list from the distinct candidate keys in lanes 0..k1 (~0 where empty): an
// empty entry becomes ~0 - lane, so all k1 + 1 keys differ and stay above every real key
// (their index reads negative); a key's rank among them is its lane in the list, and a
// forward permute moves it there.  Lanes past k1 read ~0.  The keys pass through a
// per-wave LDS row and every lane reads them back at uniform addresses (broadcast reads):
// one compare per key instead of two lane reads and a compare.  A wave's LDS operations
// complete in program order, so its reads see its own writes.
constexpr int kMaxWaves = 16;

__device__ __forceinline__ void list_from_keys(uint64_t cand, int k1, uint64_t& key,
                                               uint64_t& thr) {
  __shared__ uint64_t rank_keys[kMaxWaves][32];
  const int lane = lane_id();
  const bool mine = lane <= k1;
  const uint64_t v = !mine ? ~0ull : (cand == ~0ull ? ~0ull - (uint64_t)lane : cand);
  uint64_t* rk = rank_keys[__builtin_amdgcn_readfirstlane(threadIdx.x / kWave)];
  if (lane < 32) rk[lane] = v;
  int rank = 0;
  for (int j = 0; j <= k1; ++j) rank += rk[j] < v ? 1 : 0;
  const int dst = (mine ? rank : lane) << 2;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(dst, (int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(dst, (int)(uint32_t)(v >> 32));
  key = ((uint64_t)hi << 32) | lo;
  thr = readlane(key, k1);
}

// Build a sorted list of k1 + 1 entries from the distinct keys of pool lanes 0..np-1 (~0
// where empty, np <= 64), as list_from_keys does for k1 + 1 keys, but over the pool's real
// keys only: they are packed into the wave's LDS row in lane order, each gets its rank among
// them, the other lanes take the ranks after them in lane order, and all 64 lanes are
// permuted by rank (a bijection), so lanes 0..k1 hold the k1 + 1 smallest in order.  An
// empty entry of rank r becomes ~0 - (63 - r): distinct, ascending, above every real key,
// with a negative index.
__device__ __forceinline__ void list_from_pool(uint64_t cand, int np, int k1, uint64_t& key,
                                               uint64_t& thr) {
  __shared__ uint64_t pool_keys[kMaxWaves][kWave];
  const int lane = lane_id();
  const bool real = lane < np && cand != ~0ull;
  const uint64_t rm = ballot(real);
  const int nr = __popcll(rm);
  const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(rm >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)rm, 0));
  uint64_t* rk = pool_keys[__builtin_amdgcn_readfirstlane(threadIdx.x / kWave)];
  if (real) rk[below] = cand;
  int rank = 0;
  for (int j = 0; j < nr; ++j) rank += rk[j] < cand ? 1 : 0;
  rank = real ? rank : nr + (lane - below);
  const uint64_t v = real ? cand : ~0ull - (uint64_t)(kWave - 1 - rank);
  const int dst = rank << 2;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(dst, (int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(dst, (int)(uint32_t)(v >> 32));
  key = ((uint64_t)hi << 32) | lo;
  thr = readlane(key, k1);
}

// The k-th distance of a list as a float bound for a prefilter: +inf while the list is not
// full (its k-th key is empty), else the d^2 of the k-th key.  A candidate can enter the
// list only if its d^2 <= this bound.
__device__ __forceinline__ float thr_float(uint64_t thr) {
  const uint32_t hi = (uint32_t)(thr >> 32);
  return hi == 0xFFFFFFFFu ? INFINITY : __uint_as_float(hi);
}

// Seed a list for query t from the previous query's list: its neighbours shifted one step
// forward are admissible candidates (with their canonical d^2 at this E) and usually lie
// close to t's true neighbours, so the k-th distance starts tight and the scan that
// follows inserts few candidates.  `key` holds the previous query's list (lanes 0..E) on
// entry and the seeded list on exit.  Candidates run to `chi`; (E-1)*tau is the first.
template <int E, bool TAU1, int NQ>
__device__ __forceinline__ void seed_list(const float* x, const uint8_t* mb, int t, int tau,
                                          int chi, bool excl_self, const float (&xq)[NQ],
                                          uint64_t& key, uint64_t& thr) {
  const int lane = lane_id();
  const int nb = lane <= E ? key_idx(key) : -1;
  const int s = nb + 1;
  bool ok = nb >= 0 && s <= chi && (!excl_self || s != t);
  if (mb) ok = ok && mb[ok ? s : 0] != 0;
  const int sc = ok ? s : (E - 1) * tau;
  float xs[E];
  lag_values<E, TAU1>(x, sc, tau, xs);
  float acc = 0.0f;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const float df = xq[e] - xs[e];
    acc = acc + df * df;
  }
  list_from_keys(ok ? nkey(acc, s) : ~0ull, E, key, thr);
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
  usum = lanes32_sum(u);   // k <= 21: the list lives in lanes 0..31
  return u;
}

// Sum over each 32-lane half (lanes 0..31 and 32..63), returned in every lane of that half:
// the steps of lanes32_sum run in all four rows of 16 at once, so the upper half's sum is the
// same sequence of operations on its own lanes.
__device__ __forceinline__ double halves32_sum(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x124>(v);
  v += dpp_f64<0x128>(v);
  auto rl = [&](int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
  };
  const double lo = rl(0) + rl(16);
  const double hi = rl(32) + rl(48);
  return lane_id() < 32 ? lo : hi;
}

// Simplex weights of two finished lists at once: list a of E in lanes 0..E, list b of E + 1
// in lanes 32..33 + E (lane 32 + j holds its j-th neighbour).  Each half forms its own
// weights exactly as list_weight64 does for one list.  The query's lag values come from the
// wave's scalar copy xq (x[t - e tau]), and every lane issues the reads of its neighbour's
// E + 1 lags together (the last lag counts in the upper half only).
template <int E, bool TAU1, int NQ>
__device__ __forceinline__ double pair_weight64(const float* x, const float (&xq)[NQ], int nb,
                                                int tau, double& usum) {
  static_assert(E + 1 <= NQ, "the query's lags cover the upper list");
  const int lane = lane_id();
  const bool up = lane >= 32;
  const int El = up ? E + 1 : E;
  const bool in = (lane & 31) <= El && nb >= 0;
  float xs[E + 1];
  lag_values<E + 1, TAU1>(x, in ? nb : E * tau, tau, xs);
  double dd = 0.0;
#pragma unroll
  for (int e = 0; e <= E; ++e) {
    const double df = (double)xq[e] - (double)xs[e];
    if (e < E) dd += df * df;
    else dd = up ? dd + df * df : dd;
  }
  if (!in) dd = 0.0;
  const double d = sqrt(dd);
  const double d1a = __hiloint2double(readlane(__double2hiint(d), 0), readlane(__double2loint(d), 0));
  const double d1b = __hiloint2double(readlane(__double2hiint(d), 32), readlane(__double2loint(d), 32));
  const double d1 = up ? d1b : d1a;
  double u = 0.0;
  if (in) u = d1 > 0.0 ? exp(-d / d1) : (d == 0.0 ? 1.0 : 0.0);
  usum = halves32_sum(u);
  return u;
}

constexpr int kKnnThreads = 1024;

// The scan of one query at a compile-time E: every candidate chunk's lag reads are issued
// together, then the canonical d^2 is formed in lag order.  With `seeded`, key/thr are
// seeded from the previous query's list and all chunks are scanned in order; otherwise the
// list starts empty and the window around t is scanned first.
template <int E, bool TAU1>
__device__ __forceinline__ void knn_query(const float* x, const uint8_t* mb, int t, int lo,
                                          int hi, int tau, bool seeded, uint64_t& key,
                                          uint64_t& thr) {
  const int lane = lane_id();
  float xq[kEMax];
#pragma unroll
  for (int e = 0; e < kEMax; ++e)
    xq[e] = e < E ? __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x[t - e * tau])))
                  : 0.0f;
  if (seeded) {
    seed_list<E, TAU1, kEMax>(x, mb, t, tau, hi, true, xq, key, thr);
  } else {
    key = ~0ull;
    thr = ~0ull;
  }
  const int wb = seeded ? hi + 1 : window_base(t, lo, hi);
  const uint32_t xw = seeded ? 0 : kWave;
  // pass -1: the window around t (unseeded only); then every chunk in order
  for (int pass = seeded ? 0 : -1, base = lo; base <= hi;
       base += (pass < 0 ? 0 : kWave), pass = 0) {
    const int b = pass < 0 ? wb : base;
    const int s = b + lane;
    const bool inr = s <= hi && (uint32_t)(s - wb) >= (pass < 0 ? 0u : xw);
    // lags 0..CHK-1 first; when no lane is still within the list's bound (d^2 only grows
    // with the lags), the chunk ends there
    constexpr int CHK = E >= 9 ? E - 4 : 0;
    float xs[E];
    lag_values<E, TAU1>(x, s, tau, xs);
    float acc = 0.0f;
#pragma unroll
    for (int e = 0; e < CHK; ++e) {
      const float df = xq[e] - xs[e];
      acc = acc + df * df;
    }
    if (CHK == 0 || ballot(acc <= thr_float(thr)) != 0) {
#pragma unroll
      for (int e = CHK; e < E; ++e) {
        const float df = xq[e] - xs[e];
        acc = acc + df * df;
      }
      bool adm = inr && s != t;
      if (mb) adm = adm && mb[adm ? s : 0] != 0;   // library subsample: only marked candidates
      const uint64_t cand = adm ? nkey(acc, s) : ~0ull;
      offer_chunk(cand, key, thr, E);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Neighbour tables at each library's own E (one launch for every E).
// grid.x = n_lib, block = 1024 (16 waves, one query each at a time); LDS: the series.
// ---------------------------------------------------------------------------------------
// At most 64 VGPRs (8 waves per SIMD), so two 16-wave workgroups share a CU: 2.96 -> 2.70 ms
// for 512 tables at L = 1600, 40.1 -> 35.4 ms for 10,240, with no spill.
__global__ __launch_bounds__(kKnnThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void knn_table_kernel(const float* __restrict__ ts, int64_t ld,
                                                        int L, const int* __restrict__ lib_ids,
                                                        const int* __restrict__ lib_E, int tau,
                                                        int Tp, int k_max,
                                                        const uint8_t* __restrict__ cand_mask,
                                                        int* __restrict__ nbr_idx,
                                                        float* __restrict__ nbr_w,
                                                        float* __restrict__ nbr_d2) {
  extern __shared__ float xbuf[];
  float* x = xbuf + kPad;
  // optional candidate mask of this library (a library subsample), after the series and its
  // zero tail
  uint8_t* mb = cand_mask ? (uint8_t*)(xbuf + L + kPad + kWave) : nullptr;
  __shared__ int n_adm;
  const int lib = blockIdx.x;
  const int sid = lib_ids[lib];
  const bool sid_ok = sid >= 0 && sid < ld;   // a series outside the panel gets padding
  const int E = __builtin_amdgcn_readfirstlane(lib_E[lib]);
  const int k = E + 1;
  const int lo = (E - 1) * tau;           // first point
  const int hi = L - 1 - Tp;              // last point with a future
  if (threadIdx.x == 0) n_adm = 0;
  for (int t = threadIdx.x; t < L + kPad + kWave; t += blockDim.x)
    xbuf[t] = t < kPad || t >= L + kPad || !sid_ok ? 0.0f : ts[(int64_t)(t - kPad) * ld + sid];
  if (mb)
    for (int t = threadIdx.x; t < L; t += blockDim.x) mb[t] = cand_mask[(size_t)lib * L + t];
  __syncthreads();
  bool ok = sid_ok && E >= 1 && E <= kEMax && k <= k_max && (hi - lo + 1) - 1 >= k;
  if (mb && ok) {   // enough marked candidates for every query (one may be the query itself)
    int c = 0;
    for (int t = lo + threadIdx.x; t <= hi; t += blockDim.x) c += mb[t] != 0;
    if (c) atomicAdd(&n_adm, c);
    __syncthreads();
    ok = n_adm - 1 >= k;
  }

  const int lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int nw = blockDim.x / kWave;
  const size_t rowbase = (size_t)lib * L;

  // padding rows (outside [lo, hi], or every row of an unusable library)
  for (int t = wave; t < L; t += nw) {
    if (ok && t >= lo && t <= hi) continue;
    if (lane < k_max) {
      nbr_idx[(rowbase + t) * k_max + lane] = -1;
      nbr_w[(rowbase + t) * k_max + lane] = 0.0f;
      if (nbr_d2) nbr_d2[(rowbase + t) * k_max + lane] = INFINITY;
    }
  }
  if (!ok) return;
  // each wave walks a contiguous range of queries, seeding each list from the previous one
  const int nq = hi - lo + 1;
  const int per = (nq + nw - 1) / nw;
  const int tb = __builtin_amdgcn_readfirstlane(lo + wave * per);   // the same in every lane
  const int te = __builtin_amdgcn_readfirstlane(min(tb + per, hi + 1));
  uint64_t key = ~0ull, thr = ~0ull;
  for (int t = tb; t < te; ++t) {
    const bool seeded = t > tb;
    switch (E) {
#define CCM_E(EE)                                                 \
  case EE:                                                        \
    if (tau == 1)                                                 \
      knn_query<EE, true>(x, mb, t, lo, hi, tau, seeded, key, thr);  \
    else                                                              \
      knn_query<EE, false>(x, mb, t, lo, hi, tau, seeded, key, thr); \
    break;
      CCM_E(1) CCM_E(2) CCM_E(3) CCM_E(4) CCM_E(5) CCM_E(6) CCM_E(7) CCM_E(8) CCM_E(9) CCM_E(10)
      CCM_E(11) CCM_E(12) CCM_E(13) CCM_E(14) CCM_E(15) CCM_E(16) CCM_E(17) CCM_E(18) CCM_E(19)
      CCM_E(20)
#undef CCM_E
      default:
        break;
    }
    const float ldist = key_d2(key);
    const int lidx = key_idx(key);
    double usum;
    double u = list_weight64(x, t, lane < k ? lidx : -1, E, tau, k, usum);
    if (lane < k_max) {
      const bool in = lane < k && lidx >= 0;
      nbr_idx[(rowbase + t) * k_max + lane] = in ? lidx : -1;
      nbr_w[(rowbase + t) * k_max + lane] = in ? (float)(u / usum) : 0.0f;
      if (nbr_d2) nbr_d2[(rowbase + t) * k_max + lane] = in ? ldist : INFINITY;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Simplex projection skill, one workgroup per (series, E group).  Groups are fixed (the
// table below) and clipped to [E_min, E_max].  The squared distance is accumulated over lags
// 0..EHI-1 once; each E of the group keeps its own list.  LOO: Q_E = C_E = [(E-1)tau,
// L-1-Tp], query excluded.  HALF: C_E = [(E-1)tau, h-1-Tp], Q_E = [h+(E-1)tau, L-1-Tp],
// h = L/2, no exclusion.  Writes the FP64 skill of each E to rho64[series][E-1].
// The kernel waits on LDS and on its serial list updates far more than it computes, so the
// groups are kept small (four lists: about 80 VGPRs) and the kernel runs at kSimplexOcc
// waves per SIMD even at the cost of a small spill; the lags a group repeats are cheap next
// to that.
// ---------------------------------------------------------------------------------------
// 8-wave workgroups; 16-wave ones for long series, where a workgroup's LDS (the series, the
// bitmaps) would otherwise let fewer than kSimplexOcc waves per SIMD share a CU; 4-wave ones
// for calls over many series
constexpr int kSimplexThreads = 512;
constexpr int kSimplexMinThreads = 256;
constexpr int kSimplexMaxThreads = 1024;
constexpr int kSimplexOcc = 8;
// (group, first E, last E); every group holds an even number of lists
#define CCM_SIMPLEX_GROUPS(X) X(0, 1, 4) X(1, 5, 8) X(2, 9, 12) X(3, 13, 16) X(4, 17, 20)
constexpr int kNGroups = 5;
constexpr int kGroupE = 4;   // most lists in a group
__device__ __forceinline__ int group_lo(int g) {
#define CCM_LO(G, LO, HI) if (g == G) return LO;
  CCM_SIMPLEX_GROUPS(CCM_LO)
#undef CCM_LO
  return 1;
}
__device__ __forceinline__ int group_hi(int g) {
#define CCM_HI(G, LO, HI) if (g == G) return HI;
  CCM_SIMPLEX_GROUPS(CCM_HI)
#undef CCM_HI
  return 0;
}

// Seed every list of the group that held a list at the previous query (t - 1 >= its first
// query); lists starting at t begin empty.  List E is seeded from a pool: the previous
// query's lists of E, E - 1 and E + 1 (those of this group), each neighbour shifted one step
// forward.  Nearby E share most neighbours, and their union holds more of t's true
// neighbours than one list does, so the k-th distance starts tighter and the scan inserts
// fewer candidates.  A neighbour met in two lists enters the pool once (the first lane to
// set its bit in the wave's LDS bitmap `bm` keeps it; the bits are cleared again at once).
// `prev` carries the previous list's old index (this query's seeding has overwritten key).
template <int ELO, int G, int NG, bool TAU1, int EHI>
__device__ __forceinline__ void seed_group(const float* x, int t, int tau, int chi, bool half,
                                           int qbase, int E_lo, int E_hi,
                                           const float (&xq)[EHI], uint64_t (&key)[NG],
                                           uint64_t (&thr)[NG], uint32_t* bm, int prev) {
  if constexpr (G < NG) {
    constexpr int E = ELO + G;
    const int lane = lane_id();
    const int own = key_idx(key[G]);   // this list's previous entries, before it is reseeded
    const int qE = qbase + (E - 1) * tau;
    if (E >= E_lo && E <= E_hi && t - 1 >= qE) {
      // pool lanes: [0, E] own entries; then the E entries of list E - 1 (G > 0); then the
      // E + 2 entries of list E + 1 (G + 1 < NG): at most 3 E + 3 <= 63 lanes
      constexpr int off_hi = (E + 1) + (G > 0 ? E : 0);
      constexpr int np = off_hi + (G + 1 < NG ? E + 2 : 0);
      int nb = lane <= E ? own : -1;
      if constexpr (G > 0) {
        const int src = lane - (E + 1);
        const int v = __builtin_amdgcn_ds_bpermute((src >= 0 ? src : 0) << 2, prev);
        if (lane > E && lane < off_hi) nb = v;
      }
      if constexpr (G + 1 < NG) {
        const int src = lane - off_hi;
        const int v = __builtin_amdgcn_ds_bpermute((src >= 0 ? src : 0) << 2, key_idx(key[G + 1]));
        if (lane >= off_hi && lane < np) nb = v;
      }
      const int s = nb + 1;
      bool ok = nb >= 0 && s <= chi && s >= (E - 1) * tau && (half || s != t);
      if (ok) {   // keep the first lane holding s
        const uint32_t bit = 1u << (s & 31);
        ok = (atomicOr(&bm[s >> 5], bit) & bit) == 0u;
      }
      if (nb >= 0 && s <= chi && s >= 0) atomicAnd(&bm[s >> 5], ~(1u << (s & 31)));
      const int sc = ok ? s : (E - 1) * tau;
      float xs[E];
      lag_values<E, TAU1>(x, sc, tau, xs);
      float acc = 0.0f;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const float df = xq[e] - xs[e];
        acc = acc + df * df;
      }
      list_from_pool(ok ? nkey(acc, s) : ~0ull, np, E, key[G], thr[G]);
    }
    seed_group<ELO, G + 1, NG, TAU1, EHI>(x, t, tau, chi, half, qbase, E_lo, E_hi, xq, key, thr,
                                          bm, own);
  }
}

// The FP64 finish of the lists of E = ELO + G and ELO + G + 1 at query t (the second moves
// to lanes 32..63), then the next pair.
template <int ELO, int G, int NG, bool TAU1, int EHI>
__device__ __forceinline__ void finish_pairs(const float* x, const float (&xq)[EHI], int t,
                                             int tau, int Tp, int E_lo, int E_hi, int qbase,
                                             int lane, const uint64_t (&key)[NG], float obs,
                                             double* wm) {
  if constexpr (G < NG) {
    constexpr int Ea = ELO + G;
    const bool acta = Ea >= E_lo && Ea <= E_hi && t >= qbase + (Ea - 1) * tau;
    const bool actb = Ea + 1 >= E_lo && Ea + 1 <= E_hi && t >= qbase + Ea * tau;
    if (acta || actb) {
      const bool up = lane >= 32;
      const uint32_t blo = (uint32_t)__shfl_xor((int)(uint32_t)key[G + 1], 32);
      const uint32_t bhi = (uint32_t)__shfl_xor((int)(uint32_t)(key[G + 1] >> 32), 32);
      const uint64_t kk = up ? (((uint64_t)bhi << 32) | blo) : key[G];
      const int El = up ? Ea + 1 : Ea;
      const bool act = up ? actb : acta;
      const int li = (act && (lane & 31) <= El) ? key_idx(kk) : -1;
      double usum;
      double u = pair_weight64<Ea, TAU1, EHI>(x, xq, li, tau, usum);
      double f = ((lane & 31) <= El && li >= 0) ? (double)x[li + Tp] : 0.0;
      double pred = halves32_sum(u * f) / usum;
      const double pb = __hiloint2double(readlane(__double2hiint(pred), 32),
                                         readlane(__double2loint(pred), 32));
      if ((lane == G && acta) || (lane == G + 1 && actb)) {
        double o = obs, p = lane == G ? pred : pb;
        double* q = wm + lane * 5;
        q[0] += o;
        q[1] += o * o;
        q[2] += p;
        q[3] += p * p;
        q[4] += o * p;
      }
    }
    finish_pairs<ELO, G + 2, NG, TAU1, EHI>(x, xq, t, tau, Tp, E_lo, E_hi, qbase, lane, key, obs,
                                            wm);
  }
}

template <int ELO, int EHI, bool TAU1>
__device__ __forceinline__ void simplex_group(const float* x, int L, int E_min, int E_max, int tau,
                                              int Tp, bool half, int wave, int nw, uint32_t* bm,
                                              double (&wsum)[kSimplexMaxThreads / kWave][kGroupE][5]) {
  constexpr int NG = EHI - ELO + 1;
  const int lane = lane_id();
  const int E_lo = ELO > E_min ? ELO : E_min;
  const int E_hi = EHI < E_max ? EHI : E_max;
  const int h = L / 2;
  const int qbase = half ? h : 0;
  const int chi = half ? h - 1 - Tp : L - 1 - Tp;     // last candidate
  const int clo = (E_lo - 1) * tau;                    // first candidate over the group
  const int qlo = qbase + (E_lo - 1) * tau;
  const int qhi = L - 1 - Tp;

  // the five FP64 moment sums of E = ELO + g accumulate in wsum[wave][g] (LDS, updated once
  // per query by lane g), so the scan holds no moment registers
  double* wm = &wsum[wave][0][0];
  if (lane < kGroupE)
    for (int c = 0; c < 5; ++c) wm[lane * 5 + c] = 0.0;

  // each wave walks a contiguous range of queries; every list is carried from one query to
  // the next and re-seeded with its shifted neighbours
  const int nq = qhi - qlo + 1;
  const int per = nq > 0 ? (nq + nw - 1) / nw : 0;
  // the range is the same in every lane; reading it from the first lane keeps the query and
  // chunk loops under scalar control (the compiler otherwise kept their counters in vector
  // registers and left them through exec masks)
  const int tb = __builtin_amdgcn_readfirstlane(qlo + wave * per);
  const int te = __builtin_amdgcn_readfirstlane(min(tb + per, qhi + 1));
  uint64_t key[NG];
  uint64_t thr[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) key[g] = thr[g] = ~0ull;
  for (int t = tb; t < te; ++t) {
    float xq[EHI];
#pragma unroll
    for (int e = 0; e < EHI; ++e)
      xq[e] = __int_as_float(__builtin_amdgcn_readfirstlane(
          __float_as_int(t - e * tau >= 0 ? x[t - e * tau] : 0.0f)));
    const bool seeded = t > tb;
    if (seeded) seed_group<ELO, 0, NG, TAU1, EHI>(x, t, tau, chi, half, qbase, E_lo, E_hi, xq,
                                                  key, thr, bm, -1);
    // prefilter bound per list: -1 for a list not active at t (nothing passes)
    float tf[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int E = ELO + g;
      tf[g] = (E >= E_lo && E <= E_hi && t >= qbase + (E - 1) * tau) ? thr_float(thr[g]) : -1.0f;
    }
    // the largest bound of the group at the start of the scan (bounds only fall during it)
    float tfmax = tf[0];
#pragma unroll
    for (int g = 1; g < NG; ++g) tfmax = fmaxf(tfmax, tf[g]);
    // the window of candidates around t first when some list starts empty (HALF mode:
    // candidates are in the other half, so the window clamps to its end), then every chunk
    // in order.  Candidates that are never admissible start at d^2 = +inf; a list takes the
    // exact path (full admissibility, 64-bit keys) only when some lane passes its bound.
    const bool win = !seeded || t - 1 < qbase + (E_hi - 1) * tau;
    const int wb = win ? window_base(t, clo, chi) : chi + 1;
    const uint32_t xw = win ? kWave : 0;
    for (int pass = win ? -1 : 0, base = clo; base <= chi;
         base += (pass < 0 ? 0 : kWave), pass = 0) {
      const int b = pass < 0 ? wb : base;
      const int s = b + lane;
      const bool inr = s <= chi && (uint32_t)(s - wb) >= (pass < 0 ? 0u : xw);
      const bool okc = inr && (half || s != t);
      // lags 0..CHK-1 first; when no candidate of the chunk is still within the group's
      // largest bound (d^2 only grows with the lags), the chunk ends there
      constexpr int CHK = ELO >= 9 ? ELO - 4 : 0;
      float xs[EHI];
      lag_range<0, EHI, TAU1>(x, s, tau, xs);
      float acc = okc ? 0.0f : INFINITY;
#pragma unroll
      for (int e = 0; e < CHK; ++e) {
        const float df = xq[e] - xs[e];
        acc = acc + df * df;
      }
      if (CHK == 0 || ballot(acc <= tfmax) != 0) {
#pragma unroll
        for (int e = CHK; e < EHI; ++e) {
          const float df = xq[e] - xs[e];
          acc = acc + df * df;
          if (e + 1 >= ELO) {
            const int g = (e + 1 - ELO) >= 0 ? (e + 1 - ELO) : 0;
            if (ballot(acc <= tf[g]) != 0) {
              const int E = e + 1;
              const bool adm = okc && s >= (E - 1) * tau;
              offer_chunk(adm ? nkey(acc, s) : ~0ull, key[g], thr[g], E);
              tf[g] = thr_float(thr[g]);
            }
          }
        }
      }
    }
    const float obs = x[t + Tp];
    // the lists of E and E + 1 are finished together: the second moves to lanes 32..63
    static_assert(NG % 2 == 0, "lists are finished in pairs");
    finish_pairs<ELO, 0, NG, TAU1, EHI>(x, xq, t, tau, Tp, E_lo, E_hi, qbase, lane, key, obs, wm);
  }
}

__global__ __launch_bounds__(kSimplexMaxThreads) __attribute__((amdgpu_waves_per_eu(kSimplexOcc, kSimplexOcc))) void simplex_kernel(
    const float* __restrict__ ts, int64_t ld, int L, const int* __restrict__ ids, int E_min,
    int E_max, int tau, int Tp, int mode, double* __restrict__ rho64) {
  // dynamic LDS: the series between kPad and kWave zeros, then each wave's bitmap over
  // times (W words)
  extern __shared__ float xbuf[];
  float* x = xbuf + kPad;
  __shared__ double wsum[kSimplexMaxThreads / kWave][kGroupE][5];
  const int grp = kNGroups - 1 - (int)blockIdx.y;   // the groups of larger E (longer) first
  const int series = blockIdx.x;
  const int ELO = group_lo(grp);
  const int EHI = group_hi(grp);
  const int E_lo = ELO > E_min ? ELO : E_min;
  const int E_hi = EHI < E_max ? EHI : E_max;
  if (E_lo > E_hi) return;  // whole workgroup: group outside [E_min, E_max]
  const int sid = ids[series];
  if (sid < 0 || sid >= ld) {   // a series outside the panel: NaN skills, so optE = E_min
    if ((int)threadIdx.x >= E_lo - 1 && (int)threadIdx.x < E_hi)
      rho64[(size_t)series * kEMax + threadIdx.x] = __builtin_nan("");
    return;
  }
  for (int t = threadIdx.x; t < L + kPad + kWave; t += blockDim.x)
    xbuf[t] = t < kPad || t >= L + kPad ? 0.0f : ts[(int64_t)(t - kPad) * ld + sid];
  const int W = (L + 31) / 32;
  for (int w = threadIdx.x; w < W * (int)(blockDim.x / kWave); w += blockDim.x)
    ((uint32_t*)(xbuf + L + kPad + kWave))[w] = 0u;
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int nw = blockDim.x / kWave;
  uint32_t* bm = (uint32_t*)(xbuf + L + kPad + kWave) + (size_t)wave * W;
  const bool half = mode == 1;
  switch (grp) {
#define CCM_RUN(G, LO, HI)                                                                 \
  case G:                                                                                  \
    if (tau == 1) simplex_group<LO, HI, true>(x, L, E_min, E_max, tau, Tp, half, wave, nw, bm, wsum); \
    else simplex_group<LO, HI, false>(x, L, E_min, E_max, tau, Tp, half, wave, nw, bm, wsum);  \
    break;
    CCM_SIMPLEX_GROUPS(CCM_RUN)
#undef CCM_RUN
    default: break;
  }
  __syncthreads();
  if (threadIdx.x < kGroupE) {
    const int g = threadIdx.x;
    const int E = ELO + g;
    if (E >= E_lo && E <= E_hi) {
      double sm[5] = {0, 0, 0, 0, 0};
      for (int w = 0; w < nw; ++w)
        for (int c = 0; c < 5; ++c) sm[c] += wsum[w][g][c];
      const int qbase = half ? L / 2 : 0;
      const int qfirst = qbase + (E - 1) * tau;
      const int qhi = L - 1 - Tp;
      const double n = (double)(qhi - qfirst + 1);
      rho64[(size_t)series * kEMax + (E - 1)] =
          n > 0 ? pearson_from_moments(n, sm[0], sm[1], sm[2], sm[3], sm[4]) : __builtin_nan("");
    }
  }
}

// optE = smallest E reaching the largest non-NaN skill (E_min if all are NaN).
__global__ void simplex_finalize_kernel(const double* __restrict__ rho64, int n, int E_min,
                                        int E_max, int* __restrict__ optE,
                                        float* __restrict__ rho_E) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int nE = E_max - E_min + 1;
  double best = 0.0;
  int bestE = E_min;
  bool have = false;
  for (int E = E_min; E <= E_max; ++E) {
    const double r = rho64[(size_t)i * kEMax + (E - 1)];
    if (rho_E) rho_E[(size_t)i * nE + (E - E_min)] = (float)r;
    if (r == r && (!have || r > best)) {
      best = r;
      bestE = E;
      have = true;
    }
  }
  optE[i] = bestE;
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
    const int sid = ids[i];
    emb[g] = sid >= 0 && sid < ld ? ts[(int64_t)t * ld + sid] : __builtin_nanf("");
  }
}

}  // namespace ccm

// ---- launchers (called from the C ABI) ----------------------------------------------
// The series copy (and mask) of a long series exceeds the default 64 KB of dynamic LDS, so
// each kernel is first allowed all of the LDS its static use leaves.

extern "C" hipError_t ccm_launch_knn(const float* ts, int64_t ld, int L, const int* lib_ids,
                                     const int* lib_E, int n_lib, int tau, int Tp, int k_max,
                                     const uint8_t* cand_mask, int* nbr_idx, float* nbr_w,
                                     float* nbr_d2, hipStream_t stream) {
  if (n_lib == 0) return hipSuccess;
  static std::atomic<uint64_t> attr{0};
  hipError_t e = ccm::allow_lds_once((const void*)ccm::knn_table_kernel, attr);
  if (e != hipSuccess) return e;
  size_t lds = (size_t)(L + ccm::kPad + ccm::kWave) * sizeof(float) + (cand_mask ? (size_t)L : 0);
  hipLaunchKernelGGL(ccm::knn_table_kernel, dim3(n_lib), dim3(ccm::kKnnThreads), lds, stream, ts, ld,
                     L, lib_ids, lib_E, tau, Tp, k_max, cand_mask, nbr_idx, nbr_w, nbr_d2);
  return hipGetLastError();
}

extern "C" hipError_t ccm_launch_simplex(const float* ts, int64_t ld, int L, const int* ids, int n,
                                         int E_min, int E_max, int tau, int Tp, int mode,
                                         int* optE, float* rho_E, double* rho64,
                                         hipStream_t stream) {
  if (n == 0) return hipSuccess;
  static std::atomic<uint64_t> attr{0};
  hipError_t e = ccm::allow_lds_once((const void*)ccm::simplex_kernel, attr);
  if (e != hipSuccess) return e;
  // dynamic LDS: the series and its zero tail, then each wave's bitmap over times
  auto lds_for = [&](int threads) {
    return (size_t)(L + ccm::kPad + ccm::kWave) * sizeof(float) +
           (size_t)(threads / ccm::kWave) * ((L + 31) / 32) * sizeof(uint32_t);
  };
  // 8-wave workgroups while four of them (kSimplexOcc waves per SIMD) fit a CU's LDS with the
  // static part (under 11 KB), else 16-wave ones; calls over many series, where the chip
  // stays full anyway, take 4-wave workgroups (eight per CU), whose waves walk longer query
  // ranges (fewer unseeded starts)
  auto fits = [&](int threads, int per_cu) {
    return (size_t)per_cu * (lds_for(threads) + 11 * 1024) <= 160 * 1024;
  };
  const int threads = n >= 4096 && fits(ccm::kSimplexMinThreads, 8) ? ccm::kSimplexMinThreads
                      : fits(ccm::kSimplexThreads, 4)                ? ccm::kSimplexThreads
                                                                     : ccm::kSimplexMaxThreads;
  hipLaunchKernelGGL(ccm::simplex_kernel, dim3(n, ccm::kNGroups), dim3(threads), lds_for(threads),
                     stream, ts, ld, L, ids, E_min, E_max, tau, Tp, mode, rho64);
  hipLaunchKernelGGL(ccm::simplex_finalize_kernel, dim3((n + 255) / 256), dim3(256), 0, stream,
                     rho64, n, E_min, E_max, optE, rho_E);
  return hipGetLastError();
}

// ---- static scratch of the allocation-free optE entry point ----------------------------
// The FP64 skills [series][CCM_E_MAX] of up to kNoAllocSeries series (16 MiB), a file-scope
// device array: each GPU the library runs on holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address that hipGetSymbolAddress returns for the current
// device, looked up once per device and kept.
namespace ccm {
constexpr int kNoAllocSeries = 104857;   // floor(2^21 / 20): 2^21 doubles
constexpr int kMaxDevices = 64;
}  // namespace ccm

static __device__ __align__(256) double scratch[(size_t)ccm::kNoAllocSeries * ccm::kEMax];

extern "C" int ccm_noalloc_max_series() { return ccm::kNoAllocSeries; }

// Device address of the current device's scratch (looked up on the first call per device).
extern "C" hipError_t ccm_noalloc_scratch(double** out) {
  static std::atomic<double*> ptrs[ccm::kMaxDevices];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= ccm::kMaxDevices) return hipErrorInvalidDevice;
  double* p = ptrs[dev].load(std::memory_order_acquire);
  if (!p) {
    void* addr = nullptr;
    e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!addr) return hipErrorInvalidSymbol;
    p = (double*)addr;
    ptrs[dev].store(p, std::memory_order_release);   // same value if two threads race here
  }
  *out = p;
  return hipSuccess;
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
