// Cross-map lookup fused with Pearson correlation, FP32 gather form.
//
// Method: Sec. III-B of the paper -- one neighbour table per library (Alg. 2) is reused
// for every target; the lookup of Alg. 5 predicts yhat(t) = sum_k w[t,k] y(n_k(t)) and
// corrcoef turns each prediction into rho.  The paper runs this lookup on the CPU and
// names it memory-bandwidth bound and the next bottleneck; here it is the GPU hot loop.
//
// gfx950 design:
//   * A workgroup owns a tile of TJ = 16 targets and keeps all L rows of that tile in LDS
//     (64 B per time step), loaded once from HBM and reused by every library it visits.
//   * A wavefront works on one library at a time and 16 consecutive query times at once:
//     lane = 4 * G + l, group G = query t0 + G, and lane l reads targets 4l..4l+3 of a
//     neighbour row with one 128-bit LDS read.  The group's LDS offsets arrive with one
//     coalesced 256-byte load per four entries and are broadcast inside the quad by DPP
//     (fused into the address add); its weights arrive as one 16-byte load per four entries
//     from an address the quad shares, so each product is a plain FMA.  Each slot of four
//     entries is reloaded for the next block as soon as its products are done.
//   * LDS bank quarter of row s is s mod 4.  Four groups read in the same LDS pass
//     (lanes 16m..16m+15, queries t = 0,1,2,3 mod 4); a preparation kernel orders each
//     table row so that at step j query t prefers a neighbour with s = t + j (mod 4),
//     which keeps the four rows of a pass in distinct quarters whenever it can.
//     The order of the k products only changes FP32 rounding.
//   * Each target column is centred on its mean rounded to FP32 when the tile is loaded
//     (rho does not change under a common shift of y and yhat, and the weights sum to 1, so
//     yhat - c is the prediction of y - c); the FP32 products and moments then keep their
//     digits whatever the series' offset.
//   * Moments sum(yhat), sum(yhat^2), sum(y*yhat) are kept in FP32 for 32 blocks and folded
//     into FP64; sum(y), sum(y^2) over each library's query range come from per-tile FP64
//     column sums.  rho is formed in FP64.
//   * Waves of every workgroup visit libraries in the same order (heaviest first), so the
//     32 workgroups of one XCD read the same tables at about the same time and share L2.
//   * Series longer than the 16-target tile holds (L > 2475) use 8-target tiles in LDS up
//     to L = 5035, beyond that a global copy of 32-target tiles read through L2, with the
//     same tables and arithmetic (see gather_fp32_kernel<true>).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "wave.h"

namespace ccm {

constexpr int kTJ = 16;                 // targets per tile in LDS
constexpr int kGatherThreads = 1024;    // 16 waves

// Tile geometry for TJ targets per tile: LPR = TJ / 4 lanes per query row (each reads 16
// bytes of a neighbour row), RB = 64 / LPR query rows per wave block, SLOT = 4 RB table
// entries per slot of four steps, ROW bytes per time step of the tile.
// BANK rows of the tile share one 256-byte line of LDS banks (at least 4: the bank rule of
// the table preparation uses 4 groups for the 32-target global tile too).
template <int TJ>
struct Geo {
  static constexpr int LPR = TJ / 4;
  static constexpr int RB = kWave / LPR;
  static constexpr int SLOT = RB * 4;
  static constexpr int ROW = TJ * 4;
  static constexpr int BANK = 64 / TJ < 4 ? 4 : 64 / TJ;
};

// ---------------------------------------------------------------------------------------
// Library order: counting sort of libraries by k descending (k = 0: unusable, last).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void order_kernel(const int* __restrict__ lib_k, int n_lib,
                                                    int* __restrict__ order) {
  __shared__ int cnt[256][kKMax + 1];
  const int tid = threadIdx.x;
  const int chunk = (n_lib + 255) / 256;
  const int lo = min(tid * chunk, n_lib);
  const int hi = min(lo + chunk, n_lib);
  for (int v = 0; v <= kKMax; ++v) cnt[tid][v] = 0;
  for (int i = lo; i < hi; ++i) cnt[tid][lib_k[i]]++;
  __syncthreads();
  if (tid == 0) {
    int pos = 0;
    for (int key = kKMax; key >= 0; --key)
      for (int th = 0; th < 256; ++th) {
        int c = cnt[th][key];
        cnt[th][key] = pos;
        pos += c;
      }
  }
  __syncthreads();
  for (int i = lo; i < hi; ++i) order[cnt[tid][lib_k[i]]++] = i;
}

// ---------------------------------------------------------------------------------------
// Table preparation: per (library, t) row, reorder the k entries for bank quarters and
// write them blocked as [lib][t/RB][slot][G][l] (entry j = 4*slot + l of query t = RB b + G,
// RB = 16 for the 16-target tile, 8 for the 32-target one) as tile byte offsets + weights.
// Padding entries point at row (t+j) mod BANK with weight 0.
// ---------------------------------------------------------------------------------------
template <int TJ>
__global__ __launch_bounds__(256) void prep_tables_kernel(
    const int* __restrict__ nbr_idx, const float* __restrict__ nbr_w, const int* __restrict__ lib_E,
    int n_lib, int L, int k_max, int tau, int nblk, int KSM, uint32_t* __restrict__ poff,
    float* __restrict__ pw, int* __restrict__ lib_k) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  using Gm = Geo<TJ>;
  const int64_t per = (int64_t)nblk * Gm::RB;
  if (g >= (int64_t)n_lib * per) return;
  const int i = (int)(g / per);
  const int t = (int)(g % per);
  const int E = lib_E[i];
  const int k = E + 1;
  const int lo = (E - 1) * tau;
  bool libok = E >= 1 && E <= kEMax && k <= k_max && (L - lo) >= k + 1;
  if (libok) libok = nbr_idx[((size_t)i * L + lo) * k_max] >= 0;
  if (t == 0) lib_k[i] = libok ? k : 0;
  const bool rowok = libok && t >= lo && t < L;

  int idx[kKMax];
  float w[kKMax];
  int sel[kKMax];
  int nsel = 0;
  if (rowok) {
    const int* ri = nbr_idx + ((size_t)i * L + t) * k_max;
    const float* rw = nbr_w + ((size_t)i * L + t) * k_max;
    for (int m = 0; m < k; ++m) {
      int v = ri[m];
      bool good = v >= 0 && v < L;
      idx[m] = good ? v : -1;
      w[m] = good ? rw[m] : 0.0f;
    }
    uint32_t used = 0;
    for (int j = 0; j < k; ++j) {
      const int c = (t + j) & (Gm::BANK - 1);
      int pick = -1;
      for (int m = 0; m < k; ++m)
        if (!((used >> m) & 1) && idx[m] >= 0 && (idx[m] & (Gm::BANK - 1)) == c) {
          pick = m;
          break;
        }
      if (pick < 0)
        for (int m = 0; m < k; ++m)
          if (!((used >> m) & 1)) {
            pick = m;
            break;
          }
      used |= 1u << pick;
      sel[nsel++] = pick;
    }
  }
  const int b = t / Gm::RB;
  const int G = t % Gm::RB;
  for (int j = 0; j < KSM * 4; ++j) {
    const size_t pos = (((size_t)i * nblk + b) * KSM + (j >> 2)) * Gm::SLOT + G * 4 + (j & 3);
    uint32_t o = (uint32_t)(((t + j) & (Gm::BANK - 1)) * Gm::ROW);
    float wv = 0.0f;
    if (j < nsel) {
      int m = sel[j];
      if (idx[m] >= 0) {
        o = (uint32_t)idx[m] * Gm::ROW;
        wv = w[m];
      }
    }
    poff[pos] = o;
    pw[pos] = wv;
  }
}

// ---------------------------------------------------------------------------------------
// Targets grouped by E (the paper's Alg. 2 as printed: each target is cross-mapped with the
// libraries' tables at the target's own E).  One workgroup: a stable counting sort of the
// targets into buckets b = E - E_lo (bucket n_E: E without a table), then the tile list
// (bucket, first position, column count) with at most TJ columns per tile.
// ---------------------------------------------------------------------------------------
constexpr int kBucketThreads = 512;
constexpr int kBuckets = kEMax + 1;

template <int TJ>
__global__ __launch_bounds__(kBucketThreads) void bucket_targets_kernel(
    const int* __restrict__ tgt_E, int n_tgt, int E_lo, int n_E, int* __restrict__ perm,
    int* __restrict__ tiles, int* __restrict__ ntiles) {
  __shared__ int cnt[kBuckets][kBucketThreads];
  __shared__ int bstart[kBuckets + 1];
  __shared__ int tstart[kBuckets + 1];
  const int tid = threadIdx.x;
  const int chunk = (n_tgt + kBucketThreads - 1) / kBucketThreads;
  const int lo = min(tid * chunk, n_tgt);
  const int hi = min(lo + chunk, n_tgt);
  for (int b = 0; b < kBuckets; ++b) cnt[b][tid] = 0;
  for (int j = lo; j < hi; ++j) {
    const int e = tgt_E[j] - E_lo;
    cnt[(e >= 0 && e < n_E) ? e : n_E][tid]++;
  }
  __syncthreads();
  if (tid < kBuckets) {   // exclusive scan of bucket tid over threads
    int acc = 0;
    for (int th = 0; th < kBucketThreads; ++th) {
      const int c = cnt[tid][th];
      cnt[tid][th] = acc;
      acc += c;
    }
    bstart[tid] = acc;    // bucket size for now
  }
  __syncthreads();
  if (tid == 0) {
    int pos = 0, tl = 0;
    for (int b = 0; b < kBuckets; ++b) {
      const int c = bstart[b];
      bstart[b] = pos;
      tstart[b] = tl;
      pos += c;
      tl += (c + TJ - 1) / TJ;
    }
    bstart[kBuckets] = pos;
    tstart[kBuckets] = tl;
    *ntiles = tl;
  }
  __syncthreads();
  for (int j = lo; j < hi; ++j) {
    const int e = tgt_E[j] - E_lo;
    const int b = (e >= 0 && e < n_E) ? e : n_E;
    perm[bstart[b] + cnt[b][tid]++] = j;
  }
  for (int T = tid; T < tstart[kBuckets]; T += kBucketThreads) {
    int b = 0;
    while (tstart[b + 1] <= T) ++b;
    const int m = T - tstart[b];
    const int size = bstart[b + 1] - bstart[b];
    tiles[3 * T] = b;
    tiles[3 * T + 1] = bstart[b] + m * TJ;
    tiles[3 * T + 2] = min(TJ, size - m * TJ);
  }
}

// E of table v = e * n_lib + i (tables ordered E-major): E_lo + e.
__global__ void fill_table_E_kernel(int* __restrict__ table_E, int n_lib, int E_lo, int n_tab) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n_tab) table_E[v] = E_lo + v / n_lib;
}

// ---------------------------------------------------------------------------------------
// The gather.  grid = (target tiles, library splits), block = 1024 threads.
// LDS: tile [L][16] floats, then column sums sy[E][16], syy[E][16] (FP64, E = 1..20).
// ---------------------------------------------------------------------------------------
// Weight of step 4s + M from the slot's float4 (all four lanes of a quad hold the same four
// weights, so the products need no cross-lane broadcast).
template <int M>
__device__ __forceinline__ float wcomp(const float4& v) {
  if constexpr (M == 0) return v.x;
  else if constexpr (M == 1) return v.y;
  else if constexpr (M == 2) return v.z;
  else return v.w;
}

// acc.xyzw (+)= w * y.xyzw; FIRST: no accumulator to clear.
template <bool FIRST>
__device__ __forceinline__ void fma4(float4& acc, float wb, const float4& y) {
  if constexpr (FIRST) {
    acc.x = wb * y.x; acc.y = wb * y.y; acc.z = wb * y.z; acc.w = wb * y.w;
  } else {
    acc.x = fmaf(wb, y.x, acc.x); acc.y = fmaf(wb, y.y, acc.y);
    acc.z = fmaf(wb, y.z, acc.z); acc.w = fmaf(wb, y.w, acc.w);
  }
}

struct Moments {
  float4 sp, spp, syp;
  double dp[4], dpp[4], dyp[4];
};

__device__ __forceinline__ void fold(Moments& m) {
  m.dp[0] += m.sp.x; m.dp[1] += m.sp.y; m.dp[2] += m.sp.z; m.dp[3] += m.sp.w;
  m.dpp[0] += m.spp.x; m.dpp[1] += m.spp.y; m.dpp[2] += m.spp.z; m.dpp[3] += m.spp.w;
  m.dyp[0] += m.syp.x; m.dyp[1] += m.syp.y; m.dyp[2] += m.syp.z; m.dyp[3] += m.syp.w;
  m.sp = m.spp = m.syp = float4{0, 0, 0, 0};
}

// Table entries of one block held by one lane: slot s covers steps 4s..4s+3.  With four or
// more lanes per query row (16- and 32-target tiles), lane 4G + l holds the LDS offset of
// step 4s + l of query G (broadcast inside the quad when the read address is formed); with
// two (8 targets) each lane holds two steps' offsets, broadcast inside its pair; with one
// (4 targets) a lane holds all four and needs no broadcast.  Every lane holds all four
// weights of the slot (one 16-byte load from an address the query's lanes share, so the
// memory system fetches each weight once).
template <int TJ>
struct SlotOff {
  using type = uint32_t;
};
template <>
struct SlotOff<8> {
  using type = uint2;
};
template <>
struct SlotOff<4> {
  using type = uint4;
};

template <int KS, int TJ>
struct Slots {
  typename SlotOff<TJ>::type off[KS];
  float4 wgt[KS];
};

template <int S, int TJ, int KS>
__device__ __forceinline__ void load_slot(const uint32_t* bo, const float* bw, int lane,
                                          Slots<KS, TJ>& e) {
  using Gm = Geo<TJ>;
  const int q = (lane / Gm::LPR) * 4;   // first entry of this lane's query row
  if constexpr (Gm::LPR >= 4) e.off[S] = bo[S * Gm::SLOT + q + (lane & 3)];
  else if constexpr (Gm::LPR == 2) e.off[S] = *(const uint2*)(bo + S * Gm::SLOT + q + 2 * (lane & 1));
  else e.off[S] = *(const uint4*)(bo + S * Gm::SLOT + q);
  e.wgt[S] = *(const float4*)(bw + S * Gm::SLOT + q);
}

// LDS offset of step M (0..3) of a slot for this lane's query row.
template <int M, int TJ>
__device__ __forceinline__ uint32_t step_off(const typename SlotOff<TJ>::type& o) {
  if constexpr (Geo<TJ>::LPR >= 4) {
    return (uint32_t)quad_bcast<M>((int)o);
  } else if constexpr (Geo<TJ>::LPR == 2) {
    // lanes 4q + {0, 1} (one row) take lane 4q + M / 2, lanes 4q + {2, 3} lane 4q + 2 + M / 2
    constexpr int a = M >> 1;
    constexpr int sel = a | (a << 2) | ((2 + a) << 4) | ((2 + a) << 6);
    const int v = (M & 1) ? (int)o.y : (int)o.x;
    return (uint32_t)__builtin_amdgcn_mov_dpp(v, sel, 0xF, 0xF, true);
  } else {
    if constexpr (M == 0) return o.x;
    else if constexpr (M == 1) return o.y;
    else if constexpr (M == 2) return o.z;
    else return o.w;
  }
}

template <int J, int K, int TJ>
__device__ __forceinline__ void pair_reads(const char* tile, const Slots<(K + 3) / 4, TJ>& e,
                                           uint32_t laneoff, float4 (&y)[2]) {
  constexpr int S = J >> 2;
  if (J + 0 < K)
    y[0] = *(const float4*)(tile + step_off<(J & 3), TJ>(e.off[S]) + laneoff);
  if (J + 1 < K)
    y[1] = *(const float4*)(tile + step_off<((J + 1) & 3), TJ>(e.off[S]) + laneoff);
}

// One table row, software-pipelined by pairs of steps (reads of pair p+1 issued before the
// products of pair p).  Once the products of a slot are done its registers are reloaded
// with the same slot of the next block, a whole block ahead of use.
template <int K, int TJ, int J = 0>
__device__ __forceinline__ void gather_row_pipe(const char* tile, Slots<(K + 3) / 4, TJ>& e,
                                                const uint32_t* nbo, const float* nbw, int lane,
                                                uint32_t laneoff, float4 (&ya)[2],
                                                float4 (&yb)[2], float4& acc) {
  if constexpr (J < K) {
    constexpr int S = J >> 2;
    if constexpr (J + 2 < K) pair_reads<J + 2, K, TJ>(tile, e, laneoff, yb);
    fma4<J == 0>(acc, wcomp<(J & 3)>(e.wgt[S]), ya[0]);
    if constexpr (J + 1 < K) fma4<false>(acc, wcomp<((J + 1) & 3)>(e.wgt[S]), ya[1]);
    if constexpr ((J + 2) % 4 == 0 || J + 2 >= K) load_slot<S, TJ>(nbo, nbw, lane, e);
    gather_row_pipe<K, TJ, J + 2>(tile, e, nbo, nbw, lane, laneoff, yb, ya, acc);
  }
}

template <int K, int TJ>
__device__ __forceinline__ void gather_block(const char* smem, Slots<(K + 3) / 4, TJ>& e,
                                             const uint32_t* nbo, const float* nbw, int lane,
                                             uint32_t laneoff, int t, int L, Moments& m) {
  float4 acc, ya[2], yb[2];
  // a wave issuing its row's reads and products runs ahead of waves in their moment
  // updates (65.0 -> 61.1 ms on 512 x 101,729 at L = 1600, identical rho)
  __builtin_amdgcn_s_setprio(1);
  pair_reads<0, K, TJ>(smem, e, laneoff, ya);
  gather_row_pipe<K, TJ>(smem, e, nbo, nbw, lane, laneoff, ya, yb, acc);
  __builtin_amdgcn_s_setprio(0);
  t = t < L ? t : L - 1;
  const float4 yo = *(const float4*)(smem + laneoff + (uint32_t)t * Geo<TJ>::ROW);
  m.sp.x += acc.x; m.sp.y += acc.y; m.sp.z += acc.z; m.sp.w += acc.w;
  m.spp.x = fmaf(acc.x, acc.x, m.spp.x); m.spp.y = fmaf(acc.y, acc.y, m.spp.y);
  m.spp.z = fmaf(acc.z, acc.z, m.spp.z); m.spp.w = fmaf(acc.w, acc.w, m.spp.w);
  m.syp.x = fmaf(yo.x, acc.x, m.syp.x); m.syp.y = fmaf(yo.y, acc.y, m.syp.y);
  m.syp.z = fmaf(yo.z, acc.z, m.syp.z); m.syp.w = fmaf(yo.w, acc.w, m.syp.w);
}

template <int K, int TJ, int S = 0>
__device__ __forceinline__ void load_all(const uint32_t* bo, const float* bw, int lane,
                                         Slots<(K + 3) / 4, TJ>& e) {
  if constexpr (S < (K + 3) / 4) {
    load_slot<S, TJ>(bo, bw, lane, e);
    load_all<K, TJ, S + 1>(bo, bw, lane, e);
  }
}

// One library against the tile; FP32 moment sums (32 rows per lane) are folded into FP64
// every 32 blocks.  The workspace holds spare blocks after the last library, so the load of
// block b + 1 is always in bounds.
template <int K, int TJ>
__device__ __forceinline__ void gather_library(const char* smem, const uint32_t* __restrict__ po,
                                               const float* __restrict__ pq, int b0, int nblk,
                                               int KSM, int L, int G, uint32_t laneoff,
                                               Moments& m) {
  const int lane = lane_id();
  const size_t bstride = (size_t)KSM * Geo<TJ>::SLOT;
  const uint32_t* bo = po + (size_t)b0 * bstride;
  const float* bw = pq + (size_t)b0 * bstride;
  Slots<(K + 3) / 4, TJ> e;
  load_all<K, TJ>(bo, bw, lane, e);
  int b = b0;
  while (b < nblk) {
    const int bend = b + 32 < nblk ? b + 32 : nblk;
    for (; b < bend; ++b) {
      bo += bstride;
      bw += bstride;
      gather_block<K, TJ>(smem, e, bo, bw, lane, laneoff, b * Geo<TJ>::RB + G, L, m);
    }
    fold(m);
  }
}

// Long series (L > 2475, where the tile no longer fits in LDS): the tile of TJ target
// columns is a compact copy in global memory ([tile][L][TJ] floats, written by
// tile_copy_kernel with its FP64 column sums), read through L2.  With TJ = 32 a time step
// of the tile is a whole 128-byte line and every table is read once per 32 targets.  The
// grid is then 1-D and XCD-aware: workgroup b runs on XCD b mod 8, and all `splits`
// workgroups of one tile share that XCD (and its L2) and are dispatched together.
constexpr int kXcd = 8;

// Target column of tile column c (c < TJ) of tile T, -1 if none: columns TJ T + c, or the
// targets grouped by E (tile list entry T = bucket, first position in perm, column count).
template <int TJ>
__device__ __forceinline__ int tile_column(int T, int c, int n_tgt, const int* tiles,
                                           const int* perm) {
  if (tiles) {
    const int* te = tiles + 3 * T;
    return c < te[2] ? perm[te[1] + c] : -1;
  }
  const int j = T * TJ + c;
  return j < n_tgt ? j : -1;
}

// gtile[T][t][c] = Y(t, column c of tile T) - c_c (0 where no column), centred on the
// column's mean rounded to FP32, c_c = gsum[T][0][0][c]; and the FP64 sums of those values
// and their squares over t >= (E-1) tau for E = 1..20: gsum[T][0][E][c], gsum[T][1][E][c].
// One workgroup of 1024 threads per tile; a sum over t >= (E-1) tau is the column total less
// its first (E-1) tau terms.
constexpr int kCopyThreads = 1024;

template <int TJ>
__global__ __launch_bounds__(kCopyThreads) void tile_copy_kernel(
    const float* __restrict__ ts, int64_t ld, int L, int tau, int tgt0, int n_tgt,
    const int* __restrict__ tiles, const int* __restrict__ ntiles, const int* __restrict__ perm,
    float* __restrict__ gtile, double* __restrict__ gsum) {
  __shared__ double part[2][kCopyThreads];
  __shared__ int colmap[TJ];
  __shared__ float cref[TJ];
  const int T = blockIdx.x;
  if (tiles && T >= *ntiles) return;
  if (threadIdx.x < TJ) colmap[threadIdx.x] = tile_column<TJ>(T, threadIdx.x, n_tgt, tiles, perm);
  __syncthreads();
  const int c = threadIdx.x & (TJ - 1);
  const int j = colmap[c];
  float* out = gtile + (size_t)T * L * TJ;
  // centring value of each column: its mean rounded to FP32 (as for the LDS tile)
  double a = 0.0, a2 = 0.0;
  for (int g = threadIdx.x; g < L * TJ; g += blockDim.x)
    a += j >= 0 ? ts[(int64_t)(g / TJ) * ld + tgt0 + j] : 0.0f;
  part[0][threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x < TJ) {
    double tot = 0.0;
    for (int r = c; r < kCopyThreads; r += TJ) tot += part[0][r];
    cref[c] = (float)(tot / L);
  }
  __syncthreads();
  const float cj = cref[c];
  a = 0.0;
  for (int g = threadIdx.x; g < L * TJ; g += blockDim.x) {
    const float v = j >= 0 ? ts[(int64_t)(g / TJ) * ld + tgt0 + j] - cj : 0.0f;
    out[g] = v;
    a += v;
    a2 += (double)v * v;
  }
  part[0][threadIdx.x] = a;
  part[1][threadIdx.x] = a2;
  __syncthreads();
  if (threadIdx.x < 2 * TJ) {
    const int q = threadIdx.x / TJ;   // 0: y, 1: y^2
    double tot = 0.0;
    for (int r = c; r < kCopyThreads; r += TJ) tot += part[q][r];
    double* o = gsum + ((size_t)T * 2 + q) * (kEMax + 1) * TJ;
    double pre = 0.0;
    int t = 0;
    for (int E = 1; E <= kEMax; ++E) {
      for (; t < (E - 1) * tau && t < L; ++t) {
        const double v = j >= 0 ? (double)(ts[(int64_t)t * ld + tgt0 + j] - cj) : 0.0;
        pre += q ? v * v : v;
      }
      o[E * TJ + c] = tot - pre;
    }
    if (q == 0) o[c] = cj;   // the centring value, in the unused E = 0 slot
  }
}

// Two ways to form a workgroup's 16 target columns and its tables:
//   * tiles == NULL: columns j0..j0+15 (j0 = 16 * blockIdx.x), every library with its own
//     table (library row i = order[li], table i);
//   * tiles != NULL (targets grouped by E): tile entry blockIdx.x = (bucket b, first
//     position in perm, column count); column c is target perm[first + c], and library row
//     i uses table b * n_lib + i, the library's table at the bucket's E.  Bucket n_E holds
//     targets whose E has no table: their rho is NaN.  Entries past *ntiles exit at once.
template <bool GT, int TJ>
__global__ __launch_bounds__(kGatherThreads) void gather_fp32_kernel(
    const float* __restrict__ ts, int64_t ld, int L, int tau, int tgt0, int n_tgt,
    const uint32_t* __restrict__ poff, const float* __restrict__ pw, const int* __restrict__ order,
    const int* __restrict__ lib_k, int n_lib, int nblk, int KSM, float* __restrict__ rho,
    double* __restrict__ moments, const int* __restrict__ tiles, const int* __restrict__ ntiles,
    const int* __restrict__ perm, int n_E, const float* __restrict__ gtile,
    const double* __restrict__ gsum, int n_tiles, int gsplits) {
  static_assert(GT || TJ == 4 || TJ == 8 || TJ == kTJ, "LDS tiles of 4, 8 or 16 columns");
  using Gm = Geo<TJ>;
  extern __shared__ __align__(16) char smem[];
  __shared__ int colmap[TJ];    // target column of each tile column, -1 if none
  // tile T and library split of this workgroup
  int T, split, splits;
  if constexpr (GT) {
    const int b = blockIdx.x;
    const int q = b / kXcd;
    T = (q / gsplits) * kXcd + b % kXcd;
    split = q % gsplits;
    splits = gsplits;
    if (T >= n_tiles) return;   // whole workgroup: the grid's last round of tiles
  } else {
    T = blockIdx.x;
    split = blockIdx.y;
    splits = gridDim.y;
  }
  int vbase = 0;
  bool no_table = false;
  if (tiles) {
    if (T >= *ntiles) return;   // whole workgroup: past the tile list
    const int b = tiles[3 * T];
    vbase = b * n_lib;
    no_table = b >= n_E;
  }
  if (threadIdx.x < TJ) colmap[threadIdx.x] = tile_column<TJ>(T, threadIdx.x, n_tgt, tiles, perm);
  __syncthreads();
  // the tile, [L][TJ] floats (4 TJ bytes per time step), and its FP64 column sums of y and
  // y^2 over t >= (E-1) tau, [2][kEMax + 1][TJ]: in LDS, or the global copy
  auto tile_ptr = [&]() -> const char* {
    if constexpr (GT) return (const char*)(gtile + (size_t)T * L * TJ);
    else return smem;
  };
  auto sums_ptr = [&]() -> const double* {
    if constexpr (GT) return gsum + (size_t)T * 2 * (kEMax + 1) * TJ;
    else return (const double*)(smem + (size_t)L * Gm::ROW);
  };
  if constexpr (!GT) {
    float* tile = (float*)smem;
    double* lsy = (double*)(smem + (size_t)L * Gm::ROW);
    double* lsyy = lsy + (kEMax + 1) * TJ;
    // load the tile (rows 0..L-1, TJ columns; missing columns read as 0).  A thread always
    // handles the same column (blockDim is a multiple of TJ), so it sums that column too.
    constexpr int SH = TJ == 16 ? 4 : (TJ == 8 ? 3 : 2);   // log2 TJ
    double csum = 0.0;
    for (int g = threadIdx.x; g < L * TJ; g += blockDim.x) {
      const int t = g >> SH;
      const int j = colmap[g & (TJ - 1)];
      const float v = j >= 0 ? ts[(int64_t)t * ld + tgt0 + j] : 0.0f;
      tile[g] = v;
      csum += v;
    }
    // centre each column on c = its mean rounded to FP32 (kept in the unused E = 0 slot of
    // the sums, lsy[c]); the per-wave partial sums pass through lsy[TJ ..] first
#pragma unroll
    for (int o = TJ; o < kWave; o <<= 1) csum += __shfl_xor(csum, o);
    if (lane_id() < TJ) lsy[TJ + (threadIdx.x / kWave) * TJ + lane_id()] = csum;
    __syncthreads();
    if (threadIdx.x < TJ) {
      double tot = 0.0;
      for (int w = 0; w < kGatherThreads / kWave; ++w) tot += lsy[TJ + w * TJ + threadIdx.x];
      lsy[threadIdx.x] = (double)(float)(tot / L);
    }
    __syncthreads();
    {
      const float cj = (float)lsy[threadIdx.x & (TJ - 1)];
      for (int g = threadIdx.x; g < L * TJ; g += blockDim.x) tile[g] -= cj;
    }
    __syncthreads();
    // FP64 sums of y and y^2 over t >= (E-1) tau, per E and column
    for (int g = threadIdx.x; g < kEMax * TJ; g += blockDim.x) {
      const int E = g / TJ + 1;
      const int c = g % TJ;
      double a = 0.0, a2 = 0.0;
      for (int t = (E - 1) * tau; t < L; ++t) {
        double v = tile[t * TJ + c];
        a += v;
        a2 += v * v;
      }
      lsy[E * TJ + c] = a;
      lsyy[E * TJ + c] = a2;
    }
    __syncthreads();
  }

  const int lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int nw = blockDim.x / kWave;
  const int G = lane / Gm::LPR;   // query row of the block
  const int l = lane % Gm::LPR;   // this lane reads targets 4l .. 4l + 3
  const uint32_t laneoff = (uint32_t)l * 16;
  const size_t libstride = (size_t)nblk * KSM * Gm::SLOT;

  for (int li = split + splits * wave; li < n_lib; li += splits * nw) {
    const int i = __builtin_amdgcn_readfirstlane(order ? order[li] : li);
    const int v = vbase + i;   // table of this library row
    const int k = no_table ? 0 : __builtin_amdgcn_readfirstlane(lib_k[v]);
    if (k == 0) {
      const int j = lane < TJ ? colmap[lane] : -1;
      if (j >= 0) {
        rho[(size_t)i * n_tgt + j] = __builtin_nanf("");
        if (moments) {
          double* mo = moments + ((size_t)i * n_tgt + j) * 3;
          mo[0] = mo[1] = mo[2] = __builtin_nan("");
        }
      }
      continue;
    }
    const int E = k - 1;
    const int lo = (E - 1) * tau;
    const uint32_t* po = poff + (size_t)v * libstride;
    const float* pq = pw + (size_t)v * libstride;
    Moments m;
    m.sp = m.spp = m.syp = float4{0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c) m.dp[c] = m.dpp[c] = m.dyp[c] = 0.0;
    const int b0 = lo / Gm::RB;
    switch (k) {
#define CCM_K(KK) \
  case KK: gather_library<KK, TJ>(tile_ptr(), po, pq, b0, nblk, KSM, L, G, laneoff, m); break;
      CCM_K(2) CCM_K(3) CCM_K(4) CCM_K(5) CCM_K(6) CCM_K(7) CCM_K(8) CCM_K(9) CCM_K(10)
      CCM_K(11) CCM_K(12) CCM_K(13) CCM_K(14) CCM_K(15) CCM_K(16) CCM_K(17) CCM_K(18)
      CCM_K(19) CCM_K(20) CCM_K(21)
#undef CCM_K
      default: break;
    }
    // reduce over the query rows (lanes with equal l)
#pragma unroll
    for (int o = Gm::LPR; o < kWave; o <<= 1) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        m.dp[c] += __shfl_xor(m.dp[c], o);
        m.dpp[c] += __shfl_xor(m.dpp[c], o);
        m.dyp[c] += __shfl_xor(m.dyp[c], o);
      }
    }
    if (G == 0) {
      const double* sy = sums_ptr();
      const double* syy = sy + (kEMax + 1) * TJ;
      const double n = (double)(L - lo);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int col = 4 * l + c;
        const int j = colmap[col];
        if (j >= 0) {
          const double cref = sy[col];   // the column's centring value (E = 0 slot)
          const double r = pearson_shifted(n, cref, sy[E * TJ + col], syy[E * TJ + col],
                                           m.dp[c], m.dpp[c], m.dyp[c]);
          rho[(size_t)i * n_tgt + j] = (float)r;
          if (moments)
            unshift_moments(n, cref, sy[E * TJ + col], m.dp[c], m.dpp[c], m.dyp[c],
                            moments + ((size_t)i * n_tgt + j) * 3);
        }
      }
    }
  }
}

}  // namespace ccm

namespace ccm {
// The gather's LDS tile needs more than the default dynamic LDS limit: allow all of the
// CU's 160 KB minus the kernel's static LDS (once per tile width).
template <int TJ>
hipError_t gather_allow_lds() {
  static std::atomic<uint64_t> done{0};
  return allow_lds_once((const void*)gather_fp32_kernel<false, TJ>, done);
}

// Library splits (grid.y): enough workgroups to fill the chip when there are few tiles, no
// more than one library per wave.
int gather_splits(int n_tiles, int n_lib) {
  int splits = (1024 + n_tiles - 1) / n_tiles;
  const int max_splits = (n_lib + kGatherThreads / kWave - 1) / (kGatherThreads / kWave);
  if (splits > max_splits) splits = max_splits;
  return splits < 1 ? 1 : splits;
}

// Long series: 32 workgroups per tile (one per CU of an XCD), at most one library per wave.
int gather_splits_global(int n_lib) {
  const int per_wave = (n_lib + kGatherThreads / kWave - 1) / (kGatherThreads / kWave);
  return per_wave < 1 ? 1 : (per_wave > 32 ? 32 : per_wave);
}

}  // namespace ccm

// LDS of a tile of tj targets over L time steps: the tile plus its FP64 column sums.
static size_t gather_lds_bytes_tj(int L, int tj) {
  return (size_t)L * tj * 4 + 2 * (ccm::kEMax + 1) * (size_t)tj * sizeof(double);
}
static bool gather_fits_lds(int L, int tj) {
  return gather_lds_bytes_tj(L, tj) + (size_t)tj * sizeof(int) <= 160 * 1024;
}

// Testing switch (ccm_set_gather_tile): 0 picks the tile width from L; 4, 8 or 16 force that
// LDS tile where it fits; 32 forces the global copy.
static std::atomic<int> g_force_tile{0};
extern "C" void ccm_gather_force_tile(int tj) {
  g_force_tile.store(tj == 4 || tj == 8 || tj == 16 || tj == 32 ? tj : 0);
}

// Targets per tile of the cross-map: 16 while that tile fits in LDS (L <= 2475), then 8
// (L <= 5,035: each time step's row half as wide, each table read for half as many targets,
// but the neighbour rows stay on chip), beyond that 32 targets from a global copy.  The
// 4-target LDS tile (L <= 10,155) is built and can be forced, but at L = 8,528 it measured
// no faster than the global copy.
extern "C" int ccm_gather_tile_targets(int L) {
  const int f = g_force_tile.load();
  if (f == 32) return 32;
  if (f != 0 && gather_fits_lds(L, f)) return f;
  for (int tj = ccm::kTJ; tj >= 8; tj /= 2)
    if (gather_fits_lds(L, tj)) return tj;
  return 2 * ccm::kTJ;
}

// 1 when the cross-map's target tile is in LDS (else a global copy is made).
extern "C" int ccm_gather_tile_in_lds(int L) { return ccm_gather_tile_targets(L) <= ccm::kTJ; }

namespace ccm {
// Launch the gather on n_tiles tiles of TJ targets (library-E columns when tiles == NULL,
// else the tile list), from LDS (TJ = 4, 8, 16), else from a global copy made first.  The
// tables were blocked for TJ.
template <int TJ>
hipError_t launch_gather(const float* ts, int64_t ld, int L, int tau, int tgt0, int n_tgt,
                         const uint32_t* poff, const float* pw, const int* order, const int* lib_k,
                         int n_lib, int nblk, int KSM, float* rho, double* moments,
                         const int* tiles, const int* ntiles, const int* perm, int n_E,
                         int n_tiles, float* gtile, double* gsum, hipStream_t stream) {
  if constexpr (TJ <= kTJ) {
    hipError_t e = gather_allow_lds<TJ>();
    if (e != hipSuccess) return e;
    const int splits = gather_splits(n_tiles, n_lib);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(gather_fp32_kernel<false, TJ>), dim3(n_tiles, splits), dim3(kGatherThreads),
                       gather_lds_bytes_tj(L, TJ), stream, ts, ld, L, tau, tgt0, n_tgt, poff, pw,
                       order, lib_k, n_lib, nblk, KSM, rho, moments, tiles, ntiles, perm, n_E,
                       (const float*)nullptr, (const double*)nullptr, n_tiles, splits);
    return hipGetLastError();
  } else {
    hipLaunchKernelGGL(tile_copy_kernel<TJ>, dim3(n_tiles), dim3(kCopyThreads), 0, stream, ts, ld,
                       L, tau, tgt0, n_tgt, tiles, ntiles, perm, gtile, gsum);
    const int splits = gather_splits_global(n_lib);
    const int64_t grid = (int64_t)((n_tiles + kXcd - 1) / kXcd) * kXcd * splits;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(gather_fp32_kernel<true, TJ>), dim3((unsigned)grid), dim3(kGatherThreads), 0,
                       stream, ts, ld, L, tau, tgt0, n_tgt, poff, pw, order, lib_k, n_lib, nblk, KSM,
                       rho, moments, tiles, ntiles, perm, n_E, (const float*)gtile,
                       (const double*)gsum, n_tiles, splits);
    return hipGetLastError();
  }
}
}  // namespace ccm

extern "C" hipError_t ccm_launch_order(const int* lib_k, int n_lib, int* order, hipStream_t stream) {
  hipLaunchKernelGGL(ccm::order_kernel, dim3(1), dim3(256), 0, stream, lib_k, n_lib, order);
  return hipGetLastError();
}

extern "C" size_t ccm_gather_lds_bytes(int L) {  // tile + column sums at L's tile width
  const int tj = ccm_gather_tile_targets(L);
  return tj <= ccm::kTJ ? gather_lds_bytes_tj(L, tj) : 0;
}

extern "C" hipError_t ccm_launch_crossmap_fp32(const float* ts, int64_t ld, int L, int tau,
                                               int tgt0, int n_tgt, const int* nbr_idx,
                                               const float* nbr_w, const int* lib_E, int n_lib,
                                               int k_max, float* rho, double* moments,
                                               uint32_t* poff, float* pw, int* lib_k, int* order,
                                               float* gtile, double* gsum, hipStream_t stream) {
  if (n_lib == 0 || n_tgt == 0) return hipSuccess;
  const int KSM = (k_max + 3) / 4;
  auto run = [&](auto tj) -> hipError_t {
    constexpr int TJ = decltype(tj)::value;
    constexpr int RB = ccm::Geo<TJ>::RB;
    const int nblk = (L + RB - 1) / RB;
    const int64_t rows = (int64_t)n_lib * nblk * RB;
    hipLaunchKernelGGL(ccm::prep_tables_kernel<TJ>, dim3((unsigned)((rows + 255) / 256)), dim3(256),
                       0, stream, nbr_idx, nbr_w, lib_E, n_lib, L, k_max, tau, nblk, KSM, poff, pw,
                       lib_k);
    hipLaunchKernelGGL(ccm::order_kernel, dim3(1), dim3(256), 0, stream, lib_k, n_lib, order);
    const int n_tiles = (n_tgt + TJ - 1) / TJ;
    return ccm::launch_gather<TJ>(ts, ld, L, tau, tgt0, n_tgt, poff, pw, order, lib_k, n_lib,
                                  nblk, KSM, rho, moments, nullptr, nullptr, nullptr, 0, n_tiles,
                                  gtile, gsum, stream);
  };
  switch (ccm_gather_tile_targets(L)) {
    case 16: return run(std::integral_constant<int, 16>{});
    case 8: return run(std::integral_constant<int, 8>{});
    case 4: return run(std::integral_constant<int, 4>{});
    default: return run(std::integral_constant<int, 32>{});
  }
}

// Maximum number of tile entries for n_tgt targets in tiles of tj columns: every bucket may
// end in a partial tile.
extern "C" int ccm_target_E_max_tiles(int n_tgt, int tj) {
  return (n_tgt + tj - 1) / tj + ccm::kBuckets;
}

extern "C" hipError_t ccm_launch_crossmap_fp32_target_E(
    const float* ts, int64_t ld, int L, int tau, int tgt0, int n_tgt, const int* nbr_idx,
    const float* nbr_w, int n_lib, int E_lo, int n_E, int k_max, const int* tgt_E, float* rho,
    double* moments, uint32_t* poff, float* pw, int* lib_k, int* table_E, int* perm, int* tiles,
    int* ntiles, float* gtile, double* gsum, hipStream_t stream) {
  if (n_lib == 0 || n_tgt == 0) return hipSuccess;
  const int KSM = (k_max + 3) / 4;
  const int n_tab = n_E * n_lib;
  hipLaunchKernelGGL(ccm::fill_table_E_kernel, dim3((n_tab + 255) / 256), dim3(256), 0, stream,
                     table_E, n_lib, E_lo, n_tab);
  auto run = [&](auto tj) -> hipError_t {
    constexpr int TJ = decltype(tj)::value;
    constexpr int RB = ccm::Geo<TJ>::RB;
    const int nblk = (L + RB - 1) / RB;
    const int64_t rows = (int64_t)n_tab * nblk * RB;
    hipLaunchKernelGGL(ccm::prep_tables_kernel<TJ>, dim3((unsigned)((rows + 255) / 256)), dim3(256),
                       0, stream, nbr_idx, nbr_w, table_E, n_tab, L, k_max, tau, nblk, KSM, poff,
                       pw, lib_k);
    hipLaunchKernelGGL(ccm::bucket_targets_kernel<TJ>, dim3(1), dim3(ccm::kBucketThreads), 0,
                       stream, tgt_E, n_tgt, E_lo, n_E, perm, tiles, ntiles);
    return ccm::launch_gather<TJ>(ts, ld, L, tau, tgt0, n_tgt, poff, pw, nullptr, lib_k, n_lib,
                                  nblk, KSM, rho, moments, tiles, ntiles, perm, n_E,
                                  ccm_target_E_max_tiles(n_tgt, TJ), gtile, gsum, stream);
  };
  switch (ccm_gather_tile_targets(L)) {
    case 16: return run(std::integral_constant<int, 16>{});
    case 8: return run(std::integral_constant<int, 8>{});
    case 4: return run(std::integral_constant<int, 4>{});
    default: return run(std::integral_constant<int, 32>{});
  }
}
