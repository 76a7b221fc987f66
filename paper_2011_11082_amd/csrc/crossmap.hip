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
//     neighbour row with one 128-bit LDS read.  The group's table entries arrive with one
//     coalesced 256-byte load per four entries and are broadcast inside the quad by DPP
//     (quad_perm), so no scalar or per-lane table traffic sits in the inner loop.
//   * LDS bank quarter of row s is s mod 4.  Four groups read in the same LDS pass
//     (lanes 16m..16m+15, queries t = 0,1,2,3 mod 4); a preparation kernel orders each
//     table row so that at step j query t prefers a neighbour with s = t + j (mod 4),
//     which keeps the four rows of a pass in distinct quarters whenever it can.
//     The order of the k products only changes FP32 rounding.
//   * Moments sum(yhat), sum(yhat^2), sum(y*yhat) are kept in FP32 for 8 steps and folded
//     into FP64; sum(y), sum(y^2) over each library's query range come from per-tile FP64
//     column sums.  rho is formed in FP64.
//   * Waves of every workgroup visit libraries in the same order (heaviest first), so the
//     32 workgroups of one XCD read the same tables at about the same time and share L2.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "wave.h"

namespace ccm {

constexpr int kTJ = 16;                 // targets per tile
constexpr int kGatherThreads = 1024;    // 16 waves
constexpr int kRowBytes = kTJ * 4;

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
// write them blocked as [lib][t/16][slot][G][l] (entry j = 4*slot + l of query t = 16b+G)
// as LDS byte offsets + weights.  Padding entries point at row (t+j) mod 4 with weight 0.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void prep_tables_kernel(
    const int* __restrict__ nbr_idx, const float* __restrict__ nbr_w, const int* __restrict__ lib_E,
    int n_lib, int L, int k_max, int tau, int nblk, int KSM, uint32_t* __restrict__ poff,
    float* __restrict__ pw, int* __restrict__ lib_k) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)nblk * 16;
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
      const int c = (t + j) & 3;
      int pick = -1;
      for (int m = 0; m < k; ++m)
        if (!((used >> m) & 1) && idx[m] >= 0 && (idx[m] & 3) == c) {
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
  const int b = t / 16;
  const int G = t % 16;
  for (int j = 0; j < KSM * 4; ++j) {
    const size_t pos = (((size_t)i * nblk + b) * KSM + (j >> 2)) * kWave + G * 4 + (j & 3);
    uint32_t o = (uint32_t)(((t + j) & 3) * kRowBytes);
    float wv = 0.0f;
    if (j < nsel) {
      int m = sel[j];
      if (idx[m] >= 0) {
        o = (uint32_t)idx[m] * kRowBytes;
        wv = w[m];
      }
    }
    poff[pos] = o;
    pw[pos] = wv;
  }
}

// ---------------------------------------------------------------------------------------
// The gather.  grid = (target tiles, library splits), block = 1024 threads.
// LDS: tile [L][16] floats, then column sums sy[E][16], syy[E][16] (FP64, E = 1..20).
// ---------------------------------------------------------------------------------------
template <int J>
__device__ __forceinline__ void gather_step(const char* tile, const uint32_t (&off)[6],
                                            const float (&wgt)[6], uint32_t laneoff, float4& acc) {
  const uint32_t o = (uint32_t)quad_bcast<J & 3>((int)off[J >> 2]) + laneoff;
  const float4 y = *(const float4*)(tile + o);
  const float w = quad_bcast<J & 3>(wgt[J >> 2]);
  acc.x = fmaf(w, y.x, acc.x);
  acc.y = fmaf(w, y.y, acc.y);
  acc.z = fmaf(w, y.z, acc.z);
  acc.w = fmaf(w, y.w, acc.w);
}

__global__ __launch_bounds__(kGatherThreads) void gather_fp32_kernel(
    const float* __restrict__ ts, int64_t ld, int L, int tau, int tgt0, int n_tgt,
    const uint32_t* __restrict__ poff, const float* __restrict__ pw, const int* __restrict__ order,
    const int* __restrict__ lib_k, int n_lib, int nblk, int KSM, float* __restrict__ rho,
    double* __restrict__ moments) {
  extern __shared__ __align__(16) char smem[];
  float* tile = (float*)smem;
  double* sy = (double*)(smem + (size_t)L * kRowBytes);      // [kEMax + 1][16]
  double* syy = sy + (kEMax + 1) * kTJ;

  const int j0 = blockIdx.x * kTJ;
  // load the tile (rows 0..L-1, 16 columns; columns past n_tgt read as 0)
  for (int g = threadIdx.x; g < L * kTJ; g += blockDim.x) {
    const int t = g >> 4;
    const int c = g & 15;
    const int j = j0 + c;
    tile[g] = j < n_tgt ? ts[(int64_t)t * ld + tgt0 + j] : 0.0f;
  }
  __syncthreads();
  // FP64 sums of y and y^2 over t >= (E-1) tau, per E and column
  for (int g = threadIdx.x; g < kEMax * kTJ; g += blockDim.x) {
    const int E = g / kTJ + 1;
    const int c = g % kTJ;
    double a = 0.0, a2 = 0.0;
    for (int t = (E - 1) * tau; t < L; ++t) {
      double v = tile[t * kTJ + c];
      a += v;
      a2 += v * v;
    }
    sy[E * kTJ + c] = a;
    syy[E * kTJ + c] = a2;
  }
  __syncthreads();

  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int G = lane >> 2;
  const int l = lane & 3;
  const uint32_t laneoff = (uint32_t)l * 16;
  const int splits = gridDim.y;
  const size_t libstride = (size_t)nblk * KSM * kWave;

  for (int li = blockIdx.y + splits * wave; li < n_lib; li += splits * nw) {
    const int i = order[li];
    const int k = lib_k[i];
    if (k == 0) {
      if (lane < kTJ && j0 + lane < n_tgt) {
        rho[(size_t)i * n_tgt + j0 + lane] = __builtin_nanf("");
        if (moments) {
          double* mo = moments + ((size_t)i * n_tgt + j0 + lane) * 3;
          mo[0] = mo[1] = mo[2] = __builtin_nan("");
        }
      }
      continue;
    }
    const int E = k - 1;
    const int lo = (E - 1) * tau;
    const int KS = (k + 3) >> 2;
    const uint32_t* po = poff + (size_t)i * libstride;
    const float* pq = pw + (size_t)i * libstride;
    float4 sp = {0, 0, 0, 0}, spp = {0, 0, 0, 0}, syp = {0, 0, 0, 0};
    double dp[4] = {0, 0, 0, 0}, dpp[4] = {0, 0, 0, 0}, dyp[4] = {0, 0, 0, 0};
    int since = 0;
    for (int b = lo >> 4; b < nblk; ++b) {
      uint32_t off[6];
      float wgt[6];
#pragma unroll
      for (int s4 = 0; s4 < 6; ++s4) {
        if (s4 < KS) {
          const size_t p = ((size_t)b * KSM + s4) * kWave + lane;
          off[s4] = po[p];
          wgt[s4] = pq[p];
        } else {
          off[s4] = 0;
          wgt[s4] = 0.0f;
        }
      }
      float4 acc = {0, 0, 0, 0};
      gather_step<0>(smem, off, wgt, laneoff, acc);
      gather_step<1>(smem, off, wgt, laneoff, acc);
      if (k > 2) gather_step<2>(smem, off, wgt, laneoff, acc);
      if (k > 3) gather_step<3>(smem, off, wgt, laneoff, acc);
      if (k > 4) gather_step<4>(smem, off, wgt, laneoff, acc);
      if (k > 5) gather_step<5>(smem, off, wgt, laneoff, acc);
      if (k > 6) gather_step<6>(smem, off, wgt, laneoff, acc);
      if (k > 7) gather_step<7>(smem, off, wgt, laneoff, acc);
      if (k > 8) gather_step<8>(smem, off, wgt, laneoff, acc);
      if (k > 9) gather_step<9>(smem, off, wgt, laneoff, acc);
      if (k > 10) gather_step<10>(smem, off, wgt, laneoff, acc);
      if (k > 11) gather_step<11>(smem, off, wgt, laneoff, acc);
      if (k > 12) gather_step<12>(smem, off, wgt, laneoff, acc);
      if (k > 13) gather_step<13>(smem, off, wgt, laneoff, acc);
      if (k > 14) gather_step<14>(smem, off, wgt, laneoff, acc);
      if (k > 15) gather_step<15>(smem, off, wgt, laneoff, acc);
      if (k > 16) gather_step<16>(smem, off, wgt, laneoff, acc);
      if (k > 17) gather_step<17>(smem, off, wgt, laneoff, acc);
      if (k > 18) gather_step<18>(smem, off, wgt, laneoff, acc);
      if (k > 19) gather_step<19>(smem, off, wgt, laneoff, acc);
      if (k > 20) gather_step<20>(smem, off, wgt, laneoff, acc);
      const int t = b * 16 + G;
      if (t >= lo && t < L) {
        const float4 yo = *(const float4*)(smem + (size_t)t * kRowBytes + laneoff);
        sp.x += acc.x; sp.y += acc.y; sp.z += acc.z; sp.w += acc.w;
        spp.x = fmaf(acc.x, acc.x, spp.x); spp.y = fmaf(acc.y, acc.y, spp.y);
        spp.z = fmaf(acc.z, acc.z, spp.z); spp.w = fmaf(acc.w, acc.w, spp.w);
        syp.x = fmaf(yo.x, acc.x, syp.x); syp.y = fmaf(yo.y, acc.y, syp.y);
        syp.z = fmaf(yo.z, acc.z, syp.z); syp.w = fmaf(yo.w, acc.w, syp.w);
      }
      if (++since == 8) {
        since = 0;
        dp[0] += sp.x; dp[1] += sp.y; dp[2] += sp.z; dp[3] += sp.w;
        dpp[0] += spp.x; dpp[1] += spp.y; dpp[2] += spp.z; dpp[3] += spp.w;
        dyp[0] += syp.x; dyp[1] += syp.y; dyp[2] += syp.z; dyp[3] += syp.w;
        sp = spp = syp = float4{0, 0, 0, 0};
      }
    }
    dp[0] += sp.x; dp[1] += sp.y; dp[2] += sp.z; dp[3] += sp.w;
    dpp[0] += spp.x; dpp[1] += spp.y; dpp[2] += spp.z; dpp[3] += spp.w;
    dyp[0] += syp.x; dyp[1] += syp.y; dyp[2] += syp.z; dyp[3] += syp.w;
    // reduce over the 16 groups (lanes with equal l)
#pragma unroll
    for (int o = 4; o < kWave; o <<= 1) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        dp[c] += __shfl_xor(dp[c], o);
        dpp[c] += __shfl_xor(dpp[c], o);
        dyp[c] += __shfl_xor(dyp[c], o);
      }
    }
    if (G == 0) {
      const double n = (double)(L - lo);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int col = 4 * l + c;
        const int j = j0 + col;
        if (j < n_tgt) {
          const double r = pearson_from_moments(n, sy[E * kTJ + col], syy[E * kTJ + col], dp[c],
                                                dpp[c], dyp[c]);
          rho[(size_t)i * n_tgt + j] = (float)r;
          if (moments) {
            double* mo = moments + ((size_t)i * n_tgt + j) * 3;
            mo[0] = dp[c];
            mo[1] = dpp[c];
            mo[2] = dyp[c];
          }
        }
      }
    }
  }
}

}  // namespace ccm

extern "C" size_t ccm_gather_lds_bytes(int L) {
  return (size_t)L * ccm::kRowBytes + 2 * (ccm::kEMax + 1) * ccm::kTJ * sizeof(double);
}

extern "C" hipError_t ccm_launch_crossmap_fp32(const float* ts, int64_t ld, int L, int tau,
                                               int tgt0, int n_tgt, const int* nbr_idx,
                                               const float* nbr_w, const int* lib_E, int n_lib,
                                               int k_max, float* rho, double* moments,
                                               uint32_t* poff, float* pw, int* lib_k, int* order,
                                               hipStream_t stream) {
  if (n_lib == 0 || n_tgt == 0) return hipSuccess;
  const int nblk = (L + 15) / 16;
  const int KSM = (k_max + 3) / 4;
  const int64_t rows = (int64_t)n_lib * nblk * 16;
  hipLaunchKernelGGL(ccm::prep_tables_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0,
                     stream, nbr_idx, nbr_w, lib_E, n_lib, L, k_max, tau, nblk, KSM, poff, pw, lib_k);
  hipLaunchKernelGGL(ccm::order_kernel, dim3(1), dim3(256), 0, stream, lib_k, n_lib, order);
  const size_t lds = ccm_gather_lds_bytes(L);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)ccm::gather_fp32_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int n_tiles = (n_tgt + ccm::kTJ - 1) / ccm::kTJ;
  int splits = (1024 + n_tiles - 1) / n_tiles;
  const int max_splits = (n_lib + 15) / 16;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  hipLaunchKernelGGL(ccm::gather_fp32_kernel, dim3(n_tiles, splits), dim3(ccm::kGatherThreads), lds,
                     stream, ts, ld, L, tau, tgt0, n_tgt, poff, pw, order, lib_k, n_lib, nblk, KSM,
                     rho, moments);
  return hipGetLastError();
}
