// Cross-map lookup as a dense BF16 MFMA contraction (not in the paper).
//
// The lookup of Alg. 5 (Sec. III-B) is, for one library, yhat = W * Y where W is the
// n x L matrix holding the simplex weights of row t at the columns of its k neighbours
// (every other entry 0) and Y is the L x n_tgt target panel.  This form densifies W in
// tiles and runs the product on the matrix cores: BF16 operands (weights and targets
// rounded to nearest-even, each target column first centred on its mean rounded to FP32),
// FP32 accumulation, then the same Pearson epilogue as the FP32 gather with the observed
// targets in FP32 (centred the same way) and the moments in FP64.  Distances and
// weights are computed in FP32/FP64 exactly as for the gather; only the product operands
// are BF16.  The dense product does L / k times the multiply-adds of the gather, so this
// form is bound by MFMA throughput.
//
// gfx950 design:
//   * workgroup = 8 waves = 2 libraries (sorted by E) x one tile of 64 targets; each wave
//     owns 32 rows of a 128-row chunk of its library against the 64 targets: a 32 x 64
//     FP32 accumulator (2 tiles of v_mfma_f32_32x32x16_bf16).  With the FP64 moment sums
//     in registers the workgroup needs under 80 KB of LDS and about 100 VGPRs, so two
//     workgroups share a CU (four waves per SIMD) and one's barriers and latencies overlap
//     the other's products.
//   * K (the neighbour time s) advances in stages of 64: the workgroup stages Y^T[128][64]
//     BF16 in LDS (double-buffered, loaded two stages ahead through registers) and each wave
//     scatters the nonzeros of its 32 rows into its own zeroed A tile [32][64]; after its
//     products it writes the same positions back to zero (the tile is private to the
//     wave, so program order is the only ordering needed).  Every stage runs its products
//     unconditionally: a branch around them would make the compiler move all 128
//     accumulators between AGPRs and VGPRs at every stage.
//   * The stage loop is unrolled by two so the two B register sets alternate roles (each
//     is stored to LDS, then reloaded two stages ahead) without register copies.  Within a
//     stage the fragments of k-step kk + 1 are read from LDS while the products of kk run
//     (scheduling barriers keep the compiler from serialising reads and products again).
//   * Table entries are pre-sorted per (library, 128-row chunk) by (stage, row quarter) and
//     packed into 32 bits (row, column within stage, BF16 weight), so each wave scatters and
//     clears only its own entries; their bucket offsets are wave-uniform loads.
//   * The epilogue reads the observed FP32 y of a wave's rows at uniform strides from one
//     pointer per lane (one branch-free pass for every chunk that lies inside the series).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "wave.h"

namespace ccm {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kBTN = 64;      // targets per tile
constexpr int kBRows = 128;   // rows of A per chunk
constexpr int kHalf = 32;     // rows of A per wave
constexpr int kStage = 64;    // K per stage
// LDS row stride of the A and B tiles in BF16 elements: 64 + 8 pad, so the 16 rows read
// by one 16-lane pass of a 128-bit fragment load start 36 banks apart and never collide
constexpr int kRS = kStage + 8;
constexpr int kBThreads = 512;
constexpr int kMaxStages = 16384 / kStage;  // L <= 16384

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  __bf16 b = (__bf16)f;  // round to nearest even
  return __builtin_bit_cast(uint16_t, b);
}

// Centring value of each target column: its mean over t = 0..L-1 (FP64 sum) rounded to
// FP32.  The BF16 operands and the FP32 epilogue sums work on y - c, so a large offset of a
// series costs no digits (rho does not change under a common shift of y and yhat, and the
// weights sum to 1).  Block = 64 columns x 4 row groups.
__global__ __launch_bounds__(256) void column_ref_kernel(const float* __restrict__ ts, int64_t ld,
                                                         int L, int tgt0, int n_tgt,
                                                         float* __restrict__ cref) {
  __shared__ double part[4][64];
  const int tx = threadIdx.x & 63;
  const int ty = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + tx;
  double a = 0.0;
  if (j < n_tgt)
    for (int t = ty; t < L; t += 4) a += ts[(int64_t)t * ld + tgt0 + j];
  part[ty][tx] = a;
  __syncthreads();
  if (ty == 0 && j < n_tgt)
    cref[j] = (float)((part[0][tx] + part[1][tx] + part[2][tx] + part[3][tx]) / L);
}

// Y (time-major, FP32) -> Yt [n_tgt][Lpad] BF16 of y - c (c = cref of the column), zero
// beyond L.
__global__ __launch_bounds__(256) void transpose_bf16_kernel(const float* __restrict__ ts, int64_t ld,
                                                             int L, int tgt0, int n_tgt, int Lpad,
                                                             const float* __restrict__ cref,
                                                             uint16_t* __restrict__ yt) {
  __shared__ float tile[64][65];
  const int j0 = blockIdx.x * 64;
  const int t0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63;
  const int ty = threadIdx.x >> 6;
  const float cx = j0 + tx < n_tgt ? cref[j0 + tx] : 0.0f;
  for (int r = ty; r < 64; r += 4) {
    const int t = t0 + r, j = j0 + tx;
    tile[r][tx] = (t < L && j < n_tgt) ? ts[(int64_t)t * ld + tgt0 + j] - cx : 0.0f;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int j = j0 + r, t = t0 + tx;
    if (j < n_tgt && t < Lpad) yt[(size_t)j * Lpad + t] = bf16_bits(tile[tx][r]);
  }
}

// Per (chunk, library): sort the chunk's table entries by (stage, row quarter), quarter =
// row / 32 (the rows of one wave).  Entry = row (7 bits) | column within stage (6 bits) << 7
// | BF16 weight << 16.  Offsets [4 nst + 1] per chunk.
__global__ __launch_bounds__(kBRows) void bf16_entries_kernel(
    const int* __restrict__ nbr_idx, const float* __restrict__ nbr_w, const int* __restrict__ lib_E,
    int L, int k_max, int tau, int nchunk_max, int nst, uint32_t* __restrict__ ent,
    int* __restrict__ stage_off, int* __restrict__ lib_k) {
  __shared__ int cnt[4 * kMaxStages];
  __shared__ int cur[4 * kMaxStages];
  const int c = blockIdx.x;
  const int i = blockIdx.y;
  const int E = lib_E[i];
  const int k = E + 1;
  const int lo = (E - 1) * tau;
  bool libok = E >= 1 && E <= kEMax && k <= k_max && (L - lo) >= k + 1;
  if (libok) libok = nbr_idx[((size_t)i * L + lo) * k_max] >= 0;
  if (c == 0 && threadIdx.x == 0) lib_k[i] = libok ? k : 0;
  const int nb = 4 * nst;
  for (int q = threadIdx.x; q < nb; q += blockDim.x) cnt[q] = 0;
  __syncthreads();
  const int row = threadIdx.x;
  const int t = lo + c * kBRows + row;
  const bool rowok = libok && t < L;
  int sidx[kKMax];
  float wv[kKMax];
  if (rowok) {
    for (int m = 0; m < k; ++m) {
      const int v = nbr_idx[((size_t)i * L + t) * k_max + m];
      sidx[m] = (v >= 0 && v < L) ? v : -1;
      wv[m] = nbr_w[((size_t)i * L + t) * k_max + m];
      if (sidx[m] >= 0) atomicAdd(&cnt[4 * (sidx[m] / kStage) + (row >> 5)], 1);
    }
  }
  __syncthreads();
  int* so = stage_off + ((size_t)i * nchunk_max + c) * (nb + 1);
  if (threadIdx.x == 0) {
    int p = 0;
    for (int q = 0; q < nb; ++q) {
      cur[q] = p;
      so[q] = p;
      p += cnt[q];
    }
    so[nb] = p;
  }
  __syncthreads();
  uint32_t* eo = ent + ((size_t)i * nchunk_max + c) * (kBRows * kKMax);
  if (rowok)
    for (int m = 0; m < k; ++m)
      if (sidx[m] >= 0) {
        const int q = 4 * (sidx[m] / kStage) + (row >> 5);
        const int p = atomicAdd(&cur[q], 1);
        eo[p] = (uint32_t)row | ((uint32_t)(sidx[m] % kStage) << 7) |
                ((uint32_t)bf16_bits(wv[m]) << 16);
      }
}

__global__ __launch_bounds__(kBThreads, 2) void gather_bf16_kernel(
    const float* __restrict__ ts, int64_t ld, int L, int tau, int tgt0, int n_tgt, int Lpad,
    const uint16_t* __restrict__ yt, const float* __restrict__ cref, const uint32_t* __restrict__ ent,
    const int* __restrict__ stage_off, const int* __restrict__ order, const int* __restrict__ lib_k,
    int n_lib, int nchunk_max, int nst, float* __restrict__ rho, double* __restrict__ moments) {
  extern __shared__ __align__(16) char smem[];
  // B: two stages of Yt [64 targets][64 s] BF16 (9 KB each); A: per wave [32 rows][64 s]
  uint16_t* Bs = (uint16_t*)smem;
  uint16_t* As = (uint16_t*)(smem + 2 * kBTN * kRS * 2);
  // the current chunk's sorted entries of both libraries
  uint32_t* Es = (uint32_t*)(smem + 2 * kBTN * kRS * 2 + 8 * kHalf * kRS * 2);
  const int lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int half = wave & 3;     // rows 32*half .. 32*half+31 of each 128-row chunk
  // blockIdx.x = library pair (fastest), blockIdx.y = target tile: the workgroups resident
  // at one time share a target tile, whose BF16 and FP32 columns then stay in L2
  const int j0 = blockIdx.y * kBTN;
  const int li = blockIdx.x * 2 + (wave >> 2);
  const bool has = li < n_lib;
  const int i = has ? __builtin_amdgcn_readfirstlane(order[li]) : 0;
  const int k = has ? __builtin_amdgcn_readfirstlane(lib_k[i]) : 0;
  const int E = k - 1;
  const int lo = k > 0 ? (E - 1) * tau : 0;
  const int nrows = k > 0 ? L - lo : 0;
  const int nchunk = (nrows + kBRows - 1) / kBRows;
  __shared__ int s_nchunk[8];
  if (lane == 0) s_nchunk[wave] = nchunk;
  uint16_t* Aw = As + (size_t)wave * kHalf * kRS;
  for (int q = lane; q < kHalf * kRS / 2; q += kWave) ((uint32_t*)Aw)[q] = 0u;
  // centring values of this lane's two columns (the epilogue works on y - c, as Yt does)
  float cy[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int j = j0 + 32 * b + (lane & 31);
    cy[b] = j < n_tgt ? cref[j] : 0.0f;
  }
  // FP64 moment sums of this lane's two columns: y, y^2, yhat, yhat^2, y * yhat
  double M[5][2];
#pragma unroll
  for (int q = 0; q < 5; ++q) M[q][0] = M[q][1] = 0.0;
  __syncthreads();
  const int nch_all = max(max(max(s_nchunk[0], s_nchunk[1]), max(s_nchunk[2], s_nchunk[3])),
                          max(max(s_nchunk[4], s_nchunk[5]), max(s_nchunk[6], s_nchunk[7])));

  // B stage loader: thread -> (target row r = tid/8, eighth q = tid%8): 16 bytes
  const int br = threadIdx.x >> 3;
  const int bq = threadIdx.x & 7;
  const uint16_t* ysrc = yt + (size_t)(j0 + br) * Lpad + bq * 8;
  const bool brow_ok = j0 + br < n_tgt;

  for (int c = 0; c < nch_all; ++c) {
    f32x16 acc[1][2];
#pragma unroll
    for (int a = 0; a < 1; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    const bool mine = c < nchunk;
    // stage this chunk's entries in LDS (the four waves of a library split the copy); the
    // bucket offsets of this wave's quarter are read as uniform values from memory
    uint32_t* eo = Es + (size_t)(wave >> 2) * kBRows * kKMax;
    const int* sg = stage_off + ((size_t)i * nchunk_max + c) * (4 * nst + 1) + half;
    __syncthreads();  // previous chunk is done with Es
    if (mine) {
      const uint32_t* eg = ent + ((size_t)i * nchunk_max + c) * (kBRows * kKMax);
      const int ne = sg[4 * nst - half];
      for (int q = half * kWave + lane; q < ne; q += 4 * kWave) eo[q] = eg[q];
    }
    // B stages travel through registers two stages ahead of their use
    uint4 breg[1], breg2[1];
#pragma unroll
    for (int q = 0; q < 1; ++q) {
      breg[q] = brow_ok ? *(const uint4*)(ysrc + q * 8) : uint4{0, 0, 0, 0};
      breg2[q] = (brow_ok && nst > 1) ? *(const uint4*)(ysrc + kStage + q * 8) : uint4{0, 0, 0, 0};
    }
    __syncthreads();  // staged entries visible to both waves of each library
    // one stage; R holds this stage's B rows and is reloaded with stage st + 2 once stored,
    // so the two register sets alternate without copies
    auto stage = [&](int st, uint4 (&R)[1]) {
      const int buf = st & 1;
      // scatter this wave's nonzeros of the stage (its own bucket)
      int e0 = 0, e1 = 0;
      if (mine) {
        e0 = sg[4 * st];
        e1 = sg[4 * st + 1];
      }
      for (int e = e0 + lane; e < e1; e += kWave) {
        const uint32_t v = eo[e];
        Aw[(v & 31) * kRS + ((v >> 7) & 63)] = (uint16_t)(v >> 16);
      }
      {
        uint16_t* dst = Bs + (size_t)buf * kBTN * kRS + br * kRS + bq * 8;
        *(uint4*)dst = R[0];
      }
      __syncthreads();  // B stage `buf` complete; the other buffer is free
#pragma unroll
      for (int q = 0; q < 1; ++q)
        R[q] = (brow_ok && st + 2 < nst) ? *(const uint4*)(ysrc + (size_t)(st + 2) * kStage + q * 8)
                                         : uint4{0, 0, 0, 0};
      const uint16_t* Bb = Bs + (size_t)buf * kBTN * kRS;
      // fragments of k-step kk + 1 are read while the products of kk run
      const uint16_t* ap = Aw + (lane & 31) * kRS + 8 * (lane >> 5);
      const uint16_t* bp = Bb + (lane & 31) * kRS + 8 * (lane >> 5);
      bf16x8 fa[2], fb0[2], fb1[2];
      // raised priority while the fragments and products of the stage issue, so waves in
      // their MFMA phase run ahead of waves scattering or clearing entries (227 -> 222 ms on
      // 512 x 101,729, identical rho)
      __builtin_amdgcn_s_setprio(1);
      fa[0] = *(const bf16x8*)ap;
      fb0[0] = *(const bf16x8*)bp;
      fb1[0] = *(const bf16x8*)(bp + 32 * kRS);
#pragma unroll
      for (int kk = 0; kk < kStage / 16; ++kk) {
        const int c = kk & 1, n = c ^ 1;
        if (kk + 1 < kStage / 16) {
          fa[n] = *(const bf16x8*)(ap + 16 * (kk + 1));
          fb0[n] = *(const bf16x8*)(bp + 16 * (kk + 1));
          fb1[n] = *(const bf16x8*)(bp + 32 * kRS + 16 * (kk + 1));
        }
        __builtin_amdgcn_sched_barrier(0);   // keep the reads of kk + 1 ahead of these products
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[c], fb0[c], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[c], fb1[c], acc[0][1], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      __builtin_amdgcn_s_setprio(0);
      // clear this wave's nonzeros again (after its own reads, in program order)
      for (int e = e0 + lane; e < e1; e += kWave) Aw[(eo[e] & 31) * kRS + ((eo[e] >> 7) & 63)] = 0;
    };
    int st = 0;
    for (; st + 1 < nst; st += 2) {
      stage(st, breg);
      stage(st + 1, breg2);
    }
    if (st < nst) stage(st, breg);
    // epilogue: moments of this chunk's rows
    if (mine) {
      // accumulator element r of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4 of the
      // wave's 32; the observed y of those rows are read at uniform strides from one pointer
      const int trow = lo + c * kBRows + kHalf * half + 4 * (lane >> 5);
      const bool full = lo + c * kBRows + kHalf * half + kHalf <= L;   // uniform
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = j0 + 32 * b + (lane & 31);
        float sy = 0.f, syy = 0.f, sp = 0.f, spp = 0.f, syp = 0.f;
        if (j < n_tgt) {
          const float* yb = ts + (int64_t)trow * ld + tgt0 + j;
          if (full) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const float y = yb[(int64_t)(8 * (r >> 2) + (r & 3)) * ld] - cy[b];
              const float p = acc[0][b][r];
              sy += y;
              syy = fmaf(y, y, syy);
              sp += p;
              spp = fmaf(p, p, spp);
              syp = fmaf(y, p, syp);
            }
          } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              if (trow + 8 * (r >> 2) + (r & 3) < L) {
                const float y = yb[(int64_t)(8 * (r >> 2) + (r & 3)) * ld] - cy[b];
                const float p = acc[0][b][r];
                sy += y;
                syy = fmaf(y, y, syy);
                sp += p;
                spp = fmaf(p, p, spp);
                syp = fmaf(y, p, syp);
              }
            }
          }
        }
        M[0][b] += sy;
        M[1][b] += syy;
        M[2][b] += sp;
        M[3][b] += spp;
        M[4][b] += syp;
      }
    }
  }
  // combine lanes l, l+32 (same column, other rows), then the two row halves (waves 2m,
  // 2m+1) through LDS (the A tiles are no longer needed)
#pragma unroll
  for (int q = 0; q < 5; ++q)
#pragma unroll
    for (int b = 0; b < 2; ++b) M[q][b] += __shfl_xor(M[q][b], 32);
  __syncthreads();
  double* red = (double*)As;   // [2 libraries][3 parts][5][2][32]
  if (half >= 1 && lane < 32)
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        red[((((wave >> 2) * 3 + half - 1) * 5 + q) * 2 + b) * 32 + lane] = M[q][b];
  __syncthreads();
  if (!has || half != 0 || lane >= 32) return;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    double S[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      S[q] = M[q][b];
      for (int h = 0; h < 3; ++h) S[q] += red[((((wave >> 2) * 3 + h) * 5 + q) * 2 + b) * 32 + lane];
    }
    const int j = j0 + 32 * b + lane;
    if (j < n_tgt) {
      const double n = (double)nrows;
      const double r = k > 0 ? pearson_shifted(n, cy[b], S[0], S[1], S[2], S[3], S[4])
                             : __builtin_nan("");
      rho[(size_t)i * n_tgt + j] = (float)r;
      if (moments) {
        double* mo = moments + ((size_t)i * n_tgt + j) * 3;
        if (k > 0) {
          unshift_moments(n, cy[b], S[0], S[2], S[3], S[4], mo);
        } else {
          mo[0] = mo[1] = mo[2] = __builtin_nan("");
        }
      }
    }
  }
}

}  // namespace ccm

extern "C" hipError_t ccm_launch_order(const int* lib_k, int n_lib, int* order, hipStream_t stream);

extern "C" size_t ccm_bf16_lds_bytes() {
  return 2 * (size_t)ccm::kBTN * ccm::kRS * 2 + 8 * (size_t)ccm::kHalf * ccm::kRS * 2 +
         2 * (size_t)ccm::kBRows * ccm::kKMax * 4;
}

extern "C" hipError_t ccm_launch_crossmap_bf16(const float* ts, int64_t ld, int L, int tau, int tgt0,
                                               int n_tgt, const int* nbr_idx, const float* nbr_w,
                                               const int* lib_E, int n_lib, int k_max, float* rho,
                                               double* moments, uint16_t* yt, float* cref,
                                               uint32_t* ent, int* stage_off, int* lib_k,
                                               int* order, hipStream_t stream) {
  if (n_lib == 0 || n_tgt == 0) return hipSuccess;
  const int nst = (L + ccm::kStage - 1) / ccm::kStage;
  const int Lpad = nst * ccm::kStage;
  const int nchunk_max = (L + ccm::kBRows - 1) / ccm::kBRows;
  hipLaunchKernelGGL(ccm::column_ref_kernel, dim3((n_tgt + 63) / 64), dim3(256), 0, stream, ts, ld,
                     L, tgt0, n_tgt, cref);
  hipLaunchKernelGGL(ccm::transpose_bf16_kernel, dim3((n_tgt + 63) / 64, Lpad / 64), dim3(256), 0,
                     stream, ts, ld, L, tgt0, n_tgt, Lpad, (const float*)cref, yt);
  hipLaunchKernelGGL(ccm::bf16_entries_kernel, dim3(nchunk_max, n_lib), dim3(ccm::kBRows), 0, stream,
                     nbr_idx, nbr_w, lib_E, L, k_max, tau, nchunk_max, nst, ent, stage_off, lib_k);
  hipError_t e = ccm_launch_order(lib_k, n_lib, order, stream);
  if (e != hipSuccess) return e;
  static std::atomic<uint64_t> attr{0};
  e = ccm::allow_lds_once((const void*)ccm::gather_bf16_kernel, attr, ccm_bf16_lds_bytes());
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ccm::gather_bf16_kernel, dim3((n_lib + 1) / 2, (n_tgt + ccm::kBTN - 1) / ccm::kBTN),
                     dim3(ccm::kBThreads), ccm_bf16_lds_bytes(), stream, ts, ld, L, tau, tgt0, n_tgt,
                     Lpad, yt, (const float*)cref, ent, stage_off, order, lib_k, n_lib, nchunk_max,
                     nst, rho, moments);
  return hipGetLastError();
}
