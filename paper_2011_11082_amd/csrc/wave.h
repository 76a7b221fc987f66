// Wavefront-level helpers for gfx950 (64-lane waves).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

namespace ccm {

// Raise a kernel's dynamic LDS limit to `bytes` (or, with bytes = 0, to all of the CU's
// 160 KB left beside its static LDS) once per device: the attribute belongs to the device
// the call is made on, so `done` keeps one bit per device id (ids below 64).
inline hipError_t allow_lds_once(const void* kernel, std::atomic<uint64_t>& done,
                                 size_t bytes = 0) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const uint64_t bit = dev >= 0 && dev < 64 ? (uint64_t)1 << dev : 0;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
  if (bytes == 0) {
    hipFuncAttributes fa;
    e = hipFuncGetAttributes(&fa, kernel);
    if (e != hipSuccess) return e;
    bytes = 160 * 1024 - fa.sharedSizeBytes;
  }
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_acq_rel);
  return e;
}

constexpr int kWave = 64;
constexpr int kEMax = 20;
constexpr int kKMax = kEMax + 1;
static_assert(kKMax <= 32, "a neighbour list must fit in lanes 0..31");

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ float readlane(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ int readlane(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// DPP wave_shr:1 -- lane i receives lane i-1; lane 0 keeps `old`.
__device__ __forceinline__ float wave_shr1(float v, float old) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ int wave_shr1(int v, int old) {
  return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xF, 0xF, false);
}

// DPP quad_perm broadcast: every lane of a quad receives lane M of that quad (every source
// lane exists, so no "old" value is needed).
template <int M>
__device__ __forceinline__ int quad_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, M * 0x55, 0xF, 0xF, true);
}
template <int M>
__device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), M * 0x55, 0xF, 0xF, true));
}

// Sum over all 64 lanes (result in every lane).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// DPP move of a double (both halves), every lane a valid source.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum of lanes 0..31 (lanes 32..63 are ignored), returned in every lane: pairs and quads by
// quad_perm, then rotations by 4 and 8 inside each row of 16, then the two row sums.  No LDS
// round trip, unlike a shuffle butterfly.
__device__ __forceinline__ double lanes32_sum(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0x124>(v);   // row_ror:4
  v += dpp_f64<0x128>(v);   // row_ror:8
  const double r0 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                                     __builtin_amdgcn_readlane(__double2loint(v), 0));
  const double r1 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 16),
                                     __builtin_amdgcn_readlane(__double2loint(v), 16));
  return r0 + r1;
}

// Pearson correlation from one-pass FP64 moments of n pairs (y, p).  A variance below the
// rounding level of the data (relative 1e-10 of the raw second moment) counts as zero and
// gives NaN.
__device__ __forceinline__ double pearson_from_moments(double n, double sy, double syy, double sp,
                                                       double spp, double syp) {
  double vy = n * syy - sy * sy;
  double vp = n * spp - sp * sp;
  if (!(vy > 1e-10 * n * syy) || !(vp > 1e-10 * n * spp)) return __builtin_nan("");
  return (n * syp - sy * sp) / sqrt(vy * vp);
}

// The same from moments of shifted values y' = y - c and p' = p - c, where c is a reference
// value of the target column (its mean rounded to FP32): Pearson's rho does not change under
// a common shift, and with the column centred the FP32 products and one-pass moments no
// longer lose digits to a large mean.  The zero-variance test still compares with the raw
// second moments, sum (y' + c)^2 = syy' + c (2 sy' + n c), as for unshifted moments.
__device__ __forceinline__ double pearson_shifted(double n, double c, double sy, double syy,
                                                  double sp, double spp, double syp) {
  const double vy = n * syy - sy * sy;
  const double vp = n * spp - sp * sp;
  const double ryy = syy + c * (2.0 * sy + n * c);
  const double rpp = spp + c * (2.0 * sp + n * c);
  if (!(vy > 1e-10 * n * ryy) || !(vp > 1e-10 * n * rpp)) return __builtin_nan("");
  return (n * syp - sy * sp) / sqrt(vy * vp);
}

// Raw moments sum(p), sum(p^2), sum(y p) from shifted ones (p = p' + c, y = y' + c).
__device__ __forceinline__ void unshift_moments(double n, double c, double sy, double sp,
                                                double spp, double syp, double* out) {
  out[0] = sp + n * c;
  out[1] = spp + c * (2.0 * sp + n * c);
  out[2] = syp + c * (sy + sp + n * c);
}

}  // namespace ccm
