// Internal device helpers shared by the library's kernels (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "coulomb_disk.h"

namespace cd {

// Charges per block: one block is one 64-lane wavefront, one charge per lane.
constexpr int kBlk = 64;

// Pad charges fill the last block (or super-block).  They sit far outside
// the disk on the x axis, 1e29 apart: in FP32 every difference involving a
// pad squares to
// +inf, v_rsq_f32(+inf) = 0 and every term it feeds is exactly zero; in FP64
// a pad term is below 1e-29 relative to a real one.
__host__ __device__ inline double pad_x(int64_t k) { return 1e30 + 1e29 * (double)k; }

// DPP lane rotation within 16-lane rows: row_ror:K gives lane q the value of
// lane (q - K) mod 16 of the same row.  bound_ctrl makes the compiler fold
// the move into the consuming VALU instruction.
template <int K>
__device__ __forceinline__ float row_ror(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x120 + K, 0xf, 0xf, true));
}

// 1/sqrt(r2) in FP64: the hardware seed v_rsq_f64 (about 2^-23 relative
// error) refined by one third-order step of the Taylor series of
// (1 - e)^(-1/2): y1 = y0 (1 + e/2 + 3 e^2 / 8), e = 1 - r2 y0^2.  The
// truncation term is 5 e^3 / 16 < 2^-60, so the result is within about two
// ulp.  r2 must be finite and positive.
__device__ __forceinline__ double rsqrt64(double r2) {
  double y0 = __builtin_amdgcn_rsq(r2);
  double e = __builtin_fma(-r2 * y0, y0, 1.0);
  double p = __builtin_fma(e, 0.375, 0.5);
  return __builtin_fma(y0 * e, p, y0);
}

// Wave-wide sums (64 lanes) with a fixed butterfly order: deterministic.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmin(v, __shfl_xor(v, m, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
  return v;
}

// Wave-wide sum and maximum by DPP: lanes combine within their 16-lane row
// (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror),
// then the four row results are read by readlane and combined in row order.
// Fixed order; every lane gets the result.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int2 b = __builtin_bit_cast(int2, v);
  const int lo = __builtin_amdgcn_update_dpp(0, b.x, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, b.y, CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, make_int2(lo, hi));
}
__device__ __forceinline__ double lane_f64(double v, int lane) {
  const int2 b = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(b.x, lane),
                                              __builtin_amdgcn_readlane(b.y, lane)));
}
__device__ __forceinline__ double wave_sum_rows(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  return ((lane_f64(v, 0) + lane_f64(v, 16)) + lane_f64(v, 32)) + lane_f64(v, 48);
}
__device__ __forceinline__ double wave_max_rows(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  return fmax(fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), lane_f64(v, 32)), lane_f64(v, 48));
}

// Workspace carving: bump allocator with 256-byte alignment.
struct Carve {
  size_t off = 0;
  char* base = nullptr;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
};

inline int hip_status(hipError_t e) { return e == hipSuccess ? CD_OK : CD_ERR_HIP; }

}  // namespace cd
