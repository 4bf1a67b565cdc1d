// Border-interior split of the charges (paper Sec. II.B): the boundary
// population of Eq. 4, the initial interior radius of Eq. 5, which charges
// are boundary charges (the N_b farthest from the centre), and the
// projection of a configuration onto the split's feasible set.
//
// k_border_select: one 1024-thread workgroup.  The key of charge i is the
// bit pattern of r2 = (x*x) + (y*y) (separately rounded, non-negative, so it
// orders like the value), complemented so that far charges come first; an
// exact 8-pass radix select finds the N_b-th smallest key, then every charge
// below it and, among charges equal to it, the lowest indices are flagged.
#include <cmath>

#include "common.hpp"

namespace cd {

constexpr int kBT = 1024;

#pragma clang fp contract(off)
__device__ __forceinline__ uint64_t border_key(double x, double y) {
  const double a = x * x, b = y * y;
  const double r2 = a + b;
  return ~(uint64_t)__double_as_longlong(r2);
}
#pragma clang fp contract(on)

__global__ __launch_bounds__(kBT) void k_border_select(const double* __restrict__ x,
                                                       const double* __restrict__ y, int n,
                                                       int nb, int32_t* __restrict__ flags) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix, s_mask;
  __shared__ uint32_t s_need;
  __shared__ uint32_t lt_cnt[kBT], eq_cnt[kBT];
  const int t = threadIdx.x;
  if (t == 0) {
    s_prefix = 0;
    s_mask = 0;
    s_need = (uint32_t)nb;
  }
  __syncthreads();
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    if (t < 256) hist[t] = 0;
    __syncthreads();
    const uint64_t pre = s_prefix, msk = s_mask;
    for (int j = t; j < n; j += kBT) {
      const uint64_t key = border_key(x[j], y[j]);
      if ((key & msk) == pre) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (t == 0) {
      uint32_t need = s_need, b = 0;
      while (b < 255 && hist[b] < need) need -= hist[b++];
      s_need = need;
      s_prefix = pre | ((uint64_t)b << shift);
      s_mask = msk | ((uint64_t)255 << shift);
    }
    __syncthreads();
  }
  const uint64_t T = s_prefix;
  const uint32_t need_eq = nb > 0 ? s_need : 0u;  // charges at exactly T that are boundary
  // flags in index order: contiguous chunks per thread, so ties go to lower indices
  const int chunk = (n + kBT - 1) / kBT;
  const int j0 = min(n, t * chunk), j1 = min(n, j0 + chunk);
  uint32_t eq = 0;
  for (int j = j0; j < j1; ++j) eq += border_key(x[j], y[j]) == T;
  eq_cnt[t] = eq;
  lt_cnt[t] = 0;
  __syncthreads();
  for (int off = 1; off < kBT; off <<= 1) {
    const uint32_t b = t >= off ? eq_cnt[t - off] : 0u;
    __syncthreads();
    eq_cnt[t] += b;
    __syncthreads();
  }
  uint32_t eq_before = eq_cnt[t] - eq;
  for (int j = j0; j < j1; ++j) {
    const uint64_t key = border_key(x[j], y[j]);
    int f = 0;
    if (nb > 0) {
      if (key < T) {
        f = 1;
      } else if (key == T) {
        f = eq_before < need_eq;
        ++eq_before;
      }
    }
    flags[j] = f;
  }
}

// In-place projection onto the split's feasible set: a boundary charge onto
// the unit circle (x / r), any other charge beyond sigma onto the circle of
// radius sigma (x * (sigma / r)); every operation rounded once in FP64.
#pragma clang fp contract(off)
__global__ void k_border_project(double* __restrict__ x, double* __restrict__ y, int n,
                                 const int32_t* __restrict__ flags, double sigma) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double px = x[i], py = y[i];
  const double a = px * px, b = py * py;
  const double r = sqrt(a + b);
  if (flags && flags[i]) {
    if (r > 0.0) {
      x[i] = px / r;
      y[i] = py / r;
    }
  } else if (r > sigma) {
    const double f = sigma / r;
    x[i] = px * f;
    y[i] = py * f;
  }
}
#pragma clang fp contract(on)

// Spread of the boundary charges, the split's start before a cycle (a step
// the paper leaves open; projecting the boundary charges of an unrelaxed
// configuration along their rays lands charges of adjacent rings almost on
// top of each other): the flagged charges, ordered by theta = atan2(y, x)
// with ties to the lower index, go onto the unit circle at theta_0 +
// 2 pi k / nb (k their rank, theta_0 the angle of the first).  One
// workgroup: the flagged charges are listed in index order with their angles
// (contiguous chunks per thread and a scan), then each counts the listed
// charges before it in that order -- O(nb^2) comparisons, nb the boundary
// population of Eq. 4 (6099 at N = 1e5).  Scratch: list, rank int32 [n],
// theta double [n].
#pragma clang fp contract(off)
__global__ __launch_bounds__(kBT) void k_border_spread(double* __restrict__ x,
                                                       double* __restrict__ y, int n,
                                                       const int32_t* __restrict__ flags,
                                                       int32_t* __restrict__ list,
                                                       int32_t* __restrict__ rank,
                                                       double* __restrict__ theta) {
  __shared__ uint32_t cnt[kBT];
  __shared__ double s_th0;
  const int t = threadIdx.x;
  const int chunk = (n + kBT - 1) / kBT;
  const int j0 = min(n, t * chunk), j1 = min(n, j0 + chunk);
  uint32_t c = 0;
  for (int j = j0; j < j1; ++j) c += flags[j] != 0;
  cnt[t] = c;
  __syncthreads();
  for (int off = 1; off < kBT; off <<= 1) {
    const uint32_t b = t >= off ? cnt[t - off] : 0u;
    __syncthreads();
    cnt[t] += b;
    __syncthreads();
  }
  uint32_t pos = cnt[t] - c;
  for (int j = j0; j < j1; ++j) {
    if (flags[j]) {
      list[pos] = j;
      theta[pos] = atan2(y[j], x[j]);
      ++pos;
    }
  }
  const int nb = (int)cnt[kBT - 1];
  __syncthreads();  // the list and the angles are complete (workgroup scope)
  for (int k = t; k < nb; k += kBT) {
    const double th = theta[k];
    int r = 0;
    for (int q = 0; q < nb; ++q) {
      const double tq = theta[q];
      r += (tq < th) || (tq == th && q < k);
    }
    rank[k] = r;
    if (r == 0) s_th0 = th;
  }
  __syncthreads();
  const double th0 = s_th0;
  for (int k = t; k < nb; k += kBT) {
    const double phi = th0 + ((2.0 * 3.141592653589793) * (double)rank[k]) / (double)nb;
    const int j = list[k];
    x[j] = cos(phi);
    y[j] = sin(phi);
  }
}
#pragma clang fp contract(on)

size_t border_workspace_bytes(int64_t n) {
  if (n < 1 || n > (1 << 26)) return 0;
  return (size_t)n * 16 + 1024;
}

}  // namespace cd

using namespace cd;

extern "C" {

#pragma clang fp contract(off)
int32_t border_count(int64_t n) {
  if (n < 1) return 0;
  const double c = pow((double)n, 1.0 / 3.0);
  const double v = floor(2.84328 * c * c - 0.530196 * c - 2.32866 + 0.5);
  if (v < 0.0) return 0;
  return v > (double)n ? (int32_t)n : (int32_t)v;
}

double border_sigma0(int64_t n) {
  if (n < 1) return 1.0;
  return 1.0 - 1.0 / (2.0 * sqrt((double)n));
}

double border_sigma_ramp(int64_t n, int32_t k, int32_t stages, double sigma_start,
                         double sigma_end) {
  const double s0 = sigma_start > 0.0 ? sigma_start : border_sigma0(n);
  if (stages <= 0) return sigma_end;
  const int32_t kk = k < 0 ? 0 : (k > stages ? stages : k);
  return s0 + (sigma_end - s0) * ((double)kk / (double)stages);
}
#pragma clang fp contract(on)

int border_split(const double* x, const double* y, int64_t n, int32_t nb, int32_t* flags,
                 void* stream) {
  if (!x || !y || !flags || n < 1 || n > (1 << 26) || nb < 0 || nb > n) return CD_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_border_select, dim3(1), dim3(kBT), 0, (hipStream_t)stream, x, y, (int)n,
                     (int)nb, flags);
  return hip_status(hipGetLastError());
}

int border_spread(double* x, double* y, int64_t n, const int32_t* flags, void* ws,
                  size_t ws_bytes, void* stream) {
  if (!x || !y || !flags || n < 1 || n > (1 << 26)) return CD_ERR_INVALID_ARG;
  if (!ws || ws_bytes < border_workspace_bytes(n)) return CD_ERR_WORKSPACE;
  Carve cv;
  cv.base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  int32_t* list = cv.take<int32_t>(n);
  int32_t* rank = cv.take<int32_t>(n);
  double* theta = cv.take<double>(n);
  hipLaunchKernelGGL(k_border_spread, dim3(1), dim3(kBT), 0, (hipStream_t)stream, x, y, (int)n,
                     flags, list, rank, theta);
  return hip_status(hipGetLastError());
}

int border_project(double* x, double* y, int64_t n, const int32_t* flags, double sigma,
                   void* stream) {
  if (!x || !y || n < 1 || n > (1 << 26) || !(sigma > 0.0 && sigma <= 1.0))
    return CD_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_border_project, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, x, y, (int)n, flags, sigma);
  return hip_status(hipGetLastError());
}

}  // extern "C"
