// Defect-targeted zones of the subdomain cycle (paper Sec. II.C, steps 2-4
// and the oscillating zone radius).
//
//  - k_defect_stats: one workgroup.  Mean and population standard deviation
//    of the local energies (fixed-order FP64 sums), the threshold
//    mu + kappa*sigma_e and the list of charges above it, compacted tile by
//    tile in increasing index order.
//  - k_zone_pick: one thread per zone.  Centre (a defect charge or the
//    caller's disk point, by the caller's uniform draws) and the radius of
//    the triangle wave.
//  - k_zone_count / k_zone_fill: one workgroup per zone.  Every charge within
//    the radius, counted, then listed in increasing index order.
//  - zone_batches: host code.  Greedy assignment of the zones to batches of
//    mutually distant zones (in sequence order, or first fit), with a
//    uniform grid over the centres.
//
// The comparisons that decide membership are taken on separately rounded
// FP64 operations (no contraction), so the lists are reproducible exactly.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace cd {

constexpr int kZT = 1024;  // threads of the one-workgroup kernels
constexpr int kZW = kZT / 64;

size_t zones_workspace_bytes(int op, int64_t n, int32_t n_zones) {
  Carve c;
  if (op == CD_OP_DEFECT) {
    c.take<int32_t>((size_t)n);
    c.take<double>(4);
  } else {
    c.take<int32_t>((size_t)n_zones);
    c.take<int32_t>((size_t)n_zones + 1);
  }
  return c.off + 256;
}

// Sum of one double per thread over a 1024-thread workgroup in a fixed
// order: butterfly inside each wave, then the 16 wave sums in order.
__device__ double block_sum_fixed(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < kZW; ++q) s += red[q];
  __syncthreads();
  return s;
}

// Exclusive prefix of a 0/1 flag over the workgroup (thread order) and the
// total count.
__device__ int block_prefix_flag(bool f, int* wcnt, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t b = __ballot(f);
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  if (lane == 0) wcnt[w] = __popcll(b);
  __syncthreads();
  int before = 0;
  total = 0;
  for (int q = 0; q < kZW; ++q) {
    before += q < w ? wcnt[q] : 0;
    total += wcnt[q];
  }
  __syncthreads();
  return before + __popcll(b & lt);
}

#pragma clang fp contract(off)

__global__ __launch_bounds__(kZT) void k_defect_stats(const double* __restrict__ e, int n,
                                                      double kappa, double* __restrict__ stats,
                                                      int32_t* __restrict__ list) {
  __shared__ double red[kZW];
  __shared__ int wcnt[kZW];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int j = t; j < n; j += kZT) s += e[j];
  const double mu = block_sum_fixed(s, red) / (double)n;
  double q = 0.0;
  for (int j = t; j < n; j += kZT) {
    const double d = e[j] - mu;
    q += d * d;
  }
  const double var = block_sum_fixed(q, red) / (double)n;
  const double sigma = __dsqrt_rn(var);
  const double ks = kappa * sigma;
  const double thr = mu + ks;
  int base = 0;
  for (int j0 = 0; j0 < n; j0 += kZT) {
    const int j = j0 + t;
    const bool f = j < n && e[j] > thr;
    int total;
    const int pos = block_prefix_flag(f, wcnt, total);
    if (f) list[base + pos] = j;
    base += total;
  }
  if (t == 0) {
    stats[0] = mu;
    stats[1] = sigma;
    stats[2] = thr;
    stats[3] = (double)base;
  }
}

__global__ void k_zone_pick(const double* __restrict__ x, const double* __restrict__ y,
                            const double* __restrict__ stats, const int32_t* __restrict__ list,
                            const double* __restrict__ draws, int P, cd_zone_opts o,
                            double* __restrict__ cx, double* __restrict__ cy,
                            double* __restrict__ rz, int32_t* __restrict__ ci) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P) return;
  const double u = draws[4 * (size_t)t], v = draws[4 * (size_t)t + 1];
  const int64_t nd = (int64_t)stats[3];
  if (u < o.p_defect && nd > 0) {
    const double f = floor(v * (double)nd);
    int64_t k = f < 0.0 ? 0 : (int64_t)f;
    if (k > nd - 1) k = nd - 1;
    const int i = list[k];
    cx[t] = x[i];
    cy[t] = y[i];
    ci[t] = i;
  } else {
    cx[t] = draws[4 * (size_t)t + 2];
    cy[t] = draws[4 * (size_t)t + 3];
    ci[t] = -1;
  }
  const int64_t s = (o.t0 + t) % o.period;
  const int64_t m = s < o.period - s ? s : o.period - s;
  const double tri = (double)(2 * m) / (double)o.period;
  const double span = o.r_hi - o.r_lo;
  const double step = span * tri;
  rz[t] = o.r_lo + step;
}

__device__ __forceinline__ bool in_zone(double xj, double yj, double c0, double c1, double r2) {
  const double dx = xj - c0, dy = yj - c1;
  const double a = dx * dx, b = dy * dy;
  const double d2 = a + b;
  return d2 <= r2;
}

__global__ __launch_bounds__(kZT) void k_zone_count(const double* __restrict__ x,
                                                    const double* __restrict__ y, int n,
                                                    const double* __restrict__ cx,
                                                    const double* __restrict__ cy,
                                                    const double* __restrict__ rz,
                                                    int32_t* __restrict__ count) {
  __shared__ int wcnt[kZW];
  const int p = blockIdx.x;
  const double c0 = cx[p], c1 = cy[p], r = rz[p];
  const double r2 = r * r;
  int c = 0;
  for (int j = threadIdx.x; j < n; j += kZT) c += in_zone(x[j], y[j], c0, c1, r2);
  // integer sums are exact in any order
  for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m, 64);
  if ((threadIdx.x & 63) == 0) wcnt[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int q = 0; q < kZW; ++q) s += wcnt[q];
    count[p] = s;
  }
}

__global__ __launch_bounds__(kZT) void k_zone_fill(const double* __restrict__ x,
                                                   const double* __restrict__ y, int n,
                                                   const double* __restrict__ cx,
                                                   const double* __restrict__ cy,
                                                   const double* __restrict__ rz,
                                                   const int32_t* __restrict__ ptr,
                                                   int32_t* __restrict__ out) {
  __shared__ int wcnt[kZW];
  const int p = blockIdx.x;
  const double c0 = cx[p], c1 = cy[p], r = rz[p];
  const double r2 = r * r;
  int32_t* dst = out + ptr[p];
  const int cap = ptr[p + 1] - ptr[p];
  int base = 0;
  for (int j0 = 0; j0 < n; j0 += kZT) {
    const int j = j0 + threadIdx.x;
    const bool f = j < n && in_zone(x[j], y[j], c0, c1, r2);
    int total;
    const int pos = block_prefix_flag(f, wcnt, total);
    if (f && base + pos < cap) dst[base + pos] = j;
    base += total;
  }
}

#pragma clang fp contract(on)

}  // namespace cd

using namespace cd;

namespace {

#pragma clang fp contract(off)
bool zones_conflict(double ax, double ay, double ar, double bx, double by, double br, double gap) {
  const double dx = ax - bx, dy = ay - by;
  const double reach = ar + br + gap;
  const double a = dx * dx, b = dy * dy;
  const double d2 = a + b;
  const double r2 = reach * reach;
  return d2 < r2;
}
#pragma clang fp contract(on)

}  // namespace

extern "C" {

double zone_radius_holding(int64_t n, int64_t count) {
  if (n < 1 || count < 0) return 0.0;
  return sqrt((double)count / (double)n);
}

int defect_zones(const double* x, const double* y, const double* e, int64_t n, int32_t n_zones,
                 const double* draws, const cd_zone_opts* opts, double* cx, double* cy,
                 double* rz, int32_t* centre_idx, double* stats, int32_t* defect_idx, void* ws,
                 size_t ws_bytes, void* stream) {
  if (!x || !y || !e || !opts || n < 1 || n > (1 << 26) || n_zones < 0 ||
      (n_zones > 0 && (!draws || !cx || !cy || !rz || !centre_idx)) || opts->period < 1 ||
      opts->t0 < 0 || !(opts->r_lo >= 0.0) || !(opts->r_hi >= opts->r_lo) ||
      !std::isfinite(opts->r_hi) || !std::isfinite(opts->kappa))
    return CD_ERR_INVALID_ARG;
  if (!ws || ws_bytes < zones_workspace_bytes(CD_OP_DEFECT, n, 0)) return CD_ERR_WORKSPACE;
  Carve c;
  c.base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  int32_t* list = c.take<int32_t>((size_t)n);
  double* st_d = c.take<double>(4);
  if (defect_idx) list = defect_idx;
  if (stats) st_d = stats;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_defect_stats, dim3(1), dim3(kZT), 0, st, e, (int)n, opts->kappa, st_d,
                     list);
  if (n_zones > 0)
    hipLaunchKernelGGL(k_zone_pick, dim3((n_zones + 255) / 256), dim3(256), 0, st, x, y, st_d,
                       list, draws, n_zones, *opts, cx, cy, rz, centre_idx);
  return hip_status(hipGetLastError());
}

int zone_patches(const double* x, const double* y, int64_t n, int32_t n_zones, const double* cx,
                 const double* cy, const double* rz, int32_t* patch_ptr, int32_t* active_idx,
                 int64_t capacity, void* ws, size_t ws_bytes, void* stream) {
  if (!x || !y || !cx || !cy || !rz || !patch_ptr || n < 1 || n > (1 << 26) || n_zones < 1 ||
      capacity < 0 || (capacity > 0 && !active_idx))
    return CD_ERR_INVALID_ARG;
  if (!ws || ws_bytes < zones_workspace_bytes(CD_OP_ZONES, n, n_zones)) return CD_ERR_WORKSPACE;
  Carve c;
  c.base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  int32_t* cnt_d = c.take<int32_t>((size_t)n_zones);
  int32_t* ptr_d = c.take<int32_t>((size_t)n_zones + 1);
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zone_count, dim3(n_zones), dim3(kZT), 0, st, x, y, (int)n, cx, cy, rz,
                     cnt_d);
  int rc = hip_status(hipGetLastError());
  if (rc) return rc;
  std::vector<int32_t> cnt(n_zones);
  if ((rc = hip_status(hipMemcpyAsync(cnt.data(), cnt_d, sizeof(int32_t) * n_zones,
                                      hipMemcpyDeviceToHost, st))))
    return rc;
  if ((rc = hip_status(hipStreamSynchronize(st)))) return rc;
  int64_t total = 0;
  patch_ptr[0] = 0;
  for (int p = 0; p < n_zones; ++p) {
    total += cnt[p];
    if (total > INT32_MAX) return CD_ERR_INVALID_ARG;
    patch_ptr[p + 1] = (int32_t)total;
  }
  if (total > capacity) return CD_ERR_CAPACITY;
  if (total == 0) return CD_OK;
  if ((rc = hip_status(hipMemcpyAsync(ptr_d, patch_ptr, sizeof(int32_t) * (n_zones + 1),
                                      hipMemcpyHostToDevice, st))))
    return rc;
  hipLaunchKernelGGL(k_zone_fill, dim3(n_zones), dim3(kZT), 0, st, x, y, (int)n, cx, cy, rz,
                     ptr_d, active_idx);
  if ((rc = hip_status(hipGetLastError()))) return rc;
  // the host offsets were read by the copy above; keep them valid until it ends
  return hip_status(hipStreamSynchronize(st));
}

int zone_batches(const double* cx, const double* cy, const double* rz, int32_t n_zones,
                 double gap, int32_t cap, int32_t keep_order, int32_t* batch,
                 int32_t* n_batches) {
  if (n_zones < 0 || cap < 1 || !(gap >= 0.0) || !std::isfinite(gap) ||
      (n_zones > 0 && (!cx || !cy || !rz || !batch)))
    return CD_ERR_INVALID_ARG;
  double rmax = 0.0, x0 = 0.0, x1 = 0.0, y0 = 0.0, y1 = 0.0;
  for (int t = 0; t < n_zones; ++t) {
    if (!std::isfinite(cx[t]) || !std::isfinite(cy[t]) || !(rz[t] >= 0.0) ||
        !std::isfinite(rz[t]))
      return CD_ERR_INVALID_ARG;
    rmax = std::max(rmax, rz[t]);
    x0 = t ? std::min(x0, cx[t]) : cx[t];
    x1 = t ? std::max(x1, cx[t]) : cx[t];
    y0 = t ? std::min(y0, cy[t]) : cy[t];
    y1 = t ? std::max(y1, cy[t]) : cy[t];
  }
  // Conflicting centres are closer than 2 rmax + gap: with cells at least
  // that wide only the 3 x 3 neighbourhood of a cell can hold a conflict
  // (1e-6 of slack keeps rounding in the cell index from splitting a
  // conflicting pair two cells apart).
  const double cell = (2.0 * rmax + gap) * (1.0 + 1e-6);
  int gx = 1, gy = 1;
  if (cell > 0.0) {
    gx = (int)std::max(1.0, std::min(1024.0, std::floor((x1 - x0) / cell)));
    gy = (int)std::max(1.0, std::min(1024.0, std::floor((y1 - y0) / cell)));
  }
  const double wx = gx > 1 ? (x1 - x0) / gx : 1.0;
  const double wy = gy > 1 ? (y1 - y0) / gy : 1.0;
  auto cell_of = [&](double v, double lo, double w, int g) {
    if (g == 1) return 0;
    return std::min(g - 1, std::max(0, (int)((v - lo) / w)));
  };
  std::vector<std::vector<int32_t>> grid((size_t)gx * gy);
  std::vector<int32_t> size;
  std::vector<int32_t> mark;  // mark[b] == t + 1: batch b holds a zone in conflict with t
  int32_t nb = 0;
  for (int t = 0; t < n_zones; ++t) {
    const int ix = cell_of(cx[t], x0, wx, gx), iy = cell_of(cy[t], y0, wy, gy);
    int32_t need = 0;
    for (int a = std::max(0, ix - 1); a <= std::min(gx - 1, ix + 1); ++a)
      for (int b = std::max(0, iy - 1); b <= std::min(gy - 1, iy + 1); ++b)
        for (int32_t s : grid[(size_t)a * gy + b])
          if (zones_conflict(cx[s], cy[s], rz[s], cx[t], cy[t], rz[t], gap)) {
            need = std::max(need, batch[s] + 1);
            mark[batch[s]] = t + 1;
          }
    // ordered: after every conflicting earlier zone; first fit: the first
    // batch without a conflicting zone.  Either way a full batch is passed.
    int32_t b = keep_order ? need : 0;
    while (b < (int32_t)size.size() && (size[b] >= cap || (!keep_order && mark[b] == t + 1))) ++b;
    if (b >= (int32_t)size.size()) {
      size.resize(b + 1, 0);
      mark.resize(b + 1, 0);
    }
    ++size[b];
    batch[t] = b;
    nb = std::max(nb, b + 1);
    grid[(size_t)ix * gy + iy].push_back(t);
  }
  if (n_batches) *n_batches = nb;
  return CD_OK;
}

}  // extern "C"
