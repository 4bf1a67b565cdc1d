// Morton order of the charges: 24-bit Morton keys (12 bits per axis over
// [-1, 1]^2) and a stable least-significant-digit radix sort of
// (key, index) pairs, 3 passes of 8 bits.  Deterministic: every count is
// exact and every scatter position is a stable rank (the items of a tile are
// ranked in index order), so the permutation is the unique stable order.
//
// Per pass: per-tile digit counts (the first pass also computes the keys),
// one exclusive scan of the digit-major count table, and a stable scatter.
#include "common.hpp"

namespace cd {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;
constexpr int kScanThreads = 1024;

int sort_tiles(int n) { return (n + kSortTile - 1) / kSortTile; }

// Elements of 32-bit scratch the sort needs besides the key/value buffers.
size_t sort_scratch_elems(int n) { return (size_t)256 * sort_tiles(n) + 256; }

__device__ __forceinline__ uint32_t spread12(uint32_t v) {
  v &= 0xfffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__device__ __forceinline__ uint32_t morton_key(double x, double y) {
  double fx = (x + 1.0) * 2048.0, fy = (y + 1.0) * 2048.0;
  if (!(fx >= 0.0)) fx = 0.0;  // also maps NaN to 0
  if (!(fx <= 4095.0)) fx = 4095.0;
  if (!(fy >= 0.0)) fy = 0.0;
  if (!(fy <= 4095.0)) fy = 4095.0;
  return spread12((uint32_t)fx) | (spread12((uint32_t)fy) << 1);
}

// Digit counts of one tile.  MORTON: the keys are computed from (x, y) and
// written with the identity values first.
template <bool MORTON>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const double* __restrict__ x,
                                                            const double* __restrict__ y,
                                                            uint32_t* __restrict__ keys,
                                                            int32_t* __restrict__ vals, int n,
                                                            int shift, int ntiles,
                                                            uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortTile;
  uint32_t d[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int i = base + r * kSortThreads + threadIdx.x;
    uint32_t k = 0;
    if (i < n) {
      if (MORTON) {
        k = morton_key(x[i], y[i]);
        keys[i] = k;
        vals[i] = i;
      } else {
        k = keys[i];
      }
    }
    d[r] = i < n ? (k >> shift) & 255u : 256u;
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r)
    if (d[r] < 256u) atomicAdd(&cnt[d[r]], 1u);
  __syncthreads();
  hist[threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Inclusive scan of one value per thread over the workgroup (fixed order).
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  uint32_t before = 0;
  for (int q = 0; q < w; ++q) before += wsum[q];
  total = 0;
  for (int q = 0; q < kScanThreads / 64; ++q) total += wsum[q];
  __syncthreads();
  return v + before;
}

// Exclusive scan of hist (digit-major, length len, a multiple of 4), one
// workgroup, in chunks of 4 * kScanThreads with a running carry.
__global__ __launch_bounds__(kScanThreads) void k_sort_scan(uint32_t* __restrict__ hist,
                                                            int len) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  uint32_t carry = 0;
  for (int c0 = 0; c0 < len; c0 += 4 * kScanThreads) {
    const int i = c0 + 4 * threadIdx.x;
    uint4 q = make_uint4(0, 0, 0, 0);
    if (i < len) q = *reinterpret_cast<const uint4*>(hist + i);
    const uint32_t s = q.x + q.y + q.z + q.w;
    uint32_t total;
    const uint32_t incl = block_scan(s, wsum, total);
    uint32_t e = carry + incl - s;
    if (i < len) {
      uint4 o;
      o.x = e;
      e += q.x;
      o.y = e;
      e += q.y;
      o.z = e;
      e += q.z;
      o.w = e;
      *reinterpret_cast<uint4*>(hist + i) = o;
    }
    carry += total;
  }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin, int n, int shift,
    int ntiles, const uint32_t* __restrict__ hist, uint32_t* __restrict__ kout,
    int32_t* __restrict__ vout) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kSortThreads / 64][256];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  base[t] = hist[t * ntiles + blockIdx.x];
  run[t] = 0;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  // the whole tile is read up front, so the rounds below wait on no memory
  uint32_t key[kSortRounds];
  int32_t val[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int i = blockIdx.x * kSortTile + r * kSortThreads + t;
    key[r] = i < n ? kin[i] : 0u;
    val[r] = i < n ? vin[i] : 0;
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    for (int q = 0; q < kSortThreads / 64; ++q) wcnt[q][t] = 0;
    __syncthreads();
    const int i = blockIdx.x * kSortTile + r * kSortThreads + t;
    const bool ok = i < n;
    const uint32_t d = (key[r] >> shift) & 255u;
    uint64_t m = __ballot(ok);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t bb = __ballot((d >> bit) & 1u);
      m &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    const uint32_t lower = __popcll(m & lt);
    if (ok && lower == 0) wcnt[w][d] = __popcll(m);
    __syncthreads();
    if (ok) {
      uint32_t off = run[d] + lower;
      for (int q = 0; q < w; ++q) off += wcnt[q][d];
      const uint32_t pos = base[d] + off;
      kout[pos] = key[r];
      vout[pos] = val[r];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < kSortThreads / 64; ++q) add += wcnt[q][t];
    run[t] += add;
  }
}

// Stable Morton order of (x, y): perm[s] = index of the s-th charge.  ka, kb
// and va are scratch of n elements, hist has sort_scratch_elems(n); perm
// (n elements) also serves as scratch in the first two passes.
int morton_order(const double* x, const double* y, int n, uint32_t* ka, uint32_t* kb,
                 int32_t* va, uint32_t* hist, int32_t* perm, hipStream_t st) {
  const int nt = sort_tiles(n);
  // passes: (ka, va) -> (kb, perm) -> (ka, va) -> (kb, perm)
  uint32_t* kin[3] = {ka, kb, ka};
  int32_t* vin[3] = {va, perm, va};
  uint32_t* kout[3] = {kb, ka, kb};
  int32_t* vout[3] = {perm, va, perm};
  for (int p = 0; p < 3; ++p) {
    if (p == 0)
      hipLaunchKernelGGL(k_sort_hist<true>, dim3(nt), dim3(kSortThreads), 0, st, x, y, ka, va, n,
                         0, nt, hist);
    else
      hipLaunchKernelGGL(k_sort_hist<false>, dim3(nt), dim3(kSortThreads), 0, st, nullptr,
                         nullptr, kin[p], nullptr, n, 8 * p, nt, hist);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(kScanThreads), 0, st, hist, 256 * nt);
    hipLaunchKernelGGL(k_sort_scatter, dim3(nt), dim3(kSortThreads), 0, st, kin[p], vin[p], n,
                       8 * p, nt, hist, kout[p], vout[p]);
  }
  return hip_status(hipGetLastError());
}

}  // namespace cd
