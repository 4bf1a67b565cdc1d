// Stable least-significant-digit radix sort of (uint32 key, int32 value)
// pairs: 4 passes of 8 bits.  Used to put charges in Morton order during
// staging.  Deterministic: every count is exact and every scatter position is
// a stable rank (items of a tile are ranked in index order), so the output is
// the unique stable order.
#include "common.hpp"

namespace cd {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;

int sort_tiles(int n) { return (n + kSortTile - 1) / kSortTile; }

// Elements of 32-bit scratch the sort needs besides the two key/value pairs.
size_t sort_scratch_elems(int n) { return (size_t)256 * sort_tiles(n) + 256; }

__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint32_t* __restrict__ keys,
                                                            int n, int shift, int ntiles,
                                                            uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int i = base + r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of hist (digit-major, length 256*ntiles), one workgroup.
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t* __restrict__ hist, int len) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int seg = (len + 1023) / 1024;
  const int b = t * seg, e = min(len, b + seg);
  uint32_t s = 0;
  for (int k = b; k < e; ++k) s += hist[k];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive scan
    uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = t > 0 ? part[t - 1] : 0u;
  for (int k = b; k < e; ++k) {
    uint32_t v = hist[k];
    hist[k] = run;
    run += v;
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
  for (int r = 0; r < kSortRounds; ++r) {
    for (int q = 0; q < kSortThreads / 64; ++q) wcnt[q][t] = 0;
    __syncthreads();
    const int i = blockIdx.x * kSortTile + r * kSortThreads + t;
    const bool ok = i < n;
    uint32_t key = ok ? kin[i] : 0u;
    int32_t val = ok ? vin[i] : 0;
    const uint32_t d = (key >> shift) & 255u;
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
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < kSortThreads / 64; ++q) add += wcnt[q][t];
    run[t] += add;
    __syncthreads();
  }
}

// Sorts (ka, va) in place (result ends in ka, va after an even number of
// passes); kb, vb are same-sized scratch; hist has sort_scratch_elems(n).
int sort_pairs(uint32_t* ka, int32_t* va, uint32_t* kb, int32_t* vb, uint32_t* hist, int n,
               hipStream_t st) {
  const int nt = sort_tiles(n);
  uint32_t* kin = ka;
  int32_t* vin = va;
  uint32_t* kout = kb;
  int32_t* vout = vb;
  for (int shift = 0; shift < 32; shift += 8) {
    hipLaunchKernelGGL(k_sort_hist, dim3(nt), dim3(kSortThreads), 0, st, kin, n, shift, nt, hist);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, st, hist, 256 * nt);
    hipLaunchKernelGGL(k_sort_scatter, dim3(nt), dim3(kSortThreads), 0, st, kin, vin, n, shift, nt,
                       hist, kout, vout);
    uint32_t* tk = kin;
    kin = kout;
    kout = tk;
    int32_t* tv = vin;
    vin = vout;
    vout = tv;
  }
  return hip_status(hipGetLastError());
}

}  // namespace cd
