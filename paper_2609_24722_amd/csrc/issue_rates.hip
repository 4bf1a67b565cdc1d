// Vector-instruction issue rates of the GPU, one instruction class at a time.
//
// A stand-alone program (not part of the library): each kernel runs 2^20
// threads, every lane advancing 16 independent chains of one instruction, so
// that no dependency stalls the issue, and the rate is the lane operations
// per second over five timed launches after the clocks have ramped up.  The
// pair kernels' instruction counts divided by these rates give their issue
// bounds.  The last class interleaves twelve FP32 FMAs with one v_rsq_f32 per
// chain step and counts all thirteen instructions: it shows whether the
// transcendental costs issue time of its own next to the other instructions.
//
// Usage: issue_rates  (prints one line per class).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kChains = 16;
constexpr int kThreads = 256;

enum Op {
  kMulF32, kFmaF32, kAddF32, kSubDppF32, kMovDpp, kRsqF32,
  kFmaF64, kMulF64, kAddF64, kRsqF64, kFmaRsqF32
};

__device__ __forceinline__ float ror1(float v) {  // row rotate by one lane
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x121, 0xf, 0xf, true));
}

template <int OP, class T>
__global__ __launch_bounds__(kThreads) void k_chain(T* out, int iters, T a, T b) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  // a per-lane operand, so the DPP move folds into the subtraction (a DPP
  // instruction takes its second operand from a vector register)
  const T bv = b + (T)(threadIdx.x & 1) * (T)1e-9;
  T x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (T)1 + (T)(g & 7) * (T)0.001 + (T)c * (T)0.01;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (OP == kMulF32 || OP == kMulF64) x[c] = x[c] * a;
      else if constexpr (OP == kFmaF32) x[c] = __builtin_fmaf(x[c], a, b);
      else if constexpr (OP == kFmaF64) x[c] = __builtin_fma(x[c], a, b);
      else if constexpr (OP == kAddF32 || OP == kAddF64) x[c] = x[c] + b;
      else if constexpr (OP == kSubDppF32) x[c] = ror1(x[c]) - bv;
      else if constexpr (OP == kMovDpp) x[c] = ror1(x[c]);
      else if constexpr (OP == kRsqF32) x[c] = __builtin_amdgcn_rsqf(x[c]);
      else if constexpr (OP == kRsqF64) x[c] = __builtin_amdgcn_rsq(x[c]);
      else {
        T y = x[c];
#pragma unroll
        for (int q = 0; q < 12; ++q) y = __builtin_fmaf(y, a, b);
        x[c] = __builtin_amdgcn_rsqf(y);
      }
    }
  }
  T s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[g] = s;  // the grid covers the buffer exactly
}

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    std::fprintf(stderr, "issue_rates: %s: %s\n", what, hipGetErrorString(e));
    std::exit(1);
  }
}

constexpr int kN = 1 << 20;  // threads per launch
constexpr int kIters = 8192;

// Lane operations per second of one class (instructions per chain step
// times chain steps); prints the line when name is given.
template <int OP, class T>
double rate(const char* name, T* out, int per_step) {
  const int iters = kIters / per_step;
  const dim3 grid(kN / kThreads), block(kThreads);
  hipEvent_t e0, e1;
  check(hipEventCreate(&e0), "event");
  check(hipEventCreate(&e1), "event");
  for (int w = 0; w < 3; ++w)
    hipLaunchKernelGGL((k_chain<OP, T>), grid, block, 0, 0, out, iters, (T)0.99999, (T)1e-7);
  check(hipGetLastError(), "launch");
  const int reps = 5;
  check(hipEventRecord(e0, 0), "record");
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL((k_chain<OP, T>), grid, block, 0, 0, out, iters, (T)0.99999, (T)1e-7);
  check(hipEventRecord(e1, 0), "record");
  check(hipEventSynchronize(e1), "synchronize");
  float ms = 0.f;
  check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
  check(hipEventDestroy(e0), "event");
  check(hipEventDestroy(e1), "event");
  const double ops = (double)kN * iters * kChains * per_step * reps;
  const double r = ops / (ms * 1e-3);
  if (name) {
    std::printf("%-34s %8.3f ms/launch  %.3e lane-ops/s\n", name, ms / reps, r);
    std::fflush(stdout);
  }
  return r;
}

}  // namespace

int main() {
  float* o32 = nullptr;
  double* o64 = nullptr;
  check(hipMalloc(&o32, kN * sizeof(float)), "hipMalloc");
  check(hipMalloc(&o64, kN * sizeof(double)), "hipMalloc");
  // about a second of FP32 work first: the clocks ramp up under load
  for (int w = 0; w < 40; ++w) rate<kMulF32, float>(nullptr, o32, 1);
  rate<kMulF32, float>("v_mul_f32", o32, 1);
  rate<kFmaF32, float>("v_fma_f32", o32, 1);
  rate<kAddF32, float>("v_add_f32", o32, 1);
  rate<kSubDppF32, float>("v_sub_f32 with a DPP source", o32, 1);
  rate<kMovDpp, float>("v_mov_b32_dpp", o32, 1);
  rate<kRsqF32, float>("v_rsq_f32", o32, 1);
  rate<kFmaRsqF32, float>("12 v_fma_f32 + 1 v_rsq_f32 (all 13)", o32, 13);
  rate<kFmaF64, double>("v_fma_f64", o64, 1);
  rate<kMulF64, double>("v_mul_f64", o64, 1);
  rate<kAddF64, double>("v_add_f64", o64, 1);
  rate<kRsqF64, double>("v_rsq_f64", o64, 1);
  check(hipDeviceSynchronize(), "synchronize");
  check(hipFree(o32), "hipFree");
  check(hipFree(o64), "hipFree");
  return 0;
}
