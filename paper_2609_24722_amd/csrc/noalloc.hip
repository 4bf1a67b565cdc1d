// Allocation-free variant of coulomb_forces: the scratch lives in a
// file-scope device array of fixed size instead of a caller workspace, so a
// caller that cannot allocate (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc) only passes inputs and outputs.
//
// Each device that runs the library holds its own copy of `scratch` (64 MiB)
// until the process ends.  Host code never uses the array's name as an
// address: the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept in g_ptr.  Every
// call on a device shares that device's array, so calls that overlap on one
// device (two streams, two threads, two graph replays in flight) race.
// The forces path needs nothing cleared between calls: every partial sum it
// reads is written by the same call first.
#include <mutex>

#include "plan.hpp"

namespace cd {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_mu;
static char* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once).
static int scratch_ptr(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CD_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CD_ERR_HIP;
    g_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_ptr[dev];
  return CD_OK;
}

}  // namespace cd

extern "C" int coulomb_forces_noalloc(const double* x, const double* y, int64_t n,
                                      int precision, double* fx, double* fy, double* e_total,
                                      void* stream) {
  if (!x || !y || !fx || !fy) return CD_ERR_INVALID_ARG;
  // sizes first, on the host: too large an n is refused before anything is
  // enqueued or the scratch is looked up
  int rc = cd::forces_fixed_fits(n, precision, cd::kScratchBytes);
  if (rc == CD_ERR_CAPACITY) return CD_ERR_SCRATCH;
  if (rc) return rc;
  char* base = nullptr;
  if ((rc = cd::scratch_ptr(&base))) return rc;
  return cd::forces_fixed(x, y, n, precision, fx, fy, e_total, base, cd::kScratchBytes,
                          (hipStream_t)stream);
}
