// Internal plan of the all-pairs passes (workspace layout and launch shape),
// shared by the pair entry points and the Lanczos check.
#pragma once

#include "common.hpp"

namespace cd {

// Symmetric pass launch shape (compile-time settings): blocks of 64 charges
// per super-block (the i charges of one lane), waves per workgroup, offsets
// per chunk, and the waves per SIMD the register budget is held to.  The j
// window needs (kSymWaves + kSymChunk - 1) x kSymBlocks x 1 KiB of LDS.
#ifndef CD_SYM_BLOCKS
#define CD_SYM_BLOCKS 2
#endif
#ifndef CD_SYM_WAVES
#define CD_SYM_WAVES 8
#endif
#ifndef CD_SYM_CHUNK
#define CD_SYM_CHUNK 8
#endif
#ifndef CD_SYM_WPS
#define CD_SYM_WPS 8
#endif
constexpr int kSymBlocks = CD_SYM_BLOCKS;
constexpr int kSymWaves = CD_SYM_WAVES;
constexpr int kSymChunk = CD_SYM_CHUNK;
constexpr int kSymWavesPerSimd = CD_SYM_WPS;
static_assert(kSymBlocks >= 1 && kSymBlocks <= 4, "symmetric pass: 1..4 blocks per lane");
static_assert(kSymWaves >= 1 && kSymWaves <= 16 && kSymChunk >= 1, "symmetric pass shape");
static_assert((kSymWaves + kSymChunk - 1) * kSymBlocks * 1024 <= 65536,
              "j window exceeds 64 KiB");
// Partial sums of one batch of chunks: at most this many bytes (but at least
// one chunk), and at most kSymBatchMax chunks.
constexpr size_t kSymBatchBytes = size_t(512) << 20;
constexpr int kSymBatchMax = 1024;

struct Plan {
  int n = 0, npad = 0, nb = 0;
  int ns = 0;                              // super-blocks (symmetric pass)
  int shape = 0;                           // symmetric pass launch shape (index)
  int W = 0, L = 0, C = 0, G = 0, S = 0;  // symmetric pass
  int Cb = 0, mj = 0;                     // chunks per batch, j slots per chunk
  size_t chunk_bytes = 0;                 // partial sums of one chunk (symmetric pass)
  int splits = 0, jb = 0;                 // one-sided pass
  int nred = 0;                           // reduction workgroups
  // workspace pieces
  uint32_t *keys = nullptr, *keys2 = nullptr, *hist = nullptr;
  int32_t *perm = nullptr, *perm2 = nullptr;
  double *xs = nullptr, *ys = nullptr, *vxs = nullptr, *vys = nullptr;
  float* box = nullptr;
  double *q0 = nullptr, *q1 = nullptr, *q2 = nullptr;  // i partials / one-sided partials
  double *j0 = nullptr, *j1 = nullptr;                 // j partials
  double *dp0 = nullptr, *dp1 = nullptr;               // super-diagonal sums
  double* ep = nullptr;                                // per-workgroup energy partials
  double* eb = nullptr;                                // per-batch energy partials
  double* eblk = nullptr;
  size_t total = 0;
};


// shape: index into the symmetric pass's list of launch shapes (out of
// range: the default); the entry points pass the one coulomb_autotune chose.
// max_cb > 0 caps the chunks per batch of the symmetric pass (smaller
// scratch, more batches).
bool make_plan(int op, int64_t n64, int precision, char* base, Plan& P, int shape = -1,
               int max_cb = 0);

// Forces and energy (coulomb_forces) with the scratch carved from a fixed
// region [base, base + cap) (base 256-byte aligned): the symmetric pass's
// chunks are batched so that their partial sums fit.  Returns
// CD_ERR_CAPACITY, before anything is enqueued, when not even one chunk per
// batch fits.
int forces_fixed(const double* x, const double* y, int64_t n, int precision, double* fx,
                 double* fy, double* e_total, char* base, size_t cap, hipStream_t st);
// The same plan test alone (host only): CD_OK if the call fits in cap bytes.
int forces_fixed_fits(int64_t n, int precision, size_t cap);
int stage(const Plan& P, const double* x, const double* y, const double* vx, const double* vy,
          hipStream_t st);

// FP64 Hessian-vector products on positions staged once
size_t hvp64_bytes(int64_t n);
int hvp64_stage(Plan& P, char* base, int64_t n, const double* x, const double* y, hipStream_t st);
int hvp64_apply(const Plan& P, const double* vx, const double* vy, double* hx, double* hy,
                hipStream_t st);

}  // namespace cd
