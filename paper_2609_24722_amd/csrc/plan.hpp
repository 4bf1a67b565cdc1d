// Internal plan of the all-pairs passes (workspace layout and launch shape),
// shared by the pair entry points and the Lanczos check.
#pragma once

#include "common.hpp"

namespace cd {

struct Plan {
  int n = 0, npad = 0, nb = 0;
  int W = 0, L = 0, C = 0, G = 0, S = 0;  // symmetric pass
  int splits = 0, jb = 0;                 // one-sided pass
  int nred = 0;                           // reduction workgroups
  // workspace pieces
  uint32_t *keys = nullptr, *keys2 = nullptr, *hist = nullptr;
  int32_t *perm = nullptr, *perm2 = nullptr;
  double *xs = nullptr, *ys = nullptr, *vxs = nullptr, *vys = nullptr;
  double* cen = nullptr;
  float* box = nullptr;
  double *q0 = nullptr, *q1 = nullptr, *q2 = nullptr;  // i partials / one-sided partials
  double *j0 = nullptr, *j1 = nullptr;                 // j partials
  double* eblk = nullptr;
  size_t total = 0;
};


bool make_plan(int op, int64_t n64, int precision, char* base, Plan& P);
int stage(const Plan& P, const double* x, const double* y, const double* vx, const double* vy,
          hipStream_t st);

// FP64 Hessian-vector products on positions staged once
size_t hvp64_bytes(int64_t n);
int hvp64_stage(Plan& P, char* base, int64_t n, const double* x, const double* y, hipStream_t st);
int hvp64_apply(const Plan& P, const double* vx, const double* vy, double* hx, double* hy,
                hipStream_t st);

}  // namespace cd
