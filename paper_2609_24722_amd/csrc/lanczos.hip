// Lanczos check that a configuration is a strict local minimum on the
// tangent space of the hard wall (Eq. 3): the smallest eigenvalue of the
// tangent-space Hessian must be positive.
//
// Operator.  Charges on the wall whose force points outward (F . r_hat > 0)
// are held: they move only along the circle, and moving along a circle adds
// the curvature term F . r_hat to their tangential second derivative.  With
// P the projection that removes the radial component of held charges (and
// every component of inactive charges), the operator is
//     H_t v = P H P v + w o v,   w_i = F_i . r_hat_i for held i, else 0,
// applied with the FP64 Hessian-vector product of the energy.  Optionally
// the rigid rotation (-y, x) -- an exact zero mode of a full disk -- is
// projected out.
//
// Lanczos with full reorthogonalisation (classical Gram-Schmidt, twice) on
// the device; the tridiagonal eigenproblem is solved by Sturm bisection and
// the Ritz vector by inverse iteration with a shift just below the smallest
// eigenvalue (so the shifted matrix is positive definite and the tridiagonal
// solve needs no pivoting).  The residual ||H_t u - theta u|| of the unit
// Ritz vector is measured with one more operator application.
#include "plan.hpp"

namespace cd {

struct LzDev {
  int n, k;
  const double* x;
  const double* y;
  const int32_t* mask;
  double *fx, *fy;   // forces at the configuration
  double* wgt;       // [n] curvature term of held charges
  int32_t* held;     // [n]
  double* V;         // [k+1][2n]: vector j = (x part [n], y part [n])
  double* w;         // [2n]
  double* h;         // [2n]
  double* q;         // [2n] rotation direction
  double* c1;        // [k+1] dot products
  double* c2;        // [k+1]
  double* nrm;       // [2]
  double* alpha;     // [k]
  double* beta;      // [k]
  double* tri;       // [k + 4]: Ritz coefficients, then theta_min, theta_max, k_eff, resid
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {  // SplitMix64 finaliser
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// held set, curvature weights, rotation vector, random start vector
__global__ void k_lz_setup(LzDev L, uint64_t seed, int deflate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  const bool act = L.mask ? L.mask[i] != 0 : true;
  const double px = L.x[i], py = L.y[i];
  const double r = sqrt(px * px + py * py);
  const double fr = r > 0.0 ? (L.fx[i] * px + L.fy[i] * py) / r : 0.0;
  const bool hd = act && r >= 1.0 - 1e-14 && fr > 0.0;
  L.held[i] = hd;
  L.wgt[i] = hd ? fr : 0.0;
  double vx = act ? (double)(mix64(seed ^ (2ull * i)) >> 11) * 0x1.0p-52 - 1.0 : 0.0;
  double vy = act ? (double)(mix64(seed ^ (2ull * i + 1)) >> 11) * 0x1.0p-52 - 1.0 : 0.0;
  if (hd) {
    const double ux = px / r, uy = py / r, vr = vx * ux + vy * uy;
    vx -= vr * ux;
    vy -= vr * uy;
  }
  L.V[i] = vx;
  L.V[L.n + i] = vy;
  if (deflate) {
    L.q[i] = act ? -py : 0.0;
    L.q[L.n + i] = act ? px : 0.0;
  }
}

// out = P h + w o v
__global__ void k_lz_post(LzDev L, const double* __restrict__ v, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  const bool act = L.mask ? L.mask[i] != 0 : true;
  double hx = L.h[i], hy = L.h[L.n + i];
  if (!act) {
    hx = 0.0;
    hy = 0.0;
  } else if (L.held[i]) {
    const double px = L.x[i], py = L.y[i], r = sqrt(px * px + py * py);
    const double ux = px / r, uy = py / r, hr = hx * ux + hy * uy;
    hx = hx - hr * ux + L.wgt[i] * v[i];
    hy = hy - hr * uy + L.wgt[i] * v[L.n + i];
  }
  out[i] = hx;
  out[L.n + i] = hy;
}

// out[j] = A_j . b for j < m (A_j = A + j*len); one workgroup per j, fixed order
__global__ __launch_bounds__(256) void k_lz_dots(const double* __restrict__ A, int m, size_t len,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ out) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  if (j >= m) return;
  const double* a = A + (size_t)j * len;
  double s = 0.0;
  for (size_t e = threadIdx.x; e < len; e += blockDim.x) s += a[e] * b[e];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[j] = (red[0] + red[1]) + (red[2] + red[3]);
}

// w -= sum_j c_j A_j   (scale: c_j multiplied by 1/nrm when nrm != null, for a
// normalised direction given unnormalised)
__global__ void k_lz_axpys(double* __restrict__ w, const double* __restrict__ A, int m,
                           size_t len, const double* __restrict__ c,
                           const double* __restrict__ nrm) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const double sc = nrm ? 1.0 / nrm[0] : 1.0;
  double v = w[e];
  for (int j = 0; j < m; ++j) v -= (c[j] * sc) * A[(size_t)j * len + e];
  w[e] = v;
}

// after the two Gram-Schmidt passes: alpha_j, beta_j = ||w||, V_{j+1} = w / beta_j
__global__ void k_lz_next(LzDev L, int j) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t len = 2 * (size_t)L.n;
  const double b = sqrt(L.nrm[0]);
  if (e == 0) {
    L.alpha[j] = L.c1[j] + L.c2[j];
    L.beta[j] = b;
  }
  if (e < len) L.V[(size_t)(j + 1) * len + e] = b > 0.0 ? L.w[e] / b : 0.0;
}

__device__ int sturm_below(const double* a, const double* b, int k, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < k; ++i) {
    const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    d = a[i] - x - (i > 0 ? bb / d : 0.0);
    if (d == 0.0) d = -1e-300;
    cnt += d < 0.0;
  }
  return cnt;
}

// One thread: effective size, extreme eigenvalues by bisection, Ritz
// coefficients of the smallest by shifted inverse iteration.
__global__ void k_lz_tridiag(LzDev L) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int k = L.k;
  double amax = 0.0;
  for (int i = 0; i < k; ++i) amax = fmax(amax, fabs(L.alpha[i]) + fabs(L.beta[i]));
  int kk = k;
  for (int i = 0; i < k - 1; ++i)
    if (!(L.beta[i] > 1e-13 * amax)) {
      kk = i + 1;
      break;
    }
  const double* a = L.alpha;
  const double* b = L.beta;
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < kk; ++i) {
    const double rad = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i < kk - 1 ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - rad);
    hi = fmax(hi, a[i] + rad);
  }
  double l0 = lo, h0 = hi, l1 = lo, h1 = hi;
  for (int it = 0; it < 200; ++it) {
    const double m0 = 0.5 * (l0 + h0);
    if (sturm_below(a, b, kk, m0) >= 1) h0 = m0;
    else l0 = m0;
    const double m1 = 0.5 * (l1 + h1);
    if (sturm_below(a, b, kk, m1) >= kk) h1 = m1;
    else l1 = m1;
  }
  const double tmin = 0.5 * (l0 + h0), tmax = 0.5 * (l1 + h1);
  const double sig = tmin - 1e-10 * (fabs(tmin) + fabs(tmax));
  double* yv = L.tri;
  for (int i = 0; i < kk; ++i) yv[i] = 1.0;
  for (int pass = 0; pass < 4; ++pass) {
    // solve (T - sig I) z = y by the LDL^T recurrence (positive definite)
    double dprev = 0.0;
    for (int i = 0; i < kk; ++i) {  // forward: store multipliers in place of nothing
      const double di = a[i] - sig - (i > 0 ? b[i - 1] * b[i - 1] / dprev : 0.0);
      if (i > 0) yv[i] -= (b[i - 1] / dprev) * yv[i - 1];
      L.c1[i] = di;  // pivots
      dprev = di;
    }
    yv[kk - 1] /= L.c1[kk - 1];
    for (int i = kk - 2; i >= 0; --i) yv[i] = (yv[i] - b[i] * yv[i + 1]) / L.c1[i];
    double s = 0.0;
    for (int i = 0; i < kk; ++i) s += yv[i] * yv[i];
    s = 1.0 / sqrt(s);
    for (int i = 0; i < kk; ++i) yv[i] *= s;
  }
  L.tri[k] = tmin;
  L.tri[k + 1] = tmax;
  L.tri[k + 2] = (double)kk;
}

// u = sum_{j < kk} y_j V_j  (written to w)
__global__ void k_lz_ritz(LzDev L) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t len = 2 * (size_t)L.n;
  if (e >= len) return;
  const int kk = (int)L.tri[L.k + 2];
  double u = 0.0;
  for (int j = 0; j < kk; ++j) u += L.tri[j] * L.V[(size_t)j * len + e];
  L.w[e] = u;
}

// h = H_t u - theta u (its squared norm is taken by k_lz_dots)
__global__ void k_lz_resid(LzDev L) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * (size_t)L.n) return;
  L.h[e] = L.h[e] - L.tri[L.k] * L.w[e];
}

// v <- v / sqrt(*nrm)
__global__ void k_lz_scale(double* __restrict__ v, size_t len, const double* __restrict__ nrm) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) v[e] /= sqrt(nrm[0]);
}

struct LzPlan {
  Plan hv;
  size_t hv_bytes = 0, f_bytes = 0, total = 0;
  char* hvb = nullptr;  // workspace of the staged HVP
  char* fws = nullptr;  // workspace of the force call
  LzDev D;
};

static bool lz_plan(int64_t n, int k, char* base, LzPlan& P) {
  if (n < 2 || n > (1 << 26) || k < 2 || k > 4096) return false;
  P.hv_bytes = hvp64_bytes(n);
  P.f_bytes = coulomb_workspace_bytes(CD_OP_FORCES, n, 0, 0, CD_FP64);
  if (!P.hv_bytes || !P.f_bytes) return false;
  Carve cv;
  cv.base = base;
  P.hvb = cv.take<char>(P.hv_bytes);
  P.fws = cv.take<char>(P.f_bytes);
  const size_t len = 2 * (size_t)n;
  LzDev& D = P.D;
  D.n = (int)n;
  D.k = k;
  D.fx = cv.take<double>(n);
  D.fy = cv.take<double>(n);
  D.wgt = cv.take<double>(n);
  D.held = cv.take<int32_t>(n);
  D.V = cv.take<double>(len * (k + 1));
  D.w = cv.take<double>(len);
  D.h = cv.take<double>(len);
  D.q = cv.take<double>(len);
  D.c1 = cv.take<double>(k + 1);
  D.c2 = cv.take<double>(k + 1);
  D.nrm = cv.take<double>(2);
  D.alpha = cv.take<double>(k);
  D.beta = cv.take<double>(k);
  D.tri = cv.take<double>(k + 4);
  P.total = cv.off + 512;
  return true;
}

size_t lanczos_workspace_bytes(int64_t n, int k) {
  LzPlan P;
  return lz_plan(n, k, nullptr, P) ? P.total : 0;
}

}  // namespace cd

using namespace cd;

extern "C" int tangent_lanczos(const double* x, const double* y, int64_t n, const int32_t* mask,
                               int32_t k, int32_t deflate_rotation, uint64_t seed,
                               double* out_host, void* ws, size_t ws_bytes, void* stream) {
  if (!x || !y || !out_host) return CD_ERR_INVALID_ARG;
  LzPlan P;
  if (!lz_plan(n, k, nullptr, P)) return CD_ERR_INVALID_ARG;
  if (!ws) return CD_ERR_WORKSPACE;
  if (ws_bytes < P.total) return CD_ERR_WORKSPACE;
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  lz_plan(n, k, base, P);
  hipStream_t st = (hipStream_t)stream;
  LzDev& D = P.D;
  D.x = x;
  D.y = y;
  D.mask = mask;
  int rc = coulomb_forces(x, y, n, CD_FP64, D.fx, D.fy, nullptr, P.fws, P.f_bytes, stream);
  if (rc) return rc;
  if ((rc = hvp64_stage(P.hv, P.hvb, n, x, y, st))) return rc;
  const size_t len = 2 * (size_t)n;
  const dim3 gn((unsigned)((n + 255) / 256)), g2((unsigned)((len + 255) / 256)), b256(256);
  hipLaunchKernelGGL(k_lz_setup, gn, b256, 0, st, D, seed, deflate_rotation);
  auto deflate = [&](double* v) {
    if (!deflate_rotation) return;
    hipLaunchKernelGGL(k_lz_dots, dim3(1), b256, 0, st, D.q, 1, len, D.q, D.nrm + 1);
    hipLaunchKernelGGL(k_lz_dots, dim3(1), b256, 0, st, D.q, 1, len, v, D.c2 + D.k);
    hipLaunchKernelGGL(k_lz_axpys, g2, b256, 0, st, v, D.q, 1, len, D.c2 + D.k, D.nrm + 1);
  };
  // normalise the start vector
  deflate(D.V);
  hipLaunchKernelGGL(k_lz_dots, dim3(1), b256, 0, st, D.V, 1, len, D.V, D.nrm);
  hipLaunchKernelGGL(k_lz_scale, g2, b256, 0, st, D.V, len, D.nrm);
  auto apply = [&](const double* v, double* out) {
    int r = hvp64_apply(P.hv, v, v + n, D.h, D.h + n, st);
    hipLaunchKernelGGL(k_lz_post, gn, b256, 0, st, D, v, out);
    return r;
  };
  for (int j = 0; j < k; ++j) {
    double* vj = D.V + (size_t)j * len;
    if ((rc = apply(vj, D.w))) return rc;
    deflate(D.w);
    hipLaunchKernelGGL(k_lz_dots, dim3(j + 1), b256, 0, st, D.V, j + 1, len, D.w, D.c1);
    hipLaunchKernelGGL(k_lz_axpys, g2, b256, 0, st, D.w, D.V, j + 1, len, D.c1, nullptr);
    hipLaunchKernelGGL(k_lz_dots, dim3(j + 1), b256, 0, st, D.V, j + 1, len, D.w, D.c2);
    hipLaunchKernelGGL(k_lz_axpys, g2, b256, 0, st, D.w, D.V, j + 1, len, D.c2, nullptr);
    deflate(D.w);
    hipLaunchKernelGGL(k_lz_dots, dim3(1), b256, 0, st, D.w, 1, len, D.w, D.nrm);
    hipLaunchKernelGGL(k_lz_next, g2, b256, 0, st, D, j);
  }
  hipLaunchKernelGGL(k_lz_tridiag, dim3(1), dim3(64), 0, st, D);
  hipLaunchKernelGGL(k_lz_ritz, g2, b256, 0, st, D);
  if ((rc = apply(D.w, D.h))) return rc;
  hipLaunchKernelGGL(k_lz_resid, g2, b256, 0, st, D);
  hipLaunchKernelGGL(k_lz_dots, dim3(1), b256, 0, st, D.h, 1, len, D.h, D.tri + k + 3);
  double host[4];
  if ((rc = hip_status(hipMemcpyAsync(host, D.tri + k, 4 * sizeof(double), hipMemcpyDeviceToHost,
                                      st))))
    return rc;
  if ((rc = hip_status(hipStreamSynchronize(st)))) return rc;
  out_host[0] = host[0];
  out_host[1] = sqrt(host[3]);
  out_host[2] = host[1];
  out_host[3] = host[2];
  return CD_OK;
}
