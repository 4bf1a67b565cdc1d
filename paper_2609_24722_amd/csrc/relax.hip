// Subdomain relaxation (paper Sec. II.C step 4 and Sec. II.E): patch
// construction, the frozen-exterior field, a batched L-BFGS that relaxes many
// subdomains at once, exact FP64 energy changes, and the greedy commit of
// relaxed candidates.
//
// Objective of patch p with active set A and frozen set F (Eqs. 6-7 read as
// E_sub = sum_{i in A} e_i, e_i = 1/2 sum_{j in A} 1/r_ij + sum_{j in F} 1/r_ij):
// its gradient with respect to an active charge is the full Coulomb gradient
// from every other charge, frozen ones at their snapshot positions.
//
// Two ways to relax a batch:
//  * CD_FP64 ("plain"): every evaluation is exact -- for each active charge
//    the sum over all N charges, O(n_act N) per gradient as in Sec. II.E.
//  * CD_MIXED: the exterior is split into a halo (frozen charges within
//    halo_width of the patch, kept as explicit pairs) and the far exterior,
//    whose field at each active charge is summed exactly in FP64 (gradient
//    and Hessian) at an expansion point and used as a second-order Taylor
//    model around it.  The model (near pairs explicit, far field quadratic)
//    is minimised first with FP32 pairs, expanded at the start positions;
//    then in rounds: re-expand the far field exactly at the current
//    positions -- at the expansion point the model gradient IS the exact
//    gradient, which is tested against the tolerance -- and minimise the
//    FP64-pair model again, keeping the L-BFGS history.  Each round costs one
//    O(n_act N) FP64 pass; the iterations in between cost O(n_act (n_act +
//    n_halo)).  The endpoint is a minimiser of the exact E_sub either way.
//
// The optimiser (both paths) is L-BFGS over free charges' (x, y) and wall-held
// charges' polar angle (the paper's boundary parameterisation, Eq. 10, applied
// to the charges the hard wall of Eq. 3 actually holds), with backtracking on
// an Armijo test.  All patches advance in lock step: each round is one
// evaluation kernel over every running patch plus one update kernel with a
// workgroup per patch.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace cd {

size_t relax_workspace_bytes(int op, int64_t n, int32_t n_patches, int64_t total_active,
                             int precision);

constexpr int kMaxMem = 16;  // largest L-BFGS memory; the workspace is sized for it
// plain path: the exact evaluations take the Hessian blocks every kBlockEvery-th
// iteration, and at every one once the reduced gradient is within kBlockNear
// times the Newton switch
constexpr int kBlockEvery = 4;
constexpr double kBlockNear = 2.0;

// ------------------------------------------------------ patch construction --
__device__ __forceinline__ double dist2_rn(double ax, double ay, double bx, double by) {
  const double dx = ax - bx, dy = ay - by;
  return __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
}

// One workgroup per patch: the size-th smallest squared distance (as the bit
// pattern of a non-negative double, which orders like the value) is found by
// an exact 8-pass radix select; the patch is then every charge below that
// key plus, among charges equal to it, the lowest indices -- listed in
// increasing index order.
__global__ __launch_bounds__(1024) void k_patch_select(const double* __restrict__ x,
                                                       const double* __restrict__ y, int n,
                                                       const int32_t* __restrict__ centres,
                                                       const int32_t* __restrict__ ptr,
                                                       int32_t* __restrict__ out,
                                                       int32_t* __restrict__ err) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix, s_mask;
  __shared__ uint32_t s_need;
  __shared__ uint32_t lt_cnt[1024], eq_cnt[1024];
  const int p = blockIdx.x, t = threadIdx.x;
  const int size = ptr[p + 1] - ptr[p];
  const int ctr = centres[p];
  if (ctr < 0 || ctr >= n) {  // invalid centre: report, write nothing
    if (t == 0) atomicOr(err, 1);
    return;
  }
  const double cx = x[ctr], cy = y[ctr];
  if (t == 0) {
    s_prefix = 0;
    s_mask = 0;
    s_need = (uint32_t)size;
  }
  __syncthreads();
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    if (t < 256) hist[t] = 0;
    __syncthreads();
    const uint64_t pre = s_prefix, msk = s_mask;
    for (int j = t; j < n; j += blockDim.x) {
      const uint64_t key = __double_as_longlong(dist2_rn(x[j], y[j], cx, cy));
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
  const uint32_t need_eq = s_need;  // how many charges at exactly T belong to the patch
  const int chunk = (n + blockDim.x - 1) / blockDim.x;
  const int j0 = min(n, t * chunk), j1 = min(n, j0 + chunk);
  uint32_t lt = 0, eq = 0;
  for (int j = j0; j < j1; ++j) {
    const uint64_t key = __double_as_longlong(dist2_rn(x[j], y[j], cx, cy));
    lt += key < T;
    eq += key == T;
  }
  lt_cnt[t] = lt;
  eq_cnt[t] = eq;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const uint32_t a = t >= off ? lt_cnt[t - off] : 0u, b = t >= off ? eq_cnt[t - off] : 0u;
    __syncthreads();
    lt_cnt[t] += a;
    eq_cnt[t] += b;
    __syncthreads();
  }
  uint32_t lt_before = lt_cnt[t] - lt, eq_before = eq_cnt[t] - eq;
  int32_t* dst = out + ptr[p];
  for (int j = j0; j < j1; ++j) {
    const uint64_t key = __double_as_longlong(dist2_rn(x[j], y[j], cx, cy));
    if (key < T) {
      dst[lt_before + min(eq_before, need_eq)] = j;
      ++lt_before;
    } else if (key == T) {
      if (eq_before < need_eq) dst[lt_before + eq_before] = j;
      ++eq_before;
    }
  }
}

// ------------------------------------------------------------- relax state --
enum PStatus {
  kRunning = 0,
  kConverged = 1,      // current evaluator converged
  kIterCap = 2,
  kLineSearchFail = 3,
  kNonFinite = 4,
  kDone = 5            // exact reduced gradient met the tolerance (mixed path)
};
enum Eval { kEvalExact = 0, kEvalModel32 = 1, kEvalModel64 = 2 };
// What the next round does for a running patch: evaluate a trial point and
// accept or shorten it (kPhaseStep), or one CG iteration of a Newton step
// (kPhaseCG: the product of the tangent Hessian with the CG direction, then
// the CG update).
enum Phase { kPhaseStep = 0, kPhaseCG = 1 };

struct PState {
  double E, Et;      // objective at z and at the trial zt (current evaluator)
  double alpha;      // trial step length
  double gi;         // inf-norm of the reduced gradient at z
  double R;          // patch radius about its centre
  double cx, cy;     // patch centre (box centre of the snapshot actives)
  int it, mem, head, status, init, total_it, exact_evals, evals;
  int use32;         // mixed path: this round's model uses FP32 pairs
  int newton;        // truncated-Newton polish: directions from CG on the tangent Hessian
  int phase;         // Phase
  int cg_it;         // CG iterations of the current Newton step
  int newton_steps;  // accepted Newton steps (all rounds)
  int cg_total;      // CG iterations (all rounds)
  int nfail;         // Newton steps that did not halve the reduced gradient
  int newton_off;    // Newton mode given up for this patch (L-BFGS to the end)
  double rz;         // CG: r . M^-1 r of the current residual
  double cg_target;  // CG: the step ends when the residual's inf-norm is below this
  double gnewt;      // reduced gradient at the start of the last Newton step (0: none)
  double eta;        // relative CG target of the last Newton step
  double gexact;     // mixed path: the exact reduced gradient at the last round's check
  int force64;       // mixed path: FP64 model pairs from here on (FP32 rounds stalled)
  int skip_k;        // plain path: the next exact evaluation leaves out the Hessian blocks
  int pad2;
};

struct RelaxDev {
  // sizes
  int n, P, nbN, m, ntot, nblk, splits, jb;
  // snapshot and packed active data
  const double* x;
  const double* y;
  const int32_t* ptr;      // [P+1]
  const int32_t* idx;      // [ntot] charge index of packed active a
  int32_t* pid;            // [ntot] patch of packed active a
  int2* blk;               // [nblk] (patch, first packed active) per 64-active block
  uint64_t* maskA;         // [P][nbN] membership of A_p (original order)
  uint64_t* maskAH;        // [P][nbN] membership of A_p and its halo
  double *z0x, *z0y;       // snapshot positions of actives
  double *zx, *zy;         // current
  double *tx, *ty;         // trial
  double *gx, *gy;         // gradient at z (current evaluator)
  double *hgx, *hgy;       // gradient at the trial
  double *kxx, *kxy, *kyy;     // preconditioner: the charge's own 2x2 Hessian block at z
  double *hkxx, *hkxy, *hkyy;  // the same at the trial
  double *pkxx, *pkxy, *pkyy;  // [splits][ntot] split partials of the blocks
  double *dx, *dy;         // search direction (coordinates: held -> angle in dx)
  double *Sx, *Sy, *Yx, *Yy;  // L-BFGS history [m][ntot]
  double* rho;             // [P][m]
  int32_t* held;           // [ntot] optimisation coordinates: 0 (x, y); 1 the polar angle
                           // on the circle; kHeldTU the (t, u) of Sec. II.D
  int32_t* pin;            // [ntot] 1: boundary charge pinned to the unit circle
  const int32_t* bflag;    // [n] caller's boundary flags (null: none)
  double sigma;            // wall radius of the charges that are not pinned
  double* eterm;           // [ntot] per-active energy contribution of the last evaluation
  double *px, *py, *pe;    // [splits][ntot] split partials of the exact evaluation
  // mixed-path model
  double *fgx, *fgy;       // far-field gradient at the snapshot
  double *fhxx, *fhxy, *fhyy;  // far-field Hessian at the snapshot
  double *zrx, *zry;       // expansion point of the far-field model
  int32_t* hptr;           // [P+1] halo CSR
  int32_t* hidx;           // halo charge indices
  int hcap;
  float *a32x, *a32y;      // trial actives relative to their patch centre (FP32)
  float *h32x, *h32y;      // halo relative to the patch centre (FP32)
  double *h64x, *h64y;     // halo positions, packed (FP64)
  PState* st;              // [P]
  int32_t* running;        // [2] patches still running; [1] nonzero: a patch asks for a new halo
  // options
  double tol, step0, c1, noise_rel;
  int max_iter, eval_all;
  int32_t* ptr_w;          // [P+1] device copy of the patch offsets (in the workspace)
  double* ptol;            // [P] per-patch stage tolerance (null: tol)
  int32_t* err;            // [1] argument error found on the device
  // truncated-Newton polish: CG iterate x, residual r, direction d (all in
  // optimisation coordinates), the product q = H_t d, and d in Cartesian
  // form w (held charge: d_0 (-y, x); free: d)
  double *cgx, *cgy, *crx, *cry, *cdx, *cdy, *cqx, *cqy, *cwx, *cwy;
  int polish;              // directions of patches in Newton mode come from CG
  int max_cg;              // CG iterations per Newton step
  double newton_tol;       // Newton mode below this exact reduced gradient
  double cg_eta;           // CG target: cg_eta * |g|inf of the step's start
  double gtol;             // the call's tolerance on the exact reduced gradient
  double trust;            // mixed path: model radius about the expansion point
  double *zhx, *zhy;       // mixed path: active positions when the halo was built
  double rebuild_d2;       // squared displacement from them that asks for a new halo
  int32_t* pstats;         // [2P] or null: Newton steps and CG iterations per patch
  // (t, u) parameterisation of interior charges (Sec. II.D, Eqs. 8-9)
  int tu;                  // interior charges start in (t, u) (those beyond tu_rmin)
  double tu_rmin;          // interior charges starting closer to the centre keep (x, y)
  double *ct, *cu;         // (t, u) at z of the actives in (t, u) coordinates
  double *tct, *tcu;       // the same at the trial
};

// ------------------------------------------------------------ setup kernels --
// Feasible projection: a pinned charge onto the unit circle, any other charge
// beyond its wall radius sig onto that circle.
__device__ __forceinline__ void project_wall(double& px, double& py, int pin, double sig) {
  const double r = sqrt(px * px + py * py);
  if (pin) {
    if (r > 0.0) {
      px /= r;
      py /= r;
    }
  } else if (r > sig) {
    if (sig == 1.0) {
      px /= r;
      py /= r;
    } else {
      px *= sig / r;
      py *= sig / r;
    }
  }
}

// The (t, u) parameterisation of an interior charge (Sec. II.D): position
// r (cos u, sin u) with r = sigma sin^2 t, and the gradient in (t, u) by the
// chain rule of Eqs. 8-9: dE/dt = (g_x cos u + g_y sin u) sigma sin 2t,
// dE/du = (-g_x sin u + g_y cos u) r.
constexpr int kHeldTU = 2;
__device__ __forceinline__ void tu_position(double sig, double t, double u, double& x, double& y) {
  const double st = sin(t);
  const double r = sig * (st * st);
  double su, cu;
  sincos(u, &su, &cu);
  x = r * cu;
  y = r * su;
}
__device__ __forceinline__ void tu_grad(double sig, double t, double u, double g0, double g1,
                                        double& c0, double& c1) {
  double su, cu, st, ctt;
  sincos(u, &su, &cu);
  sincos(t, &st, &ctt);
  c0 = (g0 * cu + g1 * su) * (sig * (2.0 * st * ctt));
  c1 = (-g0 * su + g1 * cu) * (sig * (st * st));
}

__global__ void k_setup_actives(RelaxDev R, const double* __restrict__ xs,
                                const double* __restrict__ ys) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= R.ntot) return;
  // patch of a: binary search in ptr
  int lo = 0, hi = R.P;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (R.ptr[mid] <= a) lo = mid;
    else hi = mid;
  }
  R.pid[a] = lo;
  int i = R.idx[a];
  if (i < 0 || i >= R.n) {  // invalid charge index: report, stay in bounds
    atomicOr(R.err, 1);
    i = 0;
  }
  R.z0x[a] = R.x[i];
  R.z0y[a] = R.y[i];
  if (R.zhx) {  // the halo is first built about the snapshot actives
    R.zhx[a] = R.x[i];
    R.zhy[a] = R.y[i];
  }
  double sx = xs ? xs[a] : R.x[i], sy = ys ? ys[a] : R.y[i];
  const int pin = R.bflag ? (R.bflag[i] != 0) : 0;
  R.pin[a] = pin;
  project_wall(sx, sy, pin, R.sigma);
  int kind = 0;
  if (R.tu && !pin) {
    // (t, u) of Sec. II.D for an interior charge, r = sigma sin^2 t: at
    // r = 0 both derivatives of Eqs. 8-9 vanish for any force, so charges
    // starting within tu_rmin of the centre keep (x, y) (they lie almost
    // sigma from the wall).  At t = pi/2 (on the wall) dE/dt vanishes too, so
    // a charge there pushed inward could not leave: t starts at most
    // pi/2 - 1e-8 (below an ulp of r).  The position is the one (t, u) gives.
    const double r = sqrt(sx * sx + sy * sy);
    if (r >= R.tu_rmin) {
      kind = kHeldTU;
      const double t = fmin(asin(sqrt(fmin(1.0, r / R.sigma))), 0.5 * 3.141592653589793 - 1e-8);
      const double u = atan2(sy, sx);
      R.ct[a] = R.tct[a] = t;
      R.cu[a] = R.tcu[a] = u;
      tu_position(R.sigma, t, u, sx, sy);
    }
  }
  R.zx[a] = sx;
  R.zy[a] = sy;
  R.tx[a] = sx;
  R.ty[a] = sy;
  R.held[a] = kind;
  const uint64_t bit = 1ull << (i & 63);
  atomicOr((unsigned long long*)&R.maskA[(size_t)lo * R.nbN + (i >> 6)], (unsigned long long)bit);
  atomicOr((unsigned long long*)&R.maskAH[(size_t)lo * R.nbN + (i >> 6)], (unsigned long long)bit);
}

// Patch centre and radius from the snapshot actives; one workgroup per patch.
__global__ __launch_bounds__(256) void k_patch_geom(RelaxDev R) {
  __shared__ double red[4][4];
  const int p = blockIdx.x, t = threadIdx.x;
  const int a0 = R.ptr[p], a1 = R.ptr[p + 1];
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  for (int a = a0 + t; a < a1; a += blockDim.x) {
    x0 = fmin(x0, R.z0x[a]);
    x1 = fmax(x1, R.z0x[a]);
    y0 = fmin(y0, R.z0y[a]);
    y1 = fmax(y1, R.z0y[a]);
  }
  x0 = wave_min(x0);
  x1 = wave_max(x1);
  y0 = wave_min(y0);
  y1 = wave_max(y1);
  if ((t & 63) == 0) {
    red[t >> 6][0] = x0;
    red[t >> 6][1] = x1;
    red[t >> 6][2] = y0;
    red[t >> 6][3] = y1;
  }
  __syncthreads();
  const double cx = 0.5 * (fmin(fmin(red[0][0], red[1][0]), fmin(red[2][0], red[3][0])) +
                           fmax(fmax(red[0][1], red[1][1]), fmax(red[2][1], red[3][1])));
  const double cy = 0.5 * (fmin(fmin(red[0][2], red[1][2]), fmin(red[2][2], red[3][2])) +
                           fmax(fmax(red[0][3], red[1][3]), fmax(red[2][3], red[3][3])));
  double rm = 0.0;
  for (int a = a0 + t; a < a1; a += blockDim.x) {
    const double dx = R.z0x[a] - cx, dy = R.z0y[a] - cy;
    rm = fmax(rm, sqrt(dx * dx + dy * dy));
  }
  rm = wave_max(rm);
  __syncthreads();
  if ((t & 63) == 0) red[t >> 6][0] = rm;
  __syncthreads();
  if (t == 0) {
    PState s = {};
    s.cx = cx;
    s.cy = cy;
    s.R = fmax(fmax(red[0][0], red[1][0]), fmax(red[2][0], red[3][0]));
    s.status = kRunning;
    s.init = 1;
    s.alpha = 1.0;
    R.st[p] = s;
  }
}

// Halo of patch p: frozen charges within R_p + w of the patch centre.  Pass 0
// counts, pass 1 fills (index order, stable) and marks maskAH.
// geom (nullable): centre and radius [3P] to use instead of the patch state's.
__global__ __launch_bounds__(1024) void k_halo(RelaxDev R, double w, int fill,
                                               int32_t* __restrict__ counts,
                                               const double* __restrict__ geom) {
  __shared__ uint32_t cnt[1024];
  const int p = blockIdx.x, t = threadIdx.x;
  PState s = R.st[p];
  if (geom) {
    s.cx = geom[3 * p];
    s.cy = geom[3 * p + 1];
    s.R = geom[3 * p + 2];
  }
  const double lim = (s.R + w) * (s.R + w);
  const int chunk = (R.n + blockDim.x - 1) / blockDim.x;
  const int j0 = min(R.n, t * chunk), j1 = min(R.n, j0 + chunk);
  uint32_t c = 0;
  for (int j = j0; j < j1; ++j) {
    const bool act = (R.maskA[(size_t)p * R.nbN + (j >> 6)] >> (j & 63)) & 1ull;
    const double dx = R.x[j] - s.cx, dy = R.y[j] - s.cy;
    c += (!act && dx * dx + dy * dy <= lim);
  }
  cnt[t] = c;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const uint32_t v = t >= off ? cnt[t - off] : 0u;
    __syncthreads();
    cnt[t] += v;
    __syncthreads();
  }
  if (!fill) {
    if (t == 0) counts[p] = (int32_t)cnt[blockDim.x - 1];
    return;
  }
  uint32_t pos = R.hptr[p] + cnt[t] - c;
  for (int j = j0; j < j1; ++j) {
    const bool act = (R.maskA[(size_t)p * R.nbN + (j >> 6)] >> (j & 63)) & 1ull;
    const double dx = R.x[j] - s.cx, dy = R.y[j] - s.cy;
    if (!act && dx * dx + dy * dy <= lim) {
      R.hidx[pos++] = j;
      atomicOr((unsigned long long*)&R.maskAH[(size_t)p * R.nbN + (j >> 6)],
               (unsigned long long)(1ull << (j & 63)));
    }
  }
}

// Halo rebuild (mixed path), when a patch's actives have drifted from where
// its halo was built: the box centre and radius of the current actives of
// every patch, into geom [3P] (the same rule as k_patch_geom on the
// snapshot); then k_geom_commit makes them the patch's and records the
// positions the new halo is built about.
__global__ __launch_bounds__(256) void k_patch_recentre(RelaxDev R, double* __restrict__ geom) {
  __shared__ double red[4][4];
  const int p = blockIdx.x, t = threadIdx.x;
  const int a0 = R.ptr[p], a1 = R.ptr[p + 1];
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  for (int a = a0 + t; a < a1; a += blockDim.x) {
    x0 = fmin(x0, R.zx[a]);
    x1 = fmax(x1, R.zx[a]);
    y0 = fmin(y0, R.zy[a]);
    y1 = fmax(y1, R.zy[a]);
  }
  x0 = wave_min(x0);
  x1 = wave_max(x1);
  y0 = wave_min(y0);
  y1 = wave_max(y1);
  if ((t & 63) == 0) {
    red[t >> 6][0] = x0;
    red[t >> 6][1] = x1;
    red[t >> 6][2] = y0;
    red[t >> 6][3] = y1;
  }
  __syncthreads();
  const double cx = 0.5 * (fmin(fmin(red[0][0], red[1][0]), fmin(red[2][0], red[3][0])) +
                           fmax(fmax(red[0][1], red[1][1]), fmax(red[2][1], red[3][1])));
  const double cy = 0.5 * (fmin(fmin(red[0][2], red[1][2]), fmin(red[2][2], red[3][2])) +
                           fmax(fmax(red[0][3], red[1][3]), fmax(red[2][3], red[3][3])));
  double rm = 0.0;
  for (int a = a0 + t; a < a1; a += blockDim.x) {
    const double dx = R.zx[a] - cx, dy = R.zy[a] - cy;
    rm = fmax(rm, sqrt(dx * dx + dy * dy));
  }
  rm = wave_max(rm);
  __syncthreads();
  if ((t & 63) == 0) red[t >> 6][0] = rm;
  __syncthreads();
  if (t == 0) {
    geom[3 * p] = cx;
    geom[3 * p + 1] = cy;
    geom[3 * p + 2] = fmax(fmax(red[0][0], red[1][0]), fmax(red[2][0], red[3][0]));
  }
}

__global__ void k_geom_commit(RelaxDev R, const double* __restrict__ geom) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a < R.P) {
    R.st[a].cx = geom[3 * a];
    R.st[a].cy = geom[3 * a + 1];
    R.st[a].R = geom[3 * a + 2];
  }
  if (a < R.ntot) {
    R.zhx[a] = R.zx[a];
    R.zhy[a] = R.zy[a];
  }
  if (a == 0) R.running[1] = 0;
}

// ------------------------------------------------------ exact FP64 evaluation --
// Wave = 64 packed actives of one patch (grid.x over the block table), grid.y
// = split of the N snapshot charges.  Frozen charges come from the snapshot,
// skipped when the patch mask marks them; active ones from the trial
// positions of the same patch.  Charges are wave-uniform and read through the
// scalar cache.
//   kGrad : energy contribution and gradient at the trial positions
//   kFar  : far-field gradient and Hessian at the trial positions, which
//           become the model's expansion point (mask = A + halo)
//   kDelta: E_sub(trial) - E_sub(snapshot), pair differences without
//           cancellation: 1/r' - 1/r = (d - d').(d + d') / (r r' (r + r'))
enum ExactMode { kGrad = 0, kFar = 1, kDelta = 2 };

template <int MODE>
__global__ __launch_bounds__(256) void k_exact(RelaxDev R) {
  // the wave index is uniform within a wave; saying so lets the compiler keep
  // patch data in SGPRs and read the j charges through the scalar cache
  const int wb = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (wb >= R.nblk) return;
  const int2 bk = R.blk[wb];
  const int p = bk.x;
  if (MODE == kGrad && !R.eval_all && (R.st[p].status != kRunning || R.st[p].phase == kPhaseCG))
    return;
  // a re-expansion skips the patches that are finished (their far field is
  // not used again: the final outputs come from a separate exact pass)
  if (MODE == kFar && (R.st[p].status == kDone || R.st[p].status == kNonFinite)) return;
  // kGrad takes the Hessian blocks unless the patch's update said it can do
  // without them this time (plain path, between Newton phases); uniform per wave
  const bool wk = MODE == kFar || (MODE == kGrad && (R.eval_all || !R.st[p].skip_k));
  const int a0 = R.ptr[p], a1 = R.ptr[p + 1];
  const int a = bk.y + lane;
  const bool ok = a < a1;
  const int ac = ok ? a : a1 - 1;
  const double xi = R.tx[ac];
  const double yi = R.ty[ac];
  const double xo = R.z0x[ac], yo = R.z0y[ac];  // snapshot position (kDelta)
  const uint64_t* mask = (MODE == kFar ? R.maskAH : R.maskA) + (size_t)p * R.nbN;
  double G0 = 0.0, G1 = 0.0, G2 = 0.0, G3 = 0.0, G4 = 0.0, S3 = 0.0, Ee = 0.0, Ec = 0.0;
  const int J0 = blockIdx.y * R.jb, J1 = min(R.nbN, J0 + R.jb);
  auto pairs = [&](auto wk_tag) {
    constexpr bool WK = decltype(wk_tag)::value;
    for (int J = J0; J < J1; ++J) {
      const uint64_t m = mask[J];  // wave-uniform: charges of the patch (and halo) are skipped
      const int jn = min(64, R.n - J * 64);
      const double* xb = R.x + (size_t)J * 64;
      const double* yb = R.y + (size_t)J * 64;
      double eb = 0.0;
      // the skip test only in blocks that hold charges of the patch (or its
      // halo); most blocks of a large N hold none
      auto block = [&](auto masked_tag) {
        constexpr bool M = decltype(masked_tag)::value;
#pragma unroll 8
        for (int jj = 0; jj < jn; ++jj) {
          const bool skip = M && ((m >> jj) & 1ull);
          const double xj = xb[jj], yj = yb[jj];
          const double dx = xi - xj, dy = yi - yj;
          const double r2 = __builtin_fma(dx, dx, dy * dy);
          if (MODE == kDelta) {
            const double ox = xo - xj, oy = yo - yj;
            const double ro2 = __builtin_fma(ox, ox, oy * oy);
            const double ri = rsqrt64(r2), roi = rsqrt64(ro2);
            const double rn = r2 * ri, ro = ro2 * roi;
            const double num = (ox - dx) * (ox + dx) + (oy - dy) * (oy + dy);
            const double v = num * ri * roi / (rn + ro);
            eb += skip ? 0.0 : v;
          } else {
            double inv = rsqrt64(r2);
            inv = skip ? 0.0 : inv;
            const double i3 = inv * inv * inv;
            G0 = __builtin_fma(-dx, i3, G0);
            G1 = __builtin_fma(-dy, i3, G1);
            if (MODE == kGrad) eb += inv;
            if (WK) {
              // K = 3 d d^T / r^5 - I / r^3: the d d^T part here, the sum of
              // 1/r^3 (the same for both diagonal entries) apart in S3
              const double t3 = 3.0 * i3 * (inv * inv);
              const double u = t3 * dx;
              G2 = __builtin_fma(u, dx, G2);
              G3 = __builtin_fma(u, dy, G3);
              G4 = __builtin_fma(t3 * dy, dy, G4);
              S3 += i3;
            }
          }
        }
      };
      if (m)
        block(std::true_type{});
      else
        block(std::false_type{});
      const double tt = Ee + eb;  // Neumaier across 64-charge blocks
      Ec += fabs(Ee) >= fabs(eb) ? (Ee - tt) + eb : (eb - tt) + Ee;
      Ee = tt;
    }
    if (MODE != kFar && blockIdx.y == 0) {
      // active-active pairs at the trial positions (half weight in the energy)
#pragma unroll 4
      for (int b = a0; b < a1; ++b) {
        const double xj = R.tx[b], yj = R.ty[b];
        const double dx = xi - xj, dy = yi - yj;
        const double r2 = __builtin_fma(dx, dx, dy * dy);
        if (MODE == kDelta) {
          const double ox = xo - R.z0x[b], oy = yo - R.z0y[b];
          const double ro2 = __builtin_fma(ox, ox, oy * oy);
          double v = 0.0;
          if (b != ac) {
            const double ri = rsqrt64(r2), roi = rsqrt64(ro2);
            const double rn = r2 * ri, ro = ro2 * roi;
            const double num = (ox - dx) * (ox + dx) + (oy - dy) * (oy + dy);
            v = 0.5 * (num * ri * roi / (rn + ro));
          }
          const double tt = Ee + v;
          Ec += fabs(Ee) >= fabs(v) ? (Ee - tt) + v : (v - tt) + Ee;
          Ee = tt;
        } else {
          double inv = rsqrt64(r2);
          inv = (b == ac) ? 0.0 : inv;
          const double i3 = inv * inv * inv;
          const double h = 0.5 * inv;
          const double tt = Ee + h;
          Ec += fabs(Ee) >= fabs(h) ? (Ee - tt) + h : (h - tt) + Ee;
          Ee = tt;
          G0 = __builtin_fma(-dx, i3, G0);
          G1 = __builtin_fma(-dy, i3, G1);
          if (WK) {
            const double t3 = 3.0 * i3 * (inv * inv);
            const double u = t3 * dx;
            G2 = __builtin_fma(u, dx, G2);
            G3 = __builtin_fma(u, dy, G3);
            G4 = __builtin_fma(t3 * dy, dy, G4);
            S3 += i3;
          }
        }
      }
    }
  };
  if (MODE == kDelta || !wk)
    pairs(std::false_type{});
  else
    pairs(std::true_type{});
  if (!ok) return;
  const size_t q = (size_t)blockIdx.y * R.ntot + a;
  R.px[q] = G0;
  R.py[q] = G1;
  if (MODE != kFar) R.pe[q] = Ee + Ec;
  if (MODE != kDelta && wk) {
    R.pkxx[q] = G2 - S3;
    R.pkxy[q] = G3;
    R.pkyy[q] = G4 - S3;
  }
  if (MODE == kFar && blockIdx.y == 0) {
    R.zrx[a] = xi;  // the expansion point
    R.zry[a] = yi;
  }
}

// Sum the split partials: mode kDelta the energy terms, kGrad also the
// trial gradient and Hessian blocks, kFar the far-field gradient and Hessian
// (no energy).  One workgroup per 64 actives: wave w sums the splits w,
// w + kESW, ... in increasing order, then the wave partials are added in
// wave order, so the order is fixed and a long split list is read by kESW
// waves at once.
constexpr int kESW = 8;

__global__ __launch_bounds__(64 * kESW) void k_exact_sum(RelaxDev R, int mode) {
  const bool grad = mode != kDelta;
  __shared__ double part[kESW - 1][6][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int a = blockIdx.x * 64 + lane;
  int ps = kRunning;
  if (a < R.ntot && mode == kFar) ps = R.st[R.pid[a]].status;
  // finished patches were left out of the re-expansion (see k_exact)
  const bool ok = a < R.ntot && ps != kDone && ps != kNonFinite;
  // the Hessian blocks were taken for this active's patch (see k_exact)
  const bool wk = ok && (mode == kFar || (mode == kGrad && (R.eval_all || !R.st[R.pid[a]].skip_k)));
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (ok) {
    for (int sp = w; sp < R.splits; sp += kESW) {
      const size_t q = (size_t)sp * R.ntot + a;
      v[0] += R.px[q];
      v[1] += R.py[q];
      if (mode != kFar) v[2] += R.pe[q];
      if (wk) {
        v[3] += R.pkxx[q];
        v[4] += R.pkxy[q];
        v[5] += R.pkyy[q];
      }
    }
  }
  if (w > 0) {
#pragma unroll
    for (int c = 0; c < 6; ++c) part[w - 1][c][lane] = v[c];
  }
  __syncthreads();
  if (w > 0 || !ok) return;
  for (int q = 0; q < kESW - 1; ++q) {
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] += part[q][c][lane];
  }
  if (mode == kFar) {
    R.fgx[a] = v[0];
    R.fgy[a] = v[1];
    R.fhxx[a] = v[3];
    R.fhxy[a] = v[4];
    R.fhyy[a] = v[5];
    return;
  }
  if (grad) {
    R.hgx[a] = v[0];
    R.hgy[a] = v[1];
    if (wk) {  // else the last blocks taken stay (the preconditioner may lag)
      R.hkxx[a] = v[3];
      R.hkxy[a] = v[4];
      R.hkyy[a] = v[5];
    }
  }
  R.eterm[a] = v[2];
}

// ------------------------------------------------------------ model evaluation --
// Active i against its patch's other actives (trial positions) and its halo
// (snapshot), plus the far field as a Taylor model about the expansion point:
//   E_i = 1/2 sum_A 1/r + sum_halo 1/r + f.d + 1/2 d.H d,  d = z_i - zr_i
// Per patch either FP32 pairs (coordinates relative to the patch centre,
// partials of at most 64 terms folded into FP64) or FP64 pairs.
// SELF: the j range holds the actives, and every lane's own index lies in
// [diag, diag + 64) (its 64-active block); only the 64-term chunks that meet
// that range test j against the lane's index, the others need no test.
template <bool SELF, bool WK>
__device__ __forceinline__ void pairs32(const float* __restrict__ xs, const float* __restrict__ ys,
                                        int b0, int b1, int self, int diag, float xf, float yf,
                                        double& G0, double& G1, double& E, double* K, double w) {
  for (int c0 = b0; c0 < b1; c0 += 64) {
    const int c1 = min(b1, c0 + 64);
    float g0 = 0.f, g1 = 0.f, e = 0.f, k0 = 0.f, k1 = 0.f, k2 = 0.f;
    auto chunk = [&](auto self_tag) {
      constexpr bool S = decltype(self_tag)::value;
#pragma unroll 8
      for (int b = c0; b < c1; ++b) {
        const float dx = xf - xs[b], dy = yf - ys[b];
        const float r2 = __builtin_fmaf(dx, dx, dy * dy);
        float inv = __builtin_amdgcn_rsqf(r2);
        if (S) inv = (b == self) ? 0.f : inv;
        const float i3 = inv * inv * inv;
        e += inv;
        g0 = __builtin_fmaf(-dx, i3, g0);
        g1 = __builtin_fmaf(-dy, i3, g1);
        if (WK) {
          const float t3 = 3.0f * i3 * inv * inv;
          k0 += __builtin_fmaf(t3 * dx, dx, -i3);
          k1 += t3 * dx * dy;
          k2 += __builtin_fmaf(t3 * dy, dy, -i3);
        }
      }
    };
    if (SELF && c0 < diag + 64 && c1 > diag)
      chunk(std::true_type{});
    else
      chunk(std::false_type{});
    G0 += g0;
    G1 += g1;
    E += w * (double)e;
    K[0] += k0;
    K[1] += k1;
    K[2] += k2;
  }
}

template <bool SELF, bool WK>
__device__ __forceinline__ void pairs64(const double* __restrict__ xs,
                                        const double* __restrict__ ys, int b0, int b1, int self,
                                        int diag, double xi, double yi, double& G0, double& G1,
                                        double& E, double& Ec, double* K, double w) {
  for (int c0 = b0; c0 < b1; c0 += 64) {
    const int c1 = min(b1, c0 + 64);
    double e = 0.0;
    auto chunk = [&](auto self_tag) {
      constexpr bool S = decltype(self_tag)::value;
#pragma unroll 4
      for (int b = c0; b < c1; ++b) {
        const double dx = xi - xs[b], dy = yi - ys[b];
        const double r2 = __builtin_fma(dx, dx, dy * dy);
        double inv = rsqrt64(r2);
        if (S) inv = (b == self) ? 0.0 : inv;
        const double i3 = inv * inv * inv;
        e += inv;
        G0 = __builtin_fma(-dx, i3, G0);
        G1 = __builtin_fma(-dy, i3, G1);
        if (WK) {
          const double t3 = 3.0 * i3 * inv * inv;
          K[0] += __builtin_fma(t3 * dx, dx, -i3);
          K[1] += t3 * dx * dy;
          K[2] += __builtin_fma(t3 * dy, dy, -i3);
        }
      }
    };
    if (SELF && c0 < diag + 64 && c1 > diag)
      chunk(std::true_type{});
    else
      chunk(std::false_type{});
    const double v = w * e;
    const double tt = E + v;
    Ec += fabs(E) >= fabs(v) ? (E - tt) + v : (v - tt) + E;
    E = tt;
  }
}

// One workgroup per 64-active block; its MW waves split the patch's j list
// (actives, then halo) into ranges cut at multiples of 16 (at multiples of
// 64 the last waves of a workgroup often had little or nothing to do while
// the others set its time) and the partial sums are combined in LDS in wave
// order, so a large patch spreads over MW times more waves.  MW = kMW, or kMWWide when few blocks belong to
// patches still running (the chip would otherwise sit mostly idle).
constexpr int kMW = 8;
constexpr int kMWWide = 16;

template <bool WK, int MW>
__global__ __launch_bounds__(64 * MW) void k_model(RelaxDev R) {
  __shared__ double part[MW][7][64];  // G0 G1 E Ec K0 K1 K2 per wave and lane
  const int wb = blockIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (wb >= R.nblk) return;
  const int2 bk = R.blk[wb];
  const int p = bk.x;
  const PState& st = R.st[p];
  // the same for the whole workgroup; a patch in its CG phase has no trial,
  // and an evaluation at the expansion point leaves out finished patches
  if (R.eval_all ? (st.status == kDone || st.status == kNonFinite)
                 : (st.status != kRunning || st.phase == kPhaseCG))
    return;
  const bool use32 = st.use32;
  const int a0 = R.ptr[p], a1 = R.ptr[p + 1];
  const int h0 = R.hptr[p], h1 = R.hptr[p + 1];
  const int na = a1 - a0, nj = na + (h1 - h0);
  const int per = ((nj + MW - 1) / MW + 15) & ~15;
  const int j0 = min(nj, w * per), j1 = min(nj, j0 + per);
  const int a = bk.y + lane;
  const bool ok = a < a1;
  const int ac = ok ? a : a1 - 1;
  const double xi = R.tx[ac], yi = R.ty[ac];
  double G0 = 0.0, G1 = 0.0, E = 0.0, Ec = 0.0, K[3] = {0.0, 0.0, 0.0};
  if (use32) {
    const float xf = R.a32x[ac], yf = R.a32y[ac];
    pairs32<true, WK>(R.a32x, R.a32y, a0 + j0, a0 + min(j1, na), ac, bk.y, xf, yf, G0, G1, E, K,
                      0.5);
    pairs32<false, WK>(R.h32x, R.h32y, h0 + max(j0, na) - na, h0 + max(j1, na) - na, -1, 0, xf,
                       yf, G0, G1, E, K, 1.0);
  } else {
    pairs64<true, WK>(R.tx, R.ty, a0 + j0, a0 + min(j1, na), ac, bk.y, xi, yi, G0, G1, E, Ec, K,
                      0.5);
    pairs64<false, WK>(R.h64x, R.h64y, h0 + max(j0, na) - na, h0 + max(j1, na) - na, -1, 0, xi,
                       yi, G0, G1, E, Ec, K, 1.0);
  }
  part[w][0][lane] = G0;
  part[w][1][lane] = G1;
  part[w][2][lane] = E;
  part[w][3][lane] = Ec;
  part[w][4][lane] = K[0];
  part[w][5][lane] = K[1];
  part[w][6][lane] = K[2];
  __syncthreads();
  if (w != 0 || !ok) return;
  G0 = G1 = E = Ec = 0.0;
  K[0] = K[1] = K[2] = 0.0;
  for (int q = 0; q < MW; ++q) {
    G0 += part[q][0][lane];
    G1 += part[q][1][lane];
    const double v = part[q][2][lane], tt = E + v;  // Neumaier across the waves' sums
    Ec += (fabs(E) >= fabs(v) ? (E - tt) + v : (v - tt) + E) + part[q][3][lane];
    E = tt;
    K[0] += part[q][4][lane];
    K[1] += part[q][5][lane];
    K[2] += part[q][6][lane];
  }
  E += Ec;
  const double ddx = xi - R.zrx[a], ddy = yi - R.zry[a];
  const double hx = R.fhxx[a] * ddx + R.fhxy[a] * ddy, hy = R.fhxy[a] * ddx + R.fhyy[a] * ddy;
  E += R.fgx[a] * ddx + R.fgy[a] * ddy + 0.5 * (ddx * hx + ddy * hy);
  R.hgx[a] = G0 + R.fgx[a] + hx;
  R.hgy[a] = G1 + R.fgy[a] + hy;
  if (WK) {
    R.hkxx[a] = K[0] + R.fhxx[a];
    R.hkxy[a] = K[1] + R.fhxy[a];
    R.hkyy[a] = K[2] + R.fhyy[a];
  }
  R.eterm[a] = E;
}

// FP32 coordinates of trial actives relative to the patch centre; with
// halo_too also the halo, packed (FP64 and FP32 relative).
__global__ void k_model_prep(RelaxDev R, int halo_too) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a < R.ntot) {
    const PState& s = R.st[R.pid[a]];
    R.a32x[a] = (float)(R.tx[a] - s.cx);
    R.a32y[a] = (float)(R.ty[a] - s.cy);
  }
  if (halo_too && a < R.hptr[R.P]) {
    int lo = 0, hi = R.P;  // patch of halo entry a
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (R.hptr[mid] <= a) lo = mid;
      else hi = mid;
    }
    const PState& s = R.st[lo];
    const int j = R.hidx[a];
    R.h64x[a] = R.x[j];
    R.h64y[a] = R.y[j];
    R.h32x[a] = (float)(R.x[j] - s.cx);
    R.h32y[a] = (float)(R.y[j] - s.cy);
  }
}

// ------------------------------------------------- truncated-Newton product --
// q = H_t d for every patch in its CG phase (truncated-Newton polish): the
// Hessian of E_sub at z on the tangent space of the wall, applied to the CG
// direction d.  With w the Cartesian form of d,
//   (H w)_i = B_i w_i - sum_{j in A, j != i} K(z_i - z_j) w_j,
// K(r) = (3 r r^T - |r|^2 I) / |r|^5, where B_i = sum_{j != i} K(z_i - z_j)
// over every other charge is the charge's own 2x2 block: exact FP64 at z,
// written by the exact evaluation at z (plain path) or by the model
// evaluation at its expansion point z (mixed path: there the far field's
// quadratic carries the exact Hessian).  A held charge's coordinate is its
// angle, with tangent t = (-y, x): its component is t . (H w)_i - (g_i . z_i)
// d_i (the circle's curvature), a free charge's (H w)_i.  FP64 pairs.
// Workgroup layout as k_model: MW waves split the patch's actives into
// ranges cut at multiples of 16; their sums are combined in wave order.
template <int MW>
__global__ __launch_bounds__(64 * MW) void k_cg_hvp(RelaxDev R) {
  __shared__ double part[MW][2][64];
  const int wb = blockIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (wb >= R.nblk) return;
  const int2 bk = R.blk[wb];
  const int p = bk.x;
  const PState& st = R.st[p];
  if (st.status != kRunning || st.phase != kPhaseCG) return;  // uniform in the workgroup
  const int a0 = R.ptr[p], a1 = R.ptr[p + 1];
  const int na = a1 - a0;
  const int per = ((na + MW - 1) / MW + 15) & ~15;
  const int j0 = min(na, w * per), j1 = min(na, j0 + per);
  const int a = bk.y + lane;
  const bool ok = a < a1;
  const int ac = ok ? a : a1 - 1;
  const double xi = R.zx[ac], yi = R.zy[ac];
  double Q0 = 0.0, Q1 = 0.0;
  // in 64-term chunks: only the chunk that meets the block's own actives
  // [bk.y, bk.y + 64) tests j against the lane's index
  for (int c0 = a0 + j0; c0 < a0 + j1; c0 += 64) {
    const int c1 = min(a0 + j1, c0 + 64);
    auto chunk = [&](auto self_tag) {
      constexpr bool S = decltype(self_tag)::value;
#pragma unroll 4
      for (int b = c0; b < c1; ++b) {
        const double dx = xi - R.zx[b], dy = yi - R.zy[b];
        const double wx = R.cwx[b], wy = R.cwy[b];
        const double r2 = __builtin_fma(dx, dx, dy * dy);
        double inv = rsqrt64(r2);
        if (S) inv = (b == ac) ? 0.0 : inv;
        const double i3 = inv * inv * inv;
        const double sc = 3.0 * i3 * inv * inv * __builtin_fma(dx, wx, dy * wy);
        Q0 += __builtin_fma(dx, sc, -wx * i3);
        Q1 += __builtin_fma(dy, sc, -wy * i3);
      }
    };
    if (c0 < bk.y + 64 && c1 > bk.y)
      chunk(std::true_type{});
    else
      chunk(std::false_type{});
  }
  part[w][0][lane] = Q0;
  part[w][1][lane] = Q1;
  __syncthreads();
  if (w != 0 || !ok) return;
  Q0 = Q1 = 0.0;
  for (int q = 0; q < MW; ++q) {
    Q0 += part[q][0][lane];
    Q1 += part[q][1][lane];
  }
  const double wx = R.cwx[a], wy = R.cwy[a];
  const double hx = R.kxx[a] * wx + R.kxy[a] * wy - Q0;
  const double hy = R.kxy[a] * wx + R.kyy[a] * wy - Q1;
  if (R.held[a]) {
    const double px = R.zx[a], py = R.zy[a];
    const double gr = R.gx[a] * px + R.gy[a] * py;
    R.cqx[a] = -py * hx + px * hy - gr * R.cdx[a];
    R.cqy[a] = 0.0;
  } else {
    R.cqx[a] = hx;
    R.cqy[a] = hy;
  }
}

// ------------------------------------------------------------ update kernel --
// One workgroup per patch.  Accept/reject the trial (Armijo, or a reduced
// gradient decrease when the energy change is below the evaluation's noise),
// update the L-BFGS history and the wall-held set, test convergence, and
// form the next trial point.
constexpr int kUpd = 1024;
constexpr int kUpdWaves = kUpd / 64;
// actives per thread held in registers by the two-loop: kRegJ, or kRegJWide
// in a call with a patch above kRegJ * kUpd actives (one more register-held
// element per thread, so that a large patch's actives 4097 to 5120 are loaded
// one step ahead like the others instead of inside each step; for smaller
// patches it would only add masked work).  Both variants sum in the same
// order: the results are the same bit for bit.
constexpr int kRegJ = 4;
constexpr int kRegJWide = 5;

// Workgroup reductions of a kUpd-thread workgroup: each wave reduces by DPP
// (wave_sum_rows, wave_max_rows), the wave results go to LDS and every
// thread adds them in wave order.  The LDS partials alternate between two
// buffers, so one barrier per reduction suffices: a buffer is written again
// two reductions later, after every thread has passed the barrier of the
// reduction in between (and so has finished reading it).  Every thread of
// the workgroup must take part in every reduction, in the same order.
struct WgRed {
  double* buf;  // LDS, 2 * 3 * kUpdWaves doubles
  int par;
  __device__ explicit WgRed(double* b) : buf(b), par(0) {}
  __device__ double* next() {
    double* r = buf + par * 3 * kUpdWaves;
    par ^= 1;
    return r;
  }
};
#define WG_RED_LDS(name) __shared__ double name##_buf[2 * 3 * kUpdWaves]; WgRed name(name##_buf)

__device__ double block_sum(double v, WgRed& R) {
  v = wave_sum_rows(v);
  double* r = R.next();
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < kUpdWaves; ++q) t += r[q];
  return t;
}
__device__ double block_max(double v, WgRed& R) {
  v = wave_max_rows(v);
  double* r = R.next();
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = r[0];
  for (int q = 1; q < kUpdWaves; ++q) t = fmax(t, r[q]);
  return t;
}
// three sums in one pass
__device__ void block_sum3(double& a, double& b, double& c, WgRed& R) {
  a = wave_sum_rows(a);
  b = wave_sum_rows(b);
  c = wave_sum_rows(c);
  double* r = R.next();
  if ((threadIdx.x & 63) == 0) {
    const int w = threadIdx.x >> 6;
    r[3 * w] = a;
    r[3 * w + 1] = b;
    r[3 * w + 2] = c;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0, tc = 0.0;
  for (int q = 0; q < kUpdWaves; ++q) {
    ta += r[3 * q];
    tb += r[3 * q + 1];
    tc += r[3 * q + 2];
  }
  a = ta;
  b = tb;
  c = tc;
}
// a sum and a maximum in one pass
__device__ void block_sum_max(double& sm, double& mx, WgRed& R) {
  sm = wave_sum_rows(sm);
  mx = wave_max_rows(mx);
  double* r = R.next();
  if ((threadIdx.x & 63) == 0) {
    const int w = threadIdx.x >> 6;
    r[3 * w] = sm;
    r[3 * w + 1] = mx;
  }
  __syncthreads();
  double ts = 0.0, tm = r[1];
  for (int q = 0; q < kUpdWaves; ++q) {
    ts += r[3 * q];
    tm = fmax(tm, r[3 * q + 1]);
  }
  sm = ts;
  mx = tm;
}

// two maxima in one pass
__device__ void block_max2(double& a, double& b, WgRed& R) {
  a = wave_max_rows(a);
  b = wave_max_rows(b);
  double* r = R.next();
  if ((threadIdx.x & 63) == 0) {
    const int w = threadIdx.x >> 6;
    r[3 * w] = a;
    r[3 * w + 1] = b;
  }
  __syncthreads();
  double ta = r[0], tb = r[1];
  for (int q = 1; q < kUpdWaves; ++q) {
    ta = fmax(ta, r[3 * q]);
    tb = fmax(tb, r[3 * q + 1]);
  }
  a = ta;
  b = tb;
}

// Many sums at once.  rows_sum: each 16-lane row adds every one of the N
// values by DPP, the row's first lane stores the row sums, then a barrier.
// rows_total: the total of value q from its kRows row sums, in a fixed order
// (four interleaved partial sums, then (s0 + s1) + (s2 + s3)).
constexpr int kRows = kUpd / 16;
template <int N>
__device__ __forceinline__ void rows_sum(const double (&v)[N], double* part) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double x = v[q];
    x += dpp_f64<0xB1>(x);
    x += dpp_f64<0x4E>(x);
    x += dpp_f64<0x141>(x);
    x += dpp_f64<0x140>(x);
    if ((t & 15) == 0) part[q * kRows + (t >> 4)] = x;
  }
  __syncthreads();
}
__device__ __forceinline__ double rows_total(const double* part, int q) {
  const double* r = part + q * kRows;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int i = 0; i < kRows; i += 4) {
    s0 += r[i];
    s1 += r[i + 1];
    s2 += r[i + 2];
    s3 += r[i + 3];
  }
  return (s0 + s1) + (s2 + s3);
}

// reduced gradient component magnitude at position (px, py) with gradient g:
// a charge on its wall (radius sig: 1 for the hard wall of Eq. 3, the
// interior radius of the border-interior split) whose gradient points inward
// is held and keeps only the tangential part; a pinned boundary charge is
// always held
__device__ __forceinline__ bool held_rule(double px, double py, double g0, double g1, int pin,
                                          double sig) {
  if (pin) return true;
  const double r = sqrt(px * px + py * py);
  return r >= sig * (1.0 - 1e-14) && (g0 * px + g1 * py) < 0.0;
}
__device__ __forceinline__ double reduced_inf(double px, double py, double g0, double g1, int pin,
                                              double sig) {
  if (held_rule(px, py, g0, g1, pin, sig)) {
    const double r = sqrt(px * px + py * py);
    const double ux = px / r, uy = py / r, gr = g0 * ux + g1 * uy;
    return fmax(fabs(g0 - gr * ux), fabs(g1 - gr * uy));
  }
  return fmax(fabs(g0), fabs(g1));
}
// gradient in optimisation coordinates: (gx, gy) for a free charge, (dE/dtheta, 0) for a held one
__device__ __forceinline__ void coord_grad(bool h, double px, double py, double g0, double g1,
                                           double& c0, double& c1) {
  if (h) {
    c0 = -g0 * py + g1 * px;
    c1 = 0.0;
  } else {
    c0 = g0;
    c1 = g1;
  }
}

__device__ void take_step(bool h, double px, double py, double d0, double d1, double al,
                          double& nx, double& ny, int pin, double sig) {
  if (h) {
    double sn, cs;
    sincos(al * d0, &sn, &cs);
    nx = px * cs - py * sn;
    ny = px * sn + py * cs;
  } else {
    nx = px + al * d0;
    ny = py + al * d1;
  }
  project_wall(nx, ny, pin, sig);
}

__device__ __forceinline__ void prec2x2(double a, double b, double c, double q0, double q1,
                                        double& r0, double& r1);

// Preconditioner H0 = inverse of the charge's own Hessian block (its 2x2
// block for a free charge; d2E/dtheta2 = t.K.t - g.r_hat for a held one),
// with |eigenvalues| floored at 1e-3 of the largest when the block is not
// positive definite.  r = H0 q.
__device__ void apply_prec(bool held, double px, double py, double g0, double g1, double a,
                           double b, double c, double q0, double q1, double& r0, double& r1) {
  if (held) {
    const double rr = px * px + py * py;
    const double tt = (a * py * py - 2.0 * b * px * py + c * px * px) / rr;
    const double k = tt - (g0 * px + g1 * py) / sqrt(rr);
    const double f = fmax(fabs(k), 1e-3 * fmax(fabs(a), fabs(c)));
    r0 = f > 0.0 ? q0 / f : q0;
    r1 = 0.0;
    return;
  }
  prec2x2(a, b, c, q0, q1, r0, r1);
}

// r = M^-1 q for the symmetric 2x2 block M = [a b; b c], with |eigenvalues|
// floored at 1e-3 of the largest when M is not positive definite.
__device__ __forceinline__ void prec2x2(double a, double b, double c, double q0, double q1,
                                        double& r0, double& r1) {
  const double tr = a + c, det = a * c - b * b;
  if (tr > 0.0 && det > 1e-6 * tr * tr) {
    r0 = (c * q0 - b * q1) / det;
    r1 = (a * q1 - b * q0) / det;
    return;
  }
  const double m = 0.5 * tr, dd = sqrt(0.25 * (a - c) * (a - c) + b * b);
  double l1 = m + dd, l2 = m - dd;
  double vx, vy;
  if (fabs(b) > 0.0) {
    vx = b;
    vy = l1 - a;
  } else if (a >= c) {
    vx = 1.0;
    vy = 0.0;
  } else {
    vx = 0.0;
    vy = 1.0;
  }
  const double nv = sqrt(vx * vx + vy * vy);
  const double lmax = fmax(fabs(l1), fabs(l2));
  if (!(nv > 0.0) || !(lmax > 0.0)) {
    r0 = q0;
    r1 = q1;
    return;
  }
  vx /= nv;
  vy /= nv;
  l1 = fmax(fabs(l1), 1e-3 * lmax);
  l2 = fmax(fabs(l2), 1e-3 * lmax);
  const double p1 = vx * q0 + vy * q1, p2 = -vy * q0 + vx * q1;
  r0 = vx * (p1 / l1) - vy * (p2 / l2);
  r1 = vy * (p1 / l1) + vx * (p2 / l2);
}

// The same for an interior charge in (t, u): J^T B J with J = d(x, y)/d(t, u)
// (columns sigma sin 2t (cos u, sin u) and r (-sin u, cos u)) and B the
// charge's own Cartesian block.
__device__ void tu_prec(double sig, double t, double u, double a, double b, double c, double q0,
                        double q1, double& r0, double& r1) {
  double su, cu, st, ctt;
  sincos(u, &su, &cu);
  sincos(t, &st, &ctt);
  const double ft = sig * (2.0 * st * ctt), fu = sig * (st * st);
  const double jtx = ft * cu, jty = ft * su, jux = -fu * su, juy = fu * cu;
  const double btx = a * jtx + b * jty, bty = b * jtx + c * jty;
  const double bux = a * jux + b * juy, buy = b * jux + c * juy;
  prec2x2(jtx * btx + jty * bty, jtx * bux + jty * buy, jux * bux + juy * buy, q0, q1, r0, r1);
}

// Kind-dispatched pieces of the optimiser for active a (held[a]: 0 (x, y),
// 1 the angle on its circle, kHeldTU the (t, u) of Sec. II.D): the gradient
// in optimisation coordinates at z and at the trial, the position after the
// coordinate step al (d0, d1) from z (a (t, u) charge records its trial
// (t, u)), the preconditioner at z, and the length of a step's displacement.
template <bool TU>
__device__ __forceinline__ void cgrad_z(const RelaxDev& R, int a, double g0, double g1,
                                        double& c0, double& c1) {
  const int h = R.held[a];
  if (TU && h == kHeldTU) tu_grad(R.sigma, R.ct[a], R.cu[a], g0, g1, c0, c1);
  else coord_grad(h != 0, R.zx[a], R.zy[a], g0, g1, c0, c1);
}
template <bool TU>
__device__ __forceinline__ void cgrad_t(const RelaxDev& R, int a, double g0, double g1,
                                        double& c0, double& c1) {
  const int h = R.held[a];
  if (TU && h == kHeldTU) tu_grad(R.sigma, R.tct[a], R.tcu[a], g0, g1, c0, c1);
  else coord_grad(h != 0, R.tx[a], R.ty[a], g0, g1, c0, c1);
}
template <bool TU>
__device__ __forceinline__ void step_from_z(RelaxDev& R, int a, double d0, double d1, double al,
                                            double& nx, double& ny) {
  const int h = R.held[a];
  if (TU && h == kHeldTU) {
    const double t = R.ct[a] + al * d0, u = R.cu[a] + al * d1;
    R.tct[a] = t;
    R.tcu[a] = u;
    tu_position(R.sigma, t, u, nx, ny);
  } else {
    take_step(h != 0, R.zx[a], R.zy[a], d0, d1, al, nx, ny, R.pin[a], R.sigma);
  }
}
template <bool TU>
__device__ __forceinline__ void prec_z(const RelaxDev& R, int a, double q0, double q1, double& r0,
                                       double& r1) {
  const int h = R.held[a];
  if (TU && h == kHeldTU)
    tu_prec(R.sigma, R.ct[a], R.cu[a], R.kxx[a], R.kxy[a], R.kyy[a], q0, q1, r0, r1);
  else
    apply_prec(h != 0, R.zx[a], R.zy[a], R.gx[a], R.gy[a], R.kxx[a], R.kxy[a], R.kyy[a], q0, q1,
               r0, r1);
}
template <bool TU>
__device__ __forceinline__ double step_len(const RelaxDev& R, int a, double d0, double d1) {
  const int h = R.held[a];
  if (TU && h == kHeldTU) {
    double st, ctt;
    sincos(R.ct[a], &st, &ctt);
    const double lt = R.sigma * (2.0 * st * ctt) * d0, lu = R.sigma * (st * st) * d1;
    return sqrt(lt * lt + lu * lu);
  }
  return h ? fabs(d0) : sqrt(d0 * d0 + d1 * d1);
}

// Trial point of active a along the coordinate step (d0, d1) from z (held:
// rotation by the angle d0; free: translation, then the wall projection;
// (t, u): the position the stepped (t, u) gives), with the model's FP32
// coordinates of the trial on the mixed path.
template <bool TU>
__device__ __forceinline__ void set_trial(RelaxDev& R, const PState& s, int a, double d0,
                                          double d1) {
  R.dx[a] = d0;
  R.dy[a] = d1;
  double nx, ny;
  step_from_z<TU>(R, a, d0, d1, 1.0, nx, ny);
  R.tx[a] = nx;
  R.ty[a] = ny;
  if (R.a32x) {
    R.a32x[a] = (float)(nx - s.cx);
    R.a32y[a] = (float)(ny - s.cy);
  }
}

// A coordinate vector in Cartesian form: held charge d0 (-y, x), free (d0, d1).
__device__ __forceinline__ void to_cart(bool h, double px, double py, double d0, double d1,
                                        double& wx, double& wy) {
  wx = h ? -py * d0 : d0;
  wy = h ? px * d0 : d1;
}

// Start of a Newton step at z (truncated-Newton polish): preconditioned CG on
// H_t x = -g_c (g_c the coordinate gradient at z) from x = 0, with the
// block-Jacobi preconditioner of apply_prec.  The step ends when the
// residual's inf-norm falls below max(cg_eta |g_c|inf, gtol / 10).
__device__ void cg_start(RelaxDev& R, PState& s, int p, double gi, WgRed& red) {
  const int a0 = R.ptr[p], a1 = R.ptr[p + 1];
  double rz = 0.0, gm = 0.0;
  for (int a = a0 + threadIdx.x; a < a1; a += kUpd) {
    const bool h = R.held[a];
    const double px = R.zx[a], py = R.zy[a], g0 = R.gx[a], g1 = R.gy[a];
    double c0, c1, z0, z1;
    coord_grad(h, px, py, g0, g1, c0, c1);
    const double r0 = -c0, r1 = -c1;  // the residual of x = 0
    apply_prec(h, px, py, g0, g1, R.kxx[a], R.kxy[a], R.kyy[a], r0, r1, z0, z1);
    R.cgx[a] = 0.0;
    R.cgy[a] = 0.0;
    R.crx[a] = r0;
    R.cry[a] = r1;
    R.cdx[a] = z0;
    R.cdy[a] = z1;
    to_cart(h, px, py, z0, z1, R.cwx[a], R.cwy[a]);
    rz += r0 * z0 + r1 * z1;
    gm = fmax(gm, fmax(fabs(c0), fabs(c1)));
  }
  block_sum_max(rz, gm, red);
  s.rz = rz;
  s.cg_it = 0;
  s.phase = kPhaseCG;
  // forcing term: fixed (cg_eta > 0), or adaptive (Eisenstat-Walker's second
  // choice): 0.9 (g_k / g_{k-1})^2 from the reduced gradients at the starts
  // of this and the last Newton step, 0.1 for the first, kept above 0.9
  // eta_{k-1}^2 when that exceeds 0.1 and within [1e-8, 0.1]
  double eta = R.cg_eta;
  if (!(eta > 0.0)) {
    if (s.gnewt > 0.0) {
      const double q = gi / s.gnewt;
      eta = 0.9 * q * q;
      const double prev = 0.9 * s.eta * s.eta;
      if (prev > 0.1) eta = fmax(eta, prev);
      eta = fmin(0.1, fmax(eta, 1e-8));
    } else {
      eta = 0.1;
    }
  }
  s.eta = eta;
  s.gnewt = gi;
  s.cg_target = fmax(eta * gm, 0.1 * R.gtol);
}

// One CG iteration after k_cg_hvp wrote q = H_t d.  The Newton step ends --
// and its trial point is set -- when the residual meets the target, at the
// iteration cap, or when d has non-positive curvature (the step then follows
// the iterate x, a descent direction, or d itself at the first iteration).
// Its largest displacement is capped at step0, as for L-BFGS steps.
__device__ void cg_iteration(RelaxDev& R, PState& s, int p, WgRed& red) {
  const int a0 = R.ptr[p], a1 = R.ptr[p + 1];
  double dq = 0.0;
  for (int a = a0 + threadIdx.x; a < a1; a += kUpd) dq += R.cdx[a] * R.cqx[a] + R.cdy[a] * R.cqy[a];
  dq = block_sum(dq, red);
  int end = 0;  // 0: go on, 1: step along the iterate x, 2: along d
  if (!(dq > 0.0)) {
    end = s.cg_it == 0 ? 2 : 1;
  } else {
    const double al = s.rz / dq;
    double rz = 0.0, rm = 0.0;
    for (int a = a0 + threadIdx.x; a < a1; a += kUpd) {
      const double q0 = R.cqx[a], q1 = R.cqy[a];
      R.cgx[a] += al * R.cdx[a];
      R.cgy[a] += al * R.cdy[a];
      const double r0 = R.crx[a] - al * q0, r1 = R.cry[a] - al * q1;
      R.crx[a] = r0;
      R.cry[a] = r1;
      double z0, z1;
      apply_prec(R.held[a], R.zx[a], R.zy[a], R.gx[a], R.gy[a], R.kxx[a], R.kxy[a], R.kyy[a], r0,
                 r1, z0, z1);
      R.cqx[a] = z0;  // q is spent: it holds M^-1 r until d is updated
      R.cqy[a] = z1;
      rz += r0 * z0 + r1 * z1;
      rm = fmax(rm, fmax(fabs(r0), fabs(r1)));
    }
    block_sum_max(rz, rm, red);
    s.cg_it++;
    if (rm <= s.cg_target || s.cg_it >= R.max_cg || !(rz > 0.0)) {
      end = 1;
    } else {
      const double be = rz / s.rz;
      s.rz = rz;
      for (int a = a0 + threadIdx.x; a < a1; a += kUpd) {
        const double d0 = R.cqx[a] + be * R.cdx[a], d1 = R.cqy[a] + be * R.cdy[a];
        R.cdx[a] = d0;
        R.cdy[a] = d1;
        to_cart(R.held[a], R.zx[a], R.zy[a], d0, d1, R.cwx[a], R.cwy[a]);
      }
    }
  }
  if (end) {
    double dm = 0.0;
    for (int a = a0 + threadIdx.x; a < a1; a += kUpd) {
      const double d0 = end == 1 ? R.cgx[a] : R.cdx[a], d1 = end == 1 ? R.cgy[a] : R.cdy[a];
      dm = fmax(dm, R.held[a] ? fabs(d0) : sqrt(d0 * d0 + d1 * d1));
    }
    dm = block_max(dm, red);
    const double sc = dm > R.step0 ? R.step0 / dm : 1.0;
    for (int a = a0 + threadIdx.x; a < a1; a += kUpd) {
      const double d0 = end == 1 ? R.cgx[a] : R.cdx[a], d1 = end == 1 ? R.cgy[a] : R.cdy[a];
      set_trial<false>(R, s, a, d0 * sc, d1 * sc);
    }
    s.cg_total += s.cg_it;
    s.phase = kPhaseStep;
    s.alpha = 1.0;
  }
}

// HT: storage type of the L-BFGS history (FP32 on the mixed path, where it
// halves the kernel's dominant memory traffic; FP64 on the plain path).  The
// recursion itself runs in FP64.  RJ: actives per thread held in registers.
template <class HT, bool TU, int RJ>
__global__ __launch_bounds__(kUpd) void k_update(RelaxDev R) {
  HT* const Sx = reinterpret_cast<HT*>(R.Sx);
  HT* const Sy = reinterpret_cast<HT*>(R.Sy);
  HT* const Yx = reinterpret_cast<HT*>(R.Yx);
  HT* const Yy = reinterpret_cast<HT*>(R.Yy);
  WG_RED_LDS(red);
  __shared__ double s_alf[kMaxMem];
  __shared__ double s_rho[kMaxMem];  // rho of the patch: the recursion reads it from LDS
  __shared__ double s_part[8 * kRows];
  __shared__ int s_flag;
  const int p = blockIdx.x, t = threadIdx.x;
  PState s = R.st[p];
  if (s.status != kRunning) return;
  if (s.phase == kPhaseCG) {
    cg_iteration(R, s, p, red);
    if (t == 0) R.st[p] = s;
    return;
  }
  s.evals++;
  const bool was_init = s.init;
  const bool k_fresh = !s.skip_k;  // this evaluation took the Hessian blocks
  const int a0 = R.ptr[p], a1 = R.ptr[p + 1];
  const int m = R.m;
  double* rho = R.rho + (size_t)p * m;
  if (t < m) s_rho[t] = rho[t];  // before the first barrier below
  const double tol = R.ptol ? R.ptol[p] : R.tol;  // loaded ahead of the barriers

  // energy of the trial (fixed-order block sum of per-active terms) and the
  // directional derivatives along the step in optimisation coordinates:
  // pred = grad(z).s, dpt = grad(zt).s; a held charge's step is the angle
  // alpha*d (its Cartesian displacement has a second-order radial part that
  // the large wall reaction would weigh), a free charge's is zt - z
  // (every value is loaded before the held test selects the formula, so
  // the loads of an active go out together)
  double e = 0.0, pr = 0.0, pt = 0.0;
  for (int a = a0 + t; a < a1; a += kUpd) {
    e += R.eterm[a];
    if (s.init) continue;
    const int h = R.held[a];
    const double gx = R.gx[a], gy = R.gy[a], hgx = R.hgx[a], hgy = R.hgy[a];
    const double zx = R.zx[a], zy = R.zy[a], tx = R.tx[a], ty = R.ty[a], dx = R.dx[a];
    const double st = s.alpha * dx;
    if (TU && h == kHeldTU) {  // the step in (t, u) is alpha d
      double c0, c1, n0, n1;
      cgrad_z<TU>(R, a, gx, gy, c0, c1);
      cgrad_t<TU>(R, a, hgx, hgy, n0, n1);
      const double su = s.alpha * R.dy[a];
      pr += c0 * st + c1 * su;
      pt += n0 * st + n1 * su;
      continue;
    }
    const double ddx = tx - zx, ddy = ty - zy;
    const double prh = (-gx * zy + gy * zx) * st, pth = (-hgx * ty + hgy * tx) * st;
    const double prf = gx * ddx + gy * ddy, ptf = hgx * ddx + hgy * ddy;
    pr += h ? prh : prf;
    pt += h ? pth : ptf;
  }
  block_sum3(e, pr, pt, red);
  const double Et = e;
  bool accept;
  bool nonfinite = !isfinite(Et);
  double shrink = 0.5;  // backtracking factor when the trial is rejected
  if (s.init) {
    accept = true;
  } else {
    const double pred = pr, dpt = pt;
    const double dE = Et - s.E;
    const double noise = (s.use32 ? 1e-9 : R.noise_rel) * fabs(s.E);
    if (fabs(dE) > noise) {
      accept = dE <= R.c1 * pred;  // Armijo
    } else {
      // energy change below the evaluation's rounding: derivative-only test
      // (curvature condition) and a secant step back on an overshoot
      accept = pred < 0.0 && dpt <= 0.9 * fabs(pred);
      if (pred < 0.0 && dpt > pred) shrink = fmin(0.5, fmax(0.1, pred / (pred - dpt)));
    }
  }
  if (nonfinite) {
    if (t == 0) {
      s.status = kNonFinite;
      R.st[p] = s;
      atomicSub(R.running, 1);
    }
    return;
  }

  if (accept) {
    // secant pair in the coordinates of the step just taken (held flags at z)
    if (!s.init) {
      double syp = 0.0, ssp = 0.0, yyp = 0.0;
      const int k = s.head;
      for (int a = a0 + t; a < a1; a += kUpd) {
        const int hk = R.held[a];
        const bool h = hk != 0;
        const double zx = R.zx[a], zy = R.zy[a], tx = R.tx[a], ty = R.ty[a], dx = R.dx[a];
        const double gx = R.gx[a], gy = R.gy[a], hgx = R.hgx[a], hgy = R.hgy[a];
        double c0, c1, n0, n1;
        // the step in coordinates: the angle step of a held charge, alpha d
        // in (t, u), the Cartesian displacement of a free charge
        const double s0 = h ? s.alpha * dx : tx - zx;
        const double s1 = TU && hk == kHeldTU ? s.alpha * R.dy[a] : (h ? 0.0 : ty - zy);
        cgrad_z<TU>(R, a, gx, gy, c0, c1);
        cgrad_t<TU>(R, a, hgx, hgy, n0, n1);
        // the pair as stored (rounded to HT), so that rho matches the vectors
        const HT hs0 = (HT)s0, hs1 = (HT)s1, hy0 = (HT)(n0 - c0), hy1 = (HT)(n1 - c1);
        const size_t q = (size_t)k * R.ntot + a;
        Sx[q] = hs0;
        Sy[q] = hs1;
        Yx[q] = hy0;
        Yy[q] = hy1;
        const double u0 = hs0, u1 = hs1;
        const double y0 = hy0, y1 = hy1;
        syp += u0 * y0 + u1 * y1;
        ssp += u0 * u0 + u1 * u1;
        yyp += y0 * y0 + y1 * y1;
      }
      block_sum3(syp, ssp, yyp, red);
      const double sy = syp, ss = ssp, yy = yyp;
      if (sy > 1e-12 * sqrt(ss * yy)) {
        if (t == 0) rho[k] = s_rho[k] = 1.0 / sy;
        s.head = (s.head + 1) % m;
        if (s.mem < m) s.mem++;
      } else if (s.mem == m) {
        s.mem = m - 1;  // slot k held the oldest pair, now overwritten by the rejected one
      }
    }
    // move to the trial, update the held set
    if (t == 0) s_flag = 0;
    __syncthreads();
    double gm = 0.0, dz = 0.0;  // reduced gradient; mixed path: displacement from the expansion point
    for (int a = a0 + t; a < a1; a += kUpd) {
      const double px = R.tx[a], py = R.ty[a], g0 = R.hgx[a], g1 = R.hgy[a];
      if (R.zrx) {
        const double ex = px - R.zrx[a], ey = py - R.zry[a];
        dz = fmax(dz, ex * ex + ey * ey);
      }
      R.zx[a] = px;
      R.zy[a] = py;
      R.gx[a] = g0;
      R.gy[a] = g1;
      R.kxx[a] = R.hkxx[a];
      R.kxy[a] = R.hkxy[a];
      R.kyy[a] = R.hkyy[a];
      const int pin = R.pin[a];
      const int hk = R.held[a];
      if (TU && hk == kHeldTU) {  // (t, u) charges keep their coordinates: no wall to hold them
        R.ct[a] = R.tct[a];
        R.cu[a] = R.tcu[a];
      }
      const int h = TU && hk == kHeldTU ? kHeldTU : held_rule(px, py, g0, g1, pin, R.sigma);
      if (h != hk) {
        R.held[a] = h;
        if (!s.init) {
          // the charge's history into its new coordinates, keeping the
          // tangential part of every pair: angle step s_t = t.s / r and
          // angle-gradient change y_t = r t.y (t the unit tangent), and back
          // to the Cartesian vectors s_t r t and (y_t / r) t on release
          const double r = sqrt(px * px + py * py);
          const double ux = -py / r, uy = px / r;
          for (int k = 0; k < m; ++k) {
            const size_t q = (size_t)k * R.ntot + a;
            const double s0 = Sx[q], s1 = Sy[q], y0 = Yx[q], y1 = Yy[q];
            if (h) {
              Sx[q] = (HT)((ux * s0 + uy * s1) / r);
              Yx[q] = (HT)(r * (ux * y0 + uy * y1));
              Sy[q] = Yy[q] = (HT)0;
            } else {
              Sx[q] = (HT)(r * s0 * ux);
              Sy[q] = (HT)(r * s0 * uy);
              Yx[q] = (HT)(y0 / r * ux);
              Yy[q] = (HT)(y0 / r * uy);
            }
          }
        }
        s_flag = 1;
      }
      gm = fmax(gm, reduced_inf(px, py, g0, g1, pin, R.sigma));
    }
    block_max2(gm, dz, red);
    const double gi = gm;
    __syncthreads();
    if (s_flag && s.mem > 0) {
      // entries were converted: every rho again, eight pairs per pass over the
      // actives and one many-value sum (thread j < 8 finishes pair 8h + j)
      const int M = s.mem;
      for (int h = 0; 8 * h < M; ++h) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = 0.0;
        for (int a = a0 + t; a < a1; a += kUpd) {
          int sk = s.head - 8 * h;
          if (sk <= 0) sk += m;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            sk = sk == 0 ? m - 1 : sk - 1;
            if (8 * h + j < M) {
              const size_t q = (size_t)sk * R.ntot + a;
              v[j] += (double)Sx[q] * (double)Yx[q] + (double)Sy[q] * (double)Yy[q];
            }
          }
        }
        rows_sum<8>(v, s_part);
        const int jt = 8 * h + t;
        if (t < 8 && jt < M) {
          const double sy = rows_total(s_part, t);
          const int kk = s.head - 1 - jt < 0 ? s.head - 1 - jt + m : s.head - 1 - jt;
          rho[kk] = s_rho[kk] = sy > 0.0 ? 1.0 / sy : 0.0;
        }
        __syncthreads();  // s_part is written again by the next half
      }
    }
    s.E = Et;
    s.gi = gi;
    if (!s.init) {
      s.it++;
      s.total_it++;
      if (s.newton) s.newton_steps++;
    }
    s.init = 0;
    // mixed path: the model is trusted within trust of its expansion point
    // (beyond the halo the exterior is a quadratic, blind to charges an
    // active could run into); a patch that leaves that radius ends the round
    // and is re-expanded exactly where it stands
    const bool left = R.zrx && dz > R.trust * R.trust;
    if (gi <= tol || s.it >= R.max_iter || left) {
      if (t == 0) {
        s.status = (gi <= tol || left) ? kConverged : kIterCap;
        R.st[p] = s;
        atomicSub(R.running, 1);
      }
      return;
    }
    // truncated-Newton polish: the plain path enters Newton mode below
    // newton_tol (the mixed path's round check decides there)
    // (the Newton product needs the exact blocks at z: with stale ones the
    // patch takes one more L-BFGS step and enters with fresh ones)
    if (R.polish && !R.fgx && !s.newton_off && gi <= R.newton_tol && k_fresh) s.newton = 1;
    if (!R.fgx) {
      // the plain path takes each active's Hessian block (the preconditioner)
      // every kBlockEvery-th iteration, from close to the Newton switch on,
      // and in Newton mode, where the product needs it at every point
      const bool near_newton = R.polish && !s.newton_off && gi <= kBlockNear * R.newton_tol;
      s.skip_k = !(s.newton || near_newton || s.it % kBlockEvery == 0);
    }
    if (s.newton) {
      if (R.fgx && !was_init) {
        // mixed path: one Newton step per expansion of the far field; the
        // next round re-expands at the new point and tests it exactly
        if (t == 0) {
          s.status = kConverged;
          R.st[p] = s;
          atomicSub(R.running, 1);
        }
        return;
      }
      // mixed path, where each Newton step costs a round: a second Newton
      // step that fails to halve the reduced gradient ends Newton mode for
      // the patch (e.g. an indefinite Hessian or a changing held set), L-BFGS
      // from here to the end.  The plain path's steps cost one exact
      // evaluation each, like an L-BFGS iteration, so it keeps them.
      if (R.fgx && s.gnewt > 0.0 && gi > 0.5 * s.gnewt && ++s.nfail >= 2) {
        s.newton = 0;
        s.newton_off = 1;
      } else {
        cg_start(R, s, p, gi, red);
        if (t == 0) R.st[p] = s;
        return;
      }
    }
  } else {
    s.alpha *= shrink;
    if (s.newton && s.alpha < 1e-3) {
      // the Newton step failed its line search: an L-BFGS direction from z
      // (the history is kept), Newton again at the next check
      s.newton = 0;
    } else if (s.alpha >= 1e-10) {
      for (int a = a0 + t; a < a1; a += kUpd) {
        double nx, ny;
        step_from_z<TU>(R, a, R.dx[a], R.dy[a], s.alpha, nx, ny);
        R.tx[a] = nx;
        R.ty[a] = ny;
        if (R.a32x) {  // the model's FP32 coordinates of the trial
          R.a32x[a] = (float)(nx - s.cx);
          R.a32y[a] = (float)(ny - s.cy);
        }
      }
      if (t == 0) R.st[p] = s;
      return;
    } else {
      if (s.mem == 0) {
        if (t == 0) {
          s.status = kLineSearchFail;
          R.st[p] = s;
          atomicSub(R.running, 1);
        }
        return;
      }
      s.mem = 0;  // restart from steepest descent
      s.head = 0;
    }
  }

  // new direction: two-loop recursion on the coordinate gradient.  A
  // thread's first RJ actives (a0 + t + j kUpd) keep the vector in
  // registers; any further ones (patches above RJ * kUpd actives) keep it
  // in R.dx, R.dy, touched only by their own thread, inside the same steps.
  // Each thread sums its actives in increasing order, then the workgroup sum.
  __syncthreads();
  const int tail0 = a0 + t + RJ * kUpd;
  double dxr[RJ], dyr[RJ];  // the direction of the register-held elements
  {
    double qx[RJ], qy[RJ];
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      const int a = a0 + t + j * kUpd;
      qx[j] = qy[j] = 0.0;
      if (a < a1) cgrad_z<TU>(R, a, R.gx[a], R.gy[a], qx[j], qy[j]);
    }
    for (int a = tail0; a < a1; a += kUpd) {
      double c0, c1;
      cgrad_z<TU>(R, a, R.gx[a], R.gy[a], c0, c1);
      R.dx[a] = c0;
      R.dy[a] = c1;
    }
    // FP32 history: pair k + 1 is loaded while pair k is reduced (FP64
    // history has no registers to spare for it)
    constexpr bool kPre = sizeof(HT) == 4;
    HT ux[RJ], uy[RJ], wx[RJ], wy[RJ];
    auto load_pair = [&](int k, HT* u0, HT* u1, HT* w0, HT* w1) {
      const bool kin = k >= 0 && k < s.mem;  // pairs outside the memory read as zero
      const int sk = s.head - 1 - (kin ? k : 0);
      const size_t base = (size_t)(sk < 0 ? sk + m : sk) * R.ntot;
#pragma unroll
      for (int j = 0; j < RJ; ++j) {
        const int a = a0 + t + j * kUpd;
        const bool ok = kin && a < a1;
        const size_t q = base + (size_t)min(a, a1 - 1);
        const HT x0 = Sx[q], x1 = Sy[q], x2 = Yx[q], x3 = Yy[q];
        u0[j] = ok ? x0 : (HT)0;
        u1[j] = ok ? x1 : (HT)0;
        w0[j] = ok ? x2 : (HT)0;
        w1[j] = ok ? x3 : (HT)0;
      }
    };
    // FP32 history: step k reduces pair k while pair k + 1 loads.  Two steps
    // per loop trip, with the buffers' roles swapped, so no register copy
    // waits on a load in flight.
    // Raw loads at clamped, in-patch addresses (stored, finite values): no
    // branch or select stands between a load and its use.  A pair outside
    // the memory is loaded but never used; the elements past the patch end
    // meet q = 0 in the sums and are masked (mk = 0) in the updates, so q
    // stays 0 there.
    auto load_vec = [&](const HT* A0, const HT* A1, int k, HT* v0, HT* v1) {
      const bool kin = k >= 0 && k < s.mem;
      const int sk = s.head - 1 - (kin ? k : 0);
      const size_t base = (size_t)(sk < 0 ? sk + m : sk) * R.ntot;
#pragma unroll
      for (int j = 0; j < RJ; ++j) {
        const size_t q = base + (size_t)min(a0 + t + j * kUpd, a1 - 1);
        v0[j] = A0[q];
        v1[j] = A1[q];
      }
    };
    double mk[RJ];
#pragma unroll
    for (int j = 0; j < RJ; ++j) mk[j] = a0 + t + j * kUpd < a1 ? 1.0 : 0.0;
    if constexpr (kPre) {
      HT a0s[RJ], a1s[RJ], a0y[RJ], a1y[RJ];
      HT b0s[RJ], b1s[RJ], b0y[RJ], b1y[RJ];
      auto step1 = [&](int k, HT* c0s, HT* c1s, HT* c0y, HT* c1y, HT* n0s, HT* n1s, HT* n0y,
                       HT* n1y) {
        const int kk = s.head - 1 - k < 0 ? s.head - 1 - k + m : s.head - 1 - k;
        const size_t base = (size_t)kk * R.ntot;
        load_vec(Sx, Sy, k + 1, n0s, n1s);
        load_vec(Yx, Yy, k + 1, n0y, n1y);
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < RJ; ++j) v += (double)c0s[j] * qx[j] + (double)c1s[j] * qy[j];
        for (int a = tail0; a < a1; a += kUpd)
          v += (double)Sx[base + a] * R.dx[a] + (double)Sy[base + a] * R.dy[a];
        const double rk = s_rho[kk];  // read ahead of the reduction's barrier
        const double al = rk * block_sum(v, red);
        if (t == 0) s_alf[kk] = al;
#pragma unroll
        for (int j = 0; j < RJ; ++j) {
          qx[j] -= al * (mk[j] * (double)c0y[j]);
          qy[j] -= al * (mk[j] * (double)c1y[j]);
        }
        for (int a = tail0; a < a1; a += kUpd) {
          R.dx[a] -= al * (double)Yx[base + a];
          R.dy[a] -= al * (double)Yy[base + a];
        }
      };
      load_vec(Sx, Sy, 0, a0s, a1s);
      load_vec(Yx, Yy, 0, a0y, a1y);
      for (int k = 0; k < s.mem; k += 2) {
        step1(k, a0s, a1s, a0y, a1y, b0s, b1s, b0y, b1y);
        if (k + 1 < s.mem) step1(k + 1, b0s, b1s, b0y, b1y, a0s, a1s, a0y, a1y);
      }
    } else {
      if (kPre) load_pair(0, ux, uy, wx, wy);
      for (int k = 0; k < s.mem; ++k) {
        const int kk = s.head - 1 - k < 0 ? s.head - 1 - k + m : s.head - 1 - k;
        const size_t base = (size_t)kk * R.ntot;
        HT nux[RJ], nuy[RJ], nwx[RJ], nwy[RJ];
        if (kPre)
          load_pair(k + 1, nux, nuy, nwx, nwy);
        else
          load_pair(k, ux, uy, wx, wy);
        double v = 0.0;
  #pragma unroll
        for (int j = 0; j < RJ; ++j) v += (double)ux[j] * qx[j] + (double)uy[j] * qy[j];
        for (int a = tail0; a < a1; a += kUpd)
          v += (double)Sx[base + a] * R.dx[a] + (double)Sy[base + a] * R.dy[a];
        const double rk = s_rho[kk];  // read ahead of the reduction's barrier
        const double al = rk * block_sum(v, red);
        if (t == 0) s_alf[kk] = al;
  #pragma unroll
        for (int j = 0; j < RJ; ++j) {
          qx[j] -= al * (double)wx[j];
          qy[j] -= al * (double)wy[j];
          if (kPre) {
            ux[j] = nux[j];
            uy[j] = nuy[j];
            wx[j] = nwx[j];
            wy[j] = nwy[j];
          }
        }
        for (int a = tail0; a < a1; a += kUpd) {
          R.dx[a] -= al * (double)Yx[base + a];
          R.dy[a] -= al * (double)Yy[base + a];
        }
      }
    }
    // the preconditioner, in registers for the register-held elements and
    // in memory for the tail
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      const int a = a0 + t + j * kUpd;
      if (a < a1) {
        double r0, r1;
        prec_z<TU>(R, a, qx[j], qy[j], r0, r1);
        qx[j] = r0;
        qy[j] = r1;
      }
    }
    for (int a = tail0; a < a1; a += kUpd) {
      double r0, r1;
      prec_z<TU>(R, a, R.dx[a], R.dy[a], r0, r1);
      R.dx[a] = r0;
      R.dy[a] = r1;
    }
    if constexpr (kPre) {
      HT a0s[RJ], a1s[RJ], a0y[RJ], a1y[RJ];
      HT b0s[RJ], b1s[RJ], b0y[RJ], b1y[RJ];
      auto step2 = [&](int k, HT* c0s, HT* c1s, HT* c0y, HT* c1y, HT* n0s, HT* n1s, HT* n0y,
                       HT* n1y) {
        const int kk = s.head - 1 - k < 0 ? s.head - 1 - k + m : s.head - 1 - k;
        const size_t base = (size_t)kk * R.ntot;
        load_vec(Sx, Sy, k - 1, n0s, n1s);
        load_vec(Yx, Yy, k - 1, n0y, n1y);
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < RJ; ++j) v += (double)c0y[j] * qx[j] + (double)c1y[j] * qy[j];
        for (int a = tail0; a < a1; a += kUpd)
          v += (double)Yx[base + a] * R.dx[a] + (double)Yy[base + a] * R.dy[a];
        const double rk = s_rho[kk];
        const double be = rk * block_sum(v, red);
        const double coef = s_alf[kk] - be;
#pragma unroll
        for (int j = 0; j < RJ; ++j) {
          qx[j] += coef * (mk[j] * (double)c0s[j]);
          qy[j] += coef * (mk[j] * (double)c1s[j]);
        }
        for (int a = tail0; a < a1; a += kUpd) {
          R.dx[a] += coef * (double)Sx[base + a];
          R.dy[a] += coef * (double)Sy[base + a];
        }
      };
      load_vec(Sx, Sy, s.mem - 1, a0s, a1s);
      load_vec(Yx, Yy, s.mem - 1, a0y, a1y);
      for (int k = s.mem - 1; k >= 0; k -= 2) {
        step2(k, a0s, a1s, a0y, a1y, b0s, b1s, b0y, b1y);
        if (k - 1 >= 0) step2(k - 1, b0s, b1s, b0y, b1y, a0s, a1s, a0y, a1y);
      }
    } else {
      if (kPre) load_pair(s.mem - 1, ux, uy, wx, wy);
      for (int k = s.mem - 1; k >= 0; --k) {
        const int kk = s.head - 1 - k < 0 ? s.head - 1 - k + m : s.head - 1 - k;
        const size_t base = (size_t)kk * R.ntot;
        HT nux[RJ], nuy[RJ], nwx[RJ], nwy[RJ];
        if (kPre)
          load_pair(k - 1, nux, nuy, nwx, nwy);
        else
          load_pair(k, ux, uy, wx, wy);
        double v = 0.0;
  #pragma unroll
        for (int j = 0; j < RJ; ++j) v += (double)wx[j] * qx[j] + (double)wy[j] * qy[j];
        for (int a = tail0; a < a1; a += kUpd)
          v += (double)Yx[base + a] * R.dx[a] + (double)Yy[base + a] * R.dy[a];
        const double rk = s_rho[kk];
        const double be = rk * block_sum(v, red);
        const double coef = s_alf[kk] - be;
  #pragma unroll
        for (int j = 0; j < RJ; ++j) {
          qx[j] += coef * (double)ux[j];
          qy[j] += coef * (double)uy[j];
          if (kPre) {
            ux[j] = nux[j];
            uy[j] = nuy[j];
            wx[j] = nwx[j];
            wy[j] = nwy[j];
          }
        }
        for (int a = tail0; a < a1; a += kUpd) {
          R.dx[a] += coef * (double)Sx[base + a];
          R.dy[a] += coef * (double)Sy[base + a];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      dxr[j] = qx[j];
      dyr[j] = qy[j];
    }
  }
  // d = -H g; fall back to scaled steepest descent if not a descent direction
  // (the step length bound dm is taken in the same pass; the rare steepest
  // descent fallback takes it again).  Register-held elements first, then
  // the tail: the actives in increasing order, as everywhere.
  double dg = 0.0, dm = 0.0;
#pragma unroll
  for (int j = 0; j < RJ; ++j) {
    const int a = a0 + t + j * kUpd;
    if (a < a1) {
      double c0, c1;
      cgrad_z<TU>(R, a, R.gx[a], R.gy[a], c0, c1);
      const double d0 = -dxr[j], d1 = -dyr[j];
      dxr[j] = d0;
      dyr[j] = d1;
      dg += d0 * c0 + d1 * c1;
      dm = fmax(dm, step_len<TU>(R, a, d0, d1));
    }
  }
  for (int a = tail0; a < a1; a += kUpd) {
    double c0, c1;
    cgrad_z<TU>(R, a, R.gx[a], R.gy[a], c0, c1);
    const double d0 = -R.dx[a], d1 = -R.dy[a];
    R.dx[a] = d0;
    R.dy[a] = d1;
    dg += d0 * c0 + d1 * c1;
    dm = fmax(dm, step_len<TU>(R, a, d0, d1));
  }
  block_sum_max(dg, dm, red);
  const bool steep = !(dg < 0.0);
  if (steep) {
    dm = 0.0;
    for (int a = a0 + t; a < a1; a += kUpd) {
      double c0, c1, r0, r1;
      cgrad_z<TU>(R, a, R.gx[a], R.gy[a], c0, c1);
      prec_z<TU>(R, a, c0, c1, r0, r1);
      R.dx[a] = -r0;
      R.dy[a] = -r1;
      dm = fmax(dm, step_len<TU>(R, a, r0, r1));
    }
    dm = block_max(dm, red);
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      const int a = a0 + t + j * kUpd;
      if (a < a1) {
        dxr[j] = R.dx[a];
        dyr[j] = R.dy[a];
      }
    }
  }
  const double sc = dm > R.step0 ? R.step0 / dm : 1.0;
  s.alpha = 1.0;
#pragma unroll
  for (int j = 0; j < RJ; ++j) {
    const int a = a0 + t + j * kUpd;
    if (a < a1) set_trial<TU>(R, s, a, dxr[j] * sc, dyr[j] * sc);
  }
  for (int a = tail0; a < a1; a += kUpd) set_trial<TU>(R, s, a, R.dx[a] * sc, R.dy[a] * sc);
  if (t == 0) R.st[p] = s;
}

// Restart every patch not yet done on a new evaluator: the next evaluation
// is at z itself (no secant pair from it).  keep_mem keeps the L-BFGS
// history (the near-field curvature it holds is unchanged by a re-expansion
// of the far field).
__global__ void k_restart(RelaxDev R, int keep_mem) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= R.P) return;
  PState s = R.st[p];
  if (s.status == kConverged || s.status == kIterCap || s.status == kLineSearchFail)
    s.status = kRunning;
  s.init = 1;
  s.it = 0;
  s.phase = kPhaseStep;
  if (!keep_mem) {
    s.mem = 0;
    s.head = 0;
  }
  s.alpha = 1.0;
  R.st[p] = s;
}

__global__ void k_copy_z_to_t(RelaxDev R) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= R.ntot) return;
  R.tx[a] = R.zx[a];
  R.ty[a] = R.zy[a];
  R.tct[a] = R.ct[a];  // the trial's (t, u) with it (used by (t, u) charges only)
  R.tcu[a] = R.cu[a];
}

// Ends the round of every patch still running (its stage continues after the
// next re-expansion, from the point it has reached).
__global__ void k_cut(RelaxDev R) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < R.P && R.st[p].status == kRunning) R.st[p].status = kIterCap;
}

__global__ void k_count_running(RelaxDev R) {
  __shared__ int c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  for (int p = threadIdx.x; p < R.P; p += blockDim.x)
    if (R.st[p].status == kRunning) atomicAdd(&c, 1);
  __syncthreads();
  if (threadIdx.x == 0) *R.running = c;
}

// After a re-expansion at z and a model evaluation there, (hgx, hgy) is the
// exact gradient at z: a patch whose exact reduced gradient meets the
// tolerance is done.  Sets the stage tolerance of the others to a fraction
// of their current exact gradient.
__global__ __launch_bounds__(kUpd) void k_check(RelaxDev R, double tol, double frac,
                                                double tol32, double* __restrict__ ptol) {
  WG_RED_LDS(red);
  const int p = blockIdx.x, t = threadIdx.x;
  PState s = R.st[p];
  if (s.status == kNonFinite || s.status == kDone) return;
  const int a0 = R.ptr[p], a1 = R.ptr[p + 1];
  double gm = 0.0, dh = 0.0;  // reduced gradient; squared drift since the halo was built
  for (int a = a0 + t; a < a1; a += kUpd) {
    gm = fmax(gm, reduced_inf(R.zx[a], R.zy[a], R.hgx[a], R.hgy[a], R.pin[a], R.sigma));
    const double ex = R.zx[a] - R.zhx[a], ey = R.zy[a] - R.zhy[a];
    dh = fmax(dh, ex * ex + ey * ey);
  }
  block_max2(gm, dh, red);
  const double gi = gm;
  if (t == 0) {
    // (t, u) coordinates: a round on the FP32 model that failed to bring the
    // exact gradient below 0.9 of the last check's has hit the model's
    // rounding -- a charge pushed against its wall approaches it as
    // sigma sin^2 t, and its last displacement to the wall (which the exact
    // test needs within 1e-14) is below FP32 resolution: the patch's model
    // uses FP64 pairs from here on.  (In (x, y) such a charge is held on the
    // wall and a stalled round only means a slow one.)
    if (R.tu && s.use32 && s.exact_evals > 0 && gi > 0.9 * s.gexact) s.force64 = 1;
    s.gexact = gi;
    s.exact_evals++;
    s.gi = gi;
    if (gi <= tol) s.status = kDone;
    if (s.status != kDone && dh > R.rebuild_d2) atomicOr(&R.running[1], 1);
    ptol[p] = fmax(0.1 * tol, frac * gi);
    s.use32 = gi > tol32 && !s.force64;
    s.newton = R.polish && !s.use32 && !s.newton_off && gi <= R.newton_tol;
    R.st[p] = s;
  }
}

// Final per-patch outputs after an exact evaluation at z (gradient in hg,
// energy terms in eterm): positions, E_sub, exact reduced gradient, counters
// and status (0 converged, 1 iteration cap, 2 line search failed, 3 non-finite).
__global__ __launch_bounds__(kUpd) void k_finish(RelaxDev R, double tol, int exact_evals_all,
                                                 double* __restrict__ xo, double* __restrict__ yo,
                                                 double* __restrict__ esub,
                                                 double* __restrict__ gtan,
                                                 int32_t* __restrict__ iters,
                                                 int32_t* __restrict__ status) {
  WG_RED_LDS(red);
  const int p = blockIdx.x, t = threadIdx.x;
  const PState s = R.st[p];
  const int a0 = R.ptr[p], a1 = R.ptr[p + 1];
  double e = 0.0, gm = 0.0;
  for (int a = a0 + t; a < a1; a += kUpd) {
    e += R.eterm[a];
    gm = fmax(gm, reduced_inf(R.zx[a], R.zy[a], R.hgx[a], R.hgy[a], R.pin[a], R.sigma));
    if (xo) {
      xo[a] = R.zx[a];
      yo[a] = R.zy[a];
    }
  }
  const double E = block_sum(e, red);
  const double gi = block_max(gm, red);
  if (t == 0) {
    if (esub) esub[p] = E;
    if (gtan) gtan[p] = gi;
    if (iters) {
      iters[2 * p] = s.total_it;
      iters[2 * p + 1] = exact_evals_all ? s.evals + 1 : s.exact_evals + 1;
    }
    if (status)
      status[p] = !(gi <= tol) ? (s.status == kLineSearchFail ? 2 : s.status == kNonFinite ? 3 : 1)
                               : (isfinite(E) ? 0 : 3);
    if (R.pstats) {
      R.pstats[2 * p] = s.newton_steps;
      R.pstats[2 * p + 1] = s.cg_total;
    }
  }
}

__global__ __launch_bounds__(kUpd) void k_finish_delta(RelaxDev R, double* __restrict__ dE) {
  WG_RED_LDS(red);
  const int p = blockIdx.x, t = threadIdx.x;
  const int a0 = R.ptr[p], a1 = R.ptr[p + 1];
  double e = 0.0;
  for (int a = a0 + t; a < a1; a += kUpd) e += R.eterm[a];
  const double d = block_sum(e, red);
  if (t == 0 && dE) dE[p] = d;
}

// ------------------------------------------------------------------ planning --
struct RPlan {
  int n, P, nbN, m, ntot, nblk, splits, jb, hcap;
  int running;  // patches running at the last read-back (host copy)
  // schedule (relax_autotune chooses among these): lock-step rounds per graph
  // replay (the running count is read back between replays), and the
  // running-block count below which the model evaluation takes 16 waves per
  // block instead of 8
  int graph_rounds = 8;
  int64_t wide_blocks = 512;
  bool use_graphs = true;  // rounds replayed from HIP graphs (else launched one by one)
  int regj = kRegJ;        // actives per thread in registers in the update (kRegJ or kRegJWide)
  size_t total;
  RelaxDev D;
  int32_t* hcount;  // [P]
  int32_t* blk_host_dummy;
  double* geom;      // [3P] mixed path: proposed patch centre and radius of a halo rebuild
};

// The exact passes split the N charges into j ranges so that a pass launches
// about kExactWaves waves (one per 64-active block and range): at 4 waves per
// SIMD that is 16 rounds of the chip, enough to even out blocks of unequal
// patches.  A quarter of it left a 64-patch FP64 batch 47% slower per pass.
constexpr int kExactWaves = 65536;

static bool rplan(int64_t n64, int P, int64_t ntot64, int precision, int m, char* base, RPlan& R) {
  if (n64 < 2 || n64 > (1 << 26) || P < 1 || ntot64 < 1 || ntot64 > n64 * (int64_t)P) return false;
  if (precision != CD_FP64 && precision != CD_MIXED) return false;
  if (m < 1 || m > kMaxMem) return false;
  R.n = (int)n64;
  R.P = P;
  R.ntot = (int)ntot64;
  R.nbN = (R.n + 63) / 64;
  R.m = m;
  R.nblk = R.ntot / 64 + P;  // upper bound of the block table length
  int sp = (kExactWaves + R.nblk - 1) / R.nblk;
  sp = sp < 1 ? 1 : (sp > R.nbN ? R.nbN : sp);
  R.jb = (R.nbN + sp - 1) / sp;
  R.splits = (R.nbN + R.jb - 1) / R.jb;
  R.hcap = precision == CD_MIXED ? 6 * R.ntot + 4096 * P : 0;
  R.running = P;
  Carve cv;
  cv.base = base;
  RelaxDev& D = R.D;
  const size_t nt = R.ntot;
  // split partials hold nt * splits values; since splits <= ceil(kExactWaves /
  // nblk), nblk > nt / 64 and splits <= nbN, that is below both
  // kExactWaves * 64 + nt and nt * nbN, bounds that grow with nt, so the
  // workspace of a larger batch covers every smaller one (the greedy commit
  // sizes its scratch for the largest patch)
  const size_t pcap = std::min((size_t)kExactWaves * 64 + nt, nt * (size_t)R.nbN);
  D.pid = cv.take<int32_t>(nt);
  D.blk = cv.take<int2>(R.nblk);
  D.maskA = cv.take<uint64_t>((size_t)P * R.nbN);
  D.maskAH = cv.take<uint64_t>((size_t)P * R.nbN);
  D.z0x = cv.take<double>(nt);
  D.z0y = cv.take<double>(nt);
  D.zx = cv.take<double>(nt);
  D.zy = cv.take<double>(nt);
  D.tx = cv.take<double>(nt);
  D.ty = cv.take<double>(nt);
  D.gx = cv.take<double>(nt);
  D.gy = cv.take<double>(nt);
  D.hgx = cv.take<double>(nt);
  D.hgy = cv.take<double>(nt);
  D.kxx = cv.take<double>(nt);
  D.kxy = cv.take<double>(nt);
  D.kyy = cv.take<double>(nt);
  D.hkxx = cv.take<double>(nt);
  D.hkxy = cv.take<double>(nt);
  D.hkyy = cv.take<double>(nt);
  D.pkxx = cv.take<double>(pcap);
  D.pkxy = cv.take<double>(pcap);
  D.pkyy = cv.take<double>(pcap);
  D.dx = cv.take<double>(nt);
  D.dy = cv.take<double>(nt);
  D.Sx = cv.take<double>(nt * m);
  D.Sy = cv.take<double>(nt * m);
  D.Yx = cv.take<double>(nt * m);
  D.Yy = cv.take<double>(nt * m);
  D.rho = cv.take<double>((size_t)P * m);
  D.held = cv.take<int32_t>(nt);
  D.pin = cv.take<int32_t>(nt);
  D.eterm = cv.take<double>(nt);
  D.px = cv.take<double>(pcap);
  D.py = cv.take<double>(pcap);
  D.pe = cv.take<double>(pcap);
  D.st = cv.take<PState>(P);
  D.ptr_w = cv.take<int32_t>(P + 1);
  D.ptol = cv.take<double>(P);
  D.err = cv.take<int32_t>(1);
  D.running = cv.take<int32_t>(2);
  D.cgx = cv.take<double>(nt);
  D.cgy = cv.take<double>(nt);
  D.crx = cv.take<double>(nt);
  D.cry = cv.take<double>(nt);
  D.cdx = cv.take<double>(nt);
  D.cdy = cv.take<double>(nt);
  D.cqx = cv.take<double>(nt);
  D.cqy = cv.take<double>(nt);
  D.cwx = cv.take<double>(nt);
  D.cwy = cv.take<double>(nt);
  D.ct = cv.take<double>(nt);
  D.cu = cv.take<double>(nt);
  D.tct = cv.take<double>(nt);
  D.tcu = cv.take<double>(nt);
  R.hcount = cv.take<int32_t>(P);
  if (precision == CD_MIXED) {
    D.fgx = cv.take<double>(nt);
    D.fgy = cv.take<double>(nt);
    D.fhxx = cv.take<double>(nt);
    D.fhxy = cv.take<double>(nt);
    D.fhyy = cv.take<double>(nt);
    D.zrx = cv.take<double>(nt);
    D.zry = cv.take<double>(nt);
    D.hptr = cv.take<int32_t>(P + 1);
    D.hidx = cv.take<int32_t>(R.hcap);
    D.a32x = cv.take<float>(nt);
    D.a32y = cv.take<float>(nt);
    D.h32x = cv.take<float>(R.hcap);
    D.h32y = cv.take<float>(R.hcap);
    D.h64x = cv.take<double>(R.hcap);
    D.h64y = cv.take<double>(R.hcap);
    D.zhx = cv.take<double>(nt);
    D.zhy = cv.take<double>(nt);
    R.geom = cv.take<double>(3 * (size_t)P);
  } else {
    D.zhx = D.zhy = nullptr;
    R.geom = nullptr;
    D.fgx = D.fgy = D.fhxx = D.fhxy = D.fhyy = D.zrx = D.zry = nullptr;
    D.hptr = D.hidx = nullptr;
    D.a32x = D.a32y = D.h32x = D.h32y = nullptr;
    D.h64x = D.h64y = nullptr;
  }
  D.n = R.n;
  D.P = P;
  D.nbN = R.nbN;
  D.m = m;
  D.ntot = R.ntot;
  D.splits = R.splits;
  D.jb = R.jb;
  D.hcap = R.hcap;
  R.total = cv.off + 256;
  return true;
}

size_t relax_workspace_bytes(int op, int64_t n, int32_t n_patches, int64_t total_active,
                             int precision) {
  if (op == CD_OP_PATCHES)
    return n_patches > 0 ? (((size_t)n_patches + 2) * 4 + 511) & ~size_t(255) : 0;
  if (op != CD_OP_RELAX) return 0;
  RPlan R;
  if (!rplan(n, n_patches, total_active, precision, kMaxMem, nullptr, R)) return 0;
  return R.total;
}

// Mixed path: once at most this percent of the patches that started a round
// still run, their stage ends where they are (as at the iteration cap); they
// continue it after the next re-expansion, L-BFGS history kept, alongside the
// rest, instead of holding the batch in rounds that run a few patches on a
// mostly idle chip.
constexpr int kCutPercent = 50;

// Runs rounds (eval + update) until no patch is running or max rounds, or
// (cut_at > 0) until at most cut_at patches run, whose rounds it then ends.
// Returns a CD status.

// Relax schedules relax_autotune chooses among (the first is the default):
// the running-block count below which model blocks take 16 waves, lock-step
// rounds per graph replay, and the polish of a call that left it at
// CD_POLISH_DEFAULT (-1: the path's default; kOtherPolish: Newton on the
// mixed path, L-BFGS on the plain one).  The update kernel's workgroup shape
// is fixed (1024 threads, four register-held actives each: 512 and 256
// threads were slower on both the batch of 256 patches and the cycle).
struct RelaxSched {
  int64_t wide_blocks;
  int graph_rounds;
  int polish;
};
constexpr int kOtherPolish = 1;
constexpr RelaxSched kRelaxScheds[] = {{512, 8, -1},  {0, 8, -1},         {1 << 30, 8, -1},
                                       {256, 8, -1},  {1024, 8, -1},      {512, 4, -1},
                                       {512, 16, -1}, {512, 32, -1},      {512, 8, kOtherPolish}};
constexpr int kNumRelaxScheds = sizeof(kRelaxScheds) / sizeof(kRelaxScheds[0]);
static_assert(kNumRelaxScheds == CD_RELAX_SCHEDULES, "the header states the candidate count");
using RelaxKey = std::tuple<int, int, int, int64_t, int>;  // device, precision, coords, n, log2 total
static std::mutex g_rtune_mu;
static std::map<RelaxKey, int> g_rtuned;
static thread_local int g_force_sched = -1;  // the candidate relax_autotune is timing

static RelaxKey relax_key(int precision, int coords, int64_t n, int64_t ntot) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  int lg = 0;
  while ((int64_t(1) << (lg + 1)) <= ntot) ++lg;
  return std::make_tuple(dev, precision, coords, n, lg);
}

static int relax_sched_index(int precision, int coords, int64_t n, int64_t ntot) {
  if (g_force_sched >= 0) return g_force_sched;
  std::lock_guard<std::mutex> lk(g_rtune_mu);
  auto it = g_rtuned.find(relax_key(precision, coords, n, ntot));
  return it == g_rtuned.end() ? 0 : it->second;
}

// The rounds of one relax call as HIP graphs: graph_rounds rounds (model or
// exact evaluation, then the update) are captured once per evaluation shape
// on a private stream, which follows the caller's stream through events (a
// caller's default stream cannot be captured), and replayed until no patch
// runs.  The kernels and their arguments are those of the plain launches, so
// the results are the same bit for bit.  The launch option CD_LAUNCH_PLAIN
// selects the plain launches; when a graph cannot be captured or
// instantiated the rounds go on as plain launches.
struct RoundGraphs {
  hipStream_t cs = nullptr;
  hipEvent_t ev = nullptr;
  hipGraphExec_t ex[2] = {nullptr, nullptr};
  bool ok = false;
  bool broken = false;        // a capture failed: plain launches from then on
  int32_t* hc = nullptr;      // pinned host copies of the running count, one per block in flight
  hipEvent_t cev[2] = {nullptr, nullptr};
  bool begin(hipStream_t st) {
    if (!cs && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return false;
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return false;
    if (hipEventRecord(ev, st) != hipSuccess || hipStreamWaitEvent(cs, ev, 0) != hipSuccess)
      return false;
    return ok = true;
  }
  int end(hipStream_t st) {  // the caller's stream waits for the private one
    if (!ok) return CD_OK;
    ok = false;
    if (hipEventRecord(ev, cs) != hipSuccess || hipStreamWaitEvent(st, ev, 0) != hipSuccess)
      return CD_ERR_HIP;
    return CD_OK;
  }
  bool counts() {  // the pinned count slots and their events, made on first use
    if (!hc && hipHostMalloc(reinterpret_cast<void**>(&hc), 2 * sizeof(int32_t),
                             hipHostMallocDefault) != hipSuccess) {
      hc = nullptr;
      return false;
    }
    for (hipEvent_t& e : cev)
      if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return false;
    return true;
  }
  ~RoundGraphs() {
    if (cs) (void)hipStreamSynchronize(cs);  // no replay is still running below
    for (hipGraphExec_t& x : ex)
      if (x) (void)hipGraphExecDestroy(x);
    if (ev) (void)hipEventDestroy(ev);
    if (cs) (void)hipStreamDestroy(cs);
    for (hipEvent_t& e : cev)
      if (e) {
        (void)hipEventSynchronize(e);  // the copy into hc it follows has landed
        (void)hipEventDestroy(e);
      }
    if (hc) (void)hipHostFree(hc);
  }
};

template <int RJ>
static void launch_update(RPlan& R, hipStream_t s, bool hist32) {
  if (hist32 && R.D.tu)
    hipLaunchKernelGGL((k_update<float, true, RJ>), dim3(R.P), dim3(kUpd), 0, s, R.D);
  else if (hist32)
    hipLaunchKernelGGL((k_update<float, false, RJ>), dim3(R.P), dim3(kUpd), 0, s, R.D);
  else if (R.D.tu)
    hipLaunchKernelGGL((k_update<double, true, RJ>), dim3(R.P), dim3(kUpd), 0, s, R.D);
  else
    hipLaunchKernelGGL((k_update<double, false, RJ>), dim3(R.P), dim3(kUpd), 0, s, R.D);
}

template <class EvalFn>
static void launch_round(RPlan& R, hipStream_t s, bool hist32, int shape, EvalFn& eval) {
  if (R.D.polish) {  // CG iterations of patches in a Newton step, then the trial evaluations
    if (shape)
      hipLaunchKernelGGL((k_cg_hvp<kMWWide>), dim3(R.D.nblk), dim3(64 * kMWWide), 0, s, R.D);
    else
      hipLaunchKernelGGL((k_cg_hvp<kMW>), dim3(R.D.nblk), dim3(64 * kMW), 0, s, R.D);
  }
  eval(s, shape);
  // the (t, u) variant only when the call asked for it: the (x, y) kernel
  // carries none of its branches
  if (R.regj == kRegJWide)
    launch_update<kRegJWide>(R, s, hist32);
  else
    launch_update<kRegJ>(R, s, hist32);
}

// eval(stream, shape) enqueues one evaluation; shape(): 0 or 1, the
// evaluation's launch shape for the current running count.
//
// The rounds go in blocks of graph_rounds (one graph replay, or the same
// kernels launched one by one), each followed by an asynchronous copy of the
// running count into pinned host memory.  Two blocks are kept in flight: the
// host waits for the count of block k - 1 only once block k is queued, so the
// device does not idle while the host reads it.  The launch shape of block k
// comes from the count after block k - 2 (the last one read), the same on
// both launch modes, so their results agree bit for bit; blocks queued after
// the count reached zero find no running patch and change nothing.
template <class EvalFn, class ShapeFn>
static int run_rounds(RPlan& R, hipStream_t st, int max_rounds, bool hist32, RoundGraphs& G,
                      EvalFn eval, ShapeFn shape, int cut_at = 0) {
  RelaxDev& D = R.D;
  const int gr = R.graph_rounds;
  hipLaunchKernelGGL(k_count_running, dim3(1), dim3(256), 0, st, D);
  if (!G.counts()) return CD_ERR_HIP;
  const bool graphs = R.use_graphs && G.begin(st);
  hipStream_t ls = graphs ? G.cs : st;  // the stream the blocks go to
  int launched = 0, read = 0;           // blocks queued; blocks whose count was read
  bool stop = false;
  for (int r = 0;;) {
    if (!stop && r < max_rounds && launched - read < 2) {
      const int sh = shape();
      if (graphs && !G.broken && !G.ex[sh]) {
        // capture this shape's block; a capture or instantiation that fails
        // leaves nothing enqueued and hands the rounds to plain launches
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal) != hipSuccess) {
          G.broken = true;
        } else {
          for (int q = 0; q < gr; ++q) launch_round(R, ls, hist32, sh, eval);
          const hipError_t ce = hipStreamEndCapture(ls, &g);
          const hipError_t ie =
              (ce == hipSuccess && g) ? hipGraphInstantiate(&G.ex[sh], g, nullptr, nullptr, 0)
                                      : hipErrorUnknown;
          if (g) (void)hipGraphDestroy(g);
          if (ie != hipSuccess) {
            G.ex[sh] = nullptr;
            G.broken = true;
          }
        }
        (void)hipGetLastError();  // a failed capture's error is handled here
      }
      if (graphs && !G.broken) {
        if (hipGraphLaunch(G.ex[sh], ls) != hipSuccess) return CD_ERR_HIP;
      } else {
        for (int q = 0; q < gr; ++q) launch_round(R, ls, hist32, sh, eval);
      }
      const int b = launched & 1;
      if (hipMemcpyAsync(G.hc + b, D.running, sizeof(int32_t), hipMemcpyDeviceToHost, ls) !=
              hipSuccess ||
          hipEventRecord(G.cev[b], ls) != hipSuccess)
        return CD_ERR_HIP;
      ++launched;
      r += gr;
      continue;
    }
    if (read == launched) break;  // nothing in flight and nothing more to queue
    const int b = read & 1;
    if (hipEventSynchronize(G.cev[b]) != hipSuccess) return CD_ERR_HIP;
    R.running = G.hc[b];
    ++read;
    if (R.running <= 0 || R.running <= cut_at) stop = true;
  }
  if (R.running > 0 && R.running <= cut_at)
    hipLaunchKernelGGL(k_cut, dim3((R.P + 255) / 256), dim3(256), 0, ls, R.D);
  const int rc = graphs ? G.end(st) : CD_OK;
  if (rc) return rc;
  return hip_status(hipGetLastError());
}

}  // namespace cd

using namespace cd;

extern "C" {

int build_patches(const double* x, const double* y, int64_t n, int32_t n_patches,
                  const int32_t* centres, const int32_t* patch_ptr, int32_t* active_idx, void* ws,
                  size_t ws_bytes, void* stream) {
  if (!x || !y || !centres || !patch_ptr || !active_idx || n < 1 || n > (1 << 26) ||
      n_patches < 1 || patch_ptr[0] != 0)
    return CD_ERR_INVALID_ARG;
  for (int p = 0; p < n_patches; ++p) {
    const int sz = patch_ptr[p + 1] - patch_ptr[p];
    if (sz < 1 || sz > n) return CD_ERR_INVALID_ARG;
  }
  if (!ws || ws_bytes < relax_workspace_bytes(CD_OP_PATCHES, n, n_patches, 0, 0))
    return CD_ERR_WORKSPACE;
  int32_t* ptr_d =
      reinterpret_cast<int32_t*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  int32_t* err_d = ptr_d + n_patches + 1;
  hipStream_t st = (hipStream_t)stream;
  int rc = hip_status(hipMemcpyAsync(ptr_d, patch_ptr, sizeof(int32_t) * (n_patches + 1),
                                     hipMemcpyHostToDevice, st));
  if (rc) return rc;
  if ((rc = hip_status(hipMemsetAsync(err_d, 0, sizeof(int32_t), st)))) return rc;
  hipLaunchKernelGGL(k_patch_select, dim3(n_patches), dim3(1024), 0, st, x, y, (int)n, centres,
                     ptr_d, active_idx, err_d);
  rc = hip_status(hipGetLastError());
  if (rc) return rc;
  int32_t herr = 0;
  if ((rc = hip_status(hipMemcpyAsync(&herr, err_d, sizeof(int32_t), hipMemcpyDeviceToHost, st))))
    return rc;
  // also lets the caller release the host offsets array after return
  if ((rc = hip_status(hipStreamSynchronize(st)))) return rc;
  return herr ? CD_ERR_INVALID_ARG : CD_OK;
}

// scatter of committed positions: x[idx[a]] = xr[a]
__global__ void k_scatter(double* __restrict__ x, double* __restrict__ y,
                          const int32_t* __restrict__ idx, const double* __restrict__ xr,
                          const double* __restrict__ yr, int m) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= m) return;
  x[idx[a]] = xr[a];
  y[idx[a]] = yr[a];
}

int relax_subdomains(const double* x, const double* y, int64_t n, int32_t n_patches,
                     const int32_t* patch_ptr, const int32_t* active_idx, const double* x_start,
                     const double* y_start, const cd_relax_opts* opts, double* x_out,
                     double* y_out, double* dE, double* e_sub, double* gtan_inf, int32_t* iters,
                     int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  if (!x || !y || !patch_ptr || !active_idx || !opts) return CD_ERR_INVALID_ARG;
  if ((x_start == nullptr) != (y_start == nullptr)) return CD_ERR_INVALID_ARG;
  if ((x_out == nullptr) != (y_out == nullptr)) return CD_ERR_INVALID_ARG;
  if (n_patches < 1 || patch_ptr[0] != 0) return CD_ERR_INVALID_ARG;
  for (int p = 0; p < n_patches; ++p)
    if (patch_ptr[p + 1] <= patch_ptr[p] || patch_ptr[p + 1] - patch_ptr[p] > n)
      return CD_ERR_INVALID_ARG;
  cd_relax_opts o = *opts;
  if (o.exterior_model < CD_EXTERIOR_DEFAULT || o.exterior_model > CD_EXTERIOR_MODEL ||
      (o.exterior_model == CD_EXTERIOR_EXACT && o.precision != CD_FP64))
    return CD_ERR_INVALID_ARG;
  if (o.exterior_model == CD_EXTERIOR_MODEL && o.precision == CD_FP64) {
    // the model with FP64 pairs throughout: the mixed path, never below its
    // FP64 switch
    o.precision = CD_MIXED;
    o.inner_tol = 1e300;
  }
  if (!(o.gtol > 0.0) || o.max_iter < 0 || o.halo_width < 0.0 || o.inner_tol < 0.0 ||
      o.step0 < 0.0 || o.max_outer < 0 || !(o.sigma >= 0.0 && o.sigma <= 1.0))
    return CD_ERR_INVALID_ARG;
  if (o.polish < CD_POLISH_DEFAULT || o.polish > CD_POLISH_LBFGS || o.max_polish_iter < 0 ||
      !(o.newton_tol >= 0.0) || !(o.cg_eta >= 0.0 && o.cg_eta < 1.0) || !(o.trust_radius >= 0.0) ||
      (o.coords != CD_COORDS_XY && o.coords != CD_COORDS_TU) ||
      (o.launch != CD_LAUNCH_GRAPH && o.launch != CD_LAUNCH_PLAIN))
    return CD_ERR_INVALID_ARG;
  const int64_t ntot = patch_ptr[n_patches];
  if (o.lbfgs_m < 0 || o.lbfgs_m > kMaxMem) return CD_ERR_INVALID_ARG;
  const int m = o.lbfgs_m > 0 ? o.lbfgs_m : 8;
  RPlan R;
  if (!rplan(n, n_patches, ntot, o.precision, m, nullptr, R)) return CD_ERR_INVALID_ARG;
  if (!ws) return CD_ERR_WORKSPACE;
  if (ws_bytes < R.total) return CD_ERR_WORKSPACE;  // the plan actually used, memory m
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  rplan(n, n_patches, ntot, o.precision, m, base, R);
  hipStream_t st = (hipStream_t)stream;
  RelaxDev& D = R.D;
  double* const ptol_ws = D.ptol;
  D.ptol = nullptr;
  D.x = x;
  D.y = y;
  D.ptr = D.ptr_w;
  D.idx = active_idx;
  const double h = sqrt(2.0 * 3.141592653589793 / (sqrt(3.0) * (double)n));
  D.step0 = o.step0 > 0.0 ? o.step0 : 0.1 * h;
  D.c1 = 1e-4;
  D.noise_rel = 1e-14;
  D.max_iter = o.max_iter;
  D.bflag = o.boundary;
  D.sigma = o.sigma > 0.0 ? o.sigma : 1.0;
  D.eval_all = 0;
  D.tol = o.gtol;
  D.gtol = o.gtol;
  // defaults measured on the 256-patch batch at N = 1e5 (gtol 1e-3): the
  // plain path gains from Newton steps (each replaces many exact O(n_act N)
  // evaluations by CG iterations over the patch's own pairs); on the mixed
  // path a CG iteration costs a pair pass like an L-BFGS iteration, and
  // L-BFGS, which keeps its curvature pairs across rounds, is as fast
  const bool plain = o.precision == CD_FP64;
  const RelaxSched sched = kRelaxScheds[relax_sched_index(o.precision, o.coords, n, ntot)];
  R.graph_rounds = sched.graph_rounds;
  R.wide_blocks = sched.wide_blocks;
  R.use_graphs = o.launch == CD_LAUNCH_GRAPH;
  D.tu = o.coords == CD_COORDS_TU;
  D.tu_rmin = 1e-3 * D.sigma;
  // the Newton steps work in (x, y) and angle coordinates: none in (t, u); a
  // tuned schedule may flip the path's default polish
  bool newton_default = plain;
  if (sched.polish == kOtherPolish) newton_default = !newton_default;
  D.polish = !D.tu && (o.polish == CD_POLISH_NEWTON ||
                       (o.polish == CD_POLISH_DEFAULT && newton_default));
  D.max_cg = o.max_polish_iter > 0 ? o.max_polish_iter : 500;
  D.newton_tol = o.newton_tol > 0.0 ? o.newton_tol : (plain ? 3e-2 : 3e-5) / (h * h);
  D.cg_eta = o.cg_eta > 0.0 ? o.cg_eta : (plain ? 1e-2 : 0.0);  // 0: adaptive forcing
  D.pstats = o.polish_stats;
  const int max_iter_eff = o.max_iter > 0 ? o.max_iter : 1;
  // a Newton step takes up to max_cg CG rounds and a few line-search rounds;
  // the plain path may take many Newton steps in one run of rounds
  const int newton_rounds = D.polish ? (D.max_cg + 64) * (o.precision == CD_FP64 ? 32 : 1) : 0;
  // a whole number of graph replays, so that replayed and one-by-one rounds
  // stop at the same round
  const int max_rounds =
      (4 * max_iter_eff + 64 + newton_rounds + R.graph_rounds - 1) / R.graph_rounds *
      R.graph_rounds;

  std::vector<int2> blk;
  blk.reserve(R.nblk);
  int max_na = 0;
  for (int p = 0; p < n_patches; ++p) {
    max_na = std::max(max_na, patch_ptr[p + 1] - patch_ptr[p]);
    for (int a = patch_ptr[p]; a < patch_ptr[p + 1]; a += 64) blk.push_back(make_int2(p, a));
  }
  D.nblk = (int)blk.size();
  R.regj = max_na > kRegJ * kUpd ? kRegJWide : kRegJ;
  int rc;
  if ((rc = hip_status(hipMemcpyAsync(D.ptr_w, patch_ptr, sizeof(int32_t) * (n_patches + 1),
                                      hipMemcpyHostToDevice, st))))
    return rc;
  if ((rc = hip_status(hipMemcpyAsync(D.blk, blk.data(), blk.size() * sizeof(int2),
                                      hipMemcpyHostToDevice, st))))
    return rc;
  if ((rc = hip_status(hipMemsetAsync(D.maskA, 0, sizeof(uint64_t) * n_patches * R.nbN, st))))
    return rc;
  if ((rc = hip_status(hipMemsetAsync(D.maskAH, 0, sizeof(uint64_t) * n_patches * R.nbN, st))))
    return rc;
  const int tb = (int)((ntot + 255) / 256);
  const int tb64 = (int)((ntot + 63) / 64);
  if ((rc = hip_status(hipMemsetAsync(D.err, 0, sizeof(int32_t), st)))) return rc;
  hipLaunchKernelGGL(k_setup_actives, dim3(tb), dim3(256), 0, st, D, x_start, y_start);
  {
    int32_t herr = 0;
    if ((rc = hip_status(hipMemcpyAsync(&herr, D.err, sizeof(int32_t), hipMemcpyDeviceToHost, st))))
      return rc;
    if ((rc = hip_status(hipStreamSynchronize(st)))) return rc;
    if (herr) return CD_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_patch_geom, dim3(n_patches), dim3(256), 0, st, D);
  const dim3 eg((D.nblk + 3) / 4, R.splits), eb(256);
  auto exact_grad_on = [&](int all, hipStream_t s) {
    RelaxDev E = D;
    E.eval_all = all;
    hipLaunchKernelGGL(k_exact<kGrad>, eg, eb, 0, s, E);
    hipLaunchKernelGGL(k_exact_sum, dim3(tb64), dim3(64 * kESW), 0, s, E, (int)kGrad);
  };
  auto exact_grad = [&](int all) { exact_grad_on(all, st); };
  RoundGraphs graphs;

  if (o.max_iter == 0) {
    // evaluation only: the outputs describe the (projected) start positions
  } else if (o.precision == CD_FP64) {
    D.tol = o.gtol;
    if ((rc = run_rounds(R, st, max_rounds, false, graphs,
                         [&](hipStream_t s, int) { exact_grad_on(0, s); }, []() { return 0; })))
      return rc;
  } else {
    const double w = (o.halo_width > 0.0 ? o.halo_width : 4.0) * h;
    // the model is trusted within trust of its expansion point, and the halo
    // is rebuilt about the current actives once one has drifted a quarter of
    // the halo width from where it was built: within a round an active then
    // stays more than a quarter of the width from every frozen charge the
    // model does not hold explicitly
    D.trust = (o.trust_radius > 0.0 ? o.trust_radius * h : 0.5 * w);
    D.rebuild_d2 = 0.0625 * w * w;
    std::vector<int32_t> hc(n_patches), hp(n_patches + 1);
    // halo lists about geom (null: the patch state's centre and radius);
    // with geom, a halo that would not fit leaves the current one in place
    auto build_halo = [&](const double* geom, bool& built) -> int {
      built = false;
      hipLaunchKernelGGL(k_halo, dim3(n_patches), dim3(1024), 0, st, D, w, 0, R.hcount, geom);
      int e = hip_status(hipMemcpyAsync(hc.data(), R.hcount, sizeof(int32_t) * n_patches,
                                        hipMemcpyDeviceToHost, st));
      if (!e) e = hip_status(hipStreamSynchronize(st));
      if (e) return e;
      hp[0] = 0;
      for (int p = 0; p < n_patches; ++p) hp[p + 1] = hp[p] + hc[p];
      if (hp[n_patches] > R.hcap) return geom ? CD_OK : CD_ERR_WORKSPACE;
      if (geom) {
        hipLaunchKernelGGL(k_geom_commit, dim3((std::max(n_patches, (int)ntot) + 255) / 256),
                           dim3(256), 0, st, D, geom);
        if ((e = hip_status(hipMemcpyAsync(D.maskAH, D.maskA,
                                           sizeof(uint64_t) * n_patches * R.nbN,
                                           hipMemcpyDeviceToDevice, st))))
          return e;
      }
      if ((e = hip_status(hipMemcpyAsync(D.hptr, hp.data(), sizeof(int32_t) * (n_patches + 1),
                                         hipMemcpyHostToDevice, st))))
        return e;
      hipLaunchKernelGGL(k_halo, dim3(n_patches), dim3(1024), 0, st, D, w, 1, R.hcount, geom);
      const int hb = (hp[n_patches] + 255) / 256;
      hipLaunchKernelGGL(k_model_prep, dim3(tb > hb ? tb : hb), dim3(256), 0, st, D, 1);
      built = true;
      return hip_status(hipGetLastError());
    };
    if ((rc = hip_status(hipMemsetAsync(D.running + 1, 0, sizeof(int32_t), st)))) return rc;
    bool built = false;
    if ((rc = build_halo(nullptr, built))) return rc;
    int rebuilds = 0;
    bool rebuild = false;
    RelaxDev Df = D;
    Df.eval_all = 1;
    // 16-wave model blocks when the running patches hold fewer than
    // wide_blocks blocks (estimated from the running count)
    auto wide_shape = [&]() {
      return (int)((int64_t)R.running * D.nblk < R.wide_blocks * n_patches);
    };
    auto model_on = [&](int all, hipStream_t s, int wide) {
      RelaxDev E = D;
      E.eval_all = all;
      // within the rounds k_update writes the FP32 coordinates of each trial
      if (all) hipLaunchKernelGGL(k_model_prep, dim3(tb), dim3(256), 0, s, E, 0);
      // the Hessian blocks (preconditioner) are evaluated at the expansion
      // point only and kept for the rest of the round
      if (all && wide)
        hipLaunchKernelGGL((k_model<true, kMWWide>), dim3(D.nblk), dim3(64 * kMWWide), 0, s, E);
      else if (all)
        hipLaunchKernelGGL((k_model<true, kMW>), dim3(D.nblk), dim3(64 * kMW), 0, s, E);
      else if (wide)
        hipLaunchKernelGGL((k_model<false, kMWWide>), dim3(D.nblk), dim3(64 * kMWWide), 0, s, E);
      else
        hipLaunchKernelGGL((k_model<false, kMW>), dim3(D.nblk), dim3(64 * kMW), 0, s, E);
    };
    auto model = [&](int all) { model_on(all, st, wide_shape()); };
    // rounds: expand the far field exactly at z (one O(n_act N) FP64 pass);
    // the model gradient at its expansion point is the exact gradient, which
    // ends a patch when it meets gtol; otherwise minimise the model (FP32
    // pairs while the exact gradient is above tol32, FP64 pairs below) to a
    // hundredth of it, keeping the L-BFGS history across rounds
    const double tol32 = o.inner_tol > 0.0 ? o.inner_tol : 3e-2 / (h * h);
    const int outer_max = o.max_outer > 0 ? o.max_outer : 40;
    for (int outer = 0; outer < outer_max; ++outer) {
      if (rebuild) {  // a patch drifted from its halo: rebuild every patch's about its actives
        hipLaunchKernelGGL(k_patch_recentre, dim3(n_patches), dim3(256), 0, st, D, R.geom);
        if ((rc = build_halo(R.geom, built))) return rc;
        rebuilds += built;
        if (!built && (rc = hip_status(hipMemsetAsync(D.running + 1, 0, sizeof(int32_t), st))))
          return rc;
      }
      hipLaunchKernelGGL(k_copy_z_to_t, dim3(tb), dim3(256), 0, st, D);
      hipLaunchKernelGGL(k_exact<kFar>, eg, eb, 0, st, Df);
      hipLaunchKernelGGL(k_exact_sum, dim3(tb64), dim3(64 * kESW), 0, st, Df, (int)kFar);
      model(1);
      hipLaunchKernelGGL(k_check, dim3(n_patches), dim3(kUpd), 0, st, D, o.gtol, 0.01, tol32,
                         ptol_ws);
      hipLaunchKernelGGL(k_restart, dim3((n_patches + 255) / 256), dim3(256), 0, st, D, outer > 0);
      hipLaunchKernelGGL(k_count_running, dim3(1), dim3(256), 0, st, D);
      int32_t hrr[2] = {0, 0};
      if ((rc = hip_status(hipMemcpyAsync(hrr, D.running, 2 * sizeof(int32_t),
                                          hipMemcpyDeviceToHost, st))))
        return rc;
      if ((rc = hip_status(hipStreamSynchronize(st)))) return rc;
      const int32_t hr = hrr[0];
      rebuild = hrr[1] != 0;
      R.running = hr;
      if (hr == 0) break;
      D.ptol = ptol_ws;
      rc = run_rounds(R, st, max_rounds, true, graphs,
                      [&](hipStream_t s, int wide) { model_on(0, s, wide); }, wide_shape,
                      (int)((int64_t)hr * kCutPercent / 100));
      D.ptol = nullptr;
      if (rc) return rc;
    }
  }
  // exact energy and reduced gradient at the final positions, then the exact
  // energy change from the snapshot
  hipLaunchKernelGGL(k_copy_z_to_t, dim3(tb), dim3(256), 0, st, D);
  if (x_out || e_sub || gtan_inf || iters || status) {  // a call for dE alone skips them
    exact_grad(1);
    hipLaunchKernelGGL(k_finish, dim3(n_patches), dim3(kUpd), 0, st, D, o.gtol,
                       o.precision == CD_FP64 ? 1 : 0, x_out, y_out, e_sub, gtan_inf, iters,
                       status);
  }
  if (dE) {
    hipLaunchKernelGGL(k_exact<kDelta>, eg, eb, 0, st, D);
    hipLaunchKernelGGL(k_exact_sum, dim3(tb64), dim3(64 * kESW), 0, st, D, (int)kDelta);
    hipLaunchKernelGGL(k_finish_delta, dim3(n_patches), dim3(kUpd), 0, st, D, dE);
  }
  rc = hip_status(hipGetLastError());
  if (rc) return rc;
  return hip_status(hipStreamSynchronize(st));
}

// Relax schedule tuning: every schedule of kRelaxScheds relaxes the caller's
// batch once (outputs discarded; the first schedule once more beforehand, so
// that one-time start-up costs do not count), timed on the host around the
// synchronising call; the fastest is kept for later calls with the same
// device, precision, coordinates, n and floor(log2(total actives)).
int relax_autotune(const double* x, const double* y, int64_t n, int32_t n_patches,
                   const int32_t* patch_ptr, const int32_t* active_idx, const double* x_start,
                   const double* y_start, const cd_relax_opts* opts, void* ws, size_t ws_bytes,
                   void* stream, int32_t* choice_out, double* times_out) {
  if (!choice_out || !opts || !patch_ptr || n_patches < 1) return CD_ERR_INVALID_ARG;
  const int64_t ntot = patch_ptr[n_patches];
  double best_t = 0.0;
  int best = 0;
  int rc = CD_OK;
  for (int k = -1; k < kNumRelaxScheds && !rc; ++k) {
    g_force_sched = k < 0 ? 0 : k;
    const auto t0 = std::chrono::steady_clock::now();
    rc = relax_subdomains(x, y, n, n_patches, patch_ptr, active_idx, x_start, y_start, opts,
                          nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, ws,
                          ws_bytes, stream);
    const double dt =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (k < 0 || rc) continue;
    if (times_out) times_out[k] = dt;
    if (k == 0 || dt < best_t) {
      best = k;
      best_t = dt;
    }
  }
  g_force_sched = -1;
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_rtune_mu);
    g_rtuned[relax_key(opts->precision, opts->coords, n, ntot)] = best;
  }
  const RelaxSched& sc = kRelaxScheds[best];
  choice_out[0] = best;
  choice_out[1] = (int32_t)std::min<int64_t>(sc.wide_blocks, INT32_MAX);
  choice_out[2] = sc.graph_rounds;
  choice_out[3] = sc.polish;
  return CD_OK;
}

// Greedy commit of relaxed candidates.  Candidates with a negative energy
// change at the snapshot are visited in increasing order of that change
// (ties by index); one that shares a charge with an already committed
// candidate is skipped; otherwise its energy change is evaluated again,
// exactly, against the current configuration (earlier commits included,
// since the 1/r coupling makes changes non-additive) and it is committed --
// its positions written into x, y -- iff that change is negative.
int commit_patches(double* x, double* y, int64_t n, int32_t n_patches, const int32_t* patch_ptr,
                   const int32_t* active_idx, const double* x_rel, const double* y_rel,
                   const double* order_key, int32_t* committed, double* dE_commit, void* ws,
                   size_t ws_bytes, void* stream) {
  if (!x || !y || !patch_ptr || !active_idx || !x_rel || !y_rel || !order_key || !committed ||
      !dE_commit || n_patches < 1 || patch_ptr[0] != 0)
    return CD_ERR_INVALID_ARG;
  int maxp = 0;
  for (int p = 0; p < n_patches; ++p) {
    const int sz = patch_ptr[p + 1] - patch_ptr[p];
    if (sz < 1 || sz > n) return CD_ERR_INVALID_ARG;
    maxp = sz > maxp ? sz : maxp;
  }
  const size_t need = relax_workspace_bytes(CD_OP_RELAX, n, 1, maxp, CD_FP64);
  if (!need) return CD_ERR_INVALID_ARG;
  if (!ws) return CD_ERR_WORKSPACE;
  if (ws_bytes < need + 512) return CD_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  const int ntot = patch_ptr[n_patches];
  std::vector<int32_t> idx(ntot);
  int rc = hip_status(hipMemcpyAsync(idx.data(), active_idx, sizeof(int32_t) * ntot,
                                     hipMemcpyDeviceToHost, st));
  if (rc) return rc;
  if ((rc = hip_status(hipStreamSynchronize(st)))) return rc;
  for (int a = 0; a < ntot; ++a)
    if (idx[a] < 0 || idx[a] >= n) return CD_ERR_INVALID_ARG;
  std::vector<int> order;
  for (int p = 0; p < n_patches; ++p) {
    committed[p] = 0;
    dE_commit[p] = 0.0;
    if (order_key[p] < 0.0) order.push_back(p);
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return order_key[a] < order_key[b]; });
  std::vector<unsigned char> taken(n, 0);
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  double* dEd = reinterpret_cast<double*>(base);
  char* rws = base + 256;
  cd_relax_opts o = {};
  o.precision = CD_FP64;
  o.max_iter = 0;  // evaluation only: energy change of the given positions
  o.gtol = 1e300;
  for (int p : order) {
    const int a0 = patch_ptr[p], a1 = patch_ptr[p + 1];
    bool clash = false;
    for (int a = a0; a < a1 && !clash; ++a) clash = taken[idx[a]];
    if (clash) continue;
    const int32_t pp[2] = {0, a1 - a0};
    rc = relax_subdomains(x, y, n, 1, pp, active_idx + a0, x_rel + a0, y_rel + a0, &o, nullptr,
                          nullptr, dEd, nullptr, nullptr, nullptr, nullptr, rws, need, stream);
    if (rc) return rc;
    double d = 0.0;
    if ((rc = hip_status(hipMemcpyAsync(&d, dEd, sizeof(double), hipMemcpyDeviceToHost, st))))
      return rc;
    if ((rc = hip_status(hipStreamSynchronize(st)))) return rc;
    dE_commit[p] = d;
    if (d < 0.0) {
      hipLaunchKernelGGL(k_scatter, dim3((a1 - a0 + 255) / 256), dim3(256), 0, st, x, y,
                         active_idx + a0, x_rel + a0, y_rel + a0, a1 - a0);
      if ((rc = hip_status(hipGetLastError()))) return rc;
      committed[p] = 1;
      for (int a = a0; a < a1; ++a) taken[idx[a]] = 1;
    }
  }
  return hip_status(hipStreamSynchronize(st));
}

}  // extern "C"
