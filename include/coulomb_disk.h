/*
 * coulomb_disk.h -- C ABI of the MI355X (gfx950) engine for N unit charges
 * with 1/r repulsion confined to the unit disk.
 *
 * Model (paper Sec. II.A, Eqs. 2-3): energy E = sum_{i<j} 1/|r_i - r_j| in
 * units e^2/R, hard wall |r_i| <= 1.  Positions are structure-of-arrays FP64
 * (x[n], y[n]).
 *
 * Conventions shared by every entry point:
 *  - Pointers are DEVICE pointers unless the comment says host.  The caller
 *    owns every buffer; the library never allocates or frees device memory.
 *  - `ws` is caller-provided device scratch of at least
 *    coulomb_workspace_bytes(...) bytes for the same operation and sizes,
 *    256-byte aligned.  Calls sharing one workspace must not overlap.
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL = the
 *    default stream).  No call synchronises the stream except where noted
 *    (relax_subdomains and coulomb_lanczos read small per-iteration flags).
 *  - Return value: CD_OK, or a negative code detected before anything is
 *    enqueued (bad argument, workspace too small) or reported by the HIP
 *    runtime at launch.  Asynchronous kernel faults surface through the
 *    caller's next synchronisation.
 *  - Hot paths do not check the domain (finite, inside the disk, distinct
 *    positions); coulomb_validate does.  Self pairs are excluded by index;
 *    two distinct charges at the same point give non-finite results.
 *  - precision: CD_FP64 computes every pair in FP64; CD_MIXED computes pairs
 *    in FP32 on coordinates taken relative to a nearby reference point (with
 *    a hi/lo split for spatially near tiles) and folds FP32 partial sums of
 *    at most 64 terms into FP64 accumulators.
 *  - Results are deterministic for a given input, precision and device.
 */
#ifndef COULOMB_DISK_H
#define COULOMB_DISK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { CD_FP64 = 0, CD_MIXED = 1 };

enum {
  CD_OK = 0,
  CD_ERR_INVALID_ARG = -1,
  CD_ERR_WORKSPACE = -2,
  CD_ERR_HIP = -3,
  CD_ERR_DOMAIN = -4,
  CD_ERR_CAPACITY = -5,
  CD_ERR_SCRATCH = -6
};

/* operation selectors for coulomb_workspace_bytes */
enum {
  CD_OP_ENERGY = 0,
  CD_OP_FORCES = 1,
  CD_OP_HVP = 2,
  CD_OP_VALIDATE = 3,
  CD_OP_PATCHES = 4,
  CD_OP_RELAX = 5,
  CD_OP_LANCZOS = 6,
  CD_OP_DEFECT = 7,
  CD_OP_ZONES = 8,
  CD_OP_VORONOI = 9,
  CD_OP_BORDER = 10
};

/* Per-charge flags written by coulomb_validate. */
enum { CD_FLAG_NONFINITE = 1, CD_FLAG_OUTSIDE = 2, CD_FLAG_COINCIDENT = 4 };

/* Bytes of device scratch that `op` needs for these sizes (n_patches and
 * total_active matter only for CD_OP_PATCHES / CD_OP_RELAX; lanczos_k is
 * passed in n_patches for CD_OP_LANCZOS; the number of zones in n_patches
 * for CD_OP_ZONES).  Returns 0 for invalid sizes. */
size_t coulomb_workspace_bytes(int op, int64_t n, int32_t n_patches, int64_t total_active,
                               int precision);

/* Energy, Eq. 2: *e_total = sum_{i<j} 1/r_ij.  If e_local != NULL it receives
 * the local energies of Sec. II.C step 1, e_i = 1/2 sum_{j!=i} 1/r_ij (so
 * sum_i e_i = E).  n >= 1.  e_total: 1 double (device). */
int coulomb_energy(const double* x, const double* y, int64_t n, int precision,
                   double* e_total, double* e_local, void* ws, size_t ws_bytes, void* stream);

/* Forces F_i = -dE/dr_i = sum_{j!=i} (r_i - r_j)/r_ij^3 (the Cartesian
 * gradient the chain rule of Eqs. 8-10 consumes, Sec. II.D), fused with the
 * energy: fx[n], fy[n]; e_total (1 double) may be NULL. */
int coulomb_forces(const double* x, const double* y, int64_t n, int precision, double* fx,
                   double* fy, double* e_total, void* ws, size_t ws_bytes, void* stream);

/* Allocation-free coulomb_forces, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and results as coulomb_forces without
 * ws/ws_bytes: the scratch is a fixed 64 MiB region inside the library,
 * one per device, held from its first use on that device until the process
 * ends.  CD_MIXED batches the symmetric pass's chunks so that their partial
 * sums fit (more, smaller batches than coulomb_forces at large n; the sums
 * then run in another order, differences at FP64 rounding level).  Sizes
 * that do not fit return CD_ERR_SCRATCH before anything is enqueued
 * (every n up to 830,720 fits on CD_FP64, up to 706,304 on CD_MIXED).  Every call on
 * one device shares that device's region: calls that overlap on a device
 * (two streams, threads or graph replays in flight) race; serialise them.
 * Nothing needs clearing between calls.  Launches kernels only (no copy,
 * memset or synchronisation), so it can be captured in a HIP graph. */
int coulomb_forces_noalloc(const double* x, const double* y, int64_t n, int precision,
                           double* fx, double* fy, double* e_total, void* stream);

/* Riesz-s generalisation of Eq. 2 (the paper states its result in Riesz
 * terms, Sec. III.E): *e_total = sum_{i<j} r_ij^(-s) (nullable) and
 * F_i = -dE/dr_i = sum_{j!=i} s (r_i - r_j) r_ij^(-s-2): fx[n], fy[n].
 * s = 1 is the Coulomb case of coulomb_forces.  0 < s <= 6 on CD_MIXED
 * (FP32 pair terms 2^((-s/2-1) log2 r^2) from the hardware log2/exp2, so
 * close pairs must keep r^(-s-2) within FP32 range), 0 < s <= 64 on CD_FP64
 * (powers of the refined FP64 1/r when s is an integer up to 32, of its
 * square root when 2s is, else pow).  ws: coulomb_workspace_bytes(CD_OP_FORCES, n, 0, 0, precision). */
int coulomb_riesz(const double* x, const double* y, int64_t n, double s, int precision,
                  double* fx, double* fy, double* e_total, void* ws, size_t ws_bytes,
                  void* stream);

/* Hessian-vector product of Eq. 2's energy: (H v)_i = sum_{j!=i} K(d_ij)
 * (v_i - v_j), K(d) = (3 d d^T - |d|^2 I)/|d|^5, d_ij = r_i - r_j.
 * vx, vy, hx, hy: [n].  CD_MIXED: components of v must stay below 1e8 in
 * magnitude (padding charges sit at x ~ 1e30 and d.v is formed in FP32). */
int coulomb_hvp(const double* x, const double* y, const double* vx, const double* vy,
                int64_t n, int precision, double* hx, double* hy, void* ws, size_t ws_bytes,
                void* stream);

/* Launch-shape tuning of the CD_MIXED pair pass (not an operation of the
 * paper; a performance setting).  Times each candidate shape of the
 * symmetric pass (waves per workgroup, super-block offsets per chunk) for
 * `op` (CD_OP_ENERGY, CD_OP_FORCES or CD_OP_HVP, the HVP with v = r) on the
 * given positions, and keeps the fastest for later CD_MIXED calls with the
 * same op and n on the current device (process-wide, thread-safe).  Results
 * of those calls are deterministic for the chosen shape; another shape sums
 * in another order (differences at FP32 rounding level).  shape_out: host
 * int32[3] = chosen index, waves, offsets.  ws: at least
 * coulomb_workspace_bytes(op, n, 0, 0, CD_MIXED) + 16 n + 512 bytes (the
 * scratch of every pair call already covers all shapes).  Synchronises the
 * stream. */
int coulomb_autotune(const double* x, const double* y, int64_t n, int op, void* ws,
                     size_t ws_bytes, void* stream, int32_t* shape_out);

/* Domain check of positions against Eq. 3: flags_out[n] (int32) gets
 * CD_FLAG_* bits (non-finite; |r| > 1 + 4*2^-53; exactly coincident with
 * another charge).  *count_out (1 int32, device) = number of flagged
 * charges. */
int coulomb_validate(const double* x, const double* y, int64_t n, int32_t* flags_out,
                     int32_t* count_out, void* ws, size_t ws_bytes, void* stream);

/* Subdomains (paper Sec. II.C-E).  A batch of P patches is described by
 * host offsets patch_ptr[P+1] (patch_ptr[0] = 0, patch p holds the packed
 * entries patch_ptr[p] .. patch_ptr[p+1]-1) and a device array
 * active_idx[patch_ptr[P]] of charge indices.  Patches may overlap; each is
 * relaxed against the same frozen snapshot. */

/* Patch construction (Sec. II.C step 3-4, Sec. II.E sizes): patch p is the
 * patch_ptr[p+1]-patch_ptr[p] charges nearest to charge centres[p] (device
 * int32 [P]) by squared Euclidean distance computed in FP64 as
 * (dx*dx) + (dy*dy) without fused multiply-add, ties to the lower index,
 * written to active_idx in increasing index order.  ws: at least
 * coulomb_workspace_bytes(CD_OP_PATCHES, n, P, 0, 0) bytes.  Synchronises
 * the stream before returning. */
int build_patches(const double* x, const double* y, int64_t n, int32_t n_patches,
                  const int32_t* centres, const int32_t* patch_ptr, int32_t* active_idx,
                  void* ws, size_t ws_bytes, void* stream);

/* Options of relax_subdomains (host struct). */
typedef struct {
  int32_t precision; /* CD_FP64: exact FP64 evaluations throughout (O(n_act N) per
                        gradient); CD_MIXED: rounds of [exact FP64 far-field expansion
                        at the current positions (its gradient is the exact one, tested
                        against gtol); L-BFGS on the model = explicit active and halo
                        pairs (FP32 while the exact gradient exceeds inner_tol, FP64
                        after) + the expanded far field as a quadratic] */
  int32_t max_iter;  /* L-BFGS iterations: CD_FP64 in total, CD_MIXED per round;
                        0 = no iteration: the outputs evaluate the start */
  int32_t lbfgs_m;   /* L-BFGS memory, 1..16 (0 = 8); the workspace is sized for 16 */
  int32_t max_outer; /* CD_MIXED: rounds, each one exact far-field expansion (0 = 40) */
  double gtol;       /* tolerance on the inf-norm of the exact FP64 reduced gradient */
  double inner_tol;  /* CD_MIXED: FP32 pairs while the exact gradient exceeds this
                        (0 = 3e-2 / h^2) */
  double halo_width; /* CD_MIXED: halo width in units of h (0 = 4) */
  double step0;      /* largest displacement of an L-BFGS trial step (0 = 0.1 h) */
  /* Border-interior split (Sec. II.B); both zero/NULL give the hard wall of
   * Eq. 3 for every charge. */
  double sigma;              /* wall radius of the charges not pinned, in (0, 1]
                                (0 = 1) */
  const int32_t* boundary;   /* device int32 [n] or NULL: nonzero marks a boundary
                                charge, pinned to the unit circle (it moves only
                                along it); starts are projected accordingly */
  /* Truncated-Newton polish (FP64, driven by Hessian-vector products; Sec. II.C
   * step 4): below newton_tol a patch takes Newton steps -- preconditioned CG
   * (block-Jacobi: each charge's own 2x2 Hessian block) on the tangent-space
   * Hessian of E_sub at the current point, in optimisation coordinates (held
   * charges: their angle, with the circle's curvature term), stopped at
   * non-positive curvature, at a residual inf-norm of cg_eta times the gradient's
   * (but not below gtol / 10) or after max_polish_iter iterations; then the same
   * line search as an L-BFGS step (a failed one falls back to L-BFGS).  The
   * Hessian products are FP64 pairs over the patch's actives plus each charge's
   * exact block.  CD_MIXED takes one Newton step per exact expansion of the far
   * field (from the expansion point, where the model's Hessian is the exact one);
   * CD_FP64 takes them back to back. */
  int32_t polish;            /* CD_POLISH_NEWTON, CD_POLISH_LBFGS (L-BFGS to the end) or
                                CD_POLISH_DEFAULT: Newton on CD_FP64, L-BFGS on CD_MIXED
                                (the faster of the two on each path) */
  int32_t max_polish_iter;   /* CG iterations per Newton step (0 = 500) */
  double newton_tol;         /* on the exact reduced gradient's inf-norm (0 = 3e-2 / h^2
                                on CD_FP64, 3e-5 / h^2 on CD_MIXED; h the mean spacing
                                sqrt(2 pi / (sqrt(3) n))) */
  double cg_eta;             /* relative CG residual target, fixed; 0 = 1e-2 on CD_FP64,
                                adaptive on CD_MIXED: 0.1 for a first Newton step, then
                                0.9 (g_k / g_{k-1})^2 within [1e-8, 0.1]
                                (Eisenstat-Walker), and a second step that fails to
                                halve the gradient returns the patch to L-BFGS */
  int32_t* polish_stats;     /* device int32 [2P] or NULL: accepted Newton steps and CG
                                iterations per patch */
  double trust_radius;       /* CD_MIXED, in units of h (0 = half the halo width): a round
                                ends for a patch once one of its actives is farther than
                                this from the expansion point (the far field is a
                                quadratic, blind to charges beyond the halo that an
                                active could reach), and the next round re-expands where
                                the patch stands; the halos are rebuilt about the current
                                actives once one has drifted a quarter of the halo width
                                from where its halo was built */
  int32_t coords;            /* CD_COORDS_XY: interior charges move in (x, y) under the
                                wall rule (held on their wall, moving along it, when
                                pushed outward); CD_COORDS_TU: the parameterisation of
                                Sec. II.D -- an interior charge moves in (t, u), r =
                                sigma sin^2 t, x = r cos u, y = r sin u, with the
                                gradient of Eqs. 8-9, so r <= sigma holds without a wall
                                rule.  At r = 0 both derivatives vanish for any force, so
                                interior charges starting within 1e-3 sigma of the centre
                                keep (x, y).  Boundary charges move by their angle (Eq. 10)
                                either way.  No Newton polish in (t, u) (L-BFGS only). */
  int32_t launch;            /* CD_LAUNCH_GRAPH: lock-step rounds replayed from HIP graphs;
                                CD_LAUNCH_PLAIN: the same kernels launched one by one */
  int32_t exterior_model;    /* CD_EXTERIOR_DEFAULT: set by precision (CD_FP64 exact
                                evaluations, CD_MIXED the model); CD_EXTERIOR_EXACT: every
                                gradient an exact FP64 evaluation over all n (CD_FP64 only;
                                with CD_MIXED the call returns CD_ERR_INVALID_ARG);
                                CD_EXTERIOR_MODEL: the model of CD_MIXED (explicit active and
                                halo pairs plus the exactly re-expanded far field); with
                                CD_FP64 its pairs are FP64 throughout, the L-BFGS history is
                                stored in FP32 as on CD_MIXED, and the workspace is that of
                                CD_MIXED */
} cd_relax_opts;

enum { CD_COORDS_XY = 0, CD_COORDS_TU = 1 };
enum { CD_LAUNCH_GRAPH = 0, CD_LAUNCH_PLAIN = 1 };
enum { CD_EXTERIOR_DEFAULT = 0, CD_EXTERIOR_EXACT = 1, CD_EXTERIOR_MODEL = 2 };

enum { CD_POLISH_DEFAULT = 0, CD_POLISH_NEWTON = 1, CD_POLISH_LBFGS = 2 };

/* Relax every patch of the batch (Sec. II.C step 4) against the frozen
 * snapshot (x, y)[n]: minimise E_sub = sum_{i in A} e_i (Eqs. 6-7, 1/2 on
 * active-active pairs) over the active positions subject to |r| <= 1 (Eq. 3),
 * or under the border-interior split of opts (boundary charges on the unit
 * circle, the others within sigma), by L-BFGS with wall-held charges moving
 * on their circle.
 *   x_start, y_start: packed start positions [patch_ptr[P]] (device) or both
 *     NULL for the snapshot positions; starts outside the disk are projected.
 *   x_out, y_out (nullable pair): packed relaxed positions.
 *   dE[P]: E_sub(relaxed) - E_sub(snapshot), exact FP64 pair differences.
 *   e_sub[P]: exact FP64 E_sub at the relaxed positions.
 *   gtan_inf[P]: inf-norm of the exact FP64 reduced gradient there.
 *   iters[2P]: accepted iterations (L-BFGS and Newton steps, all stages)
 *     and exact FP64 evaluations per patch.
 *   status[P]: 0 converged (gtan_inf <= gtol), 1 iteration cap, 2 line search
 *     failed, 3 non-finite.
 * Output pointers other than x_out/y_out may be NULL.  ws: at least
 * coulomb_workspace_bytes(CD_OP_RELAX, n, P, patch_ptr[P], opts->precision).
 * Reads a few per-round flags back to the host and synchronises the stream
 * before returning.  The lock-step rounds are replayed from HIP graphs
 * captured on a private stream that follows `stream` (opts->launch =
 * CD_LAUNCH_PLAIN: the same kernels launched one by one, with identical
 * results). */
int relax_subdomains(const double* x, const double* y, int64_t n, int32_t n_patches,
                     const int32_t* patch_ptr, const int32_t* active_idx,
                     const double* x_start, const double* y_start, const cd_relax_opts* opts,
                     double* x_out, double* y_out, double* dE, double* e_sub,
                     double* gtan_inf, int32_t* iters, int32_t* status, void* ws,
                     size_t ws_bytes, void* stream);

/* Schedule tuning of relax_subdomains (not an operation of the paper; a
 * performance setting).  Relaxes the given batch once with each candidate
 * schedule -- the running-block count below which the model evaluation
 * spreads a 64-active block over 16 waves instead of 8 (0, 256, 512, 1024,
 * always), lock-step rounds per HIP graph replay (4, 8, 16, 32), and, for a
 * call that leaves polish at CD_POLISH_DEFAULT, the path's other polish
 * (Newton on CD_MIXED, L-BFGS on CD_FP64) -- outputs discarded, timed on the
 * host, and keeps the fastest for later relax_subdomains calls on the
 * current device with the same precision, coordinates, n and
 * floor(log2(patch_ptr[P])) (process-wide, thread-safe).  A schedule only
 * changes the order of work, and with it the rounding (the L-BFGS or Newton
 * polish choice changes the optimiser: any endpoint still meets the
 * tolerance).  Arguments as relax_subdomains; choice_out: host int32 [4] =
 * chosen index, wide-block count, rounds per replay, polish (-1 default,
 * 1 the other); times_out (nullable): host double [CD_RELAX_SCHEDULES],
 * seconds per candidate.  Synchronises the stream. */
#define CD_RELAX_SCHEDULES 9
int relax_autotune(const double* x, const double* y, int64_t n, int32_t n_patches,
                   const int32_t* patch_ptr, const int32_t* active_idx, const double* x_start,
                   const double* y_start, const cd_relax_opts* opts, void* ws, size_t ws_bytes,
                   void* stream, int32_t* choice_out, double* times_out);

/* Defect-targeted zones of a subdomain cycle (Sec. II.C).  Options (host
 * struct) of defect_zones. */
typedef struct {
  double kappa;    /* threshold mu + kappa * sigma_e of step 2 (the printed
                      rule is kappa = -1; +1 flags a high-energy tail) */
  double p_defect; /* probability that a centre is a defect charge (step 3: 0.8) */
  double r_lo;     /* zone radius range of the oscillation, 0 <= r_lo <= r_hi */
  double r_hi;
  int64_t t0;      /* index of the first zone of this call in the cycle, >= 0 */
  int32_t period;  /* zones per period of the radius oscillation, >= 1 */
  int32_t reserved;
} cd_zone_opts;

/* Steps 2-3 of Sec. II.C and the zone radius.  From the local energies
 * e[n] (device; the e_local of coulomb_energy is step 1):
 *   mu = (1/n) sum e_i and sigma_e = sqrt((1/n) sum (e_i - mu)^2) (FP64, fixed
 *   summation order), thr = mu + kappa * sigma_e, and the defect list
 *   D = {i : e_i > thr} in increasing index order (empty when e is constant
 *   or not finite).
 * Then for each zone t = 0..n_zones-1, from the caller's uniform draws
 * (device double [4 n_zones]: u, v in [0, 1) and a point (px, py) drawn
 * uniformly in the disk, per zone):
 *   centre: if u < p_defect and |D| > 0, the position of charge
 *     D[min(floor(v |D|), |D| - 1)], and centre_idx[t] = that charge;
 *     otherwise (px, py), and centre_idx[t] = -1.
 *   radius: s = (t0 + t) mod period, tri = 2 min(s, period - s) / period,
 *     rz[t] = r_lo + (r_hi - r_lo) * tri (a triangle wave), each operation
 *     rounded once in FP64.
 * cx, cy, rz: device double [n_zones]; centre_idx: device int32 [n_zones]
 * (all may be NULL when n_zones = 0: statistics only).  stats (nullable):
 * device double [4] = mu, sigma_e, thr, |D|.  defect_idx (nullable): device
 * int32 [n], its first |D| entries receive D.  ws: at least
 * coulomb_workspace_bytes(CD_OP_DEFECT, n, 0, 0, 0) bytes.  Does not
 * synchronise. */
int defect_zones(const double* x, const double* y, const double* e, int64_t n, int32_t n_zones,
                 const double* draws, const cd_zone_opts* opts, double* cx, double* cy,
                 double* rz, int32_t* centre_idx, double* stats, int32_t* defect_idx, void* ws,
                 size_t ws_bytes, void* stream);

/* The radius of a disk about a point of the unit disk that holds `count` of
 * the n charges at their mean density (n / pi): sqrt(count / n), rounded
 * once per operation; the r_lo and r_hi of cd_zone_opts for zones of a given
 * size (Sec. II.C: subdomains of a few hundred to a few thousand charges).
 * 0 for n < 1 or count < 0.  Host function, no device work. */
double zone_radius_holding(int64_t n, int64_t count);

/* Active sets of zones (Sec. II.C step 4): zone p holds every charge j with
 * (dx*dx) + (dy*dy) <= rz[p]*rz[p], dx = x[j] - cx[p], dy = y[j] - cy[p], each
 * operation rounded once in FP64, listed in increasing index order.
 * cx, cy, rz: device double [n_zones].  patch_ptr: host int32 [n_zones + 1],
 * filled with the offsets (patch_ptr[0] = 0) in every case that returns
 * CD_OK or CD_ERR_CAPACITY.  active_idx: device int32 [capacity]; if the
 * zones hold more than capacity entries in total, nothing is written and
 * CD_ERR_CAPACITY is returned (call again with patch_ptr[n_zones] entries).
 * Zones may be empty or overlap.  ws: at least
 * coulomb_workspace_bytes(CD_OP_ZONES, n, n_zones, 0, 0) bytes.
 * Synchronises the stream. */
int zone_patches(const double* x, const double* y, int64_t n, int32_t n_zones, const double* cx,
                 const double* cy, const double* rz, int32_t* patch_ptr, int32_t* active_idx,
                 int64_t capacity, void* ws, size_t ws_bytes, void* stream);

/* Batches of a cycle's zones for side-by-side relaxation (host code; all
 * pointers host).  Zones a and b conflict when (cx_a - cx_b)^2 +
 * (cy_a - cy_b)^2 < (rz_a + rz_b + gap)^2 (each operation rounded once in
 * FP64); no two zones of one batch conflict and no batch holds more than
 * cap zones.  Zones are placed in sequence order:
 *   keep_order != 0: zone t goes to the first batch after those of every
 *     earlier zone it conflicts with (conflicting zones keep their order);
 *   keep_order == 0: zone t goes to the first batch that holds no zone it
 *     conflicts with (first fit: fewer, fuller batches).
 * In both cases batches that are full are passed over.  batch: int32
 * [n_zones]; n_batches (nullable): int32 [1]. */
int zone_batches(const double* cx, const double* cy, const double* rz, int32_t n_zones,
                 double gap, int32_t cap, int32_t keep_order, int32_t* batch,
                 int32_t* n_batches);

/* Border-interior split (Sec. II.B).  border_count: N_b of Eq. 4,
 * 2.84328 N^(2/3) - 0.530196 N^(1/3) - 2.32866 rounded to the nearest integer
 * and clamped to [0, n] (6099 at N = 1e5).  border_sigma0: the initial
 * interior radius of Eq. 5, 1 - 1/(2 sqrt(N)).  Host code. */
int32_t border_count(int64_t n);
double border_sigma0(int64_t n);

/* The interior radius over a cycle (Sec. II.B: it rises from the value of
 * Eq. 5 to 1; the paper gives the end points, not the law): stage k of
 * `stages` has sigma_start + (sigma_end - sigma_start) (k / stages), k clamped
 * to [0, stages]; sigma_start <= 0 takes border_sigma0(n); stages <= 0 gives
 * sigma_end.  Host function, no device work. */
double border_sigma_ramp(int64_t n, int32_t k, int32_t stages, double sigma_start,
                         double sigma_end);

/* Boundary charges: flags[n] (device int32) = 1 for the nb charges farthest
 * from the centre by (x*x) + (y*y) (each operation rounded once in FP64),
 * ties to the lower index, 0 for the others.  0 <= nb <= n.  One workgroup;
 * needs no workspace; does not synchronise. */
int border_split(const double* x, const double* y, int64_t n, int32_t nb, int32_t* flags,
                 void* stream);

/* Projection onto the split's feasible set, in place on x, y (device [n]):
 * a charge with flags[i] != 0 onto the unit circle (x / r), any other charge
 * with r > sigma onto the circle of radius sigma (x * (sigma / r)), with
 * r = sqrt((x*x) + (y*y)) and each operation rounded once in FP64.  flags:
 * device int32 [n] or NULL (no boundary charges); 0 < sigma <= 1.  Does not
 * synchronise. */
int border_project(double* x, double* y, int64_t n, const int32_t* flags, double sigma,
                   void* stream);

/* Start of the split before a cycle (a step the paper leaves open; moving
 * the boundary charges of an unrelaxed configuration along their rays, as
 * border_project does, lands charges of adjacent rings almost on top of each
 * other): the charges with flags[i] != 0, ordered by theta = atan2(y, x)
 * (ties to the lower index), go onto the unit circle at angle theta_0 +
 * 2 pi k / nb -- k their rank, nb their number, theta_0 the angle of the
 * first -- as x = cos, y = sin, in place on x, y (device [n]); the others are
 * unchanged.  flags: device int32 [n].  One workgroup, O(nb^2) comparisons.
 * ws: coulomb_workspace_bytes(CD_OP_BORDER, n, 0, 0, 0) bytes.  Does not
 * synchronise. */
int border_spread(double* x, double* y, int64_t n, const int32_t* flags, void* ws,
                  size_t ws_bytes, void* stream);

/* Structure analysis (Sec. III): Voronoi coordination and psi_6.
 * z[n] (device int32): the number of Voronoi (Delaunay) neighbours of each
 * charge; -2 for a charge on the convex hull (unbounded cell); -1 only if a
 * cell needs more than 48 vertices or reaches 1e4 from its charge.  Each cell is certified exact: clipped
 * by every charge in a widening grid neighbourhood until 2|v| <= the
 * neighbourhood's margin for all its vertices v (relative to the charge).
 * psi6 (nullable, device double [2n]): real and imaginary part of
 * psi_6(i) = (1/z_i) sum_j ((r_j - r_i)/|r_j - r_i|)^6 over the neighbours
 * (0 for z <= 0).  Charges must be distinct and inside |r| <= 1 + 1e-9.
 * The convex hull is found on the host (monotone chain) from a copy of the
 * positions, so the call synchronises the stream.  ws:
 * coulomb_workspace_bytes(CD_OP_VORONOI, n, 0, 0, 0) bytes. */
int voronoi_coordination(const double* x, const double* y, int64_t n, int32_t* z, double* psi6,
                         void* ws, size_t ws_bytes, void* stream);

/* Radial counts: counts[nbins] (device int32) of |r| = sqrt((x*x) + (y*y))
 * (each operation rounded once) in the bins floor(|r| nbins), the last bin
 * also taking |r| >= 1.  Does not synchronise. */
int radial_histogram(const double* x, const double* y, int64_t n, int32_t nbins, int32_t* counts,
                     void* stream);

/* Statistics of a voronoi_coordination result (Sec. III: the coordination
 * fractions and the mean bond-orientational order), into out (device double
 * [9]): out[0..4] the fractions P(z) of the bounded cells with z = 4..8,
 * out[5] the mean of |psi_6| over the bounded cells (0 when psi6 is NULL or
 * no cell is bounded), out[6] the number of bounded cells (z >= 0), out[7]
 * of hull charges (z = -2), out[8] of unresolved cells (z = -1).  One
 * workgroup sums in a fixed order, so the result is reproducible.  Does not
 * synchronise. */
int structure_stats(const int32_t* z, const double* psi6, int64_t n, double* out, void* stream);

/* Greedy commit of relaxed candidates (perturb-and-relax cycles): the
 * candidates whose snapshot energy change order_key[p] (host [P], e.g. the dE
 * of relax_subdomains) is negative are visited in increasing order of it
 * (ties by index).  A candidate sharing a charge with one already committed
 * is skipped; otherwise its exact FP64 energy change is evaluated again
 * against the current configuration and, iff negative, its packed positions
 * x_rel, y_rel (device) are written into x, y (device, updated in place).
 * committed[P] (host int32): 1 if committed; dE_commit[P] (host): the
 * re-evaluated change (0 when not evaluated).  ws: at least
 * coulomb_workspace_bytes(CD_OP_RELAX, n, 1, largest patch, CD_FP64) + 512
 * bytes (the CD_OP_RELAX size never decreases as total_active grows, so this
 * covers every patch).  Synchronises the stream. */
int commit_patches(double* x, double* y, int64_t n, int32_t n_patches, const int32_t* patch_ptr,
                   const int32_t* active_idx, const double* x_rel, const double* y_rel,
                   const double* order_key, int32_t* committed, double* dE_commit, void* ws,
                   size_t ws_bytes, void* stream);

/* Local-minimum certificate (tangent space of the hard wall of Eq. 3):
 * k steps of Lanczos with full reorthogonalisation on the operator
 *   H_t v = P H P v + w o v,
 * H the Hessian of the energy (of E_sub over the active charges when mask is
 * given), P the projection removing the radial component of held charges
 * (|r| >= 1 - 1e-14 with outward force F . r_hat > 0) and every component of
 * inactive ones, w_i = F_i . r_hat_i on held charges (the circle's curvature
 * term), 0 elsewhere.  FP64 Hessian-vector products throughout.
 *   mask: device int32 [n], nonzero = active, or NULL (all active).
 *   k: 2..4096 Lanczos steps (lanczos_k, passed as n_patches to
 *      coulomb_workspace_bytes(CD_OP_LANCZOS, n, k, 0, 0)).
 *   deflate_rotation: nonzero projects out the rigid rotation (-y, x), an
 *      exact zero mode of a full-disk configuration.
 *   seed: start vector (counter-based hash, uniform in [-1, 1)).
 *   out_host[4] (host): smallest Ritz value theta, residual ||H_t u - theta u||
 *      of its unit Ritz vector, largest Ritz value, steps used.
 * A positive theta with residual below theta/2 certifies a strict local
 * minimum.  Synchronises the stream before returning. */
int tangent_lanczos(const double* x, const double* y, int64_t n, const int32_t* mask,
                    int32_t k, int32_t deflate_rotation, uint64_t seed, double* out_host,
                    void* ws, size_t ws_bytes, void* stream);

/* Measurement hook: when ev_start/ev_stop (hipEvent_t passed as void*) are
 * non-NULL, every later energy/forces/HVP call records ev_start immediately
 * before its first and ev_stop immediately after its last launch of the
 * dominant pair kernel, on the call's stream (with more than one batch of
 * chunks the span includes the reductions between them).  NULL, NULL
 * disables.  Process-wide, not thread-safe; for benchmarking only. */
void coulomb_set_kernel_events(void* ev_start, void* ev_stop);

/* Human-readable text for a return code (host string, static storage). */
const char* coulomb_status_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* COULOMB_DISK_H */
