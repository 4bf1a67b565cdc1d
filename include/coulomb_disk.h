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
  CD_ERR_DOMAIN = -4
};

/* operation selectors for coulomb_workspace_bytes */
enum {
  CD_OP_ENERGY = 0,
  CD_OP_FORCES = 1,
  CD_OP_HVP = 2,
  CD_OP_VALIDATE = 3,
  CD_OP_PATCHES = 4,
  CD_OP_RELAX = 5,
  CD_OP_LANCZOS = 6
};

/* Per-charge flags written by coulomb_validate. */
enum { CD_FLAG_NONFINITE = 1, CD_FLAG_OUTSIDE = 2, CD_FLAG_COINCIDENT = 4 };

/* Bytes of device scratch that `op` needs for these sizes (n_patches and
 * total_active matter only for CD_OP_PATCHES / CD_OP_RELAX; lanczos_k is
 * passed in n_patches for CD_OP_LANCZOS).  Returns 0 for invalid sizes. */
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

/* Hessian-vector product of Eq. 2's energy: (H v)_i = sum_{j!=i} K(d_ij)
 * (v_i - v_j), K(d) = (3 d d^T - |d|^2 I)/|d|^5, d_ij = r_i - r_j.
 * vx, vy, hx, hy: [n]. */
int coulomb_hvp(const double* x, const double* y, const double* vx, const double* vy,
                int64_t n, int precision, double* hx, double* hy, void* ws, size_t ws_bytes,
                void* stream);

/* Domain check of positions against Eq. 3: flags_out[n] (int32) gets
 * CD_FLAG_* bits (non-finite; |r| > 1 + 4*2^-53; exactly coincident with
 * another charge).  *count_out (1 int32, device) = number of flagged
 * charges. */
int coulomb_validate(const double* x, const double* y, int64_t n, int32_t* flags_out,
                     int32_t* count_out, void* ws, size_t ws_bytes, void* stream);

/* Measurement hook: when ev_start/ev_stop (hipEvent_t passed as void*) are
 * non-NULL, every later energy/forces/HVP call records ev_start immediately
 * before and ev_stop immediately after its dominant pair kernel, on the
 * call's stream.  NULL, NULL disables.  Process-wide, not thread-safe; for
 * benchmarking only. */
void coulomb_set_kernel_events(void* ev_start, void* ev_stop);

/* Human-readable text for a return code (host string, static storage). */
const char* coulomb_status_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* COULOMB_DISK_H */
