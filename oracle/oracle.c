/*
 * CPU oracle for the unit-disk Coulomb problem — TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously-correct FP64 reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * links or calls it, and it shares no code with the GPU kernels.
 *
 * Model (paper Sec. II.A, Eqs. 2-3): N unit charges in the unit disk, energy
 * E = sum_{i<j} 1/|r_i - r_j| in units e^2/R, hard wall |r_i| <= 1.
 *
 * Every sum is a Neumaier-compensated FP64 sum taken in a fixed order (rows in
 * ascending i, columns in ascending j); OpenMP only splits rows, and row
 * results are merged in row order, so results do not depend on the thread
 * count.  Each 1/r is 1.0/sqrt(r2) with IEEE sqrt and divide.
 *
 * Functions and the passage each one follows:
 *   orc_energy       Eq. 2 (pair sum) and step 1 of the cycle in Sec. II.C
 *                    (local energies e_i = 1/2 sum_{j!=i} 1/r_ij).
 *   orc_forces       F_i = -dE/dr_i, the Cartesian gradient that feeds the
 *                    chain rule of Eqs. 8-10 (Sec. II.D).
 *   orc_hvp          Hessian-vector product of Eq. 2: second derivatives of
 *                    1/|d| are (3 d d^T - |d|^2 I)/|d|^5.
 *   orc_hessian      the same Hessian as a dense 2N x 2N matrix (tiny N).
 *   orc_rows         forces, HVP rows and e_i for a subset of charges.
 *   orc_esub         subdomain objective of Eqs. 6-7 with the reading
 *                    E_sub = sum_{i in A} e_i, e_i = 1/2 sum_{j in A, j!=i}
 *                    1/r_ij + sum_{j in F} 1/r_ij, and its gradient over A.
 *   orc_esub_delta   E_sub(moved) - E_sub(snapshot) as a sum over changed pairs
 *                    of the change of 1/r, formed without cancellation.
 *   orc_esub_hvp     Hessian-vector product of E_sub over the active coordinates.
 *   orc_riesz        Riesz-s energy and forces (1/r^s pairs).
 *   orc_reduce_grad  hard-wall (Eq. 3) KKT reduction of the gradient.
 *   orc_relax        local relaxation of one subdomain (Sec. II.C step 4):
 *                    L-BFGS on free and wall-held coordinates, then
 *                    truncated Newton on the tangent-space Hessian.
 *   orc_reduce_grad_bi, orc_relax_bi  the same under the border-interior
 *                    constraint of Sec. II.B: boundary charges pinned to the
 *                    unit circle, the others confined to |r| <= sigma.
 *   orc_tu_grad, orc_relax_tu  the parameterisation of Sec. II.D: interior
 *                    charges in (t, u) with r = sigma sin^2 t, the gradient
 *                    by the chain rule of Eqs. 8-9 (boundary charges: Eq. 10),
 *                    and a relaxation in these coordinates.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double s, c; } nacc;

static inline void nadd(nacc *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}
static inline double nval(const nacc *a) { return a->s + a->c; }

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------- energy -- */
/* E = sum_{i<j} 1/r_ij.  If e_local != NULL also e_i = 1/2 sum_{j!=i} 1/r_ij. */
double orc_energy(int64_t n, const double *x, const double *y, double *e_local) {
  double *rs = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double *rc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    nacc a = {0.0, 0.0};
    for (int64_t j = i + 1; j < n; ++j) {
      double dx = x[i] - x[j], dy = y[i] - y[j];
      nadd(&a, 1.0 / sqrt(dx * dx + dy * dy));
    }
    rs[i] = a.s;
    rc[i] = a.c;
  }
  nacc t = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i) {
    nadd(&t, rs[i]);
    nadd(&t, rc[i]);
  }
  free(rs);
  free(rc);
  if (e_local) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      nacc a = {0.0, 0.0};
      for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double dx = x[i] - x[j], dy = y[i] - y[j];
        nadd(&a, 1.0 / sqrt(dx * dx + dy * dy));
      }
      e_local[i] = 0.5 * nval(&a);
    }
  }
  return nval(&t);
}

/* ---------------------------------------------------------------- forces -- */
/* F_i = sum_{j!=i} (r_i - r_j)/r_ij^3  (= -dE/dr_i). */
void orc_forces(int64_t n, const double *x, const double *y, double *fx, double *fy) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    nacc ax = {0.0, 0.0}, ay = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = x[i] - x[j], dy = y[i] - y[j];
      double r2 = dx * dx + dy * dy;
      double w = 1.0 / (r2 * sqrt(r2));
      nadd(&ax, dx * w);
      nadd(&ay, dy * w);
    }
    fx[i] = nval(&ax);
    fy[i] = nval(&ay);
  }
}

/* ----------------------------------------------------------------- Riesz -- */
/* The Riesz-s generalisation of Eq. 2 (the paper states its result in Riesz
 * terms): E = sum_{i<j} r_ij^(-s) and F_i = -dE/dr_i =
 * sum_{j!=i} s (r_i - r_j) r_ij^(-s-2).  Pair terms from pow(); sums are
 * Neumaier-compensated, rows in index order.  fx, fy may be NULL. */
double orc_riesz(int64_t n, const double *x, const double *y, double s, double *fx, double *fy) {
  double *rs = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double *rc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    nacc e = {0.0, 0.0}, ax = {0.0, 0.0}, ay = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = x[i] - x[j], dy = y[i] - y[j];
      double r2 = dx * dx + dy * dy;
      double p = pow(r2, -0.5 * s); /* r^-s */
      if (j > i) nadd(&e, p);
      double w = s * p / r2;
      nadd(&ax, dx * w);
      nadd(&ay, dy * w);
    }
    rs[i] = e.s;
    rc[i] = e.c;
    if (fx) fx[i] = nval(&ax);
    if (fy) fy[i] = nval(&ay);
  }
  nacc t = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i) {
    nadd(&t, rs[i]);
    nadd(&t, rc[i]);
  }
  free(rs);
  free(rc);
  return nval(&t);
}

/* The same sums for a subset of rows only (sampled checks at large N):
 * out0/out1 = F_i, or (H v)_i when vx != NULL; e_out = e_i (nullable). */
void orc_rows(int64_t n, const double *x, const double *y, const double *vx, const double *vy,
              int64_t nrows, const int32_t *rows, double *out0, double *out1, double *e_out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    nacc a0 = {0, 0}, a1 = {0, 0}, ae = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = x[i] - x[j], dy = y[i] - y[j];
      double r2 = dx * dx + dy * dy;
      double rr = sqrt(r2);
      nadd(&ae, 1.0 / rr);
      double i3 = 1.0 / (r2 * rr);
      if (vx) {
        double wx = vx[i] - vx[j], wy = vy[i] - vy[j];
        double i5 = i3 / r2;
        double dw = dx * wx + dy * wy;
        nadd(&a0, 3.0 * dx * dw * i5 - wx * i3);
        nadd(&a1, 3.0 * dy * dw * i5 - wy * i3);
      } else {
        nadd(&a0, dx * i3);
        nadd(&a1, dy * i3);
      }
    }
    if (out0) out0[r] = nval(&a0);
    if (out1) out1[r] = nval(&a1);
    if (e_out) e_out[r] = 0.5 * nval(&ae);
  }
}

/* ------------------------------------------------------------------- hvp -- */
/* (H v)_i = sum_{j!=i} K(d_ij) (v_i - v_j),  K(d) = (3 d d^T - |d|^2 I)/|d|^5. */
void orc_hvp(int64_t n, const double *x, const double *y, const double *vx,
             const double *vy, double *hx, double *hy) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    nacc ax = {0.0, 0.0}, ay = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = x[i] - x[j], dy = y[i] - y[j];
      double wx = vx[i] - vx[j], wy = vy[i] - vy[j];
      double r2 = dx * dx + dy * dy;
      double r = sqrt(r2);
      double i3 = 1.0 / (r2 * r);
      double i5 = i3 / r2;
      double dw = dx * wx + dy * wy;
      nadd(&ax, 3.0 * dx * dw * i5 - wx * i3);
      nadd(&ay, 3.0 * dy * dw * i5 - wy * i3);
    }
    hx[i] = nval(&ax);
    hy[i] = nval(&ay);
  }
}

/* Dense Hessian, row-major 2n x 2n, coordinate order (x0, y0, x1, y1, ...). */
void orc_hessian(int64_t n, const double *x, const double *y, double *H) {
  const int64_t m = 2 * n;
  memset(H, 0, sizeof(double) * (size_t)(m * m));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    nacc dxx = {0, 0}, dxy = {0, 0}, dyy = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = x[i] - x[j], dy = y[i] - y[j];
      double r2 = dx * dx + dy * dy;
      double r = sqrt(r2);
      double i3 = 1.0 / (r2 * r);
      double i5 = i3 / r2;
      double kxx = 3.0 * dx * dx * i5 - i3;
      double kxy = 3.0 * dx * dy * i5;
      double kyy = 3.0 * dy * dy * i5 - i3;
      H[(2 * i) * m + 2 * j] = -kxx;
      H[(2 * i) * m + 2 * j + 1] = -kxy;
      H[(2 * i + 1) * m + 2 * j] = -kxy;
      H[(2 * i + 1) * m + 2 * j + 1] = -kyy;
      nadd(&dxx, kxx);
      nadd(&dxy, kxy);
      nadd(&dyy, kyy);
    }
    H[(2 * i) * m + 2 * i] = nval(&dxx);
    H[(2 * i) * m + 2 * i + 1] = nval(&dxy);
    H[(2 * i + 1) * m + 2 * i] = nval(&dxy);
    H[(2 * i + 1) * m + 2 * i + 1] = nval(&dyy);
  }
}

/* ------------------------------------------------------------- subdomain -- */
/* Full-length position arrays with the active charges moved, plus a flag
 * array (1 = active).  Caller frees. */
static void place(int64_t n, const double *x, const double *y, int64_t na,
                  const int32_t *idx, const double *xa, const double *ya,
                  double **X, double **Y, unsigned char **act) {
  *X = (double *)malloc(sizeof(double) * (size_t)n);
  *Y = (double *)malloc(sizeof(double) * (size_t)n);
  *act = (unsigned char *)calloc((size_t)n, 1);
  memcpy(*X, x, sizeof(double) * (size_t)n);
  memcpy(*Y, y, sizeof(double) * (size_t)n);
  for (int64_t a = 0; a < na; ++a) {
    (*X)[idx[a]] = xa ? xa[a] : x[idx[a]];
    (*Y)[idx[a]] = ya ? ya[a] : y[idx[a]];
    (*act)[idx[a]] = 1;
  }
}

/* E_sub = sum_{i in A} e_i with e_i = 1/2 sum_{j in A, j != i} 1/r_ij +
 * sum_{j in F} 1/r_ij, evaluated with the active charges at (xa, ya) (NULL =
 * snapshot).  gx, gy (nullable, length na) receive dE_sub/dr_i for i in A. */
double orc_esub(int64_t n, const double *x, const double *y, int64_t na,
                const int32_t *idx, const double *xa, const double *ya,
                double *gx, double *gy) {
  double *X, *Y;
  unsigned char *act;
  place(n, x, y, na, idx, xa, ya, &X, &Y, &act);
  double *rs = (double *)malloc(sizeof(double) * (size_t)(na > 0 ? na : 1));
  double *rc = (double *)malloc(sizeof(double) * (size_t)(na > 0 ? na : 1));
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < na; ++a) {
    const int64_t i = idx[a];
    nacc e = {0, 0}, ax = {0, 0}, ay = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = X[i] - X[j], dy = Y[i] - Y[j];
      double r2 = dx * dx + dy * dy;
      double r = sqrt(r2);
      double inv = 1.0 / r;
      nadd(&e, act[j] ? 0.5 * inv : inv);
      double w = 1.0 / (r2 * r);
      nadd(&ax, -dx * w);
      nadd(&ay, -dy * w);
    }
    rs[a] = e.s;
    rc[a] = e.c;
    if (gx) gx[a] = nval(&ax);
    if (gy) gy[a] = nval(&ay);
  }
  nacc t = {0, 0};
  for (int64_t a = 0; a < na; ++a) {
    nadd(&t, rs[a]);
    nadd(&t, rc[a]);
  }
  free(rs);
  free(rc);
  free(X);
  free(Y);
  free(act);
  return nval(&t);
}

/* E_sub(active at (xa,ya)) - E_sub(active at snapshot): the sum over every
 * pair with at least one active member of 1/r_new - 1/r_old (weight 1/2 on
 * ordered active-active pairs, which appear twice).  Each difference is
 * formed without cancellation from
 *   1/r' - 1/r = (r^2 - r'^2) / (r r' (r + r')),
 *   r^2 - r'^2 = (d - d').(d + d'),  d - d' = -(delta_i - delta_j),
 * where delta is a charge's displacement (zero for frozen charges). */
double orc_esub_delta(int64_t n, const double *x, const double *y, int64_t na,
                      const int32_t *idx, const double *xa, const double *ya) {
  double *X, *Y;
  unsigned char *act;
  place(n, x, y, na, idx, xa, ya, &X, &Y, &act);
  double *rs = (double *)malloc(sizeof(double) * (size_t)(na > 0 ? na : 1));
  double *rc = (double *)malloc(sizeof(double) * (size_t)(na > 0 ? na : 1));
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < na; ++a) {
    const int64_t i = idx[a];
    const double six = X[i] - x[i], siy = Y[i] - y[i];
    nacc s = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dxo = x[i] - x[j], dyo = y[i] - y[j];
      double dxn = X[i] - X[j], dyn = Y[i] - Y[j];
      double mx = -(six - (X[j] - x[j])), my = -(siy - (Y[j] - y[j])); /* d - d' */
      double ro = sqrt(dxo * dxo + dyo * dyo), rn = sqrt(dxn * dxn + dyn * dyn);
      double num = mx * (dxo + dxn) + my * (dyo + dyn);
      double d = num / (ro * rn * (ro + rn));
      nadd(&s, act[j] ? 0.5 * d : d);
    }
    rs[a] = s.s;
    rc[a] = s.c;
  }
  nacc t = {0, 0};
  for (int64_t a = 0; a < na; ++a) {
    nadd(&t, rs[a]);
    nadd(&t, rc[a]);
  }
  free(rs);
  free(rc);
  free(X);
  free(Y);
  free(act);
  return nval(&t);
}

/* Hessian of E_sub over the active coordinates applied to (vx, vy) (length
 * na): (Hv)_i = sum_{j != i} K(d_ij)(v_i - v_j), v_j = 0 for frozen j. */
void orc_esub_hvp(int64_t n, const double *x, const double *y, int64_t na,
                  const int32_t *idx, const double *xa, const double *ya,
                  const double *vx, const double *vy, double *hx, double *hy) {
  double *X, *Y;
  unsigned char *act;
  place(n, x, y, na, idx, xa, ya, &X, &Y, &act);
  double *VX = (double *)calloc((size_t)n, sizeof(double));
  double *VY = (double *)calloc((size_t)n, sizeof(double));
  for (int64_t a = 0; a < na; ++a) {
    VX[idx[a]] = vx[a];
    VY[idx[a]] = vy[a];
  }
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < na; ++a) {
    const int64_t i = idx[a];
    nacc ax = {0, 0}, ay = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = X[i] - X[j], dy = Y[i] - Y[j];
      double wx = VX[i] - VX[j], wy = VY[i] - VY[j];
      double r2 = dx * dx + dy * dy;
      double r = sqrt(r2);
      double i3 = 1.0 / (r2 * r);
      double i5 = i3 / r2;
      double dw = dx * wx + dy * wy;
      nadd(&ax, 3.0 * dx * dw * i5 - wx * i3);
      nadd(&ay, 3.0 * dy * dw * i5 - wy * i3);
    }
    hx[a] = nval(&ax);
    hy[a] = nval(&ay);
  }
  free(VX);
  free(VY);
  free(X);
  free(Y);
  free(act);
}

/* ------------------------------------------------------------- hard wall -- */
/* Eq. 3 as a feasible set |r| <= 1.  A charge is on the wall when
 * |r| >= 1 - 1e-14; it is held by the wall (constrained) when the gradient
 * points inward there (g . r_hat < 0, i.e. the force pushes outward).  For a
 * held charge the reduced gradient is the tangential part of g; otherwise it
 * is g.  cons[i] = 1 for held charges.  Returns max_i |reduced g| (inf-norm
 * over the 2na components). */
/* Border-interior variant (Sec. II.B): pin[a] != 0 marks a boundary charge,
 * pinned to the unit circle (always held, reduced gradient = its tangential
 * part); every other charge has its wall at radius sigma (on the wall when
 * |r| >= sigma (1 - 1e-14)).  pin = NULL and sigma = 1 give the hard wall. */
double orc_reduce_grad_bi(int64_t na, const double *xa, const double *ya, const double *gx,
                          const double *gy, const int32_t *pin, double sigma, double *tx,
                          double *ty, int32_t *cons) {
  double m = 0.0;
  for (int64_t a = 0; a < na; ++a) {
    double r = sqrt(xa[a] * xa[a] + ya[a] * ya[a]);
    double ox = gx[a], oy = gy[a];
    int c = 0;
    const int pinned = pin && pin[a];
    if (pinned || r >= sigma * (1.0 - 1e-14)) {
      double ux = xa[a] / r, uy = ya[a] / r;
      double gr = gx[a] * ux + gy[a] * uy;
      if (pinned || gr < 0.0) {
        ox = gx[a] - gr * ux;
        oy = gy[a] - gr * uy;
        c = 1;
      }
    }
    if (tx) tx[a] = ox;
    if (ty) ty[a] = oy;
    if (cons) cons[a] = c;
    if (fabs(ox) > m) m = fabs(ox);
    if (fabs(oy) > m) m = fabs(oy);
  }
  return m;
}

double orc_reduce_grad(int64_t na, const double *xa, const double *ya, const double *gx,
                       const double *gy, double *tx, double *ty, int32_t *cons) {
  return orc_reduce_grad_bi(na, xa, ya, gx, gy, NULL, 1.0, tx, ty, cons);
}

/* The constraint of one relax: pinned boundary charges and the interior wall. */
typedef struct {
  const int32_t *pin;
  double sigma;
} wall_t;

/* Feasible projection: a pinned charge onto the unit circle, any other
 * charge beyond sigma onto the circle of radius sigma. */
static void project(int64_t na, double *xa, double *ya, const wall_t *w) {
  for (int64_t a = 0; a < na; ++a) {
    double r = sqrt(xa[a] * xa[a] + ya[a] * ya[a]);
    if (w->pin && w->pin[a]) {
      if (r > 0.0) {
        xa[a] /= r;
        ya[a] /= r;
      }
    } else if (r > w->sigma) {
      xa[a] *= w->sigma / r;
      ya[a] *= w->sigma / r;
    }
  }
}

/* ----------------------------------------------------------------- relax -- */
typedef struct {
  int32_t max_iter;    /* outer iterations (L-BFGS + Newton) */
  int32_t lbfgs_m;     /* L-BFGS memory */
  double gtol;         /* stop when inf-norm of the reduced gradient <= gtol */
  double newton_tol;   /* switch to truncated Newton below this inf-norm */
  double step0;        /* largest displacement of an L-BFGS trial step */
  int32_t cg_max;      /* CG iterations per Newton step */
} orc_relax_opts;

typedef struct {
  int32_t iters, newton_steps, status; /* 0 converged, 1 iteration cap, 2 line search failed */
  double gtan_inf;
} orc_relax_stats;

/* Optimisation coordinates: two slots per active charge.  A free charge uses
 * (x, y); a charge held by the wall moves on the circle and uses its polar
 * angle in slot 0 (slot 1 stays zero).  This is the angle parameterisation
 * the paper uses for boundary charges (Sec. II.D, Eq. 10), here applied only
 * to charges the wall actually holds. */
static void to_coords(int64_t na, const double *xa, const double *ya, const double *gx,
                      const double *gy, const int32_t *held, double *gc) {
  for (int64_t a = 0; a < na; ++a) {
    if (held[a]) {
      gc[2 * a] = -gx[a] * ya[a] + gy[a] * xa[a]; /* dE/dtheta = g . (-y, x) */
      gc[2 * a + 1] = 0.0;
    } else {
      gc[2 * a] = gx[a];
      gc[2 * a + 1] = gy[a];
    }
  }
}

/* Position after the coordinate step scale*s: free charges translate (then
 * are projected onto |r| <= 1), held charges rotate by the angle step. */
static void take_step(int64_t na, const double *xa, const double *ya, const int32_t *held,
                      const double *s, double scale, double *nx, double *ny, const wall_t *w) {
  for (int64_t a = 0; a < na; ++a) {
    if (held[a]) {
      double th = scale * s[2 * a];
      double c = cos(th), sn = sin(th);
      nx[a] = xa[a] * c - ya[a] * sn;
      ny[a] = xa[a] * sn + ya[a] * c;
    } else {
      nx[a] = xa[a] + scale * s[2 * a];
      ny[a] = ya[a] + scale * s[2 * a + 1];
    }
  }
  project(na, nx, ny, w);
}

/* Held-set rule of Eq. 3's hard wall: held iff on the wall and g . r_hat < 0;
 * a pinned boundary charge is always held. */
static int update_held(int64_t na, const double *xa, const double *ya, const double *gx,
                       const double *gy, int32_t *held, int32_t *changed, const wall_t *w) {
  int any = 0;
  for (int64_t a = 0; a < na; ++a) {
    double r = sqrt(xa[a] * xa[a] + ya[a] * ya[a]);
    int h = 0;
    if (w->pin && w->pin[a]) h = 1;
    else if (r >= w->sigma * (1.0 - 1e-14)) h = (gx[a] * xa[a] + gy[a] * ya[a]) < 0.0;
    changed[a] = (h != held[a]);
    any |= changed[a];
    held[a] = h;
  }
  return any;
}

/* Tangent-space Hessian in optimisation coordinates: a held charge's angle
 * direction is t = (-y, x) and its second derivative gains -(g . r_hat). */
static void tan_hvp(int64_t n, const double *x, const double *y, int64_t na,
                    const int32_t *idx, const double *xa, const double *ya,
                    const double *gx, const double *gy, const int32_t *held,
                    const double *v, double *out, double *wx, double *wy,
                    double *hx, double *hy) {
  for (int64_t a = 0; a < na; ++a) {
    if (held[a]) {
      wx[a] = -ya[a] * v[2 * a];
      wy[a] = xa[a] * v[2 * a];
    } else {
      wx[a] = v[2 * a];
      wy[a] = v[2 * a + 1];
    }
  }
  orc_esub_hvp(n, x, y, na, idx, xa, ya, wx, wy, hx, hy);
  for (int64_t a = 0; a < na; ++a) {
    if (held[a]) {
      double gr = gx[a] * xa[a] + gy[a] * ya[a];
      out[2 * a] = -ya[a] * hx[a] + xa[a] * hy[a] - gr * v[2 * a];
      out[2 * a + 1] = 0.0;
    } else {
      out[2 * a] = hx[a];
      out[2 * a + 1] = hy[a];
    }
  }
}

static double dot(int64_t m, const double *a, const double *b) {
  nacc s = {0, 0};
  for (int64_t k = 0; k < m; ++k) nadd(&s, a[k] * b[k]);
  return nval(&s);
}

/* Relax the active set idx[0..na) of the frozen snapshot (x, y): on entry
 * (xa, ya) hold the start positions, on exit the relaxed ones.  Objective is
 * E_sub (Eqs. 6-7); constraint |r| <= 1 (Eq. 3).  L-BFGS steps are accepted
 * by an Armijo test on the exact energy change (orc_esub_delta); once the
 * reduced gradient is below newton_tol, truncated-Newton steps solve the
 * tangent-Hessian system by CG and are accepted when the reduced gradient
 * shrinks.  Convergence: inf-norm of the reduced gradient <= gtol. */
void orc_relax_bi(int64_t n, const double *x, const double *y, int64_t na,
                  const int32_t *idx, const int32_t *pin, double sigma, double *xa, double *ya,
                  const orc_relax_opts *o, orc_relax_stats *st) {
  const wall_t wall = {pin, sigma}, *w = &wall;
  const int64_t m2 = 2 * na;
  const int M = o->lbfgs_m > 0 ? o->lbfgs_m : 8;
  double *gc = malloc(sizeof(double) * m2), *gcn = malloc(sizeof(double) * m2);
  double *d = malloc(sizeof(double) * m2), *q = malloc(sizeof(double) * m2);
  double *S = malloc(sizeof(double) * m2 * M), *Yv = malloc(sizeof(double) * m2 * M);
  double *rho = malloc(sizeof(double) * M), *alf = malloc(sizeof(double) * M);
  double *gx = malloc(sizeof(double) * na), *gy = malloc(sizeof(double) * na);
  double *nx = malloc(sizeof(double) * na), *ny = malloc(sizeof(double) * na);
  double *ngx = malloc(sizeof(double) * na), *ngy = malloc(sizeof(double) * na);
  double *wx = malloc(sizeof(double) * na), *wy = malloc(sizeof(double) * na);
  double *hx = malloc(sizeof(double) * na), *hy = malloc(sizeof(double) * na);
  double *cr = malloc(sizeof(double) * m2), *cp = malloc(sizeof(double) * m2);
  double *cHp = malloc(sizeof(double) * m2), *cx = malloc(sizeof(double) * m2);
  double *X0 = malloc(sizeof(double) * n), *Y0 = malloc(sizeof(double) * n);
  int32_t *held = calloc(na, sizeof(int32_t)), *chg = malloc(sizeof(int32_t) * na);
  int nmem = 0, head = 0;
  st->iters = 0;
  st->newton_steps = 0;
  st->status = 1;

  project(na, xa, ya, w);
  orc_esub(n, x, y, na, idx, xa, ya, gx, gy);
  update_held(na, xa, ya, gx, gy, held, chg, w);
  double gi = orc_reduce_grad_bi(na, xa, ya, gx, gy, pin, sigma, NULL, NULL, NULL);
  to_coords(na, xa, ya, gx, gy, held, gc);

  for (int it = 0; it < o->max_iter; ++it) {
    if (gi <= o->gtol) break;
    st->iters = it + 1;
    int took = 0;
    if (gi <= o->newton_tol) {
      /* truncated Newton: CG on H_tan p = -gc, stop at negative curvature */
      for (int64_t k = 0; k < m2; ++k) {
        cx[k] = 0.0;
        cr[k] = -gc[k];
        cp[k] = cr[k];
      }
      double rr = dot(m2, cr, cr), rr0 = rr;
      for (int c = 0; c < o->cg_max; ++c) {
        tan_hvp(n, x, y, na, idx, xa, ya, gx, gy, held, cp, cHp, wx, wy, hx, hy);
        double pHp = dot(m2, cp, cHp);
        if (pHp <= 0.0) {
          if (c == 0)
            for (int64_t k = 0; k < m2; ++k) cx[k] = cp[k];
          break;
        }
        double al = rr / pHp;
        for (int64_t k = 0; k < m2; ++k) {
          cx[k] += al * cp[k];
          cr[k] -= al * cHp[k];
        }
        double rrn = dot(m2, cr, cr);
        if (rrn <= 1e-10 * rr0) break;
        double be = rrn / rr;
        rr = rrn;
        for (int64_t k = 0; k < m2; ++k) cp[k] = cr[k] + be * cp[k];
      }
      double scale = 1.0;
      for (int h = 0; h < 8 && !took; ++h, scale *= 0.5) {
        take_step(na, xa, ya, held, cx, scale, nx, ny, w);
        orc_esub(n, x, y, na, idx, nx, ny, ngx, ngy);
        double gin = orc_reduce_grad_bi(na, nx, ny, ngx, ngy, pin, sigma, NULL, NULL, NULL);
        if (gin < gi) {
          memcpy(xa, nx, sizeof(double) * na);
          memcpy(ya, ny, sizeof(double) * na);
          memcpy(gx, ngx, sizeof(double) * na);
          memcpy(gy, ngy, sizeof(double) * na);
          update_held(na, xa, ya, gx, gy, held, chg, w);
          to_coords(na, xa, ya, gx, gy, held, gc);
          gi = gin;
          took = 1;
          st->newton_steps++;
        }
      }
      nmem = 0;
      head = 0;
      if (took) continue;
    }
    for (int attempt = 0; attempt < 2 && !took; ++attempt) {
      /* two-loop recursion on the coordinate gradient */
      memcpy(q, gc, sizeof(double) * m2);
      for (int k = 0; k < nmem; ++k) {
        int s = (head - 1 - k + M) % M;
        alf[s] = rho[s] * dot(m2, S + (int64_t)s * m2, q);
        for (int64_t t = 0; t < m2; ++t) q[t] -= alf[s] * Yv[(int64_t)s * m2 + t];
      }
      double gam = 0.0;
      if (nmem > 0) {
        int s = (head - 1 + M) % M;
        double yy = dot(m2, Yv + (int64_t)s * m2, Yv + (int64_t)s * m2);
        if (rho[s] > 0.0 && yy > 0.0) gam = 1.0 / (rho[s] * yy);
      }
      if (gam <= 0.0) gam = o->step0 / gi;
      for (int64_t t = 0; t < m2; ++t) q[t] *= gam;
      for (int k = nmem - 1; k >= 0; --k) {
        int s = (head - 1 - k + M) % M;
        double be = rho[s] * dot(m2, Yv + (int64_t)s * m2, q);
        for (int64_t t = 0; t < m2; ++t) q[t] += (alf[s] - be) * S[(int64_t)s * m2 + t];
      }
      for (int64_t t = 0; t < m2; ++t) d[t] = -q[t];
      if (dot(m2, d, gc) >= 0.0)
        for (int64_t t = 0; t < m2; ++t) d[t] = -gc[t] * (o->step0 / gi);
      /* cap the largest displacement of a trial step at step0 */
      double dm = 0.0;
      for (int64_t a = 0; a < na; ++a) {
        double l = held[a] ? fabs(d[2 * a]) : sqrt(d[2 * a] * d[2 * a] + d[2 * a + 1] * d[2 * a + 1]);
        if (l > dm) dm = l;
      }
      if (dm > o->step0)
        for (int64_t t = 0; t < m2; ++t) d[t] *= o->step0 / dm;
      /* backtracking with an Armijo test on the exact energy change */
      memcpy(X0, x, sizeof(double) * n);
      memcpy(Y0, y, sizeof(double) * n);
      for (int64_t a = 0; a < na; ++a) {
        X0[idx[a]] = xa[a];
        Y0[idx[a]] = ya[a];
      }
      double al = 1.0;
      for (int ls = 0; ls < 40; ++ls, al *= 0.5) {
        take_step(na, xa, ya, held, d, al, nx, ny, w);
        double pred = 0.0;
        for (int64_t a = 0; a < na; ++a) {
          if (held[a]) pred += gc[2 * a] * al * d[2 * a];
          else pred += gx[a] * (nx[a] - xa[a]) + gy[a] * (ny[a] - ya[a]);
        }
        if (pred >= 0.0) continue;
        double dE = orc_esub_delta(n, X0, Y0, na, idx, nx, ny);
        if (dE <= 1e-4 * pred) {
          took = 1;
          break;
        }
      }
      if (!took) {
        if (nmem > 0) {
          nmem = 0;
          head = 0;
          continue;
        }
        break;
      }
      orc_esub(n, x, y, na, idx, nx, ny, ngx, ngy);
      /* secant pair in the coordinates of the step just taken */
      to_coords(na, nx, ny, ngx, ngy, held, gcn);
      double *sv = S + (int64_t)head * m2, *yv = Yv + (int64_t)head * m2;
      for (int64_t a = 0; a < na; ++a) {
        if (held[a]) {
          sv[2 * a] = al * d[2 * a];
          sv[2 * a + 1] = 0.0;
        } else {
          sv[2 * a] = nx[a] - xa[a];
          sv[2 * a + 1] = ny[a] - ya[a];
        }
      }
      for (int64_t t = 0; t < m2; ++t) yv[t] = gcn[t] - gc[t];
      memcpy(xa, nx, sizeof(double) * na);
      memcpy(ya, ny, sizeof(double) * na);
      memcpy(gx, ngx, sizeof(double) * na);
      memcpy(gy, ngy, sizeof(double) * na);
      double sy = dot(m2, sv, yv);
      double ss = dot(m2, sv, sv), yy = dot(m2, yv, yv);
      if (sy > 1e-12 * sqrt(ss * yy)) {
        rho[head] = 1.0 / sy;
        head = (head + 1) % M;
        if (nmem < M) nmem++;
      }
      if (update_held(na, xa, ya, gx, gy, held, chg, w)) {
        /* a charge changed coordinates: drop its components from the history */
        for (int k = 0; k < nmem; ++k) {
          int s = (head - 1 - k + M) % M;
          double *sk = S + (int64_t)s * m2, *yk = Yv + (int64_t)s * m2;
          for (int64_t a = 0; a < na; ++a)
            if (chg[a]) sk[2 * a] = sk[2 * a + 1] = yk[2 * a] = yk[2 * a + 1] = 0.0;
          double syk = dot(m2, sk, yk);
          rho[s] = syk > 0.0 ? 1.0 / syk : 0.0;
        }
      }
      to_coords(na, xa, ya, gx, gy, held, gc);
      gi = orc_reduce_grad_bi(na, xa, ya, gx, gy, pin, sigma, NULL, NULL, NULL);
    }
    if (!took) {
      st->status = 2;
      break;
    }
  }
  if (gi <= o->gtol) st->status = 0;
  st->gtan_inf = gi;
  free(gc); free(gcn); free(d); free(q); free(S); free(Yv); free(rho); free(alf);
  free(gx); free(gy); free(nx); free(ny); free(ngx); free(ngy); free(wx); free(wy);
  free(hx); free(hy); free(cr); free(cp); free(cHp); free(cx); free(X0); free(Y0);
  free(held); free(chg);
}

void orc_relax(int64_t n, const double *x, const double *y, int64_t na,
               const int32_t *idx, double *xa, double *ya, const orc_relax_opts *o,
               orc_relax_stats *st) {
  orc_relax_bi(n, x, y, na, idx, NULL, 1.0, xa, ya, o, st);
}

/* ------------------------------------------------------- (t, u) coordinates -- */
/* Sec. II.D: an interior charge at (t, u) sits at r (cos u, sin u) with
 * r = sigma sin^2 t; a boundary charge at (cos u, sin u).  Chain rule:
 *   Eq. 8:  dE/dt = (dE/dx cos u + dE/dy sin u) sigma sin 2t
 *   Eq. 9:  dE/du = -dE/dx r sin u + dE/dy r cos u
 *   Eq. 10: dE/du = -dE/dx sin u + dE/dy cos u   (boundary, r = 1)
 * kind[a]: 0 Cartesian (x, y), 1 boundary (u), 2 interior (t, u). */
static void tu_pos(int64_t na, const int32_t *kind, double sigma, const double *c, double *xa,
                   double *ya) {
  for (int64_t a = 0; a < na; ++a) {
    if (kind[a] == 2) {
      double r = sigma * sin(c[2 * a]) * sin(c[2 * a]);
      xa[a] = r * cos(c[2 * a + 1]);
      ya[a] = r * sin(c[2 * a + 1]);
    } else if (kind[a] == 1) {
      xa[a] = cos(c[2 * a]);
      ya[a] = sin(c[2 * a]);
    } else {
      xa[a] = c[2 * a];
      ya[a] = c[2 * a + 1];
    }
  }
}

/* Gradient in the coordinates c from the Cartesian gradient (gx, gy). */
void orc_tu_grad(int64_t na, const int32_t *kind, double sigma, const double *c,
                 const double *gx, const double *gy, double *gc) {
  for (int64_t a = 0; a < na; ++a) {
    if (kind[a] == 2) {
      double t = c[2 * a], u = c[2 * a + 1];
      double r = sigma * sin(t) * sin(t);
      gc[2 * a] = (gx[a] * cos(u) + gy[a] * sin(u)) * sigma * sin(2.0 * t);
      gc[2 * a + 1] = -gx[a] * r * sin(u) + gy[a] * r * cos(u);
    } else if (kind[a] == 1) {
      double u = c[2 * a];
      gc[2 * a] = -gx[a] * sin(u) + gy[a] * cos(u);
      gc[2 * a + 1] = 0.0;
    } else {
      gc[2 * a] = gx[a];
      gc[2 * a + 1] = gy[a];
    }
  }
}

/* Largest Cartesian displacement of the coordinate step d (to first order). */
static double tu_step_len(int64_t na, const int32_t *kind, double sigma, const double *c,
                          const double *d) {
  double m = 0.0;
  for (int64_t a = 0; a < na; ++a) {
    double l;
    if (kind[a] == 2) {
      double t = c[2 * a];
      double lt = sigma * sin(2.0 * t) * d[2 * a], lu = sigma * sin(t) * sin(t) * d[2 * a + 1];
      l = sqrt(lt * lt + lu * lu);
    } else if (kind[a] == 1) {
      l = fabs(d[2 * a]);
    } else {
      l = sqrt(d[2 * a] * d[2 * a] + d[2 * a + 1] * d[2 * a + 1]);
    }
    if (l > m) m = l;
  }
  return m;
}

/* Relaxation in the coordinates of Sec. II.D: boundary charges (pin[a] != 0)
 * by their angle, interior charges by (t, u); interior charges starting
 * within 1e-3 sigma of the centre keep (x, y) (at r = 0 the derivatives of
 * Eqs. 8-9 vanish for any force) and are projected onto |r| <= sigma after a
 * step; t starts at most pi/2 - 1e-8 (at t = pi/2, on the wall, dE/dt
 * vanishes as well, and a charge pushed inward could not leave).  L-BFGS with H0 = gamma I (gamma = s.y / y.y of the newest pair) and
 * backtracking: Armijo on the exact energy change while that change exceeds
 * the rounding of E_sub (1e-14 |E_sub|; a boundary charge evaluated at
 * (cos u, sin u) sits an ulp off the circle, which with its radial force
 * alone moves E by more than a converged step does), below it a
 * derivative-only test (the directional derivative at the trial at most 0.9
 * of the one at the start in magnitude).  Stops when the inf-norm of the
 * reduced Cartesian gradient (orc_reduce_grad_bi) is below gtol.  On entry
 * (xa, ya) hold the start, on exit the relaxed positions. */
void orc_relax_tu(int64_t n, const double *x, const double *y, int64_t na, const int32_t *idx,
                  const int32_t *pin, double sigma, double *xa, double *ya,
                  const orc_relax_opts *o, orc_relax_stats *st) {
  const wall_t wall = {pin, sigma}, *w = &wall;
  const int64_t m2 = 2 * na;
  const int M = o->lbfgs_m > 0 ? o->lbfgs_m : 8;
  int32_t *kind = malloc(sizeof(int32_t) * na);
  double *c = malloc(sizeof(double) * m2), *cn = malloc(sizeof(double) * m2);
  double *gc = malloc(sizeof(double) * m2), *gcn = malloc(sizeof(double) * m2);
  double *d = malloc(sizeof(double) * m2), *q = malloc(sizeof(double) * m2);
  double *S = malloc(sizeof(double) * m2 * M), *Yv = malloc(sizeof(double) * m2 * M);
  double *rho = malloc(sizeof(double) * M), *alf = malloc(sizeof(double) * M);
  double *gx = malloc(sizeof(double) * na), *gy = malloc(sizeof(double) * na);
  double *nx = malloc(sizeof(double) * na), *ny = malloc(sizeof(double) * na);
  double *ngx = malloc(sizeof(double) * na), *ngy = malloc(sizeof(double) * na);
  double *X0 = malloc(sizeof(double) * n), *Y0 = malloc(sizeof(double) * n);
  int nmem = 0, head = 0;
  st->iters = 0;
  st->newton_steps = 0;
  st->status = 1;

  project(na, xa, ya, w);
  for (int64_t a = 0; a < na; ++a) {
    double r = sqrt(xa[a] * xa[a] + ya[a] * ya[a]);
    if (pin && pin[a]) {
      kind[a] = 1;
      c[2 * a] = atan2(ya[a], xa[a]);
      c[2 * a + 1] = 0.0;
    } else if (r >= 1e-3 * sigma) {
      /* at t = pi/2 dE/dt vanishes for any force: start at most pi/2 - 1e-8 */
      kind[a] = 2;
      c[2 * a] = fmin(asin(sqrt(fmin(1.0, r / sigma))), 0.5 * M_PI - 1e-8);
      c[2 * a + 1] = atan2(ya[a], xa[a]);
    } else {
      kind[a] = 0;
      c[2 * a] = xa[a];
      c[2 * a + 1] = ya[a];
    }
  }
  tu_pos(na, kind, sigma, c, xa, ya);
  double Ecur = orc_esub(n, x, y, na, idx, xa, ya, gx, gy);
  orc_tu_grad(na, kind, sigma, c, gx, gy, gc);
  double gi = orc_reduce_grad_bi(na, xa, ya, gx, gy, pin, sigma, NULL, NULL, NULL);

  for (int it = 0; it < o->max_iter; ++it) {
    if (gi <= o->gtol) break;
    st->iters = it + 1;
    int took = 0;
    for (int attempt = 0; attempt < 2 && !took; ++attempt) {
      memcpy(q, gc, sizeof(double) * m2);
      for (int k = 0; k < nmem; ++k) {
        int s = (head - 1 - k + M) % M;
        alf[s] = rho[s] * dot(m2, S + (int64_t)s * m2, q);
        for (int64_t t = 0; t < m2; ++t) q[t] -= alf[s] * Yv[(int64_t)s * m2 + t];
      }
      double gam = 0.0;
      if (nmem > 0) {
        int s = (head - 1 + M) % M;
        double yy = dot(m2, Yv + (int64_t)s * m2, Yv + (int64_t)s * m2);
        if (rho[s] > 0.0 && yy > 0.0) gam = 1.0 / (rho[s] * yy);
      }
      for (int64_t t = 0; t < m2; ++t) q[t] *= gam;
      for (int k = nmem - 1; k >= 0; --k) {
        int s = (head - 1 - k + M) % M;
        double be = rho[s] * dot(m2, Yv + (int64_t)s * m2, q);
        for (int64_t t = 0; t < m2; ++t) q[t] += (alf[s] - be) * S[(int64_t)s * m2 + t];
      }
      for (int64_t t = 0; t < m2; ++t) d[t] = -q[t];
      if (!(gam > 0.0) || dot(m2, d, gc) >= 0.0) {
        /* steepest descent scaled to a first step of step0 */
        double l = tu_step_len(na, kind, sigma, c, gc);
        for (int64_t t = 0; t < m2; ++t) d[t] = l > 0.0 ? -gc[t] * (o->step0 / l) : 0.0;
      }
      double dm = tu_step_len(na, kind, sigma, c, d);
      if (dm > o->step0)
        for (int64_t t = 0; t < m2; ++t) d[t] *= o->step0 / dm;
      memcpy(X0, x, sizeof(double) * n);
      memcpy(Y0, y, sizeof(double) * n);
      for (int64_t a = 0; a < na; ++a) {
        X0[idx[a]] = xa[a];
        Y0[idx[a]] = ya[a];
      }
      double pred0 = dot(m2, gc, d);
      double al = 1.0;
      for (int ls = 0; ls < 40 && pred0 < 0.0; ++ls, al *= 0.5) {
        for (int64_t t = 0; t < m2; ++t) cn[t] = c[t] + al * d[t];
        tu_pos(na, kind, sigma, cn, nx, ny);
        for (int64_t a = 0; a < na; ++a)
          if (kind[a] == 0) {  /* a Cartesian charge stays within sigma */
            double r = sqrt(nx[a] * nx[a] + ny[a] * ny[a]);
            if (r > sigma) {
              nx[a] *= sigma / r;
              ny[a] *= sigma / r;
              cn[2 * a] = nx[a];
              cn[2 * a + 1] = ny[a];
            }
          }
        double dE = orc_esub_delta(n, X0, Y0, na, idx, nx, ny);
        if (fabs(dE) > 1e-14 * fabs(Ecur)) {
          if (dE <= 1e-4 * al * pred0) {
            took = 1;
            break;
          }
        } else {
          orc_esub(n, x, y, na, idx, nx, ny, ngx, ngy);
          orc_tu_grad(na, kind, sigma, cn, ngx, ngy, gcn);
          if (dot(m2, gcn, d) <= 0.9 * fabs(pred0)) {
            took = 1;
            break;
          }
        }
      }
      if (!took) {
        if (nmem > 0) {
          nmem = 0;
          head = 0;
          continue;
        }
        break;
      }
      Ecur = orc_esub(n, x, y, na, idx, nx, ny, ngx, ngy);
      orc_tu_grad(na, kind, sigma, cn, ngx, ngy, gcn);
      double *sv = S + (int64_t)head * m2, *yv = Yv + (int64_t)head * m2;
      for (int64_t t = 0; t < m2; ++t) {
        sv[t] = cn[t] - c[t];
        yv[t] = gcn[t] - gc[t];
      }
      double sy = dot(m2, sv, yv), ss = dot(m2, sv, sv), yy = dot(m2, yv, yv);
      if (sy > 1e-12 * sqrt(ss * yy)) {
        rho[head] = 1.0 / sy;
        head = (head + 1) % M;
        if (nmem < M) nmem++;
      }
      memcpy(c, cn, sizeof(double) * m2);
      memcpy(gc, gcn, sizeof(double) * m2);
      memcpy(xa, nx, sizeof(double) * na);
      memcpy(ya, ny, sizeof(double) * na);
      memcpy(gx, ngx, sizeof(double) * na);
      memcpy(gy, ngy, sizeof(double) * na);
      gi = orc_reduce_grad_bi(na, xa, ya, gx, gy, pin, sigma, NULL, NULL, NULL);
    }
    if (!took) {
      st->status = 2;
      break;
    }
  }
  if (gi <= o->gtol) st->status = 0;
  st->gtan_inf = gi;
  free(kind); free(c); free(cn); free(gc); free(gcn); free(d); free(q); free(S); free(Yv);
  free(rho); free(alf); free(gx); free(gy); free(nx); free(ny); free(ngx); free(ngy);
  free(X0); free(Y0);
}
