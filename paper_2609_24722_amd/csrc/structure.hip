// Structure analysis of a configuration (paper Sec. III: Voronoi
// coordination, the bond-orientational order psi_6, the radial density).
//
// Voronoi cells.  The charges are binned on a uniform grid of cells about
// one mean spacing wide (counting sort; each cell's list is then put in
// index order, so everything downstream is deterministic).  One thread per
// charge i clips a large square around r_i by the bisector half-plane of
// every charge j in the (2R+1)^2 cells around its own (Sutherland-Hodgman in
// coordinates relative to r_i, FP64); each polygon edge remembers the charge
// whose bisector made it.  A charge j outside the searched block lies
// farther than its distance D from r_i (D: the block's margin around r_i,
// unbounded where the block reaches the grid's edge); it can cut a vertex v
// only if |r_j - r_i| < 2|v|.  So a bounded cell is final when every vertex
// satisfies 2|v| <= D; otherwise the search widens (k_voronoi).  Charges on
// the convex hull (host code, monotone chain) have unbounded cells and report
// z = -2.
// z_i = number of bisector edges = Voronoi (Delaunay) neighbours;
// psi_6(i) = (1/z_i) sum_j u_ij^6, u_ij = (r_j - r_i)/|r_j - r_i| as a complex
// number.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace cd {

constexpr int kVorR = 2;       // cells searched on each side of the charge's cell
constexpr int kVorMaxV = 48;   // polygon vertices
constexpr double kVorBox = 4.0;
constexpr double kGridL = 1.0 + 1e-9;  // the grid covers [-L, L]^2
constexpr int kScanT = 1024;

struct Grid {
  int G;       // cells per side
  double c;    // cell width
};

__host__ __device__ inline Grid make_grid(int64_t n) {
  const double h = sqrt(2.0 * 3.141592653589793 / (sqrt(3.0) * (double)n));
  double g = floor(2.0 * kGridL / h);
  if (g < 1.0) g = 1.0;
  if (g > 4096.0) g = 4096.0;
  Grid q;
  q.G = (int)g;
  q.c = 2.0 * kGridL / q.G;
  return q;
}

size_t structure_workspace_bytes(int64_t n) {
  const Grid g = make_grid(n);
  const size_t cells = (size_t)g.G * g.G;
  Carve cv;
  cv.take<int32_t>(cells + 1);  // counts, then starts
  cv.take<int32_t>(cells);      // fill cursors
  cv.take<int32_t>((size_t)n);  // cell of each charge
  cv.take<int32_t>((size_t)n);  // charges by cell
  cv.take<int32_t>((size_t)n);  // convex-hull flags
  return cv.off + 256;
}

__device__ __forceinline__ int cell_coord(double v, const Grid& g) {
  int k = (int)floor((v + kGridL) / g.c);
  return k < 0 ? 0 : (k >= g.G ? g.G - 1 : k);
}

__global__ void k_fill_int(int32_t* __restrict__ a, int m, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) a[i] = v;
}

__global__ void k_cell_count(const double* __restrict__ x, const double* __restrict__ y, int n,
                             Grid g, int32_t* __restrict__ count, int32_t* __restrict__ cell) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cell_coord(y[i], g) * g.G + cell_coord(x[i], g);
  cell[i] = c;
  atomicAdd(&count[c], 1);
}

// Exclusive scan of m counts in place (one workgroup, chunks of kScanT with a
// running carry); a[m] receives the total.
__global__ __launch_bounds__(kScanT) void k_cell_scan(int32_t* __restrict__ a, int m) {
  __shared__ int32_t ws[kScanT / 64];
  int carry = 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c0 = 0; c0 < m; c0 += kScanT) {
    const int i = c0 + threadIdx.x;
    const int v = i < m ? a[i] : 0;
    int s = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int u = __shfl_up(s, off, 64);
      if (lane >= off) s += u;
    }
    if (lane == 63) ws[w] = s;
    __syncthreads();
    int before = 0, total = 0;
    for (int q = 0; q < kScanT / 64; ++q) {
      before += q < w ? ws[q] : 0;
      total += ws[q];
    }
    __syncthreads();
    if (i < m) a[i] = carry + before + s - v;
    carry += total;
  }
  if (threadIdx.x == 0) a[m] = carry;
}

__global__ void k_cell_fill(int n, const int32_t* __restrict__ cell,
                            const int32_t* __restrict__ start, int32_t* __restrict__ cursor,
                            int32_t* __restrict__ slot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cell[i];
  slot[start[c] + atomicAdd(&cursor[c], 1)] = i;
}

// Each cell's charges in increasing index order (insertion sort; cells hold
// a handful of charges).
__global__ void k_cell_sort(int m, const int32_t* __restrict__ start, int32_t* __restrict__ slot) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  const int a = start[c], b = start[c + 1];
  for (int k = a + 1; k < b; ++k) {
    const int v = slot[k];
    int q = k - 1;
    while (q >= a && slot[q] > v) {
      slot[q + 1] = slot[q];
      --q;
    }
    slot[q + 1] = v;
  }
}

// Clip the square of half-width B around r_i by the bisectors of the charges
// in cells [x0, x1] x [y0, y1], taken ring by ring around the home cell
// (cx, cy) so that near charges cut first; a charge of ring k >= 1 lies at
// least (k - 1) c from r_i and can cut only vertices farther than half that,
// so the rings stop once (k - 1) c >= 2 max|v|.  Returns the vertex count
// (kVorMaxV + 1 on overflow) with the polygon in buffer `cur`.
__device__ __forceinline__ bool clip_one(double dx, double dy, int j, int& nv, int& cur,
                                         double (&px)[2][kVorMaxV], double (&py)[2][kVorMaxV],
                                         int (&lab)[2][kVorMaxV]) {
  const double hd = 0.5 * (dx * dx + dy * dy);
  if (!(hd > 0.0)) return true;  // a coincident charge has no bisector
  // f(v) = v.d - |d|^2/2 <= 0 keeps v
  bool any_out = false;
  for (int q = 0; q < nv; ++q) any_out |= px[cur][q] * dx + py[cur][q] * dy - hd > 0.0;
  if (!any_out) return true;
  const int nx = cur ^ 1;
  int m = 0;
  for (int q = 0; q < nv; ++q) {
    const int r = q + 1 == nv ? 0 : q + 1;
    const double ax = px[cur][q], ay = py[cur][q], bx = px[cur][r], by = py[cur][r];
    const double fa = ax * dx + ay * dy - hd, fb = bx * dx + by * dy - hd;
    if (fa <= 0.0) {
      if (m < kVorMaxV) {
        px[nx][m] = ax;
        py[nx][m] = ay;
        lab[nx][m] = lab[cur][q];
      }
      ++m;
      if (fb > 0.0) {
        const double t = fa / (fa - fb);
        if (m < kVorMaxV) {
          px[nx][m] = ax + t * (bx - ax);
          py[nx][m] = ay + t * (by - ay);
          lab[nx][m] = j;
        }
        ++m;
      }
    } else if (fb <= 0.0) {
      const double t = fa / (fa - fb);
      if (m < kVorMaxV) {
        px[nx][m] = ax + t * (bx - ax);
        py[nx][m] = ay + t * (by - ay);
        lab[nx][m] = lab[cur][q];
      }
      ++m;
    }
  }
  cur = nx;
  if (m > kVorMaxV) return false;
  nv = m;
  return true;
}

// Farthest distance from r_i of a point that could cut vertex v (relative to
// r_i): such a charge lies in the disk about V = r_i + v through r_i (radius
// |v|) and in the disk of radius Rb about the origin that holds every
// charge.  The farthest point of that lens from r_i is the point of circle V
// opposite r_i, the point of circle Rb opposite r_i, or one of the two circle
// intersections (each candidate counted when it lies in the other disk; the
// tests allow slack, which can only add candidates).  Without the Rb disk the
// bound is 2|v|; with it, the long cells of charges next to the hull, whose
// far vertices lie well outside the disk, certify at a short range.
__device__ double lens_reach(double cx, double cy, double vx, double vy, double Rb) {
  const double rho2 = vx * vx + vy * vy, rho = sqrt(rho2);
  const double Vx = cx + vx, Vy = cy + vy;
  const double Ax = Vx + vx, Ay = Vy + vy;
  const double Rb2 = Rb * Rb;
  if (Ax * Ax + Ay * Ay <= Rb2 * (1.0 + 1e-9)) return 2.0 * rho;
  double M = 0.0;
  const double cn = sqrt(cx * cx + cy * cy);
  if (cn > 0.0) {
    const double ex = -Rb * cx / cn - Vx, ey = -Rb * cy / cn - Vy;
    if (ex * ex + ey * ey <= rho2 * (1.0 + 1e-9)) M = Rb + cn;
  } else {
    M = Rb;
  }
  const double d2 = Vx * Vx + Vy * Vy, d = sqrt(d2);
  if (d > 0.0) {
    const double a = (Rb2 - rho2 + d2) / (2.0 * d);
    const double hh = Rb2 - a * a;
    if (hh > -1e-9 * Rb2) {
      const double h = sqrt(fmax(hh, 0.0));
      const double ux = Vx / d, uy = Vy / d;
      const double p1x = a * ux - h * uy - cx, p1y = a * uy + h * ux - cy;
      const double p2x = a * ux + h * uy - cx, p2y = a * uy - h * ux - cy;
      M = fmax(M, fmax(sqrt(p1x * p1x + p1y * p1y), sqrt(p2x * p2x + p2y * p2y)));
    }
  }
  return M;
}
// lens_reach with slack for rounding, over the polygon's vertices
__device__ double poly_reach(double xi, double yi, const double* px, const double* py, int nv,
                             double Rb) {
  double M = 0.0;
  for (int q = 0; q < nv; ++q) M = fmax(M, lens_reach(xi, yi, px[q], py[q], Rb));
  return M * (1.0 + 1e-9) + 1e-12;
}

__device__ int clip_cell(const double* __restrict__ x, const double* __restrict__ y, int i,
                         double xi, double yi, const Grid& g, const int32_t* __restrict__ start,
                         const int32_t* __restrict__ slot, int cx, int cy, int x0, int x1,
                         int y0, int y1, double B, double Rb, double (&px)[2][kVorMaxV],
                         double (&py)[2][kVorMaxV], int (&lab)[2][kVorMaxV], int& cur) {
  cur = 0;
  int nv = 4;
  px[0][0] = -B; py[0][0] = -B; lab[0][0] = -1;
  px[0][1] = B;  py[0][1] = -B; lab[0][1] = -1;
  px[0][2] = B;  py[0][2] = B;  lab[0][2] = -1;
  px[0][3] = -B; py[0][3] = B;  lab[0][3] = -1;
  const int kmax = max(max(cx - x0, x1 - cx), max(cy - y0, y1 - cy));
  for (int k = 0; k <= kmax; ++k) {
    if (k >= 2 && (k - 1) * g.c >= poly_reach(xi, yi, px[cur], py[cur], nv, Rb)) break;
    for (int qy = max(y0, cy - k); qy <= min(y1, cy + k); ++qy) {
      const bool edge_row = qy == cy - k || qy == cy + k;
      for (int qx = max(x0, cx - k); qx <= min(x1, cx + k); ++qx) {
        if (!edge_row && qx != cx - k && qx != cx + k) continue;  // ring k only
        const int c = qy * g.G + qx;
        for (int t = start[c]; t < start[c + 1]; ++t) {
          const int j = slot[t];
          if (j == i) continue;
          if (!clip_one(x[j] - xi, y[j] - yi, j, nv, cur, px, py, lab)) return kVorMaxV + 1;
        }
      }
    }
  }
  return nv;
}

// Charges on the convex hull (found on the host) have unbounded cells:
// z = -2, psi_6 = 0.  For the others the search widens (2, 6, 18, .. cells
// on each side, then the whole grid) until every vertex's reach (lens_reach)
// is within the block's margin: no charge outside can cut the polygon.  A
// certified polygon with an edge on the square belongs to a cell that
// extends beyond it (a charge next to the hull can have far vertices): the
// square grows to 1e4 once, at the same range; z = -1 if even that does not
// hold it, or if the polygon outgrows its vertex arrays.
__global__ __launch_bounds__(64) void k_voronoi(const double* __restrict__ x,
                                                const double* __restrict__ y, int n, Grid g,
                                                const int32_t* __restrict__ start,
                                                const int32_t* __restrict__ slot,
                                                const int32_t* __restrict__ hullf,
                                                double Rb, int32_t* __restrict__ zout,
                                                double* __restrict__ psi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (hullf[i]) {  // on the convex hull: unbounded cell
    zout[i] = -2;
    if (psi) psi[2 * (size_t)i] = psi[2 * (size_t)i + 1] = 0.0;
    return;
  }
  const double xi = x[i], yi = y[i];
  double px[2][kVorMaxV], py[2][kVorMaxV];
  int lab[2][kVorMaxV];
  const int cx = cell_coord(xi, g), cy = cell_coord(yi, g);
  int R = kVorR, cur = 0, nv = 0, z = -1;
  double B = kVorBox;
  for (;;) {
    const int x0 = max(0, cx - R), x1 = min(g.G - 1, cx + R);
    const int y0 = max(0, cy - R), y1 = min(g.G - 1, cy + R);
    nv = clip_cell(x, y, i, xi, yi, g, start, slot, cx, cy, x0, x1, y0, y1, B, Rb, px, py, lab,
                   cur);
    if (nv > kVorMaxV) break;  // z = -1: more vertices than the polygon holds
    // the searched block's margin around r_i (unbounded where it reaches the grid's edge)
    const double inf = 1e300;
    const double ml = x0 == 0 ? inf : xi - (-kGridL + x0 * g.c);
    const double mr = x1 == g.G - 1 ? inf : (-kGridL + (x1 + 1) * g.c) - xi;
    const double mb = y0 == 0 ? inf : yi - (-kGridL + y0 * g.c);
    const double mt = y1 == g.G - 1 ? inf : (-kGridL + (y1 + 1) * g.c) - yi;
    const double D = fmin(fmin(ml, mr), fmin(mb, mt));
    bool box = false;
    for (int q = 0; q < nv; ++q) box |= lab[cur][q] < 0;
    const bool full = x0 == 0 && y0 == 0 && x1 == g.G - 1 && y1 == g.G - 1;
    if (full || poly_reach(xi, yi, px[cur], py[cur], nv, Rb) <= D) {
      if (!box) {
        z = 0;
        break;
      }
      if (B < 1e4) {
        B = 1e4;
        continue;
      }
      break;  // z = -1
    }
    R *= 3;
  }
  double sre = 0.0, sim = 0.0;
  if (z == 0) {
    for (int q = 0; q < nv; ++q) {
      const int j = lab[cur][q];
      if (j < 0) continue;
      ++z;
      const double dx = x[j] - xi, dy = y[j] - yi;
      const double r = sqrt(dx * dx + dy * dy);
      const double ur = dx / r, ui = dy / r;
      const double u2r = ur * ur - ui * ui, u2i = 2.0 * ur * ui;
      const double u4r = u2r * u2r - u2i * u2i, u4i = 2.0 * u2r * u2i;
      sre += u4r * u2r - u4i * u2i;
      sim += u4r * u2i + u4i * u2r;
    }
  }
  zout[i] = z;
  if (psi) {
    psi[2 * (size_t)i] = z > 0 ? sre / z : 0.0;
    psi[2 * (size_t)i + 1] = z > 0 ? sim / z : 0.0;
  }
}

// Statistics of a coordination result in one workgroup: per thread a strided
// pass in index order, then a tree over the threads, so the sums do not
// depend on timing.  out[0..4]: fractions of the bounded cells with z = 4..8;
// out[5]: mean |psi_6| over the bounded cells; out[6..8]: the counts of
// bounded cells, hull charges and unresolved cells.
__global__ __launch_bounds__(kScanT) void k_structure_stats(const int32_t* __restrict__ z,
                                                            const double* __restrict__ psi6, int n,
                                                            double* __restrict__ out) {
  __shared__ double s_abs[kScanT];
  __shared__ int32_t s_cnt[8][kScanT];
  const int t = threadIdx.x;
  int32_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // z = 4..8, bounded, hull, unresolved
  double a = 0.0;
  for (int i = t; i < n; i += kScanT) {
    const int zi = z[i];
    if (zi >= 0) {
      ++c[5];
      if (zi >= 4 && zi <= 8) ++c[zi - 4];
      if (psi6) {
        const double re = psi6[2 * i], im = psi6[2 * i + 1];
        a += sqrt(re * re + im * im);
      }
    } else if (zi == -2) {
      ++c[6];
    } else {
      ++c[7];
    }
  }
  s_abs[t] = a;
  for (int k = 0; k < 8; ++k) s_cnt[k][t] = c[k];
  __syncthreads();
  for (int w = kScanT / 2; w > 0; w >>= 1) {
    if (t < w) {
      s_abs[t] += s_abs[t + w];
      for (int k = 0; k < 8; ++k) s_cnt[k][t] += s_cnt[k][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const int32_t b = s_cnt[5][0];
    const double inv = b > 0 ? 1.0 / (double)b : 0.0;
    for (int k = 0; k < 5; ++k) out[k] = b > 0 ? (double)s_cnt[k][0] * inv : 0.0;
    out[5] = b > 0 && psi6 ? s_abs[0] / (double)b : 0.0;
    out[6] = (double)b;
    out[7] = (double)s_cnt[6][0];
    out[8] = (double)s_cnt[7][0];
  }
}

#pragma clang fp contract(off)
__global__ void k_radial(const double* __restrict__ x, const double* __restrict__ y, int n,
                         int nbins, int32_t* __restrict__ counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = x[i] * x[i], b = y[i] * y[i];
  const double r = sqrt(a + b);
  const double f = floor(r * (double)nbins);
  int k = f < 0.0 ? 0 : (f >= (double)nbins ? nbins - 1 : (int)f);
  if (!(r == r)) k = nbins - 1;  // NaN
  atomicAdd(&counts[k], 1);
}
#pragma clang fp contract(on)

}  // namespace cd

using namespace cd;

namespace {

// Vertices of the convex hull (Andrew's monotone chain; points on an edge
// between two vertices are not vertices).  flags[i] = 1 for a vertex.
void hull_flags(const std::vector<double>& x, const std::vector<double>& y,
                std::vector<int32_t>& flags) {
  const int n = (int)x.size();
  std::vector<int> o(n);
  for (int i = 0; i < n; ++i) o[i] = i;
  std::sort(o.begin(), o.end(), [&](int a, int b) { return x[a] < x[b] || (x[a] == x[b] && y[a] < y[b]); });
  auto cross = [&](int a, int b, int c) {
    return (x[b] - x[a]) * (y[c] - y[a]) - (y[b] - y[a]) * (x[c] - x[a]);
  };
  std::vector<int> h(2 * (size_t)n + 2);
  int k = 0;
  for (int t = 0; t < n; ++t) {  // lower hull
    while (k >= 2 && cross(h[k - 2], h[k - 1], o[t]) <= 0.0) --k;
    h[k++] = o[t];
  }
  for (int t = n - 2, lo = k + 1; t >= 0; --t) {  // upper hull
    while (k >= lo && cross(h[k - 2], h[k - 1], o[t]) <= 0.0) --k;
    h[k++] = o[t];
  }
  flags.assign(n, 0);
  for (int t = 0; t < k; ++t) flags[h[t]] = 1;
}

}  // namespace

extern "C" {

int voronoi_coordination(const double* x, const double* y, int64_t n, int32_t* z, double* psi6,
                         void* ws, size_t ws_bytes, void* stream) {
  if (!x || !y || !z || n < 1 || n > (1 << 26)) return CD_ERR_INVALID_ARG;
  if (!ws || ws_bytes < structure_workspace_bytes(n)) return CD_ERR_WORKSPACE;
  const Grid g = make_grid(n);
  const int cells = g.G * g.G;
  Carve cv;
  cv.base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  int32_t* start = cv.take<int32_t>((size_t)cells + 1);
  int32_t* cursor = cv.take<int32_t>((size_t)cells);
  int32_t* cell = cv.take<int32_t>((size_t)n);
  int32_t* slot = cv.take<int32_t>((size_t)n);
  int32_t* hullf = cv.take<int32_t>((size_t)n);
  hipStream_t st = (hipStream_t)stream;
  const int nn = (int)n;
  double Rb = 0.0;  // radius of a disk about the origin that holds every charge
  {
    std::vector<double> hx(n), hy(n);
    std::vector<int32_t> hf;
    int rc = hip_status(hipMemcpyAsync(hx.data(), x, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    if (!rc) rc = hip_status(hipMemcpyAsync(hy.data(), y, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    if (!rc) rc = hip_status(hipStreamSynchronize(st));
    if (rc) return rc;
    hull_flags(hx, hy, hf);
    for (int64_t i = 0; i < n; ++i) Rb = fmax(Rb, sqrt(hx[i] * hx[i] + hy[i] * hy[i]));
    Rb = Rb * (1.0 + 1e-12) + 1e-300;
    rc = hip_status(hipMemcpyAsync(hullf, hf.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    if (!rc) rc = hip_status(hipStreamSynchronize(st));  // hf is released on return
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_fill_int, dim3((cells + 256) / 256), dim3(256), 0, st, start, cells + 1, 0);
  hipLaunchKernelGGL(k_fill_int, dim3((cells + 255) / 256), dim3(256), 0, st, cursor, cells, 0);
  hipLaunchKernelGGL(k_cell_count, dim3((nn + 255) / 256), dim3(256), 0, st, x, y, nn, g, start,
                     cell);
  hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(kScanT), 0, st, start, cells);
  hipLaunchKernelGGL(k_cell_fill, dim3((nn + 255) / 256), dim3(256), 0, st, nn, cell, start,
                     cursor, slot);
  hipLaunchKernelGGL(k_cell_sort, dim3((cells + 255) / 256), dim3(256), 0, st, cells, start, slot);
  hipLaunchKernelGGL(k_voronoi, dim3((nn + 63) / 64), dim3(64), 0, st, x, y, nn, g, start, slot,
                     hullf, Rb, z, psi6);
  return hip_status(hipGetLastError());
}

int radial_histogram(const double* x, const double* y, int64_t n, int32_t nbins, int32_t* counts,
                     void* stream) {
  if (!x || !y || !counts || n < 1 || n > (1 << 26) || nbins < 1 || nbins > (1 << 20))
    return CD_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_fill_int, dim3((nbins + 255) / 256), dim3(256), 0, st, counts, nbins, 0);
  hipLaunchKernelGGL(k_radial, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, (int)n,
                     nbins, counts);
  return hip_status(hipGetLastError());
}

int structure_stats(const int32_t* z, const double* psi6, int64_t n, double* out, void* stream) {
  if (!z || !out || n < 1 || n > (1 << 26)) return CD_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_structure_stats, dim3(1), dim3(kScanT), 0, (hipStream_t)stream, z, psi6,
                     (int)n, out);
  return hip_status(hipGetLastError());
}

}  // extern "C"
