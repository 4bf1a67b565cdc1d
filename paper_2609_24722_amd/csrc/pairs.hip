// All-pairs energy, forces and Hessian-vector products for N charges in the
// unit disk (paper Sec. II.A, Eq. 2), and the C-ABI entry points that run
// them: coulomb_energy, coulomb_forces, coulomb_hvp, coulomb_validate.
//
// Pipeline of one call (all on the caller's stream):
//   1. staging     Morton keys of the FP64 positions, a stable radix sort,
//                  gather into sorted SoA arrays padded to whole 64-charge
//                  blocks (128-charge super-blocks for CD_MIXED), per-block
//                  bounding box;
//   2. pair pass   CD_MIXED: symmetric FP32 kernel over super-block pairs
//                  (each unordered pair evaluated once, Newton's third law);
//                  CD_FP64: one-sided FP64 kernel over (i block, j range);
//   3. reduction   fixed-order sums of the partial results, scattered back
//                  to the caller's order; energy by a fixed-shape tree.
#include <map>
#include <mutex>
#include <tuple>

#include "plan.hpp"

namespace cd {

size_t sort_scratch_elems(int n);
int morton_order(const double* x, const double* y, int n, uint32_t* ka, uint32_t* kb,
                 int32_t* va, uint32_t* hist, int32_t* perm, hipStream_t st);

// kRiesz: energy and forces of the Riesz-s generalisation (1/r^s pairs);
// it takes the force path everywhere except the pair arithmetic.
enum Mode { kEnergy = 0, kForces = 1, kHvp = 2, kRiesz = 3 };

// ------------------------------------------------------------------ staging --
// Sorted, padded copies (xs[s] = x[perm[s]] for s < n, pads beyond; v only
// when given) and the bounding box of each block's real charges (+inf..-inf
// for a block of pads only).  One wave per block.
__global__ void k_gather(const double* __restrict__ x, const double* __restrict__ y,
                         const double* __restrict__ vx, const double* __restrict__ vy,
                         const int32_t* __restrict__ perm, int n, int nb,
                         double* __restrict__ xs, double* __restrict__ ys,
                         double* __restrict__ vxs, double* __restrict__ vys,
                         float* __restrict__ box) {
  const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= nb) return;  // whole waves
  const int s = b * kBlk + lane;
  const bool ok = s < n;
  const bool gv = vxs && vx;  // v is gathered only when given
  double xv = pad_x(s - n), yv = 0.0, wx = 0.0, wy = 0.0;
  if (ok) {
    const int p = perm[s];
    xv = x[p];
    yv = y[p];
    if (gv) {
      wx = vx[p];
      wy = vy[p];
    }
  }
  xs[s] = xv;
  ys[s] = yv;
  if (gv) {
    vxs[s] = wx;
    vys[s] = wy;
  }
  const double x0 = wave_min(ok ? xv : 1e300), x1 = wave_max(ok ? xv : -1e300);
  const double y0 = wave_min(ok ? yv : 1e300), y1 = wave_max(ok ? yv : -1e300);
  if (lane == 0) {
    box[4 * b + 0] = (float)x0;
    box[4 * b + 1] = (float)x1;
    box[4 * b + 2] = (float)y0;
    box[4 * b + 3] = (float)y1;
  }
}

// ------------------------------------------------- symmetric FP32 pair pass --
// Work decomposition.  Charges are grouped in super-blocks of NI x 64 (NI =
// kSymBlocks blocks of 64).  Super-blocks I and J = (I + o) mod ns interact
// for offsets o = 1..floor(ns/2) (for even ns the offset ns/2 only from
// I < ns/2): every unordered pair of super-blocks exactly once, the same work
// for every I.  A workgroup of W waves owns super-blocks I = gW..gW+W-1 (one
// per wave; each lane holds one charge of each of the NI blocks) and the
// offsets of chunk c: o = cL+1 .. cL+L.  At time step t wave w handles
// o = cL+1+t, so its j super-block lands in LDS slot w + t of the
// workgroup's window of S = L+W-1 consecutive super-blocks; no two waves
// share a slot in a step and a barrier separates steps, so the j-side sums
// accumulate in LDS without atomics and in a fixed order.  The pairs inside a
// super-block (each block's own pairs and the pairs between its blocks) are
// done by ns more workgroups at the start of the first launch's grid.
//
// A step takes the j super-block one 64-charge block at a time, each lane
// owning one j.  Within each 16-lane row the j data rotate by DPP (row_ror:k
// folded into the subtractions) and the j-side accumulators travel with them
// (row_ror:1 per step), one move serving the lane's NI i charges.  After 16
// steps the rows rotate by a lane permute, four times in all, which covers
// the (NI x 64) x 64 pairs and returns each j accumulator to its own lane.
//
// Precision.  Coordinates are taken relative to the centre of the i block's
// box (FP64 subtraction, then rounded to FP32; the j block is read once for
// each i block), so their rounding error scales with the distance from that
// centre, not with |r|.  A j block whose box lies farther from the i block's
// box than the larger box diagonal gives dx a relative rounding error of at
// most about 2 ulp; for a nearer one the low parts fl32(r - c - hi) are kept
// too, and dx = (hi_j - hi_i) + (lo_j - lo_i) is exact to the FP32 rounding
// of dx itself.  Per block pair the i and j partials are FP32 sums of 64
// terms, folded into FP64 (registers for i, LDS for j).  The total energy is
// summed per workgroup, in a fixed order.
//
// Batches.  The partial sums of one launch cover the chunks c0..c0+nc-1 and
// are reduced before the next launch, so their memory is bounded by the batch
// size Cb, not by the number of chunks C.
constexpr int NI = kSymBlocks;
constexpr int SB = NI * kBlk;  // charges per super-block

struct SymArgs {
  const double* xs;
  const double* ys;
  const double* vxs;
  const double* vys;
  const float* box;
  int ns, npad, W, L, C, G, S;
  int c0, nc, Cb;  // first chunk and chunks of this launch; chunks per batch
  double* ip0;  // i-side partials [Cb][npad]: fx | hx | e_local
  double* ip1;  //                             fy | hy
  double* jp0;  // j-side partials [G*Cb][S][SB]
  double* jp1;
  double* ep;   // per-workgroup energy partials [Cb][G] (total energy)
  double* dp0;  // sums of the pairs inside each super-block [npad]
  double* dp1;
  double* dep;  // their energy, per super-block [ns]
  double diag_scale;  // weight of the ordered within-block energy sum
  float rz_e, rz_s;   // kRiesz: -(s/2) - 1 and s
};

// One charge per lane, relative to a reference point: coordinates (hi, lo)
// and, for Hessian-vector products, v relative to a reference value (hi, lo).
struct Side {
  float xh, yh, xl, yl, vx, vy, vxl, vyl;
};

template <int MODE>
__device__ __forceinline__ Side load_side(const SymArgs& a, size_t s, double cx, double cy,
                                          double cvx, double cvy, bool lo) {
  Side q{};
  const double rx = a.xs[s] - cx, ry = a.ys[s] - cy;
  q.xh = (float)rx;
  q.yh = (float)ry;
  if (lo) {
    q.xl = (float)(rx - (double)q.xh);
    q.yl = (float)(ry - (double)q.yh);
  }
  if (MODE == kHvp) {
    const double wx = a.vxs[s] - cvx, wy = a.vys[s] - cvy;
    q.vx = (float)wx;
    q.vy = (float)wy;
    if (lo) {
      q.vxl = (float)(wx - (double)q.vx);
      q.vyl = (float)(wy - (double)q.vy);
    }
  }
  return q;
}

// The same from FP64 values already loaded (x, y, and v for HVP).
template <int MODE>
__device__ __forceinline__ Side make_side(double x, double y, double vx, double vy, double cx,
                                          double cy, double cvx, double cvy, bool lo) {
  Side q{};
  const double rx = x - cx, ry = y - cy;
  q.xh = (float)rx;
  q.yh = (float)ry;
  if (lo) {
    q.xl = (float)(rx - (double)q.xh);
    q.yl = (float)(ry - (double)q.yh);
  }
  if (MODE == kHvp) {
    const double wx = vx - cvx, wy = vy - cvy;
    q.vx = (float)wx;
    q.vy = (float)wy;
    if (lo) {
      q.vxl = (float)(wx - (double)q.vx);
      q.vyl = (float)(wy - (double)q.vy);
    }
  }
  return q;
}

template <int MODE, bool LOCAL>
struct PairOps {
  // one pair: d = r_j - r_i (FP32), w = v_j - v_i (HVP only)
  // i-side accumulators a0,a1,a2; j-side accumulators b0,b1 (already aligned)
  // re, rs: the Riesz exponents (kRiesz only)
  __device__ __forceinline__ static void apply(float dx, float dy, float wx, float wy, float& a0,
                                               float& a1, float& a2, float& b0, float& b1,
                                               float re, float rs) {
    const float r2 = __builtin_fmaf(dx, dx, dy * dy);
    if (MODE == kRiesz) {
      // q = r^(-s-2) = 2^(re log2 r2); the energy term is q r2 = r^-s.  A pad
      // gives r2 = +inf and q = exactly 0; the clamp keeps 0 * inf out.
      const float q = __builtin_amdgcn_exp2f(re * __builtin_amdgcn_logf(r2));
      a2 = __builtin_fmaf(q, fminf(r2, 1e30f), a2);
      const float c = rs * q;
      a0 = __builtin_fmaf(-dx, c, a0);
      a1 = __builtin_fmaf(-dy, c, a1);
      b0 = __builtin_fmaf(dx, c, b0);
      b1 = __builtin_fmaf(dy, c, b1);
      return;
    }
    const float inv = __builtin_amdgcn_rsqf(r2);
    if (MODE == kEnergy) {
      a2 += inv;
      if (LOCAL) b0 += inv;
    } else if (MODE == kForces) {
      a2 += inv;
      const float i3 = inv * inv * inv;
      a0 = __builtin_fmaf(-dx, i3, a0);
      a1 = __builtin_fmaf(-dy, i3, a1);
      b0 = __builtin_fmaf(dx, i3, b0);
      b1 = __builtin_fmaf(dy, i3, b1);
    } else {
      const float i2 = inv * inv;
      const float i3 = i2 * inv;
      const float q = 3.0f * i3 * i2;
      const float dw = __builtin_fmaf(dx, wx, dy * wy);
      const float s = dw * q;
      const float kx = __builtin_fmaf(dx, s, -wx * i3);
      const float ky = __builtin_fmaf(dy, s, -wy * i3);
      a0 -= kx;
      a1 -= ky;
      b0 += kx;
      b1 += ky;
    }
  }
};

// d = r_j - r_i and w = v_j - v_i for the j data rotated by row_ror:K
// (K = 0: the lane's own j).
template <int MODE, bool NEAR, int K>
__device__ __forceinline__ void diff(const Side& i, const Side& j, float& dx, float& dy,
                                     float& wx, float& wy) {
  auto rot = [](float v) {
    if constexpr (K == 0) return v;
    else return row_ror<K>(v);
  };
  dx = rot(j.xh) - i.xh;
  dy = rot(j.yh) - i.yh;
  if (NEAR) {
    dx += rot(j.xl) - i.xl;
    dy += rot(j.yl) - i.yl;
  }
  wx = 0.f;
  wy = 0.f;
  if (MODE == kHvp) {
    wx = rot(j.vx) - i.vx;
    wy = rot(j.vy) - i.vy;
    if (NEAR) {
      wx += rot(j.vxl) - i.vxl;
      wy += rot(j.vyl) - i.vyl;
    }
  }
}

// Row rotation by 16 lanes (lane q takes lane q + 16) of the j data.
template <int MODE, bool NEAR>
__device__ __forceinline__ void rotate_rows(Side& j, int src) {
  j.xh = __shfl(j.xh, src, 64);
  j.yh = __shfl(j.yh, src, 64);
  if (NEAR) {
    j.xl = __shfl(j.xl, src, 64);
    j.yl = __shfl(j.yl, src, 64);
  }
  if (MODE == kHvp) {
    j.vx = __shfl(j.vx, src, 64);
    j.vy = __shfl(j.vy, src, 64);
    if (NEAR) {
      j.vxl = __shfl(j.vxl, src, 64);
      j.vyl = __shfl(j.vyl, src, 64);
    }
  }
}

// The 64 x 64 pairs of one block pair for the calling lane (one i, one j);
// ONESIDED: the block with itself, ordered pairs, i side only.
template <int MODE, bool LOCAL, bool NEAR, bool ONESIDED>
struct BlockPair {
  __device__ __forceinline__ static void run(const Side& i, Side j, float& a0, float& a1,
                                             float& a2, float& b0, float& b1, int lane,
                                             float re = 0.f, float rs = 0.f) {
    const int src = (lane + 16) & 63;
    float dx, dy, wx, wy;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if (!(ONESIDED && p == 0)) {  // the self pair of a diagonal block is skipped
        diff<MODE, NEAR, 0>(i, j, dx, dy, wx, wy);
        PairOps<MODE, LOCAL>::apply(dx, dy, wx, wy, a0, a1, a2, b0, b1, re, rs);
      }
#define CD_SYM_STEP(K)                                                  \
  {                                                                     \
    diff<MODE, NEAR, K>(i, j, dx, dy, wx, wy);                          \
    if (!ONESIDED) {                                                    \
      b0 = row_ror<1>(b0);                                              \
      if (MODE != kEnergy) b1 = row_ror<1>(b1);                         \
    }                                                                   \
    PairOps<MODE, LOCAL>::apply(dx, dy, wx, wy, a0, a1, a2, b0, b1, re, rs); \
  }
      CD_SYM_STEP(1) CD_SYM_STEP(2) CD_SYM_STEP(3) CD_SYM_STEP(4) CD_SYM_STEP(5)
      CD_SYM_STEP(6) CD_SYM_STEP(7) CD_SYM_STEP(8) CD_SYM_STEP(9) CD_SYM_STEP(10)
      CD_SYM_STEP(11) CD_SYM_STEP(12) CD_SYM_STEP(13) CD_SYM_STEP(14) CD_SYM_STEP(15)
#undef CD_SYM_STEP
      if (!ONESIDED) {
        b0 = row_ror<1>(b0);
        if (MODE != kEnergy) b1 = row_ror<1>(b1);
        b0 = __shfl(b0, src, 64);
        if (MODE != kEnergy) b1 = __shfl(b1, src, 64);
      }
      if (p < 3) rotate_rows<MODE, NEAR>(j, src);
    }
  }
};

// The (NI x 64) x 64 pairs of the lane's NI i charges with one j block; j[q]
// holds the j block relative to the reference point of i block q.  The
// j-side accumulators are shared.
template <int MODE, bool LOCAL, bool NEAR>
struct BlockPairN {
  __device__ __forceinline__ static void run(const Side (&u)[NI], Side (&j)[NI],
                                             float (&acc)[NI][3], float& b0, float& b1,
                                             int lane, float re = 0.f, float rs = 0.f) {
    const int src = (lane + 16) & 63;
    float dx, dy, wx, wy;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
#pragma unroll
      for (int q = 0; q < NI; ++q) {
        diff<MODE, NEAR, 0>(u[q], j[q], dx, dy, wx, wy);
        PairOps<MODE, LOCAL>::apply(dx, dy, wx, wy, acc[q][0], acc[q][1], acc[q][2], b0, b1, re,
                                    rs);
      }
#define CD_SYM_STEPN(K)                                                                     \
  {                                                                                         \
    b0 = row_ror<1>(b0);                                                                    \
    if (MODE != kEnergy) b1 = row_ror<1>(b1);                                               \
    _Pragma("unroll") for (int q = 0; q < NI; ++q) {                                        \
      diff<MODE, NEAR, K>(u[q], j[q], dx, dy, wx, wy);                                      \
      PairOps<MODE, LOCAL>::apply(dx, dy, wx, wy, acc[q][0], acc[q][1], acc[q][2], b0, b1, re, \
                                  rs);                                                      \
    }                                                                                       \
  }
      CD_SYM_STEPN(1) CD_SYM_STEPN(2) CD_SYM_STEPN(3) CD_SYM_STEPN(4) CD_SYM_STEPN(5)
      CD_SYM_STEPN(6) CD_SYM_STEPN(7) CD_SYM_STEPN(8) CD_SYM_STEPN(9) CD_SYM_STEPN(10)
      CD_SYM_STEPN(11) CD_SYM_STEPN(12) CD_SYM_STEPN(13) CD_SYM_STEPN(14) CD_SYM_STEPN(15)
#undef CD_SYM_STEPN
      b0 = row_ror<1>(b0);
      if (MODE != kEnergy) b1 = row_ror<1>(b1);
      b0 = __shfl(b0, src, 64);
      if (MODE != kEnergy) b1 = __shfl(b1, src, 64);
      if (p < 3) {
#pragma unroll
        for (int q = 0; q < NI; ++q) rotate_rows<MODE, NEAR>(j[q], src);
      }
    }
  }
};

// Centre of a box side in FP64; 0 for the empty side of a block of pads.
__device__ __forceinline__ double centre(float lo, float hi) {
  return lo <= hi ? 0.5 * ((double)lo + (double)hi) : 0.0;
}

__device__ __forceinline__ bool boxes_near(const float* box, int I, int J) {
  // gap between the two boxes below the larger box diagonal
  float ix0 = box[4 * I], ix1 = box[4 * I + 1], iy0 = box[4 * I + 2], iy1 = box[4 * I + 3];
  float jx0 = box[4 * J], jx1 = box[4 * J + 1], jy0 = box[4 * J + 2], jy1 = box[4 * J + 3];
  float gx = fmaxf(0.f, fmaxf(jx0 - ix1, ix0 - jx1));
  float gy = fmaxf(0.f, fmaxf(jy0 - iy1, iy0 - jy1));
  float di = (ix1 - ix0) * (ix1 - ix0) + (iy1 - iy0) * (iy1 - iy0);
  float dj = (jx1 - jx0) * (jx1 - jx0) + (jy1 - jy0) * (jy1 - jy0);
  return gx * gx + gy * gy < fmaxf(di, dj);
}

// acc[k] += (v0, v1, v2) for the k selected by a wave-uniform index.
__device__ __forceinline__ void add_at(double (&U)[NI][3], int k, double v0, double v1,
                                       double v2) {
#pragma unroll
  for (int q = 0; q < NI; ++q)
    if (q == k) {
      U[q][0] += v0;
      U[q][1] += v1;
      U[q][2] += v2;
    }
}

// The pairs inside super-block I, by one workgroup: block pair p = (q, r),
// q <= r, of its NI blocks (q = r: the block's own ordered pairs, i side
// only) goes to wave p mod W.  The sums of each charge are combined in LDS in
// a fixed order and written to dp (forces, HVP: two components; local
// energies: one); the energy goes to dep[I].
constexpr int kDiagPairs = NI * (NI + 1) / 2;

constexpr size_t kDiagLds = sizeof(float) * kDiagPairs * 2 * 3 * kBlk;

template <int MODE, bool LOCAL>
__device__ __forceinline__ void sym_diag(const SymArgs& a, int I, int w, int lane,
                                         float (*part)[2][3][kBlk]) {
  // part[pair][i side | j side][component][lane], in the dynamic LDS
  __shared__ double red[16];
  double rvx = 0.0, rvy = 0.0;
  if (MODE == kHvp) {
    rvx = a.vxs[(size_t)I * SB];
    rvy = a.vys[(size_t)I * SB];
  }
#pragma unroll 1
  for (int p = w; p < kDiagPairs; p += a.W) {
    int q = 0, r = p;  // pair p in the order (0,0), (0,1), .., (0,NI-1), (1,1), ..
    while (r >= NI - q) {
      r -= NI - q;
      ++q;
    }
    r += q;
    const float* bq = a.box + 4 * ((size_t)NI * I + q);
    const double ccx = centre(bq[0], bq[1]), ccy = centre(bq[2], bq[3]);
    const Side sq =
        load_side<MODE>(a, (size_t)I * SB + q * kBlk + lane, ccx, ccy, rvx, rvy, true);
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, b0 = 0.f, b1 = 0.f;
    if (q == r) {
      BlockPair<MODE, false, true, true>::run(sq, sq, a0, a1, a2, b0, b1, lane, a.rz_e, a.rz_s);
      b0 = b1 = 0.f;
    } else {
      const Side sr =
          load_side<MODE>(a, (size_t)I * SB + r * kBlk + lane, ccx, ccy, rvx, rvy, true);
      BlockPair<MODE, LOCAL, true, false>::run(sq, sr, a0, a1, a2, b0, b1, lane, a.rz_e, a.rz_s);
    }
    const float dscale = q == r ? (float)a.diag_scale : 1.f;  // 0.5 or 1: exact in FP32
    part[p][0][0][lane] = a0;
    part[p][0][1][lane] = a1;
    part[p][0][2][lane] = a2 * dscale;
    // j side: forces/HVP components, or (local energies) the energy
    part[p][1][0][lane] = MODE == kEnergy ? 0.f : b0;
    part[p][1][1][lane] = MODE == kEnergy ? 0.f : b1;
    part[p][1][2][lane] = (MODE == kEnergy && LOCAL) ? b0 : 0.f;
  }
  __syncthreads();
  double es = 0.0;  // this thread's share of the energy
  for (int t = threadIdx.x; t < SB; t += blockDim.x) {
    const int k = t / kBlk, l = t % kBlk;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    int p = 0;
    for (int pq = 0; pq < NI; ++pq)
      for (int pr = pq; pr < NI; ++pr, ++p) {
        if (pq == k) {
          v0 += (double)part[p][0][0][l];
          v1 += (double)part[p][0][1][l];
          v2 += (double)part[p][0][2][l];
        }
        if (pr == k && pq != pr) {
          v0 += (double)part[p][1][0][l];
          v1 += (double)part[p][1][1][l];
          v2 += (double)part[p][1][2][l];
        }
      }
    const size_t s = (size_t)I * SB + t;
    if (MODE == kEnergy && LOCAL) {
      a.dp0[s] = v2;
    } else if (MODE != kEnergy) {
      a.dp0[s] = v0;
      a.dp1[s] = v1;
    }
    es += v2;
  }
  if (MODE != kHvp && !LOCAL) {
    const double ws = wave_sum(es);
    if (lane == 0) red[w] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
      a.dep[I] = t;
    }
  }
}

// Occupancy: the energy and force variants are held to the register budget
// of kSymWavesPerSimd waves per SIMD.
template <int MODE, bool LOCAL>
__global__ __launch_bounds__(64 * kSymWaves) __attribute__((amdgpu_waves_per_eu(
    MODE == kHvp ? 1 : kSymWavesPerSimd))) void k_sym(SymArgs a) {
  extern __shared__ double lds[];  // [S][NJ][SB]
  constexpr int NJ = (MODE == kEnergy) ? 1 : 2;
  constexpr bool JSIDE = MODE != kEnergy || LOCAL;  // j-side sums are kept
  __shared__ double ered[16];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // chunk-major dispatch: the last chunk (possibly short) ends the grid
  int bid = blockIdx.x;
  if (a.c0 == 0) {
    // first launch: workgroups 0..ns-1 do the pairs inside super-block bid,
    // dispatched first so that they overlap the chunk grid
    if (bid < a.ns) {
      sym_diag<MODE, LOCAL>(a, bid, w, lane, reinterpret_cast<float(*)[2][3][kBlk]>(lds));
      return;
    }
    bid -= a.ns;
  }
  const int cl = bid / a.G, g = bid % a.G;
  const int c = a.c0 + cl;
  const int task = g * a.Cb + cl;  // index of this workgroup's partials in the batch
  const int I = g * a.W + w;
  const bool wave_ok = I < a.ns;
  const int hmax = a.ns / 2;
  if (JSIDE)
    for (int e = threadIdx.x; e < a.S * NJ * SB; e += blockDim.x) lds[e] = 0.0;

  double U[NI][3];
  Side u[NI];
  double cx[NI], cy[NI];
  double rvx = 0.0, rvy = 0.0;
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    U[q][0] = U[q][1] = U[q][2] = 0.0;
    cx[q] = cy[q] = 0.0;
    u[q] = Side{};
  }
  if (wave_ok) {
    // reference points: the centres of the blocks' boxes (a block of pads
    // only has the empty box +inf..-inf and the centre 0)
    const float* bx = a.box + 4 * NI * (size_t)I;
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      cx[q] = centre(bx[4 * q], bx[4 * q + 1]);
      cy[q] = centre(bx[4 * q + 2], bx[4 * q + 3]);
    }
    if (MODE == kHvp) {
      // v relative to the super-block's first charge, so that differences of
      // a smooth v keep their precision
      rvx = a.vxs[(size_t)I * SB];
      rvy = a.vys[(size_t)I * SB];
    }
#pragma unroll
    for (int q = 0; q < NI; ++q)
      u[q] = load_side<MODE>(a, (size_t)I * SB + q * kBlk + lane, cx[q], cy[q], rvx, rvy, true);
  }
  if (JSIDE) __syncthreads();

  // Passes e = t * NI + h: step t, j block h of the step's super-block.  The
  // j charges of the next pass are loaded while the current one computes.
  auto pass_block = [&](int e) -> int {  // j block of pass e, -1 if none
    const int o = c * a.L + 1 + e / NI;
    if (!(wave_ok && o <= hmax && (2 * o < a.ns || I < hmax))) return -1;
    int J = I + o;
    if (J >= a.ns) J -= a.ns;
    return NI * J + e % NI;
  };
  const int npass = a.L * NI;
  double nx = 0.0, ny = 0.0, nvx = 0.0, nvy = 0.0;
  int jbn = pass_block(0);
  if (jbn >= 0) {
    const size_t sj = (size_t)jbn * kBlk + lane;
    nx = a.xs[sj];
    ny = a.ys[sj];
    if (MODE == kHvp) {
      nvx = a.vxs[sj];
      nvy = a.vys[sj];
    }
  }
#pragma unroll 1
  for (int e = 0; e < npass; ++e) {
    const int jb = jbn;
    const double jx = nx, jy = ny, jvx = nvx, jvy = nvy;
    jbn = e + 1 < npass ? pass_block(e + 1) : -1;
    if (jbn >= 0) {
      const size_t sj = (size_t)jbn * kBlk + lane;
      nx = a.xs[sj];
      ny = a.ys[sj];
      if (MODE == kHvp) {
        nvx = a.vxs[sj];
        nvy = a.vys[sj];
      }
    }
    if (jb >= 0) {
      bool near = false;
#pragma unroll
      for (int q = 0; q < NI; ++q) near = near || boxes_near(a.box, NI * I + q, jb);
      Side j[NI];
#pragma unroll
      for (int q = 0; q < NI; ++q)
        j[q] = make_side<MODE>(jx, jy, jvx, jvy, cx[q], cy[q], rvx, rvy, near);
      float acc[NI][3];
#pragma unroll
      for (int q = 0; q < NI; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.f;
      float b0 = 0.f, b1 = 0.f;
      if (near)
        BlockPairN<MODE, LOCAL, true>::run(u, j, acc, b0, b1, lane, a.rz_e, a.rz_s);
      else
        BlockPairN<MODE, LOCAL, false>::run(u, j, acc, b0, b1, lane, a.rz_e, a.rz_s);
#pragma unroll
      for (int q = 0; q < NI; ++q) {
        U[q][0] += (double)acc[q][0];
        U[q][1] += (double)acc[q][1];
        U[q][2] += (double)acc[q][2];
      }
      if (JSIDE) {
        double* sl = lds + (size_t)(w + e / NI) * NJ * SB + (e % NI) * kBlk;
        sl[lane] += (double)b0;
        if (NJ > 1) sl[SB + lane] += (double)b1;
      }
    }
    if (JSIDE && e % NI == NI - 1) __syncthreads();
  }

  const size_t si = (size_t)cl * a.npad + (size_t)I * SB + lane;
  if (MODE == kEnergy && LOCAL) {
    if (wave_ok) {
#pragma unroll
      for (int q = 0; q < NI; ++q) a.ip0[si + q * kBlk] = U[q][2];
    }
  } else {
    if (MODE != kEnergy && wave_ok) {
#pragma unroll
      for (int q = 0; q < NI; ++q) {
        a.ip0[si + q * kBlk] = U[q][0];
        a.ip1[si + q * kBlk] = U[q][1];
      }
    }
    if (MODE != kHvp) {
      double es = 0.0;
#pragma unroll
      for (int q = 0; q < NI; ++q) es += U[q][2];
      const double e = wave_sum(es);
      if (lane == 0) ered[w] = e;
      __syncthreads();
      if (threadIdx.x == 0) {
        double tt = 0.0;
        for (int q = 0; q < a.W; ++q) tt += ered[q];
        a.ep[(size_t)cl * a.G + g] = tt;  // the batch's sums are contiguous
      }
    }
  }
  if (JSIDE) {
    const size_t base = (size_t)task * a.S * SB;
    for (int e = threadIdx.x; e < a.S * SB; e += blockDim.x) {
      const int slot = e / SB, l = e % SB;
      a.jp0[base + e] = lds[(size_t)slot * NJ * SB + l];
      if (NJ > 1) a.jp1[base + e] = lds[(size_t)slot * NJ * SB + SB + l];
    }
  }
}

// Sum of one batch's partials for sorted index s, in a fixed order: the
// i-side chunks, then for each chunk the workgroups whose j window contains
// super-block B.  One workgroup of 2 x SB threads per super-block: the first
// SB threads take the first component of its charges, the others the second.
// The list of j partial slots (the same for all charges of B) is built first
// in LDS, so the loads can be issued in groups.
struct SymReduceArgs {
  const double* ip0;
  const double* ip1;
  const double* jp0;
  const double* jp1;
  const double* dp0;  // sums of the pairs inside the super-blocks (added by the first batch)
  const double* dp1;
  const int32_t* perm;
  int n, ns, npad, W, L, C, G, S;
  int c0, nc, Cb, mj;  // batch: first chunk, chunks, stride; list entries per chunk
  int first, last;     // first batch writes the outputs, later ones add to them
  double* out0;        // fx | hx | e_local (caller order)
  double* out1;        // fy | hy
  double* eblk;        // per-super-block sum of e_local (last batch)
};

template <int MODE>
__global__ __launch_bounds__(2 * SB) void k_sym_reduce(SymReduceArgs a) {
  extern __shared__ int32_t lst[];  // [nc][mj]: j partial slots, -1 for none
  __shared__ double red[SB / 64];
  const int B = blockIdx.x;
  for (int cl = threadIdx.x; cl < a.nc; cl += blockDim.x) {
    // workgroup (g, c) holds super-block J in slot (J - gW - cL - 1) mod ns
    // when that is < S; with u = (B - cL - 1) mod ns the bases gW that
    // qualify are u - slot + k*ns (k = 0, 1, 2), three disjoint ranges
    const int c = a.c0 + cl;
    int32_t* out = lst + cl * a.mj;
    int e = 0;
    int u = (B - c * a.L - 1) % a.ns;
    if (u < 0) u += a.ns;
    for (int k = 0; k < 3; ++k) {
      const int hi = u + k * a.ns, lo = hi - a.S + 1;
      const int g0 = lo <= 0 ? 0 : (lo + a.W - 1) / a.W;
      int g1 = hi / a.W;
      if (g1 > a.G - 1) g1 = a.G - 1;
      for (int g = g0; g <= g1 && e < a.mj; ++g) out[e++] = (g * a.Cb + cl) * a.S + (hi - g * a.W);
    }
    for (; e < a.mj; ++e) out[e] = -1;
  }
  __syncthreads();
  const int comp = threadIdx.x / SB, l = threadIdx.x % SB;
  const bool act = MODE != kEnergy || comp == 0;
  const int s = B * SB + l;
  const double* ip = comp ? a.ip1 : a.ip0;
  const double* jp = comp ? a.jp1 : a.jp0;
  double v = 0.0;
  if (act) {
    if (a.first) v = (comp ? a.dp1 : a.dp0)[s];
    int k = 0;
    for (; k + 8 <= a.nc; k += 8) {
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = ip[(size_t)(k + q) * a.npad + s];
#pragma unroll
      for (int q = 0; q < 8; ++q) v += t[q];
    }
    for (; k < a.nc; ++k) v += ip[(size_t)k * a.npad + s];
    const int m = a.nc * a.mj;
    k = 0;
    for (; k + 8 <= m; k += 8) {
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = lst[k + q];
        t[q] = j >= 0 ? jp[(size_t)j * SB + l] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) v += t[q];
    }
    for (; k < m; ++k) {
      const int j = lst[k];
      if (j >= 0) v += jp[(size_t)j * SB + l];
    }
    if (s < a.n) {
      double* out = comp ? a.out1 : a.out0;
      const int p = a.perm[s];
      if (!a.first) v = out[p] + v;
      if (MODE == kEnergy && a.last) v *= 0.5;
      out[p] = v;
    } else {
      v = 0.0;
    }
  }
  if (MODE == kEnergy && a.last) {
    const double ws = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && threadIdx.x < SB) red[threadIdx.x >> 6] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < SB / 64; ++q) t += red[q];
      a.eblk[B] = t;
    }
  }
}

// ---------------------------------------------------- one-sided FP64 pass --
// Wave = one i block (charges in registers), grid.y = j range split.  The j
// charges are wave-uniform, read through the scalar cache and broadcast from
// SGPRs.  The block containing i masks the self pair by index.
struct OneArgs {
  const double* xs;
  const double* ys;
  const double* vxs;
  const double* vys;
  int n, nb, npad, jb;  // jb = j blocks per split
  double rs;            // kRiesz: the exponent s
  int rn;               // kRiesz: r^-s = b^rn with b = 1/r (rh = 0) or sqrt(1/r) (rh = 1)
  int rh;               //   when s (rh = 0) or 2s (rh = 1) is an integer in 1..32; rn = 0: pow
  double* p0;        // [splits][npad]
  double* p1;
  double* p2;
};

template <int MODE, bool SELF>
__device__ __forceinline__ void one64_block(const double* __restrict__ xb,
                                            const double* __restrict__ yb,
                                            const double* __restrict__ vxb,
                                            const double* __restrict__ vyb, int jn, double xi,
                                            double yi, double vxi, double vyi, int lane,
                                            double& A0, double& A1, double& A2, double rs,
                                            int rn, int rh) {
#pragma unroll 4
  for (int jj = 0; jj < jn; ++jj) {
    const double dx = xi - xb[jj], dy = yi - yb[jj];
    const double r2 = __builtin_fma(dx, dx, dy * dy);
    if (MODE == kRiesz) {
      // r^-s: for s an integer the s-th power of 1/r (refined rsqrt, binary
      // powering), for 2s an integer the 2s-th power of sqrt(1/r); otherwise
      // pow.  The self pair is taken at r2 = 1 and zeroed.
      const bool self = SELF && jj == lane;
      const double q2 = self ? 1.0 : r2;
      double p, w;
      if (rn > 0) {
        const double inv = rsqrt64(q2);
        double b = rh ? sqrt(inv) : inv, acc = 1.0;
        for (int e = rn; e > 0; e >>= 1) {
          if (e & 1) acc *= b;
          b *= b;
        }
        p = self ? 0.0 : acc;
        w = rs * p * (inv * inv);
      } else {
        p = self ? 0.0 : pow(q2, -0.5 * rs);
        w = rs * p / q2;
      }
      A2 += p;
      A0 = __builtin_fma(dx, w, A0);
      A1 = __builtin_fma(dy, w, A1);
      continue;
    }
    double inv = rsqrt64(r2);
    if (SELF) inv = (jj == lane) ? 0.0 : inv;
    if (MODE == kEnergy) {
      A2 += inv;
    } else if (MODE == kForces) {
      A2 += inv;
      const double i3 = inv * inv * inv;
      A0 = __builtin_fma(dx, i3, A0);
      A1 = __builtin_fma(dy, i3, A1);
    } else {
      const double wx = vxi - vxb[jj], wy = vyi - vyb[jj];
      const double i2 = inv * inv;
      const double i3 = i2 * inv;
      const double q = 3.0 * i3 * i2;
      const double s = __builtin_fma(dx, wx, dy * wy) * q;
      A0 += __builtin_fma(dx, s, -wx * i3);
      A1 += __builtin_fma(dy, s, -wy * i3);
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_one64(OneArgs a) {
  const int I = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (I >= a.nb) return;
  const int si = I * kBlk + lane;
  const double xi = a.xs[si], yi = a.ys[si];
  const double vxi = MODE == kHvp ? a.vxs[si] : 0.0, vyi = MODE == kHvp ? a.vys[si] : 0.0;
  double A0 = 0.0, A1 = 0.0, A2 = 0.0;
  const int j0 = blockIdx.y * a.jb;
  const int j1 = min(a.nb, j0 + a.jb);
  for (int J = j0; J < j1; ++J) {
    const double* xb = a.xs + (size_t)J * kBlk;
    const double* yb = a.ys + (size_t)J * kBlk;
    const double* vxb = MODE == kHvp ? a.vxs + (size_t)J * kBlk : nullptr;
    const double* vyb = MODE == kHvp ? a.vys + (size_t)J * kBlk : nullptr;
    const int jn = min(kBlk, a.n - J * kBlk);  // real charges only; pads never enter
    if (J == I)
      one64_block<MODE, true>(xb, yb, vxb, vyb, jn, xi, yi, vxi, vyi, lane, A0, A1, A2, a.rs,
                              a.rn, a.rh);
    else
      one64_block<MODE, false>(xb, yb, vxb, vyb, jn, xi, yi, vxi, vyi, lane, A0, A1, A2, a.rs,
                               a.rn, a.rh);
  }
  const size_t k = (size_t)blockIdx.y * a.npad + si;
  if (MODE == kEnergy) {
    a.p0[k] = A2;
  } else {
    a.p0[k] = A0;
    a.p1[k] = A1;
    if (MODE == kForces || MODE == kRiesz) a.p2[k] = A2;
  }
}

struct OneReduceArgs {
  const double* p0;
  const double* p1;
  const double* p2;
  const int32_t* perm;
  int n, npad, splits;
  double* out0;
  double* out1;
  double* eblk;
};

template <int MODE>
__global__ __launch_bounds__(256) void k_one64_reduce(OneReduceArgs a) {
  __shared__ double red[4];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v0 = 0.0, v1 = 0.0, ve = 0.0;
  if (s < a.n) {
    for (int k = 0; k < a.splits; ++k) {
      const size_t q = (size_t)k * a.npad + s;
      if (MODE == kEnergy) {
        ve += a.p0[q];
      } else {
        v0 += a.p0[q];
        v1 += a.p1[q];
        if (MODE == kForces || MODE == kRiesz) ve += a.p2[q];
      }
    }
    ve *= 0.5;  // ordered pairs: e_i = 1/2 sum_{j != i} 1/r_ij
    const int p = a.perm[s];
    if (MODE == kEnergy) {
      if (a.out0) a.out0[p] = ve;
    } else {
      a.out0[p] = v0;
      a.out1[p] = v1;
    }
  }
  if (MODE != kHvp) {
    double ws = wave_sum(ve);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ws;
    __syncthreads();
    if (threadIdx.x == 0) a.eblk[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// Final energy: one workgroup of 1024 threads sums the m partials in a fixed
// order (per thread the elements t, t + 1024, ... in order, loads issued in
// groups of 8; then the waves' sums in order).
__global__ __launch_bounds__(1024) void k_sum_blocks(const double* __restrict__ eblk, int m,
                                                     double* __restrict__ out) {
  __shared__ double red[16];
  double v = 0.0;
  int k = threadIdx.x;
  for (; k + 7 * 1024 < m; k += 8 * 1024) {
    double t[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) t[q] = eblk[k + q * 1024];
#pragma unroll
    for (int q = 0; q < 8; ++q) v += t[q];
  }
  for (; k < m; k += 1024) v += eblk[k];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += red[q];
    *out = t;
  }
}

static void sum_blocks(const double* part, int m, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(1024), 0, st, part, m, out);
}

// ------------------------------------------------------------- validation --
__global__ void k_validate(const double* __restrict__ xs, const double* __restrict__ ys,
                           const int32_t* __restrict__ perm, int n, int32_t* __restrict__ flags,
                           int32_t* __restrict__ count) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double x = xs[s], y = ys[s];
  int f = 0;
  if (!isfinite(x) || !isfinite(y)) f |= CD_FLAG_NONFINITE;
  else if (x * x + y * y > 1.0 + 8.0 * 1.1102230246251565e-16) f |= CD_FLAG_OUTSIDE;
  // equal points have equal Morton keys, so after the stable sort an exact
  // duplicate sits next to one of its copies
  if (s > 0 && xs[s - 1] == x && ys[s - 1] == y) f |= CD_FLAG_COINCIDENT;
  if (s + 1 < n && xs[s + 1] == x && ys[s + 1] == y) f |= CD_FLAG_COINCIDENT;
  flags[perm[s]] = f;
  if (f) atomicAdd(count, 1);
}

// ------------------------------------------------------------------ shapes --
// Launch shapes of the symmetric pass (waves per workgroup W, offsets per
// chunk L) that coulomb_autotune chooses from; the first is the default.
// make_plan clamps each to the kernel's launch bound (W <= kSymWaves) and to
// the 64 KiB j window.
struct SymShape {
  int W, L;
};
constexpr SymShape kShapes[] = {{kSymWaves, kSymChunk}, {8, 6}, {8, 12}, {8, 16}, {8, 20},
                                {4, 8}, {4, 12}, {4, 16}, {4, 24}, {2, 24}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
// offsets per chunk that keep the j window (S = W + L - 1 super-blocks of
// NI KiB each, forces and HVP) within 64 KiB
constexpr int max_chunk(int W) { return 64 / NI - W + 1; }

static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int64_t>, int> g_tuned;  // (device, op, n) -> shape

static int current_device() {
  int d = -1;
  if (hipGetDevice(&d) != hipSuccess) return -1;
  return d;
}

static int tuned_shape(int op, int64_t n) {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(std::make_tuple(dev, op, n));
  return it == g_tuned.end() ? 0 : it->second;
}

// ---------------------------------------------------------------- planning --
bool make_plan(int op, int64_t n64, int precision, char* base, Plan& P, int shape, int max_cb) {
  if (n64 < 1 || n64 > (int64_t)1 << 26) return false;
  if (precision != CD_FP64 && precision != CD_MIXED) return false;
  const int n = (int)n64;
  P.n = n;
  P.nb = (n + kBlk - 1) / kBlk;
  P.npad = P.nb * kBlk;
  const int mode = op == CD_OP_ENERGY ? kEnergy : op == CD_OP_FORCES ? kForces : kHvp;
  if (precision == CD_MIXED && op != CD_OP_VALIDATE) {
    P.ns = (n + SB - 1) / SB;
    P.nb = NI * P.ns;
    P.npad = P.nb * kBlk;
    // W waves per workgroup, L offsets per chunk; S = L + W - 1 <= ns keeps
    // the j window from wrapping onto itself
    if (shape < 0 || shape >= kNumShapes) shape = 0;
    const SymShape sh = kShapes[shape];
    P.shape = shape;
    const int w = sh.W < kSymWaves ? sh.W : kSymWaves;  // the kernel's launch bound
    P.W = P.ns < w ? P.ns : w;
    const int l = P.ns + 1 - P.W, lmax = sh.L < max_chunk(w) ? sh.L : max_chunk(w);
    P.L = l < 1 ? 1 : (l > lmax ? lmax : l);
    const int hmax = P.ns / 2;
    P.C = hmax > 0 ? (hmax + P.L - 1) / P.L : 1;
    P.G = (P.ns + P.W - 1) / P.W;
    P.S = P.L + P.W - 1;
    P.mj = (P.S + P.W - 1) / P.W + 1;  // j partial slots of one super-block per chunk
    // chunks per batch: partial sums of at most kSymBatchBytes (at least one chunk)
    const size_t per = ((size_t)P.npad + (size_t)P.G * P.S * SB) * sizeof(double) *
                       (mode == kEnergy ? 1 : 2);
    size_t cb = kSymBatchBytes / per;
    if (cb < 1) cb = 1;
    if (cb > (size_t)kSymBatchMax) cb = kSymBatchMax;
    if (max_cb > 0 && cb > (size_t)max_cb) cb = max_cb;
    P.Cb = cb < (size_t)P.C ? (int)cb : P.C;
    P.chunk_bytes = per;
  } else {
    // enough waves to fill 256 CUs several times over
    int sp = (16384 + P.nb - 1) / P.nb;
    if (sp < 1) sp = 1;
    if (sp > P.nb) sp = P.nb;
    P.jb = (P.nb + sp - 1) / sp;
    P.splits = (P.nb + P.jb - 1) / P.jb;
  }
  P.nred = (n + 255) / 256;
  Carve cv;
  cv.base = base;
  P.keys = cv.take<uint32_t>(n);
  P.keys2 = cv.take<uint32_t>(n);
  P.perm = cv.take<int32_t>(n);
  P.perm2 = cv.take<int32_t>(n);
  P.hist = cv.take<uint32_t>(sort_scratch_elems(n));
  P.xs = cv.take<double>(P.npad);
  P.ys = cv.take<double>(P.npad);
  if (op == CD_OP_HVP) {
    P.vxs = cv.take<double>(P.npad);
    P.vys = cv.take<double>(P.npad);
  }
  P.box = cv.take<float>(4 * (size_t)P.nb);
  if (op != CD_OP_VALIDATE) {
    if (precision == CD_MIXED) {
      const size_t q = (size_t)P.Cb * P.npad;
      P.q0 = cv.take<double>(q);
      if (mode != kEnergy) P.q1 = cv.take<double>(q);
      const size_t jq = (size_t)P.G * P.Cb * P.S * SB;
      P.j0 = cv.take<double>(jq);
      if (mode != kEnergy) P.j1 = cv.take<double>(jq);
      P.dp0 = cv.take<double>(P.npad);
      if (mode != kEnergy) P.dp1 = cv.take<double>(P.npad);
      if (mode != kHvp) {
        P.ep = cv.take<double>((size_t)P.ns + (size_t)P.G * P.Cb);  // diagonal, then batch
        P.eb = cv.take<double>((P.C + P.Cb - 1) / P.Cb);
      }
      P.eblk = cv.take<double>(P.ns);
    } else {
      const size_t q = (size_t)P.splits * P.npad;
      P.q0 = cv.take<double>(q);
      if (mode != kEnergy) P.q1 = cv.take<double>(q);
      if (mode == kForces) P.q2 = cv.take<double>(q);
      P.eblk = cv.take<double>(P.nred);
    }
  }
  P.total = cv.off + 256;
  return true;
}

int stage(const Plan& P, const double* x, const double* y, const double* vx,
                 const double* vy, hipStream_t st) {
  const int n = P.n;
  int rc = morton_order(x, y, n, P.keys, P.keys2, P.perm2, P.hist, P.perm, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_gather, dim3((P.nb + 3) / 4), dim3(256), 0, st, x, y, vx, vy, P.perm, n,
                     P.nb, P.xs, P.ys, P.vxs, P.vys, P.box);
  return hip_status(hipGetLastError());
}

// Measurement hook (coulomb_set_kernel_events): events recorded around the
// dominant pair kernel of the next calls.
static hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

static void mark(hipEvent_t ev, hipStream_t st) {
  if (ev) (void)hipEventRecord(ev, st);
}

// Symmetric pass in batches of chunks, each followed by its reduction, and
// (forces, energy) the total energy.
template <int MODE, bool LOCAL>
static void run_sym(const Plan& P, hipStream_t st, double* out0, double* out1, double* e_total,
                    double riesz_s = 0.0) {
  SymArgs a;
  a.rz_e = (float)(-0.5 * riesz_s - 1.0);
  a.rz_s = (float)riesz_s;
  a.xs = P.xs;
  a.ys = P.ys;
  a.vxs = P.vxs;
  a.vys = P.vys;
  a.box = P.box;
  a.ns = P.ns;
  a.npad = P.npad;
  a.W = P.W;
  a.L = P.L;
  a.C = P.C;
  a.G = P.G;
  a.S = P.S;
  a.Cb = P.Cb;
  a.ip0 = P.q0;
  a.ip1 = P.q1;
  a.jp0 = P.j0;
  a.jp1 = P.j1;
  a.ep = P.ep ? P.ep + P.ns : nullptr;
  a.diag_scale = (MODE == kEnergy && LOCAL) ? 1.0 : 0.5;
  constexpr bool JSIDE = MODE != kEnergy || LOCAL;
  constexpr int NJ = (MODE == kEnergy) ? 1 : 2;
  size_t lds = JSIDE ? (size_t)P.S * NJ * SB * sizeof(double) : 0;
  if (lds < kDiagLds) lds = kDiagLds;
  SymReduceArgs r;
  r.ip0 = P.q0;
  r.ip1 = P.q1;
  r.jp0 = P.j0;
  r.jp1 = P.j1;
  r.dp0 = P.dp0;
  r.dp1 = P.dp1;
  r.perm = P.perm;
  r.n = P.n;
  r.ns = P.ns;
  r.npad = P.npad;
  r.W = P.W;
  r.L = P.L;
  r.C = P.C;
  r.G = P.G;
  r.S = P.S;
  r.Cb = P.Cb;
  r.mj = P.mj;
  r.out0 = out0;
  r.out1 = out1;
  r.eblk = P.eblk;
  const int nbatch = (P.C + P.Cb - 1) / P.Cb;
  constexpr bool ESUM = MODE != kHvp && !LOCAL;  // total energy from the per-workgroup sums
  a.dp0 = P.dp0;
  a.dp1 = P.dp1;
  a.dep = P.ep;
  mark(g_ev_start, st);
  for (int c0 = 0, b = 0; c0 < P.C; c0 += P.Cb, ++b) {
    const int nc = P.C - c0 < P.Cb ? P.C - c0 : P.Cb;
    a.c0 = c0;
    a.nc = nc;
    const int grid = P.G * nc + (c0 == 0 ? P.ns : 0);  // + the super-diagonal workgroups
    hipLaunchKernelGGL((k_sym<MODE, LOCAL>), dim3(grid), dim3(64 * P.W), lds, st, a);
    if (c0 + nc >= P.C) mark(g_ev_stop, st);
    if (ESUM && e_total) {
      // the first batch's sum includes the super-diagonal sums stored before it
      const double* part = b == 0 ? P.ep : P.ep + P.ns;
      const int m = P.G * nc + (b == 0 ? P.ns : 0);
      sum_blocks(part, m, nbatch == 1 ? e_total : P.eb + b, st);
    }
    if (JSIDE) {
      r.c0 = c0;
      r.nc = nc;
      r.first = c0 == 0;
      r.last = c0 + nc >= P.C;
      hipLaunchKernelGGL((k_sym_reduce<MODE>), dim3(P.ns), dim3(2 * SB),
                         (size_t)nc * P.mj * sizeof(int32_t), st, r);
    }
  }
  if (e_total) {
    if (MODE == kEnergy && LOCAL) sum_blocks(P.eblk, P.ns, e_total, st);
    else if (ESUM && nbatch > 1) sum_blocks(P.eb, nbatch, e_total, st);
  }
}

template <int MODE>
static void run_one64(const Plan& P, hipStream_t st, double* out0, double* out1,
                      double riesz_s = 0.0) {
  OneArgs a;
  a.rs = riesz_s;
  const double r2s = 2.0 * riesz_s;
  a.rn = 0;
  a.rh = 0;
  if (riesz_s == floor(riesz_s) && riesz_s >= 1.0 && riesz_s <= 32.0) {
    a.rn = (int)riesz_s;
  } else if (r2s == floor(r2s) && r2s >= 1.0 && r2s <= 32.0) {
    a.rn = (int)r2s;
    a.rh = 1;
  }
  a.xs = P.xs;
  a.ys = P.ys;
  a.vxs = P.vxs;
  a.vys = P.vys;
  a.n = P.n;
  a.nb = P.nb;
  a.npad = P.npad;
  a.jb = P.jb;
  a.p0 = P.q0;
  a.p1 = P.q1;
  a.p2 = P.q2;
  mark(g_ev_start, st);
  hipLaunchKernelGGL((k_one64<MODE>), dim3((P.nb + 3) / 4, P.splits), dim3(256), 0, st, a);
  mark(g_ev_stop, st);
  OneReduceArgs r;
  r.p0 = P.q0;
  r.p1 = P.q1;
  r.p2 = P.q2;
  r.perm = P.perm;
  r.n = P.n;
  r.npad = P.npad;
  r.splits = P.splits;
  r.out0 = out0;
  r.out1 = out1;
  r.eblk = P.eblk;
  hipLaunchKernelGGL((k_one64_reduce<MODE>), dim3(P.nred), dim3(256), 0, st, r);
}


// v in caller order -> sorted, padded copies (pads carry v = 0)
__global__ void k_gather_v(const double* __restrict__ vx, const double* __restrict__ vy,
                           const int32_t* __restrict__ perm, int n, int npad,
                           double* __restrict__ vxs, double* __restrict__ vys) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= npad) return;
  if (s < n) {
    const int p = perm[s];
    vxs[s] = vx[p];
    vys[s] = vy[p];
  } else {
    vxs[s] = 0.0;
    vys[s] = 0.0;
  }
}

size_t hvp64_bytes(int64_t n) {
  Plan P;
  return make_plan(CD_OP_HVP, n, CD_FP64, nullptr, P) ? P.total : 0;
}

int hvp64_stage(Plan& P, char* base, int64_t n, const double* x, const double* y,
                hipStream_t st) {
  if (!make_plan(CD_OP_HVP, n, CD_FP64, base, P)) return CD_ERR_INVALID_ARG;
  return stage(P, x, y, nullptr, nullptr, st);
}

int hvp64_apply(const Plan& P, const double* vx, const double* vy, double* hx, double* hy,
                hipStream_t st) {
  hipLaunchKernelGGL(k_gather_v, dim3((P.npad + 255) / 256), dim3(256), 0, st, vx, vy, P.perm,
                     P.n, P.npad, P.vxs, P.vys);
  run_one64<kHvp>(P, st, hx, hy);
  return hip_status(hipGetLastError());
}

size_t relax_workspace_bytes(int op, int64_t n, int32_t n_patches, int64_t total_active,
                             int precision);
size_t lanczos_workspace_bytes(int64_t n, int k);
size_t zones_workspace_bytes(int op, int64_t n, int32_t n_zones);
size_t structure_workspace_bytes(int64_t n);
size_t border_workspace_bytes(int64_t n);

}  // namespace cd

using namespace cd;

extern "C" {

size_t coulomb_workspace_bytes(int op, int64_t n, int32_t n_patches, int64_t total_active,
                               int precision) {
  (void)n_patches;
  (void)total_active;
  if (op == CD_OP_ENERGY || op == CD_OP_FORCES || op == CD_OP_HVP || op == CD_OP_VALIDATE) {
    const int prec = op == CD_OP_VALIDATE ? CD_FP64 : precision;
    size_t most = 0;
    // enough for every shape the tuner may choose
    for (int sh = 0; sh < (prec == CD_MIXED ? kNumShapes : 1); ++sh) {
      Plan P;
      if (!make_plan(op, n, prec, nullptr, P, sh)) return 0;
      most = P.total > most ? P.total : most;
    }
    return most;
  }
  if (op == CD_OP_LANCZOS) return cd::lanczos_workspace_bytes(n, n_patches);
  if (op == CD_OP_VORONOI) {
    if (n < 1 || n > (1 << 26)) return 0;
    return cd::structure_workspace_bytes(n);
  }
  if (op == CD_OP_BORDER) return cd::border_workspace_bytes(n);
  if (op == CD_OP_DEFECT || op == CD_OP_ZONES) {
    if (n < 1 || n > (1 << 26) || (op == CD_OP_ZONES && n_patches < 1)) return 0;
    return cd::zones_workspace_bytes(op, n, n_patches);
  }
  return cd::relax_workspace_bytes(op, n, n_patches, total_active, precision);
}

}  // extern "C"

namespace cd {

static int check_ws(int op, int64_t n, int precision, void* ws, size_t ws_bytes, Plan& P,
                    int shape = -1) {
  if (!ws) return CD_ERR_WORKSPACE;
  if (shape < 0 && precision == CD_MIXED) shape = tuned_shape(op, n);
  if (!make_plan(op, n, precision, nullptr, P, shape)) return CD_ERR_INVALID_ARG;
  if (ws_bytes < P.total) return CD_ERR_WORKSPACE;
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  make_plan(op, n, precision, base, P, shape);
  return CD_OK;
}

static int energy_impl(const double* x, const double* y, int64_t n, int precision,
                       double* e_total, double* e_local, void* ws, size_t ws_bytes,
                       hipStream_t st, int shape) {
  if (!x || !y || !e_total) return CD_ERR_INVALID_ARG;
  Plan P;
  int rc = check_ws(CD_OP_ENERGY, n, precision, ws, ws_bytes, P, shape);
  if (rc) return rc;
  if ((rc = stage(P, x, y, nullptr, nullptr, st))) return rc;
  if (precision == CD_MIXED) {
    if (e_local) run_sym<kEnergy, true>(P, st, e_local, nullptr, e_total);
    else run_sym<kEnergy, false>(P, st, nullptr, nullptr, e_total);
  } else {
    run_one64<kEnergy>(P, st, e_local, nullptr);
    sum_blocks(P.eblk, P.nred, e_total, st);
  }
  return hip_status(hipGetLastError());
}

static int forces_run(const Plan& P, const double* x, const double* y, int precision,
                      double* fx, double* fy, double* e_total, hipStream_t st) {
  int rc = stage(P, x, y, nullptr, nullptr, st);
  if (rc) return rc;
  if (precision == CD_MIXED) {
    run_sym<kForces, false>(P, st, fx, fy, e_total);
  } else {
    run_one64<kForces>(P, st, fx, fy);
    if (e_total) sum_blocks(P.eblk, P.nred, e_total, st);
  }
  return hip_status(hipGetLastError());
}

static int forces_impl(const double* x, const double* y, int64_t n, int precision, double* fx,
                       double* fy, double* e_total, void* ws, size_t ws_bytes, hipStream_t st,
                       int shape) {
  if (!x || !y || !fx || !fy) return CD_ERR_INVALID_ARG;
  Plan P;
  int rc = check_ws(CD_OP_FORCES, n, precision, ws, ws_bytes, P, shape);
  if (rc) return rc;
  return forces_run(P, x, y, precision, fx, fy, e_total, st);
}

// Plan of a forces call inside cap bytes: the default plan, or the same
// shape with fewer chunks per batch.
static int plan_fixed(int64_t n, int precision, char* base, size_t cap, Plan& P) {
  const int shape = precision == CD_MIXED ? tuned_shape(CD_OP_FORCES, n) : -1;
  if (!make_plan(CD_OP_FORCES, n, precision, nullptr, P, shape)) return CD_ERR_INVALID_ARG;
  int cb = P.Cb;
  if (P.total > cap) {
    if (precision != CD_MIXED || P.Cb <= 1) return CD_ERR_CAPACITY;
    const size_t over = P.total - cap;  // chunks to drop, rounded up
    const size_t drop = (over + P.chunk_bytes - 1) / P.chunk_bytes;
    if (drop >= (size_t)P.Cb) return CD_ERR_CAPACITY;
    cb = P.Cb - (int)drop;
    // the carve aligns each piece, so step down until the plan fits
    for (;; --cb) {
      if (cb < 1) return CD_ERR_CAPACITY;
      make_plan(CD_OP_FORCES, n, precision, nullptr, P, shape, cb);
      if (P.total <= cap) break;
    }
  }
  if (base) make_plan(CD_OP_FORCES, n, precision, base, P, shape, cb);
  return CD_OK;
}

int forces_fixed_fits(int64_t n, int precision, size_t cap) {
  Plan P;
  return plan_fixed(n, precision, nullptr, cap, P);
}

int forces_fixed(const double* x, const double* y, int64_t n, int precision, double* fx,
                 double* fy, double* e_total, char* base, size_t cap, hipStream_t st) {
  if (!x || !y || !fx || !fy || !base) return CD_ERR_INVALID_ARG;
  Plan P;
  const int rc = plan_fixed(n, precision, base, cap, P);
  if (rc) return rc;
  return forces_run(P, x, y, precision, fx, fy, e_total, st);
}

static int riesz_impl(const double* x, const double* y, int64_t n, double rs, int precision,
                      double* fx, double* fy, double* e_total, void* ws, size_t ws_bytes,
                      hipStream_t st) {
  if (!x || !y || !fx || !fy) return CD_ERR_INVALID_ARG;
  if (!(rs > 0.0) || rs > (precision == CD_MIXED ? 6.0 : 64.0)) return CD_ERR_INVALID_ARG;
  Plan P;
  int rc = check_ws(CD_OP_FORCES, n, precision, ws, ws_bytes, P, -1);
  if (rc) return rc;
  if ((rc = stage(P, x, y, nullptr, nullptr, st))) return rc;
  if (precision == CD_MIXED) {
    run_sym<kRiesz, false>(P, st, fx, fy, e_total, rs);
  } else {
    run_one64<kRiesz>(P, st, fx, fy, rs);
    if (e_total) sum_blocks(P.eblk, P.nred, e_total, st);
  }
  return hip_status(hipGetLastError());
}

static int hvp_impl(const double* x, const double* y, const double* vx, const double* vy,
                    int64_t n, int precision, double* hx, double* hy, void* ws, size_t ws_bytes,
                    hipStream_t st, int shape) {
  if (!x || !y || !vx || !vy || !hx || !hy) return CD_ERR_INVALID_ARG;
  Plan P;
  int rc = check_ws(CD_OP_HVP, n, precision, ws, ws_bytes, P, shape);
  if (rc) return rc;
  if ((rc = stage(P, x, y, vx, vy, st))) return rc;
  if (precision == CD_MIXED) run_sym<kHvp, false>(P, st, hx, hy, nullptr);
  else run_one64<kHvp>(P, st, hx, hy);
  return hip_status(hipGetLastError());
}

}  // namespace cd

extern "C" {

int coulomb_energy(const double* x, const double* y, int64_t n, int precision, double* e_total,
                   double* e_local, void* ws, size_t ws_bytes, void* stream) {
  return energy_impl(x, y, n, precision, e_total, e_local, ws, ws_bytes, (hipStream_t)stream,
                     -1);
}

int coulomb_forces(const double* x, const double* y, int64_t n, int precision, double* fx,
                   double* fy, double* e_total, void* ws, size_t ws_bytes, void* stream) {
  return forces_impl(x, y, n, precision, fx, fy, e_total, ws, ws_bytes, (hipStream_t)stream, -1);
}

int coulomb_riesz(const double* x, const double* y, int64_t n, double s, int precision,
                  double* fx, double* fy, double* e_total, void* ws, size_t ws_bytes,
                  void* stream) {
  return riesz_impl(x, y, n, s, precision, fx, fy, e_total, ws, ws_bytes, (hipStream_t)stream);
}

int coulomb_hvp(const double* x, const double* y, const double* vx, const double* vy, int64_t n,
                int precision, double* hx, double* hy, void* ws, size_t ws_bytes, void* stream) {
  return hvp_impl(x, y, vx, vy, n, precision, hx, hy, ws, ws_bytes, (hipStream_t)stream, -1);
}

int coulomb_autotune(const double* x, const double* y, int64_t n, int op, void* ws,
                     size_t ws_bytes, void* stream, int32_t* shape_out) {
  if (!x || !y || !shape_out) return CD_ERR_INVALID_ARG;
  if (op != CD_OP_ENERGY && op != CD_OP_FORCES && op != CD_OP_HVP) return CD_ERR_INVALID_ARG;
  const size_t need = coulomb_workspace_bytes(op, n, 0, 0, CD_MIXED);
  if (!need) return CD_ERR_INVALID_ARG;
  if (!ws) return CD_ERR_WORKSPACE;
  const size_t outb = ((size_t)n * 2 * sizeof(double) + 8 + 255) & ~size_t(255);
  if (ws_bytes < need + outb + 256) return CD_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  // outputs at the aligned start, the operation's scratch after them
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  double* o0 = reinterpret_cast<double*>(base);
  double* o1 = o0 + n;
  double* oe = o1 + n;
  char* rws = base + outb;
  const size_t rbytes = ws_bytes - (size_t)(rws - reinterpret_cast<char*>(ws));
  auto run = [&](int sh) {
    if (op == CD_OP_ENERGY) return energy_impl(x, y, n, CD_MIXED, oe, nullptr, rws, rbytes, st, sh);
    if (op == CD_OP_FORCES) return forces_impl(x, y, n, CD_MIXED, o0, o1, oe, rws, rbytes, st, sh);
    return hvp_impl(x, y, x, y, n, CD_MIXED, o0, o1, rws, rbytes, st, sh);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = hip_status(hipEventCreate(&e0));
  if (!rc) rc = hip_status(hipEventCreate(&e1));
  int best = 0;
  float best_ms = 0.f;
  for (int sh = 0; sh < kNumShapes && !rc; ++sh) {
    if ((rc = run(sh))) break;  // warm-up
    if ((rc = hip_status(hipEventRecord(e0, st)))) break;
    for (int k = 0; k < 3 && !rc; ++k) rc = run(sh);
    if (rc || (rc = hip_status(hipEventRecord(e1, st)))) break;
    if ((rc = hip_status(hipEventSynchronize(e1)))) break;
    float ms = 0.f;
    if ((rc = hip_status(hipEventElapsedTime(&ms, e0, e1)))) break;
    if (sh == 0 || ms < best_ms) {
      best = sh;
      best_ms = ms;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(current_device(), op, n)] = best;
  }
  shape_out[0] = best;
  shape_out[1] = kShapes[best].W;
  shape_out[2] = kShapes[best].L;
  return CD_OK;
}

int coulomb_validate(const double* x, const double* y, int64_t n, int32_t* flags_out,
                     int32_t* count_out, void* ws, size_t ws_bytes, void* stream) {
  if (!x || !y || !flags_out || !count_out) return CD_ERR_INVALID_ARG;
  Plan P;
  int rc = check_ws(CD_OP_VALIDATE, n, CD_FP64, ws, ws_bytes, P);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if ((rc = stage(P, x, y, nullptr, nullptr, st))) return rc;
  if ((rc = hip_status(hipMemsetAsync(count_out, 0, sizeof(int32_t), st)))) return rc;
  hipLaunchKernelGGL(k_validate, dim3((P.n + 255) / 256), dim3(256), 0, st, P.xs, P.ys, P.perm,
                     P.n, flags_out, count_out);
  return hip_status(hipGetLastError());
}

void coulomb_set_kernel_events(void* ev_start, void* ev_stop) {
  g_ev_start = (hipEvent_t)ev_start;
  g_ev_stop = (hipEvent_t)ev_stop;
}

const char* coulomb_status_string(int code) {
  switch (code) {
    case CD_OK: return "ok";
    case CD_ERR_INVALID_ARG: return "invalid argument";
    case CD_ERR_WORKSPACE: return "workspace missing or too small";
    case CD_ERR_HIP: return "HIP runtime error";
    case CD_ERR_DOMAIN: return "positions outside the domain";
    case CD_ERR_CAPACITY: return "output capacity too small (sizes reported)";
    case CD_ERR_SCRATCH: return "sizes exceed the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

}  // extern "C"
