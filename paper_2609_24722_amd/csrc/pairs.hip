// All-pairs energy, forces and Hessian-vector products for N charges in the
// unit disk (paper Sec. II.A, Eq. 2), and the C-ABI entry points that run
// them: coulomb_energy, coulomb_forces, coulomb_hvp, coulomb_validate.
//
// Pipeline of one call (all on the caller's stream):
//   1. staging     Morton keys of the FP64 positions, a stable radix sort,
//                  gather into sorted SoA arrays padded to whole 64-charge
//                  blocks, per-block centre and bounding box;
//   2. pair pass   CD_MIXED: symmetric FP32 kernel over block pairs (each
//                  unordered pair evaluated once, Newton's third law);
//                  CD_FP64: one-sided FP64 kernel over (i block, j range);
//   3. reduction   fixed-order sums of the partial results, scattered back
//                  to the caller's order; energy by a fixed-shape tree.
#include "plan.hpp"

namespace cd {

size_t sort_scratch_elems(int n);
int sort_pairs(uint32_t* ka, int32_t* va, uint32_t* kb, int32_t* vb, uint32_t* hist, int n,
               hipStream_t st);

enum Mode { kEnergy = 0, kForces = 1, kHvp = 2 };

// ------------------------------------------------------------------ staging --
__device__ __forceinline__ uint32_t spread16(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__global__ void k_morton(const double* __restrict__ x, const double* __restrict__ y, int n,
                         uint32_t* __restrict__ keys, int32_t* __restrict__ idx) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double fx = (x[i] + 1.0) * 32768.0, fy = (y[i] + 1.0) * 32768.0;
  if (!(fx >= 0.0)) fx = 0.0;
  if (!(fx <= 65535.0)) fx = 65535.0;
  if (!(fy >= 0.0)) fy = 0.0;
  if (!(fy <= 65535.0)) fy = 65535.0;
  keys[i] = spread16((uint32_t)fx) | (spread16((uint32_t)fy) << 1);
  idx[i] = i;
}

// Sorted, padded copies: xs[s] = x[perm[s]] for s < n, pads beyond.
__global__ void k_gather(const double* __restrict__ x, const double* __restrict__ y,
                         const double* __restrict__ vx, const double* __restrict__ vy,
                         const int32_t* __restrict__ perm, int n, int npad,
                         double* __restrict__ xs, double* __restrict__ ys,
                         double* __restrict__ vxs, double* __restrict__ vys) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= npad) return;
  if (s < n) {
    int p = perm[s];
    xs[s] = x[p];
    ys[s] = y[p];
    if (vxs && vx) {  // v is gathered only when given (staged HVPs gather it per call)
      vxs[s] = vx[p];
      vys[s] = vy[p];
    }
  } else {
    xs[s] = pad_x(s - n);
    ys[s] = 0.0;
    if (vxs && vx) {
      vxs[s] = 0.0;
      vys[s] = 0.0;
    }
  }
}

// Per block: bounding box of its real charges and the box centre (the
// reference point of the block's relative coordinates).  One wave per block.
__global__ void k_blockinfo(const double* __restrict__ xs, const double* __restrict__ ys, int n,
                            int nb, double* __restrict__ cen, float* __restrict__ box) {
  int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (b >= nb) return;
  int s = b * kBlk + lane;
  bool ok = s < n;
  double xv = xs[s], yv = ys[s];
  double x0 = wave_min(ok ? xv : 1e300), x1 = wave_max(ok ? xv : -1e300);
  double y0 = wave_min(ok ? yv : 1e300), y1 = wave_max(ok ? yv : -1e300);
  if (lane == 0) {
    cen[2 * b] = 0.5 * (x0 + x1);
    cen[2 * b + 1] = 0.5 * (y0 + y1);
    box[4 * b + 0] = (float)x0;
    box[4 * b + 1] = (float)x1;
    box[4 * b + 2] = (float)y0;
    box[4 * b + 3] = (float)y1;
  }
}

// ------------------------------------------------- symmetric FP32 pair pass --
// Work decomposition.  Blocks I and J = (I + o) mod nb interact for offsets
// o = 1..floor(nb/2) (for even nb the offset nb/2 only from I < nb/2): every
// unordered block pair exactly once, the same work for every I.  A workgroup
// of W waves owns blocks I = gW..gW+W-1 (one per wave, i charges in
// registers) and the offsets of chunk c: o = cL+1 .. cL+L.  At time step t
// wave w handles o = cL+1+t, so its j block lands in LDS slot w + t of the
// workgroup's window of L+W-1 consecutive j blocks; no two waves share a slot
// in a step, and a barrier separates steps, so the j-side sums accumulate in
// LDS without atomics and in a fixed order.
//
// Inside a block pair each lane owns one i and one j.  Within each 16-lane
// row the j data rotate by DPP (row_ror:k folded into the subtraction) and
// the j-side accumulators travel with them (row_ror:1 per step); after 16
// steps the rows rotate by a lane permute, four times in all, which covers
// the 64 x 64 pairs and returns each j accumulator to its own lane.
//
// Precision.  Coordinates are taken relative to the centre of block I
// (FP64 subtraction, then rounded to FP32), so their rounding error scales
// with the distance from that centre, not with |r|.  For block pairs whose
// boxes are near each other the low parts fl32(r - c - hi) are kept too and
// dx = (hi_j - hi_i) + (lo_j - lo_i) is exact to FP32 rounding of dx itself.
// Per block pair the i and j partials are FP32 sums of 64 terms, folded into
// FP64 (registers for i, LDS for j).
struct SymArgs {
  const double* xs;
  const double* ys;
  const double* vxs;
  const double* vys;
  const double* cen;
  const float* box;
  int nb, npad, W, L, C, G, S;
  double* ip0;  // i-side partials [C][npad]: fx | hx | e
  double* ip1;  //                            fy | hy
  double* ip2;  //                            e (forces mode)
  double* jp0;  // j-side partials [G*C][S][64]
  double* jp1;
  double diag_scale;  // weight of the ordered within-block energy sum
};

template <int MODE, bool LOCAL>
struct PairOps {
  // one pair: d = r_j - r_i (FP32), w = v_j - v_i (HVP only)
  // i-side accumulators a0,a1,a2; j-side accumulators b0,b1 (already aligned)
  __device__ __forceinline__ static void apply(float dx, float dy, float wx, float wy, float& a0,
                                               float& a1, float& a2, float& b0, float& b1) {
    float r2 = __builtin_fmaf(dx, dx, dy * dy);
    float inv = __builtin_amdgcn_rsqf(r2);
    if (MODE == kEnergy) {
      a2 += inv;
      if (LOCAL) b0 += inv;
    } else if (MODE == kForces) {
      a2 += inv;
      float i3 = inv * inv * inv;
      float tx = dx * i3, ty = dy * i3;
      a0 -= tx;
      a1 -= ty;
      b0 += tx;
      b1 += ty;
    } else {
      float i2 = inv * inv;
      float i3 = i2 * inv;
      float q = 3.0f * i3 * i2;
      float dw = __builtin_fmaf(dx, wx, dy * wy);
      float s = dw * q;
      float kx = __builtin_fmaf(dx, s, -wx * i3);
      float ky = __builtin_fmaf(dy, s, -wy * i3);
      a0 -= kx;
      a1 -= ky;
      b0 += kx;
      b1 += ky;
    }
  }
};

template <int MODE, bool LOCAL, bool NEAR, bool ONESIDED>
struct BlockPair {
  // Processes the 64 x 64 pairs of one block pair for the calling lane.
  // j data (xjh, yjh, xjl, yjl, vxj, vyj) are modified (rotated).
  __device__ __forceinline__ static void run(float xih, float yih, float xil, float yil, float vxi,
                                             float vyi, float vxil, float vyil, float xjh,
                                             float yjh, float xjl, float yjl, float vxj,
                                             float vyj, float vxjl, float vyjl, float& a0,
                                             float& a1, float& a2, float& b0, float& b1,
                                             int lane) {
    const int src = (lane + 16) & 63;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      // step 0: own-lane j (skipped for the self pair of a diagonal block)
      if (!(ONESIDED && p == 0)) {
        float dx = xjh - xih, dy = yjh - yih;
        if (NEAR) {
          dx += xjl - xil;
          dy += yjl - yil;
        }
        float wx = 0.f, wy = 0.f;
        if (MODE == kHvp) {
          wx = vxj - vxi;
          wy = vyj - vyi;
          if (NEAR) {
            wx += vxjl - vxil;
            wy += vyjl - vyil;
          }
        }
        PairOps<MODE, LOCAL>::apply(dx, dy, wx, wy, a0, a1, a2, b0, b1);
      }
#define CD_SYM_STEP(K)                                                      \
  {                                                                         \
    float dx = row_ror<K>(xjh) - xih, dy = row_ror<K>(yjh) - yih;           \
    if (NEAR) {                                                             \
      dx += row_ror<K>(xjl) - xil;                                          \
      dy += row_ror<K>(yjl) - yil;                                          \
    }                                                                       \
    float wx = 0.f, wy = 0.f;                                               \
    if (MODE == kHvp) {                                                     \
      wx = row_ror<K>(vxj) - vxi;                                           \
      wy = row_ror<K>(vyj) - vyi;                                           \
      if (NEAR) {                                                           \
        wx += row_ror<K>(vxjl) - vxil;                                      \
        wy += row_ror<K>(vyjl) - vyil;                                      \
      }                                                                     \
    }                                                                       \
    if (!ONESIDED) {                                                        \
      b0 = row_ror<1>(b0);                                                  \
      if (MODE != kEnergy) b1 = row_ror<1>(b1);                             \
    }                                                                       \
    PairOps<MODE, LOCAL>::apply(dx, dy, wx, wy, a0, a1, a2, b0, b1);        \
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
      if (p < 3) {
        xjh = __shfl(xjh, src, 64);
        yjh = __shfl(yjh, src, 64);
        if (NEAR) {
          xjl = __shfl(xjl, src, 64);
          yjl = __shfl(yjl, src, 64);
        }
        if (MODE == kHvp) {
          vxj = __shfl(vxj, src, 64);
          vyj = __shfl(vyj, src, 64);
          if (NEAR) {
            vxjl = __shfl(vxjl, src, 64);
            vyjl = __shfl(vyjl, src, 64);
          }
        }
      }
    }
  }
};

__device__ __forceinline__ bool boxes_near(const float* box, int I, int J) {
  // gap between the two boxes below twice the larger box diagonal
  float ix0 = box[4 * I], ix1 = box[4 * I + 1], iy0 = box[4 * I + 2], iy1 = box[4 * I + 3];
  float jx0 = box[4 * J], jx1 = box[4 * J + 1], jy0 = box[4 * J + 2], jy1 = box[4 * J + 3];
  float gx = fmaxf(0.f, fmaxf(jx0 - ix1, ix0 - jx1));
  float gy = fmaxf(0.f, fmaxf(jy0 - iy1, iy0 - jy1));
  float di = (ix1 - ix0) * (ix1 - ix0) + (iy1 - iy0) * (iy1 - iy0);
  float dj = (jx1 - jx0) * (jx1 - jx0) + (jy1 - jy0) * (jy1 - jy0);
  return gx * gx + gy * gy < 4.f * fmaxf(di, dj);
}

template <int MODE, bool LOCAL>
__global__ __launch_bounds__(1024) void k_sym(SymArgs a) {
  extern __shared__ double lds[];  // [S][NJ][64]
  constexpr int NJ = (MODE == kEnergy) ? 1 : 2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = blockIdx.x / a.C, c = blockIdx.x % a.C;
  const int I = g * a.W + w;
  const bool wave_ok = I < a.nb;
  const int hmax = a.nb / 2;
  for (int e = threadIdx.x; e < a.S * NJ * kBlk; e += blockDim.x) lds[e] = 0.0;

  double A0 = 0.0, A1 = 0.0, A2 = 0.0;
  float xih = 0.f, yih = 0.f, xil = 0.f, yil = 0.f, vxi = 0.f, vyi = 0.f, vxil = 0.f, vyil = 0.f;
  double cx = 0.0, cy = 0.0, cvx = 0.0, cvy = 0.0;
  if (wave_ok) {
    const int si = I * kBlk + lane;
    cx = a.cen[2 * I];
    cy = a.cen[2 * I + 1];
    double rx = a.xs[si] - cx, ry = a.ys[si] - cy;
    xih = (float)rx;
    yih = (float)ry;
    xil = (float)(rx - (double)xih);
    yil = (float)(ry - (double)yih);
    if (MODE == kHvp) {
      // v is also taken relative to a reference value of block I (its first
      // charge), so that differences of a smooth v keep their precision
      cvx = a.vxs[(size_t)I * kBlk];
      cvy = a.vys[(size_t)I * kBlk];
      double wx = a.vxs[si] - cvx, wy = a.vys[si] - cvy;
      vxi = (float)wx;
      vyi = (float)wy;
      vxil = (float)(wx - (double)vxi);
      vyil = (float)(wy - (double)vyi);
    }
    if (c == 0) {
      // diagonal block: ordered pairs within the block, i side only
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, b0 = 0.f, b1 = 0.f;
      BlockPair<MODE, false, true, true>::run(xih, yih, xil, yil, vxi, vyi, vxil, vyil, xih, yih,
                                              xil, yil, vxi, vyi, vxil, vyil, a0, a1, a2, b0, b1,
                                              lane);
      A0 += (double)a0;
      A1 += (double)a1;
      A2 += a.diag_scale * (double)a2;
    }
  }
  __syncthreads();

  for (int t = 0; t < a.L; ++t) {
    const int o = c * a.L + 1 + t;
    const bool ok = wave_ok && o <= hmax && (2 * o < a.nb || I < hmax);
    if (ok) {
      int J = I + o;
      if (J >= a.nb) J -= a.nb;
      const int sj = J * kBlk + lane;
      double rx = a.xs[sj] - cx, ry = a.ys[sj] - cy;
      float xjh = (float)rx, yjh = (float)ry;
      float vxj = 0.f, vyj = 0.f;
      double wx = 0.0, wy = 0.0;
      if (MODE == kHvp) {
        wx = a.vxs[sj] - cvx;
        wy = a.vys[sj] - cvy;
        vxj = (float)wx;
        vyj = (float)wy;
      }
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, b0 = 0.f, b1 = 0.f;
      if (boxes_near(a.box, I, J)) {
        float xjl = (float)(rx - (double)xjh), yjl = (float)(ry - (double)yjh);
        float vxjl = 0.f, vyjl = 0.f;
        if (MODE == kHvp) {
          vxjl = (float)(wx - (double)vxj);
          vyjl = (float)(wy - (double)vyj);
        }
        BlockPair<MODE, LOCAL, true, false>::run(xih, yih, xil, yil, vxi, vyi, vxil, vyil, xjh,
                                                 yjh, xjl, yjl, vxj, vyj, vxjl, vyjl, a0, a1, a2,
                                                 b0, b1, lane);
      } else {
        BlockPair<MODE, LOCAL, false, false>::run(xih, yih, xil, yil, vxi, vyi, vxil, vyil, xjh,
                                                  yjh, 0.f, 0.f, vxj, vyj, 0.f, 0.f, a0, a1, a2,
                                                  b0, b1, lane);
      }
      A0 += (double)a0;
      A1 += (double)a1;
      A2 += (double)a2;
      if (MODE != kEnergy || LOCAL) {
        double* sl = lds + (size_t)(w + t) * NJ * kBlk;
        sl[lane] += (double)b0;
        if (NJ > 1) sl[kBlk + lane] += (double)b1;
      }
    }
    __syncthreads();
  }

  if (wave_ok) {
    const size_t si = (size_t)c * a.npad + (size_t)I * kBlk + lane;
    if (MODE == kEnergy) {
      a.ip0[si] = A2;
    } else {
      a.ip0[si] = A0;
      a.ip1[si] = A1;
      if (MODE == kForces) a.ip2[si] = A2;
    }
  }
  if (MODE != kEnergy || LOCAL) {
    const size_t base = (size_t)blockIdx.x * a.S * kBlk;
    for (int e = threadIdx.x; e < a.S * kBlk; e += blockDim.x) {
      const int slot = e / kBlk, l = e % kBlk;
      a.jp0[base + e] = lds[(size_t)slot * NJ * kBlk + l];
      if (NJ > 1) a.jp1[base + e] = lds[(size_t)slot * NJ * kBlk + kBlk + l];
    }
  }
}

// Sum of the partials for sorted index s, in a fixed order: i-side chunks,
// then for each chunk the workgroups whose j window contains block B.
struct SymReduceArgs {
  const double* ip0;
  const double* ip1;
  const double* ip2;
  const double* jp0;
  const double* jp1;
  const int32_t* perm;
  int n, nb, npad, W, L, C, G, S;
  double* out0;  // fx | hx | e_local (caller order), may be null
  double* out1;  // fy | hy
  double* eblk;  // per-workgroup energy partial
};

template <int MODE, bool LOCAL>
__global__ __launch_bounds__(256) void k_sym_reduce(SymReduceArgs a) {
  __shared__ double red[4];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v0 = 0.0, v1 = 0.0, ve = 0.0;
  if (s < a.n) {
    const int B = s / kBlk, l = s % kBlk;
    for (int c = 0; c < a.C; ++c) {
      const size_t k = (size_t)c * a.npad + s;
      if (MODE == kEnergy) {
        ve += a.ip0[k];
      } else {
        v0 += a.ip0[k];
        v1 += a.ip1[k];
        if (MODE == kForces) ve += a.ip2[k];
      }
    }
    if (MODE != kEnergy || LOCAL) {
      for (int c = 0; c < a.C; ++c) {
        // workgroup (g, c) holds block J in slot (J - gW - cL - 1) mod nb when
        // that is < S; with u = (B - cL - 1) mod nb the bases gW that qualify
        // are u - slot + k*nb (k = 0, 1, 2), three disjoint ranges
        int u = (B - c * a.L - 1) % a.nb;
        if (u < 0) u += a.nb;
        for (int k = 0; k < 3; ++k) {
          const int hi = u + k * a.nb, lo = hi - a.S + 1;
          int g0 = lo <= 0 ? 0 : (lo + a.W - 1) / a.W;
          int g1 = hi / a.W;
          if (g1 > a.G - 1) g1 = a.G - 1;
          for (int g = g0; g <= g1; ++g) {
            const int slot = hi - g * a.W;
            const size_t q = ((size_t)(g * a.C + c) * a.S + slot) * kBlk + l;
            if (MODE == kEnergy) {
              ve += a.jp0[q];
            } else {
              v0 += a.jp0[q];
              v1 += a.jp1[q];
            }
          }
        }
      }
    }
    const int p = a.perm[s];
    if (MODE == kEnergy) {
      if (LOCAL) {
        ve *= 0.5;
        if (a.out0) a.out0[p] = ve;
      }
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
                                            double& A0, double& A1, double& A2) {
#pragma unroll 4
  for (int jj = 0; jj < jn; ++jj) {
    const double dx = xi - xb[jj], dy = yi - yb[jj];
    const double r2 = __builtin_fma(dx, dx, dy * dy);
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
      one64_block<MODE, true>(xb, yb, vxb, vyb, jn, xi, yi, vxi, vyi, lane, A0, A1, A2);
    else
      one64_block<MODE, false>(xb, yb, vxb, vyb, jn, xi, yi, vxi, vyi, lane, A0, A1, A2);
  }
  const size_t k = (size_t)blockIdx.y * a.npad + si;
  if (MODE == kEnergy) {
    a.p0[k] = A2;
  } else {
    a.p0[k] = A0;
    a.p1[k] = A1;
    if (MODE == kForces) a.p2[k] = A2;
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
        if (MODE == kForces) ve += a.p2[q];
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

// Final energy: one workgroup sums the per-workgroup partials in a fixed
// order (strided per-thread sums, then a fixed tree).
__global__ __launch_bounds__(256) void k_sum_blocks(const double* __restrict__ eblk, int m,
                                                    double* __restrict__ out) {
  __shared__ double red[4];
  double v = 0.0;
  for (int k = threadIdx.x; k < m; k += blockDim.x) v += eblk[k];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
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

// ---------------------------------------------------------------- planning --
bool make_plan(int op, int64_t n64, int precision, char* base, Plan& P) {
  if (n64 < 1 || n64 > (int64_t)1 << 26) return false;
  if (precision != CD_FP64 && precision != CD_MIXED) return false;
  const int n = (int)n64;
  P.n = n;
  P.nb = (n + kBlk - 1) / kBlk;
  P.npad = P.nb * kBlk;
  const int mode = op == CD_OP_ENERGY ? kEnergy : op == CD_OP_FORCES ? kForces : kHvp;
  if (precision == CD_MIXED && op != CD_OP_VALIDATE) {
    P.W = P.nb < 16 ? P.nb : 16;
    int l = P.nb + 1 - P.W;
    P.L = l < 1 ? 1 : (l > 32 ? 32 : l);
    const int hmax = P.nb / 2;
    P.C = hmax > 0 ? (hmax + P.L - 1) / P.L : 1;
    P.G = (P.nb + P.W - 1) / P.W;
    P.S = P.L + P.W - 1;
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
  P.perm = cv.take<int32_t>(P.npad);
  P.perm2 = cv.take<int32_t>(n);
  P.hist = cv.take<uint32_t>(sort_scratch_elems(n));
  P.xs = cv.take<double>(P.npad);
  P.ys = cv.take<double>(P.npad);
  if (op == CD_OP_HVP) {
    P.vxs = cv.take<double>(P.npad);
    P.vys = cv.take<double>(P.npad);
  }
  P.cen = cv.take<double>(2 * (size_t)P.nb);
  P.box = cv.take<float>(4 * (size_t)P.nb);
  if (op != CD_OP_VALIDATE) {
    const size_t q = (precision == CD_MIXED ? (size_t)P.C : (size_t)P.splits) * P.npad;
    P.q0 = cv.take<double>(q);
    if (mode != kEnergy) P.q1 = cv.take<double>(q);
    if (mode == kForces) P.q2 = cv.take<double>(q);
    if (precision == CD_MIXED) {
      const size_t jq = (size_t)P.G * P.C * P.S * kBlk;
      P.j0 = cv.take<double>(jq);
      if (mode != kEnergy) P.j1 = cv.take<double>(jq);
    }
    P.eblk = cv.take<double>(P.nred);
  }
  P.total = cv.off + 256;
  return true;
}

int stage(const Plan& P, const double* x, const double* y, const double* vx,
                 const double* vy, hipStream_t st) {
  const int n = P.n;
  hipLaunchKernelGGL(k_morton, dim3((n + 255) / 256), dim3(256), 0, st, x, y, n, P.keys,
                     P.perm);
  int rc = sort_pairs(P.keys, P.perm, P.keys2, P.perm2, P.hist, n, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_gather, dim3((P.npad + 255) / 256), dim3(256), 0, st, x, y, vx, vy,
                     P.perm, n, P.npad, P.xs, P.ys, P.vxs, P.vys);
  hipLaunchKernelGGL(k_blockinfo, dim3((P.nb + 3) / 4), dim3(256), 0, st, P.xs, P.ys, n, P.nb,
                     P.cen, P.box);
  return hip_status(hipGetLastError());
}

// Measurement hook (coulomb_set_kernel_events): events recorded around the
// dominant pair kernel of the next calls.
static hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

static void mark(hipEvent_t ev, hipStream_t st) {
  if (ev) (void)hipEventRecord(ev, st);
}

template <int MODE, bool LOCAL>
static void run_sym(const Plan& P, hipStream_t st, double* out0, double* out1) {
  SymArgs a;
  a.xs = P.xs;
  a.ys = P.ys;
  a.vxs = P.vxs;
  a.vys = P.vys;
  a.cen = P.cen;
  a.box = P.box;
  a.nb = P.nb;
  a.npad = P.npad;
  a.W = P.W;
  a.L = P.L;
  a.C = P.C;
  a.G = P.G;
  a.S = P.S;
  a.ip0 = P.q0;
  a.ip1 = P.q1;
  a.ip2 = P.q2;
  a.jp0 = P.j0;
  a.jp1 = P.j1;
  a.diag_scale = (MODE == kEnergy && LOCAL) ? 1.0 : 0.5;
  constexpr int NJ = (MODE == kEnergy) ? 1 : 2;
  const size_t lds = (size_t)P.S * NJ * kBlk * sizeof(double);
  mark(g_ev_start, st);
  hipLaunchKernelGGL((k_sym<MODE, LOCAL>), dim3(P.G * P.C), dim3(64 * P.W), lds, st, a);
  mark(g_ev_stop, st);
  SymReduceArgs r;
  r.ip0 = P.q0;
  r.ip1 = P.q1;
  r.ip2 = P.q2;
  r.jp0 = P.j0;
  r.jp1 = P.j1;
  r.perm = P.perm;
  r.n = P.n;
  r.nb = P.nb;
  r.npad = P.npad;
  r.W = P.W;
  r.L = P.L;
  r.C = P.C;
  r.G = P.G;
  r.S = P.S;
  r.out0 = out0;
  r.out1 = out1;
  r.eblk = P.eblk;
  hipLaunchKernelGGL((k_sym_reduce<MODE, LOCAL>), dim3(P.nred), dim3(256), 0, st, r);
}

template <int MODE>
static void run_one64(const Plan& P, hipStream_t st, double* out0, double* out1) {
  OneArgs a;
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

}  // namespace cd

using namespace cd;

extern "C" {

size_t coulomb_workspace_bytes(int op, int64_t n, int32_t n_patches, int64_t total_active,
                               int precision) {
  (void)n_patches;
  (void)total_active;
  if (op == CD_OP_ENERGY || op == CD_OP_FORCES || op == CD_OP_HVP || op == CD_OP_VALIDATE) {
    Plan P;
    if (!make_plan(op, n, op == CD_OP_VALIDATE ? CD_FP64 : precision, nullptr, P)) return 0;
    return P.total;
  }
  if (op == CD_OP_LANCZOS) return cd::lanczos_workspace_bytes(n, n_patches);
  return cd::relax_workspace_bytes(op, n, n_patches, total_active, precision);
}

static int check_ws(int op, int64_t n, int precision, void* ws, size_t ws_bytes, Plan& P) {
  if (!ws) return CD_ERR_WORKSPACE;
  if (!make_plan(op, n, precision, nullptr, P)) return CD_ERR_INVALID_ARG;
  if (ws_bytes < P.total) return CD_ERR_WORKSPACE;
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  make_plan(op, n, precision, base, P);
  return CD_OK;
}

int coulomb_energy(const double* x, const double* y, int64_t n, int precision, double* e_total,
                   double* e_local, void* ws, size_t ws_bytes, void* stream) {
  if (!x || !y || !e_total) return CD_ERR_INVALID_ARG;
  Plan P;
  int rc = check_ws(CD_OP_ENERGY, n, precision, ws, ws_bytes, P);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if ((rc = stage(P, x, y, nullptr, nullptr, st))) return rc;
  if (precision == CD_MIXED) {
    if (e_local) run_sym<kEnergy, true>(P, st, e_local, nullptr);
    else run_sym<kEnergy, false>(P, st, nullptr, nullptr);
  } else {
    run_one64<kEnergy>(P, st, e_local, nullptr);
  }
  hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(256), 0, st, P.eblk, P.nred, e_total);
  return hip_status(hipGetLastError());
}

int coulomb_forces(const double* x, const double* y, int64_t n, int precision, double* fx,
                   double* fy, double* e_total, void* ws, size_t ws_bytes, void* stream) {
  if (!x || !y || !fx || !fy) return CD_ERR_INVALID_ARG;
  Plan P;
  int rc = check_ws(CD_OP_FORCES, n, precision, ws, ws_bytes, P);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if ((rc = stage(P, x, y, nullptr, nullptr, st))) return rc;
  if (precision == CD_MIXED) run_sym<kForces, false>(P, st, fx, fy);
  else run_one64<kForces>(P, st, fx, fy);
  if (e_total)
    hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(256), 0, st, P.eblk, P.nred, e_total);
  return hip_status(hipGetLastError());
}

int coulomb_hvp(const double* x, const double* y, const double* vx, const double* vy, int64_t n,
                int precision, double* hx, double* hy, void* ws, size_t ws_bytes, void* stream) {
  if (!x || !y || !vx || !vy || !hx || !hy) return CD_ERR_INVALID_ARG;
  Plan P;
  int rc = check_ws(CD_OP_HVP, n, precision, ws, ws_bytes, P);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if ((rc = stage(P, x, y, vx, vy, st))) return rc;
  if (precision == CD_MIXED) run_sym<kHvp, false>(P, st, hx, hy);
  else run_one64<kHvp>(P, st, hx, hy);
  return hip_status(hipGetLastError());
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
    default: return "unknown status";
  }
}

}  // extern "C"
