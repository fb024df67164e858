// Element quadrature of the u-dependent terms on the finest Q1 grid:
//   G(u, x)_i = int u^2 x phi_i,  so that  M_E(u) x = 3 G(u, x) - M x
//               (Sec. 2, entries of M_E: int (3u^2 - 1) phi_i phi_j)
//   N(u)_i    = int (u^3 - u) phi_i      (weak form of u(u^2-1) in (okb))
// with u, x the Q1 interpolants.  The integrands are of degree 4 per
// direction, so the 3-point Gauss-Legendre rule per direction is exact.  The
// -M x part of M_E x is applied by the node-stencil kernels that consume G.
//
// Layout of the work: a block of 8 wavefronts covers 7 node rows of the x-y
// plane and streams along z one element layer at a time.  Wavefront w owns
// element row ey = y0 - 1 + w; lane l owns elements ex = l + 64c.  Each lane
// evaluates its element by sum factorisation (2^d corners -> 3^d Gauss points
// -> integrand -> 2^d corner contributions).  Contributions are summed into
// nodes deterministically: along x with cross-lane shuffles, along y through
// LDS (wavefront w reads w-1), along z with a carry that each lane keeps in
// its own LDS slots (one per element slot along x).
#include "ok_internal.h"

#include <algorithm>

namespace okd {

namespace {

constexpr int kRows = 7;              // node rows per block
constexpr int kWaves = kRows + 1;     // one halo element row

// Gauss points 1/2 -+ sqrt(15)/10 and 1/2 on [0,1], weights 5/18, 8/18, 5/18.
constexpr double kG0 = 0.11270166537925831148;
constexpr double kW0 = 5.0 / 18.0;
constexpr double kW1 = 8.0 / 18.0;

__device__ __forceinline__ double ld(const double* p) { return *p; }
__device__ __forceinline__ double ld(const float* p) { return (double)*p; }

// Positions of the 3 Gauss points on [0,1].
constexpr double kGq[3] = {kG0, 0.5, 1.0 - kG0};

// Values at the 3 Gauss points of the linear interpolant of (v0, v1): one
// difference and one fused multiply-add per point.
__device__ __forceinline__ void lerp3(double v0, double v1, double* o) {
  const double d = v1 - v0;
  o[0] = fma(kGq[0], d, v0);
  o[1] = fma(kGq[1], d, v0);
  o[2] = fma(kGq[2], d, v0);
}

// Transpose of lerp3 with the Gauss weights folded in: contributions of the
// 3 Gauss-point values of one direction to the 2 ends.
constexpr double kPa = (1.0 - kG0) * kW0;
constexpr double kPb = 0.5 * kW1;
constexpr double kPc = kG0 * kW0;
__device__ __forceinline__ void proj3(const double* t, double& o0, double& o1) {
  double m = kPb * t[1];
  o0 = kPa * t[0] + m + kPc * t[2];
  o1 = kPc * t[0] + m + kPa * t[2];
}

// Linear interpolant at Gauss point q from v0 and d = v1 - v0 (as lerp3
// computes it).
__device__ __forceinline__ double lerp_at(double v0, double d, int q) {
  return fma(kGq[q], d, v0);
}
// Weight of Gauss point q in the projection to end 0 / end 1 (proj3).
__device__ __forceinline__ double pw0(int q) { return q == 0 ? kPa : q == 1 ? kPb : kPc; }
__device__ __forceinline__ double pw1(int q) { return q == 0 ? kPc : q == 1 ? kPb : kPa; }

// One 3D element: corners v[az][ay][ax] of u and x; returns corner
// contributions E[az][ay][ax] without the h^3 factor.  Sum factorisation
// ordered to keep few values live: the four x-edges are interpolated to
// their Gauss points once, then for each Gauss row qy the y- and
// z-interpolants, the integrand and its z-projection, accumulated straight
// into the y-projection; the x-projection comes last.
template <int MODE>
__device__ __forceinline__ void element3(const double (&u)[2][2][2], const double (&x)[2][2][2],
                                         double (&E)[2][2][2]) {
  double ue[2][2][3], xe[2][2][3];  // [az][ay][qx]
  for (int az = 0; az < 2; az++)
    for (int ay = 0; ay < 2; ay++) {
      lerp3(u[az][ay][0], u[az][ay][1], ue[az][ay]);
      if (MODE == 0) lerp3(x[az][ay][0], x[az][ay][1], xe[az][ay]);
    }
  // y-differences of the x-edge interpolants, shared by the three Gauss rows
  double ud[2][3], xd[2][3];  // [az][qx]
  for (int az = 0; az < 2; az++)
    for (int qx = 0; qx < 3; qx++) {
      ud[az][qx] = ue[az][1][qx] - ue[az][0][qx];
      xd[az][qx] = (MODE == 0) ? xe[az][1][qx] - xe[az][0][qx] : 0.0;
    }
  double acc[2][2][3];  // [az][ay][qx]: z- and y-projected integrand
  for (int az = 0; az < 2; az++)
    for (int ay = 0; ay < 2; ay++)
      for (int qx = 0; qx < 3; qx++) acc[az][ay][qx] = 0.0;
#pragma unroll
  for (int qy = 0; qy < 3; qy++) {
    const double wy0 = pw0(qy), wy1 = pw1(qy);
#pragma unroll
    for (int qx = 0; qx < 3; qx++) {
      const double u0 = lerp_at(ue[0][0][qx], ud[0][qx], qy);
      const double u1 = lerp_at(ue[1][0][qx], ud[1][qx], qy);
      double f[3];
      if (MODE == 0) {
        const double x0 = lerp_at(xe[0][0][qx], xd[0][qx], qy);
        const double x1 = lerp_at(xe[1][0][qx], xd[1][qx], qy);
        double uq[3], xq[3];
        lerp3(u0, u1, uq);
        lerp3(x0, x1, xq);
        for (int qz = 0; qz < 3; qz++) f[qz] = (uq[qz] * uq[qz]) * xq[qz];
      } else {
        double uq[3];
        lerp3(u0, u1, uq);
        for (int qz = 0; qz < 3; qz++) f[qz] = (uq[qz] * uq[qz]) * uq[qz] - uq[qz];
      }
      double fb, ft;
      proj3(f, fb, ft);
      acc[0][0][qx] += wy0 * fb;
      acc[0][1][qx] += wy1 * fb;
      acc[1][0][qx] += wy0 * ft;
      acc[1][1][qx] += wy1 * ft;
    }
  }
  for (int az = 0; az < 2; az++)
    for (int ay = 0; ay < 2; ay++) proj3(acc[az][ay], E[az][ay][0], E[az][ay][1]);
}

template <int MODE>
__device__ __forceinline__ void element2(const double (&u)[2][2], const double (&x)[2][2],
                                         double (&E)[2][2]) {
  double uq[3][3], xq[3][3];
  {
    double a[2][3];
    for (int ay = 0; ay < 2; ay++) lerp3(u[ay][0], u[ay][1], a[ay]);
    for (int qx = 0; qx < 3; qx++) {
      double t[3];
      lerp3(a[0][qx], a[1][qx], t);
      for (int qy = 0; qy < 3; qy++) uq[qy][qx] = t[qy];
    }
  }
  if (MODE == 0) {
    double a[2][3];
    for (int ay = 0; ay < 2; ay++) lerp3(x[ay][0], x[ay][1], a[ay]);
    for (int qx = 0; qx < 3; qx++) {
      double t[3];
      lerp3(a[0][qx], a[1][qx], t);
      for (int qy = 0; qy < 3; qy++) xq[qy][qx] = t[qy];
    }
  }
  for (int qy = 0; qy < 3; qy++)
    for (int qx = 0; qx < 3; qx++) {
      double v = uq[qy][qx];
      if (MODE == 0)
        uq[qy][qx] = (v * v) * xq[qy][qx];
      else
        uq[qy][qx] = (v * v) * v - v;
    }
  double a[2][3];
  for (int qx = 0; qx < 3; qx++) {
    double t[3] = {uq[0][qx], uq[1][qx], uq[2][qx]};
    proj3(t, a[0][qx], a[1][qx]);
  }
  for (int ay = 0; ay < 2; ay++) proj3(a[ay], E[ay][0], E[ay][1]);
}

struct EShape {
  int epl;       // elements per lane along x: ceil(N/64)
  int rowtiles;  // ceil((N+1)/kRows)
  int zc, nzc;   // most planes per block, z-chunks (planes split evenly)
};

// Blocks of one launch that are resident at once: two blocks of 8 wavefronts
// per CU (at most 128 VGPRs per lane) on 256 CUs.
constexpr int64_t kResidentBlocks = 512;

// z-chunks: a block's time grows with its element layers (zc + 1, one halo
// layer), the launch's with the rounds of resident blocks; the count of
// chunks minimises rounds * (zc + 1).
EShape element_shape(const Grid& g, int count) {
  EShape s;
  s.epl = (g.N + 63) / 64;
  s.rowtiles = (g.nn + kRows - 1) / kRows;
  s.zc = 1;
  s.nzc = 1;
  if (g.dim == 3) {
    int64_t best = -1;
    for (int nzc = 1; nzc <= std::min(g.nn, 128); nzc++) {
      const int zc = (g.nn + nzc - 1) / nzc;  // planes of the largest chunk
      const int64_t blocks = (int64_t)s.rowtiles * nzc * std::max(count, 1);
      const int64_t cost = ((blocks + kResidentBlocks - 1) / kResidentBlocks) * (zc + 1);
      if (best < 0 || cost < best) {
        best = cost;
        s.nzc = nzc;
        s.zc = zc;
      }
    }
  }
  return s;
}

// Elements per lane along x (epl) from the shape; the element-slot loop is
// not unrolled, so the live registers are those of one element and two
// blocks of 8 wavefronts fit on a CU.
constexpr int kMaxEpl = 8;
template <int DIM, int MODE, class TX, class TO>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(4, 8)))
    k_element(Vec<const double> uv, Vec<const TX> xv, Vec<const double> addv, Vec<TO> outv,
              Grid g, EShape sh, Batch B, double alpha, double beta) {
  constexpr int NZ = (DIM == 3) ? 2 : 1;  // corner layers per element
  __shared__ double xch[2][kWaves][NZ][64];
  __shared__ double carry[(DIM == 3) ? kWaves : 1][kMaxEpl + 1][64];  // lane-private
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int per = sh.rowtiles * sh.nzc;
  const int inst = lb / per;
  if (B.act && !B.act[inst]) return;
  const int b = lb - inst * per;
  const int rt = b % sh.rowtiles;
  const int zch = b / sh.rowtiles;
  const double* __restrict__ u = uv.at(inst);
  const TX* __restrict__ x = xv.null() ? nullptr : xv.at(inst);
  const double* __restrict__ add = addv.null() ? nullptr : addv.at(inst);
  TO* __restrict__ out = outv.at(inst);
  const int N = g.N, nn = g.nn;
  const int64_t plane = g.plane;
  const int y0 = rt * kRows;
  const int ey = y0 - 1 + w;          // element row of this wavefront
  const bool row_ok = (ey >= 0 && ey < N);
  const bool out_row = (w >= 1 && ey <= N);  // node row ey is output by this wavefront
  const double hd = (DIM == 3) ? g.h * g.h * g.h : g.h * g.h;
  const double sc = alpha * hd;

  int z0 = 0, z1 = 1;
  if (DIM == 3) {
    z0 = (int)(((int64_t)zch * nn) / sh.nzc);
    z1 = (int)(((int64_t)(zch + 1) * nn) / sh.nzc);
  }
  const int epl = sh.epl;
  if constexpr (DIM == 3)
    for (int c = 0; c <= epl; c++) carry[w][c][lane] = 0.0;

  const int lz0 = (DIM == 3) ? z0 - 1 : 0;
  const int lz1 = (DIM == 3) ? z1 - 1 : 0;
  int buf = 0;
  for (int ez = lz0; ez <= lz1; ez++) {
    const bool layer_ok = (DIM == 2) || (ez >= 0 && ez < N);
    double prevR[2][NZ];  // lane-63 right contributions of the previous slot
    for (int a = 0; a < 2; a++)
      for (int cz = 0; cz < NZ; cz++) prevR[a][cz] = 0.0;
#pragma unroll 1
    for (int c = 0; c <= epl; c++) {
      const int i = lane + 64 * c;
      double L[2][NZ], R[2][NZ];  // [ay][cz]: left (ax=0) and right (ax=1) corner parts
      for (int a = 0; a < 2; a++)
        for (int cz = 0; cz < NZ; cz++) L[a][cz] = R[a][cz] = 0.0;
      if (c < epl && row_ok && layer_ok && i < N) {
        if (DIM == 3) {
          double uc[2][2][2], xc[2][2][2], E[2][2][2];
          for (int az = 0; az < 2; az++)
            for (int ay = 0; ay < 2; ay++) {
              int64_t base = (int64_t)(ez + az) * plane + (int64_t)(ey + ay) * nn + i;
              uc[az][ay][0] = u[base];
              uc[az][ay][1] = u[base + 1];
              if (MODE == 0) {
                xc[az][ay][0] = ld(x + base);
                xc[az][ay][1] = ld(x + base + 1);
              } else {
                xc[az][ay][0] = xc[az][ay][1] = 0.0;
              }
            }
          element3<MODE>(uc, xc, E);
          for (int ay = 0; ay < 2; ay++)
            for (int az = 0; az < 2; az++) {
              L[ay][az] = E[az][ay][0];
              R[ay][az] = E[az][ay][1];
            }
        } else {
          double uc[2][2], xc[2][2], E[2][2];
          for (int ay = 0; ay < 2; ay++) {
            int64_t base = (int64_t)(ey + ay) * nn + i;
            uc[ay][0] = u[base];
            uc[ay][1] = u[base + 1];
            if (MODE == 0) {
              xc[ay][0] = ld(x + base);
              xc[ay][1] = ld(x + base + 1);
            } else {
              xc[ay][0] = xc[ay][1] = 0.0;
            }
          }
          element2<MODE>(uc, xc, E);
          for (int ay = 0; ay < 2; ay++) {
            L[ay][0] = E[ay][0];
            R[ay][0] = E[ay][1];
          }
        }
      }
      // x: node i gets L of element i and R of element i-1 (lane-1, or lane 63
      // of the previous slot).
      double X[2][NZ];
      for (int a = 0; a < 2; a++)
        for (int cz = 0; cz < NZ; cz++) {
          double up = __shfl_up(R[a][cz], 1);
          X[a][cz] = L[a][cz] + (lane >= 1 ? up : prevR[a][cz]);
          prevR[a][cz] = __shfl(R[a][cz], 63);
        }
      // y: node row ey gets the ay=0 parts of row ey and the ay=1 parts of row ey-1.
      for (int cz = 0; cz < NZ; cz++) xch[buf][w][cz][lane] = X[1][cz];
      __syncthreads();
      if (out_row) {
        double tot[NZ];
        for (int cz = 0; cz < NZ; cz++) tot[cz] = X[0][cz] + xch[buf][w - 1][cz][lane];
        const bool node_ok = (i <= N);
        if constexpr (DIM == 2) {
          if (node_ok) {
            int64_t idx = (int64_t)ey * nn + i;
            double v = sc * tot[0];
            if (add) v += beta * add[idx];
            out[idx] = (TO)v;
          }
        } else {
          if (ez >= z0 && node_ok) {
            int64_t idx = (int64_t)ez * plane + (int64_t)ey * nn + i;
            double v = sc * (carry[w][c][lane] + tot[0]);
            if (add) v += beta * add[idx];
            out[idx] = (TO)v;
          }
          carry[w][c][lane] = tot[NZ - 1];
        }
      }
      buf ^= 1;
    }
  }
}

}  // namespace

template <class TX, class TO>
hipError_t launch_element(const Grid& g, const Batch& B, int mode, Vec<const double> u,
                          Vec<const TX> x, Vec<const double> add, double alpha, double beta,
                          Vec<TO> out, hipStream_t st) {
  EShape sh = element_shape(g, B.count);
  int64_t blocks = (int64_t)sh.rowtiles * sh.nzc * B.count;
  if (blocks > 0x7fffffff || B.count < 1) return hipErrorInvalidValue;
  dim3 grid((unsigned)blocks), block(64 * kWaves);
#define OKD_EL(D, M)                                                                        \
  hipLaunchKernelGGL((k_element<D, M, TX, TO>), grid, block, 0, st, u, x, add, out, g, sh, B, \
                     alpha, beta)
  if (g.dim == 3 && sh.epl > kMaxEpl) return hipErrorInvalidValue;
  if (g.dim == 2) {
    if (mode == 0) OKD_EL(2, 0); else OKD_EL(2, 1);
  } else {
    if (mode == 0) OKD_EL(3, 0); else OKD_EL(3, 1);
  }
#undef OKD_EL
  return hipGetLastError();
}

template hipError_t launch_element<double, double>(const Grid&, const Batch&, int,
                                                   Vec<const double>, Vec<const double>,
                                                   Vec<const double>, double, double,
                                                   Vec<double>, hipStream_t);
template hipError_t launch_element<float, double>(const Grid&, const Batch&, int,
                                                  Vec<const double>, Vec<const float>,
                                                  Vec<const double>, double, double,
                                                  Vec<double>, hipStream_t);

}  // namespace okd
