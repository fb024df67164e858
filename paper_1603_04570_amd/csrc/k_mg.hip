// Multigrid transfers between nested uniform Q1 grids and the exact
// coarse-grid solve of M + alpha K.
//
// Prolongation P is Q1 interpolation from N/2 to N elements per direction:
// a fine node copies the coarse node at an even index and averages the two
// coarse neighbours at an odd index, direction by direction (tensor product
// of the 1D weights 1 and 1/2).  Restriction is its transpose R = P^T, the
// finite-element restriction that makes P^T A_h P equal the rediscretised
// coarse operator.
//
// Coarse solve: on a uniform grid with Neumann ends the DCT-I vectors
// v_k(j) = cos(k pi j / N) diagonalise M + alpha K in the sense
// (M + alpha K) V = W V Lambda, with W the trapezoid weights and
// Lambda_k = prod mu + alpha sum kap prod mu (mu = (h/3)(2 + cos), kap =
// (2/h)(1 - cos)), and V^T W V = Gamma = diag(N/2, with N at k = 0, N).
// Hence (M + alpha K)^-1 = V (Lambda Gamma)^-1 V^T; V is symmetric.
#include "ok_internal.h"

#include <algorithm>

namespace okd {

namespace {

__device__ __forceinline__ double ld(const double* p) { return *p; }
__device__ __forceinline__ double ld(const float* p) { return (double)*p; }

// q / nn and q % nn for q < 2^31 without an integer division: the double
// product q * (1/nn) is within 5e-7 of q/nn, whose fractional part is 0 or at
// least 1/nn, so its truncation is the quotient or one less; the remainder
// test corrects it.
__device__ __forceinline__ unsigned qdiv(unsigned q, unsigned nn, double rnn, unsigned& rem) {
  unsigned d = (unsigned)((double)q * rnn);
  int r = (int)(q - d * nn);
  if (r < 0) {
    d--;
    r += (int)nn;
  } else if (r >= (int)nn) {
    d++;
    r -= (int)nn;
  }
  rem = (unsigned)r;
  return d;
}

// One thread per node of the output grid, flat index q per instance (< 2^31
// nodes): q = i + nn (j + nn k).
template <int DIM>
__device__ __forceinline__ void node_ijk(unsigned q, const Grid& g, int& i, int& j, int& k) {
  const unsigned nn = (unsigned)g.nn;
  unsigned ri, rj;
  const unsigned row = qdiv(q, nn, g.rnn, ri);
  i = (int)ri;
  if (DIM == 3) {
    k = (int)qdiv(row, nn, g.rnn, rj);
    j = (int)rj;
  } else {
    j = (int)row;
    k = 0;
  }
}

// Restriction gathers straight from global memory (its 27 loads per coarse
// node keep enough bytes in flight); every load is issued before the first
// one is used, from clamped (in-bounds) indices: terms outside the grid are loaded anyway and
// then left out of the sum, which keeps the summation order (and so every
// bit) of the plain nested loops over the stencil while no load waits behind
// a lane-dependent branch.
template <int DIM, class T>
__global__ void __launch_bounds__(256)
    k_restrict(Vec<const T> rv, Vec<T> bcv, Grid f, Grid c, Batch B, int per) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = lb / per;
  if (B.act && !B.act[inst]) return;
  const unsigned q = (unsigned)(lb - inst * per) * blockDim.x + threadIdx.x;
  if (q >= (unsigned)c.nodes) return;
  int ci, cj, ck;
  node_ijk<DIM>(q, c, ci, cj, ck);
  const T* __restrict__ r = rv.at(inst);
  constexpr int NZ = (DIM == 3) ? 3 : 1;
  int64_t off[NZ][3];
  int fi[3];
  bool ok[NZ][3], oki[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const int x = 2 * ci + d - 1;
    oki[d] = (x >= 0 && x <= f.N);
    fi[d] = x < 0 ? 0 : (x > f.N ? f.N : x);
  }
#pragma unroll
  for (int a = 0; a < NZ; a++) {
    const int z = (DIM == 3) ? 2 * ck + a - 1 : 0;
    const bool okz = (z >= 0 && z <= f.N);
    const int zc = z < 0 ? 0 : (z > f.N ? f.N : z);
#pragma unroll
    for (int bb = 0; bb < 3; bb++) {
      const int y = 2 * cj + bb - 1;
      ok[a][bb] = okz && (y >= 0 && y <= f.N);
      const int yc = y < 0 ? 0 : (y > f.N ? f.N : y);
      off[a][bb] = (int64_t)zc * f.plane + (int64_t)yc * f.nn;
    }
  }
  T v[NZ][3][3];
#pragma unroll
  for (int a = 0; a < NZ; a++)
#pragma unroll
    for (int bb = 0; bb < 3; bb++)
#pragma unroll
      for (int d = 0; d < 3; d++) v[a][bb][d] = r[off[a][bb] + fi[d]];
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < NZ; a++) {
    const double wk = (DIM == 3 && a != 1) ? 0.5 : 1.0;
#pragma unroll
    for (int bb = 0; bb < 3; bb++) {
      const double wj = wk * (bb != 1 ? 0.5 : 1.0);
#pragma unroll
      for (int d = 0; d < 3; d++) {
        const double t = wj * (d != 1 ? 0.5 : 1.0) * ld(&v[a][bb][d]);
        s += (ok[a][bb] && oki[d]) ? t : 0.0;
      }
    }
  }
  bcv.at(inst)[q] = (T)s;
}

// 3D restriction streamed along z: a block owns a tile of kRsTI x kRsTJ
// coarse nodes (x, y) and a chunk of coarse planes; each fine plane of its
// footprint (2 kRsTJ + 1 rows of 2 ti + 1 nodes, zero outside the grid) is
// read once, staged in LDS (double-buffered, one barrier per plane), combined
// along x and y with the weights (1/2, 1, 1/2), and accumulated along z in a
// register: fine plane 2K adds to coarse plane K with weight 1, plane 2K + 1
// with weight 1/2 to K and to K + 1.  The next plane's loads are issued
// before the current plane is combined.
constexpr int kRsTI = 64, kRsTJ = 4;
constexpr int kRsFC = 2 * kRsTI + 1, kRsFR = 2 * kRsTJ + 1;
constexpr int kRsLoads = (kRsFC * kRsFR + 255) / 256;

template <class T>
__global__ void __launch_bounds__(256)
    k_restrict_zs(Vec<const T> rv, Vec<T> bcv, Grid f, Grid c, Batch B, int tx, int ty, int ti,
                  int kc, int nzc) {
  __shared__ double F[2][kRsFR][kRsFC];
  const int per = tx * ty * nzc;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = lb / per;
  if (B.act && !B.act[inst]) return;
  int rem = lb - inst * per;
  const int bx = rem % tx;
  rem /= tx;
  const int by = rem % ty, bz = rem / ty;
  const int I0 = bx * ti, J0 = by * kRsTJ;
  const int K0 = bz * kc, K1 = min(K0 + kc, c.nn);
  const int z0 = max(2 * K0 - 1, 0), z1 = min(2 * K1 - 1, f.N);
  const T* __restrict__ r = rv.at(inst);
  T* __restrict__ bc = bcv.at(inst);
  // this thread's staging slots: fine (row, col) of the footprint, its
  // offset in a fine plane (-1 outside the grid) and its LDS word
  const int ncol = 2 * ti + 1, nel = kRsFR * ncol;
  int off[kRsLoads], lw[kRsLoads];
#pragma unroll
  for (int u = 0; u < kRsLoads; u++) {
    const int e = threadIdx.x + 256 * u;
    off[u] = -1;
    lw[u] = -1;
    if (e < nel) {
      const int row = e / ncol, col = e - row * ncol;
      lw[u] = row * kRsFC + col;
      const int fy = 2 * J0 - 1 + row, fx = 2 * I0 - 1 + col;
      if (fy >= 0 && fy <= f.N && fx >= 0 && fx <= f.N) off[u] = fy * f.nn + fx;
    }
  }
  // output node of this thread
  const int i = threadIdx.x % kRsTI, j = threadIdx.x / kRsTI;
  const bool out_ok = i < ti && I0 + i < c.nn && J0 + j < c.nn;
  const int64_t oq = (int64_t)(J0 + j) * c.nn + (I0 + i);
  double pf[kRsLoads];
#pragma unroll
  for (int u = 0; u < kRsLoads; u++)
    pf[u] = off[u] >= 0 ? ld(r + (int64_t)z0 * f.plane + off[u]) : 0.0;
  double acc = 0.0;
  int buf = 0;
  for (int zf = z0; zf <= z1; zf++) {
#pragma unroll
    for (int u = 0; u < kRsLoads; u++)
      if (lw[u] >= 0) (&F[buf][0][0])[lw[u]] = pf[u];
    if (zf < z1) {
#pragma unroll
      for (int u = 0; u < kRsLoads; u++)
        pf[u] = off[u] >= 0 ? ld(r + (int64_t)(zf + 1) * f.plane + off[u]) : 0.0;
    }
    __syncthreads();
    double p = 0.0;
    if (out_ok) {
#pragma unroll
      for (int dy = 0; dy < 3; dy++) {
        const double* row = &F[buf][2 * j + dy][2 * i];
        const double t = 0.5 * row[0] + row[1] + 0.5 * row[2];
        p += (dy == 1 ? 1.0 : 0.5) * t;
      }
    }
    if ((zf & 1) == 0) {
      acc += p;
      if (zf == f.N && out_ok) bc[(int64_t)(zf >> 1) * c.plane + oq] = (T)acc;
    } else {
      const int K = zf >> 1;
      acc += 0.5 * p;
      if (K >= K0 && out_ok) bc[(int64_t)K * c.plane + oq] = (T)acc;
      acc = 0.5 * p;
    }
    buf ^= 1;
  }
}

// Prolongation works on one coarse row (J, K) and a segment of at most
// kProlongW coarse nodes along x per block: the four coarse rows that the
// segment's fine nodes interpolate from are staged in LDS with coalesced
// loads, and every fine node gathers its (up to) eight coarse values from
// LDS; gathering them from global memory costs more than the HBM traffic of
// the transfer.  Sums run in the order of the nested loops over the stencil
// (z, then y, then x offsets), skipping the terms a fine node does not have.
constexpr int kProlongW = 256;    // coarse nodes per prolongation block

template <int DIM, class T>
__global__ void __launch_bounds__(256)
    k_prolong_add(Vec<const T> ecv, Vec<T> xv, Grid f, Grid c, Batch B, int nseg) {
  constexpr int NZ = (DIM == 3) ? 2 : 1;  // coarse planes K, K+1
  constexpr int LW = kProlongW + 1;       // coarse x values per staged row
  __shared__ double cr[NZ][2][LW];
  const int per = nseg * c.nn * (DIM == 3 ? c.nn : 1);
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = lb / per;
  if (B.act && !B.act[inst]) return;
  int rem = lb - inst * per;
  const int seg = rem % nseg;
  rem /= nseg;
  const int J = rem % c.nn, K = (DIM == 3) ? rem / c.nn : 0;
  const int I0 = (int)((int64_t)seg * c.nn / nseg), I1 = (int)((int64_t)(seg + 1) * c.nn / nseg);
  const T* __restrict__ ec = ecv.at(inst);
  T* __restrict__ x = xv.at(inst);
  // fine nodes (2I0 .. min(2 I1, nn_f) - 1) x rows 2J + a x planes 2K + b:
  // thread t owns columns t and t + 256 of every fine row of the block, and
  // issues all its loads of x before the first sum (enough bytes in flight
  // to stream at HBM rate), before the coarse rows are staged
  const int nfx = min(2 * I1, f.nn) - 2 * I0;
  constexpr int kCols = 2 * kProlongW / 256;  // columns per thread
  constexpr int kRowsP = 2 * NZ;              // fine rows per block
  T xo[kRowsP][kCols];
  int64_t qo[kRowsP][kCols];
#pragma unroll
  for (int rr = 0; rr < kRowsP; rr++) {
    const int a = rr & 1, b = rr >> 1;  // fine row 2J + a, plane 2K + b
    const int fj = 2 * J + a, fk = 2 * K + b;
    const bool row_ok = fj <= f.N && (DIM == 2 || fk <= f.N);
#pragma unroll
    for (int v = 0; v < kCols; v++) {
      const int ix = threadIdx.x + 256 * v;
      qo[rr][v] = -1;
      if (row_ok && ix < nfx) {
        const int fi = 2 * I0 + ix;
        const int64_t q =
            (DIM == 3) ? ((int64_t)fk * f.nn + fj) * f.nn + fi : (int64_t)fj * f.nn + fi;
        qo[rr][v] = q;
        xo[rr][v] = x[q];
      }
    }
  }
  // coarse rows J, J+1 of planes K, K+1 (clamped to the grid; a clamped row
  // only feeds fine rows that do not exist)
  for (int t = threadIdx.x; t < NZ * 2 * LW; t += blockDim.x) {
    const int o = t % LW, rr = t / LW;
    const int dy = rr & 1, dz = rr >> 1;
    const int Ic = min(I0 + o, c.N), Jc = min(J + dy, c.N), Kc = min(K + dz, c.N);
    cr[dz][dy][o] = ld(ec + ((int64_t)Kc * c.plane + (int64_t)Jc * c.nn + Ic));
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < kRowsP; rr++) {
    const int a = rr & 1, b = rr >> 1;
    const bool two_j = a != 0, two_k = b != 0;
    const double wk = two_k ? 0.5 : 1.0;
    const double wj = wk * (two_j ? 0.5 : 1.0);
#pragma unroll
    for (int v = 0; v < kCols; v++) {
      if (qo[rr][v] < 0) continue;
      const int ix = threadIdx.x + 256 * v;
      const int fi = 2 * I0 + ix;
      const int li0 = (fi >> 1) - I0, li1 = ((fi + 1) >> 1) - I0;
      const bool two_i = (fi & 1) != 0;
      const double wi = two_i ? 0.5 : 1.0;
      double s = 0.0;
#pragma unroll
      for (int za = 0; za < NZ; za++) {
        if (za && !two_k) break;
#pragma unroll
        for (int yb = 0; yb < 2; yb++) {
          if (yb && !two_j) break;
          s += wj * wi * cr[za][yb][li0];
          if (two_i) s += wj * wi * cr[za][yb][li1];
        }
      }
      x[qo[rr][v]] = (T)(ld(&xo[rr][v]) + s);
    }
  }
}

constexpr int kCoarseMax = 1024;   // nodes of the coarse grid
constexpr int kCoarseLine = 64;    // nodes per direction

// One block per instance solves (M + alpha K) x = b exactly on a grid of at
// most 1024 nodes.
template <int DIM, class T>
__global__ void __launch_bounds__(1024)
    k_coarse(Vec<const T> bv, Vec<T> xv, Grid g, Batch bt) {
  const int inst = blockIdx.x;
  if (bt.act && !bt.act[inst]) return;
  const T* __restrict__ b = bv.at(inst);
  T* __restrict__ x = xv.at(inst);
  const double alpha = bt.coef[inst].alpha;
  __shared__ double A[kCoarseMax], B[kCoarseMax];
  __shared__ double V[kCoarseLine * kCoarseLine];
  __shared__ double mu[kCoarseLine], kap[kCoarseLine], gam[kCoarseLine];
  const int nn = g.nn, N = g.N;
  const int n = (int)g.nodes;
  const int t = threadIdx.x;
  for (int q = t; q < nn * nn; q += blockDim.x) {
    int j = q / nn, k = q % nn;
    V[q] = cospi((double)(j * k % (2 * N)) / (double)N);
  }
  if (t < nn) {
    double c = cospi((double)t / (double)N);
    mu[t] = (g.h / 3.0) * (2.0 + c);
    kap[t] = (2.0 / g.h) * (1.0 - c);
    gam[t] = (t == 0 || t == N) ? (double)N : 0.5 * N;
  }
  for (int q = t; q < n; q += blockDim.x) A[q] = ld(b + q);
  __syncthreads();
  // forward transform along each axis: out[..k..] = sum_j V[j][k] in[..j..]
  double* src = A;
  double* dst = B;
  for (int ax = 0; ax < DIM; ax++) {
    int64_t stride = (ax == 0) ? 1 : (ax == 1 ? nn : (int64_t)nn * nn);
    for (int q = t; q < n; q += blockDim.x) {
      int k = (int)((q / stride) % nn);
      int base = q - k * (int)stride;
      double s = 0.0;
      for (int j = 0; j < nn; j++) s += V[j * nn + k] * src[base + j * stride];
      dst[q] = s;
    }
    __syncthreads();
    double* tt = src;
    src = dst;
    dst = tt;
  }
  for (int q = t; q < n; q += blockDim.x) {
    int k0 = q % nn, k1 = (q / nn) % nn, k2 = (DIM == 3) ? q / (nn * nn) : 0;
    double lam, gg;
    if (DIM == 3) {
      double pm = mu[k0] * mu[k1] * mu[k2];
      double sk = kap[k0] * mu[k1] * mu[k2] + mu[k0] * kap[k1] * mu[k2] + mu[k0] * mu[k1] * kap[k2];
      lam = pm + alpha * sk;
      gg = gam[k0] * gam[k1] * gam[k2];
    } else {
      double pm = mu[k0] * mu[k1];
      double sk = kap[k0] * mu[k1] + mu[k0] * kap[k1];
      lam = pm + alpha * sk;
      gg = gam[k0] * gam[k1];
    }
    src[q] = src[q] / (lam * gg);
  }
  __syncthreads();
  for (int ax = 0; ax < DIM; ax++) {
    int64_t stride = (ax == 0) ? 1 : (ax == 1 ? nn : (int64_t)nn * nn);
    for (int q = t; q < n; q += blockDim.x) {
      int k = (int)((q / stride) % nn);
      int base = q - k * (int)stride;
      double s = 0.0;
      for (int j = 0; j < nn; j++) s += V[k * nn + j] * src[base + j * stride];
      dst[q] = s;
    }
    __syncthreads();
    double* tt = src;
    src = dst;
    dst = tt;
  }
  for (int q = t; q < n; q += blockDim.x) x[q] = (T)src[q];
}

// Coarse grids larger than one block's LDS: the same fast diagonalisation,
// one pass per axis through global scratch.  Pass `ax` maps in -> out with
// out[..k..] = sum_j V[j][k] in[..j..] along axis ax (V symmetric, so the
// forward and backward transforms are the same pass); k_coarse_scale divides
// by Lambda Gamma.  V is rebuilt in LDS by every block (nn <= 64).
template <class TI, class TO>
__global__ void __launch_bounds__(256)
    k_coarse_axis(Vec<const TI> inv, Vec<TO> outv, Grid g, Batch bt, int ax, int per) {
  const int inst = blockIdx.x / per;
  if (bt.act && !bt.act[inst]) return;
  __shared__ double V[kCoarseLine * kCoarseLine];
  const int nn = g.nn, N = g.N;
  for (int q = threadIdx.x; q < nn * nn; q += blockDim.x) {
    const int j = q / nn, k = q % nn;
    V[q] = cospi((double)(j * k % (2 * N)) / (double)N);
  }
  __syncthreads();
  const unsigned q = (unsigned)(blockIdx.x - inst * per) * blockDim.x + threadIdx.x;
  if (q >= (unsigned)g.nodes) return;
  const unsigned stride = (ax == 0) ? 1u : (ax == 1 ? (unsigned)nn : (unsigned)(nn * nn));
  const int k = (int)((q / stride) % (unsigned)nn);
  const unsigned base = q - (unsigned)k * stride;
  const TI* in = inv.at(inst);
  double s = 0.0;
  for (int j = 0; j < nn; j++) s += V[j * nn + k] * ld(in + base + (unsigned)j * stride);
  outv.at(inst)[q] = (TO)s;
}

template <int DIM, class T>
__global__ void __launch_bounds__(256)
    k_coarse_scale(Vec<T> xv, Grid g, Batch bt, int per) {
  const int inst = blockIdx.x / per;
  if (bt.act && !bt.act[inst]) return;
  const unsigned q = (unsigned)(blockIdx.x - inst * per) * blockDim.x + threadIdx.x;
  if (q >= (unsigned)g.nodes) return;
  const int nn = g.nn, N = g.N;
  const double alpha = bt.coef[inst].alpha;
  int k0, k1, k2;
  node_ijk<DIM>(q, g, k0, k1, k2);
  auto mu = [&](int t) { return (g.h / 3.0) * (2.0 + cospi((double)t / (double)N)); };
  auto kap = [&](int t) { return (2.0 / g.h) * (1.0 - cospi((double)t / (double)N)); };
  auto gam = [&](int t) { return (t == 0 || t == N) ? (double)N : 0.5 * N; };
  double lam, gg;
  if (DIM == 3) {
    const double m0 = mu(k0), m1 = mu(k1), m2 = mu(k2);
    const double pm = m0 * m1 * m2;
    const double sk = kap(k0) * m1 * m2 + m0 * kap(k1) * m2 + m0 * m1 * kap(k2);
    lam = pm + alpha * sk;
    gg = gam(k0) * gam(k1) * gam(k2);
  } else {
    const double m0 = mu(k0), m1 = mu(k1);
    lam = m0 * m1 + alpha * (kap(k0) * m1 + m0 * kap(k1));
    gg = gam(k0) * gam(k1);
  }
  T* x = xv.at(inst);
  x[q] = (T)(ld(x + q) / (lam * gg));
}

}  // namespace

template <class T>
hipError_t launch_restrict(const Grid& fine, const Grid& coarse, const Batch& B, Vec<const T> r,
                           Vec<T> bc, hipStream_t st) {
  if (fine.N != 2 * coarse.N) return hipErrorInvalidValue;
  if (fine.dim == 3 && coarse.nn >= 100) {
    // streamed along z; chunks of coarse planes so that the launch holds
    // about 1500 or more blocks
    const int tx = (coarse.nn + kRsTI - 1) / kRsTI;
    const int ti = (coarse.nn + tx - 1) / tx;
    const int ty = (coarse.nn + kRsTJ - 1) / kRsTJ;
    const int64_t tiles = (int64_t)tx * ty * B.count;
    int nzc = (int)std::min<int64_t>(coarse.nn, std::max<int64_t>(1, (1536 + tiles - 1) / tiles));
    const int kc = (coarse.nn + nzc - 1) / nzc;
    nzc = (coarse.nn + kc - 1) / kc;
    const int64_t nblk = tiles * nzc;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_restrict_zs<T>), dim3((unsigned)nblk), dim3(256), 0, st, r, bc, fine,
                       coarse, B, tx, ty, ti, kc, nzc);
    return hipGetLastError();
  }
  const int per = (int)((coarse.nodes + 255) / 256);
  dim3 grid((unsigned)((int64_t)per * B.count)), block(256);
  if (fine.dim == 2)
    hipLaunchKernelGGL((k_restrict<2, T>), grid, block, 0, st, r, bc, fine, coarse, B, per);
  else
    hipLaunchKernelGGL((k_restrict<3, T>), grid, block, 0, st, r, bc, fine, coarse, B, per);
  return hipGetLastError();
}

template <class T>
hipError_t launch_prolong_add(const Grid& fine, const Grid& coarse, const Batch& B,
                              Vec<const T> ec, Vec<T> x, hipStream_t st) {
  const int nseg = (coarse.nn + kProlongW - 1) / kProlongW;
  const int64_t nblk = (int64_t)nseg * coarse.nn * (fine.dim == 3 ? coarse.nn : 1) * B.count;
  if (fine.N != 2 * coarse.N || nblk > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)nblk), block(256);
  if (fine.dim == 2)
    hipLaunchKernelGGL((k_prolong_add<2, T>), grid, block, 0, st, ec, x, fine, coarse, B, nseg);
  else
    hipLaunchKernelGGL((k_prolong_add<3, T>), grid, block, 0, st, ec, x, fine, coarse, B, nseg);
  return hipGetLastError();
}

template <class T>
hipError_t launch_coarse_solve(const Grid& g, const Batch& B, Vec<const T> b, Vec<T> x,
                               Vec<T> s1, Vec<T> s2, hipStream_t st) {
  if (g.nn > kCoarseLine) return hipErrorInvalidValue;
  if (g.nodes <= kCoarseMax) {
    if (g.dim == 2)
      hipLaunchKernelGGL((k_coarse<2, T>), dim3(B.count), dim3(1024), 0, st, b, x, g, B);
    else
      hipLaunchKernelGGL((k_coarse<3, T>), dim3(B.count), dim3(1024), 0, st, b, x, g, B);
    return hipGetLastError();
  }
  if (s1.null() || s2.null()) return hipErrorInvalidValue;
  const int per = (int)((g.nodes + 255) / 256);
  const dim3 grid((unsigned)((int64_t)per * B.count)), block(256);
  // forward: b -> s1 -> s2 (-> s1 in 3D), scale, backward to x
  Vec<const T> src = b;
  Vec<T> bufs[2] = {s1, s2};
  int w = 0;
  for (int ax = 0; ax < g.dim; ax++) {
    hipLaunchKernelGGL((k_coarse_axis<T, T>), grid, block, 0, st, src, bufs[w], g, B, ax, per);
    src = Vec<const T>{bufs[w].p, bufs[w].s};
    w ^= 1;
  }
  Vec<T> cur{const_cast<T*>(src.p), src.s};
  if (g.dim == 2)
    hipLaunchKernelGGL((k_coarse_scale<2, T>), grid, block, 0, st, cur, g, B, per);
  else
    hipLaunchKernelGGL((k_coarse_scale<3, T>), grid, block, 0, st, cur, g, B, per);
  for (int ax = 0; ax < g.dim; ax++) {
    Vec<T> dst = (ax == g.dim - 1) ? x : bufs[w];
    hipLaunchKernelGGL((k_coarse_axis<T, T>), grid, block, 0, st, src, dst, g, B, ax, per);
    src = Vec<const T>{dst.p, dst.s};
    w ^= 1;
  }
  return hipGetLastError();
}

#define OKD_MG(T)                                                                              \
  template hipError_t launch_restrict<T>(const Grid&, const Grid&, const Batch&, Vec<const T>,  \
                                         Vec<T>, hipStream_t);                                  \
  template hipError_t launch_prolong_add<T>(const Grid&, const Grid&, const Batch&,             \
                                            Vec<const T>, Vec<T>, hipStream_t);                 \
  template hipError_t launch_coarse_solve<T>(const Grid&, const Batch&, Vec<const T>, Vec<T>,   \
                                             Vec<T>, Vec<T>, hipStream_t);
OKD_MG(double)
OKD_MG(float)
#undef OKD_MG

}  // namespace okd
