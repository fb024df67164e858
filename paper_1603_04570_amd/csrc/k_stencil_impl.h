// Matrix-free Q1 node stencils of M and K on uniform grids, with the fused
// epilogues used by Chebyshev-Jacobi iterations, multigrid residuals and
// mass actions.
//
// The Q1 mass and stiffness matrices of (0,1)^d with Neumann ends are
// Kronecker sums/products of the 1D matrices
//   M1 = (h/6) tridiag(1, 4, 1)  (diagonal 2 at the two ends),
//   K1 = (1/h) tridiag(-1, 2, -1) (diagonal 1 at the two ends),
// M = M1 x M1 (x M1),  K = K1 x M1 (x M1) + M1 x K1 (x M1) (+ M1 x M1 x K1).
// A block owns a contiguous chunk of nodes of an x-y plane and streams along
// z: each plane chunk (with a one-row halo on each side) is staged in LDS, the
// in-plane partial products P_M = (M1 x M1) s and P_K = (K1 x M1 + M1 x K1) s
// are formed from LDS and kept in registers for three consecutive planes, and
// the z-direction 1D stencil combines them.  Every node is read once from HBM
// per plane pass; the halo rows come from L2 because neighbouring chunks run
// on the same XCD (see xcd_remap).
// This file is compiled twice (k_stencil_f64.hip, k_stencil_f32.hip) with
// OKD_STENCIL_PART 0 (host tables and FP64 kernels) and 1 (FP32 and mixed
// kernels), so that the two halves build in parallel.
#ifndef OKD_STENCIL_PART
#error "define OKD_STENCIL_PART (0 or 1) before including k_stencil_impl.h"
#endif
#include "ok_internal.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

// Floating-point contraction is off in this file and every fused
// multiply-add is written out (fma): the instantiations for every launch
// shape and the fused two-iteration kernel then evaluate the same
// expressions to the same bits, whatever the compiler's scheduling.
#pragma clang fp contract(off)

namespace okd {

#if OKD_STENCIL_PART == 0
Grid make_grid(int dim, int N) {
  Grid g;
  g.dim = dim;
  g.N = N;
  g.nn = N + 1;
  g.plane = (int64_t)g.nn * g.nn;
  g.nodes = (dim == 3) ? g.plane * g.nn : g.plane;
  g.h = 1.0 / N;
  g.rnn = 1.0 / g.nn;
  return g;
}

namespace {
std::mutex g_tune_mu;
// (dim, nn, nf, word) -> (items, nzc, threads)
std::map<std::tuple<int, int, int, int>, std::tuple<int, int, int>> g_tune;
}  // namespace

void stencil_tune_set(int dim, int nn, int nf, int word, int items, int nzc, int threads) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (items == 0)
    g_tune.erase(std::make_tuple(dim, nn, nf, word));
  else
    g_tune[std::make_tuple(dim, nn, nf, word)] = std::make_tuple(items, nzc, threads);
}

void stencil_tune_get(int dim, int nn, int nf, int word, int* items, int* nzc, int* threads) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(std::make_tuple(dim, nn, nf, word));
  const bool set = it != g_tune.end();
  *items = set ? std::get<0>(it->second) : 0;
  *nzc = set ? std::get<1>(it->second) : 0;
  *threads = set ? std::get<2>(it->second) : 0;
}

static StencilShape shape_with(const Grid& g, int items, int nzc, int threads = kThreads) {
  StencilShape s;
  const int64_t plane = (g.dim == 3) ? g.plane : (int64_t)g.nn;
  s.items = items;
  s.threads = threads;
  s.chunk = threads * items;
  s.nchunks = (int)((plane + s.chunk - 1) / s.chunk);
  s.nzc = std::max(1, std::min(nzc, g.nn));
  s.zc = (g.nn + s.nzc - 1) / s.nzc;
  s.blocks = s.nchunks * s.nzc;
  return s;
}

int red_blocks(int64_t n) {
  int64_t b = (n + 4095) / 4096;
  if (b > kMaxRedBlocks) b = kMaxRedBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

bool stencil_tuned(const Grid& g, int nf, int word) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(std::make_tuple(g.dim, g.nn, nf, word));
  return it != g_tune.end() && std::get<0>(it->second) > 0;
}

StencilShape stencil_shape(const Grid& g, int nf, int word) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(g.dim, g.nn, nf, word));
    if (it != g_tune.end() && std::get<0>(it->second) > 0)
      return shape_with(g, std::get<0>(it->second), std::get<1>(it->second),
                        std::get<2>(it->second));
  }
  StencilShape s;
  const int target = 1024;
  // nodes per streaming plane: an x-y plane in 3D, an x row in 2D
  const int64_t plane = (g.dim == 3) ? g.plane : (int64_t)g.nn;
  // Largest per-thread item count that still gives ~1024 blocks with at
  // least 8 planes per block; small grids fall back to 1 item, 4 planes.
  int items = (nf >= kFusedKey) ? 2 : ((nf > 1) ? 4 : 8);
  for (; items > 1; items /= 2) {
    int64_t nch = (plane + kThreads * items - 1) / (kThreads * items);
    if (nch * ((g.nn + 7) / 8) >= target) break;
  }
  s.items = items;
  s.threads = kThreads;
  s.chunk = kThreads * items;
  s.nchunks = (int)((plane + s.chunk - 1) / s.chunk);
  int64_t zc = ((int64_t)g.nn * s.nchunks) / target;
  zc = std::max<int64_t>(4, std::min<int64_t>(zc, 32));
  zc = std::min<int64_t>(zc, g.nn);
  s.nzc = (int)((g.nn + zc - 1) / zc);
  s.zc = (g.nn + s.nzc - 1) / s.nzc;
  s.blocks = s.nchunks * s.nzc;
  return s;
}
// Among the tilings of the N+1 columns into ntx tiles of equal width (the
// last one short), the one with the fewest blocks per plane whose two-node
// ring fits items + 1 slots per thread and whose LDS fits 64 KB; ties go to
// the widest tile (longest contiguous row segments).
bool cheb2_tile_geom(const Grid& g, int threads, int items, TileGeom& tg) {
  if (g.dim != 3 || (items != 1 && items != 2) || (threads != 256 && threads != 512)) return false;
  const int nn = g.nn, cap = threads * items, slots = threads * (items + 1);
  int64_t best = -1;
  for (int ntx = 1; ntx <= 32 && ntx <= nn; ntx++) {
    const int tx = (nn + ntx - 1) / ntx;
    int ty = std::min(nn, cap / tx);
    while (ty >= 1 && (tx + 4) * (ty + 4) > slots) ty--;
    if (ty < 1) continue;
    const size_t lds = (size_t)((tx + 4) * (ty + 4) + (tx + 2) * (ty + 2) + 4 * tx * ty) * 8;
    if (lds > 65536) continue;
    const int ntxr = (nn + tx - 1) / tx, nty = (nn + ty - 1) / ty;
    const int64_t blocks = (int64_t)ntxr * nty;
    if (best < 0 || blocks < best) {  // ntx ascends: ties keep the wider tile
      best = blocks;
      tg = TileGeom{tx, ty, ntxr, nty};
    }
  }
  return best > 0;
}
#endif  // OKD_STENCIL_PART == 0

// 1D stencil patterns of node i on N elements (constants h/6, 1/h applied
// later).  M pattern: [wl, 2(wl+wr), wr];  K pattern: [-wl, wl+wr, -wr].
// SCALED multiplies the weight of each neighbour j by 2 when j is an end
// node, i.e. applies the stencil to W^-1 s with W the trapezoid weights.
template <bool SCALED>
__device__ __forceinline__ void pattern(int i, int N, double& a0, double& a1, double& a2,
                                        double& b0, double& b1, double& b2) {
  double wl = (i > 0) ? 1.0 : 0.0, wr = (i < N) ? 1.0 : 0.0;
  double sl = 1.0, sc = 1.0, sr = 1.0;
  if (SCALED) {
    sl = (i - 1 == 0) ? 2.0 : 1.0;
    sc = (i == 0 || i == N) ? 2.0 : 1.0;
    sr = (i + 1 == N) ? 2.0 : 1.0;
  }
  a0 = wl * sl;
  a1 = 2.0 * (wl + wr) * sc;
  a2 = wr * sr;
  b0 = -wl * sl;
  b1 = (wl + wr) * sc;
  b2 = -wr * sr;
}

// Unscaled 1D rows of node i applied to its neighbours (l, c, r) read from a
// linearised plane: the neighbours of the end nodes (i = 0, N) lie in other
// rows and are dropped (hl, hr), the diagonal of M1 is 4 inside and 2 at the
// ends, of K1 2 and 1 (constants h/6, 1/h applied later).  Kept as masks and
// one end flag per node instead of six coefficients, which would otherwise
// occupy registers for the whole streaming loop.
__device__ __forceinline__ double m1_row(bool hl, bool hr, bool end, double l, double c,
                                         double r) {
  return fma(end ? 2.0 : 4.0, c, hl ? l : 0.0) + (hr ? r : 0.0);
}
__device__ __forceinline__ double k1_row(bool hl, bool hr, bool end, double l, double c,
                                         double r) {
  return fma(end ? 1.0 : 2.0, c, hl ? -l : 0.0) - (hr ? r : 0.0);
}

// a0 p0 + a1 p1 + a2 p2 (the 1D three-point stencil along one axis)
__device__ __forceinline__ double sum3(double a0, double a1, double a2, double p0, double p1,
                                       double p2) {
  return fma(a2, p2, fma(a1, p1, a0 * p0));
}

// Epilogues of operators without stiffness (the Chebyshev iteration on M)
// declare kMass = true; the streaming kernel then skips the K partials.
template <class E, class = void>
struct MassOnly {
  static constexpr bool value = false;
};
template <class E>
struct MassOnly<E, std::void_t<decltype(E::kMass)>> {
  static constexpr bool value = E::kMass;
};

__device__ __forceinline__ double to_d(double v) { return v; }
__device__ __forceinline__ double to_d(float v) { return (double)v; }

// ---------------------------------------------------------------------------
// The streaming kernel over NF stenciled fields of a class of instances.
// For each owned node the epilogue first issues its pointwise loads
// (Epi::load) and later receives (instance, index, #boundary coordinates,
// (M s_f)_i, (K s_f)_i, (s_f)_i for f < NF, loaded values, the instance's
// scalars).  Plane pz+1 is prefetched into registers (F loads per thread and
// field, all issued back to back) while plane pz is processed from LDS.
// ---------------------------------------------------------------------------
template <class TS, int NF>
struct Src {
  const TS* p[NF];
  int64_t s[NF];
  // optional scale of field 0 (per instance: sc0[inst * scs]): the values are
  // staged as sc0 * p[0], rounded to TS (unnormalised FGMRES basis vectors)
  const double* sc0 = nullptr;
  int64_t scs = 0;
};

template <int DIM, int NF, int NT, int P, int F, bool SCALED, class TS, class Epi>
__global__ void __launch_bounds__(NT)
    k_stencil(Src<TS, NF> src, Grid g, StencilShape sh, Batch B, Epi epi) {
  // staged planes keep the storage type: every value is read as a double
  extern __shared__ double lds_raw[];
  TS* const lds = reinterpret_cast<TS*>(lds_raw);
  using In = typename Epi::In;
  constexpr bool MASS = MassOnly<Epi>::value;
  const int tid = threadIdx.x;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = lb / sh.blocks;
  if (B.act && !B.act[inst]) return;
  const int b = lb - inst * sh.blocks;
  const int chunk = b % sh.nchunks;
  const int zch = b / sh.nchunks;
  const typename Epi::K kk = epi.prep(B.coef[inst], inst);
  const int nn = g.nn, N = g.N;
  // Streaming "plane": an x-y plane in 3D, an x row in 2D.
  const int64_t plane = (DIM == 3) ? g.plane : (int64_t)nn;
  const int halo = (DIM == 3) ? nn + 1 : 1;
  const int ldsn = sh.chunk + 2 * halo;
  const int64_t s0 = (int64_t)chunk * sh.chunk;
  const TS* sp[NF];
#pragma unroll
  for (int f = 0; f < NF; f++) sp[f] = src.p[f] + (int64_t)inst * src.s[f];

  int ii[P], jj[P];
  bool valid[P];
#pragma unroll
  for (int p = 0; p < P; p++) {
    int64_t q = s0 + tid + NT * p;
    valid[p] = q < plane;
    if (DIM == 3) {
      int j = (int)(q / nn);
      jj[p] = j;
      ii[p] = (int)(q - (int64_t)j * nn);
    } else {
      jj[p] = 0;
      ii[p] = (int)q;
    }
  }

  // Prefetch registers hold the raw storage words; every load is issued
  // unconditionally from a clamped (in-bounds) index, so no load sits in a
  // lane-divergent branch and the loads of the next plane stay in flight
  // until commit() converts them (out-of-range positions become 0 there).
  TS pre[NF][F];
  auto issue = [&](int64_t zoff) {
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
      for (int k = 0; k < F; k++) {
        const int64_t gq = s0 - halo + tid + NT * k;
        const int64_t gc = gq < 0 ? 0 : (gq >= plane ? plane - 1 : gq);
        pre[f][k] = sp[f][zoff + gc];
      }
  };
  const bool scaled0 = src.sc0 != nullptr;
  const double sc0 = scaled0 ? src.sc0[(int64_t)inst * src.scs] : 1.0;
  auto commit = [&]() {
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
      for (int k = 0; k < F; k++) {
        const int t = tid + NT * k;
        const int64_t gq = s0 - halo + t;
        TS v = pre[f][k];
        if (f == 0 && scaled0) v = (TS)(to_d(v) * sc0);
        if (t < ldsn) lds[f * ldsn + t] = (gq >= 0 && gq < plane) ? v : TS(0);
      }
  };
  // In-plane partial products: 3D P_M = (M1 x M1) s, P_K = (K1 x M1 + M1 x K1) s;
  // 2D P_M = M1 s, P_K = K1 s along x (constants applied later).
  auto plane_partials = [&](double (*pm)[P], double (*pk)[P], double (*cen)[P]) {
#pragma unroll
    for (int p = 0; p < P; p++) {
      const int L = tid + NT * p + halo;
      if constexpr (!SCALED) {
        const int ix = ii[p];
        const bool hl = ix > 0, hr = ix < N, ex = (ix == 0 || ix == N);
        if (DIM == 3) {
          const bool ey = (jj[p] == 0 || jj[p] == N);  // rows j-1, j+1 outside are zero in LDS
#pragma unroll
          for (int f = 0; f < NF; f++) {
            const TS* lf = lds + f * ldsn;
            double mr[3], kr[3];
#pragma unroll
            for (int r = 0; r < 3; r++) {
              const int base = L + (r - 1) * nn;
              const double va = lf[base - 1], vb = lf[base], vc = lf[base + 1];
              mr[r] = m1_row(hl, hr, ex, va, vb, vc);
              if (!MASS) kr[r] = k1_row(hl, hr, ex, va, vb, vc);
            }
            pm[f][p] = m1_row(true, true, ey, mr[0], mr[1], mr[2]);
            if (!MASS)
              pk[f][p] = m1_row(true, true, ey, kr[0], kr[1], kr[2]) +
                         k1_row(true, true, ey, mr[0], mr[1], mr[2]);
            cen[f][p] = lf[L];
          }
        } else {
#pragma unroll
          for (int f = 0; f < NF; f++) {
            const TS* lf = lds + f * ldsn;
            const double va = lf[L - 1], vb = lf[L], vc = lf[L + 1];
            pm[f][p] = m1_row(hl, hr, ex, va, vb, vc);
            if (!MASS) pk[f][p] = k1_row(hl, hr, ex, va, vb, vc);
            cen[f][p] = vb;
          }
        }
      } else {
        double ax0, ax1, ax2, bx0, bx1, bx2;
        pattern<SCALED>(ii[p], N, ax0, ax1, ax2, bx0, bx1, bx2);
        if (DIM == 3) {
          double ay0, ay1, ay2, by0, by1, by2;
          pattern<SCALED>(jj[p], N, ay0, ay1, ay2, by0, by1, by2);
#pragma unroll
          for (int f = 0; f < NF; f++) {
            const TS* lf = lds + f * ldsn;
            double mr[3], kr[3];
#pragma unroll
            for (int r = 0; r < 3; r++) {
              const int base = L + (r - 1) * nn;
              double va = lf[base - 1], vb = lf[base], vc = lf[base + 1];
              mr[r] = sum3(ax0, ax1, ax2, va, vb, vc);
              kr[r] = sum3(bx0, bx1, bx2, va, vb, vc);
            }
            pm[f][p] = sum3(ay0, ay1, ay2, mr[0], mr[1], mr[2]);
            pk[f][p] = MASS ? 0.0
                            : sum3(ay0, ay1, ay2, kr[0], kr[1], kr[2]) +
                                  sum3(by0, by1, by2, mr[0], mr[1], mr[2]);
            cen[f][p] = lf[L];
          }
        } else {
#pragma unroll
          for (int f = 0; f < NF; f++) {
            const TS* lf = lds + f * ldsn;
            double va = lf[L - 1], vb = lf[L], vc = lf[L + 1];
            pm[f][p] = sum3(ax0, ax1, ax2, va, vb, vc);
            pk[f][p] = MASS ? 0.0 : sum3(bx0, bx1, bx2, va, vb, vc);
            cen[f][p] = vb;
          }
        }
      }
    }
  };

  // Stream planes z0-1 .. z1 along the last axis, output planes z0 .. z1-1.
  const double h = g.h;
  const double cmass = (DIM == 3) ? h * h * h / 216.0 : h * h / 36.0;
  const double cstiff = (DIM == 3) ? h / 36.0 : 1.0 / 6.0;
  int z0, z1;
  zrange(sh, nn, zch, z0, z1);
  double pma[NF][P], pmb[NF][P], pka[NF][P], pkb[NF][P], cb[NF][P];
#pragma unroll
  for (int f = 0; f < NF; f++)
#pragma unroll
    for (int p = 0; p < P; p++) pma[f][p] = pmb[f][p] = pka[f][p] = pkb[f][p] = cb[f][p] = 0.0;
  // Loads are never skipped by a branch (a skipped load would make the
  // compiler wait for every outstanding load where the paths join): the
  // first and last trips reload a clamped plane that is already cached.
  const int zlast = min(z1, N);
  issue((int64_t)max(z0 - 1, 0) * plane);
  for (int pz = z0 - 1; pz <= z1; pz++) {
    const bool inside = (pz >= 0 && pz <= N);
    const int o = pz - 1;  // output plane
    __syncthreads();
    if (inside) commit();
    __syncthreads();
    In in[P];
    {
      const int oc = o < z0 ? z0 : o;
#pragma unroll
      for (int p = 0; p < P; p++) {  // clamped: loaded by every lane, used if valid
        const int64_t q = s0 + tid + NT * p;
        in[p] = epi.load(inst, (int64_t)oc * plane + (q < plane ? q : plane - 1));
      }
    }
    issue((int64_t)min(pz + 1, zlast) * plane);
    double pmn[NF][P], pkn[NF][P], cn[NF][P];
    if (inside) {
      plane_partials(pmn, pkn, cn);
    } else {
#pragma unroll
      for (int f = 0; f < NF; f++)
#pragma unroll
        for (int p = 0; p < P; p++) pmn[f][p] = pkn[f][p] = cn[f][p] = 0.0;
    }
    if (o >= z0) {
      double az0, az1, az2, bz0, bz1, bz2;
      pattern<SCALED>(o, N, az0, az1, az2, bz0, bz1, bz2);
      const int nbz = (o == 0 || o == N);
#pragma unroll
      for (int p = 0; p < P; p++) {
        if (!valid[p]) continue;
        double ms[NF], ks[NF], cc[NF];
#pragma unroll
        for (int f = 0; f < NF; f++) {
          ms[f] = cmass * sum3(az0, az1, az2, pma[f][p], pmb[f][p], pmn[f][p]);
          ks[f] = MASS ? 0.0
                       : cstiff * (sum3(az0, az1, az2, pka[f][p], pkb[f][p], pkn[f][p]) +
                                   sum3(bz0, bz1, bz2, pma[f][p], pmb[f][p], pmn[f][p]));
          cc[f] = cb[f][p];
        }
        int nb = (ii[p] == 0 || ii[p] == N) + nbz;
        if (DIM == 3) nb += (jj[p] == 0 || jj[p] == N);
        int64_t idx = (int64_t)o * plane + s0 + tid + NT * p;
        epi.store(inst, idx, nb, ms, ks, cc, in[p], kk);
      }
    }
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
      for (int p = 0; p < P; p++) {
        pma[f][p] = pmb[f][p];
        pmb[f][p] = pmn[f][p];
        pka[f][p] = pkb[f][p];
        pkb[f][p] = pkn[f][p];
        cb[f][p] = cn[f][p];
      }
  }
}

template <int D, int NF, int NT, int PP, bool SCALED, class TS, class Epi>
static void launch_h(int hx, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                     const Src<TS, NF>& s, const Grid& g, const StencilShape& sh, const Batch& B,
                     const Epi& e) {
  switch (hx) {
    case 3: hipLaunchKernelGGL((k_stencil<D, NF, NT, PP, PP + 3, SCALED, TS, Epi>), grid, block, lds, st, s, g, sh, B, e); break;
    case 5: hipLaunchKernelGGL((k_stencil<D, NF, NT, PP, PP + 5, SCALED, TS, Epi>), grid, block, lds, st, s, g, sh, B, e); break;
    case 9: hipLaunchKernelGGL((k_stencil<D, NF, NT, PP, PP + 9, SCALED, TS, Epi>), grid, block, lds, st, s, g, sh, B, e); break;
    default: hipLaunchKernelGGL((k_stencil<D, NF, NT, PP, PP + 17, SCALED, TS, Epi>), grid, block, lds, st, s, g, sh, B, e); break;
  }
}

#if OKD_STENCIL_PART == 0
// Launch shapes with instantiated kernels: 256 threads of 1, 2, 4 or 8 nodes
// (two stenciled fields: up to 4); in 3D, one stenciled field, also 512
// threads of 1, 2 or 4 nodes.
bool stencil_shape_ok(int dim, int nf, int items, int threads) {
  if (threads == kThreads) return items == 1 || items == 2 || items == 4 || (items == 8 && nf == 1);
  return threads == 512 && dim == 3 && nf == 1 && (items == 1 || items == 2 || items == 4);
}
#endif

template <bool SCALED, class TS, int NF, class Epi>
static hipError_t run_stencil_n(const Grid& g, const Batch& B, const Src<TS, NF>& s, const Epi& e,
                                hipStream_t st) {
  StencilShape sh = stencil_shape(g, NF, (int)sizeof(TS));
  if (!stencil_shape_ok(g.dim, NF, sh.items, sh.threads)) return hipErrorInvalidValue;
  const int NTh = sh.threads;
  const int ldsn = sh.chunk + 2 * (g.dim == 3 ? g.nn + 1 : 1);
  size_t lds = (size_t)NF * ldsn * sizeof(TS);
  // prefetch registers beyond the chunk: ceil(2*halo/threads) rounded up to 3, 5, 9, 17
  int extra = (ldsn - sh.chunk + NTh - 1) / NTh;
  int hx = extra <= 3 ? 3 : (extra <= 5 ? 5 : (extra <= 9 ? 9 : 17));
  if (extra > 17 || lds > 65536 || B.count < 1) return hipErrorInvalidValue;
  int64_t nblk = (int64_t)sh.blocks * B.count;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)nblk), block(NTh);
  if (g.dim == 2) {
    if (NF == 1) {
      switch (sh.items) {
        case 8: launch_h<2, NF, 256, 8, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
        case 4: launch_h<2, NF, 256, 4, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
        case 2: launch_h<2, NF, 256, 2, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
        default: launch_h<2, NF, 256, 1, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
      }
    } else {
      switch (sh.items) {
        case 4: launch_h<2, NF, 256, 4, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
        case 2: launch_h<2, NF, 256, 2, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
        default: launch_h<2, NF, 256, 1, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
      }
    }
  } else {
    if (hx > 5) return hipErrorInvalidValue;
    if (NF == 1) {
      if (NTh == 512) {
        switch (sh.items) {
          case 4: launch_h<3, NF, 512, 4, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
          case 2: launch_h<3, NF, 512, 2, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
          default: launch_h<3, NF, 512, 1, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
        }
      } else {
        switch (sh.items) {
          case 8: launch_h<3, NF, 256, 8, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
          case 4: launch_h<3, NF, 256, 4, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
          case 2: launch_h<3, NF, 256, 2, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
          default: launch_h<3, NF, 256, 1, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
        }
      }
    } else {
      switch (sh.items) {
        case 4: launch_h<3, NF, 256, 4, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
        case 2: launch_h<3, NF, 256, 2, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
        default: launch_h<3, NF, 256, 1, SCALED>(hx, grid, block, lds, st, s, g, sh, B, e); break;
      }
    }
  }
  return hipGetLastError();
}

template <bool SCALED, class TS, class Epi>
static hipError_t run_stencil(const Grid& g, const Batch& B, Vec<const TS> s, const Epi& e,
                              hipStream_t st, Vec<const double> sc = Vec<const double>{nullptr, 0}) {
  Src<TS, 1> src{{s.p}, {s.s}, sc.p, sc.s};
  return run_stencil_n<SCALED, TS, 1>(g, B, src, e, st);
}

// ---------------------------------------------------------------------------
// Epilogues.  prep() reads the instance's scalars once per block.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dinv_at(double dinv_int, int nb) {
  return dinv_int * (double)(1 << nb);
}

// Epilogue inputs in their storage types (converted where used, so the
// loads stay in flight until the stencil sums are ready).
struct In0 {};
template <class A>
struct In1 {
  A a;
};
template <class A, class B>
struct In2 {
  A a;
  B b;
};
struct OpK {
  double cm, ck, dinv, it, c1, c2, osc;
};
__device__ __forceinline__ const LevelCoef& level_of(const InstCoef& C, int lev) {
  return lev < 0 ? C.mass : C.lev[lev];
}
__device__ __forceinline__ OpK op_k(const InstCoef& C, int lev, int k, int osc) {
  const LevelCoef& L = level_of(C, lev);
  OpK o;
  o.cm = L.cm;
  o.ck = L.ck;
  o.dinv = L.dinv;
  o.it = L.it;
  o.c1 = (k >= 0) ? L.c1[k] : 0.0;
  o.c2 = (k >= 0) ? L.c2[k] : 0.0;
  o.osc = coef_field(C, osc);
  return o;
}

// A s = cm (M s) + ck (K s) of a level operator, and the Chebyshev direction
// c1 d + c2 D^-1 r (Saad, Alg. 12.1); shared by the one-iteration epilogues
// and the fused two-iteration kernel.
__device__ __forceinline__ double op_apply(const OpK& k, double ms, double ks) {
  return fma(k.cm, ms, k.ck * ks);
}
__device__ __forceinline__ double cheb_dir(const OpK& k, double d, double dv, double r) {
  return fma(k.c1, d, k.c2 * dv * r);
}

// out = add + a*(M s) + b*(K s)
template <class TA, class TO>
struct EpiAxpy {
  using In = In1<TA>;
  struct K {
    double a, b;
  };
  Vec<const TA> add;
  double ca, cb;
  int fa, fb;
  Vec<TO> out;
  __device__ K prep(const InstCoef& C, int) const {
    return K{ca * coef_field(C, fa), cb * coef_field(C, fb)};
  }
  __device__ In load(int inst, int64_t i) const {
    return In{add.null() ? (TA)0 : add.at(inst)[i]};
  }
  __device__ void store(int inst, int64_t i, int, const double* ms, const double* ks,
                        const double*, const In& in, const K& k) const {
    out.at(inst)[i] = (TO)fma(k.b, ks[0], fma(k.a, ms[0], to_d(in.a)));
  }
};

// out = add + a*(M s): EpiAxpy without the stiffness term (the streaming
// kernel then forms no K partials)
template <class TA, class TO>
struct EpiMassAxpy {
  static constexpr bool kMass = true;
  using In = In1<TA>;
  struct K {
    double a;
  };
  Vec<const TA> add;
  double ca;
  int fa;
  Vec<TO> out;
  __device__ K prep(const InstCoef& C, int) const { return K{ca * coef_field(C, fa)}; }
  __device__ In load(int inst, int64_t i) const {
    return In{add.null() ? (TA)0 : add.at(inst)[i]};
  }
  __device__ void store(int inst, int64_t i, int, const double* ms, const double*,
                        const double*, const In& in, const K& k) const {
    out.at(inst)[i] = (TO)fma(k.a, ms[0], to_d(in.a));
  }
};

// Two stenciled fields s0, s1 and up to two outputs:
//   out_o = add_o + c[o][0] M s0 + c[o][1] K s0 + c[o][2] M s1 + c[o][3] K s1
template <class TO>
struct EpiLin2 {
  using In = In2<double, double>;
  struct K {
    double c[2][4];
  };
  Vec<const double> add0, add1;
  double c[2][4];
  int f[2][4];
  Vec<TO> out0, out1;
  __device__ K prep(const InstCoef& C, int) const {
    K k;
    for (int o = 0; o < 2; o++)
      for (int q = 0; q < 4; q++) k.c[o][q] = c[o][q] * coef_field(C, f[o][q]);
    return k;
  }
  __device__ In load(int inst, int64_t i) const {
    return In{add0.null() ? 0.0 : add0.at(inst)[i], add1.null() ? 0.0 : add1.at(inst)[i]};
  }
  __device__ void store(int inst, int64_t i, int, const double* ms, const double* ks,
                        const double*, const In& in, const K& k) const {
    out0.at(inst)[i] = (TO)fma(k.c[0][3], ks[1],
                               fma(k.c[0][2], ms[1], fma(k.c[0][1], ks[0], fma(k.c[0][0], ms[0], in.a))));
    if (!out1.null())
      out1.at(inst)[i] = (TO)fma(k.c[1][3], ks[1],
                                 fma(k.c[1][2], ms[1], fma(k.c[1][1], ks[0], fma(k.c[1][0], ms[0], in.b))));
  }
};

// Coupling of the block preconditioner (eq. (prec), factor [I,0;-CA^-1,I]):
// with G = 3 int u^2 z1 phi, q = M_E(u) z1 + eps^2 K z1 = G - M z1 + eps^2 K z1;
// writes y = r2 + q and nq = -q (kept for the Jacobian applied to this z).
// r2s (may be null): r2 is stored unscaled and its value is r2s[0] * r2
// (the basis vectors of FGMRES carry their normalisation as a scale).
template <class TY>
struct EpiCouple {
  using In = In2<double, double>;
  struct K {
    double e2, s;
  };
  Vec<const double> g, r2, r2s;
  Vec<TY> y;
  Vec<double> nq;
  __device__ K prep(const InstCoef& C, int inst) const {
    return K{C.e2, r2s.null() ? 1.0 : r2s.at(inst)[0]};
  }
  __device__ In load(int inst, int64_t i) const { return In{g.at(inst)[i], r2.at(inst)[i]}; }
  __device__ void store(int inst, int64_t i, int, const double* ms, const double* ks,
                        const double*, const In& in, const K& k) const {
    const double q = fma(k.e2, ks[0], in.a - ms[0]);
    y.at(inst)[i] = (TY)(in.b * k.s + q);
    nq.at(inst)[i] = -q;
  }
};

// Residual of a Richardson iteration on the Schur complement (Sec. 4):
// stencil fields s0 = a = A~^-1 (dt th K z2) and s1 = z2, G = 3 int u^2 a phi;
//   S z2 = M z2 + (eps^2 K + M_E(u)) a = M z2 + G - M a + eps^2 K a,
//   res  = y - S z2.
template <class T>
struct EpiSchurRes {
  using In = In2<double, T>;
  struct K {
    double e2;
  };
  Vec<const double> g;
  Vec<const T> y;
  Vec<T> res;
  __device__ K prep(const InstCoef& C, int) const { return K{C.e2}; }
  __device__ In load(int inst, int64_t i) const { return In{g.at(inst)[i], y.at(inst)[i]}; }
  __device__ void store(int inst, int64_t i, int, const double* ms, const double* ks,
                        const double*, const In& in, const K& k) const {
    const double sz = ms[1] + fma(k.e2, ks[0], in.a - ms[0]);
    res.at(inst)[i] = (T)(to_d(in.b) - sz);
  }
};

// First Chebyshev iteration from x0 = 0; the stencil input is b and is
// applied with SCALED patterns, so (cm M + ck K) W^-1 b is available and
// A d0 = dinv * it * (cm M + ck K) W^-1 b.
template <class T, bool LAST, bool MASSOP = false>
struct EpiChebFirst {
  static constexpr bool kMass = MASSOP;
  using In = In0;
  using K = OpK;
  int lev, osc;
  Vec<T> x, r, d;
  __device__ K prep(const InstCoef& C, int) const { return op_k(C, lev, 0, osc); }
  __device__ In load(int, int64_t) const { return In{}; }
  __device__ void store(int inst, int64_t i, int nb, const double* ms, const double* ks,
                        const double* cen, const In&, const K& k) const {
    const double bi = cen[0];
    double dv = dinv_at(k.dinv, nb);
    double ad0 = k.dinv * k.it * op_apply(k, ms[0], ks[0]);
    double d0 = dv * bi * k.it;
    double r1 = bi - ad0;
    double d1 = cheb_dir(k, d0, dv, r1);
    if (LAST) {
      x.at(inst)[i] = (T)(k.osc * (d0 + d1));
    } else {
      x.at(inst)[i] = (T)d0;
      r.at(inst)[i] = (T)r1;
      d.at(inst)[i] = (T)d1;
    }
  }
};

// Iteration k: stencil input d_k.  x_{k+1} = x_k + d_k, r_{k+1} = r_k - A d_k,
// d_{k+1} = c1 d_k + c2 D^-1 r_{k+1}.  LAST also adds the final step:
// x_{k+2} = x_{k+1} + d_{k+1}, and writes only x.
template <class T, bool LAST, bool MASSOP = false>
struct EpiChebStep {
  static constexpr bool kMass = MASSOP;
  using In = In2<T, T>;
  using K = OpK;
  int lev, k, osc;
  Vec<T> x, r, dn;
  __device__ K prep(const InstCoef& C, int) const { return op_k(C, lev, k, osc); }
  __device__ In load(int inst, int64_t i) const {
    return In{x.at(inst)[i], r.at(inst)[i]};
  }
  __device__ void store(int inst, int64_t i, int nb, const double* ms, const double* ks,
                        const double* cen, const In& in, const K& kk) const {
    const double dk = cen[0];
    double dv = dinv_at(kk.dinv, nb);
    double xv = to_d(in.a) + dk;
    double rv = to_d(in.b) - op_apply(kk, ms[0], ks[0]);
    double d1 = cheb_dir(kk, dk, dv, rv);
    if (LAST) {
      x.at(inst)[i] = (T)(kk.osc * (xv + d1));
    } else {
      x.at(inst)[i] = (T)xv;
      r.at(inst)[i] = (T)rv;
      dn.at(inst)[i] = (T)d1;
    }
  }
};

// Start from a given x (stencil input x): r0 = b - A x, d0 = D^-1 r0 it.
template <class T>
struct EpiChebStart {
  using In = In1<T>;
  using K = OpK;
  int lev;
  Vec<const T> b;
  Vec<T> r, d;
  __device__ K prep(const InstCoef& C, int) const { return op_k(C, lev, -1, CF_ONE); }
  __device__ In load(int inst, int64_t i) const { return In{b.at(inst)[i]}; }
  __device__ void store(int inst, int64_t i, int nb, const double* ms, const double* ks,
                        const double*, const In& in, const K& k) const {
    double r0 = to_d(in.a) - op_apply(k, ms[0], ks[0]);
    r.at(inst)[i] = (T)r0;
    d.at(inst)[i] = (T)(dinv_at(k.dinv, nb) * r0 * k.it);
  }
};

// One Chebyshev iteration from x0 = 0: x = D^-1 b it (pointwise).
template <class T>
struct EpiChebOne {
  using In = In0;
  using K = OpK;
  int lev, osc;
  Vec<T> x;
  __device__ K prep(const InstCoef& C, int) const { return op_k(C, lev, -1, osc); }
  __device__ In load(int, int64_t) const { return In{}; }
  __device__ void store(int inst, int64_t i, int nb, const double*, const double*,
                        const double* cen, const In&, const K& k) const {
    x.at(inst)[i] = (T)(k.osc * dinv_at(k.dinv, nb) * cen[0] * k.it);
  }
};

// r = b - A x
template <class T>
struct EpiResid {
  using In = In1<T>;
  using K = OpK;
  int lev;
  Vec<const T> b;
  Vec<T> r;
  __device__ K prep(const InstCoef& C, int) const { return op_k(C, lev, -1, CF_ONE); }
  __device__ In load(int inst, int64_t i) const { return In{b.at(inst)[i]}; }
  __device__ void store(int inst, int64_t i, int, const double* ms, const double* ks,
                        const double*, const In& in, const K& k) const {
    r.at(inst)[i] = (T)(to_d(in.a) - op_apply(k, ms[0], ks[0]));
  }
};

// ---------------------------------------------------------------------------
// Two consecutive middle Chebyshev iterations k, k+1 on M (Saad, Alg. 12.1)
// in one streaming pass (temporal blocking along the streaming axis).
// Stage 1 computes r_{k+1} and d_{k+1} on the chunk plus a one-row halo for
// plane pz-1 as plane pz of d_k arrives; stage 2 applies M to d_{k+1} and
// finishes iteration k+1 for plane pz-2.  Every value the unfused kernels
// would store is rounded to T here at the same point, so the result is
// bitwise that of two launch_cheb_step calls.  LAST2: iteration k+1 is the
// final one (writes only x, scaled by osc).  r_k is read on the halo rows,
// which other blocks own, so r_{k+2} goes to a second buffer (rout != rin).
// LDS: d_k plane with a two-row halo (E2), d_{k+1} plane with a one-row halo
// (E1), and two buffers each of r_{k+1} and d_k on the chunk.  NT threads of
// P nodes each cover a chunk; a larger chunk shortens the relative halo.
// ---------------------------------------------------------------------------
template <int DIM, int NT, int P, int P1, int FA, class T, bool LAST2>
__global__ void __launch_bounds__(NT)
    k_cheb2(Grid g, StencilShape sh, Batch B, int kk, int osc, Vec<T> xv, Vec<const T> rinv,
            Vec<T> routv, Vec<const T> dinv_, Vec<T> doutv) {
  extern __shared__ double lds_raw[];  // holds words of T: every staged value is T-exact
  const int tid = threadIdx.x;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = lb / sh.blocks;
  if (B.act && !B.act[inst]) return;
  const int b = lb - inst * sh.blocks;
  const int chunk = b % sh.nchunks;
  const int zch = b / sh.nchunks;
  const InstCoef& IC = B.coef[inst];
  const OpK ka = op_k(IC, -1, kk, CF_ONE), kb = op_k(IC, -1, kk + 1, osc);
  const int nn = g.nn, N = g.N;
  const int64_t plane = (DIM == 3) ? g.plane : (int64_t)nn;
  const int H = (DIM == 3) ? nn + 1 : 1;  // one row (3D) or one node (2D) of halo
  const int CH = sh.chunk;
  const int E1 = CH + 2 * H, E2 = CH + 4 * H;
  T* LA = reinterpret_cast<T*>(lds_raw);  // d_k, positions s0-2H .. s0+CH+2H
  T* LB = LA + E2;      // d_{k+1}, positions s0-H .. s0+CH+H
  T* LR = LB + E1;      // r_{k+1} on the chunk, two buffers
  T* LD = LR + 2 * CH;  // d_k on the chunk, two buffers
  const int64_t s0 = (int64_t)chunk * CH;
  T* __restrict__ x = xv.at(inst);
  const T* __restrict__ r = rinv.at(inst);
  T* __restrict__ rout = LAST2 ? nullptr : routv.at(inst);
  const T* __restrict__ din = dinv_.at(inst);
  T* __restrict__ dout = doutv.at(inst);
  const int ystep = (DIM == 3) ? nn : 0;

  // stage-1 items: ext1 position e = tid + 256 q, in-plane index s0 - H + e
  int i1[P1], j1[P1];
  bool v1[P1];
#pragma unroll
  for (int q = 0; q < P1; q++) {
    const int e = tid + NT * q;
    const int64_t gq = s0 - H + e;
    v1[q] = (e < E1) && gq >= 0 && gq < plane;
    const int64_t gc = gq < 0 ? 0 : (gq >= plane ? plane - 1 : gq);
    j1[q] = (DIM == 3) ? (int)(gc / nn) : 0;
    i1[q] = (int)(gc - (int64_t)j1[q] * nn);
  }
  // stage-2 items: chunk position c = tid + 256 p
  int i2[P], j2[P];
  bool v2[P];
#pragma unroll
  for (int p = 0; p < P; p++) {
    const int64_t gq = s0 + tid + NT * p;
    v2[p] = gq < plane;
    const int64_t gc = gq < plane ? gq : plane - 1;
    j2[p] = (DIM == 3) ? (int)(gc / nn) : 0;
    i2[p] = (int)(gc - (int64_t)j2[p] * nn);
  }
  auto clampq = [&](int64_t gq) { return gq < 0 ? (int64_t)0 : (gq >= plane ? plane - 1 : gq); };

  // prefetch registers (raw words, clamped in-bounds loads)
  T pa[FA], pr[P1], px[P];
  auto issue_a = [&](int64_t zoff) {
#pragma unroll
    for (int k = 0; k < FA; k++) pa[k] = din[zoff + clampq(s0 - 2 * H + tid + NT * k)];
  };
  auto issue_rx = [&](int zr, int zx) {
#pragma unroll
    for (int q = 0; q < P1; q++)
      pr[q] = r[(int64_t)zr * plane + clampq(s0 - H + tid + NT * q)];
#pragma unroll
    for (int p = 0; p < P; p++) px[p] = x[(int64_t)zx * plane + clampq(s0 + tid + NT * p)];
  };
  // in-plane mass partial (M1 x M1) v at LDS position L of buffer v (the
  // arithmetic of the one-iteration kernel)
  auto mpart = [&](const T* v, int L, int i, int j) {
    const bool hl = i > 0, hr = i < N, ex = (i == 0 || i == N);
    if (DIM == 3) {
      const bool ey = (j == 0 || j == N);
      double m[3];
#pragma unroll
      for (int rr = 0; rr < 3; rr++) {
        const int bse = L + (rr - 1) * ystep;
        m[rr] = m1_row(hl, hr, ex, v[bse - 1], v[bse], v[bse + 1]);
      }
      return m1_row(true, true, ey, m[0], m[1], m[2]);
    }
    return m1_row(hl, hr, ex, v[L - 1], v[L], v[L + 1]);
  };

  const double h = g.h;
  const double cmass = (DIM == 3) ? h * h * h / 216.0 : h * h / 36.0;
  int z0, z1;
  zrange(sh, nn, zch, z0, z1);
  const int zlast = min(z1 + 1, N);
  double pa1[P1], pb1[P1], cb1[P1];  // stage 1: partials of planes pz-2, pz-1; d_k(pz-1)
  double pa2[P], pb2[P], cb2[P];     // stage 2: partials of d_{k+1} planes pz-3, pz-2; d_{k+1}(pz-2)
#pragma unroll
  for (int q = 0; q < P1; q++) pa1[q] = pb1[q] = cb1[q] = 0.0;
#pragma unroll
  for (int p = 0; p < P; p++) pa2[p] = pb2[p] = cb2[p] = 0.0;
  issue_a((int64_t)max(z0 - 2, 0) * plane);
  issue_rx(max(z0 - 1, 0), max(z0, 0));
  for (int pz = z0 - 2; pz <= z1 + 1; pz++) {
    const bool insideA = (pz >= 0 && pz <= N);
    const int q1 = pz - 1;  // stage-1 output plane
    const int o = pz - 2;   // stage-2 output plane
    const int buf = pz & 1;
    // no barrier before staging: every read of LA in the previous trip
    // precedes that trip's barrier before stage 2
    if (insideA) {
#pragma unroll
      for (int k = 0; k < FA; k++) {
        const int t = tid + NT * k;
        const int64_t gq = s0 - 2 * H + t;
        if (t < E2) LA[t] = (gq >= 0 && gq < plane) ? pa[k] : T(0);
      }
    }
    __syncthreads();
    // stage-1 pointwise inputs of plane q1 and stage-2 x of plane o arrived last trip
    T rq[P1], xq[P];
#pragma unroll
    for (int q = 0; q < P1; q++) rq[q] = pr[q];
#pragma unroll
    for (int p = 0; p < P; p++) xq[p] = px[p];
    issue_a((int64_t)max(min(pz + 1, zlast), 0) * plane);  // plane -1 is never read
    issue_rx(min(max(q1 + 1, 0), N), min(max(o + 1, 0), N));
    // stage 1: partials of d_k at plane pz over the extended chunk
    double pn1[P1], cn1[P1];
#pragma unroll
    for (int q = 0; q < P1; q++) {
      const int L = tid + NT * q + H;
      const bool use = insideA && (tid + NT * q < E1);
      pn1[q] = use ? mpart(LA, L, i1[q], j1[q]) : 0.0;
      cn1[q] = use ? LA[L] : 0.0;
    }
    if (q1 >= z0 - 1 && q1 <= z1) {
      const bool inq = (q1 >= 0 && q1 <= N);
      double az0 = 0, az1 = 0, az2 = 0, bz0, bz1, bz2;
      if (inq) pattern<false>(q1, N, az0, az1, az2, bz0, bz1, bz2);
      const int nbz = (q1 == 0 || q1 == N);
#pragma unroll
      for (int q = 0; q < P1; q++) {
        const int e = tid + NT * q;
        if (e >= E1) continue;
        double d1 = 0.0;
        if (inq && v1[q]) {
          const double ms = cmass * sum3(az0, az1, az2, pa1[q], pb1[q], pn1[q]);
          const double dk = cb1[q];
          int nb = (i1[q] == 0 || i1[q] == N) + nbz;
          if (DIM == 3) nb += (j1[q] == 0 || j1[q] == N);
          const double dv = dinv_at(ka.dinv, nb);
          const double ru = to_d(rq[q]) - op_apply(ka, ms, 0.0);
          const double rv1 = to_d((T)ru);
          d1 = to_d((T)cheb_dir(ka, dk, dv, ru));
          const int c = e - H;
          if (c >= 0 && c < CH) {
            LR[buf * CH + c] = (T)rv1;
            LD[buf * CH + c] = (T)dk;
          }
        }
        LB[e] = (T)d1;
      }
    }
#pragma unroll
    for (int q = 0; q < P1; q++) {
      pa1[q] = pb1[q];
      pb1[q] = pn1[q];
      cb1[q] = cn1[q];
    }
    __syncthreads();
    // stage 2: partials of d_{k+1} at plane q1 over the chunk; finish plane o
    if (q1 >= z0 - 1 && q1 <= z1) {
      double pn2[P], cn2[P];
#pragma unroll
      for (int p = 0; p < P; p++) {
        const int L = tid + NT * p + H;
        pn2[p] = mpart(LB, L, i2[p], j2[p]);
        cn2[p] = LB[L];
      }
      if (o >= z0 && o < z1) {
        double az0, az1, az2, bz0, bz1, bz2;
        pattern<false>(o, N, az0, az1, az2, bz0, bz1, bz2);
        const int nbz = (o == 0 || o == N);
        const int pb = buf ^ 1;
#pragma unroll
        for (int p = 0; p < P; p++) {
          if (!v2[p]) continue;
          const int c = tid + NT * p;
          const double ms = cmass * sum3(az0, az1, az2, pa2[p], pb2[p], pn2[p]);
          const double d1 = cb2[p];
          const double rv1 = LR[pb * CH + c];
          const double dk = LD[pb * CH + c];
          int nb = (i2[p] == 0 || i2[p] == N) + nbz;
          if (DIM == 3) nb += (j2[p] == 0 || j2[p] == N);
          const double dv = dinv_at(kb.dinv, nb);
          const double xv1 = to_d((T)(to_d(xq[p]) + dk));
          const double xv2 = xv1 + d1;
          const double rv2 = rv1 - op_apply(kb, ms, 0.0);
          const double d2 = cheb_dir(kb, d1, dv, rv2);
          const int64_t idx = (int64_t)o * plane + s0 + c;
          if (LAST2) {
            x[idx] = (T)(kb.osc * (xv2 + d2));
          } else {
            x[idx] = (T)xv2;
            rout[idx] = (T)rv2;
            dout[idx] = (T)d2;
          }
        }
      }
#pragma unroll
      for (int p = 0; p < P; p++) {
        pa2[p] = pb2[p];
        pb2[p] = pn2[p];
        cb2[p] = cn2[p];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same two Chebyshev iterations on M (3D) with a block owning a
// rectangular tile of TX x TY nodes of each x-y plane instead of a run of
// consecutive nodes.  A run of C nodes stages halos of whole rows (C + 2H
// nodes of d_{k+1}, C + 4H of d_k with H = N + 2), a tile the rings
// (TX+2)(TY+2) and (TX+4)(TY+4): for the same C far fewer when rows are long,
// so both halo stages fit P + 1 slots per thread.  Nodes outside the grid
// hold 0 in LDS, as the positions before and after a plane do in k_cheb2,
// and every node's arithmetic is that of k_cheb2: the results are the same
// bits.  LDS: d_k on the tile with a two-node ring (pitch TX+4), d_{k+1}
// with a one-node ring (pitch TX+2), and two buffers each of r_{k+1} and d_k
// on the tile.
// ---------------------------------------------------------------------------
template <int NT, int P, class T, bool LAST2>
__global__ void __launch_bounds__(NT)
    k_cheb2t(Grid g, StencilShape sh, TileGeom tg, Batch B, int kk, int osc, Vec<T> xv,
             Vec<const T> rinv, Vec<T> routv, Vec<const T> dinv_, Vec<T> doutv) {
  constexpr int P1 = P + 1;
  extern __shared__ double lds_raw[];  // staged as doubles: reads need no conversion
  const int tid = threadIdx.x;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = lb / sh.blocks;
  if (B.act && !B.act[inst]) return;
  const int b = lb - inst * sh.blocks;
  const int tile = b % sh.nchunks;
  const int zch = b / sh.nchunks;
  const InstCoef& IC = B.coef[inst];
  const OpK ka = op_k(IC, -1, kk, CF_ONE), kb = op_k(IC, -1, kk + 1, osc);
  const int nn = g.nn, N = g.N;
  const int64_t plane = g.plane;
  const int TX = tg.tx, TY = tg.ty;
  const int x0 = (tile % tg.ntx) * TX, y0 = (tile / tg.ntx) * TY;
  const int WA = TX + 4, WB = TX + 2;  // LDS row pitches
  const int EA = WA * (TY + 4), E1 = WB * (TY + 2), CH = TX * TY;
  double* LA = lds_raw;  // d_k: rows y0-2 .. y0+TY+1, columns x0-2 .. x0+TX+1
  double* LB = LA + EA;      // d_{k+1}: rows y0-1 .. y0+TY, columns x0-1 .. x0+TX
  double* LR = LB + E1;      // r_{k+1} on the tile, two buffers
  double* LD = LR + 2 * CH;  // d_k on the tile, two buffers
  T* __restrict__ x = xv.at(inst);
  const T* __restrict__ r = rinv.at(inst);
  T* __restrict__ rout = LAST2 ? nullptr : routv.at(inst);
  const T* __restrict__ din = dinv_.at(inst);
  T* __restrict__ dout = doutv.at(inst);
  auto cl = [&](int v) { return v < 0 ? 0 : (v > N ? N : v); };

  // d_k staging: LA position t = tid + NT k holds node (x0-2 + t % WA, y0-2 + t / WA)
  int oa[P1];       // in-plane offset of that node, clamped into the grid
  unsigned va = 0;  // bit k: the node lies in the grid (else LA holds 0)
#pragma unroll
  for (int k = 0; k < P1; k++) {
    const int t = tid + NT * k;
    const int ra = t / WA, ca = t - ra * WA;
    const int gy = y0 - 2 + ra, gx = x0 - 2 + ca;
    if (t < EA && gy >= 0 && gy <= N && gx >= 0 && gx <= N) va |= 1u << k;
    oa[k] = cl(gy) * nn + cl(gx);
  }
  // stage-1 items: LB position e = tid + NT q (node (x0-1 + e % WB, y0-1 + e / WB))
  int i1[P1], j1[P1], l1[P1];
  bool v1[P1];
#pragma unroll
  for (int q = 0; q < P1; q++) {
    const int e = tid + NT * q;
    const int rb = e / WB, cb = e - rb * WB;
    const int gy = y0 - 1 + rb, gx = x0 - 1 + cb;
    v1[q] = e < E1 && gy >= 0 && gy <= N && gx >= 0 && gx <= N;
    i1[q] = cl(gx);
    j1[q] = cl(gy);
    l1[q] = e < E1 ? (rb + 1) * WA + cb + 1 : WA + 1;  // the same node in LA
  }
  // stage-2 items: tile position c = tid + NT p (node (x0 + c % TX, y0 + c / TX))
  int i2[P], j2[P], l2[P];
  bool v2[P];
#pragma unroll
  for (int p = 0; p < P; p++) {
    const int c = tid + NT * p;
    const int a = c / TX, bb = c - a * TX;
    const int gy = y0 + a, gx = x0 + bb;
    v2[p] = c < CH && gy <= N && gx <= N;
    i2[p] = cl(gx);
    j2[p] = cl(gy);
    l2[p] = c < CH ? (a + 1) * WB + bb + 1 : WB + 1;  // the same node in LB
  }

  // prefetch registers (raw words, clamped in-bounds loads)
  T pa[P1], pr[P1], px[P];
  auto issue_a = [&](int64_t zoff) {
#pragma unroll
    for (int k = 0; k < P1; k++) pa[k] = din[zoff + oa[k]];
  };
  auto issue_rx = [&](int zr, int zx) {
#pragma unroll
    for (int q = 0; q < P1; q++) pr[q] = r[(int64_t)zr * plane + (int64_t)j1[q] * nn + i1[q]];
#pragma unroll
    for (int p = 0; p < P; p++) px[p] = x[(int64_t)zx * plane + (int64_t)j2[p] * nn + i2[p]];
  };
  // in-plane mass partial (M1 x M1) v at LDS position L of a buffer with row
  // pitch ys (the arithmetic of the one-iteration kernel).  The neighbours
  // that kernel masks out at i = 0 and i = N lie outside the grid here and
  // hold +0 in LDS, so adding them unmasked gives the same bits.
  auto mpart = [&](const double* v, int L, int ys, int i, int j) {
    const bool ex = (i == 0 || i == N);
    const bool ey = (j == 0 || j == N);
    double m[3];
#pragma unroll
    for (int rr = 0; rr < 3; rr++) {
      const int bse = L + (rr - 1) * ys;
      m[rr] = m1_row(true, true, ex, v[bse - 1], v[bse], v[bse + 1]);
    }
    return m1_row(true, true, ey, m[0], m[1], m[2]);
  };

  const double h = g.h;
  const double cmass = h * h * h / 216.0;
  int z0, z1;
  zrange(sh, nn, zch, z0, z1);
  const int zlast = min(z1 + 1, N);
  double pa1[P1], pb1[P1], cb1[P1];  // stage 1: partials of planes pz-2, pz-1; d_k(pz-1)
  double pa2[P], pb2[P], cb2[P];     // stage 2: partials of d_{k+1} planes pz-3, pz-2; d_{k+1}(pz-2)
#pragma unroll
  for (int q = 0; q < P1; q++) pa1[q] = pb1[q] = cb1[q] = 0.0;
#pragma unroll
  for (int p = 0; p < P; p++) pa2[p] = pb2[p] = cb2[p] = 0.0;
  issue_a((int64_t)max(z0 - 2, 0) * plane);
  issue_rx(max(z0 - 1, 0), max(z0, 0));
  for (int pz = z0 - 2; pz <= z1 + 1; pz++) {
    const bool insideA = (pz >= 0 && pz <= N);
    const int q1 = pz - 1;  // stage-1 output plane
    const int o = pz - 2;   // stage-2 output plane
    const int buf = pz & 1;
    // no barrier before staging: every read of LA in the previous trip
    // precedes that trip's barrier before stage 2
    if (insideA) {
#pragma unroll
      for (int k = 0; k < P1; k++) {
        const int t = tid + NT * k;
        if (t < EA) LA[t] = ((va >> k) & 1u) ? to_d(pa[k]) : 0.0;
      }
    }
    __syncthreads();
    // stage-1 pointwise inputs of plane q1 and stage-2 x of plane o arrived last trip
    T rq[P1], xq[P];
#pragma unroll
    for (int q = 0; q < P1; q++) rq[q] = pr[q];
#pragma unroll
    for (int p = 0; p < P; p++) xq[p] = px[p];
    issue_a((int64_t)max(min(pz + 1, zlast), 0) * plane);  // plane -1 is never read
    issue_rx(min(max(q1 + 1, 0), N), min(max(o + 1, 0), N));
    // stage 1: partials of d_k at plane pz over the tile and its one-node ring
    double pn1[P1], cn1[P1];
#pragma unroll
    for (int q = 0; q < P1; q++) {
      const bool use = insideA && (tid + NT * q < E1);
      pn1[q] = use ? mpart(LA, l1[q], WA, i1[q], j1[q]) : 0.0;
      cn1[q] = use ? LA[l1[q]] : 0.0;
    }
    if (q1 >= z0 - 1 && q1 <= z1) {
      const bool inq = (q1 >= 0 && q1 <= N);
      double az0 = 0, az1 = 0, az2 = 0, bz0, bz1, bz2;
      if (inq) pattern<false>(q1, N, az0, az1, az2, bz0, bz1, bz2);
      const int nbz = (q1 == 0 || q1 == N);
#pragma unroll
      for (int q = 0; q < P1; q++) {
        const int e = tid + NT * q;
        if (e >= E1) continue;
        double d1 = 0.0;
        if (inq && v1[q]) {
          const double ms = cmass * sum3(az0, az1, az2, pa1[q], pb1[q], pn1[q]);
          const double dk = cb1[q];
          const int nb = (i1[q] == 0 || i1[q] == N) + nbz + (j1[q] == 0 || j1[q] == N);
          const double dv = dinv_at(ka.dinv, nb);
          const double ru = to_d(rq[q]) - op_apply(ka, ms, 0.0);
          const double rv1 = to_d((T)ru);
          d1 = to_d((T)cheb_dir(ka, dk, dv, ru));
          const int ci = i1[q] - x0, cj = j1[q] - y0;
          if (ci >= 0 && ci < TX && cj >= 0 && cj < TY) {
            const int c = cj * TX + ci;
            LR[buf * CH + c] = rv1;
            LD[buf * CH + c] = dk;
          }
        }
        LB[e] = d1;
      }
    }
#pragma unroll
    for (int q = 0; q < P1; q++) {
      pa1[q] = pb1[q];
      pb1[q] = pn1[q];
      cb1[q] = cn1[q];
    }
    __syncthreads();
    // stage 2: partials of d_{k+1} at plane q1 over the tile; finish plane o
    if (q1 >= z0 - 1 && q1 <= z1) {
      double pn2[P], cn2[P];
#pragma unroll
      for (int p = 0; p < P; p++) {
        pn2[p] = mpart(LB, l2[p], WB, i2[p], j2[p]);
        cn2[p] = LB[l2[p]];
      }
      if (o >= z0 && o < z1) {
        double az0, az1, az2, bz0, bz1, bz2;
        pattern<false>(o, N, az0, az1, az2, bz0, bz1, bz2);
        const int nbz = (o == 0 || o == N);
        const int pb = buf ^ 1;
#pragma unroll
        for (int p = 0; p < P; p++) {
          if (!v2[p]) continue;
          const int c = tid + NT * p;
          const double ms = cmass * sum3(az0, az1, az2, pa2[p], pb2[p], pn2[p]);
          const double d1 = cb2[p];
          const double rv1 = LR[pb * CH + c];
          const double dk = LD[pb * CH + c];
          const int nb = (i2[p] == 0 || i2[p] == N) + nbz + (j2[p] == 0 || j2[p] == N);
          const double dv = dinv_at(kb.dinv, nb);
          const double xv1 = to_d((T)(to_d(xq[p]) + dk));
          const double xv2 = xv1 + d1;
          const double rv2 = rv1 - op_apply(kb, ms, 0.0);
          const double d2 = cheb_dir(kb, d1, dv, rv2);
          const int64_t idx = (int64_t)o * plane + (int64_t)j2[p] * nn + i2[p];
          if (LAST2) {
            x[idx] = (T)(kb.osc * (xv2 + d2));
          } else {
            x[idx] = (T)xv2;
            rout[idx] = (T)rv2;
            dout[idx] = (T)d2;
          }
        }
      }
#pragma unroll
      for (int p = 0; p < P; p++) {
        pa2[p] = pb2[p];
        pb2[p] = pn2[p];
        cb2[p] = cn2[p];
      }
    }
  }
}

// In-plane partial products of M and K at LDS position L of plane buffer v
// (node (i, j)): the arithmetic of the one-field streaming kernel, unscaled
// or with the W^-1-scaled patterns (SCALED).
template <int DIM, bool SCALED, class V, bool NOMASK = false>
__device__ __forceinline__ void mk_partials(const V* v, int L, int ystep, int i, int j, int N,
                                            double& pm, double& pk) {
  if constexpr (!SCALED) {
    // NOMASK: the neighbours dropped at i = 0 and i = N hold +0 (tiled layouts)
    const bool hl = NOMASK || i > 0, hr = NOMASK || i < N, ex = (i == 0 || i == N);
    if (DIM == 3) {
      const bool ey = (j == 0 || j == N);
      double mr[3], kr[3];
#pragma unroll
      for (int r = 0; r < 3; r++) {
        const int base = L + (r - 1) * ystep;
        const double va = v[base - 1], vb = v[base], vc = v[base + 1];
        mr[r] = m1_row(hl, hr, ex, va, vb, vc);
        kr[r] = k1_row(hl, hr, ex, va, vb, vc);
      }
      pm = m1_row(true, true, ey, mr[0], mr[1], mr[2]);
      pk = m1_row(true, true, ey, kr[0], kr[1], kr[2]) + k1_row(true, true, ey, mr[0], mr[1], mr[2]);
    } else {
      const double va = v[L - 1], vb = v[L], vc = v[L + 1];
      pm = m1_row(hl, hr, ex, va, vb, vc);
      pk = k1_row(hl, hr, ex, va, vb, vc);
    }
  } else {
    double ax0, ax1, ax2, bx0, bx1, bx2;
    pattern<true>(i, N, ax0, ax1, ax2, bx0, bx1, bx2);
    if (DIM == 3) {
      double ay0, ay1, ay2, by0, by1, by2;
      pattern<true>(j, N, ay0, ay1, ay2, by0, by1, by2);
      double mr[3], kr[3];
#pragma unroll
      for (int r = 0; r < 3; r++) {
        const int base = L + (r - 1) * ystep;
        const double va = v[base - 1], vb = v[base], vc = v[base + 1];
        mr[r] = sum3(ax0, ax1, ax2, va, vb, vc);
        kr[r] = sum3(bx0, bx1, bx2, va, vb, vc);
      }
      pm = sum3(ay0, ay1, ay2, mr[0], mr[1], mr[2]);
      pk = sum3(ay0, ay1, ay2, kr[0], kr[1], kr[2]) + sum3(by0, by1, by2, mr[0], mr[1], mr[2]);
    } else {
      const double va = v[L - 1], vb = v[L], vc = v[L + 1];
      pm = sum3(ax0, ax1, ax2, va, vb, vc);
      pk = sum3(bx0, bx1, bx2, va, vb, vc);
    }
  }
}

// ---------------------------------------------------------------------------
// The two Chebyshev iterations of a multigrid smoother (Saad, Alg. 12.1, on
// A = M + alpha K of level lev) fused with their neighbour in the V-cycle, in
// one streaming pass (temporal blocking along the streaming axis as in
// k_cheb2):
//   PRE  (pre-smoothing from x = 0, then the residual): stage 1 forms
//        x2 = osc (d0 + d1), d0 = D^-1 b it, on the chunk plus a one-row halo
//        from the W^-1-scaled stencil of b; stage 2 applies A to x2 and
//        writes x2 (out1) and r = b - A x2 (out2).
//   POST (post-smoothing from a given x): stage 1 forms r0 = b - A x and
//        d0 = D^-1 r0 it on the chunk plus halo; stage 2 applies A to d0 and
//        writes x + d0 + d1 to out1, a buffer other than x (x is read on halo
//        rows that other blocks own).
// Every value the one-iteration kernels store is rounded to T at the same
// point, so the outputs are bitwise those of launch_cheb_first + launch_resid
// (PRE) and launch_cheb_start + launch_cheb_step (POST).  av: the stenciled
// input (PRE b, POST x); bv: POST b.  LDS as in k_cheb2: the input plane with
// a two-row halo, the stage-1 field with a one-row halo, and two buffers each
// of the chunk values stage 2 needs (POST r0; the input's chunk values).
// ---------------------------------------------------------------------------
template <int DIM, int NT, int P, int P1, int FA, class T, bool PRE>
__global__ void __launch_bounds__(NT)
    k_mg2(Grid g, StencilShape sh, Batch B, int lev, Vec<const T> av, Vec<const T> bv,
          Vec<T> out1v, Vec<T> out2v) {
  extern __shared__ double lds_raw[];  // holds words of T: every staged value is T-exact
  const int tid = threadIdx.x;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = lb / sh.blocks;
  if (B.act && !B.act[inst]) return;
  const int b = lb - inst * sh.blocks;
  const int chunk = b % sh.nchunks;
  const int zch = b / sh.nchunks;
  const InstCoef& IC = B.coef[inst];
  const OpK k1 = PRE ? op_k(IC, lev, 0, CF_ONE) : op_k(IC, lev, -1, CF_ONE);
  const OpK k2 = PRE ? op_k(IC, lev, -1, CF_ONE) : op_k(IC, lev, 0, CF_ONE);
  const int nn = g.nn, N = g.N;
  const int64_t plane = (DIM == 3) ? g.plane : (int64_t)nn;
  const int H = (DIM == 3) ? nn + 1 : 1;
  const int CH = sh.chunk;
  const int E1 = CH + 2 * H, E2 = CH + 4 * H;
  T* LA = reinterpret_cast<T*>(lds_raw);
  T* LB = LA + E2;
  T* LR = LB + E1;
  T* LD = LR + 2 * CH;
  const int64_t s0 = (int64_t)chunk * CH;
  const T* __restrict__ a = av.at(inst);
  const T* __restrict__ bsrc = PRE ? nullptr : bv.at(inst);
  T* __restrict__ o1 = out1v.at(inst);
  T* __restrict__ o2 = PRE ? out2v.at(inst) : nullptr;
  const int ystep = (DIM == 3) ? nn : 0;

  int i1[P1], j1[P1];
  bool v1[P1];
#pragma unroll
  for (int q = 0; q < P1; q++) {
    const int e = tid + NT * q;
    const int64_t gq = s0 - H + e;
    v1[q] = (e < E1) && gq >= 0 && gq < plane;
    const int64_t gc = gq < 0 ? 0 : (gq >= plane ? plane - 1 : gq);
    j1[q] = (DIM == 3) ? (int)(gc / nn) : 0;
    i1[q] = (int)(gc - (int64_t)j1[q] * nn);
  }
  int i2[P], j2[P];
  bool v2[P];
#pragma unroll
  for (int p = 0; p < P; p++) {
    const int64_t gq = s0 + tid + NT * p;
    v2[p] = gq < plane;
    const int64_t gc = gq < plane ? gq : plane - 1;
    j2[p] = (DIM == 3) ? (int)(gc / nn) : 0;
    i2[p] = (int)(gc - (int64_t)j2[p] * nn);
  }
  auto clampq = [&](int64_t gq) { return gq < 0 ? (int64_t)0 : (gq >= plane ? plane - 1 : gq); };

  T pa[FA], pr[P1];
  auto issue_a = [&](int64_t zoff) {
#pragma unroll
    for (int k = 0; k < FA; k++) pa[k] = a[zoff + clampq(s0 - 2 * H + tid + NT * k)];
  };
  auto issue_b = [&](int zr) {
    if constexpr (!PRE) {
#pragma unroll
      for (int q = 0; q < P1; q++) pr[q] = bsrc[(int64_t)zr * plane + clampq(s0 - H + tid + NT * q)];
    }
  };

  const double h = g.h;
  const double cmass = (DIM == 3) ? h * h * h / 216.0 : h * h / 36.0;
  const double cstiff = (DIM == 3) ? h / 36.0 : 1.0 / 6.0;
  int z0, z1;
  zrange(sh, nn, zch, z0, z1);
  const int zlast = min(z1 + 1, N);
  double pa1[P1], pb1[P1], qa1[P1], qb1[P1], cb1[P1];
  double pa2[P], pb2[P], qa2[P], qb2[P], cb2[P];
#pragma unroll
  for (int q = 0; q < P1; q++) pa1[q] = pb1[q] = qa1[q] = qb1[q] = cb1[q] = 0.0;
#pragma unroll
  for (int p = 0; p < P; p++) pa2[p] = pb2[p] = qa2[p] = qb2[p] = cb2[p] = 0.0;
  issue_a((int64_t)max(z0 - 2, 0) * plane);
  issue_b(max(z0 - 1, 0));
  for (int pz = z0 - 2; pz <= z1 + 1; pz++) {
    const bool insideA = (pz >= 0 && pz <= N);
    const int q1 = pz - 1;  // stage-1 output plane
    const int o = pz - 2;   // stage-2 output plane
    const int buf = pz & 1;
    // no barrier before staging: every read of LA in the previous trip
    // precedes that trip's barrier before stage 2
    if (insideA) {
#pragma unroll
      for (int k = 0; k < FA; k++) {
        const int t = tid + NT * k;
        const int64_t gq = s0 - 2 * H + t;
        if (t < E2) LA[t] = (gq >= 0 && gq < plane) ? pa[k] : T(0);
      }
    }
    __syncthreads();
    T bq[P1];
#pragma unroll
    for (int q = 0; q < P1; q++) bq[q] = pr[q];
    issue_a((int64_t)max(min(pz + 1, zlast), 0) * plane);  // plane -1 is never read
    issue_b(min(max(q1 + 1, 0), N));
    double pn1[P1], qn1[P1], cn1[P1];
#pragma unroll
    for (int q = 0; q < P1; q++) {
      const int L = tid + NT * q + H;
      pn1[q] = qn1[q] = cn1[q] = 0.0;
      if (insideA && (tid + NT * q < E1)) {
        mk_partials<DIM, PRE>(LA, L, ystep, i1[q], j1[q], N, pn1[q], qn1[q]);
        cn1[q] = LA[L];
      }
    }
    if (q1 >= z0 - 1 && q1 <= z1) {
      const bool inq = (q1 >= 0 && q1 <= N);
      double az0 = 0, az1 = 0, az2 = 0, bz0 = 0, bz1 = 0, bz2 = 0;
      if (inq) pattern<PRE>(q1, N, az0, az1, az2, bz0, bz1, bz2);
      const int nbz = (q1 == 0 || q1 == N);
#pragma unroll
      for (int q = 0; q < P1; q++) {
        const int e = tid + NT * q;
        if (e >= E1) continue;
        double f1 = 0.0;
        if (inq && v1[q]) {
          const double ms = cmass * sum3(az0, az1, az2, pa1[q], pb1[q], pn1[q]);
          const double ks = cstiff * (sum3(az0, az1, az2, qa1[q], qb1[q], qn1[q]) +
                                      sum3(bz0, bz1, bz2, pa1[q], pb1[q], pn1[q]));
          int nb = (i1[q] == 0 || i1[q] == N) + nbz;
          if (DIM == 3) nb += (j1[q] == 0 || j1[q] == N);
          const double dv = dinv_at(k1.dinv, nb);
          const int c = e - H;
          if constexpr (PRE) {
            const double bi = cb1[q];
            const double ad0 = k1.dinv * k1.it * op_apply(k1, ms, ks);
            const double d0 = dv * bi * k1.it;
            const double r1 = bi - ad0;
            const double d1 = cheb_dir(k1, d0, dv, r1);
            f1 = to_d((T)(k1.osc * (d0 + d1)));
            if (c >= 0 && c < CH) LD[buf * CH + c] = (T)bi;
          } else {
            const double r0 = to_d(bq[q]) - op_apply(k1, ms, ks);
            f1 = to_d((T)(dv * r0 * k1.it));
            if (c >= 0 && c < CH) {
              LR[buf * CH + c] = (T)r0;
              LD[buf * CH + c] = (T)cb1[q];
            }
          }
        }
        LB[e] = (T)f1;
      }
    }
#pragma unroll
    for (int q = 0; q < P1; q++) {
      pa1[q] = pb1[q];
      pb1[q] = pn1[q];
      qa1[q] = qb1[q];
      qb1[q] = qn1[q];
      cb1[q] = cn1[q];
    }
    __syncthreads();
    if (q1 >= z0 - 1 && q1 <= z1) {
      double pn2[P], qn2[P], cn2[P];
#pragma unroll
      for (int p = 0; p < P; p++) {
        const int L = tid + NT * p + H;
        mk_partials<DIM, false>(LB, L, ystep, i2[p], j2[p], N, pn2[p], qn2[p]);
        cn2[p] = LB[L];
      }
      if (o >= z0 && o < z1) {
        double az0, az1, az2, bz0, bz1, bz2;
        pattern<false>(o, N, az0, az1, az2, bz0, bz1, bz2);
        const int nbz = (o == 0 || o == N);
        const int pb = buf ^ 1;
#pragma unroll
        for (int p = 0; p < P; p++) {
          if (!v2[p]) continue;
          const int c = tid + NT * p;
          const double ms = cmass * sum3(az0, az1, az2, pa2[p], pb2[p], pn2[p]);
          const double ks = cstiff * (sum3(az0, az1, az2, qa2[p], qb2[p], qn2[p]) +
                                      sum3(bz0, bz1, bz2, pa2[p], pb2[p], pn2[p]));
          const int64_t idx = (int64_t)o * plane + s0 + c;
          if constexpr (PRE) {
            o1[idx] = (T)cb2[p];
            o2[idx] = (T)(LD[pb * CH + c] - op_apply(k2, ms, ks));
          } else {
            int nb = (i2[p] == 0 || i2[p] == N) + nbz;
            if (DIM == 3) nb += (j2[p] == 0 || j2[p] == N);
            const double dk = cb2[p];
            const double dv = dinv_at(k2.dinv, nb);
            const double xv = LD[pb * CH + c] + dk;
            const double rv = LR[pb * CH + c] - op_apply(k2, ms, ks);
            const double d1 = cheb_dir(k2, dk, dv, rv);
            o1[idx] = (T)(k2.osc * (xv + d1));
          }
        }
      }
#pragma unroll
      for (int p = 0; p < P; p++) {
        pa2[p] = pb2[p];
        pb2[p] = pn2[p];
        qa2[p] = qb2[p];
        qb2[p] = qn2[p];
        cb2[p] = cn2[p];
      }
    }
  }
}

template <class T>
__global__ void __launch_bounds__(256)
    k_add_inplace(Batch B, Vec<T> x, Vec<const T> d, int64_t n, int per) {
  const int inst = blockIdx.x / per;
  if (B.act && !B.act[inst]) return;
  T* xi = x.at(inst);
  const T* di = d.at(inst);
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)per * blockDim.x)
    xi[i] = (T)(to_d(xi[i]) + to_d(di[i]));
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <class TS, class TA, class TO>
hipError_t launch_stencil_axpy(const Grid& g, const Batch& B, Vec<const TS> s, Vec<const TA> add,
                               double ca, int fa, double cb, int fb, Vec<TO> out, hipStream_t st) {
  if (cb == 0.0) {  // a mass action: no stiffness partials
    EpiMassAxpy<TA, TO> e{add, ca, fa, out};
    return run_stencil<false>(g, B, s, e, st);
  }
  EpiAxpy<TA, TO> e{add, ca, cb, fa, fb, out};
  return run_stencil<false>(g, B, s, e, st);
}

template <class TS>
hipError_t launch_stencil_lin2(const Grid& g, const Batch& B, Vec<const TS> s0, Vec<const TS> s1,
                               Vec<const double> add0, Vec<const double> add1,
                               const double (&c)[2][4], const int (&f)[2][4], Vec<double> out0,
                               Vec<double> out1, hipStream_t st) {
  EpiLin2<double> e;
  e.add0 = add0;
  e.add1 = add1;
  for (int o = 0; o < 2; o++)
    for (int q = 0; q < 4; q++) {
      e.c[o][q] = c[o][q];
      e.f[o][q] = f[o][q];
    }
  e.out0 = out0;
  e.out1 = out1;
  Src<TS, 2> src{{s0.p, s1.p}, {s0.s, s1.s}};
  return run_stencil_n<false, TS, 2>(g, B, src, e, st);
}

template <class T>
hipError_t launch_couple(const Grid& g, const Batch& B, Vec<const T> z1, Vec<const double> G,
                         Vec<const double> r2, Vec<const double> r2s, Vec<T> y, Vec<double> nq,
                         hipStream_t st) {
  EpiCouple<T> e{G, r2, r2s, y, nq};
  return run_stencil<false>(g, B, z1, e, st);
}

template <class T>
hipError_t launch_schur_res(const Grid& g, const Batch& B, Vec<const T> a, Vec<const T> z2,
                            Vec<const double> G, Vec<const T> y, Vec<T> res, hipStream_t st) {
  EpiSchurRes<T> e{G, y, res};
  Src<T, 2> src{{a.p, z2.p}, {a.s, z2.s}};
  return run_stencil_n<false, T, 2>(g, B, src, e, st);
}

template <class TB, class T>
hipError_t launch_cheb_one(const Grid& g, const Batch& B, int lev, int osc, Vec<const TB> b,
                           Vec<T> x, hipStream_t st, Vec<const double> bs) {
  EpiChebOne<T> e{lev, osc, x};
  return run_stencil<true>(g, B, b, e, st, bs);
}

template <class TB, class T>
hipError_t launch_cheb_first(const Grid& g, const Batch& B, int lev, int osc, bool last,
                             Vec<const TB> b, Vec<T> x, Vec<T> r, Vec<T> d, hipStream_t st,
                             Vec<const double> bs) {
  if (lev < 0) {  // M only: no stiffness partials
    if (last) {
      EpiChebFirst<T, true, true> e{lev, osc, x, r, d};
      return run_stencil<true>(g, B, b, e, st, bs);
    }
    EpiChebFirst<T, false, true> e{lev, osc, x, r, d};
    return run_stencil<true>(g, B, b, e, st, bs);
  }
  if (last) {
    EpiChebFirst<T, true> e{lev, osc, x, r, d};
    return run_stencil<true>(g, B, b, e, st, bs);
  }
  EpiChebFirst<T, false> e{lev, osc, x, r, d};
  return run_stencil<true>(g, B, b, e, st, bs);
}

template <class T>
hipError_t launch_cheb_step(const Grid& g, const Batch& B, int lev, int k, int osc, bool last,
                            Vec<T> x, Vec<T> r, Vec<const T> din, Vec<T> dout, hipStream_t st) {
  if (k < 0 || k >= kMaxCheb) return hipErrorInvalidValue;
  if (lev < 0) {  // M only: no stiffness partials
    if (last) {
      EpiChebStep<T, true, true> e{lev, k, osc, x, r, dout};
      return run_stencil<false>(g, B, din, e, st);
    }
    EpiChebStep<T, false, true> e{lev, k, osc, x, r, dout};
    return run_stencil<false>(g, B, din, e, st);
  }
  if (last) {
    EpiChebStep<T, true> e{lev, k, osc, x, r, dout};
    return run_stencil<false>(g, B, din, e, st);
  }
  EpiChebStep<T, false> e{lev, k, osc, x, r, dout};
  return run_stencil<false>(g, B, din, e, st);
}

namespace {

template <int DIM, int NT, int P, int EX1, int EXA, class T>
hipError_t launch_cheb2_p(const Grid& g, const Batch& B, const StencilShape& sh, int k, int osc,
                          bool last2, Vec<T> x, Vec<const T> r, Vec<T> rout, Vec<const T> din,
                          Vec<T> dout, hipStream_t st) {
  const int H = (DIM == 3) ? g.nn + 1 : 1;
  if (sh.chunk != NT * P) return hipErrorInvalidValue;
  const size_t lds = (size_t)(sh.chunk + 4 * H + sh.chunk + 2 * H + 4 * sh.chunk) * sizeof(T);
  if (lds > 65536) return hipErrorInvalidValue;
  const int64_t nblk = (int64_t)sh.blocks * B.count;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)nblk), block(NT);
  if (last2)
    hipLaunchKernelGGL((k_cheb2<DIM, NT, P, P + EX1, P + EXA, T, true>), grid, block, lds, st, g,
                       sh, B, k, osc, x, r, rout, din, dout);
  else
    hipLaunchKernelGGL((k_cheb2<DIM, NT, P, P + EX1, P + EXA, T, false>), grid, block, lds, st,
                       g, sh, B, k, osc, x, r, rout, din, dout);
  return hipGetLastError();
}

// Launch geometry of the fused kernel: threads of 1 or 2 nodes each.  ex1
// and exa are the extra per-thread slots of the one- and two-row halos.
struct Cheb2Geom {
  int nt, p, ex1, exa;
};
Cheb2Geom cheb2_geom(const Grid& g, const StencilShape& sh) {
  Cheb2Geom c;
  c.nt = sh.threads;
  c.p = sh.items;
  const int H = (g.dim == 3) ? g.nn + 1 : 1;
  c.ex1 = (2 * H + c.nt - 1) / c.nt;
  c.exa = (4 * H + c.nt - 1) / c.nt;
  return c;
}

template <int DIM, int NT, int P, class T>
hipError_t launch_cheb2_ex(const Grid& g, const Batch& B, const StencilShape& sh,
                           const Cheb2Geom& c, int k, int osc, bool last2, Vec<T> x,
                           Vec<const T> r, Vec<T> rout, Vec<const T> din, Vec<T> dout,
                           hipStream_t st) {
#define OK_CHEB2(E1, EA)                                                                       \
  if (c.ex1 == E1 && c.exa == EA)                                                              \
    return launch_cheb2_p<DIM, NT, P, E1, EA, T>(g, B, sh, k, osc, last2, x, r, rout, din, dout, \
                                                 st);
  if constexpr (DIM == 2) {
    OK_CHEB2(1, 1)
    return hipErrorInvalidValue;
  } else {
  OK_CHEB2(1, 1)
  OK_CHEB2(1, 2)
  OK_CHEB2(2, 3)
  OK_CHEB2(3, 5)
  OK_CHEB2(5, 9)
  return hipErrorInvalidValue;
  }
#undef OK_CHEB2
}
}  // namespace

#if OKD_STENCIL_PART == 0
namespace {
int g_fuse_cheb = 1;
int g_fuse_mg = 1;
int g_fuse_prolong = 1;
}  // namespace

void mg_fusion_set(int enable) { g_fuse_mg = enable ? 1 : 0; }

bool mg_fusion_enabled() { return g_fuse_mg != 0; }

void prolong_fusion_set(int enable) { g_fuse_prolong = enable ? 1 : 0; }

bool prolong_fusion_enabled() { return g_fuse_prolong != 0; }

bool mg2_shape_valid(const Grid& g, int key, int word) {
  const int H = (g.dim == 3) ? g.nn + 1 : 1;
  const StencilShape sh = stencil_shape(g, key, word);
  if (!cheb2_shape_ok(g.dim, sh.items, sh.threads)) return false;
  const Cheb2Geom c = cheb2_geom(g, sh);
  const bool combo = (g.dim == 2) ? (c.ex1 == 1 && c.exa == 1)
                                  : ((c.ex1 == 1 && c.exa <= 2) || (c.ex1 == 2 && c.exa == 3) ||
                                     (c.ex1 == 3 && c.exa == 5) || (c.ex1 == 5 && c.exa == 9));
  return combo && (size_t)(6 * sh.chunk + 6 * H) * (size_t)word <= 65536;
}

// The fused smoothers hold many more registers than the one-iteration
// kernels and win only on some grids: a level uses them only where the
// autotuner (or ok_set_launch_shape) has set the post-smoothing shape.
bool mg_fusion_on(const Grid& g, int word) {
  if (!g_fuse_mg) return false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(g.dim, g.nn, kMgPostKey, word));
    if (it == g_tune.end() || std::get<0>(it->second) <= 0) return false;
  }
  return mg2_shape_valid(g, kMgPreKey, word) && mg2_shape_valid(g, kMgPostKey, word);
}

void cheb_fusion_set(int enable) { g_fuse_cheb = enable ? 1 : 0; }

// Shapes of the fused kernel: 256 threads of 1 or 2 nodes, and in 3D 512
// threads of 1 or 2 nodes.
bool cheb2_shape_ok(int dim, int items, int threads) {
  if (items != 1 && items != 2) return false;
  return threads == 256 || (threads == 512 && dim == 3);
}

bool cheb_fusion_on(const Grid& g, int word) {
  if (!g_fuse_cheb) return false;
  {
    // the autotuner records items < 0 where fused pairs lost to single steps
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(g.dim, g.nn, kFusedKey, word));
    if (it != g_tune.end() && std::get<0>(it->second) < 0) return false;
  }
  StencilShape sh = stencil_shape(g, kFusedKey, word);
  if (!cheb2_shape_ok(g.dim, sh.items, sh.threads)) return false;
  const Cheb2Geom c = cheb2_geom(g, sh);
  const int H = (g.dim == 3) ? g.nn + 1 : 1;
  const bool combo = (g.dim == 2) ? (c.ex1 == 1 && c.exa == 1)
                                  : ((c.ex1 == 1 && c.exa <= 2) || (c.ex1 == 2 && c.exa == 3) ||
                                     (c.ex1 == 3 && c.exa == 5) || (c.ex1 == 5 && c.exa == 9));
  const int ch = c.nt * c.p;
  return combo && (size_t)(6 * ch + 6 * H) * (size_t)word <= 65536;
}
#endif  // OKD_STENCIL_PART == 0

#include "k_strip2.h"

#if OKD_STENCIL_PART == 0
int strip_threads(int cfg) { return (cfg >= 1 && cfg <= kStripCfgs) ? strip_cfg(cfg).nt : 0; }
int64_t strip_windows(const Grid& g, int cfg) {
  const StripCfg C = strip_cfg(cfg);
  return (int64_t)((g.nn + C.bx - 3) / (C.bx - 2)) * ((g.nn + C.by - 3) / (C.by - 2));
}
static_assert(kStripCfgs == kStripConfigs, "window configurations");
#endif

namespace {
// One launch of k_strip2 in window configuration CFG with the z-ranges of the
// table entry sh0.
template <int CFG, class T, int MODE, bool LAST2>
hipError_t launch_strip_cfg(const Grid& g, const Batch& B, const StencilShape& sh0, int lev,
                            int kk, int osc, Vec<const T> a, Vec<const T> p, Vec<T> x,
                            Vec<T> o2, Vec<T> o3, Vec<const T> ec, hipStream_t st) {
  constexpr StripCfg C = strip_cfg(CFG);
  if (g.dim != 3) return hipErrorInvalidValue;
  const int ntx = (g.nn + C.bx - 3) / (C.bx - 2), nty = (g.nn + C.by - 3) / (C.by - 2);
  StencilShape sh = sh0;
  sh.nchunks = ntx * nty;
  sh.blocks = sh.nchunks * sh.nzc;
  const int ce = (C.bx / 2 + 3) * (C.by / 2 + 3);  // coarse nodes under a window
  const size_t lds = ((size_t)2 * (C.bx + 2) * (C.by + 2) +
                      (MODE == kStripPostProlong ? 2 * (size_t)ce : 0)) * sizeof(double);
  const int64_t nblk = (int64_t)sh.blocks * B.count;
  if (nblk > 0x7fffffff || lds > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_strip2<C.bx, C.by, C.p, T, MODE, LAST2>), dim3((unsigned)nblk),
                     dim3(C.nt), lds, st, g, sh, ntx, B, lev, kk, osc, a, p, x, o2, o3, ec);
  return hipGetLastError();
}

template <class T, int MODE, bool LAST2>
hipError_t launch_strip(const Grid& g, const Batch& B, int key, int lev, int kk, int osc,
                        Vec<const T> a, Vec<const T> p, Vec<T> x, Vec<T> o2, Vec<T> o3,
                        hipStream_t st, Vec<const T> ec = Vec<const T>{nullptr, 0}) {
  const StencilShape sh = stencil_shape(g, key, (int)sizeof(T));
#define OKD_STRIP(CFG)                                                                      \
  case CFG:                                                                                 \
    return launch_strip_cfg<CFG, T, MODE, LAST2>(g, B, sh, lev, kk, osc, a, p, x, o2, o3, ec, st)
  switch (sh.items) {
    OKD_STRIP(1);
    OKD_STRIP(2);
    OKD_STRIP(3);
    OKD_STRIP(4);
    OKD_STRIP(5);
    default: return hipErrorInvalidValue;
  }
#undef OKD_STRIP
}
}  // namespace

namespace {
template <int NT, int P, class T>
hipError_t launch_cheb2t_p(const Grid& g, const Batch& B, const StencilShape& sh0, int k,
                           int osc, bool last2, Vec<T> x, Vec<const T> r, Vec<T> rout,
                           Vec<const T> din, Vec<T> dout, hipStream_t st) {
  TileGeom tg;
  if (!cheb2_tile_geom(g, NT, P, tg)) return hipErrorInvalidValue;
  StencilShape sh = sh0;
  sh.nchunks = tg.ntx * tg.nty;
  sh.blocks = sh.nchunks * sh.nzc;
  const size_t lds = (size_t)((tg.tx + 4) * (tg.ty + 4) + (tg.tx + 2) * (tg.ty + 2) +
                              4 * tg.tx * tg.ty) * sizeof(double);
  if (lds > 65536 || tg.tx * tg.ty > NT * P || (tg.tx + 4) * (tg.ty + 4) > NT * (P + 1))
    return hipErrorInvalidValue;
  const int64_t nblk = (int64_t)sh.blocks * B.count;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)nblk), block(NT);
  if (last2)
    hipLaunchKernelGGL((k_cheb2t<NT, P, T, true>), grid, block, lds, st, g, sh, tg, B, k, osc, x,
                       r, rout, din, dout);
  else
    hipLaunchKernelGGL((k_cheb2t<NT, P, T, false>), grid, block, lds, st, g, sh, tg, B, k, osc,
                       x, r, rout, din, dout);
  return hipGetLastError();
}
}  // namespace

template <class T>
hipError_t launch_cheb_step2(const Grid& g, const Batch& B, int k, int osc, bool last2, Vec<T> x,
                             Vec<const T> r, Vec<T> rout, Vec<const T> din, Vec<T> dout,
                             hipStream_t st) {
  if (k < 0 || k + 1 >= kMaxCheb || B.count < 1) return hipErrorInvalidValue;
  if (!last2 && (rout.p == r.p || rout.null())) return hipErrorInvalidValue;
  if (g.dim == 3 && stencil_tuned(g, kFusedStripKey, (int)sizeof(T))) {  // strips where selected
    const Vec<const T> din_c{din.p, din.s};
    if (last2)
      return launch_strip<T, kStripCheb, true>(g, B, kFusedStripKey, -1, k, osc, din_c, r, x,
                                               rout, dout, st);
    return launch_strip<T, kStripCheb, false>(g, B, kFusedStripKey, -1, k, osc, din_c, r, x, rout,
                                              dout, st);
  }
  if (g.dim == 3) {  // tiled kernel where the table selects it
    const StencilShape ts = stencil_shape(g, kFusedTileKey, (int)sizeof(T));
    if (stencil_tuned(g, kFusedTileKey, (int)sizeof(T)) && cheb2_shape_ok(3, ts.items, ts.threads)) {
      if (ts.threads == 512)
        return ts.items == 1
                   ? launch_cheb2t_p<512, 1, T>(g, B, ts, k, osc, last2, x, r, rout, din, dout, st)
                   : launch_cheb2t_p<512, 2, T>(g, B, ts, k, osc, last2, x, r, rout, din, dout, st);
      return ts.items == 1
                 ? launch_cheb2t_p<256, 1, T>(g, B, ts, k, osc, last2, x, r, rout, din, dout, st)
                 : launch_cheb2t_p<256, 2, T>(g, B, ts, k, osc, last2, x, r, rout, din, dout, st);
    }
  }
  const StencilShape sh = stencil_shape(g, kFusedKey, (int)sizeof(T));
  if (!cheb2_shape_ok(g.dim, sh.items, sh.threads)) return hipErrorInvalidValue;
  const Cheb2Geom c = cheb2_geom(g, sh);
  if (g.dim == 2) {
    if (c.p == 1)
      return launch_cheb2_ex<2, 256, 1, T>(g, B, sh, c, k, osc, last2, x, r, rout, din, dout, st);
    return launch_cheb2_ex<2, 256, 2, T>(g, B, sh, c, k, osc, last2, x, r, rout, din, dout, st);
  }
  if (c.nt == 512) {
    if (c.p == 1)
      return launch_cheb2_ex<3, 512, 1, T>(g, B, sh, c, k, osc, last2, x, r, rout, din, dout, st);
    return launch_cheb2_ex<3, 512, 2, T>(g, B, sh, c, k, osc, last2, x, r, rout, din, dout, st);
  }
  if (c.p == 1)
    return launch_cheb2_ex<3, 256, 1, T>(g, B, sh, c, k, osc, last2, x, r, rout, din, dout, st);
  return launch_cheb2_ex<3, 256, 2, T>(g, B, sh, c, k, osc, last2, x, r, rout, din, dout, st);
}

// The fused multigrid smoothers of k_mg2 (3D) on rectangular in-plane tiles,
// as k_cheb2t is k_cheb2 on tiles: rings of two and one nodes instead of
// whole halo rows, P + 1 slots per thread for both, LDS positions outside
// the grid holding +0 so the in-plane stencils need no boundary masks, and
// each node's arithmetic that of k_mg2 (same bits).
template <int NT, int P, class T, bool PRE>
__global__ void __launch_bounds__(NT)
    k_mg2t(Grid g, StencilShape sh, TileGeom tg, Batch B, int lev, Vec<const T> av,
           Vec<const T> bv, Vec<T> out1v, Vec<T> out2v) {
  constexpr int P1 = P + 1;
  extern __shared__ double lds_raw[];  // staged as doubles: reads need no conversion
  const int tid = threadIdx.x;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = lb / sh.blocks;
  if (B.act && !B.act[inst]) return;
  const int b = lb - inst * sh.blocks;
  const int tile = b % sh.nchunks;
  const int zch = b / sh.nchunks;
  const InstCoef& IC = B.coef[inst];
  const OpK k1 = PRE ? op_k(IC, lev, 0, CF_ONE) : op_k(IC, lev, -1, CF_ONE);
  const OpK k2 = PRE ? op_k(IC, lev, -1, CF_ONE) : op_k(IC, lev, 0, CF_ONE);
  const int nn = g.nn, N = g.N;
  const int64_t plane = g.plane;
  const int TX = tg.tx, TY = tg.ty;
  const int x0 = (tile % tg.ntx) * TX, y0 = (tile / tg.ntx) * TY;
  const int WA = TX + 4, WB = TX + 2;
  const int EA = WA * (TY + 4), E1 = WB * (TY + 2), CH = TX * TY;
  double* LA = lds_raw;      // input: rows y0-2 .. y0+TY+1, columns x0-2 .. x0+TX+1
  double* LB = LA + EA;      // stage-1 field: rows y0-1 .. y0+TY, columns x0-1 .. x0+TX
  double* LR = LB + E1;      // POST r0 on the tile, two buffers
  double* LD = LR + 2 * CH;  // the input on the tile, two buffers
  const T* __restrict__ a = av.at(inst);
  const T* __restrict__ bsrc = PRE ? nullptr : bv.at(inst);
  T* __restrict__ o1 = out1v.at(inst);
  T* __restrict__ o2 = PRE ? out2v.at(inst) : nullptr;
  auto cl = [&](int v) { return v < 0 ? 0 : (v > N ? N : v); };

  int oa[P1];
  unsigned va = 0;
#pragma unroll
  for (int k = 0; k < P1; k++) {
    const int t = tid + NT * k;
    const int ra = t / WA, ca = t - ra * WA;
    const int gy = y0 - 2 + ra, gx = x0 - 2 + ca;
    if (t < EA && gy >= 0 && gy <= N && gx >= 0 && gx <= N) va |= 1u << k;
    oa[k] = cl(gy) * nn + cl(gx);
  }
  int i1[P1], j1[P1], l1[P1];
  bool v1[P1];
#pragma unroll
  for (int q = 0; q < P1; q++) {
    const int e = tid + NT * q;
    const int rb = e / WB, cb = e - rb * WB;
    const int gy = y0 - 1 + rb, gx = x0 - 1 + cb;
    v1[q] = e < E1 && gy >= 0 && gy <= N && gx >= 0 && gx <= N;
    i1[q] = cl(gx);
    j1[q] = cl(gy);
    l1[q] = e < E1 ? (rb + 1) * WA + cb + 1 : WA + 1;
  }
  int i2[P], j2[P], l2[P];
  bool v2[P];
#pragma unroll
  for (int p = 0; p < P; p++) {
    const int c = tid + NT * p;
    const int aa = c / TX, bb = c - aa * TX;
    const int gy = y0 + aa, gx = x0 + bb;
    v2[p] = c < CH && gy <= N && gx <= N;
    i2[p] = cl(gx);
    j2[p] = cl(gy);
    l2[p] = c < CH ? (aa + 1) * WB + bb + 1 : WB + 1;
  }

  T pa[P1], pr[P1];
  auto issue_a = [&](int64_t zoff) {
#pragma unroll
    for (int k = 0; k < P1; k++) pa[k] = a[zoff + oa[k]];
  };
  auto issue_b = [&](int zr) {
    if constexpr (!PRE) {
#pragma unroll
      for (int q = 0; q < P1; q++)
        pr[q] = bsrc[(int64_t)zr * plane + (int64_t)j1[q] * nn + i1[q]];
    }
  };

  const double h = g.h;
  const double cmass = h * h * h / 216.0;
  const double cstiff = h / 36.0;
  int z0, z1;
  zrange(sh, nn, zch, z0, z1);
  const int zlast = min(z1 + 1, N);
  double pa1[P1], pb1[P1], qa1[P1], qb1[P1], cb1[P1];
  double pa2[P], pb2[P], qa2[P], qb2[P], cb2[P];
#pragma unroll
  for (int q = 0; q < P1; q++) pa1[q] = pb1[q] = qa1[q] = qb1[q] = cb1[q] = 0.0;
#pragma unroll
  for (int p = 0; p < P; p++) pa2[p] = pb2[p] = qa2[p] = qb2[p] = cb2[p] = 0.0;
  issue_a((int64_t)max(z0 - 2, 0) * plane);
  issue_b(max(z0 - 1, 0));
  for (int pz = z0 - 2; pz <= z1 + 1; pz++) {
    const bool insideA = (pz >= 0 && pz <= N);
    const int q1 = pz - 1;  // stage-1 output plane
    const int o = pz - 2;   // stage-2 output plane
    const int buf = pz & 1;
    // no barrier before staging: every read of LA in the previous trip
    // precedes that trip's barrier before stage 2
    if (insideA) {
#pragma unroll
      for (int k = 0; k < P1; k++) {
        const int t = tid + NT * k;
        if (t < EA) LA[t] = ((va >> k) & 1u) ? to_d(pa[k]) : 0.0;
      }
    }
    __syncthreads();
    T bq[P1];
#pragma unroll
    for (int q = 0; q < P1; q++) bq[q] = pr[q];
    issue_a((int64_t)max(min(pz + 1, zlast), 0) * plane);  // plane -1 is never read
    issue_b(min(max(q1 + 1, 0), N));
    double pn1[P1], qn1[P1], cn1[P1];
#pragma unroll
    for (int q = 0; q < P1; q++) {
      pn1[q] = qn1[q] = cn1[q] = 0.0;
      if (insideA && (tid + NT * q < E1)) {
        mk_partials<3, PRE, double, true>(LA, l1[q], WA, i1[q], j1[q], N, pn1[q], qn1[q]);
        cn1[q] = LA[l1[q]];
      }
    }
    if (q1 >= z0 - 1 && q1 <= z1) {
      const bool inq = (q1 >= 0 && q1 <= N);
      double az0 = 0, az1 = 0, az2 = 0, bz0 = 0, bz1 = 0, bz2 = 0;
      if (inq) pattern<PRE>(q1, N, az0, az1, az2, bz0, bz1, bz2);
      const int nbz = (q1 == 0 || q1 == N);
#pragma unroll
      for (int q = 0; q < P1; q++) {
        const int e = tid + NT * q;
        if (e >= E1) continue;
        double f1 = 0.0;
        if (inq && v1[q]) {
          const double ms = cmass * sum3(az0, az1, az2, pa1[q], pb1[q], pn1[q]);
          const double ks = cstiff * (sum3(az0, az1, az2, qa1[q], qb1[q], qn1[q]) +
                                      sum3(bz0, bz1, bz2, pa1[q], pb1[q], pn1[q]));
          const int nb = (i1[q] == 0 || i1[q] == N) + nbz + (j1[q] == 0 || j1[q] == N);
          const double dv = dinv_at(k1.dinv, nb);
          const int ci = i1[q] - x0, cj = j1[q] - y0;
          const bool own = ci >= 0 && ci < TX && cj >= 0 && cj < TY;
          const int c = cj * TX + ci;
          if constexpr (PRE) {
            const double bi = cb1[q];
            const double ad0 = k1.dinv * k1.it * op_apply(k1, ms, ks);
            const double d0 = dv * bi * k1.it;
            const double r1 = bi - ad0;
            const double d1 = cheb_dir(k1, d0, dv, r1);
            f1 = to_d((T)(k1.osc * (d0 + d1)));
            if (own) LD[buf * CH + c] = bi;
          } else {
            const double r0 = to_d(bq[q]) - op_apply(k1, ms, ks);
            f1 = to_d((T)(dv * r0 * k1.it));
            if (own) {
              LR[buf * CH + c] = to_d((T)r0);
              LD[buf * CH + c] = cb1[q];
            }
          }
        }
        LB[e] = f1;
      }
    }
#pragma unroll
    for (int q = 0; q < P1; q++) {
      pa1[q] = pb1[q];
      pb1[q] = pn1[q];
      qa1[q] = qb1[q];
      qb1[q] = qn1[q];
      cb1[q] = cn1[q];
    }
    __syncthreads();
    if (q1 >= z0 - 1 && q1 <= z1) {
      double pn2[P], qn2[P], cn2[P];
#pragma unroll
      for (int p = 0; p < P; p++) {
        mk_partials<3, false, double, true>(LB, l2[p], WB, i2[p], j2[p], N, pn2[p], qn2[p]);
        cn2[p] = LB[l2[p]];
      }
      if (o >= z0 && o < z1) {
        double az0, az1, az2, bz0, bz1, bz2;
        pattern<false>(o, N, az0, az1, az2, bz0, bz1, bz2);
        const int nbz = (o == 0 || o == N);
        const int pb = buf ^ 1;
#pragma unroll
        for (int p = 0; p < P; p++) {
          if (!v2[p]) continue;
          const int c = tid + NT * p;
          const double ms = cmass * sum3(az0, az1, az2, pa2[p], pb2[p], pn2[p]);
          const double ks = cstiff * (sum3(az0, az1, az2, qa2[p], qb2[p], qn2[p]) +
                                      sum3(bz0, bz1, bz2, pa2[p], pb2[p], pn2[p]));
          const int64_t idx = (int64_t)o * plane + (int64_t)j2[p] * nn + i2[p];
          if constexpr (PRE) {
            o1[idx] = (T)cb2[p];
            o2[idx] = (T)(LD[pb * CH + c] - op_apply(k2, ms, ks));
          } else {
            const int nb = (i2[p] == 0 || i2[p] == N) + nbz + (j2[p] == 0 || j2[p] == N);
            const double dk = cb2[p];
            const double dv = dinv_at(k2.dinv, nb);
            const double xv = LD[pb * CH + c] + dk;
            const double rv = LR[pb * CH + c] - op_apply(k2, ms, ks);
            const double d1 = cheb_dir(k2, dk, dv, rv);
            o1[idx] = (T)(k2.osc * (xv + d1));
          }
        }
      }
#pragma unroll
      for (int p = 0; p < P; p++) {
        pa2[p] = pb2[p];
        pb2[p] = pn2[p];
        qa2[p] = qb2[p];
        qb2[p] = qn2[p];
        cb2[p] = cn2[p];
      }
    }
  }
}

namespace {
template <int DIM, int NT, int P, int EX1, int EXA, class T, bool PRE>
hipError_t launch_mg2_p(const Grid& g, const Batch& B, const StencilShape& sh, int lev,
                        Vec<const T> a, Vec<const T> b, Vec<T> o1, Vec<T> o2, hipStream_t st) {
  const int H = (DIM == 3) ? g.nn + 1 : 1;
  if (sh.chunk != NT * P) return hipErrorInvalidValue;
  const size_t lds = (size_t)(sh.chunk + 4 * H + sh.chunk + 2 * H + 4 * sh.chunk) * sizeof(T);
  if (lds > 65536) return hipErrorInvalidValue;
  const int64_t nblk = (int64_t)sh.blocks * B.count;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_mg2<DIM, NT, P, P + EX1, P + EXA, T, PRE>), dim3((unsigned)nblk), dim3(NT),
                     lds, st, g, sh, B, lev, a, b, o1, o2);
  return hipGetLastError();
}

template <int DIM, int NT, int P, class T, bool PRE>
hipError_t launch_mg2_ex(const Grid& g, const Batch& B, const StencilShape& sh,
                         const Cheb2Geom& c, int lev, Vec<const T> a, Vec<const T> b, Vec<T> o1,
                         Vec<T> o2, hipStream_t st) {
#define OK_MG2(E1, EA)                                                                          \
  if (c.ex1 == E1 && c.exa == EA)                                                               \
    return launch_mg2_p<DIM, NT, P, E1, EA, T, PRE>(g, B, sh, lev, a, b, o1, o2, st);
  if constexpr (DIM == 2) {
    OK_MG2(1, 1)
    return hipErrorInvalidValue;
  } else {
  OK_MG2(1, 1)
  OK_MG2(1, 2)
  OK_MG2(2, 3)
  OK_MG2(3, 5)
  OK_MG2(5, 9)
  return hipErrorInvalidValue;
  }
#undef OK_MG2
}

template <int NT, int P, class T, bool PRE>
hipError_t launch_mg2t_p(const Grid& g, const Batch& B, const StencilShape& sh0, int lev,
                         Vec<const T> a, Vec<const T> b, Vec<T> o1, Vec<T> o2, hipStream_t st) {
  TileGeom tg;
  if (!cheb2_tile_geom(g, NT, P, tg)) return hipErrorInvalidValue;
  StencilShape sh = sh0;
  sh.nchunks = tg.ntx * tg.nty;
  sh.blocks = sh.nchunks * sh.nzc;
  const size_t lds = (size_t)((tg.tx + 4) * (tg.ty + 4) + (tg.tx + 2) * (tg.ty + 2) +
                              4 * tg.tx * tg.ty) * sizeof(double);
  if (lds > 65536 || tg.tx * tg.ty > NT * P || (tg.tx + 4) * (tg.ty + 4) > NT * (P + 1))
    return hipErrorInvalidValue;
  const int64_t nblk = (int64_t)sh.blocks * B.count;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_mg2t<NT, P, T, PRE>), dim3((unsigned)nblk), dim3(NT), lds, st, g, sh, tg,
                     B, lev, a, b, o1, o2);
  return hipGetLastError();
}

template <class T, bool PRE>
hipError_t launch_mg2(const Grid& g, const Batch& B, int lev, Vec<const T> a, Vec<const T> b,
                      Vec<T> o1, Vec<T> o2, hipStream_t st) {
  if (lev < 0 || lev >= kMaxLevels || B.count < 1) return hipErrorInvalidValue;
  const int skey = PRE ? kMgPreStripKey : kMgPostStripKey;
  if (g.dim == 3 && stencil_tuned(g, skey, (int)sizeof(T))) {  // strips where selected
    if (PRE)
      return launch_strip<T, kStripPre, false>(g, B, skey, lev, 0, CF_ONE, a,
                                               Vec<const T>{nullptr, 0}, o1, o2,
                                               Vec<T>{nullptr, 0}, st);
    return launch_strip<T, kStripPost, false>(g, B, skey, lev, 0, CF_ONE, a, b, o1,
                                              Vec<T>{nullptr, 0}, Vec<T>{nullptr, 0}, st);
  }
  if (g.dim == 3) {  // tiled kernels where the table selects them
    const int tkey = PRE ? kMgPreTileKey : kMgPostTileKey;
    const StencilShape ts = stencil_shape(g, tkey, (int)sizeof(T));
    if (stencil_tuned(g, tkey, (int)sizeof(T)) && cheb2_shape_ok(3, ts.items, ts.threads)) {
      if (ts.threads == 512)
        return ts.items == 1 ? launch_mg2t_p<512, 1, T, PRE>(g, B, ts, lev, a, b, o1, o2, st)
                             : launch_mg2t_p<512, 2, T, PRE>(g, B, ts, lev, a, b, o1, o2, st);
      return ts.items == 1 ? launch_mg2t_p<256, 1, T, PRE>(g, B, ts, lev, a, b, o1, o2, st)
                           : launch_mg2t_p<256, 2, T, PRE>(g, B, ts, lev, a, b, o1, o2, st);
    }
  }
  const StencilShape sh = stencil_shape(g, PRE ? kMgPreKey : kMgPostKey, (int)sizeof(T));
  if (!cheb2_shape_ok(g.dim, sh.items, sh.threads)) return hipErrorInvalidValue;
  const Cheb2Geom c = cheb2_geom(g, sh);
  if (g.dim == 2) {
    if (c.p == 1)
      return launch_mg2_ex<2, 256, 1, T, PRE>(g, B, sh, c, lev, a, b, o1, o2, st);
    return launch_mg2_ex<2, 256, 2, T, PRE>(g, B, sh, c, lev, a, b, o1, o2, st);
  }
  if (c.nt == 512) {
    if (c.p == 1)
      return launch_mg2_ex<3, 512, 1, T, PRE>(g, B, sh, c, lev, a, b, o1, o2, st);
    return launch_mg2_ex<3, 512, 2, T, PRE>(g, B, sh, c, lev, a, b, o1, o2, st);
  }
  if (c.p == 1)
    return launch_mg2_ex<3, 256, 1, T, PRE>(g, B, sh, c, lev, a, b, o1, o2, st);
  return launch_mg2_ex<3, 256, 2, T, PRE>(g, B, sh, c, lev, a, b, o1, o2, st);
}
}  // namespace

template <class T>
hipError_t launch_mg_pre2(const Grid& g, const Batch& B, int lev, Vec<const T> b, Vec<T> x2,
                          Vec<T> r, hipStream_t st) {
  if (x2.null() || r.null() || x2.p == r.p) return hipErrorInvalidValue;
  return launch_mg2<T, true>(g, B, lev, b, Vec<const T>{nullptr, 0}, x2, r, st);
}

template <class T>
hipError_t launch_mg_post2(const Grid& g, const Batch& B, int lev, Vec<const T> b,
                           Vec<const T> x, Vec<T> xout, hipStream_t st) {
  if (xout.null() || (const T*)xout.p == x.p) return hipErrorInvalidValue;
  return launch_mg2<T, false>(g, B, lev, x, b, xout, Vec<T>{nullptr, 0}, st);
}

// FP64 only: with single-precision vectors the folded kernel measured no
// faster than the separate prolongation pass at 256^3, so it is not built.
template <class T>
bool mg_post_prolong_ok(const Grid& g, const Grid& gc) {
  return sizeof(T) == 8 && g.dim == 3 && g.N == 2 * gc.N &&
         stencil_tuned(g, kMgPostStripKey, (int)sizeof(T));
}

template <class T>
hipError_t launch_mg_post2_prolong(const Grid& g, const Grid& gc, const Batch& B, int lev,
                                   Vec<const T> b, Vec<const T> x, Vec<const T> ec, Vec<T> xout,
                                   hipStream_t st) {
  if (lev < 0 || lev >= kMaxLevels || B.count < 1 || xout.null() || (const T*)xout.p == x.p ||
      ec.null() || !mg_post_prolong_ok<T>(g, gc))
    return hipErrorInvalidValue;
  if constexpr (sizeof(T) == 8)
    return launch_strip<T, kStripPostProlong, false>(g, B, kMgPostStripKey, lev, 0, CF_ONE, x,
                                                     b, xout, Vec<T>{nullptr, 0},
                                                     Vec<T>{nullptr, 0}, st, ec);
  return hipErrorInvalidValue;
}

template <class T>
hipError_t launch_cheb_start(const Grid& g, const Batch& B, int lev, Vec<const T> b,
                             Vec<const T> x, Vec<T> r, Vec<T> d, hipStream_t st) {
  EpiChebStart<T> e{lev, b, r, d};
  return run_stencil<false>(g, B, x, e, st);
}

template <class T>
hipError_t launch_add_inplace(const Batch& B, Vec<T> x, Vec<const T> d, int64_t n,
                              hipStream_t st) {
  int per = (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096);
  hipLaunchKernelGGL(k_add_inplace<T>, dim3((unsigned)(per * B.count)), dim3(256), 0, st, B, x, d,
                     n, per);
  return hipGetLastError();
}

template <class T>
hipError_t launch_resid(const Grid& g, const Batch& B, int lev, Vec<const T> b, Vec<const T> x,
                        Vec<T> r, hipStream_t st) {
  EpiResid<T> e{lev, b, r};
  return run_stencil<false>(g, B, x, e, st);
}

// Explicit instantiations: FP64 in part 0, FP32 and mixed in part 1.
#if OKD_STENCIL_PART == 0
template hipError_t launch_stencil_axpy<double, double, double>(const Grid&, const Batch&,
                                                                Vec<const double>,
                                                                Vec<const double>, double, int,
                                                                double, int, Vec<double>,
                                                                hipStream_t);
template hipError_t launch_stencil_lin2<double>(const Grid&, const Batch&, Vec<const double>,
                                                Vec<const double>, Vec<const double>,
                                                Vec<const double>, const double (&)[2][4],
                                                const int (&)[2][4], Vec<double>, Vec<double>,
                                                hipStream_t);
template hipError_t launch_schur_res<double>(const Grid&, const Batch&, Vec<const double>,
                                             Vec<const double>, Vec<const double>,
                                             Vec<const double>, Vec<double>, hipStream_t);
template hipError_t launch_couple<double>(const Grid&, const Batch&, Vec<const double>,
                                          Vec<const double>, Vec<const double>,
                                          Vec<const double>, Vec<double>, Vec<double>,
                                          hipStream_t);
#else
template hipError_t launch_stencil_axpy<float, float, float>(const Grid&, const Batch&,
                                                             Vec<const float>, Vec<const float>,
                                                             double, int, double, int,
                                                             Vec<float>, hipStream_t);
template hipError_t launch_stencil_axpy<float, double, float>(const Grid&, const Batch&,
                                                              Vec<const float>,
                                                              Vec<const double>, double, int,
                                                              double, int, Vec<float>,
                                                              hipStream_t);
template hipError_t launch_stencil_lin2<float>(const Grid&, const Batch&, Vec<const float>,
                                               Vec<const float>, Vec<const double>,
                                               Vec<const double>, const double (&)[2][4],
                                               const int (&)[2][4], Vec<double>, Vec<double>,
                                               hipStream_t);
template hipError_t launch_schur_res<float>(const Grid&, const Batch&, Vec<const float>,
                                            Vec<const float>, Vec<const double>, Vec<const float>,
                                            Vec<float>, hipStream_t);
template hipError_t launch_couple<float>(const Grid&, const Batch&, Vec<const float>,
                                         Vec<const double>, Vec<const double>,
                                         Vec<const double>, Vec<float>, Vec<double>,
                                         hipStream_t);
#endif
#define OKD_CHEB_TB(TB, T)                                                                    \
  template hipError_t launch_cheb_one<TB, T>(const Grid&, const Batch&, int, int,              \
                                             Vec<const TB>, Vec<T>, hipStream_t,               \
                                             Vec<const double>);                               \
  template hipError_t launch_cheb_first<TB, T>(const Grid&, const Batch&, int, int, bool,      \
                                               Vec<const TB>, Vec<T>, Vec<T>, Vec<T>,          \
                                               hipStream_t, Vec<const double>);
#define OKD_CHEB_T(T)                                                                         \
  template hipError_t launch_cheb_step<T>(const Grid&, const Batch&, int, int, int, bool,      \
                                          Vec<T>, Vec<T>, Vec<const T>, Vec<T>, hipStream_t);  \
  template hipError_t launch_cheb_step2<T>(const Grid&, const Batch&, int, int, bool, Vec<T>,  \
                                           Vec<const T>, Vec<T>, Vec<const T>, Vec<T>,         \
                                           hipStream_t);                                       \
  template hipError_t launch_cheb_start<T>(const Grid&, const Batch&, int, Vec<const T>,      \
                                           Vec<const T>, Vec<T>, Vec<T>, hipStream_t);         \
  template hipError_t launch_add_inplace<T>(const Batch&, Vec<T>, Vec<const T>, int64_t,       \
                                            hipStream_t);                                      \
  template hipError_t launch_resid<T>(const Grid&, const Batch&, int, Vec<const T>,            \
                                      Vec<const T>, Vec<T>, hipStream_t);                      \
  template hipError_t launch_mg_pre2<T>(const Grid&, const Batch&, int, Vec<const T>, Vec<T>,  \
                                        Vec<T>, hipStream_t);                                  \
  template hipError_t launch_mg_post2<T>(const Grid&, const Batch&, int, Vec<const T>,         \
                                         Vec<const T>, Vec<T>, hipStream_t);                   \
  template bool mg_post_prolong_ok<T>(const Grid&, const Grid&);                               \
  template hipError_t launch_mg_post2_prolong<T>(const Grid&, const Grid&, const Batch&, int,   \
                                                 Vec<const T>, Vec<const T>, Vec<const T>,     \
                                                 Vec<T>, hipStream_t);
#if OKD_STENCIL_PART == 0
OKD_CHEB_TB(double, double)
OKD_CHEB_T(double)
#else
OKD_CHEB_TB(float, float)
OKD_CHEB_TB(double, float)
OKD_CHEB_T(float)
#endif
#undef OKD_CHEB_TB
#undef OKD_CHEB_T

}  // namespace okd
