// Internal declarations shared by the HIP sources of libok.so.
//
// Every kernel works on a *class* of B independent instances that share the
// grid (d, N) and the precision: the launch grid is (blocks of one instance)
// x B, block b serves instance b / (blocks of one instance), every vector
// argument is a (base pointer, element stride between instances) pair, the
// per-instance constants live in a device table of InstCoef records, and an
// optional per-instance `act` flag makes the blocks of an inactive instance
// return at once.  A single solve is the class with B = 1.  The arithmetic
// of one instance does not depend on B, on the other instances or on the
// launch shape, so batched results equal solo results bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ok.h"

namespace okd {

constexpr int kMaxLevels = 16;
constexpr int kThreads = 256;   // node-stencil and vector kernels
constexpr int kMaxCheb = 32;    // Chebyshev iterations per application

// ---------------------------------------------------------------------------
// Geometry of one uniform Q1 grid level.
// ---------------------------------------------------------------------------
struct Grid {
  int dim;        // 2 or 3
  int N;          // elements per direction
  int nn;         // nodes per direction, N + 1
  int64_t plane;  // nodes per z-plane (nn*nn); the whole grid in 2D
  int64_t nodes;  // nn^dim
  double h;       // 1/N
  double rnn;     // 1/nn, for index decompositions without integer division
};
Grid make_grid(int dim, int N);

// A vector argument of a class launch: instance i starts at p + i*s.
template <class T>
struct Vec {
  T* p;
  int64_t s;
  __host__ __device__ T* at(int i) const { return p + (int64_t)i * s; }
  __host__ __device__ bool null() const { return p == nullptr; }
};
template <class T>
inline Vec<T> vec(T* p, int64_t s) {
  return Vec<T>{p, s};
}
template <class T>
inline Vec<const T> cvec(const T* p, int64_t s) {
  return Vec<const T>{p, s};
}

// Per-level operator A = cm M + ck K and its Chebyshev-Jacobi coefficients.
// diag(A) at a node = dint * 2^-(number of coordinates on the boundary),
// dinv = 1/dint.  Iteration k of Saad's Alg. 12.1 forms
// d_{k+1} = c1[k] d_k + c2[k] D^-1 r_{k+1};  it = 1/theta of the interval.
struct LevelCoef {
  double cm, ck, dinv, it;
  double c1[kMaxCheb], c2[kMaxCheb];
};

// Per-instance constants, one record per instance in device memory.
struct InstCoef {
  LevelCoef mass;             // Chebyshev on M on the finest grid
  LevelCoef lev[kMaxLevels];  // M_l + alpha K_l on each multigrid level
  double alpha;               // eps sqrt(c)
  double sA, inv_sA;          // 1 + dt theta sigma and its inverse
  double dth;                 // dt theta
  double c;                   // dt theta / (1 + dt theta sigma)
  double e2;                  // eps^2
  double dt, sigma, theta, m;
  double rtol, atol;
};

// Named per-instance scalars for stencil epilogue coefficients.
enum CoefField { CF_ONE = 0, CF_SA = 1, CF_DTH = 2, CF_E2 = 3, CF_INV_SA = 4, CF_C = 5 };
__host__ __device__ inline double coef_field(const InstCoef& c, int f) {
  switch (f) {
    case CF_SA: return c.sA;
    case CF_DTH: return c.dth;
    case CF_E2: return c.e2;
    case CF_INV_SA: return c.inv_sA;
    case CF_C: return c.c;
    default: return 1.0;
  }
}

// Class of B instances: constants table and activity flags (may be null).
struct Batch {
  int count;
  const InstCoef* coef;
  const int* act;
};

// Launch shape of the z-streaming node-stencil kernels on a grid.
struct StencilShape {
  int items;    // nodes per thread per plane (1,2,4,8)
  int threads;  // threads per block (256, or 512 for some 3D kernels)
  int chunk;    // nodes per block per plane (threads*items)
  int nchunks;  // chunks per plane
  int zc;       // most planes of a block: ceil(nn/nzc)
  int nzc;      // z-chunks; chunk c owns planes [c*nn/nzc, (c+1)*nn/nzc)
  int blocks;   // nchunks*nzc (per instance)
};
// Hardware places block b on XCD b % 8.  xcd_remap renumbers blocks so that
// each XCD receives a contiguous range of logical blocks (neighbouring
// tiles), which keeps the halo rows shared by neighbours in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb / 8, r = nb % 8;
  const int x = b % 8, t = b / 8;
  return ((x < r) ? x * (q + 1) : r * (q + 1) + (x - r) * q) + t;
}

// Planes [z0, z1) of z-chunk zch: the nn planes split as evenly as possible,
// so no block is left with a short remainder.
__device__ __forceinline__ void zrange(const StencilShape& sh, int nn, int zch, int& z0, int& z1) {
  z0 = (int)(((int64_t)zch * nn) / sh.nzc);
  z1 = (int)(((int64_t)(zch + 1) * nn) / sh.nzc);
}
StencilShape stencil_shape(const Grid& g, int nf, int word);
// Whether the table holds an entry (items > 0) for (g, key, word).
bool stencil_tuned(const Grid& g, int nf, int word);
// Shape-table key of the fused two-iteration Chebyshev kernel (in place of nf).
constexpr int kFusedKey = 17;
// Shape-table keys of the fused multigrid smoother kernels (pre-smoothing +
// residual, post-smoothing).
constexpr int kMgPreKey = 18, kMgPostKey = 19;
// Shape-table key of the 3D fused Chebyshev kernel on rectangular in-plane
// tiles; where it has an entry (items > 0) the fused pairs use it.
constexpr int kFusedTileKey = 20;
// Keys of the fused multigrid smoothers on in-plane tiles (3D), used where set.
constexpr int kMgPreTileKey = 21, kMgPostTileKey = 22;
// Keys of the fused kernels on overlapping in-plane windows with one column
// strip of nodes per thread (3D): Chebyshev pairs on M, multigrid pre- and
// post-smoothing; the entry's items field selects the window configuration
// (1..kStripCfgs), threads must be that configuration's.  Used where set (the
// multigrid ones on levels whose fused smoothers are on).
constexpr int kFusedStripKey = 23, kMgPreStripKey = 24, kMgPostStripKey = 25;
// Threads of window configuration `cfg` (0 if there is none), and its
// windows per plane of grid g.
int strip_threads(int cfg);
int64_t strip_windows(const Grid& g, int cfg);
constexpr int kStripConfigs = 5;
// In-plane tile of that kernel: tx x ty nodes, ntx tiles per row of tiles.
struct TileGeom {
  int tx, ty, ntx, nty;
};
// Tile of the 3D fused pair for `threads` threads of `items` nodes on grid g
// (false if none fits); blocks per plane = ntx * nty.
bool cheb2_tile_geom(const Grid& g, int threads, int items, TileGeom& tg);
// Launch-shape table of the stencil kernels, keyed by (dim, nodes per
// direction, stenciled fields, bytes per stenciled word); items < 0 marks the
// fused Chebyshev kernel as slower than single steps on that grid; items == 0 removes
// the entry (back to the heuristic).  Results do not depend on the shape.
void stencil_tune_set(int dim, int nn, int nf, int word, int items, int nzc, int threads = 256);
// The entry of (dim, nn, nf, word); items = nzc = threads = 0 when none is set.
void stencil_tune_get(int dim, int nn, int nf, int word, int* items, int* nzc, int* threads);

// Reduction blocks per instance for vectors of length n (a fixed function of
// n, so solo and batched runs sum in the same order).
int red_blocks(int64_t n);
constexpr int kMaxRedBlocks = 1024;

// ---------------------------------------------------------------------------
// Node-stencil launchers (asynchronous on `st`).  `lev` selects the operator
// of an instance: -1 = M on the finest grid (Chebyshev for A~^-1), l >= 0 =
// M_l + alpha K_l.  `osc` selects the output scale (a CoefField).  T is the
// storage type of the preconditioner vectors.
// ---------------------------------------------------------------------------
// out = add + a*(M s) + b*(K s), a = ca*field(fa), b = cb*field(fb)
template <class TS, class TA, class TO>
hipError_t launch_stencil_axpy(const Grid& g, const Batch& B, Vec<const TS> s, Vec<const TA> add,
                               double ca, int fa, double cb, int fb, Vec<TO> out, hipStream_t st);
// Two stenciled fields, up to two outputs (out1 may be null); coefficient
// slot q of output o is c[o][q] * field(f[o][q]) for
//   out_o = add_o + c0 M s0 + c1 K s0 + c2 M s1 + c3 K s1
template <class TS>
hipError_t launch_stencil_lin2(const Grid& g, const Batch& B, Vec<const TS> s0, Vec<const TS> s1,
                               Vec<const double> add0, Vec<const double> add1,
                               const double (&c)[2][4], const int (&f)[2][4], Vec<double> out0,
                               Vec<double> out1, hipStream_t st);
// Two consecutive middle iterations k, k+1 of the Chebyshev iteration on M
// (finest grid) in one pass, bitwise equal to two launch_cheb_step calls;
// last2: iteration k+1 is the final one.  r_{k+2} is written to rout, which
// must differ from r (r_k is read on rows other blocks own).  Returns
// hipErrorInvalidValue for grids it does not support.
template <class T>
hipError_t launch_cheb_step2(const Grid& g, const Batch& B, int k, int osc, bool last2, Vec<T> x,
                             Vec<const T> r, Vec<T> rout, Vec<const T> din, Vec<T> dout,
                             hipStream_t st);
// Process-wide switch of that fusion (on by default); results do not change.
// cheb_fusion_on: the switch is on and the fused kernel supports grid g.
void cheb_fusion_set(int enable);
// FGMRES iterations issued one ahead of the host-side stop test (default 0).
void issue_ahead_set(int enable);
bool cheb_fusion_on(const Grid& g, int word);
// Fused multigrid smoothers (two Chebyshev iterations before and after the
// coarse-grid correction, each in one pass with its neighbour).
void mg_fusion_set(int enable);
bool mg_fusion_enabled();
// Prolongation folded into the strip post-smoother (default on).
void prolong_fusion_set(int enable);
bool prolong_fusion_enabled();
bool mg2_shape_valid(const Grid& g, int key, int word);
bool mg_fusion_on(const Grid& g, int word);
template <class T>
hipError_t launch_mg_pre2(const Grid& g, const Batch& B, int lev, Vec<const T> b, Vec<T> x2,
                          Vec<T> r, hipStream_t st);
template <class T>
hipError_t launch_mg_post2(const Grid& g, const Batch& B, int lev, Vec<const T> b,
                           Vec<const T> x, Vec<T> xout, hipStream_t st);
// Post-smoothing from x + P ec (the coarse-grid correction ec on grid gc
// interpolated while x is staged): bitwise launch_prolong_add(gc -> g, ec,
// x) followed by launch_mg_post2 from the sum, without writing the sum.
// Available (mg_post_prolong_ok) for FP64 vectors where the strip
// post-smoother is selected.
template <class T>
bool mg_post_prolong_ok(const Grid& g, const Grid& gc);
template <class T>
hipError_t launch_mg_post2_prolong(const Grid& g, const Grid& gc, const Batch& B, int lev,
                                   Vec<const T> b, Vec<const T> x, Vec<const T> ec, Vec<T> xout,
                                   hipStream_t st);
// Launch shapes that have instantiated kernels (items per thread, threads).
bool stencil_shape_ok(int dim, int nf, int items, int threads);
bool cheb2_shape_ok(int dim, int items, int threads);
// Richardson residual on the Schur complement: with a = A~^-1 (dt th K z2)
// and G = 3 int u^2 a phi, res = y - (M z2 + G - M a + eps^2 K a).
template <class T>
hipError_t launch_schur_res(const Grid& g, const Batch& B, Vec<const T> a, Vec<const T> z2,
                            Vec<const double> G, Vec<const T> y, Vec<T> res, hipStream_t st);
// Preconditioner coupling: q = G - M z1 + eps^2 K z1 (G = 3 int u^2 z1 phi);
// y = r2 + q, nq = -q.  r2s (may be null): the value of r2 is r2s[0] * r2
// (per instance), rounded before the sum.
template <class T>
hipError_t launch_couple(const Grid& g, const Batch& B, Vec<const T> z1, Vec<const double> G,
                         Vec<const double> r2, Vec<const double> r2s, Vec<T> y, Vec<double> nq,
                         hipStream_t st);
// Chebyshev-Jacobi building blocks (Saad, Alg. 12.1).  bs (may be null): the
// value of b is bs[0] * b (per instance), rounded to TB as it is staged.
// one iteration from x0 = 0: x = oscale * D^-1 b * it
template <class TB, class T>
hipError_t launch_cheb_one(const Grid& g, const Batch& B, int lev, int osc, Vec<const TB> b,
                           Vec<T> x, hipStream_t st,
                           Vec<const double> bs = Vec<const double>{nullptr, 0});
// iteration 0 from x0 = 0: d0 = D^-1 b it, r1 = b - A d0, d1 = c1[0] d0 + c2[0] D^-1 r1;
// writes x = d0, r = r1, d = d1, or (last) x = oscale*(d0 + d1) only.
template <class TB, class T>
hipError_t launch_cheb_first(const Grid& g, const Batch& B, int lev, int osc, bool last,
                             Vec<const TB> b, Vec<T> x, Vec<T> r, Vec<T> d, hipStream_t st,
                             Vec<const double> bs = Vec<const double>{nullptr, 0});
// iteration k: x += d_k, r -= A d_k, d_{k+1} = c1[k] d_k + c2[k] D^-1 r (into dout);
// last: x = oscale*(x + d_k + d_{k+1}) only.
template <class T>
hipError_t launch_cheb_step(const Grid& g, const Batch& B, int lev, int k, int osc, bool last,
                            Vec<T> x, Vec<T> r, Vec<const T> din, Vec<T> dout, hipStream_t st);
// start from a given x: r = b - A x, d = D^-1 r it (x unchanged)
template <class T>
hipError_t launch_cheb_start(const Grid& g, const Batch& B, int lev, Vec<const T> b,
                             Vec<const T> x, Vec<T> r, Vec<T> d, hipStream_t st);
// x += d
template <class T>
hipError_t launch_add_inplace(const Batch& B, Vec<T> x, Vec<const T> d, int64_t n,
                              hipStream_t st);
// r = b - A x
template <class T>
hipError_t launch_resid(const Grid& g, const Batch& B, int lev, Vec<const T> b, Vec<const T> x,
                        Vec<T> r, hipStream_t st);

// Element quadrature on the finest grid:
// mode 0: out = alpha * G(u,x) + beta * add,  G_i = int u^2 x phi_i   (M_E(u) x = 3G - M x)
// mode 1: out = alpha * N(u),  N_i = int (u^3 - u) phi_i
template <class TX, class TO>
hipError_t launch_element(const Grid& g, const Batch& B, int mode, Vec<const double> u,
                          Vec<const TX> x, Vec<const double> add, double alpha, double beta,
                          Vec<TO> out, hipStream_t st);

// Multigrid transfers and the exact coarse solve (M + alpha K)^-1 (DCT-I basis).
template <class T>
hipError_t launch_restrict(const Grid& fine, const Grid& coarse, const Batch& B, Vec<const T> r,
                           Vec<T> bc, hipStream_t st);
template <class T>
hipError_t launch_prolong_add(const Grid& fine, const Grid& coarse, const Batch& B,
                              Vec<const T> ec, Vec<T> x, hipStream_t st);
// Coarse solve: grids of at most 1024 nodes in one block per instance, larger
// ones (at most 64 nodes per direction) axis by axis through the scratch
// vectors s1, s2 (nodes of g per instance).
template <class T>
hipError_t launch_coarse_solve(const Grid& g, const Batch& B, Vec<const T> b, Vec<T> x,
                               Vec<T> s1, Vec<T> s2, hipStream_t st);

// ---------------------------------------------------------------------------
// Vector and Krylov kernels (FP64 unless templated).
// ---------------------------------------------------------------------------
template <class TI, class TO>
hipError_t launch_copy_scale(const Batch& B, Vec<const TI> in, Vec<TO> out, double a, int64_t n,
                             hipStream_t st);
// out = a*x + b*y
hipError_t launch_axpby(const Batch& B, double a, Vec<const double> x, double b,
                        Vec<const double> y, Vec<double> out, int64_t n, hipStream_t st);
hipError_t launch_fill(const Batch& B, Vec<double> x, double v, int64_t n, hipStream_t st);
// partials (red_blocks(n) per instance) of sum a*b
hipError_t launch_dot_partial(const Batch& B, Vec<const double> a, Vec<const double> b,
                              int64_t n, Vec<double> partials, hipStream_t st);
// out[0] = sum(partials), out[1] = sqrt(out[0])   (partials of length red_blocks(n))
hipError_t launch_reduce_final(const Batch& B, Vec<const double> partials, int64_t n,
                               Vec<double> out, hipStream_t st);
// Fused modified Gram-Schmidt step: h = sum(pin); Hij = h; w -= h*vi;
// pout = partials of <w, vnext> (vnext null: <w, w>).
hipError_t launch_mgs_step(const Batch& B, Vec<double> w, Vec<const double> vi,
                           Vec<const double> vnext, int64_t n, Vec<const double> pin,
                           Vec<double> pout, Vec<double> Hij, hipStream_t st);
// FGMRES bookkeeping of one instance (all in device memory, per instance):
//   kr: [0] ||b||, [1] tol = rtol ||b||, [2] beta, [3] |g_{j+1}|, [4] h_{j+1,j},
//       [5] 1/h_{j+1,j}, [6] iterations of this cycle (k), [7] status flags
// Givens update of Hessenberg column j (column-major, leading dim m+1); an
// instance whose |g_{j+1}| <= tol or h_{j+1,j} == 0 is marked converged
// (act = 0, status bit 1); a non-finite value sets status bit 2 and act = 0.
// sc (may be null): sc[j+1] = 1/h_{j+1,j}, the scale of the unnormalised
// new basis vector.
hipError_t launch_givens(const Batch& B, int* act, int j, int m, Vec<double> H, Vec<double> cs,
                         Vec<double> sn, Vec<double> g, Vec<const double> pnorm, int64_t n,
                         Vec<double> kr, Vec<double> sc, hipStream_t st);
// Arnoldi projection of w against v_i = sc[i] V_i, i = 0..j, in two passes
// (modified Gram-Schmidt in inverse compact WY form): the dots <w, V_i> and
// <V_j, V_i> (partials in pd: 2m rows of red_blocks(n)), row j of L =
// lower part of V^T V (row-major, (m+1)^2), the triangular solve for the
// coefficients h (Hcol[i] = h_i, column j of the Hessenberg matrix;
// hc[i] = h_i sc[i]), then w -= sum hc_i V_i with the partials of <w, w> in
// pnorm.  V: base of the basis, vector i at V + i*vstride.  m <= 64.
constexpr int kProjGroup = 16;  // basis vectors per dot pass (2 accumulators each per thread)
hipError_t launch_proj(const Batch& B, Vec<double> w, Vec<const double> V, int64_t vstride, int j,
                       int m, int64_t n, Vec<double> pd, Vec<const double> sc, Vec<double> L,
                       Vec<double> Hcol, Vec<double> hc, Vec<double> pnorm, hipStream_t st);
// v = w * kr[5]  (normalise the new Arnoldi vector)
hipError_t launch_scale_by(const Batch& B, Vec<const double> w, Vec<double> v,
                           Vec<const double> kr, int64_t n, hipStream_t st);
// v = b / nrm[1]
hipError_t launch_scale_inv(const Batch& B, Vec<const double> b, Vec<double> v,
                            Vec<const double> nrm, int64_t n, hipStream_t st);
// Start of a cycle: g = [beta, 0, ...], kr[6] = 0 (with beta = nrm[1]), and
// the basis scales sc[0..m] = 1 (sc may be null).
hipError_t launch_cycle_init(const Batch& B, int m, Vec<double> g, Vec<const double> nrm,
                             Vec<double> kr, Vec<double> sc, hipStream_t st);
// y = H(0:k,0:k)^-1 g(0:k) with k = kr[6], then x += sum_j y_j Z_j
template <class TZ>
hipError_t launch_lsq_update(const Batch& B, int m, Vec<const double> H, Vec<const double> g,
                             Vec<double> y, Vec<const double> kr, Vec<const TZ> Z,
                             int64_t zstride, Vec<double> x, int64_t n, hipStream_t st);

// Preconditioned MINRES on the symmetric rearranged Newton system (Elman,
// Silvester and Wathen, Alg. 4.1), per instance, vectors of length n2 = 2n
// in the unknown order [dw; du].  The scalars of the recurrence live in
// device memory, MR_COUNT doubles per instance (slots below); z vectors are
// kept unnormalised (z_j = gam_j * z^_j) and the normalisation is folded
// into the kernels that read them.
enum MinresSlot {
  MR_GAM0 = 0,  // gamma_{j-1}
  MR_GAM,       // gamma_j
  MR_ETA,       // eta (the residual norm up to sign)
  MR_S0, MR_S, MR_C0, MR_C,  // Givens sines and cosines of the last two steps
  MR_TOL,       // rtol * gamma_1
  MR_DELTA,     // delta_j
  MR_WZ, MR_W0, MR_W1,  // w_{j+1} = WZ z_j + W0 w_{j-1} + W1 w_j
  MR_XC,        // x += XC w_{j+1}
  MR_ITS,       // iterations done
  MR_STATUS,    // 0 running, 1 converged, 2 non-finite, 3 iteration limit
  MR_GAM1,      // gamma_1 (initial preconditioned residual norm)
  MR_XCP,       // XC of the previous iteration (its x update is deferred to this one)
  MR_COUNT = 17
};
// Start: v1 = [s b1; b2] (s = 1/(1 + dt th sigma) if scale_first, else 1),
// and v0, w0, w1, x = 0.
hipError_t launch_mr_init(const Batch& B, Vec<const double> b, Vec<double> v1, Vec<double> v0,
                          Vec<double> w0, Vec<double> w1, Vec<double> x, int64_t n,
                          bool scale_first, hipStream_t st);
// z = [(alpha/c) z1; (c/alpha) z2] in place, and the partials of <z, v>
// (red_blocks(2n) per instance).
hipError_t launch_mr_scale_dot(const Batch& B, Vec<double> z, Vec<const double> v, int64_t n,
                               Vec<double> partials, hipStream_t st);
// gamma_1 = sqrt(sum partials); initial scalars; act = 1 unless gamma_1 is
// zero (converged, status 1) or not finite (status 2).  B.act: participating.
hipError_t launch_mr_start(const Batch& B, int* act, Vec<const double> partials, int64_t n2,
                           Vec<double> mr, hipStream_t st);
// delta = sum(partials of <A z, z>) / gamma^2;
// v2 = (A z)/gamma - (delta/gamma) v1 - (gamma/gamma0) v0.
hipError_t launch_mr_vupd(const Batch& B, Vec<const double> partials, Vec<const double> az,
                          Vec<const double> v1, Vec<const double> v0, Vec<double> v2, int64_t n2,
                          Vec<double> mr, hipStream_t st);
// gamma_{j+1} = sqrt(sum partials of <z2, v2>), the Givens step of the QR
// factorisation and the stop test (act cleared on convergence, non-finite
// values or after maxit iterations); ran = 1 for the instances that took this
// step (act set on entry), 0 otherwise.  B.act: participating.
hipError_t launch_mr_coef(const Batch& B, int* act, int* ran, Vec<const double> partials,
                          int64_t n2, int maxit, Vec<double> mr, hipStream_t st);
// w2 = WZ z + W0 w0 + W1 w1, and x += XCP w1 + XC w2 after an even number
// of iterations, x += XC w2 in an odd-numbered last one (act cleared), else
// x is left for the next iteration; swap: x is stored with its halves
// exchanged ([du; dw]).  B.act: the instances that took the step.
hipError_t launch_mr_wx(const Batch& B, const int* act, Vec<const double> z,
                        Vec<const double> w0, Vec<const double> w1, Vec<double> w2,
                        Vec<double> x, int64_t n, bool swap, Vec<const double> mr,
                        hipStream_t st);

// Residual assembly helper (FP64):
// t1 = (u - un) + dt*sigma*(th*u + (1-th)*un - m),  t2 = dt*(th*w + (1-th)*wn)
hipError_t launch_residual_prep(const Batch& B, Vec<const double> u, Vec<const double> un,
                                Vec<const double> w, Vec<const double> wn, Vec<double> t1,
                                Vec<double> t2, int64_t n, hipStream_t st);

}  // namespace okd
