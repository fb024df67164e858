// Internal declarations shared by the HIP sources of libok.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ok.h"

namespace okd {

constexpr int kMaxLevels = 16;
constexpr int kThreads = 256;          // node-stencil and vector kernels
constexpr int kRedBlocks = 1024;       // fixed grid of every reduction (determinism)

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
};

Grid make_grid(int dim, int N);

// Launch shape of the z-streaming node-stencil kernels on a grid.
struct StencilShape {
  int items;      // nodes per thread per plane (1,2,4,8)
  int chunk;      // nodes per block per plane (kThreads*items)
  int nchunks;    // chunks per plane
  int zc;         // planes per block (3D)
  int nzc;        // z-chunks
  int blocks;     // nchunks*nzc
};
StencilShape stencil_shape(const Grid& g, int nf, int word);
// Launch-shape table of the stencil kernels, keyed by (dim, nodes per
// direction, stenciled fields, bytes per stenciled word); items <= 0 removes
// the entry (back to the heuristic).
// Results do not depend on the shape: every node is computed by the same
// arithmetic in the same order whatever the tiling.
void stencil_tune_set(int dim, int nn, int nf, int word, int items, int zc);

// Operator A = cm*M + ck*K on a grid and its Jacobi diagonal:
// diag(A) at a node = dint * 2^-(number of coordinates on the boundary).
struct Op {
  double cm, ck;
  double dinv_int;  // 1/dint
};
Op make_op(const Grid& g, double cm, double ck);

// Chebyshev coefficients of Saad's Alg. 12.1 for an interval [a,b].
struct Cheb {
  double theta, delta, sigma1;
};

// ---------------------------------------------------------------------------
// Kernel launchers (asynchronous on `st`).  T is the storage type of the
// preconditioner vectors (double or float); arithmetic is FP64.
// ---------------------------------------------------------------------------
// out = scale * (M s)
template <class TI, class TO>
hipError_t launch_mass(const Grid& g, const TI* s, TO* out, double scale, hipStream_t st);

// Chebyshev-Jacobi building blocks (Saad, Alg. 12.1), on A with D = diag(A):
// one iteration from x0 = 0: x = out_scale * D^-1 b / theta
template <class TB, class T>
hipError_t launch_cheb_one(const Grid& g, const Op& A, double inv_theta, double out_scale,
                           const TB* b, T* x, hipStream_t st);
// iteration 0 from x0 = 0: d0 = D^-1 b/theta, r1 = b - A d0, d1 = c1 d0 + c2 D^-1 r1;
// writes x = d0, r = r1, d = d1, or (last) x = out_scale*(d0 + d1) only.
template <class TB, class T>
hipError_t launch_cheb_first(const Grid& g, const Op& A, double inv_theta, double c1, double c2,
                             double out_scale, bool last, const TB* b, T* x, T* r, T* d,
                             hipStream_t st);
// iteration k: x += d_k, r -= A d_k, d_{k+1} = c1 d_k + c2 D^-1 r (into dout);
// last: x = out_scale*(x + d_k + d_{k+1}) only.
template <class T>
hipError_t launch_cheb_step(const Grid& g, const Op& A, double c1, double c2, double out_scale,
                            bool last, T* x, T* r, const T* din, T* dout, hipStream_t st);
// start from a given x: r = b - A x, d = D^-1 r / theta (x unchanged)
template <class T>
hipError_t launch_cheb_start(const Grid& g, const Op& A, double inv_theta, const T* b,
                             const T* x, T* r, T* d, hipStream_t st);
template <class T>
hipError_t launch_add_inplace(T* x, const T* d, int64_t n, hipStream_t st);
// r = b - A x
template <class T>
hipError_t launch_resid(const Grid& g, const Op& A, const T* b, const T* x, T* r, hipStream_t st);
// out = add + a*(M s) + b*(K s)  (add may be null)
template <class TS, class TA, class TO>
hipError_t launch_stencil_axpy(const Grid& g, const TS* s, const TA* add, double a, double b,
                               TO* out, hipStream_t st);

// Two stenciled fields, up to two outputs (out1 may be null):
//   out0 = add0 + c0[0] M s0 + c0[1] K s0 + c0[2] M s1 + c0[3] K s1
//   out1 = add1 + c1[0] M s0 + c1[1] K s0 + c1[2] M s1 + c1[3] K s1
template <class TS>
hipError_t launch_stencil_lin2(const Grid& g, const TS* s0, const TS* s1, const double* add0,
                               const double* add1, const double* c0, const double* c1,
                               double* out0, double* out1, hipStream_t st);

// Element quadrature kernels on the finest grid:
// mode 0: out = alpha * G(u,x) + beta * add,  G_i = int u^2 x phi_i  (add may be null)
//         (M_E(u) x = 3 G(u,x) - M x)
// mode 1: out = alpha * N(u),  N_i = int (u^3 - u) phi_i
template <class TX, class TO>
hipError_t launch_element(const Grid& g, int mode, const double* u, const TX* x,
                          const double* add, double alpha, double beta, TO* out, hipStream_t st);

// Multigrid transfers and the coarse solve.
template <class T>
hipError_t launch_restrict(const Grid& fine, const Grid& coarse, const T* r, T* bc, hipStream_t st);
template <class T>
hipError_t launch_prolong_add(const Grid& fine, const Grid& coarse, const T* ec, T* x,
                              hipStream_t st);
// Exact (M + alpha K)^-1 on a small grid by the DCT-I eigenbasis.
template <class T>
hipError_t launch_coarse_solve(const Grid& g, double alpha, const T* b, T* x, hipStream_t st);

// Vector and Krylov kernels (FP64 unless templated).
template <class TI, class TO>
hipError_t launch_copy_scale(const TI* in, TO* out, double a, int64_t n, hipStream_t st);
hipError_t launch_axpby(double a, const double* x, double b, const double* y, double* out,
                        int64_t n, hipStream_t st);
hipError_t launch_fill(double* x, double v, int64_t n, hipStream_t st);
// partials[k] (kRedBlocks) of sum a*b
hipError_t launch_dot_partial(const double* a, const double* b, int64_t n, double* partials,
                              hipStream_t st);
// out[0] = sum(partials), out[1] = sqrt(out[0])
hipError_t launch_reduce_final(const double* partials, double* out, hipStream_t st);
// One fused modified Gram-Schmidt step: h = sum(pin); Hij = h; w -= h*vi;
// pout = partials of <w, vnext> (vnext == nullptr: <w, w>).
hipError_t launch_mgs_step(double* w, const double* vi, const double* vnext, int64_t n,
                           const double* pin, double* pout, double* Hij, hipStream_t st);
// Givens update of Hessenberg column j (column-major H[col*(m+1)+row]); writes
// scal[0] = |g_{j+1}|, scal[1] = h_{j+1,j}, scal[2] = 1/h_{j+1,j}.
hipError_t launch_givens(int j, int m, double* H, double* cs, double* sn, double* g,
                         const double* pnorm, double* scal, hipStream_t st);
// v = w * scal[2]
hipError_t launch_scale_by(const double* w, double* v, const double* scal, int64_t n,
                           hipStream_t st);
// y = H(0:k,0:k)^-1 g(0:k), then x += sum_j y_j Z_j
template <class TZ>
hipError_t launch_lsq_update(int k, int m, const double* H, const double* g, double* y,
                             const TZ* Z, int64_t zstride, double* x, int64_t n, hipStream_t st);
// V0 = b * (1/scal), with scal = ||b|| read from device
hipError_t launch_scale_inv(const double* b, double* v, const double* nrm, int64_t n,
                            hipStream_t st);

// Residual assembly helpers (FP64):
// t1 = (u - un) + dt*sigma*(th*u + (1-th)*un - m),  t2 = dt*(th*w + (1-th)*wn)
hipError_t launch_residual_prep(const double* u, const double* un, const double* w,
                                const double* wn, double dt, double sigma, double th, double m,
                                double* t1, double* t2, int64_t n, hipStream_t st);

}  // namespace okd
