// Vector kernels of flexible GMRES (Saad 1993) with modified Gram-Schmidt.
//
// Every reduction is deterministic: a fixed grid of kRedBlocks blocks, a
// grid-stride partial sum per thread, a fixed wavefront-shuffle + LDS tree per
// block into partials[block], and a fixed tree over the partials wherever the
// sum is needed (each consumer block recomputes it identically), so results
// are bitwise reproducible run to run.
#include "ok_internal.h"

#include <cmath>

namespace okd {

namespace {

__device__ __forceinline__ double ld(const double* p) { return *p; }
__device__ __forceinline__ double ld(const float* p) { return (double)*p; }

// Sum over the block (256 threads); result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; i++) s += sh[i];
  return s;
}

// Sum of the kRedBlocks partials, same order in every block.
__device__ __forceinline__ double sum_partials(const double* p, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) v += p[i];
  return block_sum(v, sh);
}

__global__ void __launch_bounds__(256)
    k_dot(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
          double* __restrict__ partials) {
  __shared__ double sh[8];
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v += a[i] * b[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

__global__ void __launch_bounds__(256)
    k_reduce_final(const double* __restrict__ partials, double* __restrict__ out) {
  __shared__ double sh[8];
  double s = sum_partials(partials, sh);
  if (threadIdx.x == 0) {
    out[0] = s;
    out[1] = sqrt(s);
  }
}

__global__ void __launch_bounds__(256)
    k_mgs(double* __restrict__ w, const double* __restrict__ vi, const double* __restrict__ vn,
          int64_t n, const double* __restrict__ pin, double* __restrict__ pout,
          double* __restrict__ Hij) {
  __shared__ double sh[8];
  const double h = sum_partials(pin, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) *Hij = h;
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double x = w[i] - h * vi[i];
    w[i] = x;
    v += x * (vn ? vn[i] : x);
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) pout[blockIdx.x] = v;
}

// Givens rotations on Hessenberg column j (one wavefront; thread 0 does the
// arithmetic in the order of the textbook recurrence).
__global__ void k_givens(int j, int m, double* H, double* cs, double* sn, double* g,
                         const double* pnorm, double* scal) {
  __shared__ double sh[8];
  double s = sum_partials(pnorm, sh);
  if (threadIdx.x != 0) return;
  const int ld = m + 1;
  double* col = H + (int64_t)j * ld;
  double hn = sqrt(s);
  col[j + 1] = hn;
  for (int i = 0; i < j; i++) {
    double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  double den = hypot(col[j], col[j + 1]);
  cs[j] = col[j] / den;
  sn[j] = col[j + 1] / den;
  col[j] = den;
  col[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  scal[0] = fabs(g[j + 1]);
  scal[1] = hn;
  scal[2] = 1.0 / hn;
}

__global__ void __launch_bounds__(256)
    k_scale_by(const double* __restrict__ w, double* __restrict__ v,
               const double* __restrict__ scal, int64_t n) {
  const double s = scal[2];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = w[i] * s;
}

__global__ void __launch_bounds__(256)
    k_scale_inv(const double* __restrict__ b, double* __restrict__ v,
                const double* __restrict__ nrm, int64_t n) {
  const double s = 1.0 / nrm[1];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = b[i] * s;
}

// Back substitution with the triangular H (column-major, leading dim m+1).
__global__ void k_lsq(int k, int m, const double* H, const double* g, double* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int ld = m + 1;
  for (int i = k - 1; i >= 0; i--) {
    double s = g[i];
    for (int l = i + 1; l < k; l++) s -= H[(int64_t)l * ld + i] * y[l];
    y[i] = s / H[(int64_t)i * ld + i];
  }
}

template <class TZ>
__global__ void __launch_bounds__(256)
    k_update_x(int k, const double* __restrict__ y, const TZ* __restrict__ Z, int64_t zstride,
               double* __restrict__ x, int64_t n) {
  __shared__ double ys[64];
  if (threadIdx.x < k) ys[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = x[i];
    for (int j = 0; j < k; j++) s += ys[j] * ld(Z + j * zstride + i);
    x[i] = s;
  }
}

template <class TI, class TO>
__global__ void __launch_bounds__(256)
    k_copy_scale(const TI* __restrict__ in, TO* __restrict__ out, double a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (TO)(a * ld(in + i));
}

__global__ void __launch_bounds__(256)
    k_axpby(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
            double* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a * x[i] + b * y[i];
}

__global__ void __launch_bounds__(256) k_fill(double* __restrict__ x, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void __launch_bounds__(256)
    k_residual_prep(const double* __restrict__ u, const double* __restrict__ un,
                    const double* __restrict__ w, const double* __restrict__ wn, double dt,
                    double sigma, double th, double m, double* __restrict__ t1,
                    double* __restrict__ t2, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double uu = u[i], uo = un[i], ww = w[i];
    double wo = wn ? wn[i] : ww;
    t1[i] = (uu - uo) + dt * sigma * (th * uu + (1.0 - th) * uo - m);
    t2[i] = dt * (th * ww + (1.0 - th) * wo);
  }
}

unsigned vec_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_dot_partial(const double* a, const double* b, int64_t n, double* partials,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_dot, dim3(kRedBlocks), dim3(256), 0, st, a, b, n, partials);
  return hipGetLastError();
}

hipError_t launch_reduce_final(const double* partials, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, partials, out);
  return hipGetLastError();
}

hipError_t launch_mgs_step(double* w, const double* vi, const double* vnext, int64_t n,
                           const double* pin, double* pout, double* Hij, hipStream_t st) {
  hipLaunchKernelGGL(k_mgs, dim3(kRedBlocks), dim3(256), 0, st, w, vi, vnext, n, pin, pout, Hij);
  return hipGetLastError();
}

hipError_t launch_givens(int j, int m, double* H, double* cs, double* sn, double* g,
                         const double* pnorm, double* scal, hipStream_t st) {
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(256), 0, st, j, m, H, cs, sn, g, pnorm, scal);
  return hipGetLastError();
}

hipError_t launch_scale_by(const double* w, double* v, const double* scal, int64_t n,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_scale_by, dim3(vec_blocks(n)), dim3(256), 0, st, w, v, scal, n);
  return hipGetLastError();
}

hipError_t launch_scale_inv(const double* b, double* v, const double* nrm, int64_t n,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_scale_inv, dim3(vec_blocks(n)), dim3(256), 0, st, b, v, nrm, n);
  return hipGetLastError();
}

template <class TZ>
hipError_t launch_lsq_update(int k, int m, const double* H, const double* g, double* y,
                             const TZ* Z, int64_t zstride, double* x, int64_t n, hipStream_t st) {
  if (k > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lsq, dim3(1), dim3(64), 0, st, k, m, H, g, y);
  hipLaunchKernelGGL((k_update_x<TZ>), dim3(vec_blocks(n)), dim3(256), 0, st, k, (const double*)y,
                     Z, zstride, x, n);
  return hipGetLastError();
}

template <class TI, class TO>
hipError_t launch_copy_scale(const TI* in, TO* out, double a, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_copy_scale<TI, TO>), dim3(vec_blocks(n)), dim3(256), 0, st, in, out, a,
                     n);
  return hipGetLastError();
}

hipError_t launch_axpby(double a, const double* x, double b, const double* y, double* out,
                        int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(vec_blocks(n)), dim3(256), 0, st, a, x, b, y, out, n);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, double v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(vec_blocks(n)), dim3(256), 0, st, x, v, n);
  return hipGetLastError();
}

hipError_t launch_residual_prep(const double* u, const double* un, const double* w,
                                const double* wn, double dt, double sigma, double th, double m,
                                double* t1, double* t2, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_residual_prep, dim3(vec_blocks(n)), dim3(256), 0, st, u, un, w, wn, dt,
                     sigma, th, m, t1, t2, n);
  return hipGetLastError();
}

template hipError_t launch_lsq_update<double>(int, int, const double*, const double*, double*,
                                              const double*, int64_t, double*, int64_t,
                                              hipStream_t);
template hipError_t launch_lsq_update<float>(int, int, const double*, const double*, double*,
                                             const float*, int64_t, double*, int64_t,
                                             hipStream_t);
template hipError_t launch_copy_scale<double, double>(const double*, double*, double, int64_t,
                                                      hipStream_t);
template hipError_t launch_copy_scale<double, float>(const double*, float*, double, int64_t,
                                                     hipStream_t);
template hipError_t launch_copy_scale<float, double>(const float*, double*, double, int64_t,
                                                     hipStream_t);

}  // namespace okd
