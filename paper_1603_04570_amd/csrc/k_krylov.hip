// Vector kernels of flexible GMRES (Saad 1993) with modified Gram-Schmidt,
// for a class of B instances (see ok_internal.h).
//
// Every reduction is deterministic: red_blocks(n) blocks per instance (a
// fixed function of the vector length), a grid-stride partial sum per
// thread, a fixed wavefront-shuffle + LDS tree per block into
// partials[block], and a fixed tree over the partials wherever the sum is
// needed (each consumer block recomputes it identically).  Results are
// bitwise reproducible and independent of how many instances share a launch.
#include "ok_internal.h"

#include <algorithm>
#include <cmath>

namespace okd {

namespace {

__device__ __forceinline__ double ld(const double* p) { return *p; }
__device__ __forceinline__ double ld(const float* p) { return (double)*p; }
// Streaming accesses of the Krylov vectors (each touched once per pass and
// far larger than the caches at the sizes that matter): nontemporal hints.
__device__ __forceinline__ double ldnt(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void stnt(double v, double* p) { __builtin_nontemporal_store(v, p); }

// Threads per block of the reduction kernels (k_dot, k_mgs).
constexpr int kRedThreads = 512;

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

// Sum of nblk partials, same order in every block.
__device__ __forceinline__ double sum_partials(const double* p, int nblk, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) v += p[i];
  return block_sum(v, sh);
}

__device__ __forceinline__ bool inactive(const Batch& B, int inst) {
  return B.act && !B.act[inst];
}

// Element order of a reduction over a vector of length n: thread t of
// reduction block kb visits i = kb*T + t + k*nblk*T (T = kRedThreads),
// k = 0, 1, ..., in that order (explicit fma).  Scalar nontemporal loads:
// on gfx950 this streams faster than 16-byte loads for these passes.
__global__ void __launch_bounds__(kRedThreads)
    k_dot(Batch B, Vec<const double> av, Vec<const double> bv, int64_t n, Vec<double> pv,
          int nblk) {
  __shared__ double sh[kRedThreads / 64];
  const int inst = blockIdx.x / nblk, kb = blockIdx.x % nblk;
  if (inactive(B, inst)) return;
  const double* a = av.at(inst);
  const double* b = bv.at(inst);
  double v = 0.0;
  for (int64_t i = (int64_t)kb * blockDim.x + threadIdx.x; i < n; i += (int64_t)nblk * blockDim.x)
    v = fma(ldnt(a + i), ldnt(b + i), v);
  v = block_sum(v, sh);
  if (threadIdx.x == 0) pv.at(inst)[kb] = v;
}

__global__ void __launch_bounds__(256)
    k_reduce_final(Batch B, Vec<const double> pv, int nblk, Vec<double> out) {
  __shared__ double sh[8];
  const int inst = blockIdx.x;
  if (inactive(B, inst)) return;
  double s = sum_partials(pv.at(inst), nblk, sh);
  if (threadIdx.x == 0) {
    out.at(inst)[0] = s;
    out.at(inst)[1] = sqrt(s);
  }
}

// One modified Gram-Schmidt step, fused with the next dot product:
// h = <w, v_i> (from the partials of the previous pass), w -= h v_i, and the
// partials of <w, v_next> (of <w, w> when v_next is null).  Same element
// order as k_dot.
template <bool NORM>
__global__ void __launch_bounds__(kRedThreads)
    k_mgs(Batch B, Vec<double> wv, Vec<const double> viv, Vec<const double> vnv, int64_t n,
          Vec<const double> pinv, Vec<double> poutv, Vec<double> Hv, int nblk) {
  __shared__ double sh[kRedThreads / 64];
  const int inst = blockIdx.x / nblk, kb = blockIdx.x % nblk;
  if (inactive(B, inst)) return;
  const double h = sum_partials(pinv.at(inst), nblk, sh);
  if (kb == 0 && threadIdx.x == 0) *Hv.at(inst) = h;
  double* w = wv.at(inst);
  const double* vi = viv.at(inst);
  const double* vn = NORM ? nullptr : vnv.at(inst);
  double v = 0.0;
  for (int64_t i = (int64_t)kb * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)nblk * blockDim.x) {
    const double x = fma(-h, ldnt(vi + i), ldnt(w + i));
    stnt(x, w + i);
    v = fma(x, NORM ? x : ldnt(vn + i), v);
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) poutv.at(inst)[kb] = v;
}

// Givens rotations on Hessenberg column j of one instance (thread 0 does the
// arithmetic in the order of the textbook recurrence) and the stop test.
__global__ void k_givens(Batch B, int* act, int j, int m, Vec<double> Hv, Vec<double> csv,
                         Vec<double> snv, Vec<double> gv, Vec<const double> pnv, int nblk,
                         Vec<double> krv) {
  __shared__ double sh[8];
  const int inst = blockIdx.x;
  if (inactive(B, inst)) return;
  double s = sum_partials(pnv.at(inst), nblk, sh);
  if (threadIdx.x != 0) return;
  double* col = Hv.at(inst) + (int64_t)j * (m + 1);
  double* cs = csv.at(inst);
  double* sn = snv.at(inst);
  double* g = gv.at(inst);
  double* kr = krv.at(inst);
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
  const double res = fabs(g[j + 1]);
  kr[3] = res;
  kr[4] = hn;
  kr[5] = 1.0 / hn;
  kr[6] = (double)(j + 1);
  if (!isfinite(hn) || !isfinite(res)) {
    kr[7] = 2.0;
    act[inst] = 0;
  } else if (res <= kr[1] || hn == 0.0) {
    kr[7] = 1.0;
    act[inst] = 0;
  }
}

__global__ void __launch_bounds__(256)
    k_scale_by(Batch B, Vec<const double> wv, Vec<double> vv, Vec<const double> krv, int64_t n,
               int per) {
  const int inst = blockIdx.x / per;
  if (inactive(B, inst)) return;
  const double s = krv.at(inst)[5];
  const double* w = wv.at(inst);
  double* v = vv.at(inst);
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)per * blockDim.x)
    stnt(ldnt(w + i) * s, v + i);
}

__global__ void __launch_bounds__(256)
    k_scale_inv(Batch B, Vec<const double> bv, Vec<double> vv, Vec<const double> nv, int64_t n,
                int per) {
  const int inst = blockIdx.x / per;
  if (inactive(B, inst)) return;
  const double s = 1.0 / nv.at(inst)[1];
  const double* b = bv.at(inst);
  double* v = vv.at(inst);
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)per * blockDim.x)
    v[i] = b[i] * s;
}

__global__ void k_cycle_init(Batch B, int m, Vec<double> gv, Vec<const double> nv,
                             Vec<double> krv) {
  const int inst = blockIdx.x;
  if (inactive(B, inst)) return;
  double* g = gv.at(inst);
  const double beta = nv.at(inst)[1];
  for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = (i == 0) ? beta : 0.0;
  if (threadIdx.x == 0) {
    double* kr = krv.at(inst);
    kr[2] = beta;
    kr[6] = 0.0;
    kr[7] = 0.0;
  }
}

// Back substitution with the triangular H (column-major, leading dim m+1).
__global__ void k_lsq(Batch B, int m, Vec<const double> Hv, Vec<const double> gv, Vec<double> yv,
                      Vec<const double> krv) {
  const int inst = blockIdx.x;
  if (inactive(B, inst) || threadIdx.x != 0) return;
  const double* H = Hv.at(inst);
  const double* g = gv.at(inst);
  double* y = yv.at(inst);
  const int k = (int)krv.at(inst)[6];
  const int ldh = m + 1;
  for (int i = k - 1; i >= 0; i--) {
    double s = g[i];
    for (int l = i + 1; l < k; l++) s -= H[(int64_t)l * ldh + i] * y[l];
    y[i] = s / H[(int64_t)i * ldh + i];
  }
}

template <class TZ>
__global__ void __launch_bounds__(256)
    k_update_x(Batch B, Vec<const double> yv, Vec<const double> krv, Vec<const TZ> Zv,
               int64_t zstride, Vec<double> xv, int64_t n, int per) {
  __shared__ double ys[64];
  const int inst = blockIdx.x / per;
  if (inactive(B, inst)) return;
  const int k = (int)krv.at(inst)[6];
  if (threadIdx.x < k) ys[threadIdx.x] = yv.at(inst)[threadIdx.x];
  __syncthreads();
  const TZ* Z = Zv.at(inst);
  double* x = xv.at(inst);
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)per * blockDim.x) {
    double s = x[i];
    for (int j = 0; j < k; j++) s += ys[j] * ld(Z + j * zstride + i);
    x[i] = s;
  }
}

template <class TI, class TO>
__global__ void __launch_bounds__(256)
    k_copy_scale(Batch B, Vec<const TI> inv, Vec<TO> outv, double a, int64_t n, int per) {
  const int inst = blockIdx.x / per;
  if (inactive(B, inst)) return;
  const TI* in = inv.at(inst);
  TO* out = outv.at(inst);
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)per * blockDim.x)
    out[i] = (TO)(a * ld(in + i));
}

__global__ void __launch_bounds__(256)
    k_axpby(Batch B, double a, Vec<const double> xv, double b, Vec<const double> yv,
            Vec<double> ov, int64_t n, int per) {
  const int inst = blockIdx.x / per;
  if (inactive(B, inst)) return;
  const double* x = xv.at(inst);
  const double* y = yv.at(inst);
  double* out = ov.at(inst);
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)per * blockDim.x)
    out[i] = a * x[i] + b * y[i];
}

__global__ void __launch_bounds__(256)
    k_fill(Batch B, Vec<double> xv, double v, int64_t n, int per) {
  const int inst = blockIdx.x / per;
  if (inactive(B, inst)) return;
  double* x = xv.at(inst);
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)per * blockDim.x)
    x[i] = v;
}

__global__ void __launch_bounds__(256)
    k_residual_prep(Batch B, Vec<const double> uv, Vec<const double> unv, Vec<const double> wv,
                    Vec<const double> wnv, Vec<double> t1v, Vec<double> t2v, int64_t n, int per) {
  const int inst = blockIdx.x / per;
  if (inactive(B, inst)) return;
  const InstCoef& C = B.coef[inst];
  const double dt = C.dt, sigma = C.sigma, th = C.theta, m = C.m;
  const double* u = uv.at(inst);
  const double* un = unv.at(inst);
  const double* w = wv.at(inst);
  const double* wn = wnv.null() ? nullptr : wnv.at(inst);
  double* t1 = t1v.at(inst);
  double* t2 = t2v.at(inst);
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)per * blockDim.x) {
    double uu = u[i], uo = un[i], ww = w[i];
    double wo = wn ? wn[i] : ww;
    t1[i] = (uu - uo) + dt * sigma * (th * uu + (1.0 - th) * uo - m);
    t2[i] = dt * (th * ww + (1.0 - th) * wo);
  }
}

int vec_per(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

dim3 grid_of(int per, const Batch& B) { return dim3((unsigned)((int64_t)per * B.count)); }

}  // namespace

hipError_t launch_dot_partial(const Batch& B, Vec<const double> a, Vec<const double> b,
                              int64_t n, Vec<double> partials, hipStream_t st) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_dot, grid_of(nb, B), dim3(kRedThreads), 0, st, B, a, b, n, partials, nb);
  return hipGetLastError();
}

hipError_t launch_reduce_final(const Batch& B, Vec<const double> partials, int64_t n,
                               Vec<double> out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_final, dim3(B.count), dim3(256), 0, st, B, partials, red_blocks(n),
                     out);
  return hipGetLastError();
}

hipError_t launch_mgs_step(const Batch& B, Vec<double> w, Vec<const double> vi,
                           Vec<const double> vnext, int64_t n, Vec<const double> pin,
                           Vec<double> pout, Vec<double> Hij, hipStream_t st) {
  const int nb = red_blocks(n);
  if (vnext.null())
    hipLaunchKernelGGL(k_mgs<true>, grid_of(nb, B), dim3(kRedThreads), 0, st, B, w, vi, vnext, n,
                       pin, pout, Hij, nb);
  else
    hipLaunchKernelGGL(k_mgs<false>, grid_of(nb, B), dim3(kRedThreads), 0, st, B, w, vi, vnext, n,
                       pin, pout, Hij, nb);
  return hipGetLastError();
}

hipError_t launch_givens(const Batch& B, int* act, int j, int m, Vec<double> H, Vec<double> cs,
                         Vec<double> sn, Vec<double> g, Vec<const double> pnorm, int64_t n,
                         Vec<double> kr, hipStream_t st) {
  hipLaunchKernelGGL(k_givens, dim3(B.count), dim3(256), 0, st, B, act, j, m, H, cs, sn, g, pnorm,
                     red_blocks(n), kr);
  return hipGetLastError();
}

hipError_t launch_scale_by(const Batch& B, Vec<const double> w, Vec<double> v,
                           Vec<const double> kr, int64_t n, hipStream_t st) {
  const int per = vec_per(n);
  hipLaunchKernelGGL(k_scale_by, grid_of(per, B), dim3(256), 0, st, B, w, v, kr, n, per);
  return hipGetLastError();
}

hipError_t launch_scale_inv(const Batch& B, Vec<const double> b, Vec<double> v,
                            Vec<const double> nrm, int64_t n, hipStream_t st) {
  const int per = vec_per(n);
  hipLaunchKernelGGL(k_scale_inv, grid_of(per, B), dim3(256), 0, st, B, b, v, nrm, n, per);
  return hipGetLastError();
}

hipError_t launch_cycle_init(const Batch& B, int m, Vec<double> g, Vec<const double> nrm,
                             Vec<double> kr, hipStream_t st) {
  hipLaunchKernelGGL(k_cycle_init, dim3(B.count), dim3(64), 0, st, B, m, g, nrm, kr);
  return hipGetLastError();
}

template <class TZ>
hipError_t launch_lsq_update(const Batch& B, int m, Vec<const double> H, Vec<const double> g,
                             Vec<double> y, Vec<const double> kr, Vec<const TZ> Z,
                             int64_t zstride, Vec<double> x, int64_t n, hipStream_t st) {
  if (m > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lsq, dim3(B.count), dim3(64), 0, st, B, m, H, g, y, kr);
  const int per = vec_per(n);
  hipLaunchKernelGGL((k_update_x<TZ>), grid_of(per, B), dim3(256), 0, st, B,
                     Vec<const double>{y.p, y.s}, kr, Z, zstride, x, n, per);
  return hipGetLastError();
}

template <class TI, class TO>
hipError_t launch_copy_scale(const Batch& B, Vec<const TI> in, Vec<TO> out, double a, int64_t n,
                             hipStream_t st) {
  const int per = vec_per(n);
  hipLaunchKernelGGL((k_copy_scale<TI, TO>), grid_of(per, B), dim3(256), 0, st, B, in, out, a, n,
                     per);
  return hipGetLastError();
}

hipError_t launch_axpby(const Batch& B, double a, Vec<const double> x, double b,
                        Vec<const double> y, Vec<double> out, int64_t n, hipStream_t st) {
  const int per = vec_per(n);
  hipLaunchKernelGGL(k_axpby, grid_of(per, B), dim3(256), 0, st, B, a, x, b, y, out, n, per);
  return hipGetLastError();
}

hipError_t launch_fill(const Batch& B, Vec<double> x, double v, int64_t n, hipStream_t st) {
  const int per = vec_per(n);
  hipLaunchKernelGGL(k_fill, grid_of(per, B), dim3(256), 0, st, B, x, v, n, per);
  return hipGetLastError();
}

hipError_t launch_residual_prep(const Batch& B, Vec<const double> u, Vec<const double> un,
                                Vec<const double> w, Vec<const double> wn, Vec<double> t1,
                                Vec<double> t2, int64_t n, hipStream_t st) {
  const int per = vec_per(n);
  hipLaunchKernelGGL(k_residual_prep, grid_of(per, B), dim3(256), 0, st, B, u, un, w, wn, t1, t2,
                     n, per);
  return hipGetLastError();
}

template hipError_t launch_lsq_update<double>(const Batch&, int, Vec<const double>,
                                              Vec<const double>, Vec<double>, Vec<const double>,
                                              Vec<const double>, int64_t, Vec<double>, int64_t,
                                              hipStream_t);
template hipError_t launch_lsq_update<float>(const Batch&, int, Vec<const double>,
                                             Vec<const double>, Vec<double>, Vec<const double>,
                                             Vec<const float>, int64_t, Vec<double>, int64_t,
                                             hipStream_t);
template hipError_t launch_copy_scale<double, double>(const Batch&, Vec<const double>,
                                                      Vec<double>, double, int64_t, hipStream_t);
template hipError_t launch_copy_scale<double, float>(const Batch&, Vec<const double>, Vec<float>,
                                                     double, int64_t, hipStream_t);
template hipError_t launch_copy_scale<float, double>(const Batch&, Vec<const float>, Vec<double>,
                                                     double, int64_t, hipStream_t);

}  // namespace okd
