// Vector kernels of flexible GMRES (Saad 1993) with modified Gram-Schmidt and
// of preconditioned MINRES (Paige and Saunders 1975),
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
#include <array>
#include <cmath>
#include <utility>

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
// Blocks of at least 256 threads: each thread's (at most four) partials are
// loaded together, from clamped indices, before they are added in order.
__device__ __forceinline__ double sum_partials(const double* p, int nblk, double* sh) {
  constexpr int kPer = kMaxRedBlocks / 256;
  double t[kPer];
#pragma unroll
  for (int u = 0; u < kPer; u++) t[u] = p[min((int)threadIdx.x + (int)blockDim.x * u, nblk - 1)];
  double v = 0.0;
#pragma unroll
  for (int u = 0; u < kPer; u++)
    if ((int)threadIdx.x + (int)blockDim.x * u < nblk) v += t[u];
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
                         Vec<double> krv, Vec<double> scv) {
  __shared__ double sh[8];
  __shared__ double cst[64], snt[64], ct[65];  // rotations so far and the new column, staged
  const int inst = blockIdx.x;
  if (inactive(B, inst)) return;
  double* col = Hv.at(inst) + (int64_t)j * (m + 1);
  double* cs = csv.at(inst);
  double* sn = snv.at(inst);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    ct[i] = col[i];
    if (i < j) {
      cst[i] = cs[i];
      snt[i] = sn[i];
    }
  }
  double s = sum_partials(pnv.at(inst), nblk, sh);  // its barrier also publishes the staging
  if (threadIdx.x == 0) {
    double* g = gv.at(inst);
    double* kr = krv.at(inst);
    double hn = sqrt(s);
    // the earlier rotations applied to the new column: entry i+1 is untouched
    // until rotation i, so the chain carries one running value
    double cur = ct[0];
    for (int i = 0; i < j; i++) {
      const double nxt = ct[i + 1];
      const double t = cst[i] * cur + snt[i] * nxt;
      cur = -snt[i] * cur + cst[i] * nxt;
      ct[i] = t;
    }
    const double cj = cur, cj1 = hn;
    double den = hypot(cj, cj1);
    const double csj = cj / den, snj = cj1 / den;
    cs[j] = csj;
    sn[j] = snj;
    ct[j] = den;
    ct[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -snj * gj;
    g[j] = csj * gj;
    const double res = fabs(-snj * gj);
    kr[3] = res;
    kr[4] = hn;
    kr[5] = 1.0 / hn;
    kr[6] = (double)(j + 1);
    if (!scv.null()) scv.at(inst)[j + 1] = kr[5];  // v_{j+1} = w / h_{j+1,j}, kept unscaled
    if (!isfinite(hn) || !isfinite(res)) {
      kr[7] = 2.0;
      act[inst] = 0;
    } else if (res <= kr[1] || hn == 0.0) {
      kr[7] = 1.0;
      act[inst] = 0;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) col[i] = ct[i];
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
                             Vec<double> krv, Vec<double> scv) {
  const int inst = blockIdx.x;
  if (inactive(B, inst)) return;
  double* g = gv.at(inst);
  const double beta = nv.at(inst)[1];
  for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = (i == 0) ? beta : 0.0;
  if (!scv.null())
    for (int i = threadIdx.x; i <= m; i += blockDim.x) scv.at(inst)[i] = 1.0;
  if (threadIdx.x == 0) {
    double* kr = krv.at(inst);
    kr[2] = beta;
    kr[6] = 0.0;
    kr[7] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Arnoldi projection in two passes (modified Gram-Schmidt in inverse compact
// WY form; Swirydowicz, Langou, Ananthan, Yang, Thomas, "Low synchronization
// Gram-Schmidt and GMRES algorithms", Numer. Linear Algebra Appl. 2021).
// With V = [v_0..v_j] and L the strictly lower part of V^T V, modified
// Gram-Schmidt's coefficients satisfy (I + L) h = V^T w: h_i = <w, v_i> -
// sum_{k<i} <v_i, v_k> h_k, since each projection has already removed the
// earlier components.  So one pass forms every <w, v_i> and the new row
// <v_j, v_i> of L, a one-block kernel solves the triangular system, and one
// pass forms w - V h with the partials of its squared norm: 2j+5 vector
// passes per Arnoldi step instead of 4j+7.  Basis vectors are stored
// unnormalised, v_i = s_i V_i with s_i = 1/h_{i,i-1} (s_0 = 1), so no pass
// rescales the new vector; every reader applies s_i.
// ---------------------------------------------------------------------------

// Partials of a_i = <W, V_i> and c_i = <V_j, V_i> for i = i0 .. i0+NV-1:
// pd[(2i) * nblk + kb] and pd[(2i+1) * nblk + kb].  Element order as k_dot.
// JIN: V_j is the group's last vector (i0 + NV - 1 == j), so its loaded
// values serve as V_j and it is not streamed a second time.
template <int NV, bool JIN>
__global__ void __launch_bounds__(kRedThreads)
    k_proj_dots(Batch B, Vec<const double> wv, Vec<const double> Vv, int64_t vstride, int i0,
                int j, int64_t n, Vec<double> pdv, int nblk) {
  __shared__ double sh[kRedThreads / 64][2 * NV];
  const int inst = blockIdx.x / nblk, kb = blockIdx.x % nblk;
  if (inactive(B, inst)) return;
  const double* w = wv.at(inst);
  const double* V = Vv.at(inst);
  const double* vj = V + (int64_t)j * vstride;
  const double* vi[NV];
#pragma unroll
  for (int q = 0; q < NV; q++) vi[q] = V + (int64_t)(i0 + q) * vstride;
  double a[NV], c[NV];
#pragma unroll
  for (int q = 0; q < NV; q++) a[q] = c[q] = 0.0;
  for (int64_t e = (int64_t)kb * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)nblk * blockDim.x) {
    const double x = ldnt(w + e);
    double v[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) v[q] = ldnt(vi[q] + e);
    const double y = JIN ? v[NV - 1] : ldnt(vj + e);
#pragma unroll
    for (int q = 0; q < NV; q++) {
      a[q] = fma(x, v[q], a[q]);
      c[q] = fma(y, v[q], c[q]);
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; q++) {
    double s = a[q], t = c[q];
    for (int o = 32; o > 0; o >>= 1) {
      s += __shfl_xor(s, o);
      t += __shfl_xor(t, o);
    }
    if (lane == 0) {
      sh[wave][2 * q] = s;
      sh[wave][2 * q + 1] = t;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < 2 * NV) {
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) s += sh[k][threadIdx.x];
    pdv.at(inst)[(int64_t)(2 * i0 + threadIdx.x) * nblk + kb] = s;
  }
}

// One block per instance: sum the partials (wave q%8 sums row q, a fixed
// order), scale by s_i (and s_j), store row j of L, solve (I + L) h = a by
// forward substitution, write column j of H and the update coefficients
// hc_i = h_i s_i of the stored vectors.
__global__ void __launch_bounds__(512)
    k_proj_coef(Batch B, int j, int m, Vec<const double> pdv, int nblk, Vec<const double> scv,
                Vec<double> Lv, Vec<double> Hv, Vec<double> hcv) {
  __shared__ double sums[2 * 64];
  __shared__ double scs[64];
  __shared__ double Ls[64][65];  // rows 0 .. j-1 of L, staged (padded: no bank conflicts)
  const int inst = blockIdx.x;
  if (inactive(B, inst)) return;
  const double* pd = pdv.at(inst);
  const double* sc = scv.at(inst);
  double* L = Lv.at(inst);  // row-major (m+1) x (m+1): L[i*(m+1)+k] = <v_i, v_k>, k < i
  const int ld = m + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int nq = 2 * (j + 1);
  // each lane sums partials lane, lane + 64, ... of a row in that order; the
  // loads of two rows (clamped, unconditional) are all issued before the sums
  constexpr int kPer = kMaxRedBlocks / 64;
  for (int q0 = wave; q0 < nq; q0 += 2 * nw) {
    double v[2][kPer];
#pragma unroll
    for (int r = 0; r < 2; r++) {
      const int q = min(q0 + r * nw, nq - 1);
#pragma unroll
      for (int u = 0; u < kPer; u++)
        v[r][u] = pd[(int64_t)q * nblk + min(lane + 64 * u, nblk - 1)];
    }
#pragma unroll
    for (int r = 0; r < 2; r++) {
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < kPer; u++)
        if (lane + 64 * u < nblk) s += v[r][u];
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      const int q = q0 + r * nw;
      if (lane == 0 && q < nq) sums[q] = s;
    }
  }
  // the rows of L from earlier steps and the scales, all loads in flight at once
  for (int t = threadIdx.x; t < j * j; t += blockDim.x) {
    const int i = t / j, k = t - i * j;
    if (k < i) Ls[i][k] = L[(int64_t)i * ld + k];
  }
  if ((int)threadIdx.x <= j) scs[threadIdx.x] = sc[threadIdx.x];
  __syncthreads();
  if (wave != 0) return;
  // wavefront 0: lane i owns row i.  New row j of L, then forward
  // substitution h_i = <w, v_i> sc_i - sum_{k<i} L_ik h_k with k ascending
  // (each lane's sum in the order of a row-by-row solve): after step k, lane
  // k's value is final and is broadcast to the lanes below it.
  const double sj = scs[j];
  const bool own = lane <= j;
  if (lane < j) {
    const double ljl = sums[2 * lane + 1] * scs[lane] * sj;
    L[(int64_t)j * ld + lane] = ljl;
  }
  double h = own ? sums[2 * lane] * scs[min(lane, j)] : 0.0;
  for (int k = 0; k < j; k++) {
    const double hk = __shfl(h, k);
    if (lane > k && own) {
      const double lik = (lane == j) ? sums[2 * k + 1] * scs[k] * sj : Ls[lane][k];
      h = fma(-lik, hk, h);
    }
  }
  if (own) {
    Hv.at(inst)[lane] = h;
    hcv.at(inst)[lane] = h * scs[lane];
  }
}

// w -= sum_i hc_i V_i (i = 0 .. j) and the partials of <w, w>.  Element order
// as k_dot.
__global__ void __launch_bounds__(kRedThreads)
    k_proj_update(Batch B, Vec<double> wv, Vec<const double> Vv, int64_t vstride, int j,
                  int64_t n, Vec<const double> hcv, Vec<double> pv, int nblk) {
  __shared__ double sh[kRedThreads / 64];
  __shared__ double hs[64];
  const int inst = blockIdx.x / nblk, kb = blockIdx.x % nblk;
  if (inactive(B, inst)) return;
  if ((int)threadIdx.x <= j) hs[threadIdx.x] = hcv.at(inst)[threadIdx.x];
  __syncthreads();
  double* w = wv.at(inst);
  const double* V = Vv.at(inst);
  double acc = 0.0;
  for (int64_t e = (int64_t)kb * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)nblk * blockDim.x) {
    double x = ldnt(w + e);
    int i = 0;
    for (; i + 4 <= j + 1; i += 4) {  // four loads in flight per trip
      const double v0 = ldnt(V + (int64_t)i * vstride + e);
      const double v1 = ldnt(V + (int64_t)(i + 1) * vstride + e);
      const double v2 = ldnt(V + (int64_t)(i + 2) * vstride + e);
      const double v3 = ldnt(V + (int64_t)(i + 3) * vstride + e);
      x = fma(-hs[i], v0, x);
      x = fma(-hs[i + 1], v1, x);
      x = fma(-hs[i + 2], v2, x);
      x = fma(-hs[i + 3], v3, x);
    }
    for (; i <= j; i++) x = fma(-hs[i], ldnt(V + (int64_t)i * vstride + e), x);
    stnt(x, w + e);
    acc = fma(x, x, acc);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) pv.at(inst)[kb] = acc;
}

// Back substitution with the triangular H (column-major, leading dim m+1).
__global__ void k_lsq(Batch B, int m, Vec<const double> Hv, Vec<const double> gv, Vec<double> yv,
                      Vec<const double> krv) {
  __shared__ double Hs[64][65];  // upper triangle, Hs[l][i] = H_il (padded: no bank conflicts)
  __shared__ double gs[64], ys[64];
  const int inst = blockIdx.x;
  if (inactive(B, inst)) return;
  const double* H = Hv.at(inst);
  const double* g = gv.at(inst);
  double* y = yv.at(inst);
  const int k = (int)krv.at(inst)[6];
  const int ldh = m + 1;
  // stage the triangle (all loads in flight at once), then solve from LDS
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
    const int l = t / k, i = t - l * k;
    if (i <= l) Hs[l][i] = H[(int64_t)l * ldh + i];
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) gs[i] = g[i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; i--) {
    double s = gs[i];
    for (int l = i + 1; l < k; l++) s -= Hs[l][i] * ys[l];
    ys[i] = s / Hs[i][i];
  }
  for (int i = 0; i < k; i++) y[i] = ys[i];
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
  // the directions are streamed once (nontemporal), four loads in flight
  // per trip; the sum runs over j in order
  auto ldz = [](const TZ* p) { return (double)__builtin_nontemporal_load(p); };
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)per * blockDim.x) {
    double s = x[i];
    int j = 0;
    for (; j + 4 <= k; j += 4) {
      const double z0 = ldz(Z + j * zstride + i), z1 = ldz(Z + (j + 1) * zstride + i);
      const double z2 = ldz(Z + (j + 2) * zstride + i), z3 = ldz(Z + (j + 3) * zstride + i);
      s += ys[j] * z0;
      s += ys[j + 1] * z1;
      s += ys[j + 2] * z2;
      s += ys[j + 3] * z3;
    }
    for (; j < k; j++) s += ys[j] * ldz(Z + j * zstride + i);
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

// ---------------------------------------------------------------------------
// Preconditioned MINRES (Elman, Silvester and Wathen, Alg. 4.1) on the
// symmetric rearranged Newton system.  The reductions follow k_dot's element
// order over the 2n entries of an instance.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
    k_mr_init(Batch B, Vec<const double> bv, Vec<double> v1v, Vec<double> v0v, Vec<double> w0v,
              Vec<double> w1v, Vec<double> xv, int64_t n, int scale_first, int per) {
  const int inst = blockIdx.x / per;
  if (inactive(B, inst)) return;
  const double s = scale_first ? B.coef[inst].inv_sA : 1.0;
  const double* b = bv.at(inst);
  double *v1 = v1v.at(inst), *v0 = v0v.at(inst), *w0 = w0v.at(inst), *w1 = w1v.at(inst);
  double* x = xv.at(inst);
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < 2 * n;
       i += (int64_t)per * blockDim.x) {
    v1[i] = i < n ? s * b[i] : b[i];
    v0[i] = 0.0;
    w0[i] = 0.0;
    w1[i] = 0.0;
    x[i] = 0.0;
  }
}

__global__ void __launch_bounds__(kRedThreads)
    k_mr_scale_dot(Batch B, Vec<double> zv, Vec<const double> vv, int64_t n, Vec<double> pv,
                   int nblk) {
  __shared__ double sh[kRedThreads / 64];
  const int inst = blockIdx.x / nblk, kb = blockIdx.x % nblk;
  if (inactive(B, inst)) return;
  const InstCoef& C = B.coef[inst];
  const double f1 = C.alpha / C.c, f2 = C.c / C.alpha;
  double* z = zv.at(inst);
  const double* v = vv.at(inst);
  double acc = 0.0;
  for (int64_t i = (int64_t)kb * blockDim.x + threadIdx.x; i < 2 * n;
       i += (int64_t)nblk * blockDim.x) {
    const double zi = ldnt(z + i) * (i < n ? f1 : f2);
    stnt(zi, z + i);
    acc = fma(zi, ldnt(v + i), acc);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) pv.at(inst)[kb] = acc;
}

__global__ void __launch_bounds__(256)
    k_mr_start(Batch B, int* act, Vec<const double> pv, int nblk, Vec<double> mrv) {
  __shared__ double sh[8];
  const int inst = blockIdx.x;
  if (inactive(B, inst)) {
    if (threadIdx.x == 0) act[inst] = 0;
    return;
  }
  const double s = sum_partials(pv.at(inst), nblk, sh);
  if (threadIdx.x != 0) return;
  double* mr = mrv.at(inst);
  const double g1 = sqrt(s);
  for (int k = 0; k < MR_COUNT; k++) mr[k] = 0.0;
  mr[MR_GAM0] = 1.0;
  mr[MR_GAM] = g1;
  mr[MR_ETA] = g1;
  mr[MR_C0] = 1.0;
  mr[MR_C] = 1.0;
  mr[MR_TOL] = B.coef[inst].rtol * g1;
  mr[MR_GAM1] = g1;
  int a = 1;
  if (!isfinite(g1)) {
    mr[MR_STATUS] = 2.0;
    a = 0;
  } else if (g1 == 0.0) {
    mr[MR_STATUS] = 1.0;
    a = 0;
  }
  act[inst] = a;
}

__global__ void __launch_bounds__(kRedThreads)
    k_mr_vupd(Batch B, Vec<const double> pv, Vec<const double> azv, Vec<const double> v1v,
              Vec<const double> v0v, Vec<double> v2v, int64_t n2, Vec<double> mrv, int nblk) {
  __shared__ double sh[kRedThreads / 64];
  const int inst = blockIdx.x / nblk, kb = blockIdx.x % nblk;
  if (inactive(B, inst)) return;
  double* mr = mrv.at(inst);
  const double gam = mr[MR_GAM], gam0 = mr[MR_GAM0];
  const double delta = sum_partials(pv.at(inst), nblk, sh) / (gam * gam);
  if (kb == 0 && threadIdx.x == 0) mr[MR_DELTA] = delta;
  const double ca = 1.0 / gam, c1 = -delta / gam, c0 = -gam / gam0;
  const double* az = azv.at(inst);
  const double* v1 = v1v.at(inst);
  const double* v0 = v0v.at(inst);
  double* v2 = v2v.at(inst);
  for (int64_t i = (int64_t)kb * blockDim.x + threadIdx.x; i < n2;
       i += (int64_t)nblk * blockDim.x)
    stnt(fma(c0, ldnt(v0 + i), fma(c1, ldnt(v1 + i), ca * ldnt(az + i))), v2 + i);
}

__global__ void __launch_bounds__(256)
    k_mr_coef(Batch B, int* act, int* ran, Vec<const double> pv, int nblk, int maxit,
              Vec<double> mrv) {
  __shared__ double sh[8];
  const int inst = blockIdx.x;
  if (inactive(B, inst) || !act[inst]) {
    if (threadIdx.x == 0) ran[inst] = 0;
    return;
  }
  const double s2 = sum_partials(pv.at(inst), nblk, sh);
  if (threadIdx.x != 0) return;
  ran[inst] = 1;
  double* mr = mrv.at(inst);
  const double gnew = sqrt(s2);
  const double gam = mr[MR_GAM], delta = mr[MR_DELTA];
  const double s = mr[MR_S], s0 = mr[MR_S0], cc = mr[MR_C], c0 = mr[MR_C0];
  // QR step of the Lanczos tridiagonal matrix: rotate the new column with
  // the last two rotations, then build the rotation that removes gamma_{j+1}
  const double a0 = cc * delta - c0 * s * gam;
  const double a1 = sqrt(a0 * a0 + gnew * gnew);
  const double a2 = s * delta + c0 * cc * gam;
  const double a3 = s0 * gam;
  const double cn = a0 / a1, sn = gnew / a1;
  const double eta = mr[MR_ETA];
  mr[MR_WZ] = 1.0 / (gam * a1);
  mr[MR_W0] = -a3 / a1;
  mr[MR_W1] = -a2 / a1;
  mr[MR_XCP] = mr[MR_XC];
  mr[MR_XC] = cn * eta;
  const double en = -sn * eta;
  mr[MR_ETA] = en;
  const double its = mr[MR_ITS] + 1.0;
  mr[MR_ITS] = its;
  mr[MR_GAM0] = gam;
  mr[MR_GAM] = gnew;
  mr[MR_C0] = cc;
  mr[MR_C] = cn;
  mr[MR_S0] = s;
  mr[MR_S] = sn;
  if (!isfinite(en) || !isfinite(gnew)) {
    mr[MR_STATUS] = 2.0;
    act[inst] = 0;
  } else if (fabs(en) <= mr[MR_TOL] || gnew == 0.0) {
    mr[MR_STATUS] = 1.0;
    act[inst] = 0;
  } else if (its >= (double)maxit) {
    mr[MR_STATUS] = 3.0;
    act[inst] = 0;
  }
}

__global__ void __launch_bounds__(256)
    k_mr_wx(Batch B, const int* act, Vec<const double> zv, Vec<const double> w0v,
            Vec<const double> w1v, Vec<double> w2v, Vec<double> xv, int64_t n, int swap,
            Vec<const double> mrv, int per) {
  const int inst = blockIdx.x / per;
  if (inactive(B, inst)) return;
  const double* mr = mrv.at(inst);
  const double cz = mr[MR_WZ], c0 = mr[MR_W0], c1 = mr[MR_W1], cx = mr[MR_XC];
  const double cxp = mr[MR_XCP];
  // x is updated in every second iteration with both directions (w_j, the
  // previous one, is read here anyway), and in the last one: the same fused
  // multiply-adds in the same order as one update per iteration, with one
  // pass over x per two iterations
  const int t = (int)mr[MR_ITS];  // iterations done, this one included
  const int mode = (t % 2 == 0) ? 2 : (act[inst] ? 0 : 1);
  const double* z = zv.at(inst);
  const double* w0 = w0v.at(inst);
  const double* w1 = w1v.at(inst);
  double* w2 = w2v.at(inst);
  double* x = xv.at(inst);
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < 2 * n;
       i += (int64_t)per * blockDim.x) {
    const double wp = ldnt(w1 + i);
    const double w = fma(c1, wp, fma(c0, ldnt(w0 + i), cz * ldnt(z + i)));
    stnt(w, w2 + i);
    if (mode == 0) continue;
    const int64_t k = swap ? (i < n ? i + n : i - n) : i;
    x[k] = (mode == 2) ? fma(cx, w, fma(cxp, wp, x[k])) : fma(cx, w, x[k]);
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
                         Vec<double> kr, Vec<double> sc, hipStream_t st) {
  hipLaunchKernelGGL(k_givens, dim3(B.count), dim3(256), 0, st, B, act, j, m, H, cs, sn, g, pnorm,
                     red_blocks(n), kr, sc);
  return hipGetLastError();
}

namespace {
template <int NV>
void launch_dots_nv(const Batch& B, Vec<const double> w, Vec<const double> V, int64_t vstride,
                    int i0, int j, int64_t n, Vec<double> pd, int nb, hipStream_t st) {
  if (i0 + NV - 1 == j)
    hipLaunchKernelGGL((k_proj_dots<NV, true>), dim3((unsigned)((int64_t)nb * B.count)),
                       dim3(kRedThreads), 0, st, B, w, V, vstride, i0, j, n, pd, nb);
  else
    hipLaunchKernelGGL((k_proj_dots<NV, false>), dim3((unsigned)((int64_t)nb * B.count)),
                       dim3(kRedThreads), 0, st, B, w, V, vstride, i0, j, n, pd, nb);
}
using DotsFn = void (*)(const Batch&, Vec<const double>, Vec<const double>, int64_t, int, int,
                        int64_t, Vec<double>, int, hipStream_t);
template <int... K>
constexpr std::array<DotsFn, sizeof...(K)> dots_table(std::integer_sequence<int, K...>) {
  return {&launch_dots_nv<K + 1>...};
}
}  // namespace

hipError_t launch_proj(const Batch& B, Vec<double> w, Vec<const double> V, int64_t vstride, int j,
                       int m, int64_t n, Vec<double> pd, Vec<const double> sc, Vec<double> L,
                       Vec<double> Hcol, Vec<double> hc, Vec<double> pnorm, hipStream_t st) {
  if (j < 0 || j >= m || m > 64) return hipErrorInvalidValue;
  static constexpr auto kDots = dots_table(std::make_integer_sequence<int, kProjGroup>{});
  const int nb = red_blocks(n);
  for (int i0 = 0; i0 <= j; i0 += kProjGroup) {
    const int nv = std::min(kProjGroup, j + 1 - i0);
    kDots[nv - 1](B, Vec<const double>{w.p, w.s}, V, vstride, i0, j, n, pd, nb, st);
  }
  hipLaunchKernelGGL(k_proj_coef, dim3(B.count), dim3(512), 0, st, B, j, m,
                     Vec<const double>{pd.p, pd.s}, nb, sc, L, Hcol, hc);
  hipLaunchKernelGGL(k_proj_update, dim3((unsigned)((int64_t)nb * B.count)), dim3(kRedThreads), 0,
                     st, B, w, V, vstride, j, n, Vec<const double>{hc.p, hc.s}, pnorm, nb);
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
                             Vec<double> kr, Vec<double> sc, hipStream_t st) {
  hipLaunchKernelGGL(k_cycle_init, dim3(B.count), dim3(64), 0, st, B, m, g, nrm, kr, sc);
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

hipError_t launch_mr_init(const Batch& B, Vec<const double> b, Vec<double> v1, Vec<double> v0,
                          Vec<double> w0, Vec<double> w1, Vec<double> x, int64_t n,
                          bool scale_first, hipStream_t st) {
  const int per = vec_per(2 * n);
  hipLaunchKernelGGL(k_mr_init, grid_of(per, B), dim3(256), 0, st, B, b, v1, v0, w0, w1, x, n,
                     scale_first ? 1 : 0, per);
  return hipGetLastError();
}

hipError_t launch_mr_scale_dot(const Batch& B, Vec<double> z, Vec<const double> v, int64_t n,
                               Vec<double> partials, hipStream_t st) {
  const int nb = red_blocks(2 * n);
  hipLaunchKernelGGL(k_mr_scale_dot, grid_of(nb, B), dim3(kRedThreads), 0, st, B, z, v, n,
                     partials, nb);
  return hipGetLastError();
}

hipError_t launch_mr_start(const Batch& B, int* act, Vec<const double> partials, int64_t n2,
                           Vec<double> mr, hipStream_t st) {
  hipLaunchKernelGGL(k_mr_start, dim3(B.count), dim3(256), 0, st, B, act, partials,
                     red_blocks(n2), mr);
  return hipGetLastError();
}

hipError_t launch_mr_vupd(const Batch& B, Vec<const double> partials, Vec<const double> az,
                          Vec<const double> v1, Vec<const double> v0, Vec<double> v2, int64_t n2,
                          Vec<double> mr, hipStream_t st) {
  const int nb = red_blocks(n2);
  hipLaunchKernelGGL(k_mr_vupd, grid_of(nb, B), dim3(kRedThreads), 0, st, B, partials, az, v1, v0,
                     v2, n2, mr, nb);
  return hipGetLastError();
}

hipError_t launch_mr_coef(const Batch& B, int* act, int* ran, Vec<const double> partials,
                          int64_t n2, int maxit, Vec<double> mr, hipStream_t st) {
  hipLaunchKernelGGL(k_mr_coef, dim3(B.count), dim3(256), 0, st, B, act, ran, partials,
                     red_blocks(n2), maxit, mr);
  return hipGetLastError();
}

hipError_t launch_mr_wx(const Batch& B, const int* act, Vec<const double> z,
                        Vec<const double> w0, Vec<const double> w1, Vec<double> w2,
                        Vec<double> x, int64_t n, bool swap, Vec<const double> mr,
                        hipStream_t st) {
  const int per = vec_per(2 * n);
  hipLaunchKernelGGL(k_mr_wx, grid_of(per, B), dim3(256), 0, st, B, act, z, w0, w1, w2, x, n,
                     swap ? 1 : 0, mr, per);
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
