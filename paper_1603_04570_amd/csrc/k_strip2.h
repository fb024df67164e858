// Fused two-stage streaming kernels of the 3D node stencils on overlapping
// in-plane windows, one column strip of P nodes per thread.  Included by
// k_stencil_impl.h (inside namespace okd), after the one-iteration and fused
// kernels whose arithmetic it repeats.
//
// A block owns a BX x BY window of every x-y plane of its z-range.  Windows
// overlap by two nodes: only the (BX-2) x (BY-2) interior of a window is
// output, and the window origin of tile (tx, ty) is (tx (BX-2) - 1,
// ty (BY-2) - 1).  Thread t owns column cx = t % BX and rows cy0 .. cy0+P-1,
// cy0 = (t / BX) P, of the window, in both stages: stage 1 (the first
// Chebyshev iteration) runs on the whole window, stage 2 (the second, or the
// residual) on the interior nodes, which need stage 1 on their one-node
// ring.  So
//   * what stage 2 needs from stage 1 at a node stays in the thread's
//     registers (the tiled kernels pass it through LDS);
//   * the x-row partials of M1 and K1 along the thread's column are formed
//     once for the P+2 rows it touches and shared by its P nodes, whose
//     y-combinations only add them (the tiled kernels form 3 rows per node);
//   * the boundary masks and pattern coefficients of a node are constants of
//     the thread for the whole stream; per plane only the z pattern changes.
// LDS holds the input plane on the window plus a one-node ring (LA; nodes
// outside the grid +0) and the stage-1 field on the window with a +0 ring
// (LB).  Each node's arithmetic is that of the one-iteration kernels (same
// expressions, same rounding points, neighbours outside the grid +0 instead
// of masked, as in the tiled kernels), so results are bitwise those of the
// single steps, of k_cheb2/k_cheb2t and of k_mg2/k_mg2t.
//
// Modes: kStripCheb (two middle Chebyshev iterations k, k+1 on M, as
// k_cheb2t), kStripPre (pre-smoothing from x = 0 plus the residual, as
// k_mg2t<PRE>), kStripPost (post-smoothing from a given x, as
// k_mg2t<POST>), kStripPostProlong (post-smoothing from x + P e with the
// coarse-grid correction e interpolated while x is staged: the bits of
// k_prolong_add followed by kStripPost, without the pass over x between).
#pragma once

constexpr int kStripCheb = 0, kStripPre = 1, kStripPost = 2, kStripPostProlong = 3;

// Window configurations, selected by the `items` field of a shape-table entry.
struct StripCfg {
  int bx, by, p, nt;
};
__host__ __device__ constexpr StripCfg strip_cfg(int id) {
  return id == 1   ? StripCfg{32, 32, 4, 256}
         : id == 2 ? StripCfg{32, 16, 2, 256}
         : id == 3 ? StripCfg{64, 16, 4, 256}
         : id == 4 ? StripCfg{32, 24, 3, 256}
                   : StripCfg{64, 12, 3, 256};
}
constexpr int kStripCfgs = 5;
// Strips of 3 nodes are compiled for three wavefronts per SIMD (at most 168
// VGPRs; the stiffness variants then spill a few values), the others for the
// compiler's own choice (two wavefronts per SIMD at 4 nodes per thread).
constexpr int strip_min_waves(int p, int mode) {
  return p == 3 ? 3 : (mode == kStripPostProlong ? 2 : 1);
}

template <int BX, int BY, int P, class T, int MODE, bool LAST2>
__global__ void __launch_bounds__(BX * BY / P)
    __attribute__((amdgpu_waves_per_eu(strip_min_waves(P, MODE), 8)))
    k_strip2(Grid g, StencilShape sh, int ntx, Batch B, int lev, int kk, int osc,
             Vec<const T> av, Vec<const T> pv, Vec<T> xv, Vec<T> o2v, Vec<T> o3v,
             Vec<const T> ecv) {
  constexpr int NT = BX * BY / P;
  constexpr int WA = BX + 2;                        // LDS row pitch (window + ring)
  constexpr int EA = WA * (BY + 2);                 // LDS words per plane buffer
  constexpr int KA = (EA + NT - 1) / NT;            // staging slots per thread
  constexpr bool MASS = (MODE == kStripCheb);       // operator M only
  constexpr bool SC1 = (MODE == kStripPre);         // stage 1 on the W^-1-scaled input
  constexpr bool PROL = (MODE == kStripPostProlong);
  // prolongation: the coarse nodes under the window (CW x CH per coarse
  // plane, two coarse planes in LDS) and the coarse staging slots per thread
  constexpr int CW = BX / 2 + 3, CH = BY / 2 + 3, CE = CW * CH;
  constexpr int KC = PROL ? (CE + NT - 1) / NT : 0;
  extern __shared__ double lds_raw[];
  double* LA = lds_raw;
  double* LB = lds_raw + EA;
  double* LC = lds_raw + 2 * EA;  // PROL: two coarse planes, plane K in buffer K & 1
  const int tid = threadIdx.x;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int inst = lb / sh.blocks;
  if (B.act && !B.act[inst]) return;
  const int b = lb - inst * sh.blocks;
  const int tile = b % sh.nchunks;
  const int zch = b / sh.nchunks;
  const InstCoef& IC = B.coef[inst];
  const OpK k1 = MODE == kStripCheb ? op_k(IC, -1, kk, CF_ONE)
                                    : (MODE == kStripPre ? op_k(IC, lev, 0, CF_ONE)
                                                         : op_k(IC, lev, -1, CF_ONE));
  const OpK k2 = MODE == kStripCheb ? op_k(IC, -1, kk + 1, osc)
                                    : (MODE == kStripPre ? op_k(IC, lev, -1, CF_ONE)
                                                         : op_k(IC, lev, 0, CF_ONE));
  const int nn = g.nn, N = g.N;
  const int64_t plane = g.plane;
  const int X0 = (tile % ntx) * (BX - 2) - 1, Y0 = (tile / ntx) * (BY - 2) - 1;
  const T* __restrict__ a = av.at(inst);
  const T* __restrict__ pw = (MODE == kStripPre) ? nullptr : pv.at(inst);
  T* __restrict__ xo = xv.at(inst);
  T* __restrict__ o2 = (MODE == kStripPost || PROL || (MODE == kStripCheb && LAST2))
                           ? nullptr
                           : o2v.at(inst);
  T* __restrict__ o3 = (MODE == kStripCheb && !LAST2) ? o3v.at(inst) : nullptr;

  // zero the stage-1 buffer once (its ring is never written; the barrier
  // after the first trip's staging orders this before any stage-1 write)
  for (int t = tid; t < EA; t += NT) LB[t] = 0.0;

  // input staging: slot t = tid + NT k holds window node (t % WA - 1, t / WA - 1)
  int oa[KA];       // in-plane offset of that node, clamped into the grid
  unsigned va = 0;  // bit k: the node lies in the grid (else the slot holds +0)
  // pre-smoothing stages its input scaled by 2^(boundary coordinates of the
  // node), an exact power of two: the unscaled stencil of the scaled input is
  // then, rounding for rounding, the W^-1-scaled stencil of the input
  double fsl[KA];
#pragma unroll
  for (int k = 0; k < KA; k++) {
    const int t = tid + NT * k;
    const int gy = Y0 - 1 + t / WA, gx = X0 - 1 + t % WA;
    if (t < EA && gy >= 0 && gy <= N && gx >= 0 && gx <= N) va |= 1u << k;
    oa[k] = min(max(gy, 0), N) * nn + min(max(gx, 0), N);
    fsl[k] = (double)(1 << ((gx == 0 || gx == N) + (gy == 0 || gy == N)));
  }
  // prolongation of the staged nodes (the coarse grid has N/2 elements):
  // coarse window origin; a fine node at an even index copies its coarse
  // node, at an odd one averages two
  const int Nc = N >> 1, nnc = Nc + 1;
  const int CI0 = (X0 - 1) >> 1, CJ0 = (Y0 - 1) >> 1;
  const T* __restrict__ ec = PROL ? ecv.at(inst) : nullptr;
  auto stage_coarse = [&](int kc, T (&cv)[KC > 0 ? KC : 1]) {  // load coarse plane kc
#pragma unroll
    for (int k2 = 0; k2 < KC; k2++) {
      const int j = tid + NT * k2;
      const int gj = min(max(CJ0 + j / CW, 0), Nc), gi = min(max(CI0 + j % CW, 0), Nc);
      cv[k2] = ec[((int64_t)kc * nnc + gj) * nnc + gi];
    }
  };
  auto commit_coarse = [&](int kc, const T (&cv)[KC > 0 ? KC : 1]) {
#pragma unroll
    for (int k2 = 0; k2 < KC; k2++) {
      const int j = tid + NT * k2;
      if (j < CE) LC[(kc & 1) * CE + j] = to_d(cv[k2]);
    }
  };
  // each slot's coarse offset and odd-index bits, 16 bits per slot: offset
  // in bits 0-8, odd x in bit 9, odd y in bit 10
  static_assert(!PROL || CE <= 512, "coarse window offsets take 9 bits");
  constexpr int KW = (KA + 1) / 2;
  unsigned pinfo[PROL ? KW : 1] = {};
  if constexpr (PROL) {
#pragma unroll
    for (int k = 0; k < KA; k++) {
      const int t = tid + NT * k;
      const int gy = Y0 - 1 + t / WA, gx = X0 - 1 + t % WA;
      const unsigned cl = (unsigned)(((gy >> 1) - CJ0) * CW + ((gx >> 1) - CI0));
      const unsigned v = (t < EA) ? (cl | (unsigned)(gx & 1) << 9 | (unsigned)(gy & 1) << 10) : 0u;
      pinfo[k >> 1] |= v << (16 * (k & 1));
    }
  }
  // P e at staging slot k of fine plane pz, summed in the order of
  // k_prolong_add (coarse plane, then row, then the one or two columns).
  // Every weight product is the exact power of two 2^-(number of odd
  // indices); the terms an even index does not have are added with weight 0
  // (reading a neighbour inside the staged window: finite, so each adds a
  // zero), which keeps the lanes of a wavefront on one path.
  auto prolong = [&](int k, int pz, const unsigned (&pi)[PROL ? KW : 1]) {
    const unsigned inf = (pi[k >> 1] >> (16 * (k & 1))) & 0xffffu;
    const int cl = (int)(inf & 511u);
    const bool two_i = inf & 512u, two_j = inf & 1024u;
    const int K = pz >> 1;
    const bool two_k = pz & 1;
    const int hi = (1023 - (int)two_k - (int)two_i - (int)two_j) << 20;
    const double w = __hiloint2double(hi, 0);
    const double wi = __hiloint2double(two_i ? hi : 0, 0);
    const double wj = __hiloint2double(two_j ? hi : 0, 0);
    const double wij = __hiloint2double((two_i && two_j) ? hi : 0, 0);
    double sum = 0.0;
#pragma unroll
    for (int za = 0; za < 2; za++) {
      if (za && !two_k) break;
      const double* cr = LC + ((K + za) & 1) * CE + cl;
      sum += w * cr[0];
      sum += wi * cr[1];
      sum += wj * cr[CW];
      sum += wij * cr[CW + 1];
    }
    return sum;
  };

  // the thread's strip
  const int cx = tid % BX, cy0 = (tid / BX) * P;
  const int gx = X0 + cx, ic = min(max(gx, 0), N);
  const bool xin = gx >= 0 && gx <= N;
  const bool ex = (ic == 0 || ic == N);
  const bool xout = cx >= 1 && cx <= BX - 2 && xin;
  bool in[P], out[P];
  bool ey[P];
  int off[P];      // in-plane offset of node p (clamped)
  int nbxy[P];     // boundary coordinates of node p in the plane
  double dvxy[P];  // stage-1 D^-1 without the z factor: dinv 2^nbxy (exact)
#pragma unroll
  for (int p = 0; p < P; p++) {
    const int cy = cy0 + p, gy = Y0 + cy, jc = min(max(gy, 0), N);
    in[p] = xin && gy >= 0 && gy <= N;
    out[p] = in[p] && xout && cy >= 1 && cy <= BY - 2;
    ey[p] = (jc == 0 || jc == N);
    off[p] = jc * nn + ic;
    nbxy[p] = (int)ex + (int)ey[p];
    dvxy[p] = dinv_at(k1.dinv, nbxy[p]);
  }

  // in-plane partials of the P nodes of the strip from buffer v (pitch WA;
  // row r of the strip's column is v[(cy0 + r) * WA + cx + 0..2], r = 0..P+1):
  // the arithmetic of mk_partials with +0 outside the grid
  auto partials = [&](const double* v, double (&pm)[P], double (&pk)[P], double (&cen)[P]) {
    double mr[P + 2], kr[P + 2];
#pragma unroll
    for (int r = 0; r < P + 2; r++) {
      const double* row = v + (cy0 + r) * WA + cx;
      const double l = row[0], c = row[1], rr = row[2];
      if (r >= 1 && r <= P) cen[r - 1] = c;
      mr[r] = m1_row(true, true, ex, l, c, rr);
      kr[r] = MASS ? 0.0 : k1_row(true, true, ex, l, c, rr);
    }
#pragma unroll
    for (int p = 0; p < P; p++) {
      pm[p] = m1_row(true, true, ey[p], mr[p], mr[p + 1], mr[p + 2]);
      pk[p] = MASS ? 0.0
                   : m1_row(true, true, ey[p], kr[p], kr[p + 1], kr[p + 2]) +
                         k1_row(true, true, ey[p], mr[p], mr[p + 1], mr[p + 2]);
    }
  };
  const double h = g.h;
  const double cmass = h * h * h / 216.0;
  const double cstiff = h / 36.0;
  // z-combination of the partials of planes z-1, z, z+1 at a node: the
  // expressions of the one-iteration kernels with the pattern of plane z;
  // inside the grid the pattern is [1, 4, 1] / [-1, 2, -1], and
  // sum3(1, 4, 1, a, b, n) = fma(4, b, a) + n, sum3(-1, 2, -1, a, b, n) =
  // fma(2, b, -a) - n exactly (the unit products are exact)
  auto zcomb = [&](bool zin, const double (&az)[3], const double (&bz)[3], double pa, double pb,
                   double pn, double qa, double qb, double qn, double& ms, double& ks) {
    if (zin) {
      ms = cmass * (fma(4.0, pb, pa) + pn);
      if (!MASS) ks = cstiff * ((fma(4.0, qb, qa) + qn) + (fma(2.0, pb, -pa) - pn));
    } else {
      ms = cmass * sum3(az[0], az[1], az[2], pa, pb, pn);
      if (!MASS)
        ks = cstiff * (sum3(az[0], az[1], az[2], qa, qb, qn) + sum3(bz[0], bz[1], bz[2], pa, pb, pn));
    }
  };

  int z0, z1;
  zrange(sh, nn, zch, z0, z1);
  const int zlast = min(z1 + 1, N);
  const int pl = (int)plane;  // a grid of one instance has fewer than 2^31 nodes
  // stage 1: partials of input planes pz-2, pz-1 and the input at pz-1
  double pa1[P], pb1[P], qa1[P], qb1[P], cb1[P];
  // stage 2: partials of stage-1 planes pz-3, pz-2 and the stage-1 field at pz-2
  double pa2[P], pb2[P], qa2[P], qb2[P], cb2[P];
  // what stage 2 of plane o needs from stage 1 of plane o (two planes in flight)
  double ca[P], cbv[P], na[P], nbv[P];
#pragma unroll
  for (int p = 0; p < P; p++) {
    pa1[p] = pb1[p] = qa1[p] = qb1[p] = cb1[p] = 0.0;
    pa2[p] = pb2[p] = qa2[p] = qb2[p] = cb2[p] = 0.0;
    ca[p] = cbv[p] = na[p] = nbv[p] = 0.0;
  }
  // prefetch registers (raw words from clamped, always in-bounds addresses)
  T pre_a[KA], pre_p[P], pre_x[P];
#pragma unroll
  for (int p = 0; p < P; p++) pre_p[p] = pre_x[p] = T(0);
  auto issue_a = [&](int z) {
    const int zo = z * pl;
#pragma unroll
    for (int k = 0; k < KA; k++) pre_a[k] = a[zo + oa[k]];
  };
  auto issue_p = [&](int zq, int zx) {
    if constexpr (MODE != kStripPre) {
      const int zo = zq * pl;
#pragma unroll
      for (int p = 0; p < P; p++) pre_p[p] = pw[zo + off[p]];
    }
    if constexpr (MODE == kStripCheb) {
      const int zo = zx * pl;
#pragma unroll
      for (int p = 0; p < P; p++) pre_x[p] = xo[zo + off[p]];
    }
  };
  issue_a(max(z0 - 2, 0));
  issue_p(max(z0 - 1, 0), max(z0, 0));
  T cpre[KC > 0 ? KC : 1];
  if constexpr (PROL) {
    // the coarse planes under the first staged plane (the barrier after the
    // first trip's staging is not enough: that staging reads them)
    const int K0 = max(z0 - 2, 0) >> 1;
    stage_coarse(K0, cpre);
    commit_coarse(K0, cpre);
    stage_coarse(min(K0 + 1, Nc), cpre);
    commit_coarse(K0 + 1, cpre);
    __syncthreads();
  }
  for (int pz = z0 - 2; pz <= z1 + 1; pz++) {
    const bool insideA = (pz >= 0 && pz <= N);
    const int q1 = pz - 1;  // stage-1 plane
    const int o = pz - 2;   // stage-2 (output) plane
    // no barrier before staging: every read of LA in the previous trip
    // precedes that trip's barrier before stage 2, and stage 2 reads only LB
    // PROL: coarse plane pz/2 + 1 is first read by trip pz + 1; loaded now,
    // stored after this trip's barrier (its buffer was last read by trip
    // pz - 1), visible after the barrier before stage 2
    const bool cstage = PROL && insideA && !(pz & 1) && (pz >> 1) + 1 <= Nc;
    if (cstage) stage_coarse((pz >> 1) + 1, cpre);
    if (insideA) {
      const double fz = (SC1 && (pz == 0 || pz == N)) ? 2.0 : 1.0;
      // the packed slot words made opaque per trip: unpacked here, not held
      // unpacked in registers across the plane loop
      unsigned pi[PROL ? KW : 1];
#pragma unroll
      for (int q = 0; q < (PROL ? KW : 1); q++) {
        pi[q] = pinfo[q];
        if constexpr (PROL) asm volatile("" : "+v"(pi[q]));
      }
#pragma unroll
      for (int k = 0; k < KA; k++) {
        const int t = tid + NT * k;
        double v = 0.0;
        if ((va >> k) & 1u) {
          if constexpr (PROL)
            v = to_d((T)(to_d(pre_a[k]) + prolong(k, pz, pi)));
          else
            v = to_d(pre_a[k]);
        }
        if (SC1) v = v * fsl[k] * fz;
        if (t < EA) LA[t] = v;
      }
    }
    __syncthreads();
    if (cstage) commit_coarse((pz >> 1) + 1, cpre);
    T pq[P], xq[P];  // stage-1 pointwise input of plane q1, stage-2 x of plane o
#pragma unroll
    for (int p = 0; p < P; p++) {
      pq[p] = pre_p[p];
      xq[p] = pre_x[p];
    }
    issue_a(max(min(pz + 1, zlast), 0));  // plane -1 is never read
    issue_p(min(max(q1 + 1, 0), N), min(max(o + 1, 0), N));
    // stage 1: partials of the input at plane pz on the strip
    double pn1[P], qn1[P], cn1[P];
    if (insideA) {
      partials(LA, pn1, qn1, cn1);
    } else {
#pragma unroll
      for (int p = 0; p < P; p++) pn1[p] = qn1[p] = cn1[p] = 0.0;
    }
    const bool s1 = (q1 >= z0 - 1 && q1 <= z1);
    if (s1) {
      const bool inq = (q1 >= 0 && q1 <= N);
      const bool zin = (q1 > 0 && q1 < N);
      double az[3] = {0, 0, 0}, bz[3] = {0, 0, 0};
      if (inq) pattern<false>(q1, N, az[0], az[1], az[2], bz[0], bz[1], bz[2]);
      const int nbz = (q1 == 0 || q1 == N);
      const double fz = nbz ? 2.0 : 1.0, fzi = nbz ? 0.5 : 1.0;
#pragma unroll
      for (int p = 0; p < P; p++) {
        double f1 = 0.0;
        na[p] = nbv[p] = 0.0;
        if (inq && in[p]) {
          double ms, ks = 0.0;
          zcomb(zin, az, bz, pa1[p], pb1[p], pn1[p], qa1[p], qb1[p], qn1[p], ms, ks);
          const double dv = dvxy[p] * fz;  // dinv_at(dinv, nbxy + nbz), exactly
          if constexpr (MODE == kStripCheb) {
            const double dk = cb1[p];
            const double ru = to_d(pq[p]) - op_apply(k1, ms, 0.0);
            na[p] = to_d((T)ru);
            nbv[p] = dk;
            f1 = to_d((T)cheb_dir(k1, dk, dv, ru));
          } else if constexpr (MODE == kStripPre) {
            // the staged input is b 2^nb: d0 = (dv b) it = (dinv (b 2^nb)) it
            const double bs = cb1[p];
            const double bi = bs * (fzi / (double)(1 << nbxy[p]));
            const double ad0 = k1.dinv * k1.it * op_apply(k1, ms, ks);
            const double d0 = k1.dinv * bs * k1.it;
            const double r1 = bi - ad0;
            const double d1 = cheb_dir(k1, d0, dv, r1);
            f1 = to_d((T)(k1.osc * (d0 + d1)));
            na[p] = bi;
          } else {
            const double r0 = to_d(pq[p]) - op_apply(k1, ms, ks);
            f1 = to_d((T)(dv * r0 * k1.it));
            na[p] = to_d((T)r0);
            nbv[p] = cb1[p];
          }
        }
        LB[(cy0 + p + 1) * WA + cx + 1] = f1;
      }
    }
#pragma unroll
    for (int p = 0; p < P; p++) {
      pa1[p] = pb1[p];
      pb1[p] = pn1[p];
      qa1[p] = qb1[p];
      qb1[p] = qn1[p];
      cb1[p] = cn1[p];
    }
    __syncthreads();
    // stage 2: partials of the stage-1 field at plane q1; finish plane o
    if (s1) {
      double pn2[P], qn2[P], cn2[P];
      partials(LB, pn2, qn2, cn2);
      if (o >= z0 && o < z1) {
        double az[3], bz[3];
        pattern<false>(o, N, az[0], az[1], az[2], bz[0], bz[1], bz[2]);
        const bool zin = (o > 0 && o < N);
        const double fz = (o == 0 || o == N) ? 2.0 : 1.0;
        const int zo = o * pl;
#pragma unroll
        for (int p = 0; p < P; p++) {
          if (!out[p]) continue;
          double ms, ks = 0.0;
          zcomb(zin, az, bz, pa2[p], pb2[p], pn2[p], qa2[p], qb2[p], qn2[p], ms, ks);
          const int idx = zo + off[p];
          if constexpr (MODE == kStripCheb) {
            const double d1 = cb2[p];
            const double rv1 = ca[p], dk = cbv[p];
            const double dv = dvxy[p] * fz;  // both iterations use M's diagonal
            const double xv1 = to_d((T)(to_d(xq[p]) + dk));
            const double xv2 = xv1 + d1;
            const double rv2 = rv1 - op_apply(k2, ms, 0.0);
            const double d2 = cheb_dir(k2, d1, dv, rv2);
            if (LAST2) {
              xo[idx] = (T)(k2.osc * (xv2 + d2));
            } else {
              xo[idx] = (T)xv2;
              o2[idx] = (T)rv2;
              o3[idx] = (T)d2;
            }
          } else if constexpr (MODE == kStripPre) {
            xo[idx] = (T)cb2[p];
            o2[idx] = (T)(ca[p] - op_apply(k2, ms, ks));
          } else {
            const double dk = cb2[p];
            const double dv = dvxy[p] * fz;  // both iterations on the same level
            const double xv = cbv[p] + dk;
            const double rv = ca[p] - op_apply(k2, ms, ks);
            const double d1 = cheb_dir(k2, dk, dv, rv);
            xo[idx] = (T)(k2.osc * (xv + d1));
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
        ca[p] = na[p];
        cbv[p] = nbv[p];
      }
    }
  }
}
