// Host engine: class layout, per-instance constants, and the lockstep solver
// operations.  Every vector operation runs in the kernels of this library;
// the host only sequences launches and reads back a few flags and norms.
#include "engine.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstring>

namespace okd {

void ClassExec::clear_graphs() {
  for (auto& g : iter)
    if (g) (void)hipGraphExecDestroy(g);
  iter.clear();
  key = nullptr;
}

ClassExec::~ClassExec() {
  clear_graphs();
  if (fork) (void)hipEventDestroy(fork);
  if (join) (void)hipEventDestroy(join);
  if (xs) (void)hipStreamDestroy(xs);
}

SideStream::~SideStream() {
  if (fork) (void)hipEventDestroy(fork);
  if (join) (void)hipEventDestroy(join);
  if (s) (void)hipStreamDestroy(s);
}

FlagPipe::~FlagPipe() {
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (h) (void)hipHostFree(h);
}

Prof::~Prof() {
  for (auto& e : ev) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
}

namespace {

int set_err(std::string* err, int code, const std::string& msg) {
  if (err) *err = msg;
  return code;
}

#define OKE(c, ...)                                                                          \
  do {                                                                                       \
    hipError_t e_ = (__VA_ARGS__);                                                           \
    if (e_ != hipSuccess)                                                                    \
      return set_err((c).err, OK_E_HIP,                                                      \
                     std::string(#__VA_ARGS__).substr(0, 60) + ": " + hipGetErrorString(e_)); \
  } while (0)

// HIP-event bracket around launches of one kernel class (see ok_profile_*).
struct ProfScope {
  Prof* p;
  ProfPair* pp = nullptr;
  hipStream_t st;
  ProfScope(const ClassCtx& c, int cls, double bytes, hipStream_t s, int count = 1)
      : p(c.prof), st(s) {
    if (!p || p->capturing || cls == OK_K_NONE) return;
    if (!((p->mask >> cls) & 1)) return;
    if (p->used == p->ev.size()) {
      ProfPair q{};
      (void)hipEventCreate(&q.a);
      (void)hipEventCreate(&q.b);
      p->ev.push_back(q);
    }
    pp = &p->ev[p->used++];
    pp->bytes = bytes;
    pp->count = count;
    pp->cls = cls;
    (void)hipEventRecord(pp->a, st);
  }
  ~ProfScope() {
    if (pp) (void)hipEventRecord(pp->b, st);
  }
};

// Bump allocator over a 256-byte aligned region (base == nullptr: size only).
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// D^-1 (M + alpha K) on the DCT-I mode with cosines c_d (multilinear in c).
double dct_lambda(const Grid& g, double alpha, const double* c) {
  double h = g.h, num = 1.0, sk = 0.0;
  for (int d = 0; d < g.dim; d++) num *= (h / 3.0) * (2.0 + c[d]);
  for (int d = 0; d < g.dim; d++) {
    double t = (2.0 / h) * (1.0 - c[d]);
    for (int e = 0; e < g.dim; e++)
      if (e != d) t *= (h / 3.0) * (2.0 + c[e]);
    sk += t;
  }
  double mi = 2.0 * h / 3.0;
  double den = std::pow(mi, g.dim) + alpha * g.dim * (2.0 / h) * std::pow(mi, g.dim - 1);
  return (num + alpha * sk) / den;
}

// Fill a LevelCoef: operator cm M + ck K on grid g with Chebyshev interval [lo, hi].
void level_coef(LevelCoef& L, const Grid& g, double cm, double ck, double lo, double hi) {
  double mi = 2.0 * g.h / 3.0, ki = 2.0 / g.h;
  double dm = 1.0, dk = g.dim * ki;
  for (int d = 0; d < g.dim; d++) dm *= mi;
  for (int d = 0; d < g.dim - 1; d++) dk *= mi;
  L.cm = cm;
  L.ck = ck;
  L.dinv = 1.0 / (cm * dm + ck * dk);
  // Saad, Alg. 12.1: theta, delta, sigma1; rho_0 = 1/sigma1,
  // rho_{k+1} = 1/(2 sigma1 - rho_k), c1 = rho_{k+1} rho_k, c2 = 2 rho_{k+1}/delta.
  double th = 0.5 * (hi + lo), de = 0.5 * (hi - lo), s1 = th / de;
  L.it = 1.0 / th;
  double rho = 1.0 / s1;
  for (int k = 0; k < kMaxCheb; k++) {
    double rho1 = 1.0 / (2.0 * s1 - rho);
    L.c1[k] = rho1 * rho;
    L.c2[k] = 2.0 * rho1 / de;
    rho = rho1;
  }
}

// Smoother interval of D^-1 (M + alpha K): the largest eigenvalue (a corner of
// the cosine box) and the smallest over the upper half of the spectrum
// (vertices with some cosine in {-1, 0}); exact for Q1 on uniform grids.
void smoother_interval(const Grid& g, double alpha, double& lo, double& hi) {
  lo = 1e300;
  hi = -1e300;
  int nv = 1;
  for (int d = 0; d < g.dim; d++) nv *= 3;
  for (int s = 0; s < nv; s++) {
    int t[3] = {s % 3, (s / 3) % 3, s / 9};
    double c[3];
    bool corner = true, high = false;
    for (int d = 0; d < g.dim; d++) {
      c[d] = t[d] == 0 ? -1.0 : (t[d] == 1 ? 0.0 : 1.0);
      if (t[d] == 1) corner = false;
      if (t[d] <= 1) high = true;
    }
    double l = dct_lambda(g, alpha, c);
    if (corner && l > hi) hi = l;
    if (high && l < lo) lo = l;
  }
}

void inst_coef(InstCoef& C, const ok_params& p, const Grid* lev, int L) {
  std::memset(&C, 0, sizeof(C));
  // Sec. 2: c = dt theta / (1 + dt theta sigma), S^ = M + eps sqrt(c) K.
  C.dth = p.dt * p.theta;
  C.sA = 1.0 + C.dth * p.sigma;
  C.inv_sA = 1.0 / C.sA;
  const double cc = C.dth / C.sA;
  C.c = cc;
  C.alpha = p.eps * std::sqrt(cc);
  C.e2 = p.eps * p.eps;
  C.dt = p.dt;
  C.sigma = p.sigma;
  C.theta = p.theta;
  C.m = p.m;
  C.rtol = p.gmres_rtol;
  C.atol = p.newton_atol;
  // D^-1 M has spectrum [2^-d, (3/2)^d].
  level_coef(C.mass, lev[0], 1.0, 0.0, std::pow(0.5, p.dim), std::pow(1.5, p.dim));
  for (int l = 0; l < L; l++) {
    double lo, hi;
    smoother_interval(lev[l], C.alpha, lo, hi);
    level_coef(C.lev[l], lev[l], 1.0, C.alpha, lo, hi);
  }
}

void carve(ClassCtx& c, char* base, bool with_state, size_t* total) {
  Carver cv{base};
  const int B = c.B, m = c.m;
  const int64_t n = c.n, n2 = 2 * n;
  const size_t ps = c.psz;
  c.coef = cv.take<InstCoef>(B);
  c.act = cv.take<int>(B);
  c.part = cv.take<int>(B);
  c.incyc = cv.take<int>(B);
  c.aux = cv.take<int>(B);
  c.vs = (n2 + 63) & ~(int64_t)63;
  c.V = cv.take<double>((size_t)B * c.nv * c.vs);
  c.Z = cv.take<char>((size_t)B * m * c.vs * ps);
  c.X = cv.take<double>((size_t)B * n2);
  c.Bv = cv.take<double>((size_t)B * n2);
  c.T1 = cv.take<double>((size_t)B * n2);
  c.un = cv.take<double>((size_t)B * n);
  c.wn = cv.take<double>((size_t)B * n);
  c.G = cv.take<double>((size_t)B * n);
  c.Q = cv.take<double>((size_t)B * n);
  c.su = with_state ? cv.take<double>((size_t)B * n) : nullptr;
  c.sw = with_state ? cv.take<double>((size_t)B * n) : nullptr;
  c.zt = c.mixed ? cv.take<char>((size_t)B * n2 * ps) : nullptr;
  c.cr = cv.take<char>((size_t)B * n * ps);
  c.cr2 = cv.take<char>((size_t)B * n * ps);
  c.rich = c.shape.schur_richardson > 1 ? cv.take<char>((size_t)B * 4 * n * ps) : nullptr;
  c.cda = cv.take<char>((size_t)B * n * ps);
  c.cdb = cv.take<char>((size_t)B * n * ps);
  c.yv = cv.take<char>((size_t)B * n * ps);
  c.tv = cv.take<char>((size_t)B * n * ps);
  c.sv = cv.take<char>((size_t)B * n * ps);
  const bool two_sets = c.shape.linear_solver == OK_SOLVER_MINRES;
  for (int l = 0; l < c.L; l++) {
    const int64_t nl = c.lev[l].nodes;
    for (int k = 0; k < 5; k++) {
      c.mg[l][k] = (l == 0 && k < 2) ? nullptr : cv.take<char>((size_t)B * nl * ps);
      c.mg2[l][k] = (two_sets && !(l == 0 && k < 2)) ? cv.take<char>((size_t)B * nl * ps)
                                                      : nullptr;
    }
  }
  c.pA = cv.take<double>((size_t)B * kMaxRedBlocks);
  c.pB = cv.take<double>((size_t)B * kMaxRedBlocks);
  c.H = cv.take<double>((size_t)B * (m + 1) * m);
  c.cs = cv.take<double>((size_t)B * (m + 1));
  c.sn = cv.take<double>((size_t)B * (m + 1));
  c.g = cv.take<double>((size_t)B * (m + 1));
  c.y = cv.take<double>((size_t)B * (m + 1));
  c.kr = cv.take<double>((size_t)B * 8);
  c.nrm = cv.take<double>((size_t)B * 8);
  c.sc = cv.take<double>((size_t)B * (m + 1));
  c.Lm = cv.take<double>((size_t)B * (m + 1) * (m + 1));
  c.hcf = cv.take<double>((size_t)B * (m + 1));
  c.pd = cv.take<double>((size_t)B * 2 * m * red_blocks(n2));
  c.mr = cv.take<double>((size_t)B * MR_COUNT);
  *total = (cv.off + 255) & ~(size_t)255;
}

void setup_shape(ClassCtx& c, const ok_params& shape, int B) {
  c.shape = shape;
  c.B = B;
  c.dim = shape.dim;
  c.L = levels_for(&shape);
  c.m = shape.gmres_restart;
  // MINRES keeps nine work vectors of 2n (three each of v, z and w) in V
  c.nv = shape.linear_solver == OK_SOLVER_MINRES ? std::max(c.m + 1, 9) : c.m + 1;
  c.mixed = (shape.precision == OK_MIXED);
  c.psz = c.mixed ? sizeof(float) : sizeof(double);
  int nl = shape.n;
  for (int l = 0; l < c.L; l++) {
    c.lev[l] = make_grid(shape.dim, nl);
    nl /= 2;
  }
  c.n = c.lev[0].nodes;
}

// ---------------------------------------------------------------------------
// Strides of the SoA arrays.
// ---------------------------------------------------------------------------
inline int64_t sV(const ClassCtx& c) { return (int64_t)c.nv * c.vs; }
inline int64_t sZ(const ClassCtx& c) { return (int64_t)c.m * c.vs; }
inline int64_t sH(const ClassCtx& c) { return (int64_t)(c.m + 1) * c.m; }
inline int64_t sM(const ClassCtx& c) { return (int64_t)c.m + 1; }
inline int64_t sL(const ClassCtx& c) { return (int64_t)(c.m + 1) * (c.m + 1); }
inline int64_t sPd(const ClassCtx& c) { return (int64_t)2 * c.m * red_blocks(c.n2()); }

template <class P>
Vec<P> pvec(void* p, int64_t s) {
  return Vec<P>{(P*)p, s};
}
template <class T>
Vec<const T> cst(Vec<T> v) {
  return Vec<const T>{v.p, v.s};
}
template <class T>
Vec<T> off(Vec<T> v, int64_t o) {
  return Vec<T>{v.p + o, v.s};
}

// ---------------------------------------------------------------------------
// Chebyshev drivers (Saad, Alg. 12.1); coefficients come from the constants
// table, iteration k uses c1[k], c2[k].  `cls` tags launches for profiling;
// `step_cls` the middle iterations, which are timed as one contiguous run.
// ---------------------------------------------------------------------------
template <class TB, class P>
int cheb_zero(ClassCtx& c, const int* fl, int cls, int step_cls, const Grid& g, int lev, int osc,
              int K, Vec<const TB> b, Vec<P> x, Vec<P> r, Vec<P> da, Vec<P> db, hipStream_t st,
              Vec<P> r2 = Vec<P>{nullptr, 0},
              Vec<const double> bs = Vec<const double>{nullptr, 0}) {
  const Batch B = c.batch(fl);
  const double w = (double)c.psz * g.nodes * c.B, wb = (double)sizeof(TB) * g.nodes * c.B;
  if (K > kMaxCheb) return set_err(c.err, OK_E_INVALID, "too many Chebyshev iterations");
  if (K <= 1) {
    ProfScope ps(c, cls, wb + w, st);
    OKE(c, launch_cheb_one<TB, P>(g, B, lev, osc, b, x, st, bs));
    return OK_SUCCESS;
  }
  {
    ProfScope ps(c, cls, wb + (K == 2 ? w : 3.0 * w), st);
    OKE(c, launch_cheb_first<TB, P>(g, B, lev, osc, K == 2, b, x, r, da, st, bs));
  }
  if (K == 2) return OK_SUCCESS;
  Vec<P> dc = da, dn = db;
  if (lev < 0 && K >= 4 && !r2.null() && cheb_fusion_on(g, (int)sizeof(P))) {
    // iterations 1 .. K-2 (the last one final) in fused pairs; an odd count
    // starts with one single iteration; r alternates between r and r2
    Vec<P> rc = r, rn = r2;
    int k = 1;
    if ((K - 2) % 2) {
      ProfScope ps(c, step_cls, 6.0 * w, st);
      OKE(c, launch_cheb_step<P>(g, B, lev, k, osc, false, x, rc, cst(dc), dn, st));
      std::swap(dc, dn);
      k++;
    }
    // the middle pairs timed as one contiguous run (events between launches
    // would hold up each launch), the final pair on its own
    const int mid = (K - 1 - k) / 2 - 1;  // K >= 4: at least the final pair
    if (mid > 0) {
      ProfScope ps(c, step_cls, 6.0 * w * mid, st, mid);
      for (int q = 0; q < mid; q++, k += 2) {
        OKE(c, launch_cheb_step2<P>(g, B, k, osc, false, x, cst(rc), rn, cst(dc), dn, st));
        std::swap(dc, dn);
        std::swap(rc, rn);
      }
    }
    ProfScope ps(c, cls, 4.0 * w, st);
    OKE(c, launch_cheb_step2<P>(g, B, k, osc, true, x, cst(rc), rn, cst(dc), dn, st));
    return OK_SUCCESS;
  }
  {
    const int mid = K > 3 ? K - 3 : 0;
    ProfScope ps(c, step_cls, 6.0 * w * mid, st, mid);
    for (int k = 1; k <= K - 3; k++) {
      OKE(c, launch_cheb_step<P>(g, B, lev, k, osc, false, x, r, cst(dc), dn, st));
      std::swap(dc, dn);
    }
  }
  {
    ProfScope ps(c, cls, 4.0 * w, st);
    OKE(c, launch_cheb_step<P>(g, B, lev, K - 2, osc, true, x, r, cst(dc), dn, st));
  }
  return OK_SUCCESS;
}

template <class P>
int cheb_from(ClassCtx& c, const int* fl, int cls, const Grid& g, int lev, int K, Vec<const P> b,
              Vec<P> x, Vec<P> r, Vec<P> da, Vec<P> db, hipStream_t st) {
  const Batch B = c.batch(fl);
  const double w = (double)c.psz * g.nodes * c.B;
  if (K > kMaxCheb + 1) return set_err(c.err, OK_E_INVALID, "too many Chebyshev iterations");
  {
    ProfScope ps(c, cls, 4.0 * w, st);
    OKE(c, launch_cheb_start<P>(g, B, lev, b, cst(x), r, da, st));
  }
  if (K <= 1) {
    OKE(c, launch_add_inplace<P>(B, x, cst(da), g.nodes, st));
    return OK_SUCCESS;
  }
  Vec<P> dc = da, dn = db;
  for (int k = 0; k <= K - 2; k++) {
    const bool last = (k == K - 2);
    ProfScope ps(c, cls, last ? 4.0 * w : 6.0 * w, st);
    OKE(c, launch_cheb_step<P>(g, B, lev, k, CF_ONE, last, x, r, cst(dc), dn, st));
    std::swap(dc, dn);
  }
  return OK_SUCCESS;
}

// ---------------------------------------------------------------------------
// Multigrid V-cycle for S^ = M + alpha K (Sec. 2 after eq. (schurinv)).
// ---------------------------------------------------------------------------
// set: which work buffers (c.mg, or c.mg2 for a second concurrent cycle).
template <class P>
int mg_vcycle(ClassCtx& c, const int* fl, int l, Vec<const P> b, Vec<P> x, bool zero_start,
              hipStream_t st, int set = 0) {
  const Grid& g = c.lev[l];
  const Batch B = c.batch(fl);
  void* const(*mgw)[5] = set ? c.mg2 : c.mg;
  if (l == c.L - 1) {
    OKE(c, launch_coarse_solve<P>(g, B, b, x, pvec<P>(mgw[l][2], g.nodes),
                                  pvec<P>(mgw[l][3], g.nodes), st));
    return OK_SUCCESS;
  }
  const int64_t nl = g.nodes;
  Vec<P> r = pvec<P>(mgw[l][2], nl), da = pvec<P>(mgw[l][3], nl), db = pvec<P>(mgw[l][4], nl);
  const int cls = (l == 0) ? OK_K_MG_SMOOTH : OK_K_NONE;
  const Grid& gc = c.lev[l + 1];
  Vec<P> xc = pvec<P>(mgw[l + 1][0], gc.nodes), bc = pvec<P>(mgw[l + 1][1], gc.nodes);
  if (zero_start && c.shape.mg_pre == 2 && c.shape.mg_post == 2 &&
      mg_fusion_on(g, (int)sizeof(P))) {
    // pre-smoothing and residual in one pass (smoothed x kept in db), the
    // coarse-grid correction added to db, post-smoothing from db into x
    {
      ProfScope ps(c, cls, 3.0 * c.psz * nl * c.B, st);
      OKE(c, launch_mg_pre2<P>(g, B, l, b, db, r, st));
    }
    OKE(c, launch_restrict<P>(g, gc, B, cst(r), bc, st));
    int e = mg_vcycle<P>(c, fl, l + 1, cst(bc), xc, true, st, set);
    if (e) return e;
    if (prolong_fusion_enabled() && mg_post_prolong_ok<P>(g, gc)) {
      // the correction interpolated while db is staged: db is not rewritten
      ProfScope ps(c, cls, (3.0 + 0.125) * c.psz * nl * c.B, st);
      OKE(c, launch_mg_post2_prolong<P>(g, gc, B, l, b, cst(db), cst(xc), x, st));
      return OK_SUCCESS;
    }
    OKE(c, launch_prolong_add<P>(g, gc, B, cst(xc), db, st));
    ProfScope ps(c, cls, 3.0 * c.psz * nl * c.B, st);
    OKE(c, launch_mg_post2<P>(g, B, l, b, cst(db), x, st));
    return OK_SUCCESS;
  }
  int e = zero_start
              ? cheb_zero<P, P>(c, fl, cls, cls, g, l, CF_ONE, c.shape.mg_pre, b, x, r, da, db, st)
              : cheb_from<P>(c, fl, cls, g, l, c.shape.mg_pre, b, x, r, da, db, st);
  if (e) return e;
  {
    ProfScope ps(c, cls, 3.0 * c.psz * nl * c.B, st);
    OKE(c, launch_resid<P>(g, B, l, b, cst(x), r, st));
  }
  OKE(c, launch_restrict<P>(g, gc, B, cst(r), bc, st));
  e = mg_vcycle<P>(c, fl, l + 1, cst(bc), xc, true, st, set);
  if (e) return e;
  OKE(c, launch_prolong_add<P>(g, gc, B, cst(xc), x, st));
  return cheb_from<P>(c, fl, cls, g, l, c.shape.mg_post, b, x, r, da, db, st);
}

template <class P>
int mg_apply(ClassCtx& c, const int* fl, Vec<const P> b, Vec<P> x, int cycles, hipStream_t st,
             int set = 0) {
  for (int k = 0; k < cycles; k++) {
    int e = mg_vcycle<P>(c, fl, 0, b, x, k == 0, st, set);
    if (e) return e;
  }
  return OK_SUCCESS;
}

// x = S~^-1 b = S^^-1 M S^^-1 b, eq. (schurinv); t, s: work vectors.
template <class P>
int schur_tilde_inv(ClassCtx& c, const int* fl, Vec<const P> b, Vec<P> x, Vec<P> t, Vec<P> s,
                    hipStream_t st) {
  const Grid& g = c.lev[0];
  const Batch B = c.batch(fl);
  int e = mg_apply<P>(c, fl, b, t, c.shape.mg_cycles, st);
  if (e) return e;
  OKE(c, launch_stencil_axpy<P, P, P>(g, B, cst(t), Vec<const P>{nullptr, 0}, 1.0, CF_ONE, 0.0,
                                      CF_ONE, s, st));
  return mg_apply<P>(c, fl, cst(s), x, c.shape.mg_cycles, st);
}

// z = [z1; z2] = P^-1 [r1; r2], eq. (prec) with S~^-1 = S^^-1 M S^^-1.
// rs (may be null): r is stored unscaled, its value is rs[0] * r.
template <class P>
int precond(ClassCtx& c, const int* fl, Vec<const double> u, Vec<const double> r, Vec<P> z,
            hipStream_t st, Vec<const double> rs = Vec<const double>{nullptr, 0}) {
  const Grid& g = c.lev[0];
  const Batch B = c.batch(fl);
  const int64_t n = c.n;
  Vec<const double> r1 = r, r2 = off(r, n);
  Vec<P> z1 = z, z2 = off(z, n);
  Vec<P> cr = pvec<P>(c.cr, n), cda = pvec<P>(c.cda, n), cdb = pvec<P>(c.cdb, n);
  // z1 = A~^-1 r1: Chebyshev on M, scaled by 1/(1 + dt th sigma).
  int e = cheb_zero<double, P>(c, fl, OK_K_NONE, OK_K_CHEB_MASS, g, -1, CF_INV_SA,
                               c.shape.cheb_A_its, r1, z1, cr, cda, cdb, st, pvec<P>(c.cr2, n),
                               rs);
  if (e) return e;
  // y = r2 - C z1 = r2 + eps^2 K z1 + M_E(u) z1, M_E z1 = 3G - M z1 (G in FP64);
  // Q = -(eps^2 K z1 + M_E(u) z1) is kept: the Jacobian applied to this z needs it.
  Vec<double> G = vec(c.G, n);
  {
    ProfScope ps(c, OK_K_ELEMENT, (double)n * c.B * (8.0 + c.psz + 8.0), st);
    OKE(c, launch_element<P, double>(g, B, 0, u, cst(z1), Vec<const double>{nullptr, 0}, 3.0, 0.0,
                                     G, st));
  }
  Vec<P> y = pvec<P>(c.yv, n), t = pvec<P>(c.tv, n), s = pvec<P>(c.sv, n);
  OKE(c, launch_couple<P>(g, B, cst(z1), cst(G), r2, rs, y, vec(c.Q, n), st));
  // z2 = S~^-1 y = S^^-1 M S^^-1 y
  e = schur_tilde_inv<P>(c, fl, cst(y), z2, t, s, st);
  if (e) return e;
  // Sec. 4: further Richardson iterations z2 += S~^-1 (y - S z2), with
  // S z2 = M z2 + (eps^2 K + M_E(u)) A~^-1 (dt th K z2) applied matrix-free
  if (c.shape.schur_richardson > 1) {
    const int64_t sp = (int64_t)4 * n;
    Vec<P> rt = pvec<P>(c.rich, sp), ra = off(rt, n), res = off(rt, 2 * n), cor = off(rt, 3 * n);
    rt.s = ra.s = res.s = cor.s = sp;
    for (int it = 1; it < c.shape.schur_richardson; it++) {
      OKE(c, launch_stencil_axpy<P, P, P>(g, B, cst(z2), Vec<const P>{nullptr, 0}, 0.0, CF_ONE,
                                          1.0, CF_DTH, rt, st));
      e = cheb_zero<P, P>(c, fl, OK_K_NONE, OK_K_NONE, g, -1, CF_INV_SA, c.shape.cheb_A_its,
                          cst(rt), ra, cr, cda, cdb, st, pvec<P>(c.cr2, n));
      if (e) return e;
      OKE(c, launch_element<P, double>(g, B, 0, u, cst(ra), Vec<const double>{nullptr, 0}, 3.0,
                                       0.0, G, st));
      OKE(c, launch_schur_res<P>(g, B, cst(ra), cst(z2), cst(G), cst(y), res, st));
      e = schur_tilde_inv<P>(c, fl, cst(res), cor, t, s, st);
      if (e) return e;
      OKE(c, launch_add_inplace<P>(B, z2, cst(cor), n, st));
    }
  }
  return OK_SUCCESS;
}

// y = J(u) x, eq. (newton); x of type TX (2n), y FP64 (2n).
template <class TX>
int jac(ClassCtx& c, const int* fl, Vec<const double> u, Vec<const TX> x, Vec<double> y,
        hipStream_t st) {
  const Grid& g = c.lev[0];
  const Batch B = c.batch(fl);
  const int64_t n = c.n;
  Vec<double> G = vec(c.G, n);
  {
    ProfScope ps(c, OK_K_ELEMENT, (double)n * c.B * (8.0 + sizeof(TX) + 8.0), st);
    OKE(c, launch_element<TX, double>(g, B, 0, u, x, Vec<const double>{nullptr, 0}, -3.0, 0.0,
                                      G, st));
  }
  // y1 = sA M x1 + dt th K x2;  y2 = -M_E x1 - eps^2 K x1 + M x2 = -3G + M x1 - eps^2 K x1 + M x2
  const double cf[2][4] = {{1.0, 0.0, 0.0, 1.0}, {1.0, -1.0, 1.0, 0.0}};
  const int ff[2][4] = {{CF_SA, CF_ONE, CF_ONE, CF_DTH}, {CF_ONE, CF_E2, CF_ONE, CF_ONE}};
  OKE(c, launch_stencil_lin2<TX>(g, B, x, off(x, n), Vec<const double>{nullptr, 0}, cst(G), cf, ff,
                                 y, off(y, n), st));
  return OK_SUCCESS;
}

// y = J(u) z for z = P^-1 v just computed by precond (same instances): the
// coupling term of row 2 is the stored Q, so no quadrature pass is needed.
//   y1 = sA M z1 + dt th K z2;  y2 = Q + M z2
template <class P>
int jac_z(ClassCtx& c, const int* fl, Vec<const P> z, Vec<double> y, hipStream_t st) {
  const Grid& g = c.lev[0];
  const Batch B = c.batch(fl);
  const int64_t n = c.n;
  const double cf[2][4] = {{1.0, 0.0, 0.0, 1.0}, {0.0, 0.0, 1.0, 0.0}};
  const int ff[2][4] = {{CF_SA, CF_ONE, CF_ONE, CF_DTH}, {CF_ONE, CF_ONE, CF_ONE, CF_ONE}};
  OKE(c, launch_stencil_lin2<P>(g, B, z, off(z, n), Vec<const double>{nullptr, 0},
                                Vec<const double>{c.Q, n}, cf, ff, y, off(y, n), st));
  return OK_SUCCESS;
}

template <class T>
int d2h(ClassCtx& c, std::vector<T>& h, const T* d, size_t count, hipStream_t st) {
  h.resize(count);
  OKE(c, hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, st));
  return OK_SUCCESS;
}

int sync(ClassCtx& c, hipStream_t st) {
  OKE(c, hipStreamSynchronize(st));
  return OK_SUCCESS;
}

int push_flags(ClassCtx& c, int* dflags, const std::vector<int>& h, hipStream_t st) {
  OKE(c, hipMemcpyAsync(dflags, h.data(), sizeof(int) * c.B, hipMemcpyHostToDevice, st));
  // The host vector may change right after this call returns: make the copy complete.
  OKE(c, hipStreamSynchronize(st));
  return OK_SUCCESS;
}

int g_ortho = 0;

// One FGMRES iteration j (Arnoldi step + Givens) for the active instances.
template <class P>
int fgmres_iteration(ClassCtx& c, int j, Vec<const double> u, hipStream_t st) {
  const int64_t n2 = c.n2();
  const Batch B = c.batch(c.act);
  Vec<double> Vj = Vec<double>{c.V + (int64_t)j * c.vs, sV(c)};
  Vec<double> W = Vec<double>{c.V + (int64_t)(j + 1) * c.vs, sV(c)};
  Vec<P> Zj = Vec<P>{(P*)c.Z + (int64_t)j * c.vs, sZ(c)};
  const bool proj = (g_ortho == 0);
  int e = precond<P>(c, c.act, u, cst(Vj), Zj, st,
                     proj ? Vec<const double>{c.sc + j, sM(c)} : Vec<const double>{nullptr, 0});
  if (e) return e;
  e = jac_z<P>(c, c.act, cst(Zj), W, st);
  if (e) return e;
  Vec<double> pin = vec(c.pA, (int64_t)kMaxRedBlocks), pout = vec(c.pB, (int64_t)kMaxRedBlocks);
  if (proj) {
    {
      // modified Gram-Schmidt's algorithmic bytes (w and v_i read, w written
      // per projection i = 0..j); the two passes move 2j+5 vectors
      ProfScope ps(c, OK_K_KRYLOV, 24.0 * (j + 1) * n2 * c.B, st, j / kProjGroup + 3);
      OKE(c, launch_proj(B, W, Vec<const double>{c.V, sV(c)}, c.vs, j, c.m, n2, vec(c.pd, sPd(c)),
                         Vec<const double>{c.sc, sM(c)}, vec(c.Lm, sL(c)),
                         Vec<double>{c.H + (int64_t)j * (c.m + 1), sH(c)}, vec(c.hcf, sM(c)),
                         pin, st));
    }
    OKE(c, launch_givens(B, c.act, j, c.m, vec(c.H, sH(c)), vec(c.cs, sM(c)), vec(c.sn, sM(c)),
                         vec(c.g, sM(c)), cst(pin), n2, vec(c.kr, (int64_t)8), vec(c.sc, sM(c)),
                         st));
    return OK_SUCCESS;
  }
  {
    // the Gram-Schmidt chain (one dot, j+1 fused steps) timed as one run;
    // algorithmic bytes of modified Gram-Schmidt: per projection i = 0..j,
    // w and v_i read and w written (the kernels also read v_{i+1} for the
    // fused next dot, and the dot reads w and v_0 once more)
    ProfScope ps(c, OK_K_KRYLOV, 24.0 * (j + 1) * n2 * c.B, st, j + 2);
    OKE(c, launch_dot_partial(B, cst(W), Vec<const double>{c.V, sV(c)}, n2, pin, st));
    for (int i = 0; i <= j; i++) {
      Vec<const double> vi{c.V + (int64_t)i * c.vs, sV(c)};
      Vec<const double> vn{(i < j) ? c.V + (int64_t)(i + 1) * c.vs : nullptr, sV(c)};
      OKE(c, launch_mgs_step(B, W, vi, vn, n2, cst(pin), pout,
                             Vec<double>{c.H + (int64_t)j * (c.m + 1) + i, sH(c)}, st));
      std::swap(pin, pout);
    }
  }
  OKE(c, launch_givens(B, c.act, j, c.m, vec(c.H, sH(c)), vec(c.cs, sM(c)), vec(c.sn, sM(c)),
                       vec(c.g, sM(c)), cst(pin), n2, vec(c.kr, (int64_t)8),
                       Vec<double>{nullptr, 0}, st));
  OKE(c, launch_scale_by(B, cst(W), W, Vec<const double>{c.kr, 8}, n2, st));
  return OK_SUCCESS;
}

// Iteration j on stream s: replayed from a graph captured on the class stream
// (kernel arguments depend only on j, the state pointer and the tuned launch
// shapes), or launched kernel by kernel.  No graphs while kernels are profiled.
int run_iteration(ClassCtx& c, int j, Vec<const double> u, hipStream_t s) {
  ClassExec* x = c.ex.get();
  const bool profiling = c.prof && c.prof->mask != 0;
  if (!x || !x->graphs || profiling)
    return c.mixed ? fgmres_iteration<float>(c, j, u, s) : fgmres_iteration<double>(c, j, u, s);
  if (x->key != (const void*)u.p || (int)x->iter.size() != c.m) {
    x->clear_graphs();
    x->iter.assign(c.m, nullptr);
    x->key = u.p;
  }
  if (!x->iter[j]) {
    OKE(c, hipStreamBeginCapture(x->xs, hipStreamCaptureModeThreadLocal));
    if (c.prof) c.prof->capturing = true;
    int e = c.mixed ? fgmres_iteration<float>(c, j, u, x->xs)
                    : fgmres_iteration<double>(c, j, u, x->xs);
    if (c.prof) c.prof->capturing = false;
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(x->xs, &g);
    if (e || ee != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      if (e) return e;
      OKE(c, ee);
    }
    hipError_t ei = hipGraphInstantiate(&x->iter[j], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) x->iter[j] = nullptr;
    OKE(c, ei);
  }
  OKE(c, hipGraphLaunch(x->iter[j], s));
  return OK_SUCCESS;
}

template <class P>
int lsq_update(ClassCtx& c, Vec<double> x, hipStream_t st) {
  const Batch B = c.batch(c.incyc);
  OKE(c, launch_lsq_update<P>(B, c.m, Vec<const double>{c.H, sH(c)},
                              Vec<const double>{c.g, sM(c)}, vec(c.y, sM(c)),
                              Vec<const double>{c.kr, 8}, Vec<const P>{(const P*)c.Z, sZ(c)},
                              c.vs, x, c.n2(), st));
  return OK_SUCCESS;
}

bool any(const std::vector<int>& v) {
  for (int a : v)
    if (a) return true;
  return false;
}

}  // namespace

// ---------------------------------------------------------------------------
// Parameters and layout
// ---------------------------------------------------------------------------
int levels_for(const ok_params* p) {
  if (p->mg_levels > 0) return p->mg_levels;
  int L = 1, n = p->n;
  while (n > 8 && n % 2 == 0 && L < kMaxLevels) {
    n /= 2;
    L++;
  }
  return L;
}

int validate_params(const ok_params* p, std::string& why) {
  auto bad = [&](const char* w) {
    why = w;
    return OK_E_INVALID;
  };
  if (!p) return bad("null params");
  if (p->dim != 2 && p->dim != 3) return bad("dim must be 2 or 3");
  if (p->n < 2) return bad("n must be >= 2");
  if (p->dim == 3 && p->n > 512) return bad("3D n must be <= 512");
  if (p->dim == 2 && p->n > 4096) return bad("2D n must be <= 4096");
  if (!(p->eps > 0) || !std::isfinite(p->eps)) return bad("eps must be > 0");
  if (!(p->sigma >= 0) || !std::isfinite(p->sigma)) return bad("sigma must be >= 0");
  if (!(std::fabs(p->m) < 1)) return bad("|m| must be < 1");
  if (!(p->dt > 0) || !std::isfinite(p->dt)) return bad("dt must be > 0");
  if (!(p->theta > 0 && p->theta <= 1)) return bad("theta must be in (0,1]");
  if (p->precision != OK_FP64 && p->precision != OK_MIXED) return bad("bad precision");
  if (p->gmres_restart < 1 || p->gmres_restart > 64) return bad("gmres_restart in 1..64");
  if (p->gmres_max_restarts < 0) return bad("gmres_max_restarts >= 0");
  if (!(p->gmres_rtol > 0)) return bad("gmres_rtol > 0");
  if (!(p->newton_atol >= 0)) return bad("newton_atol >= 0");
  if (p->newton_max_it < 0) return bad("newton_max_it >= 0");
  if (p->cheb_A_its < 1 || p->cheb_A_its > kMaxCheb) return bad("cheb_A_its in 1..32");
  if (p->schur_richardson < 1) return bad("schur_richardson >= 1");
  if (p->mg_pre < 1 || p->mg_post < 1 || p->mg_cycles < 1) return bad("mg_pre/post/cycles >= 1");
  if (p->mg_pre > kMaxCheb || p->mg_post > kMaxCheb) return bad("mg_pre/post <= 32");
  if (p->linear_solver != OK_SOLVER_FGMRES && p->linear_solver != OK_SOLVER_MINRES)
    return bad("linear_solver must be OK_SOLVER_FGMRES or OK_SOLVER_MINRES");
  if (p->linear_solver == OK_SOLVER_MINRES && p->precision != OK_FP64)
    return bad("OK_SOLVER_MINRES requires precision OK_FP64");
  int L = levels_for(p);
  if (L < 1 || L > kMaxLevels) return bad("bad mg_levels");
  if (p->n % (1 << (L - 1))) return bad("n not divisible by 2^(levels-1)");
  int nc = p->n >> (L - 1);
  if (nc < 1 || nc + 1 > 64) return bad("coarsest grid must have <= 64 nodes per direction");
  return OK_SUCCESS;
}

bool same_class(const ok_params& a, const ok_params& b) {
  return a.dim == b.dim && a.n == b.n && a.precision == b.precision &&
         a.gmres_restart == b.gmres_restart && a.gmres_max_restarts == b.gmres_max_restarts &&
         a.newton_max_it == b.newton_max_it && a.cheb_A_its == b.cheb_A_its &&
         a.schur_richardson == b.schur_richardson && levels_for(&a) == levels_for(&b) &&
         a.mg_pre == b.mg_pre && a.mg_post == b.mg_post && a.mg_cycles == b.mg_cycles &&
         a.linear_solver == b.linear_solver;
}

size_t class_bytes(const ok_params& shape, int B, bool with_state) {
  ClassCtx c;
  setup_shape(c, shape, B);
  size_t total = 0;
  carve(c, nullptr, with_state, &total);
  return total;
}

int class_init(ClassCtx& c, const ok_params* ps, int B, char* base, bool with_state,
               hipStream_t st, std::string& err) {
  setup_shape(c, ps[0], B);
  size_t total = 0;
  carve(c, base, with_state, &total);
  c.ip.assign(ps, ps + B);
  c.hcoef.resize(B);
  for (int i = 0; i < B; i++) inst_coef(c.hcoef[i], ps[i], c.lev, c.L);
  c.h_act.assign(B, 0);
  c.h_part.assign(B, 0);
  c.h_aux.assign(B, 0);
  c.h_hasF.assign(B, 0);
  c.out.assign(B, InstOut{});
  c.nits.assign(B, 0);
  hipError_t e = hipMemcpyAsync(c.coef, c.hcoef.data(), sizeof(InstCoef) * B,
                                hipMemcpyHostToDevice, st);
  for (int* f : {c.act, c.part, c.incyc, c.aux})
    if (e == hipSuccess) e = hipMemsetAsync(f, 0, sizeof(int) * B, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    err = std::string("class setup: ") + hipGetErrorString(e);
    return OK_E_HIP;
  }
  return OK_SUCCESS;
}

int push_part(ClassCtx& c, hipStream_t st) { return push_flags(c, c.part, c.h_part, st); }

int set_instance(ClassCtx& c, int i, const ok_params& p, hipStream_t st) {
  if (i < 0 || i >= c.B || !same_class(c.shape, p)) return OK_E_INVALID;
  c.ip[i] = p;
  inst_coef(c.hcoef[i], p, c.lev, c.L);
  OKE(c, hipMemcpyAsync(c.coef + i, &c.hcoef[i], sizeof(InstCoef), hipMemcpyHostToDevice, st));
  // the host entry may be rewritten by the next call: complete the copy
  OKE(c, hipStreamSynchronize(st));
  return OK_SUCCESS;
}

int enable_exec(ClassCtx& c, bool graphs) {
  if (!c.ex) {
    c.ex.reset(new ClassExec());
    OKE(c, hipStreamCreateWithFlags(&c.ex->xs, hipStreamNonBlocking));
    OKE(c, hipEventCreateWithFlags(&c.ex->fork, hipEventDisableTiming));
    OKE(c, hipEventCreateWithFlags(&c.ex->join, hipEventDisableTiming));
  }
  c.ex->graphs = graphs;
  c.ex->clear_graphs();
  return OK_SUCCESS;
}

// ---------------------------------------------------------------------------
// Single operations (FP64 in/out)
// ---------------------------------------------------------------------------
int jac_apply_d(ClassCtx& c, const int* flags, Vec<const double> u, Vec<const double> x,
                Vec<double> y, hipStream_t st) {
  return jac<double>(c, flags, u, x, y, st);
}

int precond_apply_d(ClassCtx& c, const int* flags, Vec<const double> u, Vec<const double> r,
                    Vec<double> z, hipStream_t st) {
  if (!c.mixed) return precond<double>(c, flags, u, r, z, st);
  Vec<float> zt = pvec<float>(c.zt, c.n2());
  int e = precond<float>(c, flags, u, r, zt, st);
  if (e) return e;
  OKE(c, launch_copy_scale<float, double>(c.batch(flags), cst(zt), z, 1.0, c.n2(), st));
  return OK_SUCCESS;
}

int cheb_mass_d(ClassCtx& c, const int* flags, Vec<const double> r, Vec<double> x,
                hipStream_t st) {
  const Grid& g = c.lev[0];
  const int64_t n = c.n;
  if (!c.mixed)
    return cheb_zero<double, double>(c, flags, OK_K_NONE, OK_K_CHEB_MASS, g, -1, CF_ONE,
                                     c.shape.cheb_A_its, r, x, pvec<double>(c.cr, n),
                                     pvec<double>(c.cda, n), pvec<double>(c.cdb, n), st,
                                     pvec<double>(c.cr2, n));
  Vec<float> xf = pvec<float>(c.zt, c.n2());
  int e = cheb_zero<double, float>(c, flags, OK_K_NONE, OK_K_CHEB_MASS, g, -1, CF_ONE,
                                   c.shape.cheb_A_its, r, xf, pvec<float>(c.cr, n),
                                   pvec<float>(c.cda, n), pvec<float>(c.cdb, n), st,
                                   pvec<float>(c.cr2, n));
  if (e) return e;
  OKE(c, launch_copy_scale<float, double>(c.batch(flags), cst(xf), x, 1.0, n, st));
  return OK_SUCCESS;
}

int mg_apply_d(ClassCtx& c, const int* flags, Vec<const double> b, Vec<double> x, int cycles,
               hipStream_t st) {
  if (!c.mixed) return mg_apply<double>(c, flags, b, x, cycles, st);
  const int64_t n = c.n;
  Vec<float> bf = Vec<float>{(float*)c.zt, c.n2()}, xf = Vec<float>{(float*)c.zt + n, c.n2()};
  OKE(c, launch_copy_scale<double, float>(c.batch(flags), b, bf, 1.0, n, st));
  int e = mg_apply<float>(c, flags, cst(bf), xf, cycles, st);
  if (e) return e;
  OKE(c, launch_copy_scale<float, double>(c.batch(flags), cst(xf), x, 1.0, n, st));
  return OK_SUCCESS;
}

int initial_w_d(ClassCtx& c, Vec<const double> u, Vec<double> w, int* rounds, hipStream_t st) {
  const Grid& g = c.lev[0];
  const Batch B = c.batch(nullptr);
  const int64_t n = c.n;
  // rhs = N(u) + eps^2 K u  (weak form of (okb) at u)
  Vec<double> G = vec(c.G, n), rhs = vec(c.Bv, c.n2()), res = vec(c.T1, c.n2()),
              dl = vec(c.X, c.n2());
  OKE(c, launch_element<double, double>(g, B, 1, u, Vec<const double>{nullptr, 0},
                                        Vec<const double>{nullptr, 0}, 1.0, 0.0, G, st));
  OKE(c, launch_stencil_axpy<double, double, double>(g, B, u, cst(G), 0.0, CF_ONE, 1.0, CF_E2,
                                                      rhs, st));
  OKE(c, launch_fill(B, w, 0.0, n, st));
  // Chebyshev work vectors in the (idle) Krylov basis, FP64 in every precision
  const int64_t sv = sV(c);
  Vec<double> cr{c.V, sv}, ca{c.V + n, sv}, cb{c.V + 2 * n, sv}, cr2{c.V + 3 * n, sv};
  auto norm = [&](Vec<const double> v, double* out) -> int {
    OKE(c, launch_dot_partial(B, v, v, n, vec(c.pA, (int64_t)kMaxRedBlocks), st));
    OKE(c, launch_reduce_final(B, Vec<const double>{c.pA, kMaxRedBlocks}, n, vec(c.nrm, 8), st));
    if (d2h(c, c.h_nrm, c.nrm, (size_t)8 * c.B, st) || sync(c, st)) return OK_E_HIP;
    *out = c.h_nrm[1];
    return OK_SUCCESS;
  };
  double bn = 0.0;
  if (norm(cst(rhs), &bn)) return OK_E_HIP;
  int k = 0;
  for (; k < 8; k++) {
    // res = rhs - M w; w += Cheb_M(res)
    OKE(c, launch_stencil_axpy<double, double, double>(g, B, cst(w), cst(rhs), -1.0, CF_ONE, 0.0,
                                                        CF_ONE, res, st));
    double rn = 0.0;
    if (norm(cst(res), &rn)) return OK_E_HIP;
    if (!std::isfinite(rn)) return set_err(c.err, OK_E_NONFINITE, "non-finite initial w");
    if (rn <= 1e-15 * bn) break;
    int e = cheb_zero<double, double>(c, nullptr, OK_K_NONE, OK_K_NONE, g, -1, CF_ONE, kMaxCheb,
                                      cst(res), dl, cr, ca, cb, st, cr2);
    if (e) return e;
    OKE(c, launch_add_inplace<double>(B, w, cst(dl), n, st));
  }
  if (rounds) *rounds = k;
  return OK_SUCCESS;
}

hipError_t residual_launch(const Grid& g, const Batch& B, Vec<const double> u,
                           Vec<const double> w, Vec<const double> un, Vec<const double> wn,
                           Vec<double> F, Vec<double> t1, Vec<double> t2, Vec<double> G,
                           Vec<double> part, Vec<double> nrm, hipStream_t st) {
  const int64_t n = g.nodes;
  hipError_t e = launch_residual_prep(B, u, un, w, wn, t1, t2, n, st);
  if (e != hipSuccess) return e;
  Vec<double> F1 = F, F2 = Vec<double>{F.p + n, F.s};
  const double a[2][4] = {{1.0, 0.0, 0.0, 1.0}, {0.0, 0.0, 0.0, 0.0}};  // F1 = M t1 + K t2
  const int fa[2][4] = {{CF_ONE, CF_ONE, CF_ONE, CF_ONE}, {CF_ONE, CF_ONE, CF_ONE, CF_ONE}};
  e = launch_stencil_lin2<double>(g, B, cst(t1), cst(t2), Vec<const double>{nullptr, 0},
                                  Vec<const double>{nullptr, 0}, a, fa, F1,
                                  Vec<double>{nullptr, 0}, st);
  if (e != hipSuccess) return e;
  e = launch_element<double, double>(g, B, 1, u, Vec<const double>{nullptr, 0},
                                     Vec<const double>{nullptr, 0}, -1.0, 0.0, G, st);
  if (e != hipSuccess) return e;
  // F2 = -N(u) + M w - eps^2 K u
  const double b2[2][4] = {{1.0, 0.0, 0.0, -1.0}, {0.0, 0.0, 0.0, 0.0}};
  const int fb[2][4] = {{CF_ONE, CF_ONE, CF_ONE, CF_E2}, {CF_ONE, CF_ONE, CF_ONE, CF_ONE}};
  e = launch_stencil_lin2<double>(g, B, w, u, cst(G), Vec<const double>{nullptr, 0}, b2, fb, F2,
                                  Vec<double>{nullptr, 0}, st);
  if (e != hipSuccess) return e;
  e = launch_dot_partial(B, cst(F), cst(F), 2 * n, part, st);
  if (e != hipSuccess) return e;
  return launch_reduce_final(B, cst(part), 2 * n, nrm, st);
}

void instance_constants(const ok_params& p, InstCoef& C, Grid* lev, int& L) {
  L = levels_for(&p);
  for (int l = 0; l < L; l++) lev[l] = make_grid(p.dim, p.n >> l);
  inst_coef(C, p, lev, L);
}

int residual_d(ClassCtx& c, const int* flags, Vec<const double> u, Vec<const double> w,
               Vec<const double> un, Vec<const double> wn, Vec<double> F, hipStream_t st) {
  const Grid& g = c.lev[0];
  const Batch B = c.batch(flags);
  const int64_t n = c.n;
  if (F.null()) F = vec(c.Bv, c.n2());
  Vec<double> t1 = vec(c.T1, c.n2()), t2 = off(vec(c.T1, c.n2()), n);
  Vec<const double> wnv = (c.shape.theta < 1.0 || !wn.null()) ? wn : Vec<const double>{nullptr, 0};
  OKE(c, residual_launch(g, B, u, w, un, wnv, F, t1, t2, vec(c.G, n),
                         vec(c.pA, (int64_t)kMaxRedBlocks), vec(c.nrm, 8), st));
  if (d2h(c, c.h_nrm, c.nrm, (size_t)8 * c.B, st)) return OK_E_HIP;
  if (sync(c, st)) return OK_E_HIP;
  std::vector<int> hf(c.B, 1);
  if (flags == c.part) hf = c.h_part;
  else if (flags == c.act) hf = c.h_act;
  else if (flags == c.aux) hf = c.h_aux;
  for (int i = 0; i < c.B; i++)
    if (hf[i]) c.out[i].fnorm = c.h_nrm[8 * i + 1];
  return OK_SUCCESS;
}

// ---------------------------------------------------------------------------
// FGMRES (Saad 1993) in lockstep over a group of classes
// ---------------------------------------------------------------------------
namespace {
int g_issue_ahead = 0;
}  // namespace
void issue_ahead_set(int enable) { g_issue_ahead = enable ? 1 : 0; }
void ortho_set(int mode) { g_ortho = mode ? 1 : 0; }

bool g_trace_ranges = false;
void trace_ranges_set(int enable) { g_trace_ranges = enable != 0; }
void trace_push(const char* name) { roctxRangePushA(name); }
void trace_pop() { roctxRangePop(); }

int fgmres_group(const Group& grp, const std::vector<Vec<const double>>& u,
                 const std::vector<Vec<const double>>& b, const std::vector<Vec<double>>& x,
                 hipStream_t st) {
  const size_t nc = grp.size();
  std::vector<std::vector<double>> bnorm(nc), tol(nc);
  // x = 0, ||b||
  for (size_t k = 0; k < nc; k++) {
    ClassCtx& c = *grp[k];
    for (int i = 0; i < c.B; i++)
      if (c.h_part[i]) c.out[i] = InstOut{0, 0, 0, c.out[i].fnorm, 0.0};
    if (!any(c.h_part)) continue;
    if (push_part(c, st)) return OK_E_HIP;
    const Batch B = c.batch(c.part);
    OKE(c, launch_fill(B, x[k], 0.0, c.n2(), st));
    OKE(c, launch_dot_partial(B, b[k], b[k], c.n2(), vec(c.pA, (int64_t)kMaxRedBlocks), st));
    OKE(c, launch_reduce_final(B, Vec<const double>{c.pA, kMaxRedBlocks}, c.n2(), vec(c.nrm, 8),
                               st));
    if (d2h(c, c.h_nrm, c.nrm, (size_t)8 * c.B, st)) return OK_E_HIP;
  }
  for (size_t k = 0; k < nc; k++)
    if (any(grp[k]->h_part) && sync(*grp[k], st)) return OK_E_HIP;
  for (size_t k = 0; k < nc; k++) {
    ClassCtx& c = *grp[k];
    bnorm[k].assign(c.B, 0.0);
    tol[k].assign(c.B, 0.0);
    c.h_kr.assign((size_t)8 * c.B, 0.0);
    for (int i = 0; i < c.B; i++) {
      c.h_act[i] = 0;
      if (!c.h_part[i]) continue;
      const double bn = c.h_nrm[8 * i + 1];
      bnorm[k][i] = bn;
      if (!std::isfinite(bn)) {
        c.out[i].status = OK_E_NONFINITE;
        continue;
      }
      if (bn == 0.0) continue;
      tol[k][i] = c.ip[i].gmres_rtol * bn;
      c.h_kr[8 * i + 0] = bn;
      c.h_kr[8 * i + 1] = tol[k][i];
      c.h_act[i] = 1;
      c.out[i].status = OK_E_GMRES_MAXIT;
    }
    if (!any(c.h_act)) continue;
    OKE(c, hipMemcpyAsync(c.kr, c.h_kr.data(), sizeof(double) * 8 * c.B, hipMemcpyHostToDevice,
                          st));
    if (push_flags(c, c.act, c.h_act, st)) return OK_E_HIP;
  }
  std::vector<bool> first(nc, true);
  const int max_restarts = grp.empty() ? 0 : grp[0]->shape.gmres_max_restarts;
  for (int cycle = 0; cycle <= max_restarts; cycle++) {
    TraceRange cycle_range("fgmres cycle");
    bool anyact = false;
    for (size_t k = 0; k < nc; k++) {
      ClassCtx& c = *grp[k];
      if (!any(c.h_act)) continue;
      anyact = true;
      const Batch B = c.batch(c.act);
      Vec<const double> src = first[k] ? b[k] : Vec<const double>{c.T1, c.n2()};
      OKE(c, launch_scale_inv(B, src, Vec<double>{c.V, sV(c)}, Vec<const double>{c.nrm, 8},
                              c.n2(), st));
      OKE(c, launch_cycle_init(B, c.m, vec(c.g, sM(c)), Vec<const double>{c.nrm, 8},
                               vec(c.kr, (int64_t)8), vec(c.sc, sM(c)), st));
      OKE(c, hipMemcpyAsync(c.incyc, c.act, sizeof(int) * c.B, hipMemcpyDeviceToDevice, st));
      first[k] = false;
    }
    if (!anyact) break;
    std::vector<std::vector<int>> incyc(nc);
    for (size_t k = 0; k < nc; k++) incyc[k] = grp[k]->h_act;
    const int m = grp[0]->m;
    // Classes with a stream of their own run their iterations there, so the
    // classes of a group overlap on the device.  Iterations are issued one
    // ahead of the stop test: the host launches iteration j, then waits for
    // the activity flags of iteration j-1, so the device does not idle while
    // the host decides whether to go on.
    for (size_t k = 0; k < nc; k++) {
      ClassCtx& c = *grp[k];
      if (!c.ex || !any(c.h_act)) continue;
      OKE(c, hipEventRecord(c.ex->fork, st));
      OKE(c, hipStreamWaitEvent(c.ex->xs, c.ex->fork, 0));
    }
    for (int j = 0; j < m; j++) {
      TraceRange it_range("fgmres iteration");
      bool launched = false;
      for (size_t k = 0; k < nc; k++) {
        ClassCtx& c = *grp[k];
        if (!any(c.h_act)) continue;
        hipStream_t s = c.ex ? c.ex->xs : st;
        int e = run_iteration(c, j, u[k], s);
        if (e) return e;
        if (!c.fp) {
          auto f = std::make_unique<FlagPipe>();
          OKE(c, hipHostMalloc((void**)&f->h, sizeof(int) * 2 * c.B, hipHostMallocDefault));
          for (hipEvent_t& ev : f->ev) OKE(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
          c.fp = std::move(f);
        }
        const int slot = j & 1;
        OKE(c, hipMemcpyAsync(c.fp->h + (size_t)slot * c.B, c.act, sizeof(int) * c.B,
                              hipMemcpyDeviceToHost, s));
        OKE(c, hipEventRecord(c.fp->ev[slot], s));
        c.fp->pend[slot] = j;
        launched = true;
      }
      if (!launched) break;
      // stop test of iteration j-1, read while iteration j runs (an iteration
      // issued after every instance of a class stopped finds the activity
      // flags cleared on the device and does nothing); without issue-ahead,
      // the stop test of iteration j itself
      const int jt = g_issue_ahead ? j - 1 : j;
      if (jt < 0) continue;
      bool still = false;
      for (size_t k = 0; k < nc; k++) {
        ClassCtx& c = *grp[k];
        FlagPipe* f = c.fp.get();
        const int slot = jt & 1;
        if (f && f->pend[slot] == jt) {
          OKE(c, hipEventSynchronize(f->ev[slot]));
          f->pend[slot] = -1;
          c.h_act.assign(f->h + (size_t)slot * c.B, f->h + (size_t)(slot + 1) * c.B);
        }
        still = still || any(c.h_act);
      }
      if (!still) break;
    }
    for (size_t k = 0; k < nc; k++)
      if (grp[k]->fp) grp[k]->fp->pend[0] = grp[k]->fp->pend[1] = -1;
    for (size_t k = 0; k < nc; k++) {
      ClassCtx& c = *grp[k];
      if (!c.ex || !any(incyc[k])) continue;
      OKE(c, hipEventRecord(c.ex->join, c.ex->xs));
      OKE(c, hipStreamWaitEvent(st, c.ex->join, 0));
    }
    // least squares and x update for the instances of this cycle; stop tests
    bool restart_any = false;
    for (size_t k = 0; k < nc; k++) {
      ClassCtx& c = *grp[k];
      if (!any(incyc[k])) continue;
      int e = c.mixed ? lsq_update<float>(c, x[k], st) : lsq_update<double>(c, x[k], st);
      if (e) return e;
      if (d2h(c, c.h_kr, c.kr, (size_t)8 * c.B, st)) return OK_E_HIP;
      if (sync(c, st)) return OK_E_HIP;
      for (int i = 0; i < c.B; i++) {
        c.h_act[i] = 0;
        if (!incyc[k][i]) continue;
        const double* kr = &c.h_kr[8 * i];
        c.out[i].fgmres_its += (int)kr[6];
        c.out[i].lin_res = kr[3] / bnorm[k][i];
        if (kr[7] == 1.0) {
          c.out[i].status = OK_SUCCESS;
        } else if (kr[7] == 2.0) {
          c.out[i].status = OK_E_NONFINITE;
        } else if (cycle < max_restarts) {
          c.h_act[i] = 1;  // restart from the true residual
          restart_any = true;
        } else {
          c.out[i].status = OK_E_GMRES_MAXIT;
        }
      }
    }
    if (!restart_any) break;
    // restart: r = b - J x for the instances still going
    for (size_t k = 0; k < nc; k++) {
      ClassCtx& c = *grp[k];
      if (!any(c.h_act)) continue;
      if (push_flags(c, c.act, c.h_act, st)) return OK_E_HIP;
      const Batch B = c.batch(c.act);
      Vec<double> T1 = vec(c.T1, c.n2());
      int e = jac<double>(c, c.act, u[k], cst(x[k]), T1, st);
      if (e) return e;
      OKE(c, launch_axpby(B, 1.0, b[k], -1.0, cst(T1), T1, c.n2(), st));
      OKE(c, launch_dot_partial(B, cst(T1), cst(T1), c.n2(), vec(c.pA, (int64_t)kMaxRedBlocks),
                                st));
      OKE(c, launch_reduce_final(B, Vec<const double>{c.pA, kMaxRedBlocks}, c.n2(),
                                 vec(c.nrm, 8), st));
      if (d2h(c, c.h_nrm, c.nrm, (size_t)8 * c.B, st)) return OK_E_HIP;
      if (sync(c, st)) return OK_E_HIP;
      for (int i = 0; i < c.B; i++) {
        if (!c.h_act[i]) continue;
        const double beta = c.h_nrm[8 * i + 1];
        c.out[i].lin_res = beta / bnorm[k][i];
        if (!std::isfinite(beta)) {
          c.out[i].status = OK_E_NONFINITE;
          c.h_act[i] = 0;
        } else if (beta <= tol[k][i]) {
          c.out[i].status = OK_SUCCESS;
          c.h_act[i] = 0;
        } else {
          c.out[i].restarts++;
        }
      }
      if (push_flags(c, c.act, c.h_act, st)) return OK_E_HIP;
    }
  }
  return OK_SUCCESS;
}

// ---------------------------------------------------------------------------
// The symmetric rearranged system (Sec. 2, after eq. (schurapprox)) and
// preconditioned MINRES on it
// ---------------------------------------------------------------------------
int sym_apply_d(ClassCtx& c, const int* flags, Vec<const double> u, Vec<const double> x,
                Vec<double> y, hipStream_t st) {
  if (c.mixed) return set_err(c.err, OK_E_INVALID, "the symmetric system is FP64 only");
  const Grid& g = c.lev[0];
  const Batch B = c.batch(flags);
  const int64_t n = c.n;
  Vec<double> G = vec(c.G, n);
  {
    ProfScope ps(c, OK_K_ELEMENT, (double)n * c.B * 24.0, st);
    OKE(c, launch_element<double, double>(g, B, 0, u, off(x, n), Vec<const double>{nullptr, 0},
                                          -3.0, 0.0, G, st));
  }
  // y1 = c K x1 + M x2;  y2 = M x1 + M x2 - eps^2 K x2 + G,  G = -3 (u^2 x2, phi)
  // (M_E x2 = 3 (u^2 x2, phi) - M x2)
  const double cf[2][4] = {{0.0, 1.0, 1.0, 0.0}, {1.0, 0.0, 1.0, -1.0}};
  const int ff[2][4] = {{CF_ONE, CF_C, CF_ONE, CF_ONE}, {CF_ONE, CF_ONE, CF_ONE, CF_E2}};
  OKE(c, launch_stencil_lin2<double>(g, B, x, off(x, n), Vec<const double>{nullptr, 0}, cst(G), cf,
                                     ff, y, off(y, n), st));
  return OK_SUCCESS;
}

namespace {

// z = diag((alpha/c) S^^-1, (c/alpha) S^^-1) v (each block one multigrid
// application of S^), with the partials of <z, v> in c.pA.
// The two V-cycles share no buffer (the second uses the class's second set of
// multigrid work vectors) and run at once: the second half's on the class's
// side stream, forked from and joined back into st.
int sym_precond(ClassCtx& c, const int* fl, Vec<const double> v, Vec<double> z, hipStream_t st) {
  const int64_t n = c.n;
  if (!c.side) {
    auto sd = std::make_unique<SideStream>();
    OKE(c, hipStreamCreateWithFlags(&sd->s, hipStreamNonBlocking));
    OKE(c, hipEventCreateWithFlags(&sd->fork, hipEventDisableTiming));
    OKE(c, hipEventCreateWithFlags(&sd->join, hipEventDisableTiming));
    c.side = std::move(sd);
  }
  SideStream* sd = c.side.get();
  OKE(c, hipEventRecord(sd->fork, st));
  OKE(c, hipStreamWaitEvent(sd->s, sd->fork, 0));
  int e = mg_apply<double>(c, fl, off(v, n), off(z, n), c.shape.mg_cycles, sd->s, 1);
  if (e) return e;
  e = mg_apply<double>(c, fl, v, z, c.shape.mg_cycles, st, 0);
  if (e) return e;
  OKE(c, hipEventRecord(sd->join, sd->s));
  OKE(c, hipStreamWaitEvent(st, sd->join, 0));
  OKE(c, launch_mr_scale_dot(c.batch(fl), z, v, n, vec(c.pA, (int64_t)kMaxRedBlocks), st));
  return OK_SUCCESS;
}

int flag_pipe(ClassCtx& c) {
  if (c.fp) return OK_SUCCESS;
  auto f = std::make_unique<FlagPipe>();
  OKE(c, hipHostMalloc((void**)&f->h, sizeof(int) * 2 * c.B, hipHostMallocDefault));
  for (hipEvent_t& ev : f->ev) OKE(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  c.fp = std::move(f);
  return OK_SUCCESS;
}

}  // namespace

int minres_class(ClassCtx& c, Vec<const double> u, Vec<const double> b, Vec<double> x,
                 bool newton, hipStream_t st) {
  if (c.mixed) return set_err(c.err, OK_E_INVALID, "MINRES requires precision OK_FP64");
  TraceRange range("minres");
  const int64_t n = c.n, n2 = c.n2();
  for (int i = 0; i < c.B; i++)
    if (c.h_part[i]) c.out[i] = InstOut{0, 0, 0, c.out[i].fnorm, 0.0};
  if (!any(c.h_part)) return OK_SUCCESS;
  if (push_part(c, st)) return OK_E_HIP;
  // work vectors in V: v_{j-1}, v_j, v_{j+1}; z_j, z_{j+1}; A z_j; w_{j-1}, w_j, w_{j+1}
  int v0 = 0, v1 = 1, v2 = 2, z1 = 3, z2 = 4, w0 = 6, w1 = 7, w2 = 8;
  const int az = 5;
  auto slot = [&](int k) { return Vec<double>{c.V + (int64_t)k * c.vs, sV(c)}; };
  const Batch P = c.batch(c.part), A = c.batch(c.act), R = c.batch(c.incyc);
  Vec<double> mr = vec(c.mr, (int64_t)MR_COUNT);
  Vec<double> pa = vec(c.pA, (int64_t)kMaxRedBlocks), pb = vec(c.pB, (int64_t)kMaxRedBlocks);
  OKE(c, launch_mr_init(P, b, slot(v1), slot(v0), slot(w0), slot(w1), x, n, newton, st));
  int e = sym_precond(c, c.part, cst(slot(v1)), slot(z1), st);
  if (e) return e;
  OKE(c, launch_mr_start(P, c.act, cst(pa), n2, mr, st));
  e = flag_pipe(c);
  if (e) return e;
  const int maxit = c.m * (c.shape.gmres_max_restarts + 1);
  // Iterations are issued one ahead of the stop test, as in FGMRES: an
  // iteration issued after every instance stopped finds act cleared on the
  // device and does nothing.
  FlagPipe* f = c.fp.get();
  f->pend[0] = f->pend[1] = -1;
  for (int j = 0; j < maxit; j++) {
    TraceRange it_range("minres iteration");
    e = sym_apply_d(c, c.act, u, cst(slot(z1)), slot(az), st);
    if (e) return e;
    OKE(c, launch_dot_partial(A, cst(slot(az)), cst(slot(z1)), n2, pb, st));
    OKE(c, launch_mr_vupd(A, cst(pb), cst(slot(az)), cst(slot(v1)), cst(slot(v0)), slot(v2), n2,
                          mr, st));
    e = sym_precond(c, c.act, cst(slot(v2)), slot(z2), st);
    if (e) return e;
    OKE(c, launch_mr_coef(P, c.act, c.incyc, cst(pa), n2, maxit, mr, st));
    OKE(c, launch_mr_wx(R, c.act, cst(slot(z1)), cst(slot(w0)), cst(slot(w1)), slot(w2), x, n,
                        newton, cst(mr), st));
    int t = v0;
    v0 = v1, v1 = v2, v2 = t;
    std::swap(z1, z2);
    t = w0;
    w0 = w1, w1 = w2, w2 = t;
    const int s = j & 1;
    OKE(c, hipMemcpyAsync(f->h + (size_t)s * c.B, c.act, sizeof(int) * c.B, hipMemcpyDeviceToHost,
                          st));
    OKE(c, hipEventRecord(f->ev[s], st));
    f->pend[s] = j;
    const int jt = g_issue_ahead ? j - 1 : j;
    if (jt < 0) continue;
    const int ts = jt & 1;
    if (f->pend[ts] != jt) continue;
    OKE(c, hipEventSynchronize(f->ev[ts]));
    f->pend[ts] = -1;
    bool still = false;
    for (int i = 0; i < c.B; i++) still = still || f->h[(size_t)ts * c.B + i];
    if (!still) break;
  }
  f->pend[0] = f->pend[1] = -1;
  std::vector<double> h;
  if (d2h(c, h, c.mr, (size_t)MR_COUNT * c.B, st)) return OK_E_HIP;
  if (sync(c, st)) return OK_E_HIP;
  for (int i = 0; i < c.B; i++) {
    if (!c.h_part[i]) continue;
    const double* q = &h[(size_t)MR_COUNT * i];
    InstOut& o = c.out[i];
    o.fgmres_its = (int)q[MR_ITS];
    o.lin_res = q[MR_GAM1] > 0.0 ? std::fabs(q[MR_ETA]) / q[MR_GAM1] : 0.0;
    const int stt = (int)q[MR_STATUS];
    o.status = stt == 1 ? OK_SUCCESS : stt == 2 ? OK_E_NONFINITE : OK_E_GMRES_MAXIT;
  }
  c.h_act.assign(c.B, 0);
  return OK_SUCCESS;
}

int newton_solve_group(const Group& grp, const std::vector<Vec<const double>>& u,
                       const std::vector<Vec<const double>>& b, const std::vector<Vec<double>>& x,
                       hipStream_t st) {
  Group fg;
  std::vector<Vec<const double>> fu, fb;
  std::vector<Vec<double>> fx;
  for (size_t k = 0; k < grp.size(); k++) {
    if (grp[k]->shape.linear_solver == OK_SOLVER_MINRES) {
      int e = minres_class(*grp[k], u[k], b[k], x[k], true, st);
      if (e) return e;
      continue;
    }
    fg.push_back(grp[k]);
    fu.push_back(u[k]);
    fb.push_back(b[k]);
    fx.push_back(x[k]);
  }
  return fg.empty() ? OK_SUCCESS : fgmres_group(fg, fu, fb, fx, st);
}

// ---------------------------------------------------------------------------
// Newton in lockstep (Sec. 2: one linear solve per Newton iteration)
// ---------------------------------------------------------------------------
int newton_group_iters(const Group& grp, const std::vector<Vec<double>>& u,
                       const std::vector<Vec<double>>& w, const std::vector<Vec<const double>>& un,
                       const std::vector<Vec<const double>>& wn, std::vector<NewtonLog>& log,
                       int max_iters, hipStream_t st) {
  const size_t nc = grp.size();
  // Sec. 2 (C3 order): test ||F|| <= atol, else solve J dx = -F and update.
  auto test = [&](ClassCtx& c, size_t k, const std::vector<int>& which) {
    for (int i = 0; i < c.B; i++) {
      if (!which[i]) continue;
      const double f = c.out[i].fnorm;
      log[k].fnorm[i].push_back(f);
      c.h_hasF[i] = 1;
      if (!std::isfinite(f)) {
        c.out[i].status = OK_E_NONFINITE;
        c.h_part[i] = 0;
      } else if (f <= c.ip[i].newton_atol) {
        c.out[i].status = OK_SUCCESS;
        c.h_part[i] = 0;
      } else if (c.nits[i] >= c.shape.newton_max_it) {
        c.out[i].status = OK_E_NEWTON_MAXIT;
        c.h_part[i] = 0;
      } else {
        c.out[i].status = 1;  // still iterating
      }
    }
  };
  // residual of the instances that have none for their current iterate
  for (size_t k = 0; k < nc; k++) {
    ClassCtx& c = *grp[k];
    bool fresh = false;
    for (int i = 0; i < c.B; i++) {
      c.h_aux[i] = c.h_part[i] && !c.h_hasF[i];
      fresh = fresh || c.h_aux[i];
    }
    if (!fresh) continue;
    if (push_flags(c, c.aux, c.h_aux, st)) return OK_E_HIP;
    int e = residual_d(c, c.aux, cst(u[k]), cst(w[k]), un[k], wn[k], vec(c.Bv, c.n2()), st);
    if (e) return e;
    std::vector<int> which = c.h_aux;
    test(c, k, which);
  }
  for (int it = 0; max_iters < 0 || it < max_iters; it++) {
    bool anyp = false;
    for (size_t k = 0; k < nc; k++) anyp = anyp || any(grp[k]->h_part);
    if (!anyp) break;
    TraceRange newton_range("newton iteration");
    std::vector<Vec<const double>> bb(nc);
    std::vector<Vec<double>> xx(nc);
    std::vector<Vec<const double>> uu(nc);
    for (size_t k = 0; k < nc; k++) {
      ClassCtx& c = *grp[k];
      bb[k] = Vec<const double>{c.Bv, c.n2()};
      xx[k] = vec(c.X, c.n2());
      uu[k] = cst(u[k]);
      if (!any(c.h_part)) continue;
      if (push_part(c, st)) return OK_E_HIP;
      OKE(c, launch_copy_scale<double, double>(c.batch(c.part), bb[k], vec(c.Bv, c.n2()), -1.0,
                                               c.n2(), st));
    }
    int e = newton_solve_group(grp, uu, bb, xx, st);
    if (e) return e;
    for (size_t k = 0; k < nc; k++) {
      ClassCtx& c = *grp[k];
      if (!any(c.h_part)) continue;
      for (int i = 0; i < c.B; i++) {
        if (!c.h_part[i]) continue;
        log[k].its[i].push_back(c.out[i].fgmres_its);
        c.nits[i]++;
        // a linear solve that stopped at its iteration limit still gives the
        // step; the Newton test decides
        if (c.out[i].status == OK_E_NONFINITE) c.h_part[i] = 0;
      }
      if (!any(c.h_part)) continue;
      if (push_part(c, st)) return OK_E_HIP;
      const Batch B = c.batch(c.part);
      OKE(c, launch_axpby(B, 1.0, cst(u[k]), 1.0, Vec<const double>{c.X, c.n2()}, u[k], c.n, st));
      OKE(c, launch_axpby(B, 1.0, cst(w[k]), 1.0, Vec<const double>{c.X + c.n, c.n2()}, w[k], c.n,
                          st));
      e = residual_d(c, c.part, cst(u[k]), cst(w[k]), un[k], wn[k], vec(c.Bv, c.n2()), st);
      if (e) return e;
      std::vector<int> which = c.h_part;
      test(c, k, which);
    }
  }
  return OK_SUCCESS;
}

int newton_group(const Group& grp, const std::vector<Vec<double>>& u,
                 const std::vector<Vec<double>>& w, const std::vector<Vec<const double>>& un,
                 const std::vector<Vec<const double>>& wn, std::vector<NewtonLog>& log,
                 hipStream_t st) {
  return newton_group_iters(grp, u, w, un, wn, log, -1, st);
}

// ---------------------------------------------------------------------------
// Tile autotuner
// ---------------------------------------------------------------------------
namespace {

template <class F>
double time_best(hipStream_t st, F&& launch) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return 1e30;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return 1e30;
  }
  double best = 1e30;
  if (launch() == hipSuccess) {
    for (int r = 0; r < 5; r++) {  // best of five: near-equal shapes are close
      (void)hipEventRecord(a, st);
      if (launch() != hipSuccess) {
        best = 1e30;
        break;
      }
      (void)hipEventRecord(b, st);
      (void)hipEventSynchronize(b);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      best = std::min(best, (double)ms);
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

// Candidate z-chunk counts of a streaming stencil launch: chunks of 4 to 32
// planes, and the counts that make the whole grid (all instances) about
// 512 ... 6144 blocks, i.e. one or a few full rounds of resident blocks.
// z-range counts to try for a kernel with nch blocks per plane
std::vector<int> zchunk_candidates_n(const Grid& g, int64_t nch, int count) {
  std::vector<int> v;
  for (int zc : {4, 8, 16, 32}) v.push_back((g.nn + zc - 1) / zc);
  for (int64_t t : {512, 1024, 2048, 3072, 4096, 6144}) v.push_back((int)(t / (nch * count)));
  for (int& z : v) z = std::max(1, std::min(z, g.nn));
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  return v;
}

std::vector<int> zchunk_candidates(const Grid& g, int chunk, int count) {
  const int64_t plane = (g.dim == 3) ? g.plane : (int64_t)g.nn;
  return zchunk_candidates_n(g, (plane + chunk - 1) / chunk, count);
}

template <class P>
int autotune_impl(ClassCtx& c, hipStream_t st, int* entries) {
  const int word = (int)sizeof(P);
  const Batch B = c.batch(nullptr);
  for (int l = 0; l < c.L; l++) {
    const Grid& g = c.lev[l];
    if (l == c.L - 1 && c.L > 1) break;  // the coarsest level is a direct solve
    const int64_t nl = g.nodes;
    Vec<P> x, r, d0, d1;
    if (l == 0) {
      x = pvec<P>(c.yv, nl); r = pvec<P>(c.cr, nl); d0 = pvec<P>(c.cda, nl); d1 = pvec<P>(c.cdb, nl);
    } else {
      x = pvec<P>(c.mg[l][0], nl); r = pvec<P>(c.mg[l][2], nl);
      d0 = pvec<P>(c.mg[l][3], nl); d1 = pvec<P>(c.mg[l][4], nl);
    }
    double best = 1e30;
    int bi = 0, bz = 0, bt = 256;
    for (int threads : {256, 512})
      for (int items = 1; items <= 8; items *= 2) {
        if (!stencil_shape_ok(g.dim, 1, items, threads)) continue;
        for (int zc : zchunk_candidates(g, items * threads, B.count)) {
          stencil_tune_set(g.dim, g.nn, 1, word, items, zc, threads);
          double t = time_best(st, [&]() {
            return launch_cheb_step<P>(g, B, l, 0, CF_ONE, false, x, r, cst(d0), d1, st);
          });
          if (t < best) {
            best = t;
            bi = items;
            bz = zc;
            bt = threads;
          }
        }
      }
    stencil_tune_set(g.dim, g.nn, 1, word, bi, bz, bt);
    if (bi) (*entries)++;
    // fused smoothers of this level (pre-smoothing + residual, post-
    // smoothing): shapes tuned one kernel at a time, kept where the pair
    // beats the four one-iteration kernels it replaces
    stencil_tune_set(g.dim, g.nn, kMgPreKey, word, 0, 0);
    stencil_tune_set(g.dim, g.nn, kMgPostKey, word, 0, 0);
    stencil_tune_set(g.dim, g.nn, kMgPreTileKey, word, 0, 0);
    stencil_tune_set(g.dim, g.nn, kMgPostTileKey, word, 0, 0);
    stencil_tune_set(g.dim, g.nn, kMgPreStripKey, word, 0, 0);
    stencil_tune_set(g.dim, g.nn, kMgPostStripKey, word, 0, 0);
    if (c.shape.mg_pre == 2 && c.shape.mg_post == 2 && mg_fusion_enabled()) {
      Vec<P> bb = (l == 0) ? pvec<P>(c.cr2, nl) : pvec<P>(c.mg[l][1], nl);
      const double unfused = time_best(st, [&]() {
        hipError_t e = launch_cheb_first<P, P>(g, B, l, CF_ONE, true, cst(bb), x, r, d0, st);
        if (e == hipSuccess) e = launch_resid<P>(g, B, l, cst(bb), cst(x), r, st);
        if (e == hipSuccess) e = launch_cheb_start<P>(g, B, l, cst(bb), cst(x), r, d0, st);
        if (e == hipSuccess)
          e = launch_cheb_step<P>(g, B, l, 0, CF_ONE, true, x, r, cst(d0), d1, st);
        return e;
      });
      double fused = 0.0;
      for (int key : {kMgPreKey, kMgPostKey}) {
        double kbest = 1e30;
        int ki = 0, kz = 0, kt = 256;
        for (int threads : {256, 512})
          for (int items = 1; items <= 2; items++) {
            if (!cheb2_shape_ok(g.dim, items, threads)) continue;
            for (int zc : zchunk_candidates(g, items * threads, B.count)) {
              stencil_tune_set(g.dim, g.nn, key, word, items, zc, threads);
              if (!mg2_shape_valid(g, key, word)) continue;
              double t = time_best(st, [&]() {
                return key == kMgPreKey ? launch_mg_pre2<P>(g, B, l, cst(bb), x, r, st)
                                        : launch_mg_post2<P>(g, B, l, cst(bb), cst(x), d1, st);
              });
              if (t < kbest) {
                kbest = t;
                ki = items;
                kz = zc;
                kt = threads;
              }
            }
          }
        stencil_tune_set(g.dim, g.nn, key, word, ki, kz, kt);
        // the same kernel on in-plane tiles (3D); it needs a valid row-run
        // entry beside it, which switches the fused smoothers on
        double tbest = 1e30;
        int ti = 0, tz = 0, tt = 256;
        const int tkey = key == kMgPreKey ? kMgPreTileKey : kMgPostTileKey;
        if (g.dim == 3 && ki) {
          for (int threads : {256, 512})
            for (int items = 1; items <= 2; items++) {
              TileGeom tg;
              if (!cheb2_tile_geom(g, threads, items, tg)) continue;
              for (int zc : zchunk_candidates_n(g, (int64_t)tg.ntx * tg.nty, B.count)) {
                stencil_tune_set(g.dim, g.nn, tkey, word, items, zc, threads);
                double t = time_best(st, [&]() {
                  return key == kMgPreKey
                             ? launch_mg_pre2<P>(g, B, l, cst(bb), x, r, st)
                             : launch_mg_post2<P>(g, B, l, cst(bb), cst(x), d1, st);
                });
                if (t < tbest) {
                  tbest = t;
                  ti = items;
                  tz = zc;
                  tt = threads;
                }
              }
            }
          stencil_tune_set(g.dim, g.nn, tkey, word, 0, 0);
          if (ti && tbest < kbest) stencil_tune_set(g.dim, g.nn, tkey, word, ti, tz, tt);
        }
        // and on overlapping windows with a column strip per thread (3D)
        double sbest = 1e30;
        int si = 0, sz = 0;
        const int skey = key == kMgPreKey ? kMgPreStripKey : kMgPostStripKey;
        if (g.dim == 3 && ki) {
          for (int cfg = 1; cfg <= kStripConfigs; cfg++)
            for (int zc : zchunk_candidates_n(g, strip_windows(g, cfg), B.count)) {
              stencil_tune_set(g.dim, g.nn, skey, word, cfg, zc, strip_threads(cfg));
              double t = time_best(st, [&]() {
                return key == kMgPreKey
                           ? launch_mg_pre2<P>(g, B, l, cst(bb), x, r, st)
                           : launch_mg_post2<P>(g, B, l, cst(bb), cst(x), d1, st);
              });
              if (t < sbest) {
                sbest = t;
                si = cfg;
                sz = zc;
              }
            }
          stencil_tune_set(g.dim, g.nn, skey, word, 0, 0);
          if (si && sbest < std::min(kbest, tbest))
            stencil_tune_set(g.dim, g.nn, skey, word, si, sz, strip_threads(si));
        }
        fused += ki ? std::min(std::min(kbest, tbest), sbest) : 1e30;
      }
      if (!(fused < unfused)) {
        stencil_tune_set(g.dim, g.nn, kMgPreKey, word, 0, 0);
        stencil_tune_set(g.dim, g.nn, kMgPostKey, word, 0, 0);
        stencil_tune_set(g.dim, g.nn, kMgPreTileKey, word, 0, 0);
        stencil_tune_set(g.dim, g.nn, kMgPostTileKey, word, 0, 0);
        stencil_tune_set(g.dim, g.nn, kMgPreStripKey, word, 0, 0);
        stencil_tune_set(g.dim, g.nn, kMgPostStripKey, word, 0, 0);
      }
      (*entries)++;
    }
  }
  stencil_tune_set(c.lev[0].dim, c.lev[0].nn, kFusedKey, word, 0, 0);
  stencil_tune_set(c.lev[0].dim, c.lev[0].nn, kFusedTileKey, word, 0, 0);
  stencil_tune_set(c.lev[0].dim, c.lev[0].nn, kFusedStripKey, word, 0, 0);
  if (cheb_fusion_on(c.lev[0], word)) {  // fused pairs of Chebyshev iterations on M
    const Grid& g = c.lev[0];
    const int64_t nl = g.nodes;
    Vec<P> x = pvec<P>(c.yv, nl), r = pvec<P>(c.cr, nl), d0 = pvec<P>(c.cda, nl),
           d1 = pvec<P>(c.cdb, nl);
    double best = 1e30;
    int bi = 0, bz = 0, bt = 256;
    for (int threads : {256, 512})
      for (int items = 1; items <= 2; items++) {
        if (!cheb2_shape_ok(g.dim, items, threads)) continue;
        for (int zc : zchunk_candidates(g, items * threads, B.count)) {
          stencil_tune_set(g.dim, g.nn, kFusedKey, word, items, zc, threads);
          if (!cheb_fusion_on(g, word)) continue;
          double t = time_best(st, [&]() {
            return launch_cheb_step2<P>(g, B, 1, CF_ONE, false, x, cst(r), pvec<P>(c.cr2, nl),
                                        cst(d0), d1, st);
          });
          if (t < best) {
            best = t;
            bi = items;
            bz = zc;
            bt = threads;
          }
        }
      }
    // the same pairs on rectangular in-plane tiles (3D)
    double tbest = 1e30;
    int ti = 0, tz = 0, tt = 256;
    stencil_tune_set(g.dim, g.nn, kFusedKey, word, bi, bz, bt);  // bi = 0: built-in shape
    if (g.dim == 3) {
      for (int threads : {256, 512})
        for (int items = 1; items <= 2; items++) {
          TileGeom tg;
          if (!cheb2_tile_geom(g, threads, items, tg)) continue;
          for (int zc : zchunk_candidates_n(g, (int64_t)tg.ntx * tg.nty, B.count)) {
            stencil_tune_set(g.dim, g.nn, kFusedTileKey, word, items, zc, threads);
            double t = time_best(st, [&]() {
              return launch_cheb_step2<P>(g, B, 1, CF_ONE, false, x, cst(r),
                                          pvec<P>(c.cr2, nl), cst(d0), d1, st);
            });
            if (t < tbest) {
              tbest = t;
              ti = items;
              tz = zc;
              tt = threads;
            }
          }
        }
      stencil_tune_set(g.dim, g.nn, kFusedTileKey, word, 0, 0);
    }
    // and on overlapping windows with a column strip per thread (3D)
    double sbest = 1e30;
    int si = 0, sz = 0;
    if (g.dim == 3) {
      for (int cfg = 1; cfg <= kStripConfigs; cfg++)
        for (int zc : zchunk_candidates_n(g, strip_windows(g, cfg), B.count)) {
          stencil_tune_set(g.dim, g.nn, kFusedStripKey, word, cfg, zc, strip_threads(cfg));
          double t = time_best(st, [&]() {
            return launch_cheb_step2<P>(g, B, 1, CF_ONE, false, x, cst(r), pvec<P>(c.cr2, nl),
                                        cst(d0), d1, st);
          });
          if (t < sbest) {
            sbest = t;
            si = cfg;
            sz = zc;
          }
        }
      stencil_tune_set(g.dim, g.nn, kFusedStripKey, word, 0, 0);
    }
    // keep the fusion only where a pair beats two single iterations on M
    const double single = time_best(st, [&]() {
      hipError_t e = launch_cheb_step<P>(g, B, -1, 1, CF_ONE, false, x, r, cst(d0), d1, st);
      if (e == hipSuccess)
        e = launch_cheb_step<P>(g, B, -1, 2, CF_ONE, false, x, r, cst(d1), d0, st);
      return e;
    });
    if ((bi && best < single) || (ti && tbest < single) || (si && sbest < single)) {
      if (si && sbest < std::min(best, tbest))
        stencil_tune_set(g.dim, g.nn, kFusedStripKey, word, si, sz, strip_threads(si));
      else if (ti && tbest < best)
        stencil_tune_set(g.dim, g.nn, kFusedTileKey, word, ti, tz, tt);
    } else {
      stencil_tune_set(g.dim, g.nn, kFusedKey, word, -1, 0);
    }
    (*entries)++;
  }
  {
    const Grid& g = c.lev[0];
    Vec<const P> z{(const P*)c.Z, sZ(c)};
    const double cf[2][4] = {{1.0, 0.0, 0.0, 1.0}, {1.0, -1.0, 1.0, 0.0}};
    const int ff[2][4] = {{CF_SA, CF_ONE, CF_ONE, CF_DTH}, {CF_ONE, CF_E2, CF_ONE, CF_ONE}};
    double best = 1e30;
    int bi = 0, bz = 0;
    for (int items = 1; items <= 4; items *= 2)
      for (int zc : zchunk_candidates(g, items * 256, B.count)) {
        stencil_tune_set(g.dim, g.nn, 2, word, items, zc);
        double t = time_best(st, [&]() {
          return launch_stencil_lin2<P>(g, B, z, off(z, c.n), Vec<const double>{nullptr, 0},
                                        Vec<const double>{c.G, c.n}, cf, ff, vec(c.T1, c.n2()),
                                        off(vec(c.T1, c.n2()), c.n), st);
        });
        if (t < best) {
          best = t;
          bi = items;
          bz = zc;
        }
      }
    stencil_tune_set(g.dim, g.nn, 2, word, bi, bz);
    if (bi) (*entries)++;
  }
  return OK_SUCCESS;
}

}  // namespace

int autotune_class(ClassCtx& c, hipStream_t st, int* entries) {
  if (c.ex) c.ex->clear_graphs();  // captured launch shapes would be stale
  int n = 0;
  int e = c.mixed ? autotune_impl<float>(c, st, &n) : autotune_impl<double>(c, st, &n);
  if (entries) *entries = n;
  if (e) return e;
  OKE(c, hipStreamSynchronize(st));
  return OK_SUCCESS;
}

}  // namespace okd
