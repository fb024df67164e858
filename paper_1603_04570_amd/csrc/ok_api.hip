// C ABI of libok.so: problem setup, the block preconditioner, flexible GMRES,
// Newton and the timestep loop.  Host code only orchestrates; every vector
// operation runs in the HIP kernels of this library.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ok_internal.h"

using namespace okd;

namespace {

struct ProfPair {
  hipEvent_t a, b;
  double bytes;
  int count;  // kernel launches between the two events
};

}  // namespace

struct ok_ctx {
  ok_params p;
  int dim = 0, L = 0;
  bool mixed = false;
  Grid lev[kMaxLevels];
  Op opA[kMaxLevels];   // M_l + alpha K_l
  Cheb chA[kMaxLevels]; // smoother interval of D^-1 (M_l + alpha K_l)
  Op opM;               // M on the finest grid
  Cheb chM;             // [2^-d, (3/2)^d]
  double c = 0, alpha = 0, sA = 0, dth = 0;
  int64_t n = 0;        // finest nodes
  int m = 0;            // FGMRES restart length
  size_t psz = 8;       // bytes per preconditioner word
  // FP64 vectors
  double *V = nullptr, *X = nullptr, *B = nullptr, *T1 = nullptr, *un = nullptr, *wn = nullptr;
  double *G = nullptr, *pA = nullptr, *pB = nullptr;
  double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *ycoef = nullptr;
  double *scal = nullptr, *nrm = nullptr;
  // preconditioner-precision vectors (double or float)
  void* Z = nullptr;          // m x 2n
  void* zt = nullptr;         // 2n (ok_precond_apply staging in mixed mode)
  void *cr = nullptr, *cda = nullptr, *cdb = nullptr;
  void *y = nullptr, *t = nullptr, *s = nullptr;
  void* mg[kMaxLevels][5] = {};  // x, b, r, da, db
  // profiling
  int prof_class = OK_K_NONE;
  std::vector<ProfPair> prof;
  size_t prof_used = 0;
  int64_t prof_launches = 0;
  double prof_ms = 0.0, prof_bytes = 0.0;
  std::string err;
};

namespace {

const char* kStatusNames[] = {"success", "invalid argument", "workspace too small or misaligned",
                              "HIP error", "FGMRES did not converge",
                              "Newton did not converge", "non-finite value"};

int fail(ok_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define OK_HIP(ctx, ...)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (__VA_ARGS__);                                                         \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, OK_E_HIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
  } while (0)

int levels_for(const ok_params* p) {
  if (p->mg_levels > 0) return p->mg_levels;
  int L = 1, n = p->n;
  while (n > 8 && n % 2 == 0 && L < kMaxLevels) {
    n /= 2;
    L++;
  }
  return L;
}

int validate(const ok_params* p, std::string& why) {
  if (!p) { why = "null params"; return OK_E_INVALID; }
  if (p->dim != 2 && p->dim != 3) { why = "dim must be 2 or 3"; return OK_E_INVALID; }
  if (p->n < 2) { why = "n must be >= 2"; return OK_E_INVALID; }
  if (p->dim == 3 && p->n > 512) { why = "3D n must be <= 512"; return OK_E_INVALID; }
  if (p->dim == 2 && p->n > 2048) { why = "2D n must be <= 2048"; return OK_E_INVALID; }
  if (!(p->eps > 0) || !std::isfinite(p->eps)) { why = "eps must be > 0"; return OK_E_INVALID; }
  if (!(p->sigma >= 0) || !std::isfinite(p->sigma)) { why = "sigma must be >= 0"; return OK_E_INVALID; }
  if (!(std::fabs(p->m) < 1)) { why = "|m| must be < 1"; return OK_E_INVALID; }
  if (!(p->dt > 0) || !std::isfinite(p->dt)) { why = "dt must be > 0"; return OK_E_INVALID; }
  if (!(p->theta > 0 && p->theta <= 1)) { why = "theta must be in (0,1]"; return OK_E_INVALID; }
  if (p->precision != OK_FP64 && p->precision != OK_MIXED) { why = "bad precision"; return OK_E_INVALID; }
  if (p->gmres_restart < 1 || p->gmres_restart > 64) { why = "gmres_restart in 1..64"; return OK_E_INVALID; }
  if (p->gmres_max_restarts < 0) { why = "gmres_max_restarts >= 0"; return OK_E_INVALID; }
  if (!(p->gmres_rtol > 0)) { why = "gmres_rtol > 0"; return OK_E_INVALID; }
  if (!(p->newton_atol >= 0)) { why = "newton_atol >= 0"; return OK_E_INVALID; }
  if (p->newton_max_it < 0) { why = "newton_max_it >= 0"; return OK_E_INVALID; }
  if (p->cheb_A_its < 1) { why = "cheb_A_its >= 1"; return OK_E_INVALID; }
  if (p->schur_richardson < 1) { why = "schur_richardson >= 1"; return OK_E_INVALID; }
  if (p->mg_pre < 1 || p->mg_post < 1 || p->mg_cycles < 1) { why = "mg_pre/post/cycles >= 1"; return OK_E_INVALID; }
  int L = levels_for(p);
  if (L < 1 || L > kMaxLevels) { why = "bad mg_levels"; return OK_E_INVALID; }
  if (p->n % (1 << (L - 1))) { why = "n not divisible by 2^(levels-1)"; return OK_E_INVALID; }
  int nc = p->n >> (L - 1);
  int64_t cn = (int64_t)(nc + 1) * (nc + 1) * (p->dim == 3 ? (nc + 1) : 1);
  if (nc < 1 || cn > 1024 || nc + 1 > 64) { why = "coarsest grid must have <= 1024 nodes"; return OK_E_INVALID; }
  return OK_SUCCESS;
}

// Bump allocator over the caller's workspace (base 0 -> size only).
struct Carver {
  char* base;
  size_t off = 0;
  void* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

void carve(ok_ctx* c, char* base, size_t* total) {
  Carver cv{base};
  const int64_t n = c->n, n2 = 2 * n;
  const int m = c->m;
  const size_t d8 = sizeof(double), ps = c->psz;
  c->V = (double*)cv.take(d8 * n2 * (m + 1));
  c->Z = cv.take(ps * n2 * m);
  c->X = (double*)cv.take(d8 * n2);
  c->B = (double*)cv.take(d8 * n2);
  c->T1 = (double*)cv.take(d8 * n2);
  c->un = (double*)cv.take(d8 * n);
  c->wn = (double*)cv.take(d8 * n);
  c->G = (double*)cv.take(d8 * n);
  c->zt = c->mixed ? cv.take(ps * n2) : nullptr;
  c->cr = cv.take(ps * n);
  c->cda = cv.take(ps * n);
  c->cdb = cv.take(ps * n);
  c->y = cv.take(ps * n);
  c->t = cv.take(ps * n);
  c->s = cv.take(ps * n);
  for (int l = 0; l < c->L; l++) {
    int64_t nl = c->lev[l].nodes;
    for (int k = 0; k < 5; k++) {
      if (l == 0 && k < 2) { c->mg[l][k] = nullptr; continue; }
      c->mg[l][k] = cv.take(ps * nl);
    }
  }
  c->pA = (double*)cv.take(d8 * kRedBlocks);
  c->pB = (double*)cv.take(d8 * kRedBlocks);
  c->H = (double*)cv.take(d8 * (m + 1) * m);
  c->cs = (double*)cv.take(d8 * (m + 1));
  c->sn = (double*)cv.take(d8 * (m + 1));
  c->g = (double*)cv.take(d8 * (m + 1));
  c->ycoef = (double*)cv.take(d8 * (m + 1));
  c->scal = (double*)cv.take(d8 * 8);
  c->nrm = (double*)cv.take(d8 * 8);
  *total = (cv.off + 255) & ~(size_t)255;
}

// D^-1 (M + alpha K) on the DCT-I mode with cosines c_d; numerator and
// denominator of the closed form (both multilinear in c).
double dct_lambda(const Grid& g, double alpha, const double* c) {
  double h = g.h, num = 1.0, sk = 0.0;
  for (int d = 0; d < g.dim; d++) num *= (h / 3.0) * (2.0 + c[d]);
  for (int d = 0; d < g.dim; d++) {
    double t = (2.0 / h) * (1.0 - c[d]);
    for (int e = 0; e < g.dim; e++)
      if (e != d) t *= (h / 3.0) * (2.0 + c[e]);
    sk += t;
  }
  double mi = 2.0 * h / 3.0, den = std::pow(mi, g.dim) + alpha * g.dim * (2.0 / h) * std::pow(mi, g.dim - 1);
  return (num + alpha * sk) / den;
}

// Smoother interval: the largest eigenvalue of D^-1 A (a corner of the
// cosine box, since the eigenvalue is multilinear in the cosines) and the
// smallest one over the upper half of the spectrum (vertices with some
// cosine in {-1, 0}); exact for Q1 on uniform grids with Neumann ends.
Cheb smoother_interval(const Grid& g, double alpha) {
  double lo = 1e300, hi = -1e300;
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
  Cheb ch;
  ch.theta = 0.5 * (hi + lo);
  ch.delta = 0.5 * (hi - lo);
  ch.sigma1 = ch.theta / ch.delta;
  return ch;
}

// ---------------------------------------------------------------------------
// Profiling of one kernel class with HIP events on the launch stream.
// ---------------------------------------------------------------------------
struct ProfScope {
  ok_ctx* c;
  bool on;
  ProfPair* pp = nullptr;
  hipStream_t st;
  ProfScope(ok_ctx* cc, int cls, double bytes, hipStream_t s, int count = 1) : c(cc), st(s) {
    on = (c->prof_class == cls) || (c->prof_class == OK_K_STENCIL_ANY && cls != OK_K_KRYLOV &&
                                     cls != OK_K_ELEMENT);
    if (!on) return;
    if (c->prof_used == c->prof.size()) {
      ProfPair p{};
      (void)hipEventCreate(&p.a);
      (void)hipEventCreate(&p.b);
      c->prof.push_back(p);
    }
    pp = &c->prof[c->prof_used++];
    pp->bytes = bytes;
    pp->count = count;
    (void)hipEventRecord(pp->a, st);
  }
  ~ProfScope() {
    if (on) (void)hipEventRecord(pp->b, st);
  }
};

// ---------------------------------------------------------------------------
// Preconditioner pieces, templated on the precision P of its vectors.
// ---------------------------------------------------------------------------
// Chebyshev drivers (Saad, Alg. 12.1): rho_0 = 1/sigma1, rho_{k+1} =
// 1/(2 sigma1 - rho_k), d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1}/delta) D^-1 r_{k+1}.
// `cls` tags the launches for profiling; `step_cls` tags the middle iterations.
struct ChebRho {
  double rho, s1, de;
  explicit ChebRho(const Cheb& c) : rho(1.0 / c.sigma1), s1(c.sigma1), de(c.delta) {}
  void next(double& c1, double& c2) {
    double rho1 = 1.0 / (2.0 * s1 - rho);
    c1 = rho1 * rho;
    c2 = 2.0 * rho1 / de;
    rho = rho1;
  }
};

// K iterations from x0 = 0: x = out_scale * x_K.
template <class TB, class P>
int cheb_zero(ok_ctx* c, int cls, int step_cls, const Grid& g, const Op& A, const Cheb& ch, int K,
              const TB* b, P* x, P* r, P* da, P* db, double out_scale, hipStream_t st) {
  const double w = (double)c->psz * g.nodes, wb = (double)sizeof(TB) * g.nodes;
  const double it = 1.0 / ch.theta;
  if (K <= 1) {
    ProfScope ps(c, cls, wb + w, st);
    OK_HIP(c, launch_cheb_one<TB, P>(g, A, it, out_scale, b, x, st));
    return OK_SUCCESS;
  }
  ChebRho rr(ch);
  double c1, c2;
  rr.next(c1, c2);
  {
    ProfScope ps(c, cls, wb + (K == 2 ? w : 3.0 * w), st);
    OK_HIP(c, launch_cheb_first<TB, P>(g, A, it, c1, c2, out_scale, K == 2, b, x, r, da, st));
  }
  if (K == 2) return OK_SUCCESS;
  P* dc = da;
  P* dn = db;
  // middle iterations (x, r, d -> x, r, d) back to back, timed as one run
  {
    const int mid = K > 3 ? K - 3 : 0;
    ProfScope ps(c, step_cls, 6.0 * w * mid, st, mid);
    for (int k = 1; k <= K - 3; k++) {
      rr.next(c1, c2);
      OK_HIP(c, launch_cheb_step<P>(g, A, c1, c2, out_scale, false, x, r, dc, dn, st));
      P* t = dc;
      dc = dn;
      dn = t;
    }
  }
  {
    rr.next(c1, c2);
    ProfScope ps(c, cls, 4.0 * w, st);
    OK_HIP(c, launch_cheb_step<P>(g, A, c1, c2, out_scale, true, x, r, dc, dn, st));
  }
  return OK_SUCCESS;
}

// K iterations from the x passed in (updated in place).
template <class P>
int cheb_from(ok_ctx* c, int cls, const Grid& g, const Op& A, const Cheb& ch, int K, const P* b,
              P* x, P* r, P* da, P* db, hipStream_t st) {
  const double w = (double)c->psz * g.nodes;
  {
    ProfScope ps(c, cls, 4.0 * w, st);
    OK_HIP(c, launch_cheb_start<P>(g, A, 1.0 / ch.theta, b, x, r, da, st));
  }
  if (K <= 1) {
    OK_HIP(c, launch_add_inplace<P>(x, da, g.nodes, st));
    return OK_SUCCESS;
  }
  ChebRho rr(ch);
  double c1, c2;
  P* dc = da;
  P* dn = db;
  for (int k = 0; k <= K - 2; k++) {
    rr.next(c1, c2);
    const bool last = (k == K - 2);
    ProfScope ps(c, cls, last ? 4.0 * w : 6.0 * w, st);
    OK_HIP(c, launch_cheb_step<P>(g, A, c1, c2, 1.0, last, x, r, dc, dn, st));
    P* t = dc;
    dc = dn;
    dn = t;
  }
  return OK_SUCCESS;
}

template <class P>
int mg_vcycle(ok_ctx* c, int l, const P* b, P* x, bool zero_start, hipStream_t st) {
  const Grid& g = c->lev[l];
  if (l == c->L - 1) {
    OK_HIP(c, launch_coarse_solve<P>(g, c->alpha, b, x, st));
    return OK_SUCCESS;
  }
  P* r = (P*)c->mg[l][2];
  P* da = (P*)c->mg[l][3];
  P* db = (P*)c->mg[l][4];
  const double w = (double)c->psz * g.nodes;
  const int cls = (l == 0) ? OK_K_MG_SMOOTH : OK_K_NONE;
  int e = zero_start ? cheb_zero<P, P>(c, cls, cls, g, c->opA[l], c->chA[l], c->p.mg_pre, b, x, r,
                                       da, db, 1.0, st)
                     : cheb_from<P>(c, cls, g, c->opA[l], c->chA[l], c->p.mg_pre, b, x, r, da, db,
                                    st);
  if (e) return e;
  {
    ProfScope ps(c, cls, 3.0 * w, st);
    OK_HIP(c, launch_resid<P>(g, c->opA[l], b, x, r, st));
  }
  const Grid& gc = c->lev[l + 1];
  P* bc = (P*)c->mg[l + 1][1];
  P* xc = (P*)c->mg[l + 1][0];
  OK_HIP(c, launch_restrict<P>(g, gc, r, bc, st));
  e = mg_vcycle<P>(c, l + 1, bc, xc, true, st);
  if (e) return e;
  OK_HIP(c, launch_prolong_add<P>(g, gc, xc, x, st));
  return cheb_from<P>(c, cls, g, c->opA[l], c->chA[l], c->p.mg_post, b, x, r, da, db, st);
}

template <class P>
int mg_apply(ok_ctx* c, const P* b, P* x, int cycles, hipStream_t st) {
  for (int k = 0; k < cycles; k++) {
    int e = mg_vcycle<P>(c, 0, b, x, k == 0, st);
    if (e) return e;
  }
  return OK_SUCCESS;
}

// z = [z1; z2] = P^-1 [r1; r2] with u the current Newton iterate.
template <class P>
int precond(ok_ctx* c, const double* u, const double* r, P* z, hipStream_t st) {
  const Grid& g = c->lev[0];
  const int64_t n = c->n;
  const double* r1 = r;
  const double* r2 = r + n;
  P* z1 = z;
  P* z2 = z + n;
  P* cr = (P*)c->cr;
  P* cda = (P*)c->cda;
  P* cdb = (P*)c->cdb;
  // z1 = A~^-1 r1: Chebyshev on M, scaled by 1/(1 + dt th sigma).
  {
    int e = cheb_zero<double, P>(c, OK_K_NONE, OK_K_CHEB_MASS, g, c->opM, c->chM, c->p.cheb_A_its,
                                 r1, z1, cr, cda, cdb, 1.0 / c->sA, st);
    if (e) return e;
  }
  // y = r2 - C z1 = r2 + eps^2 K z1 + M_E(u) z1  (M_E in FP64)
  {
    ProfScope ps(c, OK_K_ELEMENT, (double)n * (8.0 + 8.0 + c->psz + 8.0), st);
    OK_HIP(c, launch_element<P, double>(g, 0, u, z1, r2, 3.0, 1.0, c->G, st));  // 3G + r2
  }
  P* y = (P*)c->y;
  // y = r2 + 3G - M z1 + eps^2 K z1 = r2 + M_E z1 + eps^2 K z1
  OK_HIP(c, launch_stencil_axpy<P, double, P>(g, z1, c->G, -1.0, c->p.eps * c->p.eps, y, st));
  if (c->p.schur_richardson > 1) return fail(c, OK_E_INVALID, "schur_richardson > 1 not built");
  // z2 = S^^-1 M S^^-1 y
  P* t = (P*)c->t;
  P* s = (P*)c->s;
  int e = mg_apply<P>(c, y, t, c->p.mg_cycles, st);
  if (e) return e;
  OK_HIP(c, launch_mass<P, P>(g, t, s, 1.0, st));
  return mg_apply<P>(c, s, z2, c->p.mg_cycles, st);
}

// y = J(u) x for x of type TX (2n), y FP64 (2n).
template <class TX>
int jac_apply(ok_ctx* c, const double* u, const TX* x, double* y, hipStream_t st) {
  const Grid& g = c->lev[0];
  const int64_t n = c->n;
  const TX* x1 = x;
  const TX* x2 = x + n;
  double* y1 = y;
  double* y2 = y + n;
  const double e2 = c->p.eps * c->p.eps;
  {
    ProfScope ps(c, OK_K_ELEMENT, (double)n * (8.0 + sizeof(TX) + 8.0), st);
    OK_HIP(c, launch_element<TX, double>(g, 0, u, x1, nullptr, -3.0, 0.0, c->G, st));  // -3G
  }
  // y1 = sA M x1 + dt th K x2;
  // y2 = -M_E x1 - eps^2 K x1 + M x2 = -3G + M x1 - eps^2 K x1 + M x2
  const double c0[4] = {c->sA, 0.0, 0.0, c->dth};
  const double c1[4] = {1.0, -e2, 1.0, 0.0};
  {
    ProfScope ps(c, OK_K_NONE, (double)n * (2.0 * sizeof(TX) + 3.0 * 8.0), st);
    OK_HIP(c, launch_stencil_lin2<TX>(g, x1, x2, nullptr, c->G, c0, c1, y1, y2, st));
  }
  return OK_SUCCESS;
}

int residual(ok_ctx* c, const double* u, const double* w, const double* un, const double* wn,
             double* F, double* norm, hipStream_t st) {
  const Grid& g = c->lev[0];
  const int64_t n = c->n;
  const ok_params& p = c->p;
  double* t1 = c->T1;
  double* t2 = c->T1 + n;
  OK_HIP(c, launch_residual_prep(u, un, w, (p.theta < 1.0) ? wn : nullptr, p.dt, p.sigma,
                                 p.theta, p.m, t1, t2, n, st));
  double* F1 = F;
  double* F2 = F + n;
  const double a0[4] = {1.0, 0.0, 0.0, 1.0};  // F1 = M t1 + K t2
  OK_HIP(c, launch_stencil_lin2<double>(g, t1, t2, nullptr, nullptr, a0, nullptr, F1, nullptr, st));
  OK_HIP(c, launch_element<double, double>(g, 1, u, (const double*)nullptr, nullptr, -1.0, 0.0,
                                           c->G, st));
  const double b0[4] = {1.0, 0.0, 0.0, -p.eps * p.eps};  // F2 = -N(u) + M w - eps^2 K u
  OK_HIP(c, launch_stencil_lin2<double>(g, w, u, c->G, nullptr, b0, nullptr, F2, nullptr, st));
  if (norm) {
    OK_HIP(c, launch_dot_partial(F, F, 2 * n, c->pA, st));
    OK_HIP(c, launch_reduce_final(c->pA, c->nrm, st));
    double h[2];
    OK_HIP(c, hipMemcpyAsync(h, c->nrm, sizeof(h), hipMemcpyDeviceToHost, st));
    OK_HIP(c, hipStreamSynchronize(st));
    *norm = h[1];
  }
  return OK_SUCCESS;
}

template <class P>
int fgmres_impl(ok_ctx* c, const double* u, const double* b, double* x, int32_t* its_out,
                int32_t* restarts_out, double* lin_res, hipStream_t st) {
  const int64_t n2 = 2 * c->n;
  const int m = c->m;
  P* Z = (P*)c->Z;
  int its = 0, restarts = 0;
  int status = OK_E_GMRES_MAXIT;
  double hbuf[2];
  auto finish = [&](int s) {
    if (its_out) *its_out = its;
    if (restarts_out) *restarts_out = restarts;
    return s;
  };
  OK_HIP(c, launch_fill(x, 0.0, n2, st));
  OK_HIP(c, launch_dot_partial(b, b, n2, c->pA, st));
  OK_HIP(c, launch_reduce_final(c->pA, c->nrm, st));
  OK_HIP(c, hipMemcpyAsync(hbuf, c->nrm, sizeof(hbuf), hipMemcpyDeviceToHost, st));
  OK_HIP(c, hipStreamSynchronize(st));
  const double bnorm = hbuf[1];
  if (lin_res) *lin_res = 0.0;
  if (!std::isfinite(bnorm)) return finish(fail(c, OK_E_NONFINITE, "non-finite right-hand side"));
  if (bnorm == 0.0) return finish(OK_SUCCESS);
  const double tol = c->p.gmres_rtol * bnorm;
  double beta = bnorm;
  const double* src = b;
  for (int cycle = 0; cycle <= c->p.gmres_max_restarts; cycle++) {
    if (cycle > 0) restarts++;
    OK_HIP(c, launch_scale_inv(src, c->V, c->nrm, n2, st));
    OK_HIP(c, launch_fill(c->g, 0.0, m + 1, st));
    OK_HIP(c, launch_fill(c->g, beta, 1, st));
    int k = 0;
    bool conv = false;
    double res = beta;
    for (int j = 0; j < m; j++) {
      double* vj = c->V + (int64_t)j * n2;
      double* wv = c->V + (int64_t)(j + 1) * n2;
      P* zj = Z + (int64_t)j * n2;
      int e = precond<P>(c, u, vj, zj, st);
      if (e) return finish(e);
      e = jac_apply<P>(c, u, zj, wv, st);
      if (e) return finish(e);
      double* pin = c->pA;
      double* pout = c->pB;
      {
        ProfScope ps(c, OK_K_KRYLOV, 16.0 * n2, st);
        OK_HIP(c, launch_dot_partial(wv, c->V, n2, pin, st));
      }
      for (int i = 0; i <= j; i++) {
        const double* vi = c->V + (int64_t)i * n2;
        const double* vn = (i < j) ? c->V + (int64_t)(i + 1) * n2 : nullptr;
        ProfScope ps(c, OK_K_KRYLOV, (vn ? 32.0 : 24.0) * n2, st);
        OK_HIP(c, launch_mgs_step(wv, vi, vn, n2, pin, pout, c->H + (int64_t)j * (m + 1) + i, st));
        double* tt = pin;
        pin = pout;
        pout = tt;
      }
      OK_HIP(c, launch_givens(j, m, c->H, c->cs, c->sn, c->g, pin, c->scal, st));
      OK_HIP(c, hipMemcpyAsync(hbuf, c->scal, sizeof(hbuf), hipMemcpyDeviceToHost, st));
      OK_HIP(c, hipStreamSynchronize(st));
      its++;
      k = j + 1;
      res = hbuf[0];
      const double hn = hbuf[1];
      if (!std::isfinite(hn) || !std::isfinite(res))
        return finish(fail(c, OK_E_NONFINITE, "non-finite value in the Arnoldi recurrence"));
      if (res <= tol || hn == 0.0) {
        conv = true;
        break;
      }
      OK_HIP(c, launch_scale_by(wv, wv, c->scal, n2, st));
    }
    OK_HIP(c, launch_lsq_update<P>(k, m, c->H, c->g, c->ycoef, Z, n2, x, n2, st));
    if (lin_res) *lin_res = res / bnorm;
    if (conv) {
      status = OK_SUCCESS;
      break;
    }
    // restart from the true residual r = b - J x
    int e = jac_apply<double>(c, u, x, c->T1, st);
    if (e) return finish(e);
    OK_HIP(c, launch_axpby(1.0, b, -1.0, c->T1, c->T1, n2, st));
    OK_HIP(c, launch_dot_partial(c->T1, c->T1, n2, c->pA, st));
    OK_HIP(c, launch_reduce_final(c->pA, c->nrm, st));
    OK_HIP(c, hipMemcpyAsync(hbuf, c->nrm, sizeof(hbuf), hipMemcpyDeviceToHost, st));
    OK_HIP(c, hipStreamSynchronize(st));
    beta = hbuf[1];
    if (lin_res) *lin_res = beta / bnorm;
    if (!std::isfinite(beta)) return finish(fail(c, OK_E_NONFINITE, "non-finite restart residual"));
    if (beta <= tol) {
      status = OK_SUCCESS;
      break;
    }
    src = c->T1;
  }
  if (status == OK_E_GMRES_MAXIT) fail(c, status, "FGMRES reached gmres_max_restarts");
  return finish(status);
}

int fgmres_dispatch(ok_ctx* c, const double* u, const double* b, double* x, int32_t* its,
                    int32_t* restarts, double* lin_res, hipStream_t st) {
  if (c->mixed) return fgmres_impl<float>(c, u, b, x, its, restarts, lin_res, st);
  return fgmres_impl<double>(c, u, b, x, its, restarts, lin_res, st);
}

// One Newton update given F already in c->B: solve J dx = -F, (u,w) += dx.
int newton_update(ok_ctx* c, double* u, double* w, int32_t* its, int32_t* restarts,
                  double* lin_res, hipStream_t st) {
  const int64_t n = c->n;
  OK_HIP(c, launch_copy_scale<double, double>(c->B, c->B, -1.0, 2 * n, st));
  int e = fgmres_dispatch(c, u, c->B, c->X, its, restarts, lin_res, st);
  if (e == OK_E_NONFINITE || e == OK_E_HIP || e == OK_E_INVALID) return e;
  OK_HIP(c, launch_axpby(1.0, u, 1.0, c->X, u, n, st));
  OK_HIP(c, launch_axpby(1.0, w, 1.0, c->X + n, w, n, st));
  return e;
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

}  // namespace

extern "C" {

int ok_default_params(ok_params* p) {
  if (!p) return OK_E_INVALID;
  p->dim = 3;
  p->n = 128;
  p->eps = 0.01;
  p->sigma = 1000.0;
  p->m = 0.1;
  p->dt = 2e-5;
  p->theta = 1.0;
  p->precision = OK_FP64;
  p->gmres_restart = 30;
  p->gmres_max_restarts = 10;
  p->gmres_rtol = 1e-8;
  p->newton_atol = 1e-10;
  p->newton_max_it = 25;
  p->cheb_A_its = 10;
  p->schur_richardson = 1;
  p->mg_levels = 0;
  p->mg_pre = 2;
  p->mg_post = 2;
  p->mg_cycles = 1;
  return OK_SUCCESS;
}

static void setup_levels(ok_ctx* c) {
  const ok_params& p = c->p;
  c->dim = p.dim;
  c->L = levels_for(&p);
  c->mixed = (p.precision == OK_MIXED);
  c->psz = c->mixed ? sizeof(float) : sizeof(double);
  c->m = p.gmres_restart;
  int n = p.n;
  for (int l = 0; l < c->L; l++) {
    c->lev[l] = make_grid(p.dim, n);
    n /= 2;
  }
  c->n = c->lev[0].nodes;
  // Sec. 2: c = dt theta / (1 + dt theta sigma), S^ = M + eps sqrt(c) K.
  c->dth = p.dt * p.theta;
  c->sA = 1.0 + c->dth * p.sigma;
  c->c = c->dth / c->sA;
  c->alpha = p.eps * std::sqrt(c->c);
  for (int l = 0; l < c->L; l++) {
    c->opA[l] = make_op(c->lev[l], 1.0, c->alpha);
    c->chA[l] = smoother_interval(c->lev[l], c->alpha);
  }
  c->opM = make_op(c->lev[0], 1.0, 0.0);
  // D^-1 M has spectrum [2^-d, (3/2)^d].
  double lo = std::pow(0.5, p.dim), hi = std::pow(1.5, p.dim);
  c->chM.theta = 0.5 * (hi + lo);
  c->chM.delta = 0.5 * (hi - lo);
  c->chM.sigma1 = c->chM.theta / c->chM.delta;
}

int ok_workspace_bytes(const ok_params* p, size_t* bytes) {
  std::string why;
  int v = validate(p, why);
  if (v) return v;
  if (!bytes) return OK_E_INVALID;
  ok_ctx c;
  c.p = *p;
  setup_levels(&c);
  carve(&c, nullptr, bytes);
  return OK_SUCCESS;
}

int ok_assemble_mesh(const ok_params* p, void* d_ws, size_t ws_bytes, void* stream,
                     ok_ctx** out) {
  (void)stream;
  if (!out) return OK_E_INVALID;
  *out = nullptr;
  std::string why;
  int v = validate(p, why);
  if (v) return v;
  ok_ctx* c = new (std::nothrow) ok_ctx();
  if (!c) return OK_E_INVALID;
  c->p = *p;
  setup_levels(c);
  size_t need = 0;
  carve(c, nullptr, &need);
  if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < need) {
    delete c;
    return OK_E_WORKSPACE;
  }
  carve(c, (char*)d_ws, &need);
  *out = c;
  return OK_SUCCESS;
}

int ok_destroy(ok_ctx* c) {
  if (!c) return OK_E_INVALID;
  for (auto& pp : c->prof) {
    (void)hipEventDestroy(pp.a);
    (void)hipEventDestroy(pp.b);
  }
  delete c;
  return OK_SUCCESS;
}

int ok_residual(ok_ctx* c, const double* u, const double* w, const double* un, const double* wn,
                double* F, double* h_norm, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !w || !un || (c->p.theta < 1.0 && !wn)) return fail(c, OK_E_INVALID, "null state");
  if (!aligned8(u) || !aligned8(w) || !aligned8(un) || !aligned8(F)) return fail(c, OK_E_INVALID, "misaligned");
  hipStream_t st = (hipStream_t)stream;
  double* dst = F ? F : c->B;
  double nrm = 0.0;
  int e = residual(c, u, w, un, wn, dst, h_norm ? &nrm : nullptr, st);
  if (e) return e;
  if (h_norm) *h_norm = nrm;
  return OK_SUCCESS;
}

int ok_jacobian_apply(ok_ctx* c, const double* u, const double* x, double* y, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !x || !y || x == y) return fail(c, OK_E_INVALID, "null or aliased vectors");
  if (!aligned8(u) || !aligned8(x) || !aligned8(y)) return fail(c, OK_E_INVALID, "misaligned");
  return jac_apply<double>(c, u, x, y, (hipStream_t)stream);
}

int ok_precond_apply(ok_ctx* c, const double* u, const double* r, double* z, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !r || !z || r == z) return fail(c, OK_E_INVALID, "null or aliased vectors");
  if (!aligned8(u) || !aligned8(r) || !aligned8(z)) return fail(c, OK_E_INVALID, "misaligned");
  hipStream_t st = (hipStream_t)stream;
  if (!c->mixed) return precond<double>(c, u, r, z, st);
  int e = precond<float>(c, u, r, (float*)c->zt, st);
  if (e) return e;
  OK_HIP(c, launch_copy_scale<float, double>((const float*)c->zt, z, 1.0, 2 * c->n, st));
  return OK_SUCCESS;
}

int ok_cheb_mass(ok_ctx* c, const double* r, double* x, void* stream) {
  if (!c || !r || !x) return OK_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  const Grid& g = c->lev[0];
  if (!c->mixed)
    return cheb_zero<double, double>(c, OK_K_NONE, OK_K_CHEB_MASS, g, c->opM, c->chM,
                                     c->p.cheb_A_its, r, x, (double*)c->cr, (double*)c->cda,
                                     (double*)c->cdb, 1.0, st);
  float* xf = (float*)c->zt;
  int e = cheb_zero<double, float>(c, OK_K_NONE, OK_K_CHEB_MASS, g, c->opM, c->chM,
                                   c->p.cheb_A_its, r, xf, (float*)c->cr, (float*)c->cda,
                                   (float*)c->cdb, 1.0, st);
  if (e) return e;
  OK_HIP(c, launch_copy_scale<float, double>(xf, x, 1.0, c->n, st));
  return OK_SUCCESS;
}

int ok_mg_apply(ok_ctx* c, const double* b, double* x, int32_t cycles, void* stream) {
  if (!c || !b || !x || b == x || cycles < 1) return OK_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  if (!c->mixed) return mg_apply<double>(c, b, x, cycles, st);
  float* bf = (float*)c->zt;
  float* xf = bf + c->n;
  OK_HIP(c, launch_copy_scale<double, float>(b, bf, 1.0, c->n, st));
  int e = mg_apply<float>(c, bf, xf, cycles, st);
  if (e) return e;
  OK_HIP(c, launch_copy_scale<float, double>(xf, x, 1.0, c->n, st));
  return OK_SUCCESS;
}

int ok_fgmres(ok_ctx* c, const double* u, const double* b, double* x, int32_t* its, void* stream) {
  if (!c || !u || !b || !x || b == x) return OK_E_INVALID;
  return fgmres_dispatch(c, u, b, x, its, nullptr, nullptr, (hipStream_t)stream);
}

int ok_newton_step(ok_ctx* c, double* u, double* w, const double* un, const double* wn,
                   ok_newton_info* info, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !w || !un || (c->p.theta < 1.0 && !wn)) return fail(c, OK_E_INVALID, "null state");
  hipStream_t st = (hipStream_t)stream;
  double nrm = 0.0;
  int e = residual(c, u, w, un, wn, c->B, &nrm, st);
  if (e) return e;
  ok_newton_info inf{};
  inf.fnorm = nrm;
  if (!std::isfinite(nrm)) {
    inf.status = fail(c, OK_E_NONFINITE, "non-finite residual");
    if (info) *info = inf;
    return inf.status;
  }
  e = newton_update(c, u, w, &inf.fgmres_its, &inf.restarts, &inf.lin_res, st);
  inf.status = e;
  if (info) *info = inf;
  if (e == OK_SUCCESS) OK_HIP(c, hipStreamSynchronize(st));
  return e;
}

int ok_timestep(ok_ctx* c, double* u, double* w, int32_t nsteps, ok_stats* stats, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !w || nsteps < 0) return fail(c, OK_E_INVALID, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  ok_stats S;
  std::memset(&S, 0, sizeof(S));
  const int64_t n = c->n;
  hipEvent_t e0, e1;
  OK_HIP(c, hipEventCreate(&e0));
  OK_HIP(c, hipEventCreate(&e1));
  int status = OK_SUCCESS;
  for (int s = 0; s < nsteps && status == OK_SUCCESS; s++) {
    OK_HIP(c, hipEventRecord(e0, st));
    OK_HIP(c, launch_copy_scale<double, double>(u, c->un, 1.0, n, st));
    OK_HIP(c, launch_copy_scale<double, double>(w, c->wn, 1.0, n, st));
    int newton = 0;
    for (;;) {
      double nrm = 0.0;
      int e = residual(c, u, w, c->un, c->wn, c->B, &nrm, st);
      if (e) { status = e; break; }
      if (S.fnorm_count < OK_HIST) S.fnorm[S.fnorm_count++] = nrm;
      if (!std::isfinite(nrm)) { status = fail(c, OK_E_NONFINITE, "non-finite residual"); break; }
      if (nrm <= c->p.newton_atol) break;
      if (newton >= c->p.newton_max_it) {
        status = fail(c, OK_E_NEWTON_MAXIT, "Newton reached newton_max_it");
        break;
      }
      int32_t its = 0, rs = 0;
      double lr = 0.0;
      e = newton_update(c, u, w, &its, &rs, &lr, st);
      if (S.newton_its < OK_HIST) S.fgmres_its[S.newton_its] = its;
      S.newton_its++;
      S.fgmres_its_total += its;
      newton++;
      if (e == OK_E_NONFINITE || e == OK_E_HIP || e == OK_E_INVALID) { status = e; break; }
    }
    OK_HIP(c, hipEventRecord(e1, st));
    OK_HIP(c, hipEventSynchronize(e1));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (s < OK_HIST) {
      S.newton_per_step[s] = newton;
      S.step_ms[s] = ms;
    }
    if (status == OK_SUCCESS) S.steps_done++;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  S.status = status;
  if (stats) *stats = S;
  return status;
}

}  // extern "C"

namespace {

// Time one candidate launch shape: one warm launch, then the best of three.
template <class F>
double time_best(hipStream_t st, F&& launch) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return 1e30;
  if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return 1e30; }
  double best = 1e30;
  if (launch() == hipSuccess) {
    for (int r = 0; r < 3; r++) {
      (void)hipEventRecord(a, st);
      if (launch() != hipSuccess) { best = 1e30; break; }
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

template <class P>
int autotune_impl(ok_ctx* c, hipStream_t st, int* entries) {
  const int zcs[4] = {4, 8, 16, 32};
  const int word = (int)sizeof(P);
  for (int l = 0; l < c->L; l++) {
    const Grid& g = c->lev[l];
    if (l == c->L - 1 && c->L > 1) break;  // the coarsest level is a direct solve
    P *x, *r, *d0, *d1;
    if (l == 0) {
      x = (P*)c->y; r = (P*)c->cr; d0 = (P*)c->cda; d1 = (P*)c->cdb;
    } else {
      x = (P*)c->mg[l][0]; r = (P*)c->mg[l][2]; d0 = (P*)c->mg[l][3]; d1 = (P*)c->mg[l][4];
    }
    const Op A = c->opA[l];
    double best = 1e30;
    int bi = 0, bz = 0;
    for (int items = 1; items <= 8; items *= 2)
      for (int zc : zcs) {
        if (zc > g.nn && zc != 4) continue;
        stencil_tune_set(g.dim, g.nn, 1, word, items, zc);
        double t = time_best(st, [&]() {
          return launch_cheb_step<P>(g, A, 0.5, 0.5, 1.0, false, x, r, d0, d1, st);
        });
        if (t < best) { best = t; bi = items; bz = zc; }
      }
    if (bi) { stencil_tune_set(g.dim, g.nn, 1, word, bi, bz); (*entries)++; }
    else stencil_tune_set(g.dim, g.nn, 1, word, 0, 0);
  }
  // two-field kernels (Jacobian apply) on the finest grid, for Z's precision
  {
    const Grid& g = c->lev[0];
    const P* z = (const P*)c->Z;
    const double c0[4] = {1.0, 0.0, 0.0, 1.0}, c1[4] = {0.0, 1.0, 1.0, 0.0};
    double best = 1e30;
    int bi = 0, bz = 0;
    for (int items = 1; items <= 4; items *= 2)
      for (int zc : zcs) {
        if (zc > g.nn && zc != 4) continue;
        stencil_tune_set(g.dim, g.nn, 2, word, items, zc);
        double t = time_best(st, [&]() {
          return launch_stencil_lin2<P>(g, z, z + c->n, nullptr, c->G, c0, c1, c->T1,
                                        c->T1 + c->n, st);
        });
        if (t < best) { best = t; bi = items; bz = zc; }
      }
    if (bi) { stencil_tune_set(g.dim, g.nn, 2, word, bi, bz); (*entries)++; }
    else stencil_tune_set(g.dim, g.nn, 2, word, 0, 0);
  }
  return OK_SUCCESS;
}

}  // namespace

extern "C" {

int ok_autotune(ok_ctx* c, void* stream, int32_t* entries) {
  if (!c) return OK_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  int n = 0;
  int e = c->mixed ? autotune_impl<float>(c, st, &n) : autotune_impl<double>(c, st, &n);
  if (entries) *entries = n;
  if (e) return e;
  OK_HIP(c, hipStreamSynchronize(st));
  return OK_SUCCESS;
}

int ok_profile_enable(ok_ctx* c, int32_t kernel_class) {
  if (!c) return OK_E_INVALID;
  c->prof_class = kernel_class;
  c->prof_used = 0;
  return OK_SUCCESS;
}

int ok_profile_read(ok_ctx* c, int64_t* launches, double* total_ms, double* bytes) {
  if (!c) return OK_E_INVALID;
  double ms = 0.0, by = 0.0;
  int64_t cnt = 0;
  for (size_t i = 0; i < c->prof_used; i++) {
    cnt += c->prof[i].count;
    (void)hipEventSynchronize(c->prof[i].b);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, c->prof[i].a, c->prof[i].b);
    ms += t;
    by += c->prof[i].bytes;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = ms;
  if (bytes) *bytes = by;
  c->prof_used = 0;
  return OK_SUCCESS;
}

const char* ok_error_string(int status) {
  int i = -status;
  if (i < 0 || i > 6) return "unknown status";
  return kStatusNames[i];
}

const char* ok_last_error(const ok_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
