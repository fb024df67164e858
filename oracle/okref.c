/*
 * okref.c -- plain FP64 CPU oracle for the Ohta-Kawasaki Newton-Krylov
 * timestep of Farrell & Pearson, "A preconditioner for the Ohta-Kawasaki
 * equation" (arXiv:1603.04570).
 *
 * TEST INFRASTRUCTURE ONLY: this file is the correctness reference that the
 * GPU library is compared against.  The product library never includes,
 * links or calls it.  It is serial, unblocked and assembles every operator
 * as a CSR matrix so that each step can be checked against the paper by eye:
 *
 *   Sec. 1, eqs. (oka)-(okb), (okbcs):  the PDE, natural Neumann BCs.
 *   Sec. 2, eq. (newton):               the theta-method residual F and its
 *                                        Jacobian J = [sA M, dt th K; -eps^2 K - M_E, M].
 *   Sec. 2, eq. (prec):                  block lower-triangular preconditioner.
 *   Sec. 2, eqs. (outer_approx),(schurinv): matching Schur approximation
 *                                        S~^-1 = S^^-1 M S^^-1, S^ = M + eps sqrt(c) K.
 *   Sec. 3 (after the second display):   A^-1 by Chebyshev semi-iteration.
 *   Sec. 4:                              GMRES outer solver; Richardson on S.
 *
 * Where the paper leaves a choice open, the readings are:
 *   Q1 elements on a uniform quad/hex grid of (0,1)^d; every integral is
 *   computed exactly with 3-point Gauss-Legendre per direction; Chebyshev
 *   with Jacobi (diagonal) preconditioning in Saad's three-vector form; the
 *   S^^-1 action by a geometric multigrid V(nu1,nu2) cycle with Chebyshev-
 *   Jacobi smoothing, R = P^T, rediscretised level operators and a dense
 *   Cholesky coarse solve; flexible GMRES(m) with modified Gram-Schmidt and
 *   Givens rotations, right preconditioned, zero initial guess; Newton from
 *   the previous time level with full steps.
 */
#include "okref.h"

/* Coarse grids up to this many nodes are solved with a dense Cholesky
 * factor; larger ones (e.g. 26^3 nodes when N = 25 * 2^k) with CG. */
#define OKREF_DENSE_COARSE 4096

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Mesh and quadrature                                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
  int dim, N, nn;     /* elements and nodes per direction */
  int64_t nodes;      /* nn^dim */
  double h;           /* 1/N */
} mesh_t;

static mesh_t mesh_make(int dim, int N) {
  mesh_t g;
  g.dim = dim;
  g.N = N;
  g.nn = N + 1;
  g.nodes = (dim == 2) ? (int64_t)g.nn * g.nn : (int64_t)g.nn * g.nn * g.nn;
  g.h = 1.0 / N;
  return g;
}

static void node_ijk(const mesh_t *g, int64_t idx, int *i, int *j, int *k) {
  *i = (int)(idx % g->nn);
  *j = (int)((idx / g->nn) % g->nn);
  *k = (g->dim == 3) ? (int)(idx / ((int64_t)g->nn * g->nn)) : 0;
}

static int64_t node_at(const mesh_t *g, int i, int j, int k) {
  return (int64_t)i + (int64_t)g->nn * ((int64_t)j + (int64_t)g->nn * k);
}

/* 3-point Gauss-Legendre on [0,1]: exact for polynomials of degree 5 per
 * direction.  The integrands (3u^2-1) phi_i phi_j and (u^3-u) phi_i are of
 * degree 4 per direction for multilinear u, so every integral is exact. */
static double GX[3], GW[3];
static void gauss_init(void) {
  GX[0] = 0.5 - sqrt(0.15);
  GX[1] = 0.5;
  GX[2] = 0.5 + sqrt(0.15);
  GW[0] = 5.0 / 18.0;
  GW[1] = 8.0 / 18.0;
  GW[2] = 5.0 / 18.0;
}

/* Local Q1 basis on the reference element: local node a has bits (ax,ay,az). */
static double phi1(int a, double xi) { return a ? xi : 1.0 - xi; }

typedef struct {
  int nq, nloc;             /* 3^d points, 2^d local nodes */
  double W[27];             /* weights, including h^d */
  double phi[27][8];        /* phi_a(x_q) */
  double grad[27][8][3];    /* d phi_a / d x (physical) */
} quad_t;

static void quad_make(const mesh_t *g, quad_t *Q) {
  int d = g->dim;
  Q->nq = (d == 2) ? 9 : 27;
  Q->nloc = (d == 2) ? 4 : 8;
  for (int q = 0; q < Q->nq; q++) {
    int qx = q % 3, qy = (q / 3) % 3, qz = q / 9;
    double xi[3] = {GX[qx], GX[qy], (d == 3) ? GX[qz] : 0.0};
    double w = GW[qx] * GW[qy] * g->h * g->h;
    if (d == 3) w *= GW[qz] * g->h;
    Q->W[q] = w;
    for (int a = 0; a < Q->nloc; a++) {
      int ab[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
      double p = 1.0;
      for (int e = 0; e < d; e++) p *= phi1(ab[e], xi[e]);
      Q->phi[q][a] = p;
      for (int e = 0; e < 3; e++) {
        double gr = 0.0;
        if (e < d) {
          gr = (ab[e] ? 1.0 : -1.0) / g->h;
          for (int f = 0; f < d; f++)
            if (f != e) gr *= phi1(ab[f], xi[f]);
        }
        Q->grad[q][a][e] = gr;
      }
    }
  }
}

/* Global indices of the local nodes of the element with lower corner (ei,ej,ek). */
static void element_nodes(const mesh_t *g, int ei, int ej, int ek, int64_t *idx) {
  int nloc = (g->dim == 2) ? 4 : 8;
  for (int a = 0; a < nloc; a++)
    idx[a] = node_at(g, ei + (a & 1), ej + ((a >> 1) & 1), ek + ((a >> 2) & 1));
}

static int64_t mesh_elements(const mesh_t *g) {
  return (g->dim == 2) ? (int64_t)g->N * g->N : (int64_t)g->N * g->N * g->N;
}

static void element_corner(const mesh_t *g, int64_t e, int *ei, int *ej, int *ek) {
  *ei = (int)(e % g->N);
  *ej = (int)((e / g->N) % g->N);
  *ek = (g->dim == 3) ? (int)(e / ((int64_t)g->N * g->N)) : 0;
}

/* ------------------------------------------------------------------------ */
/* CSR                                                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t nrows, ncols, nnz;
  int64_t *rp;
  int32_t *ci;
  double *v;
  int owns_pattern;
} csr_t;

static void csr_free(csr_t *A) {
  if (!A) return;
  if (A->owns_pattern) {
    free(A->rp);
    free(A->ci);
  }
  free(A->v);
  free(A);
}

/* Sparsity of a Q1 operator: node i couples with every node of the elements
 * containing it, i.e. the (up to) 3^d nodes at offsets in {-1,0,1}^d.  The
 * columns come out sorted because the loops run z, y, x outermost first. */
static csr_t *csr_pattern(const mesh_t *g) {
  csr_t *A = (csr_t *)calloc(1, sizeof(csr_t));
  if (!A) return NULL;
  A->nrows = A->ncols = g->nodes;
  A->rp = (int64_t *)malloc(sizeof(int64_t) * (g->nodes + 1));
  if (!A->rp) { free(A); return NULL; }
  A->rp[0] = 0;
  int kz = (g->dim == 3) ? 1 : 0;
  for (int64_t r = 0; r < g->nodes; r++) {
    int i, j, k;
    node_ijk(g, r, &i, &j, &k);
    int cnt = 0;
    for (int dk = -kz; dk <= kz; dk++)
      for (int dj = -1; dj <= 1; dj++)
        for (int di = -1; di <= 1; di++) {
          int ii = i + di, jj = j + dj, kk = k + dk;
          if (ii < 0 || ii > g->N || jj < 0 || jj > g->N) continue;
          if (g->dim == 3 && (kk < 0 || kk > g->N)) continue;
          cnt++;
        }
    A->rp[r + 1] = A->rp[r] + cnt;
  }
  A->nnz = A->rp[g->nodes];
  A->ci = (int32_t *)malloc(sizeof(int32_t) * A->nnz);
  if (!A->ci) { free(A->rp); free(A); return NULL; }
  for (int64_t r = 0; r < g->nodes; r++) {
    int i, j, k;
    node_ijk(g, r, &i, &j, &k);
    int64_t p = A->rp[r];
    for (int dk = -kz; dk <= kz; dk++)
      for (int dj = -1; dj <= 1; dj++)
        for (int di = -1; di <= 1; di++) {
          int ii = i + di, jj = j + dj, kk = k + dk;
          if (ii < 0 || ii > g->N || jj < 0 || jj > g->N) continue;
          if (g->dim == 3 && (kk < 0 || kk > g->N)) continue;
          A->ci[p++] = (int32_t)node_at(g, ii, jj, kk);
        }
  }
  A->owns_pattern = 1;
  return A;
}

/* A new matrix with the same pattern as P and zeroed values. */
static csr_t *csr_like(const csr_t *P) {
  csr_t *A = (csr_t *)calloc(1, sizeof(csr_t));
  if (!A) return NULL;
  *A = *P;
  A->owns_pattern = 0;
  A->v = (double *)calloc(A->nnz, sizeof(double));
  if (!A->v) { free(A); return NULL; }
  return A;
}

static void csr_add(csr_t *A, int64_t r, int64_t c, double val) {
  for (int64_t p = A->rp[r]; p < A->rp[r + 1]; p++)
    if (A->ci[p] == c) {
      A->v[p] += val;
      return;
    }
  fprintf(stderr, "okref: csr_add outside pattern (%lld,%lld)\n", (long long)r, (long long)c);
  abort();
}

/* y = A x */
static void csr_mv(const csr_t *A, const double *x, double *y) {
  for (int64_t r = 0; r < A->nrows; r++) {
    double s = 0.0;
    for (int64_t p = A->rp[r]; p < A->rp[r + 1]; p++) s += A->v[p] * x[A->ci[p]];
    y[r] = s;
  }
}

/* y = A^T x  (A is nrows x ncols, x has nrows entries, y has ncols entries) */
static void csr_mtv(const csr_t *A, const double *x, double *y) {
  for (int64_t c = 0; c < A->ncols; c++) y[c] = 0.0;
  for (int64_t r = 0; r < A->nrows; r++)
    for (int64_t p = A->rp[r]; p < A->rp[r + 1]; p++) y[A->ci[p]] += A->v[p] * x[r];
}

static void csr_diag(const csr_t *A, double *d) {
  for (int64_t r = 0; r < A->nrows; r++) {
    d[r] = 0.0;
    for (int64_t p = A->rp[r]; p < A->rp[r + 1]; p++)
      if (A->ci[p] == r) d[r] = A->v[p];
  }
}

/* ------------------------------------------------------------------------ */
/* Finite element assembly (Sec. 2, definitions of M, K, M_E below (newton)) */
/* ------------------------------------------------------------------------ */

/* M_ij = int phi_i phi_j and K_ij = int grad phi_i . grad phi_j, by element
 * loops with exact quadrature.  alpha_m * M + alpha_k * K into one matrix. */
static csr_t *assemble_MK(const mesh_t *g, const csr_t *pat, double am, double ak) {
  csr_t *A = csr_like(pat);
  if (!A) return NULL;
  quad_t Q;
  quad_make(g, &Q);
  double Ae[8][8];
  for (int a = 0; a < Q.nloc; a++)
    for (int b = 0; b < Q.nloc; b++) {
      double s = 0.0;
      for (int q = 0; q < Q.nq; q++) {
        double gg = 0.0;
        for (int e = 0; e < g->dim; e++) gg += Q.grad[q][a][e] * Q.grad[q][b][e];
        s += Q.W[q] * (am * Q.phi[q][a] * Q.phi[q][b] + ak * gg);
      }
      Ae[a][b] = s;
    }
  int64_t ne = mesh_elements(g);
  for (int64_t e = 0; e < ne; e++) {
    int ei, ej, ek;
    int64_t idx[8];
    element_corner(g, e, &ei, &ej, &ek);
    element_nodes(g, ei, ej, ek, idx);
    for (int a = 0; a < Q.nloc; a++)
      for (int b = 0; b < Q.nloc; b++) csr_add(A, idx[a], idx[b], Ae[a][b]);
  }
  return A;
}

/* (M_E)_ij = int (3u^2 - 1) phi_i phi_j with u the Q1 interpolant. */
static int assemble_ME(const mesh_t *g, const double *u, csr_t *A) {
  quad_t Q;
  quad_make(g, &Q);
  memset(A->v, 0, sizeof(double) * A->nnz);
  int64_t ne = mesh_elements(g);
  for (int64_t e = 0; e < ne; e++) {
    int ei, ej, ek;
    int64_t idx[8];
    element_corner(g, e, &ei, &ej, &ek);
    element_nodes(g, ei, ej, ek, idx);
    double coef[27];
    for (int q = 0; q < Q.nq; q++) {
      double uq = 0.0;
      for (int a = 0; a < Q.nloc; a++) uq += u[idx[a]] * Q.phi[q][a];
      coef[q] = Q.W[q] * (3.0 * uq * uq - 1.0);
    }
    for (int a = 0; a < Q.nloc; a++)
      for (int b = 0; b < Q.nloc; b++) {
        double s = 0.0;
        for (int q = 0; q < Q.nq; q++) s += coef[q] * Q.phi[q][a] * Q.phi[q][b];
        csr_add(A, idx[a], idx[b], s);
      }
  }
  return 0;
}

/* N(u)_i = int (u^3 - u) phi_i: the weak form of the nonlinearity in (okb). */
static void assemble_N(const mesh_t *g, const double *u, double *nv) {
  quad_t Q;
  quad_make(g, &Q);
  memset(nv, 0, sizeof(double) * g->nodes);
  int64_t ne = mesh_elements(g);
  for (int64_t e = 0; e < ne; e++) {
    int ei, ej, ek;
    int64_t idx[8];
    element_corner(g, e, &ei, &ej, &ek);
    element_nodes(g, ei, ej, ek, idx);
    for (int q = 0; q < Q.nq; q++) {
      double uq = 0.0;
      for (int a = 0; a < Q.nloc; a++) uq += u[idx[a]] * Q.phi[q][a];
      double f = Q.W[q] * (uq * uq * uq - uq);
      for (int a = 0; a < Q.nloc; a++) nv[idx[a]] += f * Q.phi[q][a];
    }
  }
}

/* Q1 interpolation from the mesh with Nc = N/2 elements to the mesh with N:
 * a fine node at an even index copies the coarse node, at an odd index it
 * averages the two coarse neighbours, direction by direction. */
static csr_t *assemble_P(const mesh_t *fine, const mesh_t *coarse) {
  csr_t *P = (csr_t *)calloc(1, sizeof(csr_t));
  if (!P) return NULL;
  P->nrows = fine->nodes;
  P->ncols = coarse->nodes;
  P->owns_pattern = 1;
  P->rp = (int64_t *)malloc(sizeof(int64_t) * (fine->nodes + 1));
  int64_t cap = fine->nodes * ((fine->dim == 3) ? 8 : 4);
  P->ci = (int32_t *)malloc(sizeof(int32_t) * cap);
  P->v = (double *)malloc(sizeof(double) * cap);
  if (!P->rp || !P->ci || !P->v) { csr_free(P); return NULL; }
  int64_t p = 0;
  P->rp[0] = 0;
  for (int64_t r = 0; r < fine->nodes; r++) {
    int ijk[3];
    node_ijk(fine, r, &ijk[0], &ijk[1], &ijk[2]);
    int lc[3][2], nl[3];
    double lw[3][2];
    for (int e = 0; e < 3; e++) {
      if (e >= fine->dim) { lc[e][0] = 0; lw[e][0] = 1.0; nl[e] = 1; continue; }
      if (ijk[e] % 2 == 0) { lc[e][0] = ijk[e] / 2; lw[e][0] = 1.0; nl[e] = 1; }
      else {
        lc[e][0] = (ijk[e] - 1) / 2; lw[e][0] = 0.5;
        lc[e][1] = (ijk[e] + 1) / 2; lw[e][1] = 0.5;
        nl[e] = 2;
      }
    }
    for (int c = 0; c < nl[2]; c++)
      for (int b = 0; b < nl[1]; b++)
        for (int a = 0; a < nl[0]; a++) {
          P->ci[p] = (int32_t)node_at(coarse, lc[0][a], lc[1][b], lc[2][c]);
          P->v[p] = lw[0][a] * lw[1][b] * lw[2][c];
          p++;
        }
    P->rp[r + 1] = p;
  }
  P->nnz = p;
  return P;
}

/* ------------------------------------------------------------------------ */
/* Chebyshev intervals                                                      */
/* ------------------------------------------------------------------------ */

/* For the Q1 mass and stiffness matrices on a uniform grid with Neumann ends,
 * the DCT-I vectors v(j) = prod_d cos(k_d pi j_d / N) satisfy
 *   M v = W v prod_d mu(c_d),   K v = W v sum_d kap(c_d) prod_{e!=d} mu(c_e),
 * with c = cos(k pi/N), mu(c) = (h/3)(2+c), kap(c) = (2/h)(1-c) and W the
 * diagonal of trapezoid weights (1/2 at each end).  The diagonal D of
 * M + alpha K is W times the interior diagonal, so D^-1 (M + alpha K) has
 * these vectors as eigenvectors with eigenvalue lam(c) below. */
static double dct_lambda(const mesh_t *g, double alpha, const double *c) {
  double h = g->h, num = 1.0, sk = 0.0;
  for (int d = 0; d < g->dim; d++) num *= (h / 3.0) * (2.0 + c[d]);
  for (int d = 0; d < g->dim; d++) {
    double t = (2.0 / h) * (1.0 - c[d]);
    for (int e = 0; e < g->dim; e++)
      if (e != d) t *= (h / 3.0) * (2.0 + c[e]);
    sk += t;
  }
  double den = pow(2.0 * h / 3.0, g->dim) + alpha * g->dim * (2.0 / h) * pow(2.0 * h / 3.0, g->dim - 1);
  return (num + alpha * sk) / den;
}

/* lam is multilinear in c, so its extremes over a box of c are at vertices.
 * hi: max over all corners c in {-1,1}^d.  lo (smoother, hf=1): min over the
 * high-frequency vertices, i.e. some c_d in {-1,0} and the others in {-1,1};
 * lo (hf=0): min over all corners (the whole spectrum). */
static void cheb_interval(const mesh_t *g, double alpha, int hf, double *lo, double *hi) {
  int d = g->dim;
  double mx = -1e300, mn = 1e300;
  int ncorner = 1 << d;
  for (int s = 0; s < ncorner; s++) {
    double c[3];
    for (int e = 0; e < d; e++) c[e] = (s >> e & 1) ? 1.0 : -1.0;
    double l = dct_lambda(g, alpha, c);
    if (l > mx) mx = l;
    if (!hf && l < mn) mn = l;
  }
  if (hf) {
    int nv = (d == 2) ? 9 : 27;
    for (int s = 0; s < nv; s++) {
      int t[3] = {s % 3, (s / 3) % 3, s / 9};
      double c[3];
      int high = 0;
      for (int e = 0; e < d; e++) {
        c[e] = (t[e] == 0) ? -1.0 : (t[e] == 1 ? 0.0 : 1.0);
        if (t[e] <= 1) high = 1;
      }
      if (d == 2 && t[2] != 0) continue;
      if (!high) continue;
      double l = dct_lambda(g, alpha, c);
      if (l < mn) mn = l;
    }
  }
  *lo = mn;
  *hi = mx;
}

/* ------------------------------------------------------------------------ */
/* The oracle context                                                       */
/* ------------------------------------------------------------------------ */

#define MAXLEV 16

struct okref {
  okref_params p;
  int L;                        /* number of multigrid levels */
  mesh_t lev[MAXLEV];
  csr_t *pat[MAXLEV];           /* sparsity of each level */
  csr_t *M, *K;                 /* finest-level mass and stiffness */
  csr_t *ME;                    /* M_E(u) at the finest level */
  double *Mdiag;                /* diag(M) for Chebyshev-Jacobi on A = sA M */
  csr_t *A[MAXLEV];             /* M_l + alpha K_l */
  double *Ad[MAXLEV];           /* diag(A_l) */
  double lo[MAXLEV], hi[MAXLEV];
  csr_t *P[MAXLEV];             /* prolongation level l+1 -> l */
  double *chol;                 /* dense Cholesky factor of A_{L-1} (lower) */
  int64_t ncoarse;
  double c, alpha, sA;          /* c = dt th/(1+dt th sigma), alpha = eps sqrt(c), sA = 1+dt th sigma */
  double mlo, mhi;              /* Chebyshev interval for D^-1 M */
  const double *me_u;           /* u that ME currently holds (identity + copy) */
  double *me_ucopy;
};

int64_t okref_nodes(const okref *h, int level) {
  if (!h || level < 0 || level >= h->L) return -1;
  return h->lev[level].nodes;
}
int okref_levels(const okref *h) { return h ? h->L : -1; }

void okref_destroy(okref *h) {
  if (!h) return;
  csr_free(h->M);
  csr_free(h->K);
  csr_free(h->ME);
  free(h->Mdiag);
  for (int l = 0; l < MAXLEV; l++) {
    csr_free(h->A[l]);
    free(h->Ad[l]);
    csr_free(h->P[l]);
    csr_free(h->pat[l]);
  }
  free(h->chol);
  free(h->me_ucopy);
  free(h);
}

static int dense_cholesky(double *a, int64_t n) {
  for (int64_t j = 0; j < n; j++) {
    double s = a[j * n + j];
    for (int64_t k = 0; k < j; k++) s -= a[j * n + k] * a[j * n + k];
    if (!(s > 0.0)) return -1;
    double ljj = sqrt(s);
    a[j * n + j] = ljj;
    for (int64_t i = j + 1; i < n; i++) {
      double t = a[i * n + j];
      for (int64_t k = 0; k < j; k++) t -= a[i * n + k] * a[j * n + k];
      a[i * n + j] = t / ljj;
    }
    for (int64_t i = 0; i < j; i++) a[i * n + j] = 0.0;
  }
  return 0;
}

static void dense_chol_solve(const double *l, int64_t n, const double *b, double *x) {
  for (int64_t i = 0; i < n; i++) {
    double s = b[i];
    for (int64_t k = 0; k < i; k++) s -= l[i * n + k] * x[k];
    x[i] = s / l[i * n + i];
  }
  for (int64_t i = n - 1; i >= 0; i--) {
    double s = x[i];
    for (int64_t k = i + 1; k < n; k++) s -= l[k * n + i] * x[k];
    x[i] = s / l[i * n + i];
  }
}

int okref_create(const okref_params *p, okref **out) {
  gauss_init();
  *out = NULL;
  if (!p || (p->dim != 2 && p->dim != 3) || p->n < 1) return OKREF_E_INVALID;
  if (!(p->eps > 0) || !(p->dt > 0) || !(p->theta > 0) || p->theta > 1 || p->sigma < 0)
    return OKREF_E_INVALID;
  okref *h = (okref *)calloc(1, sizeof(okref));
  if (!h) return OKREF_E_NOMEM;
  h->p = *p;
  /* Sec. 2: c = dt theta / (1 + dt theta sigma); S^ = M + eps sqrt(c) K. */
  double dth = p->dt * p->theta;
  h->sA = 1.0 + dth * p->sigma;
  h->c = dth / h->sA;
  h->alpha = p->eps * sqrt(h->c);
  /* Levels: halve until 8 elements per direction (or the requested count). */
  int L = p->mg_levels;
  if (L <= 0) {
    L = 1;
    int n = p->n;
    while (n > 8 && n % 2 == 0 && L < MAXLEV) { n /= 2; L++; }
  }
  if (L > MAXLEV) { free(h); return OKREF_E_INVALID; }
  {
    int n = p->n;
    for (int l = 0; l < L; l++) {
      if (n < 1) { free(h); return OKREF_E_INVALID; }
      h->lev[l] = mesh_make(p->dim, n);
      if (l < L - 1) {
        if (n % 2) { free(h); return OKREF_E_INVALID; }
        n /= 2;
      }
    }
  }
  h->L = L;
  for (int l = 0; l < L; l++) {
    h->pat[l] = csr_pattern(&h->lev[l]);
    if (!h->pat[l]) goto nomem;
  }
  mesh_t *g = &h->lev[0];
  h->M = assemble_MK(g, h->pat[0], 1.0, 0.0);
  h->K = assemble_MK(g, h->pat[0], 0.0, 1.0);
  h->ME = csr_like(h->pat[0]);
  h->Mdiag = (double *)malloc(sizeof(double) * g->nodes);
  h->me_ucopy = (double *)malloc(sizeof(double) * g->nodes);
  if (!h->M || !h->K || !h->ME || !h->Mdiag || !h->me_ucopy) goto nomem;
  csr_diag(h->M, h->Mdiag);
  /* Chebyshev for A = sA M: D^-1 A = D_M^-1 M has spectrum [2^-d, (3/2)^d]. */
  cheb_interval(g, 0.0, 0, &h->mlo, &h->mhi);
  for (int l = 0; l < L; l++) {
    h->A[l] = assemble_MK(&h->lev[l], h->pat[l], 1.0, h->alpha);
    h->Ad[l] = (double *)malloc(sizeof(double) * h->lev[l].nodes);
    if (!h->A[l] || !h->Ad[l]) goto nomem;
    csr_diag(h->A[l], h->Ad[l]);
    cheb_interval(&h->lev[l], h->alpha, 1, &h->lo[l], &h->hi[l]);
    if (l < L - 1) {
      h->P[l] = assemble_P(&h->lev[l], &h->lev[l + 1]);
      if (!h->P[l]) goto nomem;
    }
  }
  if (h->A[L - 1]->nrows <= OKREF_DENSE_COARSE) {
    const csr_t *Ac = h->A[L - 1];
    int64_t n = Ac->nrows;
    h->ncoarse = n;
    h->chol = (double *)calloc((size_t)(n * n), sizeof(double));
    if (!h->chol) goto nomem;
    for (int64_t r = 0; r < n; r++)
      for (int64_t q = Ac->rp[r]; q < Ac->rp[r + 1]; q++) h->chol[r * n + Ac->ci[q]] = Ac->v[q];
    if (dense_cholesky(h->chol, n)) { okref_destroy(h); return OKREF_E_INVALID; }
  }
  *out = h;
  return OKREF_OK;
nomem:
  okref_destroy(h);
  return OKREF_E_NOMEM;
}

static int ensure_ME(okref *h, const double *u) {
  int64_t n = h->lev[0].nodes;
  if (h->me_u == u && memcmp(h->me_ucopy, u, sizeof(double) * n) == 0) return 0;
  assemble_ME(&h->lev[0], u, h->ME);
  memcpy(h->me_ucopy, u, sizeof(double) * n);
  h->me_u = u;
  return 0;
}

int okref_matrix(okref *h, int which, int level, const double *u, int64_t *nrows,
                 int64_t *ncols, int64_t *nnz, int64_t *rp, int32_t *ci, double *v) {
  if (!h || level < 0 || level >= h->L) return OKREF_E_INVALID;
  const csr_t *A = NULL;
  switch (which) {
    case OKREF_MAT_M: if (level) return OKREF_E_INVALID; A = h->M; break;
    case OKREF_MAT_K: if (level) return OKREF_E_INVALID; A = h->K; break;
    case OKREF_MAT_ME:
      if (level || !u) return OKREF_E_INVALID;
      ensure_ME(h, u);
      A = h->ME;
      break;
    case OKREF_MAT_A: A = h->A[level]; break;
    case OKREF_MAT_P: if (level >= h->L - 1) return OKREF_E_INVALID; A = h->P[level]; break;
    default: return OKREF_E_INVALID;
  }
  *nrows = A->nrows;
  *ncols = A->ncols;
  *nnz = A->nnz;
  if (rp) memcpy(rp, A->rp, sizeof(int64_t) * (A->nrows + 1));
  if (ci) memcpy(ci, A->ci, sizeof(int32_t) * A->nnz);
  if (v) memcpy(v, A->v, sizeof(double) * A->nnz);
  return OKREF_OK;
}

int okref_nonlinear(okref *h, const double *u, double *nv) {
  assemble_N(&h->lev[0], u, nv);
  return OKREF_OK;
}

int okref_cheb_interval(const okref *h, int level, int mass, double *lo, double *hi) {
  if (!h || level < 0 || level >= h->L) return OKREF_E_INVALID;
  if (mass) { *lo = h->mlo; *hi = h->mhi; }
  else { *lo = h->lo[level]; *hi = h->hi[level]; }
  return OKREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Residual and Jacobian (Sec. 2, eq. (newton) and the theta-method of (oka)-(okb)) */
/* ------------------------------------------------------------------------ */

static double dot(const double *a, const double *b, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

/* Conjugate gradients (Hestenes-Stiefel) on an SPD CSR matrix from x = 0,
 * until ||b - A x|| <= tol ||b|| or maxit iterations.  Used for coarse grids
 * too large for a dense factor, and for the mass solve of w0. */
static void cg_solve(const csr_t *A, const double *b, double *x, double tol, int maxit) {
  int64_t n = A->nrows;
  double *r = (double *)malloc(sizeof(double) * n);
  double *pv = (double *)malloc(sizeof(double) * n);
  double *q = (double *)malloc(sizeof(double) * n);
  for (int64_t i = 0; i < n; i++) {
    x[i] = 0.0;
    r[i] = b[i];
    pv[i] = b[i];
  }
  double rr = dot(r, r, n);
  const double stop = tol * tol * rr;
  for (int it = 0; it < maxit && rr > stop && rr > 0.0; it++) {
    csr_mv(A, pv, q);
    double al = rr / dot(pv, q, n);
    for (int64_t i = 0; i < n; i++) {
      x[i] += al * pv[i];
      r[i] -= al * q[i];
    }
    double rn = dot(r, r, n);
    double be = rn / rr;
    rr = rn;
    for (int64_t i = 0; i < n; i++) pv[i] = r[i] + be * pv[i];
  }
  free(r);
  free(pv);
  free(q);
}

/* w from u by (okb) in weak form: M w = eps^2 K u + N(u) (the initial
 * chemical potential of the paper's experiment, Sec. 4). */
int okref_initial_w(okref *h, const double *u, double *w) {
  int64_t n = h->lev[0].nodes;
  double *rhs = (double *)malloc(sizeof(double) * n);
  double *t = (double *)malloc(sizeof(double) * n);
  if (!rhs || !t) {
    free(rhs);
    free(t);
    return OKREF_E_NOMEM;
  }
  csr_mv(h->K, u, t);
  assemble_N(&h->lev[0], u, rhs);
  for (int64_t i = 0; i < n; i++) rhs[i] += h->p.eps * h->p.eps * t[i];
  cg_solve(h->M, rhs, w, 1e-15, 10000);
  free(rhs);
  free(t);
  return OKREF_OK;
}

/* F1 = M(u - un) + dt K (th w + (1-th) wn) + dt sigma M (th u + (1-th) un - m 1)
 * F2 = M w - eps^2 K u - N(u)
 * i.e. (oka) integrated over one step by the theta-method, and (okb) at the
 * new time level, both in weak form with natural Neumann boundaries (okbcs). */
double okref_residual(okref *h, const double *u, const double *w, const double *un,
                      const double *wn, double *F) {
  const okref_params *p = &h->p;
  int64_t n = h->lev[0].nodes;
  double th = p->theta;
  double *t1 = (double *)calloc(n, sizeof(double));
  double *t2 = (double *)calloc(n, sizeof(double));
  double *nv = (double *)calloc(n, sizeof(double));
  for (int64_t i = 0; i < n; i++)
    t1[i] = (u[i] - un[i]) + p->dt * p->sigma * (th * u[i] + (1.0 - th) * un[i] - p->m);
  csr_mv(h->M, t1, F);
  for (int64_t i = 0; i < n; i++) t1[i] = p->dt * (th * w[i] + (1.0 - th) * (wn ? wn[i] : w[i]));
  csr_mv(h->K, t1, t2);
  for (int64_t i = 0; i < n; i++) F[i] += t2[i];
  csr_mv(h->M, w, F + n);
  csr_mv(h->K, u, t2);
  assemble_N(&h->lev[0], u, nv);
  for (int64_t i = 0; i < n; i++) F[n + i] -= p->eps * p->eps * t2[i] + nv[i];
  free(t1);
  free(t2);
  free(nv);
  return sqrt(dot(F, F, 2 * n));
}

static void jac_apply_assembled(okref *h, const double *x, double *y) {
  const okref_params *p = &h->p;
  int64_t n = h->lev[0].nodes;
  double *t = (double *)malloc(sizeof(double) * n);
  /* y1 = (1 + dt th sigma) M x1 + dt th K x2 */
  csr_mv(h->M, x, y);
  csr_mv(h->K, x + n, t);
  for (int64_t i = 0; i < n; i++) y[i] = h->sA * y[i] + p->dt * p->theta * t[i];
  /* y2 = -eps^2 K x1 - M_E x1 + M x2 */
  csr_mv(h->M, x + n, y + n);
  csr_mv(h->K, x, t);
  for (int64_t i = 0; i < n; i++) y[n + i] -= p->eps * p->eps * t[i];
  csr_mv(h->ME, x, t);
  for (int64_t i = 0; i < n; i++) y[n + i] -= t[i];
  free(t);
}

int okref_jacobian_apply(okref *h, const double *u, const double *x, double *y) {
  ensure_ME(h, u);
  jac_apply_assembled(h, x, y);
  return OKREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Chebyshev semi-iteration with Jacobi preconditioning                      */
/* ------------------------------------------------------------------------ */

/* Saad, Iterative Methods for Sparse Linear Systems (2nd ed.), Alg. 12.1,
 * applied to D^-1 A x = D^-1 b with the spectrum of D^-1 A in [a, b].  Starts
 * from the x passed in (zero_start: x = 0) and runs K iterations. */
static void chebyshev(const csr_t *A, const double *D, double a, double b, int K,
                      const double *rhs, double *x, int zero_start) {
  int64_t n = A->nrows;
  double th = 0.5 * (a + b), de = 0.5 * (b - a), s1 = th / de;
  double *r = (double *)malloc(sizeof(double) * n);
  double *d = (double *)malloc(sizeof(double) * n);
  double *t = (double *)malloc(sizeof(double) * n);
  if (zero_start) {
    for (int64_t i = 0; i < n; i++) { x[i] = 0.0; r[i] = rhs[i]; }
  } else {
    csr_mv(A, x, t);
    for (int64_t i = 0; i < n; i++) r[i] = rhs[i] - t[i];
  }
  double rho = 1.0 / s1;
  for (int64_t i = 0; i < n; i++) d[i] = r[i] / D[i] / th;
  for (int k = 0; k < K; k++) {
    for (int64_t i = 0; i < n; i++) x[i] += d[i];
    if (k + 1 == K) break;
    csr_mv(A, d, t);
    for (int64_t i = 0; i < n; i++) r[i] -= t[i];
    double rho1 = 1.0 / (2.0 * s1 - rho);
    for (int64_t i = 0; i < n; i++) d[i] = rho1 * rho * d[i] + (2.0 * rho1 / de) * r[i] / D[i];
    rho = rho1;
  }
  free(r);
  free(d);
  free(t);
}

int okref_cheb_mass(okref *h, const double *r, double *x) {
  chebyshev(h->M, h->Mdiag, h->mlo, h->mhi, h->p.cheb_A_its, r, x, 1);
  return OKREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Geometric multigrid V-cycle for S^ = M + alpha K (Sec. 2, after (schurinv)) */
/* ------------------------------------------------------------------------ */

static void vcycle(okref *h, int l, const double *b, double *x, int zero_start) {
  int64_t n = h->lev[l].nodes;
  if (l == h->L - 1) {
    if (h->chol)
      dense_chol_solve(h->chol, h->ncoarse, b, x);
    else
      cg_solve(h->A[l], b, x, 1e-15, 5000);
    return;
  }
  const csr_t *A = h->A[l];
  chebyshev(A, h->Ad[l], h->lo[l], h->hi[l], h->p.mg_pre, b, x, zero_start);
  double *r = (double *)malloc(sizeof(double) * n);
  csr_mv(A, x, r);
  for (int64_t i = 0; i < n; i++) r[i] = b[i] - r[i];
  int64_t nc = h->lev[l + 1].nodes;
  double *bc = (double *)malloc(sizeof(double) * nc);
  double *ec = (double *)calloc(nc, sizeof(double));
  csr_mtv(h->P[l], r, bc);            /* restriction R = P^T */
  vcycle(h, l + 1, bc, ec, 1);
  csr_mv(h->P[l], ec, r);             /* prolongation of the correction */
  for (int64_t i = 0; i < n; i++) x[i] += r[i];
  chebyshev(A, h->Ad[l], h->lo[l], h->hi[l], h->p.mg_post, b, x, 0);
  free(r);
  free(bc);
  free(ec);
}

int okref_mg(okref *h, const double *b, double *x, int cycles) {
  int64_t n = h->lev[0].nodes;
  for (int64_t i = 0; i < n; i++) x[i] = 0.0;
  for (int c = 0; c < cycles; c++) vcycle(h, 0, b, x, c == 0);
  return OKREF_OK;
}

/* S~^-1 y = S^^-1 M S^^-1 y, eq. (schurinv). */
static void schur_tilde_inv(okref *h, const double *y, double *z) {
  int64_t n = h->lev[0].nodes;
  double *t = (double *)malloc(sizeof(double) * n);
  double *s = (double *)malloc(sizeof(double) * n);
  okref_mg(h, y, t, h->p.mg_cycles);
  csr_mv(h->M, t, s);
  okref_mg(h, s, z, h->p.mg_cycles);
  free(t);
  free(s);
}

/* S x = D x - C A~^-1 B x = M x + (eps^2 K + M_E) A~^-1 (dt th K x), with
 * A~^-1 the Chebyshev approximation of ((1+dt th sigma) M)^-1. */
static void schur_apply_assembled(okref *h, const double *x, double *y) {
  const okref_params *p = &h->p;
  int64_t n = h->lev[0].nodes;
  double *t = (double *)malloc(sizeof(double) * n);
  double *a = (double *)malloc(sizeof(double) * n);
  csr_mv(h->K, x, t);
  for (int64_t i = 0; i < n; i++) t[i] *= p->dt * p->theta;
  chebyshev(h->M, h->Mdiag, h->mlo, h->mhi, p->cheb_A_its, t, a, 1);
  for (int64_t i = 0; i < n; i++) a[i] /= h->sA;
  csr_mv(h->K, a, t);
  csr_mv(h->ME, a, y);
  for (int64_t i = 0; i < n; i++) y[i] += p->eps * p->eps * t[i];
  csr_mv(h->M, x, t);
  for (int64_t i = 0; i < n; i++) y[i] += t[i];
  free(t);
  free(a);
}

int okref_schur_apply(okref *h, const double *u, const double *x, double *y) {
  ensure_ME(h, u);
  schur_apply_assembled(h, x, y);
  return OKREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Block preconditioner, eq. (prec) with A~^-1 and S~^-1                    */
/* ------------------------------------------------------------------------ */

static void precond_assembled(okref *h, const double *r, double *z) {
  const okref_params *p = &h->p;
  int64_t n = h->lev[0].nodes;
  const double *r1 = r, *r2 = r + n;
  double *z1 = z, *z2 = z + n;
  double *y = (double *)malloc(sizeof(double) * n);
  double *t = (double *)malloc(sizeof(double) * n);
  /* z1 = A~^-1 r1: Chebyshev on M, then divide by 1 + dt th sigma. */
  chebyshev(h->M, h->Mdiag, h->mlo, h->mhi, p->cheb_A_its, r1, z1, 1);
  for (int64_t i = 0; i < n; i++) z1[i] /= h->sA;
  /* y = r2 - C z1 with C = -eps^2 K - M_E. */
  csr_mv(h->K, z1, t);
  csr_mv(h->ME, z1, y);
  for (int64_t i = 0; i < n; i++) y[i] = r2[i] + p->eps * p->eps * t[i] + y[i];
  /* z2 ~ S^-1 y: Richardson iterations preconditioned by S~^-1 (Sec. 4); one
   * iteration is z2 = S~^-1 y. */
  schur_tilde_inv(h, y, z2);
  if (p->schur_richardson > 1) {
    double *res = (double *)malloc(sizeof(double) * n);
    double *cor = (double *)malloc(sizeof(double) * n);
    for (int it = 1; it < p->schur_richardson; it++) {
      schur_apply_assembled(h, z2, res);
      for (int64_t i = 0; i < n; i++) res[i] = y[i] - res[i];
      schur_tilde_inv(h, res, cor);
      for (int64_t i = 0; i < n; i++) z2[i] += cor[i];
    }
    free(res);
    free(cor);
  }
  free(y);
  free(t);
}

int okref_precond_apply(okref *h, const double *u, const double *r, double *z) {
  ensure_ME(h, u);
  precond_assembled(h, r, z);
  return OKREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Flexible GMRES(m) (Saad 1993), right preconditioned, modified Gram-Schmidt */
/* ------------------------------------------------------------------------ */

static int fgmres_assembled(okref *h, const double *b, double *x, int32_t *its_out) {
  const okref_params *p = &h->p;
  int64_t n2 = 2 * h->lev[0].nodes;
  int m = p->gmres_restart;
  double *V = (double *)malloc(sizeof(double) * n2 * (m + 1));
  double *Z = (double *)malloc(sizeof(double) * n2 * m);
  double *w = (double *)malloc(sizeof(double) * n2);
  double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
  double *cs = (double *)malloc(sizeof(double) * m);
  double *sn = (double *)malloc(sizeof(double) * m);
  double *g = (double *)malloc(sizeof(double) * (m + 1));
  double *y = (double *)malloc(sizeof(double) * m);
  int status = OKREF_E_GMRES_MAXIT, its = 0;
  for (int64_t i = 0; i < n2; i++) x[i] = 0.0;
  double bnorm = sqrt(dot(b, b, n2));
  if (!isfinite(bnorm)) { status = OKREF_E_NONFINITE; goto done; }
  if (bnorm == 0.0) { status = OKREF_OK; goto done; }
  double tol = p->gmres_rtol * bnorm;
  /* r0 = b - J x0 = b. */
  double beta = bnorm;
  memcpy(w, b, sizeof(double) * n2);
  for (int cycle = 0; cycle <= p->gmres_max_restarts; cycle++) {
    for (int64_t i = 0; i < n2; i++) V[i] = w[i] / beta;
    for (int i = 0; i <= m; i++) g[i] = 0.0;
    g[0] = beta;
    int k = 0, conv = 0;
    for (int j = 0; j < m; j++) {
      double *vj = V + (int64_t)j * n2, *zj = Z + (int64_t)j * n2;
      precond_assembled(h, vj, zj);
      jac_apply_assembled(h, zj, w);
      for (int i = 0; i <= j; i++) {
        const double *vi = V + (int64_t)i * n2;
        double hij = dot(w, vi, n2);
        H[i * m + j] = hij;
        for (int64_t q = 0; q < n2; q++) w[q] -= hij * vi[q];
      }
      double hn = sqrt(dot(w, w, n2));
      H[(j + 1) * m + j] = hn;
      if (!isfinite(hn)) { status = OKREF_E_NONFINITE; goto done; }
      for (int i = 0; i < j; i++) {
        double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
        H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
        H[i * m + j] = t;
      }
      double den = hypot(H[j * m + j], H[(j + 1) * m + j]);
      cs[j] = H[j * m + j] / den;
      sn[j] = H[(j + 1) * m + j] / den;
      H[j * m + j] = den;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      its++;
      k = j + 1;
      if (fabs(g[j + 1]) <= tol || hn == 0.0) { conv = 1; break; }
      double *vn = V + (int64_t)(j + 1) * n2;
      for (int64_t q = 0; q < n2; q++) vn[q] = w[q] / hn;
    }
    /* Least squares: back substitution with the triangular H. */
    for (int i = k - 1; i >= 0; i--) {
      double s = g[i];
      for (int l = i + 1; l < k; l++) s -= H[i * m + l] * y[l];
      y[i] = s / H[i * m + i];
    }
    for (int j = 0; j < k; j++) {
      const double *zj = Z + (int64_t)j * n2;
      for (int64_t q = 0; q < n2; q++) x[q] += y[j] * zj[q];
    }
    if (conv) { status = OKREF_OK; break; }
    /* Restart from the true residual. */
    jac_apply_assembled(h, x, w);
    for (int64_t q = 0; q < n2; q++) w[q] = b[q] - w[q];
    beta = sqrt(dot(w, w, n2));
    if (!isfinite(beta)) { status = OKREF_E_NONFINITE; break; }
    if (beta <= tol) { status = OKREF_OK; break; }
  }
done:
  if (its_out) *its_out = its;
  free(V); free(Z); free(w); free(H); free(cs); free(sn); free(g); free(y);
  return status;
}

int okref_fgmres(okref *h, const double *u, const double *b, double *x, int32_t *its) {
  ensure_ME(h, u);
  return fgmres_assembled(h, b, x, its);
}

/* ------------------------------------------------------------------------ */
/* The symmetric rearranged system (Sec. 2, after (schurapprox)) and MINRES */
/* ------------------------------------------------------------------------ */

/* Row 1 of (newton) divided by 1 + dt th sigma, unknowns in the order
 * [dw; du]:  y1 = c K x1 + M x2,  y2 = M x1 - eps^2 K x2 - M_E x2. */
static void sym_apply_assembled(okref *h, const double *x, double *y) {
  const okref_params *p = &h->p;
  int64_t n = h->lev[0].nodes;
  double *t = (double *)malloc(sizeof(double) * n);
  csr_mv(h->K, x, y);
  csr_mv(h->M, x + n, t);
  for (int64_t i = 0; i < n; i++) y[i] = h->c * y[i] + t[i];
  csr_mv(h->M, x, y + n);
  csr_mv(h->K, x + n, t);
  for (int64_t i = 0; i < n; i++) y[n + i] -= p->eps * p->eps * t[i];
  csr_mv(h->ME, x + n, t);
  for (int64_t i = 0; i < n; i++) y[n + i] -= t[i];
  free(t);
}

int okref_sym_apply(okref *h, const double *u, const double *x, double *y) {
  ensure_ME(h, u);
  sym_apply_assembled(h, x, y);
  return OKREF_OK;
}

/* Block-diagonal preconditioner of the symmetric system.  The singular
 * (1,1)-block c K is replaced by the positive definite (c/alpha) S^ =
 * c K + (sqrt(c)/eps) M; with M_E dropped, the Schur complement of that block,
 * eps^2 K + M ((c/alpha) S^)^-1 M, is approximated by S^ ((c/alpha) S^)^-1 S^
 * = (alpha/c) S^.  Both blocks are applied with the V-cycle of S^. */
static void sym_precond_assembled(okref *h, const double *r, double *z) {
  int64_t n = h->lev[0].nodes;
  okref_mg(h, r, z, h->p.mg_cycles);
  okref_mg(h, r + n, z + n, h->p.mg_cycles);
  for (int64_t i = 0; i < n; i++) {
    z[i] *= h->alpha / h->c;
    z[n + i] *= h->c / h->alpha;
  }
}

int okref_sym_precond(okref *h, const double *r, double *z) {
  sym_precond_assembled(h, r, z);
  return OKREF_OK;
}

/* Preconditioned MINRES (Paige and Saunders 1975) for a symmetric matrix
 * with a symmetric positive definite preconditioner P, in the three-term
 * Lanczos form in which P^-1 is applied once per iteration (Elman, Silvester
 * and Wathen, Finite Elements and Fast Iterative Solvers, 2nd ed., Alg. 4.1):
 * v_{j+1} = A z_j - (delta_j/gamma_j) v_j - (gamma_j/gamma_{j-1}) v_{j-1},
 * z_{j+1} = P^-1 v_{j+1}, gamma_{j+1} = <z_{j+1}, v_{j+1}>^(1/2), with z_j
 * scaled to unit P-norm; the QR factorisation of the tridiagonal Lanczos
 * matrix by Givens rotations (c, s) gives the update direction w_{j+1} and
 * the P^-1-norm of the residual, |eta|.  x0 = 0. */
static int minres_assembled(okref *h, const double *b, double *x, int32_t *its_out) {
  const okref_params *p = &h->p;
  int64_t n2 = 2 * h->lev[0].nodes;
  const int maxit = p->gmres_restart * (p->gmres_max_restarts + 1);
  double *v0 = (double *)calloc(n2, sizeof(double));
  double *v1 = (double *)malloc(sizeof(double) * n2);
  double *v2 = (double *)malloc(sizeof(double) * n2);
  double *z1 = (double *)malloc(sizeof(double) * n2);
  double *z2 = (double *)malloc(sizeof(double) * n2);
  double *az = (double *)malloc(sizeof(double) * n2);
  double *w0 = (double *)calloc(n2, sizeof(double));
  double *w1 = (double *)calloc(n2, sizeof(double));
  double *w2 = (double *)malloc(sizeof(double) * n2);
  int status = OKREF_E_GMRES_MAXIT, its = 0;
  memset(x, 0, sizeof(double) * n2);
  memcpy(v1, b, sizeof(double) * n2);
  sym_precond_assembled(h, v1, z1);
  double gam1 = sqrt(dot(z1, v1, n2));
  if (!isfinite(gam1)) { status = OKREF_E_NONFINITE; goto done; }
  if (gam1 == 0.0) { status = OKREF_OK; goto done; }
  {
    double gam0 = 1.0, gam = gam1, eta = gam1;
    double s0 = 0.0, s = 0.0, c0 = 1.0, cc = 1.0;
    const double tol = p->gmres_rtol * gam1;
    for (int j = 1; j <= maxit; j++) {
      for (int64_t i = 0; i < n2; i++) z1[i] /= gam;
      sym_apply_assembled(h, z1, az);
      double delta = dot(az, z1, n2);
      for (int64_t i = 0; i < n2; i++) v2[i] = az[i] - (delta / gam) * v1[i] - (gam / gam0) * v0[i];
      sym_precond_assembled(h, v2, z2);
      double gnew = sqrt(dot(z2, v2, n2));
      double a0 = cc * delta - c0 * s * gam;
      double a1 = sqrt(a0 * a0 + gnew * gnew);
      double a2 = s * delta + c0 * cc * gam;
      double a3 = s0 * gam;
      double cn = a0 / a1, sn = gnew / a1;
      for (int64_t i = 0; i < n2; i++) w2[i] = (z1[i] - a3 * w0[i] - a2 * w1[i]) / a1;
      for (int64_t i = 0; i < n2; i++) x[i] += cn * eta * w2[i];
      eta = -sn * eta;
      its = j;
      if (!isfinite(eta) || !isfinite(gnew)) { status = OKREF_E_NONFINITE; break; }
      if (fabs(eta) <= tol || gnew == 0.0) { status = OKREF_OK; break; }
      /* shift: (v0, v1) <- (v1, v2), z1 <- z2, (w0, w1) <- (w1, w2) */
      double *t = v0; v0 = v1; v1 = v2; v2 = t;
      t = z1; z1 = z2; z2 = t;
      t = w0; w0 = w1; w1 = w2; w2 = t;
      gam0 = gam; gam = gnew;
      c0 = cc; cc = cn; s0 = s; s = sn;
    }
  }
done:
  if (its_out) *its_out = its;
  free(v0); free(v1); free(v2); free(z1); free(z2); free(az); free(w0); free(w1); free(w2);
  return status;
}

int okref_minres(okref *h, const double *u, const double *b, double *x, int32_t *its) {
  ensure_ME(h, u);
  return minres_assembled(h, b, x, its);
}

/* ------------------------------------------------------------------------ */
/* Newton and the timestep loop (Sec. 2: one linear solve per Newton step)  */
/* ------------------------------------------------------------------------ */

/* Solve J(u) dx = -F (FGMRES on (newton), or MINRES on its symmetric
 * rearrangement) and take the full step (u,w) += dx.  F is overwritten. */
static int newton_update(okref *h, double *u, double *w, double *F, int32_t *its) {
  int64_t n = h->lev[0].nodes;
  double *dx = (double *)malloc(sizeof(double) * 2 * n);
  for (int64_t i = 0; i < 2 * n; i++) F[i] = -F[i];
  ensure_ME(h, u);
  int st;
  if (h->p.linear_solver == 1) {
    /* [f1/(1+dt th sigma); f2] for the unknowns [dw; du] */
    for (int64_t i = 0; i < n; i++) F[i] /= h->sA;
    st = minres_assembled(h, F, dx, its);
    if (st != OKREF_E_NONFINITE)
      for (int64_t i = 0; i < n; i++) { w[i] += dx[i]; u[i] += dx[n + i]; }
  } else {
    st = fgmres_assembled(h, F, dx, its);
    if (st != OKREF_E_NONFINITE)
      for (int64_t i = 0; i < n; i++) { u[i] += dx[i]; w[i] += dx[n + i]; }
  }
  free(dx);
  return st;
}

int okref_newton_step(okref *h, double *u, double *w, const double *un, const double *wn,
                      double *fnorm, int32_t *its) {
  int64_t n = h->lev[0].nodes;
  double *F = (double *)malloc(sizeof(double) * 2 * n);
  double nf = okref_residual(h, u, w, un, wn, F);
  if (fnorm) *fnorm = nf;
  if (its) *its = 0;
  int st = isfinite(nf) ? newton_update(h, u, w, F, its) : OKREF_E_NONFINITE;
  free(F);
  return st;
}

int okref_newton_solve(okref *h, double *u, double *w, const double *un, const double *wn,
                       okref_info *info) {
  int64_t n = h->lev[0].nodes;
  double *F = (double *)malloc(sizeof(double) * 2 * n);
  int st;
  for (int k = 0;; k++) {
    double nf = okref_residual(h, u, w, un, wn, F);
    int slot = info->newton_its < OKREF_HIST ? info->newton_its : OKREF_HIST;
    info->fnorm[slot] = nf;
    if (!isfinite(nf)) { st = OKREF_E_NONFINITE; break; }
    if (nf <= h->p.newton_atol) { st = OKREF_OK; break; }
    if (k >= h->p.newton_max_it) { st = OKREF_E_NEWTON_MAXIT; break; }
    int32_t its = 0;
    int s2 = newton_update(h, u, w, F, &its);
    if (info->newton_its < OKREF_HIST) info->fgmres_its[info->newton_its] = its;
    info->newton_its++;
    info->fgmres_its_total += its;
    if (s2 == OKREF_E_NONFINITE) { st = s2; break; }
  }
  free(F);
  return st;
}

int okref_timestep(okref *h, double *u, double *w, int32_t nsteps, okref_info *info) {
  int64_t n = h->lev[0].nodes;
  memset(info, 0, sizeof(*info));
  double *un = (double *)malloc(sizeof(double) * n);
  double *wn = (double *)malloc(sizeof(double) * n);
  int st = OKREF_OK;
  for (int s = 0; s < nsteps; s++) {
    memcpy(un, u, sizeof(double) * n);
    memcpy(wn, w, sizeof(double) * n);
    st = okref_newton_solve(h, u, w, un, wn, info);
    if (st) break;
  }
  info->status = st;
  free(un);
  free(wn);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Matrix-free local rows (same integrals, element by element around a node) */
/* ------------------------------------------------------------------------ */

/* Contribution of one element to the row of local node a, for the residual:
 * returns F1_a and F2_a on that element. */
static void element_residual_row(const mesh_t *g, const quad_t *Q, const okref_params *p,
                                 const int64_t *idx, int a, const double *u, const double *w,
                                 const double *un, const double *wn, double *f1, double *f2) {
  double th = p->theta, s1 = 0.0, s2 = 0.0;
  for (int q = 0; q < Q->nq; q++) {
    double uq = 0, wq = 0, unq = 0, wnq = 0;
    double gu[3] = {0, 0, 0}, gw[3] = {0, 0, 0};
    for (int b = 0; b < Q->nloc; b++) {
      double ph = Q->phi[q][b];
      uq += u[idx[b]] * ph;
      wq += w[idx[b]] * ph;
      unq += un[idx[b]] * ph;
      wnq += (wn ? wn[idx[b]] : w[idx[b]]) * ph;
      for (int e = 0; e < g->dim; e++) {
        gu[e] += u[idx[b]] * Q->grad[q][b][e];
        gw[e] += (th * w[idx[b]] + (1.0 - th) * (wn ? wn[idx[b]] : w[idx[b]])) * Q->grad[q][b][e];
      }
    }
    double ga_u = 0, ga_w = 0;
    for (int e = 0; e < g->dim; e++) {
      ga_u += gu[e] * Q->grad[q][a][e];
      ga_w += gw[e] * Q->grad[q][a][e];
    }
    double pa = Q->phi[q][a];
    s1 += Q->W[q] * ((uq - unq) * pa + p->dt * ga_w +
                     p->dt * p->sigma * (th * uq + (1.0 - th) * unq - p->m) * pa);
    s2 += Q->W[q] * (wq * pa - p->eps * p->eps * ga_u - (uq * uq * uq - uq) * pa);
  }
  *f1 += s1;
  *f2 += s2;
}

static void element_jacobian_row(const mesh_t *g, const quad_t *Q, const okref_params *p,
                                 const int64_t *idx, int a, const double *u, const double *x,
                                 double *y1, double *y2) {
  int64_t n = g->nodes;
  double dth = p->dt * p->theta, sA = 1.0 + dth * p->sigma, s1 = 0.0, s2 = 0.0;
  for (int q = 0; q < Q->nq; q++) {
    double uq = 0, x1 = 0, x2 = 0, g1[3] = {0, 0, 0}, g2[3] = {0, 0, 0};
    for (int b = 0; b < Q->nloc; b++) {
      double ph = Q->phi[q][b];
      uq += u[idx[b]] * ph;
      x1 += x[idx[b]] * ph;
      x2 += x[n + idx[b]] * ph;
      for (int e = 0; e < g->dim; e++) {
        g1[e] += x[idx[b]] * Q->grad[q][b][e];
        g2[e] += x[n + idx[b]] * Q->grad[q][b][e];
      }
    }
    double k1 = 0, k2 = 0;
    for (int e = 0; e < g->dim; e++) {
      k1 += g1[e] * Q->grad[q][a][e];
      k2 += g2[e] * Q->grad[q][a][e];
    }
    double pa = Q->phi[q][a];
    s1 += Q->W[q] * (sA * x1 * pa + dth * k2);
    s2 += Q->W[q] * (-p->eps * p->eps * k1 - (3.0 * uq * uq - 1.0) * x1 * pa + x2 * pa);
  }
  *y1 += s1;
  *y2 += s2;
}



static int local_rows(const okref_params *p, const int64_t *nodes, int64_t count, double *out,
                      int kind, const double *a0, const double *a1, const double *a2,
                      const double *a3) {
  gauss_init();
  if (!p || (p->dim != 2 && p->dim != 3) || p->n < 1) return OKREF_E_INVALID;
  mesh_t g = mesh_make(p->dim, p->n);
  quad_t Q;
  quad_make(&g, &Q);
  for (int64_t c = 0; c < count; c++) {
    int64_t r = nodes[c];
    if (r < 0 || r >= g.nodes) return OKREF_E_INVALID;
    int i, j, k;
    node_ijk(&g, r, &i, &j, &k);
    double f1 = 0.0, f2 = 0.0;
    int kz = (g.dim == 3) ? 1 : 0;
    /* every element with this node as a corner */
    for (int ek = k - kz; ek <= k; ek++)
      for (int ej = j - 1; ej <= j; ej++)
        for (int ei = i - 1; ei <= i; ei++) {
          if (ei < 0 || ej < 0 || ei >= g.N || ej >= g.N) continue;
          if (g.dim == 3 && (ek < 0 || ek >= g.N)) continue;
          int64_t idx[8];
          element_nodes(&g, ei, ej, ek, idx);
          int a = (i - ei) | ((j - ej) << 1) | ((k - ek) << 2);
          if (kind == 0)
            element_residual_row(&g, &Q, p, idx, a, a0, a1, a2, a3, &f1, &f2);
          else
            element_jacobian_row(&g, &Q, p, idx, a, a0, a1, &f1, &f2);
        }
    out[c] = f1;
    out[count + c] = f2;
  }
  return OKREF_OK;
}

int okref_local_residual(const okref_params *p, const double *u, const double *w,
                         const double *un, const double *wn, const int64_t *nodes,
                         int64_t count, double *out) {
  return local_rows(p, nodes, count, out, 0, u, w, un, wn);
}

int okref_local_jacobian(const okref_params *p, const double *u, const double *x,
                         const int64_t *nodes, int64_t count, double *out) {
  return local_rows(p, nodes, count, out, 1, u, x, NULL, NULL);
}
