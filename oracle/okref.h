/*
 * okref.h -- plain FP64 CPU oracle for the Ohta-Kawasaki Newton-Krylov
 * timestep of Farrell & Pearson, "A preconditioner for the Ohta-Kawasaki
 * equation" (arXiv:1603.04570).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes this
 * header, links this code or calls it.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark load it (through oracle/okref.py).
 *
 * Everything is serial FP64 over assembled CSR matrices on the uniform Q1
 * quad (d=2) / hex (d=3) mesh of the unit square/cube with N elements per
 * direction.  Node index: i + (N+1)*(j + (N+1)*k), x fastest.  Two-field
 * vectors are [u-block; w-block].
 */
#ifndef OKREF_H
#define OKREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t dim, n;                         /* d in {2,3}; N elements per direction  */
  double eps, sigma, m, dt, theta;        /* problem statement, Sec. 1 and 2        */
  int32_t gmres_restart, gmres_max_restarts;
  double gmres_rtol, newton_atol;
  int32_t newton_max_it, cheb_A_its;
  int32_t schur_richardson, mg_levels, mg_pre, mg_post, mg_cycles;
  int32_t linear_solver;                  /* 0: FGMRES on (newton); 1: MINRES on the
                                             symmetric rearranged system (Sec. 2)   */
} okref_params;

#define OKREF_HIST 256
typedef struct {
  int32_t status;                         /* 0 ok, <0 error (codes below)           */
  int32_t newton_its;                     /* Newton iterations (linear solves)      */
  int32_t fgmres_its_total;
  int32_t fgmres_its[OKREF_HIST];         /* per Newton iteration                   */
  double fnorm[OKREF_HIST + 1];           /* ||F||_2 before each Newton iteration   */
} okref_info;

enum { OKREF_OK = 0, OKREF_E_INVALID = -1, OKREF_E_GMRES_MAXIT = -4,
       OKREF_E_NEWTON_MAXIT = -5, OKREF_E_NONFINITE = -6, OKREF_E_NOMEM = -7 };

enum { OKREF_MAT_M = 0, OKREF_MAT_K = 1, OKREF_MAT_ME = 2, OKREF_MAT_A = 3, OKREF_MAT_P = 4 };

typedef struct okref okref;

int okref_create(const okref_params *p, okref **out);
void okref_destroy(okref *h);
int64_t okref_nodes(const okref *h, int level);
int okref_levels(const okref *h);

/* CSR export for the pin tests.  which: M, K, ME (needs u), A (=M+alpha K of a
 * level), P (prolongation level+1 -> level).  Call with rp==NULL to get sizes. */
int okref_matrix(okref *h, int which, int level, const double *u,
                 int64_t *nrows, int64_t *ncols, int64_t *nnz,
                 int64_t *rp, int32_t *ci, double *v);
int okref_nonlinear(okref *h, const double *u, double *nvec);          /* N(u)   */
int okref_initial_w(okref *h, const double *u, double *w);  /* M w = eps^2 K u + N(u) (okb) */
int okref_cheb_interval(const okref *h, int level, int mass, double *lo, double *hi);

double okref_residual(okref *h, const double *u, const double *w, const double *un,
                      const double *wn, double *F);
int okref_jacobian_apply(okref *h, const double *u, const double *x, double *y);
int okref_cheb_mass(okref *h, const double *r, double *x);              /* x = Cheb_M(r) */
int okref_mg(okref *h, const double *b, double *x, int cycles);          /* x = MG(b)     */
int okref_schur_apply(okref *h, const double *u, const double *x, double *y); /* S x with Cheb A^-1 */
int okref_precond_apply(okref *h, const double *u, const double *r, double *z);
int okref_fgmres(okref *h, const double *u, const double *b, double *x, int32_t *its);
int okref_newton_step(okref *h, double *u, double *w, const double *un, const double *wn,
                      double *fnorm, int32_t *its);
int okref_newton_solve(okref *h, double *u, double *w, const double *un, const double *wn,
                       okref_info *info);
int okref_timestep(okref *h, double *u, double *w, int32_t nsteps, okref_info *info);

/* The symmetric rearrangement of (newton) (Sec. 2, after (schurapprox)):
 *   [c K, M; M, -eps^2 K - M_E(u)] [dw; du] = [f1/(1+dt th sigma); f2],
 * x, y: [w-block; u-block] (2n).  Its block-diagonal preconditioner
 * z = diag((alpha/c) S^^-1, (c/alpha) S^^-1) r with S^ = M + alpha K, alpha =
 * eps sqrt(c), each S^^-1 mg_cycles V-cycles; and preconditioned MINRES
 * (x0 = 0; stop when the preconditioned residual norm falls to gmres_rtol of
 * its initial value; at most gmres_restart*(gmres_max_restarts+1) its). */
int okref_sym_apply(okref *h, const double *u, const double *x, double *y);
int okref_sym_precond(okref *h, const double *r, double *z);
int okref_minres(okref *h, const double *u, const double *b, double *x, int32_t *its);

/* Matrix-free local evaluation at selected nodes (no assembly): the residual
 * rows F_i and Jacobian rows (J x)_i, for sampled checks at sizes where CSR
 * assembly is too large.  out has 2*count entries: [F1 rows; F2 rows]. */
int okref_local_residual(const okref_params *p, const double *u, const double *w,
                         const double *un, const double *wn, const int64_t *nodes,
                         int64_t count, double *out);
int okref_local_jacobian(const okref_params *p, const double *u, const double *x,
                         const int64_t *nodes, int64_t count, double *out);

#ifdef __cplusplus
}
#endif
#endif
