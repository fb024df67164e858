/*
 * ok.h -- C ABI of libok.so: the preconditioned Newton-Krylov timestep of the
 * Ohta-Kawasaki equations on one MI355X (gfx950) GPU.
 *
 * Method: Farrell & Pearson, "A preconditioner for the Ohta-Kawasaki
 * equation" (arXiv:1603.04570).
 *   Sec. 1, eqs. (oka)-(okb) with Neumann conditions (okbcs): the PDE
 *     u_t - lap w + sigma (u - m) = 0,   w + eps^2 lap u - u(u^2 - 1) = 0.
 *   Sec. 2, eq. (newton): each Newton iteration of the theta-method solves
 *     J [du; dw] = [f1; f2],  J = [(1+dt th sigma) M, dt th K; -eps^2 K - M_E(u), M].
 *   Sec. 2, eq. (prec): block lower-triangular preconditioner
 *     P^-1 = diag(A~^-1, S~^-1) [I, 0; -C A~^-1, I],
 *   with, eqs. (outer_approx)/(schurinv), S~^-1 = S^^-1 M S^^-1 and
 *     S^ = M + eps sqrt(c) K,  c = dt th / (1 + dt th sigma).
 *   Sec. 3: A~^-1 by Chebyshev semi-iteration on the (scaled) mass matrix.
 *   Sec. 4: GMRES as the outer solver; S^^-1 by multigrid V-cycles.
 *
 * Discretisation: Q1 (bilinear/trilinear) elements on the uniform grid of
 * Omega = (0,1)^d, d in {2,3}, with N elements per direction; all integrals
 * exact (3-point Gauss per direction).  The S^^-1 action is one geometric
 * multigrid V(pre,post) cycle with Chebyshev-Jacobi smoothing, R = P^T and an
 * exact coarse solve; A~^-1 is Chebyshev-Jacobi on M; the outer solver is
 * flexible GMRES(m), right preconditioned, modified Gram-Schmidt.
 *
 * Data layout (every array argument): FP64, contiguous, device memory, node
 * index i + (N+1)*(j + (N+1)*k) with x fastest; a field has n = (N+1)^d
 * entries; a two-field vector is [u-block; w-block] (2n entries).  Arrays must
 * be 8-byte aligned; 256-byte alignment is recommended.
 *
 * Memory ownership: the caller allocates all device memory -- the state
 * vectors and one workspace blob of ok_workspace_bytes() bytes -- and keeps it
 * alive until ok_destroy().  The library never allocates device memory; it
 * owns only its host-side context and a few HIP events/graphs.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  Apply functions (ok_jacobian_apply, ok_precond_apply, ...) are
 * asynchronous on that stream.  Functions that return host scalars or stats
 * (ok_residual, ok_newton_step, ok_timestep, ok_fgmres) synchronise it.
 * A context must not be used from two streams or threads at once.
 *
 * Errors: every entry point returns 0 on success or a negative ok_status.
 * Nothing throws across the ABI.  ok_last_error() gives a message for the
 * last failure on a context.  On a solver failure the state holds the last
 * iterate and the info/stats structs are filled.
 */
#ifndef OK_H
#define OK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ok_status {
  OK_SUCCESS = 0,
  OK_E_INVALID = -1,       /* bad d, N, parameter range, null/misaligned pointer */
  OK_E_WORKSPACE = -2,     /* workspace null, misaligned or smaller than required */
  OK_E_HIP = -3,           /* a HIP runtime call or kernel launch failed */
  OK_E_GMRES_MAXIT = -4,   /* FGMRES hit gmres_max_restarts without converging
                              (MINRES: its iteration limit)                    */
  OK_E_NEWTON_MAXIT = -5,  /* Newton hit newton_max_it without converging */
  OK_E_NONFINITE = -6,     /* NaN/Inf in ||F|| or in the Krylov recurrence */
  OK_E_REJECTED = -7       /* serving: request refused (queue full) or dropped at a stop */
};

/* Preconditioner precision. */
#define OK_FP64 0   /* everything in FP64 */
#define OK_MIXED 1  /* Chebyshev (A~^-1), multigrid (S^^-1), mass action and the
                       stored preconditioned vectors in FP32; FGMRES, J, the
                       residual and the M_E(u) coupling stay FP64 */

typedef struct ok_ctx ok_ctx;

typedef struct {
  int32_t dim;             /* d in {2,3}                                         */
  int32_t n;               /* N elements per direction; N = Nc * 2^(levels-1),  */
                           /* Nc >= 2 (default levels: halve down to N <= 8)     */
  double eps;              /* interfacial thickness epsilon > 0 (Sec. 1)        */
  double sigma;            /* nonlocal coefficient sigma >= 0 (Sec. 1)          */
  double m;                /* mean value m of u, |m| < 1 (Sec. 1)               */
  double dt;               /* timestep > 0                                       */
  double theta;            /* theta-method parameter, 0 < theta <= 1 (Sec. 2)    */
  int32_t precision;       /* OK_FP64 or OK_MIXED                                */
  int32_t gmres_restart;   /* m of FGMRES(m), 1..64 (default 30)                 */
  int32_t gmres_max_restarts; /* restarts allowed after the first cycle (10)     */
  double gmres_rtol;       /* stop at ||r||_2 <= rtol ||b||_2 (1e-8)             */
  double newton_atol;      /* stop at ||F||_2 <= atol (1e-10)                    */
  int32_t newton_max_it;   /* (25)                                               */
  int32_t cheb_A_its;      /* Chebyshev iterations for A~^-1, >= 1 (10)          */
  int32_t schur_richardson;/* Richardson iterations on S with S~^-1, >= 1 (1)    */
  int32_t mg_levels;       /* 0 = automatic                                      */
  int32_t mg_pre, mg_post; /* Chebyshev smoothing iterations, >= 1 (2, 2)        */
  int32_t mg_cycles;       /* V-cycles per S^^-1 application, >= 1 (1)           */
  int32_t linear_solver;   /* Newton's linear solver (OK_SOLVER_FGMRES)           */
} ok_params;

/* Newton's linear solver.
 *   OK_SOLVER_FGMRES: FGMRES(m) on eq. (newton) with the block preconditioner
 *     of eq. (prec) (the paper's method).
 *   OK_SOLVER_MINRES: preconditioned MINRES on the symmetric rearrangement of
 *     (newton) that Sec. 2 notes after (schurapprox),
 *       [c K, M; M, -eps^2 K - M_E(u)] [dw; du] = [f1/(1+dt th sigma); f2],
 *     with the block-diagonal preconditioner diag((alpha/c) S^^-1,
 *     (c/alpha) S^^-1), S^ = M + alpha K, alpha = eps sqrt(c): the singular
 *     (1,1)-block c K is replaced by (c/alpha) S^ = c K + (sqrt(c)/eps) M and
 *     the Schur complement of that block (M_E dropped) by S^ ((c/alpha)
 *     S^)^-1 S^ = (alpha/c) S^; for M_E = 0 the preconditioned spectrum is
 *     +-sqrt(1+x^2)/(1+x), x = alpha lambda, inside +-[1/sqrt(2), 1].  Stops
 *     when the preconditioned residual norm falls to gmres_rtol of its
 *     initial value, after at most gmres_restart*(gmres_max_restarts+1)
 *     iterations.  FP64 only (precision must be OK_FP64). */
#define OK_SOLVER_FGMRES 0
#define OK_SOLVER_MINRES 1

typedef struct {
  int32_t status;          /* result of this Newton iteration's linear solve    */
  int32_t fgmres_its;      /* FGMRES iterations (all cycles); MINRES iterations
                              for OK_SOLVER_MINRES                               */
  int32_t restarts;        /* FGMRES restarts taken (0 for MINRES)               */
  double fnorm;            /* ||F(u,w)||_2 before the update                     */
  double lin_res;          /* final FGMRES residual estimate / ||F||; MINRES:
                              preconditioned residual norm / its initial value */
} ok_newton_info;

#define OK_HIST 256
typedef struct {
  int32_t status;
  int32_t steps_done;
  int32_t newton_its;                  /* total over all steps                   */
  int32_t fgmres_its_total;
  int32_t newton_per_step[OK_HIST];    /* Newton iterations of each step         */
  int32_t fgmres_its[OK_HIST];         /* linear-solver iterations of each Newton
                                          iteration (FGMRES, or MINRES)          */
  double fnorm[OK_HIST];               /* ||F|| at each residual evaluation      */
  int32_t fnorm_count;
  double step_ms[OK_HIST];             /* wall time of each step (HIP events)    */
} ok_stats;

/* Fill *p with the defaults above (dim=3, n=128, eps=0.01, sigma=1000,
 * m=0.1, dt=2e-5, theta=1, OK_FP64). */
int ok_default_params(ok_params *p);

/* Bytes of device workspace ok_assemble_mesh needs for these parameters
 * (the whole per-problem HBM footprint apart from the caller's u, w). */
int ok_workspace_bytes(const ok_params *p, size_t *bytes);

/* Set up a problem (Sec. 2: the preconditioner needs no reassembly between
 * Newton steps, so everything is built once here): derived constants c,
 * eps sqrt(c), 1 + dt th sigma; the multigrid levels and closed-form
 * Chebyshev intervals; the coarse-level exact solver; the carving of d_ws.
 * d_ws: device pointer, 256-byte aligned, ws_bytes >= ok_workspace_bytes().
 * On success *out owns a host context; free it with ok_destroy(). */
int ok_assemble_mesh(const ok_params *p, void *d_ws, size_t ws_bytes, void *stream,
                     ok_ctx **out);

/* Newton residual of the theta-method (Sec. 2, the right-hand side of
 * (newton) is f = -F):
 *   F1 = M(u - un) + dt K (th w + (1-th) wn) + dt sigma M (th u + (1-th) un - m)
 *   F2 = M w - eps^2 K u - N(u),  N_i = int (u^3 - u) phi_i.
 * u, w, un: n each; wn: n (may be NULL when theta == 1); d_F: 2n output (may
 * be NULL).  *h_norm (may be NULL) receives ||F||_2.  Synchronises. */
int ok_residual(ok_ctx *ctx, const double *d_u, const double *d_w, const double *d_un,
                const double *d_wn, double *d_F, double *h_norm, void *stream);

/* ok_residual for callers that cannot allocate device memory or take a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same F and ||F||_2, bit for bit, with no ctx
 * and no workspace.  Its scratch (constants record, three fields of n
 * doubles, reduction partials) is a static device array of 64 MiB that each
 * GPU the library runs on holds until the process ends; it calls no
 * hipMalloc/hipFree and no allocating library routine.  Sizes whose scratch
 * exceeds 64 MiB (more than about 2.79M nodes: 3D N > 140, 2D N > 1670) are
 * rejected with OK_E_WORKSPACE before anything runs; invalid parameters,
 * null or misaligned pointers give OK_E_INVALID.  *p is validated as by
 * ok_workspace_bytes (only dim, n and the physical parameters are used).
 * Calls on one GPU share its scratch: they are serialised by a host lock
 * and each synchronises its stream before returning; kernels of two calls
 * that overlapped on one GPU would race.  Arguments as for ok_residual. */
int ok_residual_noalloc(const ok_params *p, const double *d_u, const double *d_w,
                        const double *d_un, const double *d_wn, double *d_F, double *h_norm,
                        void *stream);

/* y = J(u) x, eq. (newton): y1 = (1+dt th sigma) M x1 + dt th K x2,
 * y2 = -eps^2 K x1 - M_E(u) x1 + M x2.  u: n; x, y: 2n (x != y).  Async. */
int ok_jacobian_apply(ok_ctx *ctx, const double *d_u, const double *d_x, double *d_y,
                      void *stream);

/* The symmetric rearranged system (OK_SOLVER_MINRES above): y = A_sym x with
 * x, y in the order [w-block; u-block] (2n each, x != y); and its solution by
 * preconditioned MINRES from x = 0 (b, x in the same order; *its receives
 * the iterations).  ok_minres synchronises; it returns OK_E_GMRES_MAXIT when
 * the iteration limit is reached first (x then holds the last iterate).
 * Both require precision OK_FP64; ok_minres also needs a context created with
 * linear_solver = OK_SOLVER_MINRES (its work vectors, and a second set of
 * multigrid work vectors: the two V-cycles of the block preconditioner run
 * concurrently, the second on a stream the context creates and owns, joined
 * back into `stream` before the next step), else OK_E_INVALID. */
int ok_sym_apply(ok_ctx *ctx, const double *d_u, const double *d_x, double *d_y, void *stream);
int ok_minres(ok_ctx *ctx, const double *d_u, const double *d_b, double *d_x, int32_t *its,
              void *stream);

/* z = P^-1 r, eq. (prec) with the matching Schur approximation (schurinv):
 *   z1 = Chebyshev_M(r1) / (1 + dt th sigma)
 *   y  = r2 + eps^2 K z1 + M_E(u) z1                (= r2 - C z1)
 *   z2 = S^^-1 M S^^-1 y  (multigrid; Richardson on S if schur_richardson > 1)
 * u: n; r, z: 2n (r != z).  Async. */
int ok_precond_apply(ok_ctx *ctx, const double *d_u, const double *d_r, double *d_z,
                     void *stream);

/* Components of the preconditioner, exposed for testing:
 * x = Chebyshev_M(r) (cheb_A_its iterations on M, no 1+dt th sigma scaling);
 * x = MG(b) (`cycles` V-cycles on M + eps sqrt(c) K from x = 0).
 * FP64 in/out of n entries regardless of precision.  Async. */
int ok_cheb_mass(ok_ctx *ctx, const double *d_r, double *d_x, void *stream);
int ok_mg_apply(ok_ctx *ctx, const double *d_b, double *d_x, int32_t cycles, void *stream);

/* Solve J(u) x = b with FGMRES(m) from x = 0 (Sec. 2 and 4).  u: n; b, x: 2n.
 * *its (may be NULL) receives the iteration count.  Synchronises. */
int ok_fgmres(ok_ctx *ctx, const double *d_u, const double *d_b, double *d_x, int32_t *its,
              void *stream);

/* ONE Newton iteration in place: F(u,w), then J dx = -F by the context's
 * linear solver (FGMRES, or MINRES on the symmetric rearrangement), then
 * (u,w) += dx.  un, wn: previous time level (wn may be NULL if theta == 1).
 * info (may be NULL) is filled.  Synchronises. */
int ok_newton_step(ok_ctx *ctx, double *d_u, double *d_w, const double *d_un,
                   const double *d_wn, ok_newton_info *info, void *stream);

/* nsteps timesteps in place: for each, (un,wn) <- (u,w) and Newton from
 * (u,w) = (un,wn) until ||F||_2 <= newton_atol.  stats may be NULL.
 * Synchronises. */
int ok_timestep(ok_ctx *ctx, double *d_u, double *d_w, int32_t nsteps, ok_stats *stats,
                void *stream);

/* Per-kernel timing for roofline reporting: after ok_profile_enable(ctx,
 * mask) every launch of a kernel class c with bit (1 << c) set in mask is
 * bracketed by HIP events on the stream it runs on (captured graphs are not
 * used meanwhile); ok_profile_read(ctx, c, ...) returns, for class c, the
 * number of launches, their summed duration and the algorithmic bytes they
 * moved (each vector read once and written once).  ok_profile_enable resets
 * the records; mask 0 stops profiling.
 *   OK_K_CHEB_MASS: middle Chebyshev iterations on M (the A~^-1 block)
 *   OK_K_MG_SMOOTH: finest-level smoother and residual launches of the V-cycle
 *   OK_K_ELEMENT:   quadrature passes (M_E(u) x, N(u))
 *   OK_K_KRYLOV:    Gram-Schmidt steps and dot products of FGMRES */
enum ok_kernel_class {
  OK_K_NONE = 0, OK_K_CHEB_MASS = 1, OK_K_MG_SMOOTH = 2, OK_K_ELEMENT = 3,
  OK_K_KRYLOV = 5
};
int ok_profile_enable(ok_ctx *ctx, int32_t class_mask);
int ok_profile_read(ok_ctx *ctx, int32_t kernel_class, int64_t *launches, double *total_ms,
                    double *bytes);

/* Tile autotuner: time the candidate launch shapes (nodes per thread x planes
 * per block) of the stencil kernels on this problem's grids -- every
 * multigrid level for the one-field kernels, the finest grid for the
 * two-field Jacobian kernel -- with HIP events on `stream`, and keep the
 * fastest.  The choice is stored process-wide, keyed by (d, N+1, fields,
 * precision), and used by every later launch on such a grid.  Results are
 * bitwise the same for every shape.  *entries (may be NULL) receives the
 * number of table entries set.  Synchronises; run it outside timed regions. */
int ok_autotune(ok_ctx *ctx, void *stream, int32_t *entries);

/* Initial chemical potential w0 from (okb) in weak form, as the paper's
 * experiments derive it from u0 (Sec. 4): solves M w = eps^2 K u + N(u) by
 * restarted Chebyshev iterations on M in FP64 until the residual is below
 * 1e-15 of the right-hand side.  d_u, d_w: n entries; synchronises. */
int ok_initial_w(ok_ctx *ctx, const double *d_u, double *d_w, void *stream);

/* Process-wide tuning options (results are bitwise the same either way,
 * except for OK_OPT_GRAM_SCHMIDT, whose two forms agree to rounding):
 *   OK_OPT_FUSE_CHEB: 1 (default) runs consecutive middle iterations of the
 *   Chebyshev iteration on M two per pass (each vector read and written once
 *   per pair); 0 runs them one per pass.
 *   OK_OPT_FUSE_MG: 1 (default) runs, on multigrid levels where ok_autotune
 *   found it faster (or where ok_set_launch_shape set OK_SHAPE_MG_POST), the
 *   two pre-smoothing iterations with the residual in one pass and the two
 *   post-smoothing iterations in one pass (V(2,2) cycles); 0 runs every
 *   iteration and the residual in passes of their own everywhere.
 *   OK_OPT_ISSUE_AHEAD: 0 (default) waits for each FGMRES iteration's stop
 *   test before issuing the next; 1 issues iteration j before the host reads
 *   the stop test of iteration j-1 (one iteration after the last is issued
 *   and does nothing).  Measured on 3D 128^3 and in serving it gained
 *   nothing, so it is off by default.
 *   OK_OPT_TRACE_RANGES: 0 (default); 1 opens a host-side ROCTX range
 *   (rocprofv3 --marker-trace) around every timestep ("timestep"), Newton
 *   iteration ("newton iteration"), FGMRES restart cycle ("fgmres cycle"),
 *   FGMRES iteration ("fgmres iteration") and serving-pool tick ("serve
 *   tick").  Ranges cover the host's issue and wait, so with the default
 *   (no issue-ahead) an FGMRES iteration's range spans its device work.
 *   OK_OPT_GRAM_SCHMIDT: orthogonalisation of each Arnoldi step of FGMRES.
 *   0 (default): modified Gram-Schmidt in inverse compact WY form (Sec. 4's
 *   GMRES; Swirydowicz et al., Numer. Linear Algebra Appl. 2021): one pass
 *   forms <w, v_i> for every basis vector and the new row of V^T V, a
 *   triangular solve gives modified Gram-Schmidt's coefficients, one pass
 *   subtracts the projections; basis vectors are kept unnormalised with a
 *   scale.  1: modified Gram-Schmidt one projection per pass (each fused
 *   with the next dot product), normalised basis vectors.  Both compute the
 *   same Arnoldi relation; results agree to rounding.
 *   OK_OPT_FUSE_PROLONG: 1 (default) adds the interpolated coarse-grid
 *   correction while the post-smoother stages its input, on 3D levels that
 *   run the strip post-smoother (OK_SHAPE_MG_POST_STRIP set by ok_autotune
 *   or ok_set_launch_shape) with the fused V(2,2) smoothers in FP64; 0 adds
 *   it in a pass of its own first.  Single-precision smoothers (OK_MIXED)
 *   always use the separate pass. */
enum ok_option {
  OK_OPT_FUSE_CHEB = 1, OK_OPT_FUSE_MG = 2, OK_OPT_ISSUE_AHEAD = 3, OK_OPT_TRACE_RANGES = 4,
  OK_OPT_GRAM_SCHMIDT = 5, OK_OPT_FUSE_PROLONG = 6
};
int ok_set_option(int32_t option, int32_t value);

/* Launch shape of the streaming node-stencil kernels on one grid: the
 * process-wide table entry that ok_autotune writes, set by hand (to pin a
 * shape for timing, or to check that results do not depend on it).
 *   dim, n: the grid (n elements per direction; any level of a hierarchy);
 *   kernel: OK_SHAPE_STENCIL (one stenciled field: Chebyshev iterations,
 *     multigrid residuals, coupling), OK_SHAPE_STENCIL2 (two fields: the
 *     mass/stiffness pairs of residual and Jacobian), OK_SHAPE_CHEB2 (two
 *     fused Chebyshev iterations on M), OK_SHAPE_MG_PRE / OK_SHAPE_MG_POST
 *     (the fused smoothers of a multigrid level);
 *   precision: OK_FP64 or OK_MIXED (the preconditioner's storage type);
 *   items, threads: a block of `threads` threads covers items*threads nodes
 *     of a plane.  STENCIL: 256 threads of 1, 2, 4 or 8 nodes, in 3D also 512
 *     threads of 1, 2 or 4; STENCIL2: 256 threads of 1, 2 or 4; CHEB2,
 *     MG_PRE, MG_POST: 256 threads (3D also 512) of 1 or 2; CHEB2_TILE,
 *     MG_PRE_TILE, MG_POST_TILE (3D only): 256 or 512 threads of 1 or 2
 *     nodes, the tile (about items*threads nodes) chosen by the library;
 *     CHEB2_STRIP, MG_PRE_STRIP, MG_POST_STRIP (3D only): items selects the
 *     window (1: 32x32 nodes, strips of 4; 2: 32x16, strips of 2; 3: 64x16,
 *     strips of 4; 4: 32x24, strips of 3; 5: 64x12, strips of 3), threads
 *     must be 256.  items = 0 removes the entry
 *     (built-in default shape; threads and zchunks are then ignored);
 *   zchunks: the n+1 planes of the streaming axis are split evenly into
 *     1..n+1 ranges, one block per (plane chunk, range).
 * Every node's arithmetic is the same for every shape, so results are
 * bitwise equal.  Launches read the table when issued; HIP graphs captured
 * earlier (ok_use_graphs) keep the shapes they were captured with.  Returns
 * OK_E_INVALID for an argument out of range. */
enum ok_shape_kernel {
  OK_SHAPE_STENCIL = 1,
  OK_SHAPE_STENCIL2 = 2,
  OK_SHAPE_CHEB2 = 3,
  OK_SHAPE_MG_PRE = 4,  /* fused pre-smoothing + residual of a multigrid level */
  OK_SHAPE_MG_POST = 5, /* fused post-smoothing of a multigrid level */
  OK_SHAPE_CHEB2_TILE = 6, /* CHEB2 on rectangular in-plane tiles (3D); while set,
                              the fused pairs of that grid use it */
  OK_SHAPE_MG_PRE_TILE = 7, /* MG_PRE / MG_POST on in-plane tiles (3D); used while */
  OK_SHAPE_MG_POST_TILE = 8, /* set on a level whose fused smoothers are on */
  OK_SHAPE_CHEB2_STRIP = 9,  /* CHEB2, MG_PRE, MG_POST on overlapping in-plane windows */
  OK_SHAPE_MG_PRE_STRIP = 10, /* with a column strip of nodes per thread (3D); used */
  OK_SHAPE_MG_POST_STRIP = 11 /* while set, before any TILE entry */
};
int ok_set_launch_shape(int32_t dim, int32_t n, int32_t kernel, int32_t precision, int32_t items,
                        int32_t threads, int32_t zchunks);
/* The table entry ok_set_launch_shape or ok_autotune last wrote for (dim, n,
 * kernel, precision): *items, *threads, *zchunks as ok_set_launch_shape takes
 * them, all three 0 when the grid uses the built-in default.  Host-side only
 * (no device access); lets a caller save the autotuned shapes and pin them
 * in another process.  OK_E_INVALID for an argument out of range or a null
 * output pointer. */
int ok_get_launch_shape(int32_t dim, int32_t n, int32_t kernel, int32_t precision, int32_t *items,
                        int32_t *threads, int32_t *zchunks);

/* Launch mode of the FGMRES iterations.  enable != 0: the context gets a HIP
 * stream of its own (default priority) and captures each Arnoldi iteration j
 * (preconditioner, Jacobian, Gram-Schmidt, Givens) once as a HIP graph, keyed
 * by the state pointer, and replays it; later calls with another state
 * pointer, or an ok_autotune, re-capture.  Results are bitwise the same as
 * with enable == 0 (kernels launched one by one on the caller's stream, the
 * default).  While a kernel class is profiled (ok_profile_enable) kernels are
 * launched one by one. */
int ok_use_graphs(ok_ctx *ctx, int32_t enable);

/* ---- Batched sweeps: many independent problems in lockstep ----
 * Instances whose parameters agree on (dim, n, precision and the solver
 * counts) form a class; each class is one set of grouped kernel launches
 * (grid = blocks of one instance x instances in the class), with the
 * per-instance physics (eps, sigma, m, dt, theta, tolerances) in a device
 * table and per-instance activity flags, so an instance that has converged
 * costs nothing in later launches.  The solver state (u, w) of every instance
 * lives in the batch workspace; ok_batch_set_state / ok_batch_get_state copy
 * it in and out (device to device).  The arithmetic of each instance is the
 * same as in a single-problem run: results are bitwise identical. */
typedef struct ok_batch ok_batch;

/* Workspace bytes for `count` instances with parameters params[0..count). */
int ok_batch_workspace_bytes(const ok_params *params, int32_t count, size_t *bytes);
/* Create a batch over the caller's workspace (256-byte aligned, at least
 * ok_batch_workspace_bytes bytes).  Synchronises `stream`. */
int ok_batch_create(const ok_params *params, int32_t count, void *d_ws, size_t ws_bytes,
                    void *stream, ok_batch **out);
/* Copy instance i's state in (from) or out (to) device arrays of n entries each. */
int ok_batch_set_state(ok_batch *b, int32_t i, const double *d_u, const double *d_w,
                       void *stream);
int ok_batch_get_state(ok_batch *b, int32_t i, double *d_u, double *d_w, void *stream);
/* nsteps timesteps of every instance (Newton and FGMRES in lockstep across
 * all instances and classes).  stats (may be NULL): `count` entries.
 * Returns the first failure of any instance (its stats carry its status);
 * the batch stops after the step in which an instance failed, the others
 * having completed that step (stats.steps_done). */
int ok_batch_timestep(ok_batch *b, int32_t nsteps, ok_stats *stats, void *stream);
/* ok_autotune for every class of the batch. */
int ok_batch_autotune(ok_batch *b, void *stream, int32_t *entries);
/* Number of classes (grouped launch sets) the instances fell into. */
int ok_batch_classes(const ok_batch *b);
/* As ok_use_graphs, for every class of the batch.  A batch starts with
 * graphs on: each class runs its FGMRES iterations from captured graphs on a
 * stream of its own, so the classes of a batch overlap on the device. */
int ok_batch_use_graphs(ok_batch *b, int32_t enable);
int ok_batch_destroy(ok_batch *b);
const char *ok_batch_last_error(const ok_batch *b);

/* ---- Serving: timestep requests of many resident simulations ----
 * A server holds the state (u, w) of `nsims` simulations resident in the
 * caller's workspace and advances them on request.  A request (simulation,
 * nsteps, arrival time) waits in a bounded queue until its simulation has no
 * other request in flight (FIFO per simulation) and a slot is free: slots
 * live in pools, one pool per class (same grid, precision and solver
 * counts), carved on demand from the rest of the workspace (the HBM budget);
 * idle pools are released when a waiting request of another class needs the
 * room.  The worker thread runs ticks: one Newton iteration (residual test,
 * FGMRES solve, update, residual test, Sec. 2) of every occupied slot of
 * every pool in grouped launches; requests admitted between ticks join the
 * next tick (continuous batching).  Each simulation's arithmetic is that of a
 * single-problem ok_timestep: results are bitwise the same alone and in the
 * mix.  Times are seconds since the server was created (ok_server_now). */
typedef struct ok_server ok_server;
typedef struct {
  int32_t max_queue;           /* arrived requests waiting for a slot; arrivals
                                  beyond it are rejected (OK_E_REJECTED); 256 */
  int32_t max_slots_per_pool;  /* instances per pool (upper bound); 16 */
  int32_t graphs;              /* replay captured FGMRES iterations; 1 */
  int32_t reserved;
  double pool_bytes;           /* a pool holds fewer slots if its bytes would
                                  exceed this; 32 GiB */
} ok_server_config;
typedef struct {
  int64_t ticket;
  int32_t sim, nsteps, status, steps_done, newton_its, fgmres_its;
  double t_arrival, t_admit, t_done; /* t_admit < 0: never admitted */
} ok_request_result;
typedef struct {
  int64_t submitted, admitted, completed, failed, rejected, deferred;
  int64_t ticks, pools_created, pools_freed, pools_live;
  int64_t max_active, max_queue_seen, peak_bytes, bytes_in_use;
  double dof_steps;   /* sum over completed requests of 2(N+1)^d x steps */
  double busy_s;      /* wall time spent in ticks */
  double now;         /* ok_server_now at the time of the call */
} ok_server_stats;

int ok_server_default_config(ok_server_config *cfg);
/* Bytes of resident state (u and w of every simulation, 256-byte aligned). */
int ok_server_state_bytes(const ok_params *sims, int32_t nsims, size_t *bytes);
/* Create a server over the caller's workspace (256-byte aligned): the first
 * ok_server_state_bytes hold the states, the rest is the pool budget, which
 * must hold at least one slot of the largest class.  cfg may be NULL.  The
 * server creates a stream of its own (default priority); `stream` is unused. */
int ok_server_create(const ok_params *sims, int32_t nsims, const ok_server_config *cfg,
                     void *d_ws, size_t ws_bytes, void *stream, ok_server **out);
/* Copy a simulation's state in or out (n entries each); only while stopped. */
int ok_server_set_state(ok_server *s, int32_t sim, const double *d_u, const double *d_w,
                        void *stream);
int ok_server_get_state(ok_server *s, int32_t sim, double *d_u, double *d_w, void *stream);
/* Start the worker thread (on the calling thread's current device). */
int ok_server_start(ok_server *s);
double ok_server_now(const ok_server *s);
/* Enqueue `nsteps` timesteps of simulation `sim`, arriving at t_arrival
 * (seconds, ok_server_now's clock; < 0: now).  Thread-safe. */
int ok_server_submit(ok_server *s, int32_t sim, int32_t nsteps, double t_arrival,
                     int64_t *ticket);
/* Up to `max` finished requests (done, failed or rejected) into out[];
 * waits up to wait_s seconds for the first one while the server runs. */
int ok_server_poll(ok_server *s, ok_request_result *out, int32_t max, int32_t *count,
                   double wait_s);
/* Stop the worker.  drain != 0: first serve every submitted request
 * (including future arrivals); drain == 0: stop after the current tick,
 * reporting unstarted and unfinished requests as OK_E_REJECTED (the state
 * of an unfinished one is its last Newton iterate).  Returns a fatal error
 * of the worker, if any. */
int ok_server_stop(ok_server *s, int32_t drain);
int ok_server_get_stats(ok_server *s, ok_server_stats *out);
int ok_server_reset_stats(ok_server *s);
int ok_server_destroy(ok_server *s);
const char *ok_server_last_error(const ok_server *s);

/* Destroy a context (frees host state only; the caller frees its memory). */
int ok_destroy(ok_ctx *ctx);

const char *ok_error_string(int status);
const char *ok_last_error(const ok_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* OK_H */
