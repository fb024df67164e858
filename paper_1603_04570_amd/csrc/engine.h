// Host engine of libok.so: a class of B instances that share the grid and the
// precision, its device memory layout, and the lockstep solver operations
// (preconditioner, Jacobian, residual, FGMRES, Newton, timestep) over groups
// of classes.  A single solve is one class with B = 1.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "ok_internal.h"

namespace okd {

// Profiling of one kernel class with HIP events on the launch stream.
struct ProfPair {
  hipEvent_t a, b;
  double bytes;
  int count;  // kernel launches between the two events
  int cls;    // kernel class of those launches
};
struct Prof {
  int mask = 0;  // bit c set: launches of kernel class c are timed
  bool capturing = false;  // no events while a graph is being captured
  std::vector<ProfPair> ev;
  size_t used = 0;
  ~Prof();
};

// Per-instance results of a group operation.
struct InstOut {
  int status = 0;      // ok_status of this instance's last operation
  int fgmres_its = 0;  // FGMRES iterations of the last linear solve
  int restarts = 0;
  double fnorm = 0.0;  // ||F|| of the last residual evaluation
  double lin_res = 0.0;
};

// Execution resources of a class that runs its FGMRES iterations from captured
// graphs on a stream of its own (owned; released with the class).
struct ClassExec {
  hipStream_t xs = nullptr;           // class stream (default priority, non-blocking)
  hipEvent_t fork = nullptr, join = nullptr;
  std::vector<hipGraphExec_t> iter;   // one graph per Arnoldi index j
  const void* key = nullptr;          // state pointer the graphs were captured with
  bool graphs = true;
  void clear_graphs();
  ~ClassExec();
};

// A second stream of a MINRES class with its fork and join events: the two
// V-cycles of the block-diagonal preconditioner run concurrently (owned;
// default priority; released with the class).
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  ~SideStream();
};

// Pinned two-slot host copy of the activity flags with an event per slot:
// the FGMRES driver reads the flags that iteration j-1 left while iteration j
// already runs (owned; released with the class).
struct FlagPipe {
  int* h = nullptr;                      // [2][B]
  hipEvent_t ev[2] = {nullptr, nullptr};
  int pend[2] = {-1, -1};               // iteration whose flags each slot receives
  ~FlagPipe();
};

struct ClassCtx {
  // ---- configuration (common to the class) ----
  ok_params shape{};  // dim, n, precision, solver counts (physics per instance below)
  int B = 0;          // instances
  int dim = 0, L = 0, m = 0;
  int nv = 0;         // vectors of 2n per instance in V (FGMRES basis or MINRES work)
  int64_t vs = 0;     // entries between consecutive vectors of V and of Z: 2n rounded up
                      // to 64, so every vector starts 256-byte aligned
  bool mixed = false;
  size_t psz = 8;  // bytes per preconditioner word
  int64_t n = 0;   // finest nodes per instance
  Grid lev[kMaxLevels]{};
  std::vector<ok_params> ip;      // per-instance parameters
  std::vector<InstCoef> hcoef;    // host copy of the constants table
  // ---- device memory (SoA: every array is [instance][length]) ----
  InstCoef* coef = nullptr;
  int *act = nullptr, *part = nullptr, *incyc = nullptr, *aux = nullptr;  // [B] flags
  double *V = nullptr, *X = nullptr, *Bv = nullptr, *T1 = nullptr;
  double *un = nullptr, *wn = nullptr, *G = nullptr, *su = nullptr, *sw = nullptr;
  double* Q = nullptr;  // -(M_E(u) z1 + eps^2 K z1) of the last preconditioner application
  double *pA = nullptr, *pB = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr;
  double *g = nullptr, *y = nullptr, *kr = nullptr, *nrm = nullptr;
  // two-pass Arnoldi projection: basis scales (m+1), lower part of V^T V
  // ((m+1)^2), update coefficients (m+1), dot partials (2m rows of
  // red_blocks(2n))
  double *sc = nullptr, *Lm = nullptr, *hcf = nullptr, *pd = nullptr;
  double* mr = nullptr;  // MINRES scalars (MR_COUNT per instance)
  void *Z = nullptr, *zt = nullptr;
  void *cr = nullptr, *cda = nullptr, *cdb = nullptr, *yv = nullptr, *tv = nullptr, *sv = nullptr;
  void* cr2 = nullptr;  // second Chebyshev residual (fused iterations ping-pong r)
  void* rich = nullptr;  // Richardson on S (schur_richardson > 1): 4 vectors of n
  void* mg[kMaxLevels][5]{};  // x, b, r, d, d' per level
  void* mg2[kMaxLevels][5]{};  // a second set (MINRES classes): its two V-cycles run at once
  // ---- host mirrors ----
  std::vector<int> h_act, h_part, h_aux;
  std::vector<int> h_hasF;  // Bv holds F of the current iterate (Newton ticks)
  std::vector<double> h_kr, h_nrm;
  std::vector<InstOut> out;
  std::vector<int> nits;  // Newton iterations of the current timestep, per instance
  Prof* prof = nullptr;  // shared profiling state (may be null)
  std::string* err = nullptr;
  std::unique_ptr<ClassExec> ex;  // null: iterations are launched one kernel at a time on
                                  // the caller's stream
  std::unique_ptr<FlagPipe> fp;   // created by the first FGMRES solve
  std::unique_ptr<SideStream> side;  // created by the first MINRES solve

  int64_t n2() const { return 2 * n; }
  Batch batch(const int* flags) const { return Batch{B, coef, flags}; }
};

// Parameter checks shared by every entry point.
int validate_params(const ok_params* p, std::string& why);
int levels_for(const ok_params* p);
// Two parameter sets can share a class (same grid, precision and solver counts).
bool same_class(const ok_params& a, const ok_params& b);

// Layout: bytes of device memory for a class of B instances of `shape`.
size_t class_bytes(const ok_params& shape, int B, bool with_state);
// Carve a class out of `base` (256-byte aligned) and upload its constants.
int class_init(ClassCtx& c, const ok_params* ps, int B, char* base, bool with_state,
               hipStream_t st, std::string& err);

// ---- group operations (lockstep over all classes of a group) ----
using Group = std::vector<ClassCtx*>;
// y = J(u) x  (u: n, x/y: 2n per instance; FP64 x)
int jac_apply_d(ClassCtx& c, const int* flags, Vec<const double> u, Vec<const double> x,
                Vec<double> y, hipStream_t st);
// z = P^-1 r (FP64 in/out; mixed classes stage through FP32)
int precond_apply_d(ClassCtx& c, const int* flags, Vec<const double> u, Vec<const double> r,
                    Vec<double> z, hipStream_t st);
int cheb_mass_d(ClassCtx& c, const int* flags, Vec<const double> r, Vec<double> x, hipStream_t st);
int mg_apply_d(ClassCtx& c, const int* flags, Vec<const double> b, Vec<double> x, int cycles,
               hipStream_t st);
// The launches of the residual of eq. (newton)'s system on a class: F (2n
// per instance), with t1, t2, G (n each) and the reduction partials part
// (kMaxRedBlocks) as scratch, and nrm[0] = ||F||^2, nrm[1] = ||F|| on the
// device.  wn null: wn is not read (theta = 1).
hipError_t residual_launch(const Grid& g, const Batch& B, Vec<const double> u,
                           Vec<const double> w, Vec<const double> un, Vec<const double> wn,
                           Vec<double> F, Vec<double> t1, Vec<double> t2, Vec<double> G,
                           Vec<double> part, Vec<double> nrm, hipStream_t st);
// The constants-table record of one instance and the grids of its multigrid
// hierarchy (L levels).  p must be valid (validate_params).
void instance_constants(const ok_params& p, InstCoef& C, Grid* lev, int& L);
// F and ||F|| per instance (norms in c.out[i].fnorm); F may be null (uses Bv).
int residual_d(ClassCtx& c, const int* flags, Vec<const double> u, Vec<const double> w,
               Vec<const double> un, Vec<const double> wn, Vec<double> F, hipStream_t st);
// w from u by (okb): M w = eps^2 K u + N(u), restarted Chebyshev on M (FP64)
// until ||rhs - M w|| <= 1e-15 ||rhs|| (at most 8 rounds of 32 iterations).
// Single instance (B = 1); rounds: restarts used.
int initial_w_d(ClassCtx& c, Vec<const double> u, Vec<double> w, int* rounds, hipStream_t st);
// y = A_sym x for the symmetric rearrangement of eq. (newton)'s system,
// x = [dw; du] (2n per instance, FP64 class only):
//   y1 = c K x1 + M x2,  y2 = M x1 - eps^2 K x2 - M_E(u) x2
int sym_apply_d(ClassCtx& c, const int* flags, Vec<const double> u, Vec<const double> x,
                Vec<double> y, hipStream_t st);
// Preconditioned MINRES on the symmetric system for the instances with
// h_part set (FP64 class), from x = 0.  newton: b is the right-hand side of
// eq. (newton) in its row order, scaled here to [b1/(1 + dt th sigma); b2],
// and x is returned in the order [du; dw]; otherwise b and x are in the
// symmetric system's order [dw; du].  Results per instance in out[]
// (fgmres_its: MINRES iterations; lin_res: final preconditioned residual
// norm relative to the initial one).
int minres_class(ClassCtx& c, Vec<const double> u, Vec<const double> b, Vec<double> x,
                 bool newton, hipStream_t st);
// Newton's linear solve J x = b on every class of the group, each with its
// class's solver (FGMRES classes in lockstep, MINRES classes one after
// another); x in the order [du; dw].
int newton_solve_group(const Group& grp, const std::vector<Vec<const double>>& u,
                       const std::vector<Vec<const double>>& b, const std::vector<Vec<double>>& x,
                       hipStream_t st);
// Solve J x = b by FGMRES for the instances with part[i] set (host masks in
// h_part of each class).  Results per instance in out[].
int fgmres_group(const Group& grp, const std::vector<Vec<const double>>& u,
                 const std::vector<Vec<const double>>& b, const std::vector<Vec<double>>& x,
                 hipStream_t st);
// Newton until ||F|| <= atol for the participating instances (h_part);
// un/wn: previous time level.  Records per-instance Newton and FGMRES counts.
struct NewtonLog {
  std::vector<std::vector<int>> its;       // per instance: FGMRES its per Newton iteration
  std::vector<std::vector<double>> fnorm;  // per instance: ||F|| per residual evaluation
};
int newton_group(const Group& grp, const std::vector<Vec<double>>& u,
                 const std::vector<Vec<double>>& w, const std::vector<Vec<const double>>& un,
                 const std::vector<Vec<const double>>& wn, std::vector<NewtonLog>& log,
                 hipStream_t st);
// At most max_iters Newton updates (max_iters < 0: until every participating
// instance stops).  Instances without a current residual (h_hasF == 0) are
// tested first; every update is followed by the residual and its test, so a
// bounded call (one serving tick) ends with each instance's status known:
// OK_SUCCESS when converged, 1 while still iterating, or an error.
int newton_group_iters(const Group& grp, const std::vector<Vec<double>>& u,
                       const std::vector<Vec<double>>& w, const std::vector<Vec<const double>>& un,
                       const std::vector<Vec<const double>>& wn, std::vector<NewtonLog>& log,
                       int max_iters, hipStream_t st);
// Orthogonalisation of the Arnoldi step: 0 (default) two passes over the
// basis (modified Gram-Schmidt in inverse compact WY form, unnormalised
// basis vectors with scales); 1 fused modified Gram-Schmidt, one pass per
// projection, normalised basis vectors.
void ortho_set(int mode);
// Upload host flags (h_part) to the device part/act arrays.
int push_part(ClassCtx& c, hipStream_t st);
// Replace the physical parameters of instance i (same class) and upload its
// constants; stream-ordered.
int set_instance(ClassCtx& c, int i, const ok_params& p, hipStream_t st);
// Give the class its own stream and graph cache (graphs: capture FGMRES
// iterations once per state pointer and replay them).
int enable_exec(ClassCtx& c, bool graphs);
// Tile autotuner over the class's grids.
int autotune_class(ClassCtx& c, hipStream_t st, int* entries);

// Host-side ROCTX ranges for rocprofv3 --marker-trace: one per timestep,
// Newton iteration, FGMRES restart cycle and FGMRES iteration, and per tick of
// a serving pool.  Off by default (no ROCTX call is made then).
extern bool g_trace_ranges;
void trace_ranges_set(int enable);
void trace_push(const char* name);
void trace_pop();
struct TraceRange {
  const bool on;
  explicit TraceRange(const char* name) : on(g_trace_ranges) {
    if (on) trace_push(name);
  }
  ~TraceRange() {
    if (on) trace_pop();
  }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace okd
