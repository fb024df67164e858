// C ABI of libok.so.  The single-problem entry points drive a class of one
// instance; the ok_batch_* entry points drive classes of many instances in
// lockstep (grouped kernel launches, per-instance activity flags).
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "engine.h"

using namespace okd;

struct ok_ctx {
  ClassCtx cls;
  Prof prof;
  std::string err;
};

struct ok_batch {
  std::vector<ClassCtx> classes;
  std::vector<int> cls_of, idx_of;  // instance -> (class, index in class)
  Prof prof;
  std::string err;
  int count = 0;
};

namespace {

const char* kStatusNames[] = {"success", "invalid argument", "workspace too small or misaligned",
                              "HIP error", "FGMRES did not converge",
                              "Newton did not converge", "non-finite value",
                              "request rejected"};

int fail(std::string* err, int code, const std::string& msg) {
  if (err) *err = msg;
  return code;
}

#define OK_HIP(errp, ...)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (__VA_ARGS__);                                                           \
    if (e_ != hipSuccess)                                                                    \
      return fail(errp, OK_E_HIP, std::string(#__VA_ARGS__).substr(0, 60) + ": " +           \
                                      hipGetErrorString(e_));                                \
  } while (0)

bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

template <class T>
Vec<T> one(T* p) {
  return Vec<T>{p, 0};
}

// Run nsteps timesteps of every instance of a group whose state lives in
// (u[k], w[k]); fills one ok_stats per instance (order: class, index).
int timestep_group(const Group& grp, const std::vector<Vec<double>>& u,
                   const std::vector<Vec<double>>& w, int nsteps,
                   std::vector<std::vector<ok_stats>>& stats, std::string* err, hipStream_t st) {
  const size_t nc = grp.size();
  stats.resize(nc);
  for (size_t k = 0; k < nc; k++) {
    stats[k].assign(grp[k]->B, ok_stats{});
    for (auto& s : stats[k]) std::memset(&s, 0, sizeof(s));
  }
  hipEvent_t e0, e1;
  OK_HIP(err, hipEventCreate(&e0));
  OK_HIP(err, hipEventCreate(&e1));
  int status = OK_SUCCESS;
  for (int s = 0; s < nsteps && status == OK_SUCCESS; s++) {
    TraceRange step_range("timestep");
    OK_HIP(err, hipEventRecord(e0, st));
    std::vector<Vec<const double>> un(nc), wn(nc);
    std::vector<NewtonLog> log(nc);
    for (size_t k = 0; k < nc; k++) {
      ClassCtx& c = *grp[k];
      const Batch all = c.batch(nullptr);
      OK_HIP(err, launch_copy_scale<double, double>(all, Vec<const double>{u[k].p, u[k].s},
                                                    vec(c.un, c.n), 1.0, c.n, st));
      OK_HIP(err, launch_copy_scale<double, double>(all, Vec<const double>{w[k].p, w[k].s},
                                                    vec(c.wn, c.n), 1.0, c.n, st));
      un[k] = Vec<const double>{c.un, c.n};
      wn[k] = Vec<const double>{c.wn, c.n};
      c.h_part.assign(c.B, 1);
      c.h_hasF.assign(c.B, 0);
      c.nits.assign(c.B, 0);
      log[k].its.assign(c.B, {});
      log[k].fnorm.assign(c.B, {});
    }
    int e = newton_group(grp, u, w, un, wn, log, st);
    OK_HIP(err, hipEventRecord(e1, st));
    OK_HIP(err, hipEventSynchronize(e1));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    for (size_t k = 0; k < nc; k++) {
      ClassCtx& c = *grp[k];
      for (int i = 0; i < c.B; i++) {
        ok_stats& S = stats[k][i];
        for (size_t q = 0; q < log[k].fnorm[i].size(); q++)
          if (S.fnorm_count < OK_HIST) S.fnorm[S.fnorm_count++] = log[k].fnorm[i][q];
        for (size_t q = 0; q < log[k].its[i].size(); q++) {
          if (S.newton_its < OK_HIST) S.fgmres_its[S.newton_its] = log[k].its[i][q];
          S.newton_its++;
          S.fgmres_its_total += log[k].its[i][q];
        }
        if (s < OK_HIST) {
          S.newton_per_step[s] = (int)log[k].its[i].size();
          S.step_ms[s] = ms;
        }
        int st_i = c.out[i].status;
        if (st_i != OK_SUCCESS) {
          S.status = st_i;
          if (status == OK_SUCCESS) {
            status = st_i;
            if (err && st_i < 0 && st_i >= -7)
              *err = std::string("instance failed: ") + kStatusNames[-st_i];
          }
        } else {
          S.steps_done++;
        }
      }
    }
    if (e) {
      status = e;
      break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return status;
}

}  // namespace

extern "C" {

int ok_default_params(ok_params* p) {
  if (!p) return OK_E_INVALID;
  std::memset(p, 0, sizeof(*p));
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
  p->linear_solver = OK_SOLVER_FGMRES;
  return OK_SUCCESS;
}

int ok_workspace_bytes(const ok_params* p, size_t* bytes) {
  std::string why;
  int v = validate_params(p, why);
  if (v) return v;
  if (!bytes) return OK_E_INVALID;
  *bytes = class_bytes(*p, 1, false);
  return OK_SUCCESS;
}

int ok_assemble_mesh(const ok_params* p, void* d_ws, size_t ws_bytes, void* stream,
                     ok_ctx** out) {
  if (!out) return OK_E_INVALID;
  *out = nullptr;
  std::string why;
  int v = validate_params(p, why);
  if (v) return v;
  size_t need = class_bytes(*p, 1, false);
  if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < need) return OK_E_WORKSPACE;
  ok_ctx* c = new (std::nothrow) ok_ctx();
  if (!c) return OK_E_INVALID;
  c->cls.err = &c->err;
  c->cls.prof = &c->prof;
  int e = class_init(c->cls, p, 1, (char*)d_ws, false, (hipStream_t)stream, c->err);
  if (e) {
    delete c;
    return e;
  }
  *out = c;
  return OK_SUCCESS;
}

int ok_destroy(ok_ctx* c) {
  if (!c) return OK_E_INVALID;
  delete c;
  return OK_SUCCESS;
}

int ok_residual(ok_ctx* c, const double* u, const double* w, const double* un, const double* wn,
                double* F, double* h_norm, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !w || !un || (c->cls.shape.theta < 1.0 && !wn))
    return fail(&c->err, OK_E_INVALID, "null state");
  if (!aligned8(u) || !aligned8(w) || !aligned8(un) || !aligned8(F))
    return fail(&c->err, OK_E_INVALID, "misaligned");
  ClassCtx& k = c->cls;
  int e = residual_d(k, nullptr, one(u), one(w), one(un), one(wn), Vec<double>{F, 0},
                     (hipStream_t)stream);
  if (e) return e;
  if (h_norm) *h_norm = k.out[0].fnorm;
  return OK_SUCCESS;
}

int ok_jacobian_apply(ok_ctx* c, const double* u, const double* x, double* y, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !x || !y || x == y) return fail(&c->err, OK_E_INVALID, "null or aliased vectors");
  if (!aligned8(u) || !aligned8(x) || !aligned8(y)) return fail(&c->err, OK_E_INVALID, "misaligned");
  return jac_apply_d(c->cls, nullptr, one(u), one(x), one(y), (hipStream_t)stream);
}

int ok_precond_apply(ok_ctx* c, const double* u, const double* r, double* z, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !r || !z || r == z) return fail(&c->err, OK_E_INVALID, "null or aliased vectors");
  if (!aligned8(u) || !aligned8(r) || !aligned8(z)) return fail(&c->err, OK_E_INVALID, "misaligned");
  return precond_apply_d(c->cls, nullptr, one(u), one(r), one(z), (hipStream_t)stream);
}

int ok_cheb_mass(ok_ctx* c, const double* r, double* x, void* stream) {
  if (!c || !r || !x || r == x) return OK_E_INVALID;
  return cheb_mass_d(c->cls, nullptr, one(r), one(x), (hipStream_t)stream);
}

int ok_mg_apply(ok_ctx* c, const double* b, double* x, int32_t cycles, void* stream) {
  if (!c || !b || !x || b == x || cycles < 1) return OK_E_INVALID;
  return mg_apply_d(c->cls, nullptr, one(b), one(x), cycles, (hipStream_t)stream);
}

int ok_fgmres(ok_ctx* c, const double* u, const double* b, double* x, int32_t* its, void* stream) {
  if (!c || !u || !b || !x || b == x) return OK_E_INVALID;
  ClassCtx& k = c->cls;
  k.h_part.assign(1, 1);
  Group grp{&k};
  int e = fgmres_group(grp, {one(u)}, {one(b)}, {one(x)}, (hipStream_t)stream);
  if (its) *its = k.out[0].fgmres_its;
  if (e) return e;
  if (k.out[0].status) return fail(&c->err, k.out[0].status, kStatusNames[-k.out[0].status]);
  return OK_SUCCESS;
}

int ok_sym_apply(ok_ctx* c, const double* u, const double* x, double* y, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !x || !y || x == y) return fail(&c->err, OK_E_INVALID, "null or aliased vectors");
  if (!aligned8(u) || !aligned8(x) || !aligned8(y)) return fail(&c->err, OK_E_INVALID, "misaligned");
  if (c->cls.mixed) return fail(&c->err, OK_E_INVALID, "the symmetric system is FP64 only");
  return sym_apply_d(c->cls, nullptr, one(u), one(x), one(y), (hipStream_t)stream);
}

int ok_minres(ok_ctx* c, const double* u, const double* b, double* x, int32_t* its, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !b || !x || b == x) return fail(&c->err, OK_E_INVALID, "null or aliased vectors");
  if (!aligned8(u) || !aligned8(b) || !aligned8(x)) return fail(&c->err, OK_E_INVALID, "misaligned");
  ClassCtx& k = c->cls;
  if (k.mixed) return fail(&c->err, OK_E_INVALID, "MINRES requires precision OK_FP64");
  if (k.shape.linear_solver != OK_SOLVER_MINRES)
    return fail(&c->err, OK_E_INVALID, "context not created for MINRES (linear_solver)");
  k.h_part.assign(1, 1);
  int e = minres_class(k, one(u), one(b), one(x), false, (hipStream_t)stream);
  if (its) *its = k.out[0].fgmres_its;
  if (e) return e;
  if (k.out[0].status) return fail(&c->err, k.out[0].status, kStatusNames[-k.out[0].status]);
  return OK_SUCCESS;
}

int ok_newton_step(ok_ctx* c, double* u, double* w, const double* un, const double* wn,
                   ok_newton_info* info, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !w || !un || (c->cls.shape.theta < 1.0 && !wn))
    return fail(&c->err, OK_E_INVALID, "null state");
  hipStream_t st = (hipStream_t)stream;
  ClassCtx& k = c->cls;
  int e = residual_d(k, nullptr, one((const double*)u), one((const double*)w), one(un), one(wn),
                     vec(k.Bv, 0), st);
  if (e) return e;
  ok_newton_info inf{};
  inf.fnorm = k.out[0].fnorm;
  if (!std::isfinite(inf.fnorm)) {
    inf.status = fail(&c->err, OK_E_NONFINITE, "non-finite residual");
    if (info) *info = inf;
    return inf.status;
  }
  const Batch all{1, k.coef, nullptr};
  OK_HIP(&c->err, launch_copy_scale<double, double>(all, Vec<const double>{k.Bv, 0}, vec(k.Bv, 0),
                                                    -1.0, k.n2(), st));
  k.h_part.assign(1, 1);
  Group grp{&k};
  e = newton_solve_group(grp, {one((const double*)u)}, {Vec<const double>{k.Bv, 0}},
                         {vec(k.X, 0)}, st);
  if (e) return e;
  inf.status = k.out[0].status;
  inf.fgmres_its = k.out[0].fgmres_its;
  inf.restarts = k.out[0].restarts;
  inf.lin_res = k.out[0].lin_res;
  if (inf.status != OK_E_NONFINITE) {
    OK_HIP(&c->err, launch_axpby(all, 1.0, one((const double*)u), 1.0, Vec<const double>{k.X, 0},
                                 one(u), k.n, st));
    OK_HIP(&c->err, launch_axpby(all, 1.0, one((const double*)w), 1.0,
                                 Vec<const double>{k.X + k.n, 0}, one(w), k.n, st));
    OK_HIP(&c->err, hipStreamSynchronize(st));
  }
  if (info) *info = inf;
  if (inf.status) fail(&c->err, inf.status, kStatusNames[-inf.status]);
  return inf.status;
}

int ok_timestep(ok_ctx* c, double* u, double* w, int32_t nsteps, ok_stats* stats, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !w || nsteps < 0) return fail(&c->err, OK_E_INVALID, "bad arguments");
  Group grp{&c->cls};
  std::vector<std::vector<ok_stats>> S;
  int e = timestep_group(grp, {one(u)}, {one(w)}, nsteps, S, &c->err, (hipStream_t)stream);
  if (stats) {
    *stats = S[0][0];
    stats->status = e;
  }
  return e;
}

int ok_initial_w(ok_ctx* c, const double* u, double* w, void* stream) {
  if (!c) return OK_E_INVALID;
  if (!u || !w || u == w) return fail(&c->err, OK_E_INVALID, "null or aliased vectors");
  if (!aligned8(u) || !aligned8(w)) return fail(&c->err, OK_E_INVALID, "misaligned");
  return initial_w_d(c->cls, one(u), one(w), nullptr, (hipStream_t)stream);
}

int ok_set_option(int32_t option, int32_t value) {
  switch (option) {
    case OK_OPT_FUSE_CHEB:
      cheb_fusion_set(value);
      return OK_SUCCESS;
    case OK_OPT_FUSE_MG:
      mg_fusion_set(value);
      return OK_SUCCESS;
    case OK_OPT_ISSUE_AHEAD:
      issue_ahead_set(value);
      return OK_SUCCESS;
    case OK_OPT_TRACE_RANGES:
      trace_ranges_set(value);
      return OK_SUCCESS;
    case OK_OPT_GRAM_SCHMIDT:
      ortho_set(value);
      return OK_SUCCESS;
    case OK_OPT_FUSE_PROLONG:
      prolong_fusion_set(value);
      return OK_SUCCESS;
    default:
      return OK_E_INVALID;
  }
}

namespace {
// Table key of an ok_shape_kernel value, or -1.
int shape_key(int32_t kernel) {
  switch (kernel) {
    case OK_SHAPE_STENCIL: return 1;
    case OK_SHAPE_STENCIL2: return 2;
    case OK_SHAPE_CHEB2: return kFusedKey;
    case OK_SHAPE_MG_PRE: return kMgPreKey;
    case OK_SHAPE_MG_POST: return kMgPostKey;
    case OK_SHAPE_CHEB2_TILE: return kFusedTileKey;
    case OK_SHAPE_MG_PRE_TILE: return kMgPreTileKey;
    case OK_SHAPE_MG_POST_TILE: return kMgPostTileKey;
    case OK_SHAPE_CHEB2_STRIP: return kFusedStripKey;
    case OK_SHAPE_MG_PRE_STRIP: return kMgPreStripKey;
    case OK_SHAPE_MG_POST_STRIP: return kMgPostStripKey;
    default: return -1;
  }
}
}  // namespace

int ok_get_launch_shape(int32_t dim, int32_t n, int32_t kernel, int32_t precision, int32_t* items,
                        int32_t* threads, int32_t* zchunks) {
  if ((dim != 2 && dim != 3) || n < 1 || n > (1 << 20)) return OK_E_INVALID;
  if (precision != OK_FP64 && precision != OK_MIXED) return OK_E_INVALID;
  const int nf = shape_key(kernel);
  if (nf < 0 || !items || !threads || !zchunks) return OK_E_INVALID;
  int it = 0, nz = 0, th = 0;
  stencil_tune_get(dim, n + 1, nf, precision == OK_MIXED ? 4 : 8, &it, &nz, &th);
  *items = it;
  *threads = th;
  *zchunks = nz;
  return OK_SUCCESS;
}

int ok_set_launch_shape(int32_t dim, int32_t n, int32_t kernel, int32_t precision, int32_t items,
                        int32_t threads, int32_t zchunks) {
  if ((dim != 2 && dim != 3) || n < 1 || n > (1 << 20)) return OK_E_INVALID;
  if (precision != OK_FP64 && precision != OK_MIXED) return OK_E_INVALID;
  const int nf = shape_key(kernel);
  if (nf < 0) return OK_E_INVALID;
  const int word = precision == OK_MIXED ? 4 : 8;
  if (items == 0) {
    stencil_tune_set(dim, n + 1, nf, word, 0, 0);
    return OK_SUCCESS;
  }
  TileGeom tg;
  const bool strip = (nf == kFusedStripKey || nf == kMgPreStripKey || nf == kMgPostStripKey);
  const bool ok_shape =
      strip ? (dim == 3 && strip_threads(items) > 0 && strip_threads(items) == threads)
      : (nf == kFusedTileKey || nf == kMgPreTileKey || nf == kMgPostTileKey)
          ? cheb2_tile_geom(make_grid(dim, n), threads, items, tg)
      : (nf >= kFusedKey)   ? cheb2_shape_ok(dim, items, threads)
                            : stencil_shape_ok(dim, nf, items, threads);
  if (!ok_shape || zchunks < 1 || zchunks > n + 1) return OK_E_INVALID;
  stencil_tune_set(dim, n + 1, nf, word, items, zchunks, threads);
  return OK_SUCCESS;
}

int ok_use_graphs(ok_ctx* c, int32_t enable) {
  if (!c) return OK_E_INVALID;
  if (!enable && !c->cls.ex) return OK_SUCCESS;
  return enable_exec(c->cls, enable != 0);
}

int ok_autotune(ok_ctx* c, void* stream, int32_t* entries) {
  if (!c) return OK_E_INVALID;
  int n = 0;
  int e = autotune_class(c->cls, (hipStream_t)stream, &n);
  if (entries) *entries = n;
  return e;
}

int ok_profile_enable(ok_ctx* c, int32_t class_mask) {
  if (!c || class_mask < 0) return OK_E_INVALID;
  c->prof.mask = class_mask;
  c->prof.used = 0;
  return OK_SUCCESS;
}

int ok_profile_read(ok_ctx* c, int32_t kernel_class, int64_t* launches, double* total_ms,
                    double* bytes) {
  if (!c) return OK_E_INVALID;
  double ms = 0.0, by = 0.0;
  int64_t cnt = 0;
  for (size_t i = 0; i < c->prof.used; i++) {
    ProfPair& q = c->prof.ev[i];
    if (q.cls != kernel_class) continue;
    cnt += q.count;
    (void)hipEventSynchronize(q.b);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, q.a, q.b);
    ms += t;
    by += q.bytes;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = ms;
  if (bytes) *bytes = by;
  return OK_SUCCESS;
}

const char* ok_error_string(int status) {
  int i = -status;
  if (i < 0 || i > 7) return "unknown status";
  return kStatusNames[i];
}

const char* ok_last_error(const ok_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched instances
// ---------------------------------------------------------------------------
namespace {

// Group instance parameter sets into classes in order of first appearance.
void plan_classes(const ok_params* ps, int count, std::vector<std::vector<int>>& members) {
  members.clear();
  for (int i = 0; i < count; i++) {
    bool placed = false;
    for (auto& m : members)
      if (same_class(ps[m[0]], ps[i])) {
        m.push_back(i);
        placed = true;
        break;
      }
    if (!placed) members.push_back({i});
  }
}

size_t batch_bytes(const ok_params* ps, const std::vector<std::vector<int>>& members) {
  size_t total = 0;
  for (auto& m : members) total += class_bytes(ps[m[0]], (int)m.size(), true);
  return total;
}

}  // namespace

extern "C" {

int ok_batch_workspace_bytes(const ok_params* params, int32_t count, size_t* bytes) {
  if (!params || count < 1 || !bytes) return OK_E_INVALID;
  std::string why;
  for (int i = 0; i < count; i++)
    if (validate_params(&params[i], why)) return OK_E_INVALID;
  std::vector<std::vector<int>> members;
  plan_classes(params, count, members);
  *bytes = batch_bytes(params, members);
  return OK_SUCCESS;
}

int ok_batch_create(const ok_params* params, int32_t count, void* d_ws, size_t ws_bytes,
                    void* stream, ok_batch** out) {
  if (!out || !params || count < 1) return OK_E_INVALID;
  *out = nullptr;
  std::string why;
  for (int i = 0; i < count; i++)
    if (validate_params(&params[i], why)) return OK_E_INVALID;
  std::vector<std::vector<int>> members;
  plan_classes(params, count, members);
  if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < batch_bytes(params, members))
    return OK_E_WORKSPACE;
  ok_batch* b = new (std::nothrow) ok_batch();
  if (!b) return OK_E_INVALID;
  b->count = count;
  b->classes.resize(members.size());
  b->cls_of.assign(count, 0);
  b->idx_of.assign(count, 0);
  char* base = (char*)d_ws;
  for (size_t k = 0; k < members.size(); k++) {
    std::vector<ok_params> ps;
    for (size_t j = 0; j < members[k].size(); j++) {
      ps.push_back(params[members[k][j]]);
      b->cls_of[members[k][j]] = (int)k;
      b->idx_of[members[k][j]] = (int)j;
    }
    ClassCtx& c = b->classes[k];
    c.err = &b->err;
    c.prof = &b->prof;
    int e = class_init(c, ps.data(), (int)ps.size(), base, true, (hipStream_t)stream, b->err);
    if (e) {
      delete b;
      return e;
    }
    base += class_bytes(ps[0], (int)ps.size(), true);
    e = enable_exec(c, true);
    if (e) {
      delete b;
      return e;
    }
  }
  *out = b;
  return OK_SUCCESS;
}

int ok_batch_destroy(ok_batch* b) {
  if (!b) return OK_E_INVALID;
  delete b;
  return OK_SUCCESS;
}

int ok_batch_set_state(ok_batch* b, int32_t i, const double* d_u, const double* d_w,
                       void* stream) {
  if (!b || i < 0 || i >= b->count || !d_u || !d_w) return OK_E_INVALID;
  ClassCtx& c = b->classes[b->cls_of[i]];
  const int j = b->idx_of[i];
  hipStream_t st = (hipStream_t)stream;
  OK_HIP(&b->err, hipMemcpyAsync(c.su + (int64_t)j * c.n, d_u, sizeof(double) * c.n,
                                 hipMemcpyDeviceToDevice, st));
  OK_HIP(&b->err, hipMemcpyAsync(c.sw + (int64_t)j * c.n, d_w, sizeof(double) * c.n,
                                 hipMemcpyDeviceToDevice, st));
  return OK_SUCCESS;
}

int ok_batch_get_state(ok_batch* b, int32_t i, double* d_u, double* d_w, void* stream) {
  if (!b || i < 0 || i >= b->count || !d_u || !d_w) return OK_E_INVALID;
  ClassCtx& c = b->classes[b->cls_of[i]];
  const int j = b->idx_of[i];
  hipStream_t st = (hipStream_t)stream;
  OK_HIP(&b->err, hipMemcpyAsync(d_u, c.su + (int64_t)j * c.n, sizeof(double) * c.n,
                                 hipMemcpyDeviceToDevice, st));
  OK_HIP(&b->err, hipMemcpyAsync(d_w, c.sw + (int64_t)j * c.n, sizeof(double) * c.n,
                                 hipMemcpyDeviceToDevice, st));
  return OK_SUCCESS;
}

int ok_batch_timestep(ok_batch* b, int32_t nsteps, ok_stats* stats, void* stream) {
  if (!b || nsteps < 0) return OK_E_INVALID;
  Group grp;
  std::vector<Vec<double>> u, w;
  for (auto& c : b->classes) {
    grp.push_back(&c);
    u.push_back(vec(c.su, c.n));
    w.push_back(vec(c.sw, c.n));
  }
  std::vector<std::vector<ok_stats>> S;
  int e = timestep_group(grp, u, w, nsteps, S, &b->err, (hipStream_t)stream);
  if (stats)
    for (int i = 0; i < b->count; i++) stats[i] = S[b->cls_of[i]][b->idx_of[i]];
  return e;
}

int ok_batch_autotune(ok_batch* b, void* stream, int32_t* entries) {
  if (!b) return OK_E_INVALID;
  int total = 0;
  for (auto& c : b->classes) {
    int n = 0;
    int e = autotune_class(c, (hipStream_t)stream, &n);
    if (e) return e;
    total += n;
  }
  if (entries) *entries = total;
  return OK_SUCCESS;
}

int ok_batch_use_graphs(ok_batch* b, int32_t enable) {
  if (!b) return OK_E_INVALID;
  for (auto& c : b->classes) {
    int e = enable_exec(c, enable != 0);
    if (e) return e;
  }
  return OK_SUCCESS;
}

int ok_batch_classes(const ok_batch* b) { return b ? (int)b->classes.size() : OK_E_INVALID; }

const char* ok_batch_last_error(const ok_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
