// Serving loop of libok.so: timestep requests of many resident simulations,
// admitted by HBM footprint into slot pools (one pool = one class of
// instances sharing grid, precision and solver counts) and advanced together
// one Newton iteration per tick (continuous batching: a request admitted
// between ticks joins the next tick's grouped launches).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "engine.h"

using namespace okd;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over byte offsets [0, size) of the pool region.
struct Arena {
  std::map<size_t, size_t> free_;  // offset -> length, coalesced
  size_t size = 0, used = 0, peak = 0;
  void init(size_t n) {
    free_.clear();
    size = n;
    used = peak = 0;
    if (n) free_[0] = n;
  }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      size_t rest = it->second - n, at = it->first + n;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used += n;
      peak = std::max(peak, used);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~(size_t)255;
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Request {
  int sim = 0, nsteps = 0;
  double t_arr = 0, t_admit = -1, t_done = -1;
  int status = 1, steps_done = 0, newton_its = 0, fgmres_its = 0;
  bool deferred = false;
};

struct Pool {
  ClassCtx c;
  size_t off = 0, bytes = 0;
  std::vector<int64_t> slot;   // request in each slot, -1 = free
  std::vector<char> starting;  // slot begins a new timestep at its next tick
  std::thread th;              // the pool's worker: ticks on the class stream
  std::condition_variable cv;  // new slots or quit
  bool quit = false;
  std::string err;
  int live() const {
    int k = 0;
    for (int64_t r : slot) k += (r >= 0);
    return k;
  }
};

struct Sim {
  ok_params p{};
  double *u = nullptr, *w = nullptr;
  int64_t nodes = 0;
  bool busy = false;  // a request of this simulation is in a slot
};

}  // namespace

// Threads: the dispatcher (admission, pool creation and release) and one
// worker per pool (its ticks).  Every field is guarded by `mu`; the device
// work of a tick runs without it, from a snapshot of the pool's slots.
struct ok_server {
  ok_server_config cfg{};
  std::vector<Sim> sims;
  char* pool_base = nullptr;
  Arena arena;
  std::vector<std::unique_ptr<Pool>> pools;
  std::vector<std::unique_ptr<Pool>> retiring;  // idle pools being shut down
  hipStream_t st = nullptr;     // the dispatcher's stream (default priority)
  std::deque<Request> reqs;     // by ticket
  std::deque<int64_t> future;   // submitted, not yet arrived (sorted by arrival)
  std::deque<int64_t> queue;    // arrived, waiting for a slot (arrival order)
  std::deque<int64_t> done;     // completed, not yet polled
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool running = false, stop = false, drain = false;
  Clock::time_point t0 = Clock::now();
  ok_server_stats stats{};
  std::string err;
  int fatal = OK_SUCCESS;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

int fail(std::string* err, int code, const std::string& msg) {
  if (err) *err = msg;
  return code;
}

#define SV_HIP(errp, ...)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (__VA_ARGS__);                                                           \
    if (e_ != hipSuccess)                                                                    \
      return fail(errp, OK_E_HIP, std::string(#__VA_ARGS__).substr(0, 60) + ": " +           \
                                      hipGetErrorString(e_));                                \
  } while (0)

size_t sim_bytes(const ok_params& p) {
  int64_t nodes = 1;
  for (int d = 0; d < p.dim; d++) nodes *= (p.n + 1);
  return ((size_t)nodes * 2 * sizeof(double) + 255) & ~(size_t)255;
}

int pool_capacity(const ok_server* s, const ok_params& p) {
  int cap = std::max(1, s->cfg.max_slots_per_pool);
  while (cap > 1 && (double)class_bytes(p, cap, true) > s->cfg.pool_bytes) cap--;
  return cap;
}

void complete(ok_server* s, int64_t r, int status) {
  Request& q = s->reqs[r];
  q.status = status;
  q.t_done = s->now();
  s->sims[q.sim].busy = false;
  s->done.push_back(r);
  s->stats.completed++;
  if (status == OK_SUCCESS) {
    s->stats.dof_steps += 2.0 * (double)s->sims[q.sim].nodes * q.steps_done;
  } else {
    s->stats.failed++;
  }
}

// What a tick needs to know of a live slot (copied under the lock).
struct SlotView {
  int slot;
  int sim;
  bool starting;
};
struct SlotOut {
  int slot;
  int status;  // 1: iterating; else the step's outcome
  int newton_its = 0, fgmres_its = 0;
  bool copied_out = false;  // the request's last step ended; state written back
};

// One Newton iteration (Sec. 2: residual test, FGMRES solve, update, residual
// test) of the pool's live slots, on the class stream; no lock held.
int pool_tick(ok_server* s, Pool& q, const std::vector<SlotView>& v,
              const std::vector<int>& last_step, std::vector<SlotOut>& out) {
  ClassCtx& c = q.c;
  hipStream_t st = c.ex->xs;
  std::fill(c.h_aux.begin(), c.h_aux.end(), 0);
  std::fill(c.h_part.begin(), c.h_part.end(), 0);
  bool any_start = false;
  for (const SlotView& x : v) {
    c.h_part[x.slot] = 1;
    if (x.starting) {
      c.h_aux[x.slot] = 1;
      c.h_hasF[x.slot] = 0;
      c.nits[x.slot] = 0;
      any_start = true;
    }
  }
  if (any_start) {  // previous time level <- current state
    SV_HIP(&q.err, hipMemcpyAsync(c.aux, c.h_aux.data(), sizeof(int) * c.B,
                                  hipMemcpyHostToDevice, st));
    const Batch fb = c.batch(c.aux);
    SV_HIP(&q.err, launch_copy_scale<double, double>(fb, cvec(c.su, c.n), vec(c.un, c.n), 1.0,
                                                     c.n, st));
    SV_HIP(&q.err, launch_copy_scale<double, double>(fb, cvec(c.sw, c.n), vec(c.wn, c.n), 1.0,
                                                     c.n, st));
    SV_HIP(&q.err, hipStreamSynchronize(st));  // h_aux is reused by the Newton tick
  }
  std::vector<NewtonLog> log(1);
  log[0].its.assign(c.B, {});
  log[0].fnorm.assign(c.B, {});
  int e = newton_group_iters(Group{&c}, {vec(c.su, c.n)}, {vec(c.sw, c.n)}, {cvec(c.un, c.n)},
                             {cvec(c.wn, c.n)}, log, 1, st);
  if (e) return e;
  bool copied = false;
  out.clear();
  for (size_t k = 0; k < v.size(); k++) {
    const int i = v[k].slot;
    SlotOut o;
    o.slot = i;
    o.status = c.out[i].status;
    for (int f : log[0].its[i]) {
      o.newton_its++;
      o.fgmres_its += f;
    }
    // the request ends with this step (or with an error): write the state back
    if (o.status != 1 && (o.status != OK_SUCCESS || last_step[k])) {
      const Sim& sm = s->sims[v[k].sim];  // sims is fixed after creation
      SV_HIP(&q.err, hipMemcpyAsync(sm.u, c.su + (int64_t)i * c.n, sizeof(double) * c.n,
                                    hipMemcpyDeviceToDevice, st));
      SV_HIP(&q.err, hipMemcpyAsync(sm.w, c.sw + (int64_t)i * c.n, sizeof(double) * c.n,
                                    hipMemcpyDeviceToDevice, st));
      o.copied_out = copied = true;
    }
    out.push_back(o);
  }
  if (copied) SV_HIP(&q.err, hipStreamSynchronize(st));
  return OK_SUCCESS;
}

void pool_main(ok_server* s, Pool* q, int dev) {
  (void)hipSetDevice(dev);
  std::unique_lock<std::mutex> lk(s->mu);
  std::vector<SlotView> v;
  std::vector<int> last;
  std::vector<SlotOut> out;
  for (;;) {
    while (!q->quit && !s->fatal && q->live() == 0) q->cv.wait(lk);
    if (q->quit || s->fatal) break;
    v.clear();
    last.clear();
    for (int i = 0; i < q->c.B; i++) {
      const int64_t r = q->slot[i];
      if (r < 0) continue;
      const Request& rq = s->reqs[r];
      v.push_back(SlotView{i, rq.sim, q->starting[i] != 0});
      last.push_back(rq.steps_done + 1 >= rq.nsteps);
      q->starting[i] = 0;
    }
    lk.unlock();
    const double ta = s->now();
    int e;
    {
      TraceRange tick_range("serve tick");
      e = pool_tick(s, *q, v, last, out);
    }
    const double tb = s->now();
    lk.lock();
    s->stats.ticks++;
    s->stats.busy_s += tb - ta;
    bool freed = false;
    for (const SlotOut& o : out) {
      const int64_t r = q->slot[o.slot];
      Request& rq = s->reqs[r];
      rq.newton_its += o.newton_its;
      rq.fgmres_its += o.fgmres_its;
      if (o.status == 1) continue;
      if (o.status == OK_SUCCESS) rq.steps_done++;
      if (!o.copied_out) {  // next timestep of the same request
        q->starting[o.slot] = 1;
        continue;
      }
      q->slot[o.slot] = -1;
      complete(s, r, o.status);
      freed = true;
    }
    if (e) {
      s->err = q->err;
      s->fatal = e;
    }
    if (freed || e) {
      s->cv_done.notify_all();
      s->cv_work.notify_all();
    }
    if (e) break;
  }
}

// Retire pools with no live slot: their workers stop; the dispatcher joins
// them and returns their memory to the arena (join_retired).
void retire_idle_pools(ok_server* s) {
  for (size_t k = 0; k < s->pools.size();) {
    if (s->pools[k]->live() == 0) {
      std::unique_ptr<Pool> q = std::move(s->pools[k]);
      s->pools.erase(s->pools.begin() + (long)k);
      q->quit = true;
      q->cv.notify_all();
      s->retiring.push_back(std::move(q));
    } else {
      k++;
    }
  }
}

void join_retired(ok_server* s, std::unique_lock<std::mutex>& lk) {
  if (s->retiring.empty()) return;
  std::vector<std::unique_ptr<Pool>> r;
  r.swap(s->retiring);
  lk.unlock();
  for (auto& q : r)
    if (q->th.joinable()) q->th.join();
  lk.lock();
  for (auto& q : r) {
    s->arena.release(q->off, q->bytes);
    s->stats.pools_freed++;
  }
  lk.unlock();
  r.clear();  // streams and graphs of the pools
  lk.lock();
}

// A free slot of a pool of this class, else a new pool if the arena has room.
int find_slot(ok_server* s, const ok_params& p, int dev, Pool** pool, int* slot) {
  *pool = nullptr;
  for (auto& up : s->pools) {
    Pool& q = *up;
    if (!same_class(q.c.shape, p)) continue;
    for (int i = 0; i < q.c.B; i++)
      if (q.slot[i] < 0) {
        *pool = &q;
        *slot = i;
        return OK_SUCCESS;
      }
  }
  const int cap = pool_capacity(s, p);
  const size_t bytes = class_bytes(p, cap, true);
  size_t off = 0;
  if (!s->arena.alloc(bytes, &off)) return OK_SUCCESS;  // no room now
  std::unique_ptr<Pool> q(new (std::nothrow) Pool());
  if (!q) {
    s->arena.release(off, bytes);
    return fail(&s->err, OK_E_INVALID, "out of host memory");
  }
  q->off = off;
  q->bytes = bytes;
  q->c.err = &q->err;
  std::vector<ok_params> ps(cap, p);
  int e = class_init(q->c, ps.data(), cap, s->pool_base + off, true, s->st, q->err);
  if (!e) e = enable_exec(q->c, s->cfg.graphs != 0);
  if (e) {
    s->err = q->err;
    s->arena.release(off, bytes);
    return e;
  }
  q->slot.assign(cap, -1);
  q->starting.assign(cap, 0);
  Pool* raw = q.get();
  try {
    q->th = std::thread(pool_main, s, raw, dev);
  } catch (...) {
    s->arena.release(off, bytes);
    return fail(&s->err, OK_E_INVALID, "cannot start a pool worker");
  }
  s->stats.pools_created++;
  s->pools.push_back(std::move(q));
  *pool = raw;
  *slot = 0;
  return OK_SUCCESS;
}

// Move arrived requests into the queue (rejecting beyond max_queue), then
// admit queued requests in arrival order.  Called with the lock held.
int admit(ok_server* s, int dev) {
  const double t = s->now();
  while (!s->future.empty() && s->reqs[s->future.front()].t_arr <= t) {
    const int64_t r = s->future.front();
    s->future.pop_front();
    if ((int)s->queue.size() >= s->cfg.max_queue) {
      s->reqs[r].status = OK_E_REJECTED;
      s->reqs[r].t_done = t;
      s->done.push_back(r);
      s->stats.rejected++;
    } else {
      s->queue.push_back(r);
    }
  }
  s->stats.max_queue_seen = std::max<int64_t>(s->stats.max_queue_seen, (int64_t)s->queue.size());
  std::vector<char> held(s->sims.size(), 0);  // a simulation's earlier request waits
  std::vector<Pool*> woken;
  bool short_of_memory = false;
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    const int64_t r = *it;
    Request& q = s->reqs[r];
    Sim& sm = s->sims[q.sim];
    if (sm.busy || held[q.sim]) {  // FIFO per simulation: one request in flight
      held[q.sim] = 1;
      ++it;
      continue;
    }
    Pool* pool = nullptr;
    int slot = -1;
    int e = find_slot(s, sm.p, dev, &pool, &slot);
    if (e) return e;
    if (!pool) {
      if (!q.deferred) s->stats.deferred++;
      q.deferred = true;
      held[q.sim] = 1;
      short_of_memory = true;
      ++it;
      continue;
    }
    ClassCtx& c = pool->c;
    e = set_instance(c, slot, sm.p, s->st);
    if (e) {
      s->err = pool->err;
      return e;
    }
    SV_HIP(&s->err, hipMemcpyAsync(c.su + (int64_t)slot * c.n, sm.u, sizeof(double) * c.n,
                                   hipMemcpyDeviceToDevice, s->st));
    SV_HIP(&s->err, hipMemcpyAsync(c.sw + (int64_t)slot * c.n, sm.w, sizeof(double) * c.n,
                                   hipMemcpyDeviceToDevice, s->st));
    pool->slot[slot] = r;  // the worker sees it once the lock is released
    pool->starting[slot] = 1;
    sm.busy = true;
    q.t_admit = t;
    s->stats.admitted++;
    woken.push_back(pool);
    it = s->queue.erase(it);
  }
  if (!woken.empty()) {
    // the pool workers read the slots on their own streams: complete the
    // copies before the lock is released
    SV_HIP(&s->err, hipStreamSynchronize(s->st));
    for (Pool* pool : woken) pool->cv.notify_all();
  }
  int live = 0;
  for (auto& up : s->pools) live += up->live();
  s->stats.max_active = std::max<int64_t>(s->stats.max_active, live);
  if (short_of_memory) retire_idle_pools(s);
  s->stats.peak_bytes = std::max<int64_t>(s->stats.peak_bytes, (int64_t)s->arena.peak);
  return OK_SUCCESS;
}

void fail_all(ok_server* s) {
  for (auto& up : s->pools)
    for (int64_t& r : up->slot)
      if (r >= 0) {
        complete(s, r, s->fatal);
        r = -1;
      }
  for (int64_t r : s->queue) complete(s, r, s->fatal);
  s->queue.clear();
}

void dispatcher_main(ok_server* s, int dev) {
  (void)hipSetDevice(dev);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    join_retired(s, lk);
    if (!s->fatal) {
      int e = admit(s, dev);
      if (e) s->fatal = e;
    }
    if (s->fatal) break;
    bool live = false;
    for (auto& up : s->pools) live = live || up->live() > 0;
    if (s->stop) {
      const bool idle = !live && s->queue.empty() && s->future.empty();
      if (!s->drain || idle) break;
    }
    if (!s->retiring.empty()) continue;  // their memory may admit a waiting request
    if (s->future.empty()) {
      s->cv_work.wait(lk);
    } else {
      const double dt = s->reqs[s->future.front()].t_arr - s->now();
      if (dt > 0) s->cv_work.wait_for(lk, std::chrono::duration<double>(std::min(dt, 1.0)));
    }
  }
  // stop the pool workers (each ends after its current tick)
  for (auto& up : s->pools) {
    up->quit = true;
    up->cv.notify_all();
  }
  std::vector<Pool*> ps;
  for (auto& up : s->pools) ps.push_back(up.get());
  lk.unlock();
  for (Pool* q : ps)
    if (q->th.joinable()) q->th.join();
  lk.lock();
  join_retired(s, lk);
  if (s->fatal) fail_all(s);
  s->running = false;
  s->cv_done.notify_all();
}

}  // namespace

extern "C" {

int ok_server_default_config(ok_server_config* c) {
  if (!c) return OK_E_INVALID;
  std::memset(c, 0, sizeof(*c));
  c->max_queue = 256;
  c->max_slots_per_pool = 16;
  c->graphs = 1;
  c->pool_bytes = 32.0 * (1ull << 30);
  return OK_SUCCESS;
}

int ok_server_state_bytes(const ok_params* sims, int32_t nsims, size_t* bytes) {
  if (!sims || nsims < 1 || !bytes) return OK_E_INVALID;
  std::string why;
  size_t t = 0;
  for (int i = 0; i < nsims; i++) {
    if (validate_params(&sims[i], why)) return OK_E_INVALID;
    t += sim_bytes(sims[i]);
  }
  *bytes = t;
  return OK_SUCCESS;
}

int ok_server_create(const ok_params* sims, int32_t nsims, const ok_server_config* cfg,
                     void* d_ws, size_t ws_bytes, void* stream, ok_server** out) {
  if (!out) return OK_E_INVALID;
  *out = nullptr;
  size_t state = 0;
  int v = ok_server_state_bytes(sims, nsims, &state);
  if (v) return v;
  ok_server_config c{};
  if (cfg) c = *cfg;
  else ok_server_default_config(&c);
  if (c.max_queue < 0 || c.max_slots_per_pool < 1 || !(c.pool_bytes > 0)) return OK_E_INVALID;
  if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < state) return OK_E_WORKSPACE;
  // the smallest pool of every simulation's class must fit next to the state
  size_t need = 0;
  for (int i = 0; i < nsims; i++) need = std::max(need, class_bytes(sims[i], 1, true));
  if (ws_bytes - state < need) return OK_E_WORKSPACE;
  ok_server* s = new (std::nothrow) ok_server();
  if (!s) return OK_E_INVALID;
  s->cfg = c;
  char* base = (char*)d_ws;
  s->sims.resize(nsims);
  for (int i = 0; i < nsims; i++) {
    Sim& sm = s->sims[i];
    sm.p = sims[i];
    sm.nodes = 1;
    for (int d = 0; d < sm.p.dim; d++) sm.nodes *= (sm.p.n + 1);
    sm.u = (double*)base;
    sm.w = sm.u + sm.nodes;
    base += sim_bytes(sm.p);
  }
  s->pool_base = (char*)d_ws + state;
  s->arena.init(ws_bytes - state);
  if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return OK_E_HIP;
  }
  (void)stream;
  *out = s;
  return OK_SUCCESS;
}

int ok_server_set_state(ok_server* s, int32_t sim, const double* d_u, const double* d_w,
                        void* stream) {
  if (!s || sim < 0 || sim >= (int)s->sims.size() || !d_u || !d_w) return OK_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->running) return fail(&s->err, OK_E_INVALID, "state access while the server runs");
  const Sim& sm = s->sims[sim];
  hipStream_t st = (hipStream_t)stream;
  SV_HIP(&s->err, hipMemcpyAsync(sm.u, d_u, sizeof(double) * sm.nodes, hipMemcpyDeviceToDevice, st));
  SV_HIP(&s->err, hipMemcpyAsync(sm.w, d_w, sizeof(double) * sm.nodes, hipMemcpyDeviceToDevice, st));
  SV_HIP(&s->err, hipStreamSynchronize(st));
  return OK_SUCCESS;
}

int ok_server_get_state(ok_server* s, int32_t sim, double* d_u, double* d_w, void* stream) {
  if (!s || sim < 0 || sim >= (int)s->sims.size() || !d_u || !d_w) return OK_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->running) return fail(&s->err, OK_E_INVALID, "state access while the server runs");
  const Sim& sm = s->sims[sim];
  hipStream_t st = (hipStream_t)stream;
  SV_HIP(&s->err, hipMemcpyAsync(d_u, sm.u, sizeof(double) * sm.nodes, hipMemcpyDeviceToDevice, st));
  SV_HIP(&s->err, hipMemcpyAsync(d_w, sm.w, sizeof(double) * sm.nodes, hipMemcpyDeviceToDevice, st));
  SV_HIP(&s->err, hipStreamSynchronize(st));
  return OK_SUCCESS;
}

int ok_server_start(ok_server* s) {
  if (!s) return OK_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->running) return fail(&s->err, OK_E_INVALID, "already running");
  if (s->fatal) return fail(&s->err, s->fatal, "server failed earlier: " + s->err);
  int dev = 0;
  SV_HIP(&s->err, hipGetDevice(&dev));
  s->stop = s->drain = false;
  try {
    for (auto& up : s->pools)  // pools kept from an earlier run get new workers
      if (!up->th.joinable()) {
        up->quit = false;
        up->th = std::thread(pool_main, s, up.get(), dev);
      }
    s->worker = std::thread(dispatcher_main, s, dev);
  } catch (...) {
    s->stop = true;
    for (auto& up : s->pools) {
      up->quit = true;
      up->cv.notify_all();
    }
    return fail(&s->err, OK_E_INVALID, "cannot start the server threads");
  }
  s->running = true;
  return OK_SUCCESS;
}

double ok_server_now(const ok_server* s) { return s ? s->now() : 0.0; }

int ok_server_submit(ok_server* s, int32_t sim, int32_t nsteps, double t_arrival,
                     int64_t* ticket) {
  if (!s || sim < 0 || sim >= (int)s->sims.size() || nsteps < 1) return OK_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->fatal) return s->fatal;
  Request r;
  r.sim = sim;
  r.nsteps = nsteps;
  r.t_arr = t_arrival < 0 ? s->now() : t_arrival;
  s->reqs.push_back(r);
  const int64_t id = (int64_t)s->reqs.size() - 1;
  // keep arrival order (ties: submission order)
  auto pos = std::upper_bound(s->future.begin(), s->future.end(), r.t_arr,
                              [s](double t, int64_t b) { return t < s->reqs[b].t_arr; });
  s->future.insert(pos, id);
  s->stats.submitted++;
  if (ticket) *ticket = id;
  s->cv_work.notify_all();
  return OK_SUCCESS;
}

int ok_server_poll(ok_server* s, ok_request_result* out, int32_t max, int32_t* count,
                   double wait_s) {
  if (!s || !count || max < 0 || (max > 0 && !out)) return OK_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_s > 0 && s->running)
    s->cv_done.wait_for(lk, std::chrono::duration<double>(wait_s),
                        [s] { return !s->done.empty() || !s->running; });
  int k = 0;
  while (k < max && !s->done.empty()) {
    const int64_t id = s->done.front();
    s->done.pop_front();
    const Request& r = s->reqs[id];
    ok_request_result& o = out[k++];
    o.ticket = id;
    o.sim = r.sim;
    o.nsteps = r.nsteps;
    o.status = r.status;
    o.steps_done = r.steps_done;
    o.newton_its = r.newton_its;
    o.fgmres_its = r.fgmres_its;
    o.t_arrival = r.t_arr;
    o.t_admit = r.t_admit;
    o.t_done = r.t_done;
  }
  *count = k;
  return OK_SUCCESS;
}

int ok_server_stop(ok_server* s, int32_t drain) {
  if (!s) return OK_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->drain = drain != 0;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  std::lock_guard<std::mutex> lk(s->mu);
  if (!drain) {  // requests never started stay unserved: report them rejected
    for (int64_t r : s->future) {
      s->reqs[r].status = OK_E_REJECTED;
      s->done.push_back(r);
      s->stats.rejected++;
    }
    s->future.clear();
    for (int64_t r : s->queue) {
      s->reqs[r].status = OK_E_REJECTED;
      s->done.push_back(r);
      s->stats.rejected++;
    }
    s->queue.clear();
    // requests in slots are finished in place: they hold their last iterate
    for (auto& up : s->pools)
      for (int i = 0; i < up->c.B; i++) {
        const int64_t r = up->slot[i];
        if (r < 0) continue;
        Request& q = s->reqs[r];
        Sim& sm = s->sims[q.sim];
        ClassCtx& c = up->c;
        SV_HIP(&s->err, hipMemcpyAsync(sm.u, c.su + (int64_t)i * c.n, sizeof(double) * c.n,
                                 hipMemcpyDeviceToDevice, s->st));
        SV_HIP(&s->err, hipMemcpyAsync(sm.w, c.sw + (int64_t)i * c.n, sizeof(double) * c.n,
                                 hipMemcpyDeviceToDevice, s->st));
        up->slot[i] = -1;
        complete(s, r, OK_E_REJECTED);
      }
    SV_HIP(&s->err, hipStreamSynchronize(s->st));
  }
  return s->fatal;
}

int ok_server_get_stats(ok_server* s, ok_server_stats* out) {
  if (!s || !out) return OK_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->pools_live = (int64_t)s->pools.size();
  out->bytes_in_use = (int64_t)s->arena.used;
  out->now = s->now();
  return OK_SUCCESS;
}

int ok_server_reset_stats(ok_server* s) {
  if (!s) return OK_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(&s->stats, 0, sizeof(s->stats));
  s->arena.peak = s->arena.used;
  return OK_SUCCESS;
}

int ok_server_destroy(ok_server* s) {
  if (!s) return OK_E_INVALID;
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
      s->drain = false;
      s->cv_work.notify_all();
    }
    s->worker.join();
  }
  for (auto& up : s->pools) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      up->quit = true;
      up->cv.notify_all();
    }
    if (up->th.joinable()) up->th.join();
  }
  s->pools.clear();
  if (s->st) (void)hipStreamSynchronize(s->st);
  if (s->st) (void)hipStreamDestroy(s->st);
  delete s;
  return OK_SUCCESS;
}

const char* ok_server_last_error(const ok_server* s) { return s ? s->err.c_str() : "null server"; }

}  // extern "C"
