// Continuous-batching request loop over the plan API (include/vofserve.h).
//
// One scheduler thread owns every plan, stream and event.  Client threads
// only touch the incoming queue, the cancel list, the finished table and the
// counters, all under one mutex.  Each turn of the scheduler:
//   1. takes newly submitted requests into its pending list (arrival order);
//   2. applies cancellations and queue timeouts to pending requests;
//   3. retires batches whose completion event has fired;
//   4. dispatches: for the class of the oldest pending request that can run,
//      picks a lane with room, a plan of that class that is idle or already
//      owned by the lane (creating one within the memory budget, evicting idle
//      plans least recently used first), gathers up to max_batch pending
//      requests of the same class and kind in arrival order and launches them
//      as one batched call on the lane's stream, followed by an event.
// A plan serves one stream at a time: it belongs to the lane that has batches
// in flight on it until they retire, so consecutive batches of a class on one
// lane reuse it without waiting, and other lanes take another instance.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <tuple>
#include <vector>

#include "bc.hpp"
#include "vofpoisson.h"
#include "vofserve.h"

namespace {

constexpr int kLaneDepth = 2;  // batches in flight per lane
constexpr int kMaxLanes = 8;

// Timed condition waits take system-clock deadlines (pthread_cond_timedwait,
// which thread sanitizers model; the steady-clock form is not modelled).
std::chrono::system_clock::time_point deadline_in(double ms) {
  return std::chrono::system_clock::now() +
         std::chrono::duration_cast<std::chrono::system_clock::duration>(
             std::chrono::duration<double, std::milli>(ms));
}

double clock_us() {
  return std::chrono::duration<double, std::micro>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct ClassKey {
  int nx, ny, nz, precision;
  double dx, dy;
  char bc[7];  // the six end letters (x-, x+, y-, y+, z-, z+), NUL-terminated
  std::vector<double> dz;
  bool operator<(const ClassKey& o) const {
    const auto a = std::tie(nx, ny, nz, precision, dx, dy);
    const auto b = std::tie(o.nx, o.ny, o.nz, o.precision, o.dx, o.dy);
    if (a != b) return a < b;
    const int c = std::strcmp(bc, o.bc);
    if (c != 0) return c < 0;
    return dz < o.dz;
  }
  bool operator==(const ClassKey& o) const { return !(*this < o) && !(o < *this); }
};

struct Req {
  long long ticket = 0;
  vp_request r{};  // r.dz / r.bc are not used after submit (see key)
  ClassKey key;
  double t_submit = 0, t_dispatch = 0, t_done = 0, deadline = 0;
  int status = VP_OK, batch = 0, lane = -1;
};

struct PlanEntry {
  ClassKey key;
  poisson_plan* plan = nullptr;  // null in a dry run
  long long bytes = 0;
  int owner = -1;  // lane with batches in flight on this plan
  int inflight = 0;
  double last_used = 0;
};

struct BatchRun {
  std::vector<Req*> reqs;
  PlanEntry* pe = nullptr;
  int lane = 0;
  hipEvent_t ev = nullptr;
  double t_ready = 0;  // dry run: completion time
};

// a request to create plans ahead of traffic (vp_server_prewarm)
struct Warm {
  ClassKey key;
  int instances = 0;
  int created = 0;
  int status = VP_OK;
  bool done = false;
  bool abandoned = false;  // the caller stopped waiting: the scheduler frees it
};

struct Lane {
  hipStream_t stream = nullptr;
  int inflight = 0;
  double busy_until = 0;  // dry run
  std::vector<hipEvent_t> events;
};

}  // namespace

struct vp_server {
  vp_server_config cfg{};
  int device = 0;

  // shared state (mu)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> incoming;
  std::deque<Warm*> warm_incoming;
  std::vector<long long> cancels;
  std::map<long long, Req*> finished;
  std::set<long long> live;  // submitted, result not yet taken
  long long next_ticket = 1;
  long long queued = 0;  // submitted, not yet dispatched or ended
  bool stopping = false;
  vp_server_stats st{};
  int fault_launch = 0, fault_plan = 0;

  // scheduler thread only
  std::list<Req*> pending;
  std::list<PlanEntry*> plans;
  std::vector<Lane> lanes;
  std::list<BatchRun*> running;
  long long bytes_resident = 0;
  std::thread worker;

  void finish(std::vector<Req*>& done);
  void publish();
  bool poll_running(std::vector<Req*>& done);
  PlanEntry* acquire(const ClassKey& key, int lane, bool may_create, int* status);
  void prewarm(Warm* w);
  bool dispatch(std::vector<Req*>& done);
  void launch(BatchRun* b, std::vector<Req*>& done);
  void run();
  void release_all();
};

namespace {

ClassKey key_of(const vp_request& r) {
  ClassKey k;
  k.nx = r.nx;
  k.ny = r.ny;
  k.nz = r.nz;
  k.precision = r.precision;
  k.dx = r.dx;
  k.dy = r.dy;
  // checked by poisson_plan_check at submit: "NNN" and "NNNNNN" are one class
  (void)vp::parse_ends(r.bc, k.bc);
  k.bc[6] = '\0';
  k.dz.assign(r.dz, r.dz + r.nz);
  return k;
}

long long footprint_of(const ClassKey& k, int max_batch) {
  return poisson_plan_footprint(k.nx, k.ny, k.nz, k.precision, max_batch);
}

}  // namespace

// hand ended requests to their waiters (scheduler thread)
void vp_server::finish(std::vector<Req*>& done) {
  if (done.empty()) return;
  const double now = clock_us();
  {
    std::lock_guard<std::mutex> lk(mu);
    for (Req* q : done) {
      if (q->t_done == 0) q->t_done = now;
      switch (q->status) {
        case VP_OK: ++st.completed; break;
        case VP_ECANCELED: ++st.cancelled; break;
        case VP_ETIMEDOUT: ++st.timed_out; break;
        default: ++st.failed; break;
      }
      if (q->t_dispatch == 0) --queued;
      finished[q->ticket] = q;
    }
  }
  done.clear();
  cv_done.notify_all();
}

// publish the scheduler's view to the counters (drain and stats read them)
void vp_server::publish() {
  {
    std::lock_guard<std::mutex> lk(mu);
    st.pending = (long long)pending.size();
    st.running = (long long)running.size();
    st.plans_resident = (long long)plans.size();
    st.bytes_resident = bytes_resident;
  }
  cv_done.notify_all();
}

bool vp_server::poll_running(std::vector<Req*>& done) {
  bool any = false;
  const double now = clock_us();
  for (auto it = running.begin(); it != running.end();) {
    BatchRun* b = *it;
    int status = VP_OK;
    bool ready;
    if (cfg.dry_run) {
      ready = now >= b->t_ready;
    } else {
      const hipError_t e = hipEventQuery(b->ev);
      ready = e != hipErrorNotReady;
      if (ready && e != hipSuccess) status = VP_EHIP;
    }
    if (!ready) {
      ++it;
      continue;
    }
    for (Req* q : b->reqs) {
      q->status = status;
      q->t_done = now;
      done.push_back(q);
    }
    Lane& L = lanes[b->lane];
    if (b->ev) L.events.push_back(b->ev);
    --L.inflight;
    PlanEntry* pe = b->pe;
    pe->last_used = now;
    if (--pe->inflight == 0) pe->owner = -1;
    delete b;
    it = running.erase(it);
    any = true;
  }
  return any;
}

// A plan of class `key` usable on `lane`: one the lane already owns, an idle
// one, or (if may_create) a new one within the budget (evicting idle plans,
// least recently used first).  nullptr with *status VP_OK means "not now"
// (memory held by running batches, or no new instance wanted); another
// status is a hard failure for the class.
PlanEntry* vp_server::acquire(const ClassKey& key, int lane, bool may_create, int* status) {
  *status = VP_OK;
  for (PlanEntry* pe : plans)
    if (pe->owner == lane && pe->key == key) return pe;
  for (PlanEntry* pe : plans)
    if (pe->owner == -1 && pe->key == key) return pe;
  if (!may_create) return nullptr;
  const long long need = footprint_of(key, cfg.max_batch);
  long long busy = 0;  // bytes of plans with batches in flight
  for (PlanEntry* pe : plans)
    if (pe->owner != -1) busy += pe->bytes;
  if (busy + need > cfg.hbm_budget) return nullptr;  // wait for running batches to retire
  auto evict_one = [&]() -> bool {
    PlanEntry* victim = nullptr;
    for (PlanEntry* pe : plans)
      if (pe->owner == -1 && (!victim || pe->last_used < victim->last_used)) victim = pe;
    if (!victim) return false;
    if (victim->plan) poisson_plan_destroy(victim->plan);
    bytes_resident -= victim->bytes;
    plans.remove(victim);
    delete victim;
    std::lock_guard<std::mutex> lk(mu);
    ++st.plans_evicted;
    return true;
  };
  while (bytes_resident + need > cfg.hbm_budget)
    if (!evict_one()) return nullptr;  // wait for running batches to retire
  for (int attempt = 0; attempt < 2; ++attempt) {
    bool injected = false;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (fault_plan > 0) {
        --fault_plan;
        injected = true;
      }
    }
    int s = VP_ENOMEM;
    poisson_plan* plan = nullptr;
    if (!injected) {
      if (cfg.dry_run) {
        s = VP_OK;
      } else {
        plan = poisson_plan_create(key.nx, key.ny, key.nz, key.dx, key.dy, key.dz.data(), key.bc,
                                   key.precision, cfg.max_batch, &s);
      }
    }
    if (s == VP_OK) {
      PlanEntry* pe = new PlanEntry();
      pe->key = key;
      pe->plan = plan;
      pe->bytes = need;
      plans.push_back(pe);
      bytes_resident += need;
      std::lock_guard<std::mutex> lk(mu);
      ++st.plans_created;
      st.bytes_peak = std::max(st.bytes_peak, bytes_resident);
      return pe;
    }
    // device memory may be short for reasons outside the budget: free every
    // idle plan once and try again, then give up on this class
    if (s != VP_ENOMEM || attempt == 1) {
      *status = s;
      return nullptr;
    }
    while (evict_one()) {
    }
  }
  *status = VP_ENOMEM;
  return nullptr;
}

void vp_server::launch(BatchRun* b, std::vector<Req*>& done) {
  Lane& L = lanes[b->lane];
  const double now = clock_us();
  const int n = (int)b->reqs.size();
  for (Req* q : b->reqs) {
    q->t_dispatch = now;
    q->batch = n;
    q->lane = b->lane;
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    queued -= n;
    ++st.batches;
    st.batched_requests += n;
  }
  bool injected = false;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (fault_launch > 0) {
      --fault_launch;
      injected = true;
    }
  }
  int status = injected ? VP_EHIP : VP_OK;
  if (!injected && !cfg.dry_run) {
    const int kind = b->reqs[0]->r.kind;
    if (kind == VP_REQ_SOLVE) {
      const double* rhs[VP_MAX_BATCH];
      double* sol[VP_MAX_BATCH];
      for (int i = 0; i < n; ++i) {
        rhs[i] = b->reqs[i]->r.rhs;
        sol[i] = b->reqs[i]->r.sol;
      }
      status = poisson_solve_batched(b->pe->plan, n, rhs, sol, L.stream);
    } else {
      vp_extend_fields f[VP_MAX_BATCH];
      for (int i = 0; i < n; ++i) f[i] = b->reqs[i]->r.ext;
      status = extend_liquid_velocity_batched(b->pe->plan, n, f, L.stream);
    }
    if (status == VP_OK) {
      hipEvent_t ev = nullptr;
      if (!L.events.empty()) {
        ev = L.events.back();
        L.events.pop_back();
      } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
      }
      if (!ev || hipEventRecord(ev, L.stream) != hipSuccess) {
        // no way to observe completion: wait for the lane here
        (void)hipStreamSynchronize(L.stream);
        if (ev) L.events.push_back(ev);
        ev = nullptr;
        status = VP_EHIP;
      }
      b->ev = ev;
    }
  }
  if (status != VP_OK) {
    // A launch chain that failed part way may have left passes queued on the
    // lane's stream, still writing the plan's workspace: wait for them before
    // the plan can be handed to another lane (an injected failure launched
    // nothing).
    if (!injected && !cfg.dry_run) (void)hipStreamSynchronize(L.stream);
    for (Req* q : b->reqs) {
      q->status = status;
      done.push_back(q);
    }
    b->pe->last_used = now;
    delete b;
    return;
  }
  if (cfg.dry_run) {
    L.busy_until = std::max(L.busy_until, now) + cfg.dry_run_us;
    b->t_ready = L.busy_until;
  }
  ++L.inflight;
  b->pe->owner = b->lane;
  ++b->pe->inflight;
  b->pe->last_used = now;
  running.push_back(b);
}

bool vp_server::dispatch(std::vector<Req*>& done) {
  bool progress = false;
  for (;;) {
    bool launched = false;
    std::set<std::pair<ClassKey, int>> tried;
    for (Req* head : pending) {
      const std::pair<ClassKey, int> grp(head->key, head->r.kind);
      if (tried.count(grp)) continue;
      tried.insert(grp);
      // lanes with room: those already owning a plan of this class first,
      // then the least loaded
      std::vector<int> order;
      for (int l = 0; l < (int)lanes.size(); ++l)
        if (lanes[l].inflight < kLaneDepth) order.push_back(l);
      if (order.empty()) return progress;
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        auto owns = [&](int l) {
          for (PlanEntry* pe : plans)
            if (pe->owner == l && pe->key == head->key) return 1;
          return 0;
        };
        const int oa = owns(a), ob = owns(b);
        if (oa != ob) return oa > ob;
        return lanes[a].inflight < lanes[b].inflight;
      });
      // Another instance of a class whose plans are all busy on full lanes
      // costs a device allocation on this thread (stalling every lane), so
      // one is made only for a backlog of half a batch or more; otherwise the
      // group waits for its plan's lane.  Beyond its own plans, acquire does
      // not depend on the lane: one try.
      bool exists = false;
      for (PlanEntry* pe : plans) exists = exists || pe->key == head->key;
      int backlog = 0;
      for (Req* q : pending) backlog += q->key == head->key && q->r.kind == head->r.kind;
      const bool may_create = !exists || 2 * backlog >= cfg.max_batch;
      const int lane = order[0];
      int status = VP_OK;
      PlanEntry* pe = acquire(head->key, lane, may_create, &status);
      if (!pe && status != VP_OK) {
        // the class cannot get a plan: end its pending requests
        for (auto it = pending.begin(); it != pending.end();) {
          if ((*it)->key == head->key) {
            (*it)->status = status;
            done.push_back(*it);
            it = pending.erase(it);
          } else {
            ++it;
          }
        }
        launched = true;
        break;
      }
      if (!pe) continue;
      BatchRun* b = new BatchRun();
      b->pe = pe;
      b->lane = lane;
      for (auto it = pending.begin(); it != pending.end() && (int)b->reqs.size() < cfg.max_batch;) {
        if ((*it)->key == head->key && (*it)->r.kind == head->r.kind) {
          b->reqs.push_back(*it);
          it = pending.erase(it);
        } else {
          ++it;
        }
      }
      launch(b, done);
      launched = true;
      break;  // pending changed: rescan from the oldest request
    }
    if (!launched) return progress;
    progress = true;
  }
}

// create idle plans of one class until `instances` exist (scheduler thread)
void vp_server::prewarm(Warm* w) {
  // hold the class's idle plans (and each new one) aside while creating, so
  // acquire neither returns nor evicts them
  std::vector<PlanEntry*> held;
  int have = 0;
  for (PlanEntry* pe : plans) {
    if (!(pe->key == w->key)) continue;
    ++have;
    if (pe->owner == -1) {
      pe->owner = -2;
      held.push_back(pe);
    }
  }
  while (have < w->instances) {
    int status = VP_OK;
    PlanEntry* pe = acquire(w->key, -3, true, &status);
    if (!pe) {
      w->status = status != VP_OK ? status : VP_ENOMEM;
      break;
    }
    pe->owner = -2;
    held.push_back(pe);
    ++have;
    ++w->created;
  }
  for (PlanEntry* pe : held) pe->owner = -1;
}

void vp_server::run() {
  if (!cfg.dry_run) (void)hipSetDevice(device);
  std::vector<Req*> done;
  for (;;) {
    std::vector<long long> cx;
    std::vector<Warm*> warms;
    bool stop;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (running.empty() && incoming.empty() && cancels.empty() && warm_incoming.empty() &&
          !stopping) {
        // idle, or waiting only for queue timeouts / plan memory
        if (pending.empty()) cv_work.wait(lk);
        else cv_work.wait_until(lk, deadline_in(0.2));
      }
      while (!incoming.empty()) {
        pending.push_back(incoming.front());
        incoming.pop_front();
      }
      cx.swap(cancels);
      while (!warm_incoming.empty()) {
        warms.push_back(warm_incoming.front());
        warm_incoming.pop_front();
      }
      stop = stopping;
      st.pending = (long long)pending.size();
    }
    const double now = clock_us();
    for (auto it = pending.begin(); it != pending.end();) {
      Req* q = *it;
      const bool cancelled = std::find(cx.begin(), cx.end(), q->ticket) != cx.end();
      const bool expired = q->deadline > 0 && now > q->deadline;
      if (cancelled || expired) {
        q->status = cancelled ? VP_ECANCELED : VP_ETIMEDOUT;
        done.push_back(q);
        it = pending.erase(it);
      } else {
        ++it;
      }
    }
    if (!warms.empty()) {
      for (Warm* w : warms) prewarm(w);
      {
        std::lock_guard<std::mutex> lk(mu);
        for (Warm* w : warms) {
          if (w->abandoned) delete w;
          else w->done = true;
        }
      }
      publish();
    }
    const bool retired = poll_running(done);
    const bool launched = dispatch(done);
    finish(done);
    if (retired || launched || !cx.empty()) publish();
    if (stop && pending.empty() && running.empty()) {
      std::lock_guard<std::mutex> lk(mu);
      if (incoming.empty() && warm_incoming.empty()) break;
    }
    if (!running.empty() && !retired && !launched) std::this_thread::yield();
  }
}

void vp_server::release_all() {
  for (PlanEntry* pe : plans) {
    if (pe->plan) poisson_plan_destroy(pe->plan);
    delete pe;
  }
  plans.clear();
  for (Lane& L : lanes) {
    for (hipEvent_t e : L.events) (void)hipEventDestroy(e);
    L.events.clear();
    if (L.stream) (void)hipStreamDestroy(L.stream);
    L.stream = nullptr;
  }
  for (auto& kv : finished) delete kv.second;
  finished.clear();
  for (Req* q : incoming) delete q;
  incoming.clear();
  for (Warm* w : warm_incoming) delete w;
  warm_incoming.clear();
  for (Req* q : pending) delete q;
  pending.clear();
}

extern "C" {

double vp_server_now_us(void) { return clock_us(); }

vp_server* vp_server_create(const vp_server_config* cfg, int* status) {
  auto fail = [&](int s) -> vp_server* {
    if (status) *status = s;
    return nullptr;
  };
  if (!cfg || cfg->hbm_budget <= 0 || cfg->lanes < 1 || cfg->lanes > kMaxLanes ||
      cfg->max_batch < 1 || cfg->max_batch > VP_MAX_BATCH || cfg->max_pending < 1 ||
      (cfg->dry_run && !(cfg->dry_run_us >= 0)))
    return fail(VP_EINVAL);
  vp_server* S = new (std::nothrow) vp_server();
  if (!S) return fail(VP_ENOMEM);
  S->cfg = *cfg;
  S->lanes.resize(cfg->lanes);
  if (!cfg->dry_run) {
    if (hipGetDevice(&S->device) != hipSuccess) {
      delete S;
      return fail(VP_EHIP);
    }
    for (Lane& L : S->lanes) {
      if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess) {
        S->release_all();
        delete S;
        return fail(VP_EHIP);
      }
    }
  }
  S->worker = std::thread([S] { S->run(); });
  if (status) *status = VP_OK;
  return S;
}

int vp_server_submit(vp_server* S, const vp_request* r, long long* ticket) {
  if (!S || !r || !ticket) return VP_EINVAL;
  auto reject = [&](int s) {
    std::lock_guard<std::mutex> lk(S->mu);
    ++S->st.rejected;
    return s;
  };
  if (r->kind != VP_REQ_SOLVE && r->kind != VP_REQ_EXTEND) return reject(VP_EINVAL);
  const int chk = poisson_plan_check(r->nx, r->ny, r->nz, r->dx, r->dy, r->dz, r->bc,
                                     r->precision, S->cfg.max_batch);
  if (chk != VP_OK) return reject(chk);
  if (r->kind == VP_REQ_SOLVE) {
    if (!r->rhs || !r->sol) return reject(VP_EINVAL);
  } else {
    const vp_extend_fields& e = r->ext;
    if (!e.u || !e.v || !e.w || !e.src || !e.ue || !e.ve || !e.we) return reject(VP_EINVAL);
    const bool hq = e.qx && e.qy && e.qz, hg = e.ug && e.vg && e.wg;
    if (((e.qx || e.qy || e.qz) && !hq) || ((e.ug || e.vg || e.wg) && !hg) || hq != hg)
      return reject(VP_EINVAL);
    if (r->precision == VP_PRECISION_MIXED && !e.phi) return reject(VP_EINVAL);
  }
  Req* q = new (std::nothrow) Req();
  if (!q) return reject(VP_ENOMEM);
  q->r = *r;
  q->r.dz = nullptr;
  q->r.bc = nullptr;
  const ClassKey& k = q->key = key_of(*r);
  if (footprint_of(k, S->cfg.max_batch) > S->cfg.hbm_budget) {
    delete q;
    return reject(VP_ETOOBIG);
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping || S->queued >= S->cfg.max_pending) {
      delete q;
      ++S->st.rejected;
      return VP_EAGAIN;
    }
    q->ticket = S->next_ticket++;
    q->t_submit = clock_us();
    if (r->queue_timeout_ms > 0) q->deadline = q->t_submit + 1e3 * r->queue_timeout_ms;
    S->incoming.push_back(q);
    S->live.insert(q->ticket);
    ++S->queued;
    ++S->st.submitted;
    *ticket = q->ticket;
  }
  S->cv_work.notify_one();
  return VP_OK;
}

int vp_server_prewarm(vp_server* S, const vp_request* r, int instances, double timeout_ms,
                      int* created) {
  if (!S || !r || instances < 1 || instances > S->cfg.lanes) return VP_EINVAL;
  const int chk = poisson_plan_check(r->nx, r->ny, r->nz, r->dx, r->dy, r->dz, r->bc,
                                     r->precision, S->cfg.max_batch);
  if (chk != VP_OK) return chk;
  Warm* w = new (std::nothrow) Warm();
  if (!w) return VP_ENOMEM;
  w->key = key_of(*r);
  w->instances = instances;
  if ((long long)instances * footprint_of(w->key, S->cfg.max_batch) > S->cfg.hbm_budget) {
    delete w;
    return VP_ETOOBIG;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->stopping) {
    delete w;
    return VP_EAGAIN;
  }
  S->warm_incoming.push_back(w);
  S->cv_work.notify_one();
  auto ready = [&] { return w->done; };
  bool ok = true;
  if (timeout_ms < 0) S->cv_done.wait(lk, ready);
  else ok = S->cv_done.wait_until(lk, deadline_in(timeout_ms), ready);
  if (!ok) {
    w->abandoned = true;  // the scheduler frees it when it gets to it
    return VP_EAGAIN;
  }
  const int st = w->status;
  if (created) *created = w->created;
  delete w;
  return st;
}

int vp_server_wait(vp_server* S, long long ticket, double timeout_ms, vp_result* res) {
  if (!S || !res) return VP_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  if (!S->live.count(ticket)) return VP_EINVAL;
  auto ready = [&] { return S->finished.count(ticket) > 0; };
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, ready);
  } else if (!ready()) {
    S->cv_done.wait_until(lk, deadline_in(timeout_ms), ready);
  }
  auto it = S->finished.find(ticket);
  if (it == S->finished.end()) return VP_EAGAIN;
  Req* q = it->second;
  res->status = q->status;
  res->batch = q->batch;
  res->lane = q->lane;
  res->t_submit_us = q->t_submit;
  res->t_dispatch_us = q->t_dispatch;
  res->t_done_us = q->t_done;
  S->finished.erase(it);
  S->live.erase(ticket);
  delete q;
  return VP_OK;
}

int vp_server_cancel(vp_server* S, long long ticket) {
  if (!S) return VP_EINVAL;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->live.count(ticket)) return VP_EINVAL;
    S->cancels.push_back(ticket);
  }
  S->cv_work.notify_one();
  return VP_OK;
}

int vp_server_drain(vp_server* S, double timeout_ms) {
  if (!S) return VP_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto idle = [&] {
    return S->queued == 0 && S->incoming.empty() && S->st.running == 0 && S->st.pending == 0;
  };
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, idle);
    return VP_OK;
  }
  return S->cv_done.wait_until(lk, deadline_in(timeout_ms), idle) ? VP_OK : VP_EAGAIN;
}

int vp_server_get_stats(vp_server* S, vp_server_stats* out) {
  if (!S || !out) return VP_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  return VP_OK;
}

int vp_server_inject(vp_server* S, int fault, int count) {
  if (!S || count < 0) return VP_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  if (fault == VP_FAULT_LAUNCH) S->fault_launch = count;
  else if (fault == VP_FAULT_PLAN) S->fault_plan = count;
  else return VP_EINVAL;
  return VP_OK;
}

void vp_server_destroy(vp_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv_work.notify_one();
  if (S->worker.joinable()) S->worker.join();
  if (!S->cfg.dry_run) {
    for (Lane& L : S->lanes)
      if (L.stream) (void)hipStreamSynchronize(L.stream);
  }
  S->release_all();
  delete S;
}

}  // extern "C"
