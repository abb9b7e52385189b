// Multi-threaded stress of the request server's host logic, built with a
// thread or address sanitizer on the CPU (dry-run mode: no device calls).
// Client threads submit, wait, poll and cancel concurrently against one
// server while a fault injector runs; every ticket must end exactly once
// with a valid status and the counters must add up.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "vofserve.h"

// The dry-run server never creates plans or launches work; these definitions
// stand in for the device half of the library and abort if reached.
extern "C" {
poisson_plan* poisson_plan_create(int, int, int, double, double, const double*, const char*, int,
                                  int, int*) {
  std::abort();
}
void poisson_plan_destroy(poisson_plan*) { std::abort(); }
int poisson_solve_batched(poisson_plan*, int, const double* const*, double* const*, void*) {
  std::abort();
}
int extend_liquid_velocity_batched(poisson_plan*, int, const vp_extend_fields*, void*) {
  std::abort();
}
}

static int fail(const char* what) {
  std::fprintf(stderr, "serve_stress: %s\n", what);
  return 1;
}

int main() {
  vp_server_config cfg{};
  cfg.lanes = 3;
  cfg.max_batch = 4;
  cfg.max_pending = 64;
  cfg.dry_run = 1;
  cfg.dry_run_us = 50;
  // room for little more than the largest plan: eviction runs all the time
  cfg.hbm_budget = poisson_plan_footprint(32, 16, 16, VP_PRECISION_MIXED, 4) +
                   poisson_plan_footprint(16, 16, 16, VP_PRECISION_MIXED, 4) / 2;
  int st = 0;
  vp_server* S = vp_server_create(&cfg, &st);
  if (!S) return fail("create");

  const int kThreads = 6, kPerThread = 400;
  std::atomic<long long> ok{0}, ended{0}, refused{0}, bad{0};
  auto client = [&](int id) {
    std::mt19937 rng(1234 + id);
    std::vector<double> dz(64, 1.0 / 64);
    static char fake[64];
    double* p = reinterpret_cast<double*>(fake);
    std::vector<long long> mine;
    for (int i = 0; i < kPerThread; ++i) {
      vp_request r{};
      const int c = rng() % 4;
      r.kind = (rng() & 1) ? VP_REQ_EXTEND : VP_REQ_SOLVE;
      r.precision = (rng() & 1) ? VP_PRECISION_MIXED : VP_PRECISION_FP64;
      r.nx = 16 << (c & 1);
      r.ny = 16;
      r.nz = 8 * (1 + (c >> 1));
      r.dx = r.dy = 0.1;
      r.dz = dz.data();
      r.bc = (c == 3) ? "NNN" : "PPN";
      r.rhs = p;
      r.sol = p;
      r.ext = vp_extend_fields{p, p, p, p, nullptr, nullptr, nullptr, p, p, p,
                               nullptr, nullptr, nullptr, p};
      r.queue_timeout_ms = (rng() % 8 == 0) ? 0.05 : 0.0;
      long long t = 0;
      const int s = vp_server_submit(S, &r, &t);
      if (s == VP_EAGAIN) {  // back off, as a client of a full queue would
        ++refused;
        std::this_thread::sleep_for(std::chrono::microseconds(100));
        continue;
      }
      if (s != VP_OK) {
        ++bad;
        continue;
      }
      mine.push_back(t);
      if (rng() % 5 == 0) vp_server_cancel(S, t);
      if (rng() % 3 == 0 && !mine.empty()) {  // poll the oldest
        vp_result res{};
        if (vp_server_wait(S, mine.front(), 0.0, &res) == VP_OK) {
          ++ended;
          if (res.status == VP_OK) ++ok;
          mine.erase(mine.begin());
        }
      }
    }
    for (long long t : mine) {
      vp_result res{};
      if (vp_server_wait(S, t, 10000.0, &res) != VP_OK) {
        ++bad;
        continue;
      }
      ++ended;
      if (res.status == VP_OK) ++ok;
      if (res.status != VP_OK && res.status != VP_ECANCELED && res.status != VP_ETIMEDOUT &&
          res.status != VP_EHIP && res.status != VP_ENOMEM)
        ++bad;
      vp_result again{};
      if (vp_server_wait(S, t, 0.0, &again) != VP_EINVAL) ++bad;  // released once
    }
  };
  std::atomic<bool> stop{false};
  std::thread injector([&] {
    int k = 0;
    std::vector<double> dz(16, 1.0 / 16);
    while (!stop) {
      vp_server_inject(S, (k++ & 1) ? VP_FAULT_LAUNCH : VP_FAULT_PLAN, 1);
      vp_server_stats s{};
      vp_server_get_stats(S, &s);
      // prewarm requests, some abandoned by a short timeout
      vp_request w{};
      w.nx = w.ny = w.nz = 16;
      w.dx = w.dy = 0.1;
      w.dz = dz.data();
      w.bc = "PPN";
      w.precision = k % 3 == 0 ? VP_PRECISION_MIXED : VP_PRECISION_FP64;
      vp_server_prewarm(S, &w, 1 + k % 2, (k % 4 == 0) ? 0.001 : 50.0, nullptr);
      std::this_thread::sleep_for(std::chrono::milliseconds(2));
    }
  });
  std::vector<std::thread> th;
  for (int i = 0; i < kThreads; ++i) th.emplace_back(client, i);
  for (auto& t : th) t.join();
  stop = true;
  injector.join();
  if (vp_server_drain(S, 10000.0) != VP_OK) return fail("drain");
  vp_server_stats s{};
  vp_server_get_stats(S, &s);
  vp_server_destroy(S);
  const long long accepted = (long long)kThreads * kPerThread - refused - bad;
  std::printf("accepted %lld ended %lld ok %lld refused %lld bad %lld batches %lld evicted %lld\n",
              accepted, ended.load(), ok.load(), refused.load(), bad.load(), s.batches,
              s.plans_evicted);
  if (bad != 0) return fail("bad statuses or lost tickets");
  if (ended != accepted) return fail("ended != accepted");
  if (s.submitted != accepted) return fail("submitted counter");
  if (s.completed + s.failed + s.cancelled + s.timed_out != accepted) return fail("end counters");
  if (s.completed != ok) return fail("completed counter");
  if (s.bytes_peak > cfg.hbm_budget) return fail("budget exceeded");
  return 0;
}
