// Threading of the request server: client threads submit, poll and wait;
// one worker thread owns the scheduler (slp_scheduler.hpp) and the device.
// No HIP here: the device is a template parameter, so the same code runs in
// libslp (slp_server.cpp) and against a simulated device in a CPU test built
// with the thread sanitizer.
//
// Clients and the worker share only a small state under one mutex: the inbox
// of submitted requests, the mirrored state of every ticket and the
// accumulated statistics. The worker takes the inbox, runs a scheduling step
// (retire finished launches, admit, set up or evict geometries, launch) with
// the mutex released, then publishes the tickets whose state changed and the
// latencies of the requests that completed. So a submission never waits for
// a launch, a setup or an eviction, and its arrival time is taken before it
// takes the mutex. Latency runs from that arrival time to the step that
// observes the launch's completion.
#pragma once

#include "slp_scheduler.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

namespace slp {

inline double server_now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct ServerTotals {
  std::vector<double> latency;   // seconds, completed requests since the last reset
  int64_t completed = 0, failed = 0, points = 0, setups = 0, evictions = 0, launches = 0;
  double first_submit = -1.0, last_done = -1.0;
  int64_t queued = 0, in_flight = 0, resident_bytes = 0;   // at the last step
};

// Dev: the scheduler's device interface (slp_scheduler.hpp) plus
//   using Payload = ...;          // what a geometry needs on the device side
//   void add(Payload &&p);        // the next geometry id's payload (worker thread)
template <class Dev>
class ServerCore {
 public:
  using Payload = typename Dev::Payload;

  // init() runs on the worker thread before anything else (e.g. selects the
  // device); a non-empty return is an error message and stops the worker.
  template <class Init>
  ServerCore(Dev &dev, int64_t budget, int n_slots, int max_groups, int max_batch, Init init)
      : dev_(dev), sched_(dev, budget, n_slots, max_groups, max_batch) {
    worker_ = std::thread([this, init] { run(init); });
  }
  ~ServerCore() { shutdown(); }

  // Registers a geometry (its device bytes if known in advance, else -1);
  // the worker hands the payload to the device before its next step.
  int64_t add_geometry(int64_t bytes, Payload &&payload) {
    std::lock_guard<std::mutex> lk(mu_);
    pending_geoms_.emplace_back(bytes, std::move(payload));
    cv_work_.notify_one();
    return next_geom_++;
  }
  int64_t geometries() {
    std::lock_guard<std::mutex> lk(mu_);
    return next_geom_;
  }

  // Queues a request; returns its ticket (> 0), or 0 if the worker has failed.
  uint64_t submit(int64_t geom, const void *dens, void *phi) {
    SchedRequest r;
    r.t_submit = server_now_s();   // arrival, before any waiting on the mutex
    r.geom = geom;
    r.dens = dens;
    r.phi = phi;
    std::lock_guard<std::mutex> lk(mu_);
    if (!worker_ok_) return 0;
    r.ticket = ++last_ticket_;
    inbox_.push_back(r);
    states_[r.ticket] = kPending;
    if (totals_.first_submit < 0) totals_.first_submit = r.t_submit;
    cv_work_.notify_one();
    return r.ticket;
  }

  // kPending, kRunning, kDone, a negative status or kUnknown.
  int state(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = states_.find(ticket);
    return it == states_.end() ? (int)kUnknown : it->second;
  }

  // Waits until the ticket is done or failed (returns its state), or until
  // timeout_s passes (returns kPending / kRunning). timeout_s <= 0: no limit.
  int wait(uint64_t ticket, double timeout_s) {
    std::unique_lock<std::mutex> lk(mu_);
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                              std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 1e9));
    for (;;) {
      auto it = states_.find(ticket);
      if (it == states_.end()) return kUnknown;
      if (it->second == kDone || it->second < 0) return it->second;
      if (!worker_ok_) return kUnknown;
      if (cv_done_.wait_until(lk, deadline) == std::cv_status::timeout) {
        it = states_.find(ticket);
        return it == states_.end() ? (int)kUnknown : it->second;
      }
    }
  }

  // Copy of the totals; reset clears latencies and counters (the measured
  // phase starts afresh).
  ServerTotals totals(bool reset) {
    std::lock_guard<std::mutex> lk(mu_);
    ServerTotals t = totals_;
    if (reset) {
      totals_.latency.clear();
      totals_.completed = totals_.failed = totals_.points = 0;
      totals_.setups = totals_.evictions = totals_.launches = 0;
      totals_.first_submit = totals_.last_done = -1.0;
    }
    return t;
  }

  bool worker_ok(std::string *err) {
    std::lock_guard<std::mutex> lk(mu_);
    if (err) *err = worker_err_;
    return worker_ok_;
  }

  // Finishes everything admitted or queued, stops the worker and releases
  // every resident geometry.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopped_) return;
      stop_ = true;
      cv_work_.notify_all();
    }
    if (worker_.joinable()) worker_.join();
    std::lock_guard<std::mutex> lk(mu_);
    stopped_ = true;
  }

 private:
  template <class Init>
  void run(Init init) {
    const std::string err = init();
    if (!err.empty()) {
      std::lock_guard<std::mutex> lk(mu_);
      worker_ok_ = false;
      worker_err_ = err;
      cv_done_.notify_all();
      return;
    }
    std::vector<SchedRequest> in;
    std::vector<std::pair<int64_t, Payload>> new_geoms;
    for (;;) {
      bool stopping;
      {
        std::lock_guard<std::mutex> lk(mu_);
        in.swap(inbox_);
        new_geoms.swap(pending_geoms_);
        stopping = stop_;
      }
      for (auto &pg : new_geoms) {
        dev_.add(std::move(pg.second));
        sched_.add_geometry(pg.first);
      }
      new_geoms.clear();
      for (const SchedRequest &r : in) sched_.submit(r, r.t_submit);
      in.clear();
      if (stopping && sched_.idle()) break;
      sched_.step(server_now_s());
      publish();
      std::unique_lock<std::mutex> lk(mu_);
      if (sched_.idle())
        cv_work_.wait(lk, [&] { return stop_ || !inbox_.empty() || !pending_geoms_.empty(); });
      else   // poll the launches again shortly; submissions wake us earlier
        cv_work_.wait_for(lk, std::chrono::microseconds(20),
                          [&] { return stop_ || !inbox_.empty(); });
    }
    sched_.release_all();
    publish();
  }

  void publish() {
    auto &st = sched_.stats();
    std::lock_guard<std::mutex> lk(mu_);
    for (uint64_t t : sched_.changed()) states_[t] = sched_.state(t);
    totals_.latency.insert(totals_.latency.end(), st.latency.begin(), st.latency.end());
    totals_.completed += st.completed;
    totals_.failed += st.failed;
    totals_.points += st.points;
    totals_.setups += st.setups;
    totals_.evictions += st.evictions;
    totals_.launches += st.launches;
    if (st.last_done >= 0) totals_.last_done = st.last_done;
    totals_.queued = sched_.queued();
    totals_.in_flight = sched_.in_flight();
    totals_.resident_bytes = sched_.resident_bytes();
    st.latency.clear();
    st.completed = st.failed = st.points = st.setups = st.evictions = st.launches = 0;
    st.last_done = -1.0;
    if (!sched_.changed().empty()) cv_done_.notify_all();
  }

  Dev &dev_;
  Scheduler<Dev> sched_;   // owned by the worker thread
  std::thread worker_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  // under mu_
  std::vector<SchedRequest> inbox_;
  std::vector<std::pair<int64_t, Payload>> pending_geoms_;
  int64_t next_geom_ = 0;
  std::unordered_map<uint64_t, int> states_;
  ServerTotals totals_;
  uint64_t last_ticket_ = 0;
  bool stop_ = false, stopped_ = false;
  bool worker_ok_ = true;
  std::string worker_err_;
};

// p-quantile of sorted values by linear interpolation.
inline double quantile_sorted(const std::vector<double> &v, double q) {
  if (v.empty()) return 0.0;
  const double pos = q * (double)(v.size() - 1);
  const size_t i = (size_t)std::floor(pos);
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace slp
