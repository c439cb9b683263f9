// Scheduling policy of the request server (no HIP here: the device is a
// template parameter, so the same code runs on the GPU in libslp and against
// a simulated device in the CPU tests).
//
// Policy:
//  * Requests are served in arrival order, except that a request whose
//    geometry is busy never blocks later requests for other geometries.
//  * A geometry runs on at most one slot (stream) at a time: its device work
//    buffers are reused by every request. Requests arriving while their
//    geometry is running are chained onto the same slot's stream at once
//    (continuous batching, at most max_chain in flight per slot).
//  * Geometries are built on the device when first needed and stay resident.
//    When admitting one would exceed the memory budget, idle geometries are
//    evicted, least recently used first (those with no queued requests go
//    first). A geometry larger than the whole budget fails its requests with
//    ENOMEM; otherwise the request waits until memory frees up.
//  * A device error of a request fails that request only.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

namespace slp {

struct SchedRequest {
  uint64_t ticket = 0;
  int64_t geom = -1;
  const void *dens = nullptr;
  void *phi = nullptr;
  double t_submit = 0.0;
};

enum SchedState : int { kPending = 1, kRunning = 2, kDone = 0, kUnknown = -1000 };

// Device interface expected from Dev:
//   int  setup(int64_t geom, int64_t *bytes);    // build device tables; 0 or status < 0
//   void release(int64_t geom);                  // free them
//   int  launch(int slot, const SchedRequest &); // enqueue the solve on the slot's stream
//   int  query(int slot, const SchedRequest &);  // 0 done, 1 still running, < 0 error
//   int64_t points(int64_t geom);                // M_q + N of one solve
template <class Dev>
class Scheduler {
 public:
  struct Stats {
    std::vector<double> latency;   // seconds, completed requests
    int64_t completed = 0, failed = 0, setups = 0, evictions = 0;
    int64_t points = 0;
    double first_submit = -1.0, last_done = -1.0;
  };

  Scheduler(Dev &dev, int64_t budget, int n_slots, int max_chain = 64)
      : dev_(dev), budget_(budget), slots_(n_slots), max_chain_(max_chain) {}

  int64_t add_geometry(int64_t known_bytes = -1) {
    const int64_t id = (int64_t)geoms_.size();
    GeomState g;
    g.bytes = known_bytes;
    geoms_.push_back(g);
    return id;
  }

  // Returns the ticket (> 0).
  uint64_t submit(const SchedRequest &r0, double now) {
    SchedRequest r = r0;
    r.ticket = ++last_ticket_;
    r.t_submit = now;
    pending_.push_back(r);
    state_[r.ticket] = kPending;
    geoms_[r.geom].queued += 1;
    if (stats_.first_submit < 0) stats_.first_submit = now;
    return r.ticket;
  }

  // State of a ticket: kPending, kRunning, kDone (result written), a
  // negative status (failed) or kUnknown.
  int state(uint64_t ticket) const {
    auto it = state_.find(ticket);
    return it == state_.end() ? (int)kUnknown : it->second;
  }

  // One scheduling round: retire finished work, then admit.
  void step(double now) {
    retire(now);
    admit(now);
  }

  bool idle() const {
    if (!pending_.empty()) return false;
    for (const Slot &s : slots_)
      if (!s.reqs.empty()) return false;
    return true;
  }

  int64_t resident_bytes() const { return resident_; }
  int64_t in_flight() const {
    int64_t n = 0;
    for (const Slot &s : slots_) n += (int64_t)s.reqs.size();
    return n;
  }
  int64_t queued() const { return (int64_t)pending_.size(); }
  Stats &stats() { return stats_; }
  bool geometry_resident(int64_t g) const { return geoms_[g].resident; }
  int busy_slots() const {
    int n = 0;
    for (const Slot &s : slots_) n += s.reqs.empty() ? 0 : 1;
    return n;
  }

  // Release every resident geometry (shutdown; nothing may be in flight).
  void release_all() {
    for (size_t g = 0; g < geoms_.size(); ++g)
      if (geoms_[g].resident) {
        dev_.release((int64_t)g);
        geoms_[g].resident = false;
      }
    resident_ = 0;
  }

 private:
  struct GeomState {
    bool resident = false;
    int64_t bytes = -1;       // known after the first setup
    int slot = -1;            // slot running it, or -1
    uint64_t last_use = 0;
    int64_t queued = 0;       // pending requests
  };
  struct Slot {
    int64_t geom = -1;
    std::deque<SchedRequest> reqs;   // in stream order
  };

  void retire(double now) {
    for (int si = 0; si < (int)slots_.size(); ++si) {
      Slot &s = slots_[si];
      while (!s.reqs.empty()) {
        const int q = dev_.query(si, s.reqs.front());
        if (q == 1) break;
        const SchedRequest &r = s.reqs.front();
        if (q == 0) {
          state_[r.ticket] = kDone;
          stats_.completed += 1;
          stats_.latency.push_back(now - r.t_submit);
          stats_.points += dev_.points(r.geom);
          stats_.last_done = now;
        } else {
          state_[r.ticket] = q;
          stats_.failed += 1;
        }
        s.reqs.pop_front();
      }
      if (s.reqs.empty() && s.geom >= 0) {
        geoms_[s.geom].slot = -1;
        s.geom = -1;
      }
    }
  }

  int free_slot() const {
    for (int si = 0; si < (int)slots_.size(); ++si)
      if (slots_[si].reqs.empty()) return si;
    return -1;
  }

  // Evict idle geometries (LRU, those without queued requests first) until
  // `need` more bytes fit in the budget. Returns false if impossible.
  bool make_room(int64_t need, int64_t keep) {
    while (resident_ + need > budget_) {
      int64_t victim = -1;
      for (int pass = 0; pass < 2 && victim < 0; ++pass) {
        uint64_t best = UINT64_MAX;
        for (size_t g = 0; g < geoms_.size(); ++g) {
          const GeomState &st = geoms_[g];
          if (!st.resident || st.slot >= 0 || (int64_t)g == keep) continue;
          if (pass == 0 && st.queued > 0) continue;
          if (st.last_use < best) { best = st.last_use; victim = (int64_t)g; }
        }
      }
      if (victim < 0) return false;
      dev_.release(victim);
      geoms_[victim].resident = false;
      resident_ -= geoms_[victim].bytes;
      stats_.evictions += 1;
    }
    return true;
  }

  // Make geometry g resident. 0 ok, 1 retry later, < 0 failure status.
  int ensure_resident(int64_t g) {
    GeomState &st = geoms_[g];
    if (st.resident) return 0;
    if (st.bytes > budget_) return -2;   // ENOMEM: can never fit
    if (st.bytes >= 0 && !make_room(st.bytes, g)) return 1;
    int64_t bytes = 0;
    const int rc = dev_.setup(g, &bytes);
    if (rc < 0) return rc;
    stats_.setups += 1;
    st.bytes = bytes;
    st.resident = true;
    resident_ += bytes;
    if (resident_ > budget_ && !make_room(0, g)) {
      // only now known to be too large for the free memory
      dev_.release(g);
      st.resident = false;
      resident_ -= bytes;
      return bytes > budget_ ? -2 : 1;
    }
    return 0;
  }

  void fail(const SchedRequest &r, int status) {
    state_[r.ticket] = status;
    stats_.failed += 1;
  }

  void admit(double now) {
    (void)now;
    for (auto it = pending_.begin(); it != pending_.end();) {
      SchedRequest &r = *it;
      GeomState &st = geoms_[r.geom];
      int si = st.slot;
      if (si >= 0) {
        // geometry already running: chain onto its stream
        if ((int)slots_[si].reqs.size() >= max_chain_) { ++it; continue; }
      } else {
        si = free_slot();
        if (si < 0) { ++it; continue; }
        const int rc = ensure_resident(r.geom);
        if (rc == 1) { ++it; continue; }             // wait for memory
        if (rc < 0) {
          st.queued -= 1;
          fail(r, rc);
          it = pending_.erase(it);
          continue;
        }
      }
      const int lrc = dev_.launch(si, r);
      st.queued -= 1;
      if (lrc < 0) {
        fail(r, lrc);
        it = pending_.erase(it);
        continue;
      }
      st.slot = si;
      st.last_use = ++clock_;
      slots_[si].geom = r.geom;
      slots_[si].reqs.push_back(r);
      state_[r.ticket] = kRunning;
      it = pending_.erase(it);
    }
  }

  Dev &dev_;
  int64_t budget_;
  std::vector<Slot> slots_;
  int max_chain_;
  std::vector<GeomState> geoms_;
  std::deque<SchedRequest> pending_;
  std::map<uint64_t, int> state_;
  uint64_t last_ticket_ = 0;
  uint64_t clock_ = 0;
  int64_t resident_ = 0;
  Stats stats_;
};

}  // namespace slp
