// Scheduling policy of the request server (no HIP here: the device is a
// template parameter, so the same code runs on the GPU in libslp and against
// a simulated device in the CPU tests).
//
// Policy:
//  * Requests are served in arrival order, except that a request whose
//    geometry is busy never blocks later requests for other geometries.
//  * A geometry runs on at most one slot (stream) at a time: its device work
//    buffers are reused by every request. Pending requests for one geometry
//    are coalesced: one launch takes up to max_batch of them (in arrival
//    order) as one batched evaluation, on a free slot or chained behind the
//    geometry's work already on its slot (continuous batching, at most
//    max_groups launches in flight per slot).
//  * Fairness: once an older request is waiting for a slot or for memory, no
//    further work is chained onto busy slots, so the next slot to drain goes
//    to the oldest waiter; a waiting geometry is thus served after at most
//    max_groups launches of any slot, whatever the load on the others.
//  * Geometries are built on the device when first needed and stay resident.
//    When admitting one would exceed the memory budget, idle geometries are
//    evicted, least recently used first (those with no queued requests go
//    first). A geometry larger than the whole budget fails its requests with
//    ENOMEM; otherwise the request waits until memory frees up.
//  * A device error of a launch fails the requests of that launch only.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <list>
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
//   int  max_batch(int64_t geom);                // largest launch the geometry takes (>= 1)
//   int  launch(int slot, const std::vector<SchedRequest> &group);
//                                                // enqueue one (batched) solve of the
//                                                // group on the slot's stream
//   int  query(int slot, const std::vector<SchedRequest> &group);
//                                                // 0 done, 1 still running, < 0 error
//   int64_t points(int64_t geom);                // M_q + N of one solve
template <class Dev>
class Scheduler {
 public:
  struct Stats {
    std::vector<double> latency;   // seconds, completed requests
    int64_t completed = 0, failed = 0, setups = 0, evictions = 0, launches = 0;
    int64_t points = 0;
    double first_submit = -1.0, last_done = -1.0;
  };

  Scheduler(Dev &dev, int64_t budget, int n_slots, int max_groups = 4, int max_batch = 64)
      : dev_(dev), budget_(budget), slots_(n_slots), max_groups_(max_groups),
        max_batch_(max_batch) {}

  int64_t add_geometry(int64_t known_bytes = -1) {
    const int64_t id = (int64_t)geoms_.size();
    GeomState g;
    g.bytes = known_bytes;
    geoms_.push_back(g);
    return id;
  }

  // Queues a request. Uses r0.ticket if non-zero (the caller numbers them in
  // submission order), else assigns the next number. Returns the ticket (> 0).
  uint64_t submit(const SchedRequest &r0, double now) {
    SchedRequest r = r0;
    if (r.ticket == 0) r.ticket = ++last_ticket_;
    else last_ticket_ = std::max(last_ticket_, r.ticket);
    if (r.t_submit <= 0.0) r.t_submit = now;
    pending_.push_back(r);
    state_[r.ticket] = kPending;
    geoms_[r.geom].queued += 1;
    if (stats_.first_submit < 0 || r.t_submit < stats_.first_submit)
      stats_.first_submit = r.t_submit;
    return r.ticket;
  }

  // State of a ticket: kPending, kRunning, kDone (result written), a
  // negative status (failed) or kUnknown.
  int state(uint64_t ticket) const {
    auto it = state_.find(ticket);
    return it == state_.end() ? (int)kUnknown : it->second;
  }

  // Tickets whose state changed in the last step (for callers that mirror the
  // states elsewhere); cleared by every step.
  const std::vector<uint64_t> &changed() const { return changed_; }

  // One scheduling round: retire finished work, then admit.
  void step(double now) {
    changed_.clear();
    retire(now);
    admit(now);
  }

  bool idle() const {
    if (!pending_.empty()) return false;
    for (const Slot &s : slots_)
      if (!s.groups.empty()) return false;
    return true;
  }

  int64_t resident_bytes() const { return resident_; }
  int64_t in_flight() const {
    int64_t n = 0;
    for (const Slot &s : slots_)
      for (const Group &g : s.groups) n += (int64_t)g.size();
    return n;
  }
  int64_t queued() const { return (int64_t)pending_.size(); }
  Stats &stats() { return stats_; }
  bool geometry_resident(int64_t g) const { return geoms_[g].resident; }
  int busy_slots() const {
    int n = 0;
    for (const Slot &s : slots_) n += s.groups.empty() ? 0 : 1;
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
  using Group = std::vector<SchedRequest>;
  struct GeomState {
    bool resident = false;
    int64_t bytes = -1;       // known after the first setup
    int slot = -1;            // slot running it, or -1
    uint64_t last_use = 0;
    int64_t queued = 0;       // pending requests
  };
  struct Slot {
    int64_t geom = -1;
    std::deque<Group> groups;   // launches in stream order
  };

  void set_state(uint64_t t, int st) {
    state_[t] = st;
    changed_.push_back(t);
  }

  void retire(double now) {
    for (int si = 0; si < (int)slots_.size(); ++si) {
      Slot &s = slots_[si];
      while (!s.groups.empty()) {
        const Group &g = s.groups.front();
        const int q = dev_.query(si, g);
        if (q == 1) break;
        for (const SchedRequest &r : g) {
          if (q == 0) {
            set_state(r.ticket, kDone);
            stats_.completed += 1;
            stats_.latency.push_back(now - r.t_submit);
            stats_.points += dev_.points(r.geom);
            stats_.last_done = now;
          } else {
            set_state(r.ticket, q);
            stats_.failed += 1;
          }
        }
        s.groups.pop_front();
      }
      if (s.groups.empty() && s.geom >= 0) {
        geoms_[s.geom].slot = -1;
        s.geom = -1;
      }
    }
  }

  int free_slot() const {
    for (int si = 0; si < (int)slots_.size(); ++si)
      if (slots_[si].groups.empty()) return si;
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

  // Take up to the geometry's batch limit of pending requests for geometry g,
  // starting at `first`, in arrival order.
  Group take_group(typename std::list<SchedRequest>::iterator first, int64_t g) {
    Group grp;
    const int cap = std::max(1, std::min(max_batch_, dev_.max_batch(g)));
    for (auto it = first; it != pending_.end() && (int)grp.size() < cap;) {
      if (it->geom == g) {
        grp.push_back(*it);
        it = pending_.erase(it);
      } else {
        ++it;
      }
    }
    geoms_[g].queued -= (int64_t)grp.size();
    return grp;
  }

  void admit(double now) {
    (void)now;
    bool waiter = false;   // an older request waits for a slot or for memory
    for (auto it = pending_.begin(); it != pending_.end();) {
      const int64_t g = it->geom;
      GeomState &st = geoms_[g];
      int si = st.slot;
      if (si >= 0) {
        // geometry already running: chain behind its work unless an older
        // request waits, or the slot holds enough launches already
        if (waiter || (int)slots_[si].groups.size() >= max_groups_) { ++it; continue; }
      } else {
        si = free_slot();
        if (si < 0) { waiter = true; ++it; continue; }
        const int rc = ensure_resident(g);
        if (rc == 1) { waiter = true; ++it; continue; }   // wait for memory
        if (rc < 0) {
          st.queued -= 1;
          set_state(it->ticket, rc);
          stats_.failed += 1;
          it = pending_.erase(it);
          continue;
        }
      }
      // `it` is the oldest pending request of g: the group starts with it;
      // afterwards the scan resumes at the first request that arrived after
      // it (pending requests are in ticket order), leftovers of g included
      const uint64_t first_ticket = it->ticket;
      Group grp = take_group(it, g);
      const int lrc = dev_.launch(si, grp);
      if (lrc < 0) {
        for (const SchedRequest &r : grp) set_state(r.ticket, lrc);
        stats_.failed += (int64_t)grp.size();
      } else {
        stats_.launches += 1;
        st.slot = si;
        st.last_use = ++clock_;
        slots_[si].geom = g;
        for (const SchedRequest &r : grp) set_state(r.ticket, kRunning);
        slots_[si].groups.push_back(std::move(grp));
      }
      it = pending_.begin();
      while (it != pending_.end() && it->ticket <= first_ticket) ++it;
    }
  }

  Dev &dev_;
  int64_t budget_;
  std::vector<Slot> slots_;
  int max_groups_, max_batch_;
  std::vector<GeomState> geoms_;
  std::list<SchedRequest> pending_;
  std::map<uint64_t, int> state_;
  std::vector<uint64_t> changed_;
  uint64_t last_ticket_ = 0;
  uint64_t clock_ = 0;
  int64_t resident_ = 0;
  Stats stats_;
};

}  // namespace slp
