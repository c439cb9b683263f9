// CPU simulation of the request scheduler (paper_1305_3162_amd/csrc/slp_scheduler.hpp)
// against a fake device with a simulated clock: checks admission by memory,
// back-pressure, eviction, continuous batching, fairness, error isolation and
// that no slot or ticket leaks. Prints "OK <scenario>" lines; exits non-zero on
// the first violated invariant.
#include "slp_scheduler.hpp"

#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "CHECK failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

struct FakeDevice {
  double now = 0.0;
  std::vector<int64_t> size;          // device bytes per geometry
  std::vector<double> dur;            // solve duration per geometry
  std::vector<bool> resident;
  std::map<uint64_t, double> finish;  // ticket -> completion time
  std::map<uint64_t, int> slot_of;
  std::vector<double> slot_free;      // time the slot's stream drains
  std::set<uint64_t> fail_tickets;    // injected device errors
  int setups = 0, releases = 0;
  int64_t live_bytes = 0, peak_bytes = 0;
  std::vector<std::vector<uint64_t>> order;   // completion order per geometry

  int setup(int64_t g, int64_t *bytes) {
    CHECK(!resident[g]);
    resident[g] = true;
    *bytes = size[g];
    live_bytes += size[g];
    if (live_bytes > peak_bytes) peak_bytes = live_bytes;
    ++setups;
    return 0;
  }
  void release(int64_t g) {
    CHECK(resident[g]);
    resident[g] = false;
    live_bytes -= size[g];
    ++releases;
  }
  int launch(int slot, const slp::SchedRequest &r) {
    CHECK(resident[r.geom]);
    const double start = std::max(now, slot_free[slot]);
    slot_free[slot] = start + dur[r.geom];
    finish[r.ticket] = slot_free[slot];
    slot_of[r.ticket] = slot;
    return 0;
  }
  int query(int slot, const slp::SchedRequest &r) {
    CHECK(slot_of.at(r.ticket) == slot);
    if (now < finish.at(r.ticket)) return 1;
    order[r.geom].push_back(r.ticket);
    return fail_tickets.count(r.ticket) ? -3 : 0;
  }
  int64_t points(int64_t g) { return 1000 + g; }
};

static FakeDevice make_dev(const std::vector<int64_t> &size, const std::vector<double> &dur, int slots) {
  FakeDevice d;
  d.size = size;
  d.dur = dur;
  d.resident.assign(size.size(), false);
  d.slot_free.assign(slots, 0.0);
  d.order.resize(size.size());
  return d;
}

static void run_until_idle(slp::Scheduler<FakeDevice> &s, FakeDevice &d, double dt, int64_t budget) {
  for (int it = 0; it < 1000000 && !s.idle(); ++it) {
    s.step(d.now);
    CHECK(s.resident_bytes() <= budget);
    d.now += dt;
  }
  s.step(d.now);
  CHECK(s.idle());
}

static void scenario_chain_and_skip() {
  // two geometries, one slot each time; g0 busy must not block g1
  FakeDevice d = make_dev({40, 40}, {1.0, 1.0}, 2);
  slp::Scheduler<FakeDevice> s(d, 100, 2);
  const int64_t g0 = s.add_geometry(), g1 = s.add_geometry();
  slp::SchedRequest r;
  r.geom = g0;
  const uint64_t a = s.submit(r, d.now), b = s.submit(r, d.now);   // g0 twice
  r.geom = g1;
  const uint64_t c = s.submit(r, d.now);                             // g1 behind them
  s.step(d.now);
  // both g0 requests chained on one slot, g1 on the other: all running at once
  CHECK(s.state(a) == slp::kRunning && s.state(b) == slp::kRunning && s.state(c) == slp::kRunning);
  CHECK(s.busy_slots() == 2 && d.setups == 2);
  run_until_idle(s, d, 0.25, 100);
  CHECK(s.state(a) == slp::kDone && s.state(b) == slp::kDone && s.state(c) == slp::kDone);
  CHECK(d.order[g0].size() == 2 && d.order[g0][0] == a && d.order[g0][1] == b);
  CHECK(s.busy_slots() == 0 && s.in_flight() == 0 && s.queued() == 0);
  std::printf("OK chain_and_skip\n");
}

static void scenario_memory_backpressure_and_eviction() {
  // budget fits two of three equal geometries
  FakeDevice d = make_dev({60, 60, 60}, {1.0, 1.0, 1.0}, 3);
  slp::Scheduler<FakeDevice> s(d, 130, 3);
  for (int i = 0; i < 3; ++i) s.add_geometry(60);   // sizes known before setup
  slp::SchedRequest r;
  std::vector<uint64_t> t;
  for (int g = 0; g < 3; ++g) {
    r.geom = g;
    t.push_back(s.submit(r, d.now));
  }
  s.step(d.now);
  CHECK(s.state(t[0]) == slp::kRunning && s.state(t[1]) == slp::kRunning);
  CHECK(s.state(t[2]) == slp::kPending);        // back-pressure: no memory yet
  CHECK(s.resident_bytes() <= 130);
  run_until_idle(s, d, 0.1, 130);
  for (uint64_t x : t) CHECK(s.state(x) == slp::kDone);
  CHECK(s.stats().evictions >= 1 && d.peak_bytes <= 130);
  // the evicted geometry is rebuilt when asked again
  r.geom = 0;
  const uint64_t again = s.submit(r, d.now);
  run_until_idle(s, d, 0.1, 130);
  CHECK(s.state(again) == slp::kDone);
  std::printf("OK memory_backpressure_and_eviction\n");
}

static void scenario_oversized_and_errors() {
  FakeDevice d = make_dev({500, 20}, {1.0, 0.5}, 2);
  slp::Scheduler<FakeDevice> s(d, 100, 2);
  const int64_t big = s.add_geometry(500), small = s.add_geometry();
  slp::SchedRequest r;
  r.geom = big;
  const uint64_t a = s.submit(r, d.now);
  r.geom = small;
  const uint64_t b = s.submit(r, d.now), c = s.submit(r, d.now), e = s.submit(r, d.now);
  d.fail_tickets.insert(c);
  run_until_idle(s, d, 0.1, 100);
  CHECK(s.state(a) == -2);                      // can never fit
  CHECK(s.state(b) == slp::kDone && s.state(e) == slp::kDone);
  CHECK(s.state(c) == -3);                      // injected device error, isolated
  CHECK(s.stats().failed == 2 && s.stats().completed == 2);
  CHECK(s.state(999999) == slp::kUnknown);
  std::printf("OK oversized_and_errors\n");
}

static void scenario_random_stress() {
  std::mt19937_64 rng(12345);
  const int G = 12, SLOTS = 4;
  std::vector<int64_t> size(G);
  std::vector<double> dur(G);
  for (int g = 0; g < G; ++g) {
    size[g] = 10 + (int64_t)(rng() % 90);
    dur[g] = 0.2 + (rng() % 100) / 50.0;
  }
  const int64_t budget = 250;
  FakeDevice d = make_dev(size, dur, SLOTS);
  slp::Scheduler<FakeDevice> s(d, budget, SLOTS, 8);
  for (int g = 0; g < G; ++g) s.add_geometry(size[g]);
  std::vector<uint64_t> tickets;
  std::map<uint64_t, int64_t> geom_of;
  std::exponential_distribution<double> gap(4.0);
  double next = 0.0;
  int submitted = 0;
  for (int it = 0; it < 2000000 && (submitted < 3000 || !s.idle()); ++it) {
    while (submitted < 3000 && next <= d.now) {
      slp::SchedRequest r;
      r.geom = (int64_t)(rng() % G);
      const uint64_t t = s.submit(r, d.now);
      tickets.push_back(t);
      geom_of[t] = r.geom;
      ++submitted;
      next += gap(rng);
    }
    s.step(d.now);
    CHECK(s.resident_bytes() <= budget);
    CHECK(d.peak_bytes <= budget);
    CHECK(s.busy_slots() <= SLOTS);
    d.now += 0.05;
  }
  CHECK(s.idle());
  for (uint64_t t : tickets) CHECK(s.state(t) == slp::kDone);
  // per geometry: completions in submission order
  for (int g = 0; g < G; ++g)
    for (size_t i = 1; i < d.order[g].size(); ++i) CHECK(d.order[g][i - 1] < d.order[g][i]);
  CHECK(s.stats().completed == 3000);
  CHECK(d.live_bytes == s.resident_bytes());
  s.release_all();
  CHECK(d.live_bytes == 0);
  std::printf("OK random_stress setups=%lld evictions=%lld\n", (long long)s.stats().setups,
              (long long)s.stats().evictions);
}

int main() {
  scenario_chain_and_skip();
  scenario_memory_backpressure_and_eviction();
  scenario_oversized_and_errors();
  scenario_random_stress();
  std::printf("ALL OK\n");
  return 0;
}
