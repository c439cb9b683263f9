// The request server's threading (paper_1305_3162_amd/csrc/slp_server_core.hpp,
// the code libslp's server runs) against a simulated device on the CPU: client
// threads submit, poll and wait while the worker schedules, and a statistics
// thread reads and resets the totals. Built with the thread sanitizer (and
// separately with the address and undefined-behaviour sanitizers) by
// tests/test_scheduler.py. Checks that every request completes with the value
// its launch wrote, that ticket states only move forward, and that the totals
// add up. Prints "ALL OK"; exits non-zero on the first violated invariant.
#include "slp_server_core.hpp"

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <thread>
#include <vector>

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "CHECK failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

// A device whose launches finish after a simulated duration on the real clock
// and whose "result" is the density value plus the geometry id, written at
// launch time (as the real device writes phi before the completion event).
struct ClockDevice {
  using Payload = int64_t;   // device bytes of the geometry
  std::vector<int64_t> bytes;
  std::vector<double> slot_free;
  std::map<uint64_t, double> finish;
  int setups = 0, releases = 0;

  void add(int64_t &&b) { bytes.push_back(b); }
  int setup(int64_t g, int64_t *b) {
    *b = bytes[g];
    ++setups;
    return 0;
  }
  void release(int64_t) { ++releases; }
  int max_batch(int64_t g) { return 1 + (int)(g % 8); }
  int launch(int slot, const std::vector<slp::SchedRequest> &grp) {
    const double now = slp::server_now_s();
    const double start = std::max(now, slot_free[slot]);
    slot_free[slot] = start + 2e-5 * (1.0 + 0.25 * (double)(grp.size() - 1));
    finish[grp[0].ticket] = slot_free[slot];
    for (const auto &r : grp)
      *static_cast<double *>(r.phi) = *static_cast<const double *>(r.dens) + (double)r.geom;
    return 0;
  }
  int query(int, const std::vector<slp::SchedRequest> &grp) {
    return slp::server_now_s() >= finish.at(grp[0].ticket) ? 0 : 1;
  }
  int64_t points(int64_t g) { return 100 + g; }
};

int main() {
  const int G = 12, SLOTS = 3, CLIENTS = 4, PER = 400;
  ClockDevice dev;
  dev.slot_free.assign(SLOTS, 0.0);
  int64_t total_bytes = 0;
  {
    slp::ServerCore<ClockDevice> core(dev, 300, SLOTS, 4, 64, [] { return std::string(); });
    for (int g = 0; g < G; ++g) {
      int64_t b = 20 + 10 * (g % 5);
      total_bytes += b;
      CHECK(core.add_geometry(b, std::move(b)) == g);
    }
    std::atomic<int> done_clients{0};
    std::atomic<int64_t> completed{0};
    std::thread stats([&] {
      // reads (and now and then resets) the totals while requests run
      int k = 0;
      while (done_clients.load() < CLIENTS) {
        slp::ServerTotals t = core.totals(++k % 50 == 0);
        CHECK(t.completed >= 0 && t.failed == 0 && (int64_t)t.latency.size() == t.completed);
        std::this_thread::sleep_for(std::chrono::microseconds(200));
      }
    });
    std::vector<std::thread> clients;
    for (int c = 0; c < CLIENTS; ++c)
      clients.emplace_back([&, c] {
        std::mt19937_64 rng(100 + c);
        std::vector<double> dens(PER), phi(PER, -1.0);
        std::vector<uint64_t> tk(PER);
        std::vector<int64_t> gof(PER);
        for (int i = 0; i < PER; ++i) {
          dens[i] = 1000.0 * c + i;
          gof[i] = (int64_t)(rng() % G);
          tk[i] = core.submit(gof[i], &dens[i], &phi[i]);
          CHECK(tk[i] > 0);
          if (rng() % 7 == 0) {
            const int st = core.state(tk[i]);
            CHECK(st == slp::kPending || st == slp::kRunning || st == slp::kDone);
          }
          if (rng() % 16 == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
        for (int i = 0; i < PER; ++i) {
          CHECK(core.wait(tk[i], 60.0) == slp::kDone);
          CHECK(phi[i] == dens[i] + (double)gof[i]);   // the launch's result is visible
          CHECK(core.state(tk[i]) == slp::kDone);
        }
        completed += PER;
        done_clients += 1;
      });
    for (auto &t : clients) t.join();
    stats.join();
    CHECK(completed.load() == CLIENTS * PER);
    CHECK(core.state(999999999) == slp::kUnknown);
    std::string err;
    CHECK(core.worker_ok(&err) && err.empty());
  }   // shutdown: the worker finishes and releases every resident geometry
  CHECK(dev.setups >= G - 1 && dev.releases == dev.setups);
  (void)total_bytes;
  std::printf("ALL OK setups=%d releases=%d\n", dev.setups, dev.releases);
  return 0;
}
