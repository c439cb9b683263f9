// Request server: a worker thread that keeps geometries resident on the
// device, admits solves by memory, runs them on a pool of streams and
// chains requests for a running geometry onto its stream (the policy is in
// slp_scheduler.hpp). Latency is measured from submit to the moment the
// worker observes the solve's completion event.
#include "slp.h"
#include "slp_internal.hpp"
#include "slp_scheduler.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct HostGeometry {
  std::vector<double> nodes;
  std::vector<int32_t> tris;
  std::vector<double> es_w, es_gamma;
  slp_params params{};
  double near_eps = 0.0;         // near-field correction within this distance (0: none)
  slp_geom *geom = nullptr;
  int64_t points = 0;
};

struct HipDevice {
  std::vector<HostGeometry> *geoms = nullptr;
  std::vector<hipStream_t> streams;
  hipStream_t setup_stream = nullptr;
  std::map<uint64_t, hipEvent_t> events;   // ticket -> completion event
  std::vector<hipEvent_t> free_events;

  int setup(int64_t g, int64_t *bytes) {
    HostGeometry &h = (*geoms)[g];
    slp_params p = h.params;
    p.es_w = h.es_w.data();
    p.es_gamma = h.es_gamma.data();
    int rc = slp_setup_geometry(&h.geom, h.nodes.data(), (int64_t)h.nodes.size() / 3, h.tris.data(),
                                (int64_t)h.tris.size() / 3, &p, setup_stream);
    if (rc) return rc;
    if (h.near_eps > 0.0) {
      rc = slp_setup_near_field(h.geom, h.near_eps, setup_stream);
      if (rc) {
        slp_geom_destroy(h.geom);
        h.geom = nullptr;
        return rc;
      }
    }
    slp_geom_info info;
    slp_geom_get_info(h.geom, &info);
    *bytes = info.device_bytes;
    h.points = info.n_src + info.n_nodes;
    return 0;
  }
  void release(int64_t g) {
    HostGeometry &h = (*geoms)[g];
    if (h.geom) slp_geom_destroy(h.geom);
    h.geom = nullptr;
  }
  int launch(int slot, const slp::SchedRequest &r) {
    HostGeometry &h = (*geoms)[r.geom];
    hipStream_t st = streams[slot];
    int rc = slp_set_density(h.geom, static_cast<const double *>(r.dens), st);
    if (!rc) rc = slp_eval_single_layer(h.geom, static_cast<double *>(r.phi), st);
    if (rc) return rc;
    hipEvent_t ev;
    if (!free_events.empty()) {
      ev = free_events.back();
      free_events.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      return SLP_EDEVICE;
    }
    if (hipEventRecord(ev, st) != hipSuccess) {
      free_events.push_back(ev);
      return SLP_EDEVICE;
    }
    events[r.ticket] = ev;
    return 0;
  }
  int query(int slot, const slp::SchedRequest &r) {
    (void)slot;
    auto it = events.find(r.ticket);
    if (it == events.end()) return SLP_EDEVICE;
    const hipError_t e = hipEventQuery(it->second);
    if (e == hipErrorNotReady) return 1;
    free_events.push_back(it->second);
    events.erase(it);
    return e == hipSuccess ? 0 : SLP_EDEVICE;
  }
  int64_t points(int64_t g) { return (*geoms)[g].points; }
};

int srv_fail(int code, const char *msg) {
  slp::set_error_message(msg);
  return code;
}

}  // namespace

struct slp_server {
  std::vector<HostGeometry> geoms;
  HipDevice dev;
  slp::Scheduler<HipDevice> *sched = nullptr;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  bool worker_ok = true;
  std::string worker_err;

  void run() {
    if (hipSetDevice(device) != hipSuccess) {
      std::lock_guard<std::mutex> lk(mu);
      worker_ok = false;
      worker_err = "worker: hipSetDevice failed";
      cv_done.notify_all();
      return;
    }
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
      const int64_t before = sched->stats().completed + sched->stats().failed;
      sched->step(now_s());
      if (sched->stats().completed + sched->stats().failed != before) cv_done.notify_all();
      if (sched->idle()) {
        cv_work.wait(lk, [&] { return stop || !sched->idle(); });
      } else {
        // poll the completion events again shortly; submissions wake us earlier
        cv_work.wait_for(lk, std::chrono::microseconds(20));
      }
    }
  }
};

extern "C" {

int slp_server_create(slp_server **out, size_t device_budget_bytes, int32_t n_slots) {
  if (!out || n_slots < 1 || n_slots > 64 || device_budget_bytes == 0)
    return srv_fail(SLP_EINVAL, "server: need out != NULL, 1 <= n_slots <= 64, budget > 0");
  *out = nullptr;
  slp_server *s = new (std::nothrow) slp_server();
  if (!s) return srv_fail(SLP_ENOMEM, "server: host allocation failed");
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return srv_fail(SLP_EDEVICE, "server: hipGetDevice failed");
  }
  s->dev.geoms = &s->geoms;
  for (int i = 0; i < n_slots; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->dev.streams) (void)hipStreamDestroy(x);
      delete s;
      return srv_fail(SLP_EDEVICE, "server: hipStreamCreate failed");
    }
    s->dev.streams.push_back(st);
  }
  if (hipStreamCreateWithFlags(&s->dev.setup_stream, hipStreamNonBlocking) != hipSuccess) {
    for (hipStream_t x : s->dev.streams) (void)hipStreamDestroy(x);
    delete s;
    return srv_fail(SLP_EDEVICE, "server: hipStreamCreate failed");
  }
  s->sched = new (std::nothrow) slp::Scheduler<HipDevice>(s->dev, (int64_t)device_budget_bytes, n_slots);
  if (!s->sched) {
    delete s;
    return srv_fail(SLP_ENOMEM, "server: host allocation failed");
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return SLP_OK;
}

int slp_server_add_geometry_near(slp_server *s, const double *nodes, int64_t n_nodes,
                                 const int32_t *tris, int64_t n_tris, const slp_params *p,
                                 double eps, int64_t *geom_id) {
  if (!s || !nodes || !tris || !p || !geom_id || n_nodes < 3 || n_tris < 1 || p->es_terms < 1 ||
      !p->es_w || !p->es_gamma || !std::isfinite(eps))
    return srv_fail(SLP_EINVAL, "server: invalid geometry arguments");
  HostGeometry h;
  h.nodes.assign(nodes, nodes + 3 * n_nodes);
  h.tris.assign(tris, tris + 3 * n_tris);
  h.es_w.assign(p->es_w, p->es_w + p->es_terms);
  h.es_gamma.assign(p->es_gamma, p->es_gamma + p->es_terms);
  h.params = *p;
  h.near_eps = eps > 0.0 ? eps : 0.0;
  int64_t bytes = 0;
  int rc = slp_geometry_device_bytes(nodes, n_nodes, tris, n_tris, p, &bytes);
  if (rc) return rc;
  if (h.near_eps > 0.0) {
    int64_t nb = 0;
    rc = slp_near_field_device_bytes(nodes, n_nodes, tris, n_tris, nullptr, 0, h.near_eps,
                                     p->precision, &nb);
    if (rc) return rc;
    bytes += nb;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  s->geoms.push_back(std::move(h));
  *geom_id = s->sched->add_geometry(bytes);
  return SLP_OK;
}

int slp_server_add_geometry(slp_server *s, const double *nodes, int64_t n_nodes, const int32_t *tris,
                            int64_t n_tris, const slp_params *p, int64_t *geom_id) {
  return slp_server_add_geometry_near(s, nodes, n_nodes, tris, n_tris, p, 0.0, geom_id);
}

int slp_server_submit(slp_server *s, int64_t geom_id, const double *dens, double *phi,
                      uint64_t *ticket) {
  if (!s || !dens || !phi || !ticket) return srv_fail(SLP_EINVAL, "server: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->worker_ok) return srv_fail(SLP_EDEVICE, s->worker_err.c_str());
  if (geom_id < 0 || geom_id >= (int64_t)s->geoms.size())
    return srv_fail(SLP_EINVAL, "server: unknown geometry id");
  slp::SchedRequest r;
  r.geom = geom_id;
  r.dens = dens;
  r.phi = phi;
  *ticket = s->sched->submit(r, now_s());
  s->cv_work.notify_one();
  return SLP_OK;
}

int slp_server_poll(slp_server *s, uint64_t ticket, int32_t *done) {
  if (!s || !done) return srv_fail(SLP_EINVAL, "server: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  const int st = s->sched->state(ticket);
  if (st == slp::kUnknown) return srv_fail(SLP_EINVAL, "server: unknown ticket");
  if (st < 0) {
    *done = 1;
    return srv_fail(st, "server: request failed");
  }
  *done = st == slp::kDone ? 1 : 0;
  return SLP_OK;
}

int slp_server_wait(slp_server *s, uint64_t ticket, double timeout_s) {
  if (!s) return srv_fail(SLP_EINVAL, "server: NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  const auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                            std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 1e9));
  for (;;) {
    const int st = s->sched->state(ticket);
    if (st == slp::kUnknown) return srv_fail(SLP_EINVAL, "server: unknown ticket");
    if (st == slp::kDone) return SLP_OK;
    if (st < 0) return srv_fail(st, "server: request failed");
    if (!s->worker_ok) return srv_fail(SLP_EDEVICE, s->worker_err.c_str());
    if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout &&
        s->sched->state(ticket) != slp::kDone)
      return srv_fail(SLP_ENOTREADY, "server: wait timed out");
  }
}

int slp_server_get_stats(slp_server *s, slp_server_stats *out, int32_t reset) {
  if (!s || !out) return srv_fail(SLP_EINVAL, "server: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto &st = s->sched->stats();
  std::memset(out, 0, sizeof(*out));
  std::vector<double> lat = st.latency;
  std::sort(lat.begin(), lat.end());
  auto pct = [&](double q) {
    if (lat.empty()) return 0.0;
    const double pos = q * (lat.size() - 1);
    const size_t i = (size_t)std::floor(pos);
    const double f = pos - i;
    return i + 1 < lat.size() ? lat[i] * (1 - f) + lat[i + 1] * f : lat[i];
  };
  out->p50_s = pct(0.50);
  out->p99_s = pct(0.99);
  double sum = 0;
  for (double v : lat) sum += v;
  out->mean_s = lat.empty() ? 0.0 : sum / lat.size();
  const double span = st.last_done - st.first_submit;
  out->pts_per_s = span > 0 ? st.points / span : 0.0;
  out->completed = st.completed;
  out->failed = st.failed;
  out->queued = s->sched->queued();
  out->in_flight = s->sched->in_flight();
  out->resident_bytes = s->sched->resident_bytes();
  out->setups = st.setups;
  out->evictions = st.evictions;
  if (reset) {
    st.latency.clear();
    st.completed = st.failed = st.points = 0;
    st.first_submit = st.last_done = -1.0;
  }
  return SLP_OK;
}

int slp_server_destroy(slp_server *s) {
  if (!s) return SLP_OK;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // finish what was admitted
    while (s->worker_ok && !s->sched->idle()) s->cv_done.wait_for(lk, std::chrono::milliseconds(1));
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  for (hipStream_t st : s->dev.streams) (void)hipStreamSynchronize(st);
  s->sched->release_all();
  for (auto &kv : s->dev.events) (void)hipEventDestroy(kv.second);
  for (hipEvent_t e : s->dev.free_events) (void)hipEventDestroy(e);
  for (hipStream_t st : s->dev.streams) (void)hipStreamDestroy(st);
  if (s->dev.setup_stream) (void)hipStreamDestroy(s->dev.setup_stream);
  delete s->sched;
  delete s;
  return SLP_OK;
}

}  // extern "C"
