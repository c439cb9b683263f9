// Request server: a worker thread that keeps geometries resident on the
// device, admits solves by memory, coalesces the pending requests of one
// geometry into batched launches on a pool of streams (the policy is in
// slp_scheduler.hpp, the threading in slp_server_core.hpp). Latency is
// measured from submission to the moment the worker observes the launch's
// completion event.
#include "slp.h"
#include "slp_internal.hpp"
#include "slp_scheduler.hpp"
#include "slp_server_core.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

namespace {

constexpr int kServerBatch = 8;        // largest launch of one geometry
constexpr int kServerLaunches = 4;     // launches in flight per stream

struct HostGeometry {
  std::vector<double> nodes;
  std::vector<int32_t> tris;
  std::vector<double> es_w, es_gamma;
  slp_params params{};
  double near_eps = 0.0;         // near-field correction within this distance (0: none)
  slp_geom *geom = nullptr;
  int64_t points = 0;
  int batch = 1;                 // requests one launch takes (work buffers reserved for them)
};

// The device side of the scheduler; every method runs on the worker thread.
struct HipDevice {
  using Payload = HostGeometry;
  std::vector<HostGeometry> geoms;
  std::vector<hipStream_t> streams;
  hipStream_t setup_stream = nullptr;
  int64_t budget = 0;
  std::map<uint64_t, hipEvent_t> events;   // first ticket of a launch -> completion event
  std::vector<hipEvent_t> free_events;

  void add(HostGeometry &&h) { geoms.push_back(std::move(h)); }

  int setup(int64_t g, int64_t *bytes) {
    HostGeometry &h = geoms[g];
    slp_params p = h.params;
    p.es_w = h.es_w.data();
    p.es_gamma = h.es_gamma.data();
    int rc = slp_setup_geometry(&h.geom, h.nodes.data(), (int64_t)h.nodes.size() / 3, h.tris.data(),
                                (int64_t)h.tris.size() / 3, &p, setup_stream);
    if (!rc && h.near_eps > 0.0) rc = slp_setup_near_field(h.geom, h.near_eps, setup_stream);
    // work buffers for batched launches: as many more items as fit in 1/16 of
    // the budget (at most kServerBatch in all; one where even that is too much)
    if (!rc) {
      const int64_t ib = std::max<int64_t>(slp::item_device_bytes(h.geom), 1);
      h.batch = (int)std::min<int64_t>(kServerBatch, 1 + (budget / 16) / ib);
      if (slp::reserve_items(h.geom, h.batch, setup_stream) != SLP_OK) h.batch = 1;
    }
    if (rc) {
      if (h.geom) slp::destroy_idle(h.geom);
      h.geom = nullptr;
      return rc;
    }
    slp_geom_info info;
    slp_geom_get_info(h.geom, &info);
    *bytes = info.device_bytes;
    h.points = info.n_src + info.n_targets;
    return 0;
  }
  void release(int64_t g) {
    HostGeometry &h = geoms[g];
    // the scheduler evicts only geometries whose launches have all completed
    if (h.geom) slp::destroy_idle(h.geom);
    h.geom = nullptr;
  }
  int max_batch(int64_t g) { return geoms[g].batch; }
  int launch(int slot, const std::vector<slp::SchedRequest> &grp) {
    HostGeometry &h = geoms[grp[0].geom];
    hipStream_t st = streams[slot];
    int rc;
    if (grp.size() == 1) {
      rc = slp_set_density(h.geom, static_cast<const double *>(grp[0].dens), st);
      if (!rc) rc = slp_eval_single_layer(h.geom, static_cast<double *>(grp[0].phi), st);
    } else {
      std::vector<slp_geom *> gs(grp.size(), h.geom);
      std::vector<const double *> ds(grp.size());
      std::vector<double *> ps(grp.size());
      for (size_t i = 0; i < grp.size(); ++i) {
        ds[i] = static_cast<const double *>(grp[i].dens);
        ps[i] = static_cast<double *>(grp[i].phi);
      }
      rc = slp_eval_batched(gs.data(), ds.data(), ps.data(), (int32_t)grp.size(), st);
    }
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
    events[grp[0].ticket] = ev;
    return 0;
  }
  int query(int slot, const std::vector<slp::SchedRequest> &grp) {
    (void)slot;
    auto it = events.find(grp[0].ticket);
    if (it == events.end()) return SLP_EDEVICE;
    const hipError_t e = hipEventQuery(it->second);
    if (e == hipErrorNotReady) return 1;
    free_events.push_back(it->second);
    events.erase(it);
    return e == hipSuccess ? 0 : SLP_EDEVICE;
  }
  int64_t points(int64_t g) { return geoms[g].points; }
};

int srv_fail(int code, const char *msg) {
  slp::set_error_message(msg);
  return code;
}

}  // namespace

struct slp_server {
  HipDevice dev;
  slp::ServerCore<HipDevice> *core = nullptr;
  int device = 0;
  ~slp_server() {
    delete core;   // finishes admitted work and releases the geometries
    for (auto &kv : dev.events) (void)hipEventDestroy(kv.second);
    for (hipEvent_t e : dev.free_events) (void)hipEventDestroy(e);
    for (hipStream_t st : dev.streams) (void)hipStreamDestroy(st);
    if (dev.setup_stream) (void)hipStreamDestroy(dev.setup_stream);
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
  s->dev.budget = (int64_t)device_budget_bytes;
  for (int i = 0; i < n_slots; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      delete s;
      return srv_fail(SLP_EDEVICE, "server: hipStreamCreate failed");
    }
    s->dev.streams.push_back(st);
  }
  if (hipStreamCreateWithFlags(&s->dev.setup_stream, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return srv_fail(SLP_EDEVICE, "server: hipStreamCreate failed");
  }
  const int device = s->device;
  s->core = new (std::nothrow) slp::ServerCore<HipDevice>(
      s->dev, (int64_t)device_budget_bytes, n_slots, kServerLaunches, slp::kMaxBatch,
      [device]() -> std::string {
        return hipSetDevice(device) == hipSuccess ? std::string() : "worker: hipSetDevice failed";
      });
  if (!s->core) {
    delete s;
    return srv_fail(SLP_ENOMEM, "server: host allocation failed");
  }
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
  *geom_id = s->core->add_geometry(bytes, std::move(h));
  return SLP_OK;
}

int slp_server_add_geometry(slp_server *s, const double *nodes, int64_t n_nodes, const int32_t *tris,
                            int64_t n_tris, const slp_params *p, int64_t *geom_id) {
  return slp_server_add_geometry_near(s, nodes, n_nodes, tris, n_tris, p, 0.0, geom_id);
}

int slp_server_submit(slp_server *s, int64_t geom_id, const double *dens, double *phi,
                      uint64_t *ticket) {
  if (!s || !dens || !phi || !ticket) return srv_fail(SLP_EINVAL, "server: NULL argument");
  if (geom_id < 0 || geom_id >= s->core->geometries())
    return srv_fail(SLP_EINVAL, "server: unknown geometry id");
  const uint64_t t = s->core->submit(geom_id, dens, phi);
  if (t == 0) {
    std::string err;
    s->core->worker_ok(&err);
    slp::set_error_message(err.c_str());
    return SLP_EDEVICE;
  }
  *ticket = t;
  return SLP_OK;
}

int slp_server_poll(slp_server *s, uint64_t ticket, int32_t *done) {
  if (!s || !done) return srv_fail(SLP_EINVAL, "server: NULL argument");
  const int st = s->core->state(ticket);
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
  const int st = s->core->wait(ticket, timeout_s);
  if (st == slp::kDone) return SLP_OK;
  if (st < 0 && st != slp::kUnknown) return srv_fail(st, "server: request failed");
  std::string err;
  if (!s->core->worker_ok(&err)) return srv_fail(SLP_EDEVICE, err.c_str());
  if (st == slp::kUnknown) return srv_fail(SLP_EINVAL, "server: unknown ticket");
  return srv_fail(SLP_ENOTREADY, "server: wait timed out");
}

int slp_server_get_stats(slp_server *s, slp_server_stats *out, int32_t reset) {
  if (!s || !out) return srv_fail(SLP_EINVAL, "server: NULL argument");
  slp::ServerTotals t = s->core->totals(reset != 0);
  std::memset(out, 0, sizeof(*out));
  std::sort(t.latency.begin(), t.latency.end());
  out->p50_s = slp::quantile_sorted(t.latency, 0.50);
  out->p99_s = slp::quantile_sorted(t.latency, 0.99);
  double sum = 0;
  for (double v : t.latency) sum += v;
  out->mean_s = t.latency.empty() ? 0.0 : sum / (double)t.latency.size();
  const double span = t.last_done - t.first_submit;
  out->pts_per_s = span > 0 ? (double)t.points / span : 0.0;
  out->completed = t.completed;
  out->failed = t.failed;
  out->queued = t.queued;
  out->in_flight = t.in_flight;
  out->resident_bytes = t.resident_bytes;
  out->setups = t.setups;
  out->evictions = t.evictions;
  out->launches = t.launches;
  return SLP_OK;
}

int slp_server_destroy(slp_server *s) {
  delete s;
  return SLP_OK;
}

}  // extern "C"
