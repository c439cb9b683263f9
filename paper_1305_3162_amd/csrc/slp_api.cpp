// Host side of libslp: argument checking, the setup phase (scaling, quadrature
// sources, binning, kernel tables) and the orchestration of the evaluation
// passes. Every arithmetic step of the evaluation runs in slp_kernels.hip.
#include "slp.h"
#include "slp_internal.hpp"
#include "slp_near.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <utility>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <queue>
#include <string>
#include <thread>
#include <vector>

using slp::kTile;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(SLP_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                  __FILE__, __LINE__);                                                   \
  } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.141592653589793238462643383279502884;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// The collapsed Gauss rule on the unit triangle, [order^2][3]: xi_1 = u (1 - v),
// xi_2 = u v, weight w_u w_v u (weights sum to 1/2).
std::vector<double> collapsed_rule(int order) {
  std::vector<double> glx, glw, rule;
  gauss_legendre(order, glx, glw);
  for (int a = 0; a < order; ++a)
    for (int b = 0; b < order; ++b) {
      const double u = 0.5 * (glx[a] + 1.0), v = 0.5 * (glx[b] + 1.0);
      rule.push_back(u * (1.0 - v));
      rule.push_back(u * v);
      rule.push_back(0.25 * glw[a] * glw[b] * u);
    }
  return rule;
}

// Stable counting sort of items by bin id; returns order (sorted -> item) and
// bin_start [nbins + 1].
void counting_sort(const std::vector<int32_t> &bin, int64_t nbins, std::vector<int32_t> &order,
                   std::vector<int32_t> &start) {
  start.assign(nbins + 1, 0);
  for (int32_t b : bin) start[b + 1]++;
  for (int64_t i = 0; i < nbins; ++i) start[i + 1] += start[i];
  std::vector<int32_t> fill(start.begin(), start.end() - 1);
  order.resize(bin.size());
  for (size_t i = 0; i < bin.size(); ++i) order[fill[bin[i]]++] = (int32_t)i;
}

}  // namespace

void slp::set_error_message(const char *msg) { g_err = msg; }

static std::atomic<uint64_t> g_geom_serial{1};

struct slp_geom {
  uint64_t serial = g_geom_serial++;   // never reused: identifies the context in cached plans
  int prec = SLP_FP64;
  int N[3]{}, n[3]{}, alpha = 2, m = 4;
  double b = 0.0;                // window shape
  int32_t window = SLP_WINDOW_GAUSS;
  double kb_inv_norm = 1.0;      // m / sinh(b m) (Kaiser-Bessel scaled to 1 at tau = 0)
  std::vector<double> kb_coef = std::vector<double>(slp::kKbCoef, 0.0);   // KB stencil polynomials
  double c[3]{}, s[3]{};
  int64_t n_nodes = 0, n_tris = 0, n_src = 0;
  int64_t n_tgt = 0;             // evaluation points (the nodes unless given separately)
  int32_t lo[3]{}, R[3]{}, P[3]{}, tiles[3]{}, K[3]{};
  int32_t terms_kept = 0;
  int32_t n_slots = 0;           // segments (padded gridding blocks)
  int64_t share = 0;             // sources per segment piece in effect
  int32_t reduce_cells = 0;      // block-sum cells per thread (0 = automatic)
  int32_t n_units = 0;           // gridding work units (workgroups per item)
  int32_t cap = 1;               // batch items the per-item buffers hold
  int64_t item_elems[5]{};       // per item: scratch, grid_a, S1 (complex), S2 (complex), grid_g
  const double *dens = nullptr;  // density of the next single evaluation (caller's device buffer)
  int32_t n_tgt_tiles = 0;       // tiles holding targets
  std::vector<int32_t> unit_len; // host: sources of each gridding work unit (unit order)
  std::vector<int32_t> tgt_len;  // host: targets of each active tile (active order)
  // device buffers
  void *src_frac = nullptr;
  double *src_w = nullptr;
  int32_t *src_perm = nullptr;
  int4 *units = nullptr;
  int4 *chunks = nullptr;
  int32_t *runs = nullptr;
  int4 *tile_slots = nullptr;
  void *scratch = nullptr;
  int32_t *tgt_cell = nullptr;
  void *tgt_frac = nullptr;
  int32_t *tgt_perm = nullptr;
  int4 *tgt_rec = nullptr;       // per active tile: {tile, first target, end target, cell box}
  void *kb_tab = nullptr;        // Kaiser-Bessel window polynomials in the working precision
  void *grid_a = nullptr;
  void *S1 = nullptr;
  void *S2 = nullptr;
  void *grid_g = nullptr;
  void *mu = nullptr;
  void *tw[3] = {nullptr, nullptr, nullptr};
  int32_t *tri_v = nullptr;      // [3][M] vertex indices, component-major
  double *tri_n = nullptr;       // [3][M] unit outward normals, component-major
  double *own_dens = nullptr;    // [3M] density formed by slp_set_density_from_m
  // host copies kept for the near-field setup: physical nodes, triangles,
  // targets, the kept exponential-sum terms and the body diameter
  std::vector<double> h_nodes, h_tgt, kept_w, kept_g;
  std::vector<int32_t> h_tris;
  double r_max = 0.0;
  // near-field correction (empty unless slp_setup_near_field ran with eps > 0)
  double nf_eps = 0.0;
  int64_t nf_nnz = 0;            // pairs
  int64_t nf_stored = 0;         // entries including the padding of every row to a group
  int64_t *nf_rowptr = nullptr;
  int32_t *nf_cols = nullptr;    // unless packed
  int32_t *nf_bases = nullptr;   // packed: chunk bases
  uint16_t *nf_offs = nullptr;   // packed: per-entry offsets
  bool nf_packed = false;
  bool nf_chunked = false;
  std::vector<int64_t> nf_rows;  // host: pairs per row (to strip the padding on copies)
  void *nf_vals = nullptr;
  double *nf_gbar = nullptr;     // [cap][M] element means of the densities
  int32_t nf_rule = 0;           // integrated-gridding order the values were built for (0: points)
  int32_t nf_prec = SLP_FP64;    // storage precision of the near-field values
  // integrated-window gridding (slp_setup_integrated_gridding): the window
  // integrated over each triangle, by cell of the region, in the near-field
  // layout; when set, a = A gbar replaces the gridding of the point sources
  int32_t iw_order = 0;          // Gauss points per direction of the rule; 0 = off
  int64_t iw_nnz = 0, iw_stored = 0, iw_rows = 0;
  int64_t *iw_rowptr = nullptr;
  int32_t *iw_cols = nullptr, *iw_bases = nullptr;
  uint16_t *iw_offs = nullptr;
  bool iw_packed = false;
  void *iw_vals = nullptr;
  double *iw_gbar = nullptr;     // [cap][M]
  int64_t bytes = 0;
  std::vector<void *> allocs;
  // captured evaluations, one per batch size (replayed when use_graph is set)
  struct Captured {
    int nb = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t spread_node = nullptr, interp_node = nullptr;
    hipGraphNode_t gbar_node = nullptr, near_node = nullptr;
    hipKernelNodeParams spread_p{}, interp_p{}, gbar_p{}, near_p{};
  };
  bool use_graph = false;
  std::vector<Captured> graphs;
  hipStream_t cap_stream = nullptr;
  void drop_graphs() {
    for (Captured &cg : graphs) {
      if (cg.exec) (void)hipGraphExecDestroy(cg.exec);
      if (cg.graph) (void)hipGraphDestroy(cg.graph);
    }
    graphs.clear();
  }
  // timing: a ring of event sets, one per evaluation, read back lazily
  static constexpr int kRing = 32;
  bool timing = false;
  int32_t every = 1;             // record the stage events of every k-th evaluation
  int64_t evals = 0;             // evaluations since timing was enabled
  bool ev_ready = false;
  static constexpr int kStages = 9;
  hipEvent_t ev[kRing][kStages + 1]{};
  bool used[kRing]{};
  bool with_near[kRing]{};       // the set recorded the near-field stage
  int cur = 0;
  double acc_ms[kStages]{};
  int64_t count = 0;
  hipEvent_t *evs() { return ev[cur]; }

  size_t esz() const { return prec == SLP_FP64 ? sizeof(double) : sizeof(float); }

  static constexpr size_t kMinAlloc = 256;
  hipError_t alloc(void **p, size_t bytes_) {
    *p = nullptr;
    if (bytes_ < kMinAlloc) bytes_ = kMinAlloc;
    hipError_t e = hipMalloc(p, bytes_);
    if (e == hipSuccess) {
      allocs.push_back(*p);
      alloc_bytes.push_back((int64_t)bytes_);
      bytes += (int64_t)bytes_;
    }
    return e;
  }
  void release(void *p) {
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == p) {
        (void)hipFree(p);
        bytes -= alloc_bytes[i];
        allocs.erase(allocs.begin() + i);
        alloc_bytes.erase(alloc_bytes.begin() + i);
        return;
      }
  }
  std::vector<int64_t> alloc_bytes;
  ~slp_geom() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void *p : allocs) (void)hipFree(p);
    if (ev_ready)
      for (auto &set : ev)
        for (auto &e : set) (void)hipEventDestroy(e);
  }
};

namespace {

int validate_params(const slp_params *p) {
  if (!p) return fail(SLP_EINVAL, "params is NULL");
  if (p->alpha < 2) return fail(SLP_EINVAL, "alpha must be >= 2 (got %d)", p->alpha);
  if (p->m < 1 || p->m > slp::kMaxM)
    return fail(SLP_EINVAL, "m must be in [1, %d] (got %d)", slp::kMaxM, p->m);
  if (p->precision != SLP_FP64 && p->precision != SLP_FP32)
    return fail(SLP_EINVAL, "precision must be SLP_FP64 or SLP_FP32");
  if (p->window != SLP_WINDOW_GAUSS && p->window != SLP_WINDOW_KB)
    return fail(SLP_EINVAL, "window must be SLP_WINDOW_GAUSS or SLP_WINDOW_KB");
  for (int q = 0; q < 3; ++q) {
    const int N = p->grid[q];
    if (!is_pow2(N) || N < 8 || N > 2048)
      return fail(SLP_EINVAL, "grid[%d] = %d: must be a power of two in [8, 2048]", q, N);
    if (N % p->alpha != 0 || (N / p->alpha) % 2 != 0)
      return fail(SLP_EINVAL, "grid[%d] = %d: must be alpha * n with n even", q, N);
  }
  if (p->es_terms < 1 || !p->es_w || !p->es_gamma)
    return fail(SLP_EINVAL, "exponential sum: es_terms >= 1 and both arrays required");
  for (int t = 0; t < p->es_terms; ++t)
    if (!std::isfinite(p->es_w[t]) || !std::isfinite(p->es_gamma[t]) || p->es_gamma[t] <= 0.0)
      return fail(SLP_EINVAL, "exponential sum term %d is not finite / gamma <= 0", t);
  if (!(p->eta2 > 0.0) || !std::isfinite(p->eta2))
    return fail(SLP_EINVAL, "eta2 must be positive and finite");
  if (p->seg_share != 0 && (p->seg_share < 64 || p->seg_share > (1 << 24)))
    return fail(SLP_EINVAL, "seg_share must be 0 (automatic) or in [64, 2^24] (got %d)",
                p->seg_share);
  if (p->reduce_cells < 0 || p->reduce_cells > 2)
    return fail(SLP_EINVAL, "reduce_cells must be 0 (automatic), 1 or 2 (got %d)",
                p->reduce_cells);
  return SLP_OK;
}

template <typename T>
void split_coords(const std::vector<double> &t, const std::vector<int32_t> &order,
                  const int32_t lo[3], int64_t n, std::vector<int32_t> &cell, std::vector<T> &frac) {
  cell.resize(3 * n);
  frac.resize(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t o = order[i];
    for (int q = 0; q < 3; ++q) {
      const double v = t[3 * o + q];
      const double f = std::floor(v);
      cell[q * n + i] = (int32_t)f - lo[q];
      frac[q * n + i] = (T)(v - f);
    }
  }
}

template <typename T>
int upload_tables(slp_geom *G, const std::vector<double> &ts, const std::vector<int32_t> &sorder,
                  const std::vector<double> &tt, const std::vector<int32_t> &torder,
                  hipStream_t st, std::vector<int32_t> &cellbuf_s, std::vector<T> &fracbuf_s,
                  std::vector<int32_t> &cellbuf_t, std::vector<T> &fracbuf_t) {
  split_coords<T>(ts, sorder, G->lo, G->n_src, cellbuf_s, fracbuf_s);
  split_coords<T>(tt, torder, G->lo, G->n_tgt, cellbuf_t, fracbuf_t);
  HIP_TRY(hipMemcpyAsync(G->src_frac, fracbuf_s.data(), fracbuf_s.size() * sizeof(T), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->tgt_cell, cellbuf_t.data(), cellbuf_t.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->tgt_frac, fracbuf_t.data(), fracbuf_t.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return SLP_OK;
}

template <typename T>
int upload_twiddles(slp_geom *G, hipStream_t st, std::vector<std::vector<T>> &hold) {
  const double pi = 3.141592653589793238462643383279502884;
  hold.resize(3);
  for (int q = 0; q < 3; ++q) {
    const int N = G->N[q];
    hold[q].resize(2 * (size_t)N);
    for (int k = 0; k < N; ++k) {
      const double a = 2.0 * pi * (double)k / (double)N;
      hold[q][2 * k] = (T)std::cos(a);
      hold[q][2 * k + 1] = (T)(-std::sin(a));
    }
    HIP_TRY(hipMemcpyAsync(G->tw[q], hold[q].data(), hold[q].size() * sizeof(T), hipMemcpyHostToDevice, st));
  }
  return SLP_OK;
}

// Kaiser-Bessel window polynomials of the gridding and interpolation (the
// window of eq. KBfct in grid units, scaled to 1 at tau = 0): for stencil
// point j of a point with fraction f the window is taken at tau = f + m - 1 - j,
// i.e. on one unit interval per j; there it is interpolated at the deg + 1
// Chebyshev points in u = 2 f - 1 and the interpolant converted to monomial
// coefficients. The window is an entire function of tau (sinh(b s) / s is even
// in s = sqrt(m^2 - tau^2)), so the interpolant converges fast: at degree 16
// its error is below 1.1e-14 of the peak for every m <= 8 (degree 8: below FP32
// rounding). Other slots stay zero.
std::vector<double> kb_polynomials(int m, double b, double inv_norm, int deg) {
  const double pi = 3.141592653589793238462643383279502884;
  std::vector<double> out(slp::kKbCoef, 0.0);
  auto window = [&](double tau) {
    const double s2 = (double)m * m - tau * tau;
    const double s = s2 > 0.0 ? std::sqrt(s2) : 0.0;
    if (s < 1e-12) return b * inv_norm;
    return std::sinh(b * s) / s * inv_norm;
  };
  const int n = deg + 1;
  for (int j = 0; j < m; ++j) {
    // Chebyshev coefficients from the values at the Chebyshev points
    std::vector<double> y(n), cc(n, 0.0);
    for (int k = 0; k < n; ++k) {
      const double u = std::cos(pi * (k + 0.5) / n);
      y[k] = window((u + 1.0) / 2.0 + m - 1 - j);
    }
    for (int l = 0; l < n; ++l) {
      double acc = 0.0;
      for (int k = 0; k < n; ++k) acc += y[k] * std::cos(pi * l * (k + 0.5) / n);
      cc[l] = (l == 0 ? 1.0 : 2.0) * acc / n;
    }
    // sum_l cc[l] T_l(u) in monomials: T_{l+1} = 2 u T_l - T_{l-1}
    std::vector<double> tprev(n, 0.0), tcur(n, 0.0), mono(n, 0.0);
    tprev[0] = 1.0;                       // T_0
    if (n > 1) tcur[1] = 1.0;             // T_1
    for (int d = 0; d < n; ++d) mono[d] += cc[0] * tprev[d];
    for (int l = 1; l < n; ++l) {
      for (int d = 0; d < n; ++d) mono[d] += cc[l] * tcur[d];
      std::vector<double> tnext(n, 0.0);
      for (int d = 0; d + 1 < n; ++d) tnext[d + 1] += 2.0 * tcur[d];
      for (int d = 0; d < n; ++d) tnext[d] -= tprev[d];
      tprev.swap(tcur);
      tcur.swap(tnext);
    }
    // the window is even, so the interval 2m - 1 - j holds P_j(-u): stored
    // exactly so (the kernels evaluate each pair from P_j's coefficients)
    for (int d = 0; d < n; ++d) {
      out[(size_t)j * n + d] = mono[d];
      out[(size_t)(2 * m - 1 - j) * n + d] = (d % 2 ? -mono[d] : mono[d]);
    }
  }
  return out;
}

// Grow the per-item work buffers to hold nb batch items (synchronises the
// stream before freeing the old ones).
int ensure_capacity(slp_geom *G, int nb, hipStream_t st) {
  if (nb <= G->cap) return SLP_OK;
  HIP_TRY(hipStreamSynchronize(st));
  if (!G->graphs.empty()) {
    HIP_TRY(hipDeviceSynchronize());   // captured evaluations may still run elsewhere
    G->drop_graphs();                  // they hold the old buffer addresses
  }
  for (double **gb : {&G->nf_gbar, &G->iw_gbar}) {   // element means, nb items
    if (!*gb) continue;
    void *q = nullptr;
    if (G->alloc(&q, (size_t)G->n_tris * 8 * nb) != hipSuccess)
      return fail(SLP_ENOMEM, "element-mean buffer for %d items: allocation failed", nb);
    G->release(*gb);
    *gb = static_cast<double *>(q);
  }
  void **bufs[5] = {&G->scratch, &G->grid_a, &G->S1, &G->S2, &G->grid_g};
  const size_t e = G->esz();
  const size_t per[5] = {e, e, 2 * e, 2 * e, e};
  for (int i = 0; i < 5; ++i) {
    G->release(*bufs[i]);
    *bufs[i] = nullptr;
  }
  for (int i = 0; i < 5; ++i)
    if (G->alloc(bufs[i], (size_t)G->item_elems[i] * per[i] * nb) != hipSuccess) {
      // leave a usable single-item context behind
      for (int k = 0; k < 5; ++k)
        if (*bufs[k]) { G->release(*bufs[k]); *bufs[k] = nullptr; }
      bool ok = true;
      for (int k = 0; k < 5; ++k) ok = ok && G->alloc(bufs[k], (size_t)G->item_elems[k] * per[k]) == hipSuccess;
      G->cap = 1;
      return fail(ok ? SLP_ENOMEM : SLP_EDEVICE, "batch buffers for %d items: allocation failed", nb);
    }
  G->cap = nb;
  return SLP_OK;
}

// Per-evaluation work buffers of one evaluation (blocks of the gridding
// segments, region grid, both half spectra, grid after the inverse FFT,
// element means of the near field and of integrated-window gridding) and
// their per-item element counts: the context's own buffers, or a carve-out
// of the static workspace (slp_eval_single_layer_static).
struct WorkBufs {
  void *scratch = nullptr, *grid_a = nullptr, *S1 = nullptr, *S2 = nullptr, *grid_g = nullptr;
  double *nf_gbar = nullptr, *iw_gbar = nullptr;
  int64_t elems[5]{};
};

WorkBufs ctx_work(const slp_geom *G) {
  WorkBufs W;
  W.scratch = G->scratch;
  W.grid_a = G->grid_a;
  W.S1 = G->S1;
  W.S2 = G->S2;
  W.grid_g = G->grid_g;
  W.nf_gbar = G->nf_gbar;
  W.iw_gbar = G->iw_gbar;
  for (int i = 0; i < 5; ++i) W.elems[i] = G->item_elems[i];
  return W;
}

template <typename T>
slp::SpreadBinsArgs<T> spread_args(const slp_geom *G, const WorkBufs &W) {
  slp::SpreadBinsArgs<T> a{};
  a.frac = static_cast<const T *>(G->src_frac);
  a.w = G->src_w;
  a.perm = G->src_perm;
  a.units = G->units;
  a.chunks = G->chunks;
  a.runs = G->runs;
  a.scratch = static_cast<T *>(W.scratch);
  a.ns = G->n_src;
  a.scratch_bstride = W.elems[0];
  a.inv_b = (T)(1.0 / G->b);
  a.step_ratio = (T)std::exp(-2.0 / G->b);
  a.window = G->window;
  for (int i = 0; i < slp::kKbCoef; ++i) a.kb_c[i] = (T)G->kb_coef[i];
  return a;
}

template <typename T>
slp::InterpArgs<T> interp_args(const slp_geom *G, const WorkBufs &W) {
  slp::InterpArgs<T> a{};
  a.cell = G->tgt_cell;
  a.frac = static_cast<const T *>(G->tgt_frac);
  a.perm = G->tgt_perm;
  a.rec = G->tgt_rec;
  a.kb_tab = static_cast<const T *>(G->kb_tab);
  a.g = static_cast<const T *>(W.grid_g);
  a.g_bstride = W.elems[4];
  for (int i = 0; i < 3; ++i) {
    a.R[i] = G->R[i];
    a.tiles[i] = G->tiles[i];
  }
  a.nt = G->n_tgt;
  a.inv_b = (T)(1.0 / G->b);
  a.window = G->window;
  return a;
}

template <typename T>
slp::SpreadReduceArgs<T> reduce_args(const slp_geom *G, const WorkBufs &W) {
  slp::SpreadReduceArgs<T> r{};
  r.scratch = static_cast<const T *>(W.scratch);
  r.tile_slots = G->tile_slots;
  r.grid = static_cast<T *>(W.grid_a);
  r.scratch_bstride = W.elems[0];
  r.grid_bstride = W.elems[1];
  for (int i = 0; i < 3; ++i) r.tiles[i] = G->tiles[i];
  return r;
}

// The five FFT passes of an evaluation (Sec. 3, steps 2-4): x forward (real
// region rows -> kx = 0..n_x/2), y forward (region y -> ky = -n_y/2..n_y/2),
// z forward with the multiplication by mu on kz = -n_z/2..n_z/2 and the z
// inverse back to the region, y inverse (ky -> region y), x inverse
// (Hermitian half spectrum -> real region rows). Line lengths in G->N.
template <typename T>
void fft_passes(const slp_geom *G, const WorkBufs &W, slp::FftPass<T> (&ps)[5]) {
  const int64_t Rx = G->R[0], Ry = G->R[1], Rz = G->R[2];
  const int64_t Px = G->P[0], Py = G->P[1];
  const int64_t Kx = G->K[0], Ky = G->K[1], Kz = G->K[2];
  const int ny = G->n[1], nz = G->n[2];
  for (slp::FftPass<T> &p : ps) p = slp::FftPass<T>{};
  {
    slp::FftPass<T> &p = ps[0];
    p.in = W.grid_a; p.out = W.S1; p.tw = G->tw[0];
    p.n_lines = Ry * Rz; p.l1 = Ry;
    p.in_s1 = Px; p.in_s2 = Py * Px; p.in_es = 1; p.in_cnt = (int)Rx; p.in_shift = G->lo[0];
    p.out_s1 = Kx; p.out_s2 = Ry * Kx; p.out_es = 1; p.out_cnt = (int)Kx; p.out_shift = 0;
    p.sign = -1; p.in_real = 1;
    p.in_bstride = W.elems[1]; p.out_bstride = W.elems[2];
  }
  {
    slp::FftPass<T> &p = ps[1];
    p.in = W.S1; p.out = W.S2; p.tw = G->tw[1];
    p.n_lines = Kx * Rz; p.l1 = Kx;
    p.in_s1 = 1; p.in_s2 = Ry * Kx; p.in_es = Kx; p.in_cnt = (int)Ry; p.in_shift = G->lo[1];
    p.out_s1 = 1; p.out_s2 = Ky * Kx; p.out_es = Kx; p.out_cnt = (int)Ky; p.out_shift = -ny / 2;
    p.sign = -1;
    p.in_bstride = W.elems[2]; p.out_bstride = W.elems[3];
  }
  {
    slp::FftPass<T> &p = ps[2];
    p.in = W.S2; p.out = W.S2; p.tw = G->tw[2];
    p.mu = static_cast<const T *>(G->mu);
    p.n_lines = Kx * Ky; p.l1 = Kx;
    p.in_s1 = 1; p.in_s2 = Kx; p.in_es = Ky * Kx; p.in_cnt = (int)Rz; p.in_shift = G->lo[2];
    p.mu_cnt = (int)Kz; p.mu_shift = -nz / 2;
    for (int q = 0; q < 3; ++q) p.mu_n[q] = G->n[q];
    p.out_s1 = 1; p.out_s2 = Kx; p.out_es = Ky * Kx; p.out_cnt = (int)Rz; p.out_shift = G->lo[2];
    p.sign = -1; p.mul_inv = 1;
    p.in_bstride = W.elems[3]; p.out_bstride = W.elems[3];
  }
  {
    slp::FftPass<T> &p = ps[3];
    p.in = W.S2; p.out = W.S1; p.tw = G->tw[1];
    p.n_lines = Kx * Rz; p.l1 = Kx;
    p.in_s1 = 1; p.in_s2 = Ky * Kx; p.in_es = Kx; p.in_cnt = (int)Ky; p.in_shift = -ny / 2;
    p.out_s1 = 1; p.out_s2 = Ry * Kx; p.out_es = Kx; p.out_cnt = (int)Ry; p.out_shift = G->lo[1];
    p.sign = +1;
    p.in_bstride = W.elems[3]; p.out_bstride = W.elems[2];
  }
  {
    slp::FftPass<T> &p = ps[4];
    p.in = W.S1; p.out = W.grid_g; p.tw = G->tw[0];
    p.n_lines = Ry * Rz; p.l1 = Ry;
    p.in_s1 = Kx; p.in_s2 = Ry * Kx; p.in_es = 1; p.in_cnt = (int)Kx; p.in_shift = 0;
    p.in_hermitian = 1;
    p.out_s1 = Rx; p.out_s2 = Ry * Rx; p.out_es = 1; p.out_cnt = (int)Rx; p.out_shift = G->lo[0];
    p.out_real = 1; p.sign = +1;
    p.in_bstride = W.elems[2]; p.out_bstride = W.elems[4];
  }
}

// Axis of each of the five passes.
constexpr int kPassAxis[5] = {0, 1, 2, 1, 0};

template <typename T>
slp::NearArgs<T> near_args(const slp_geom *G, const WorkBufs &W) {
  slp::NearArgs<T> a{};
  a.rowptr = G->nf_rowptr;
  a.cols = G->nf_cols;
  a.bases = G->nf_bases;
  a.offs = G->nf_offs;
  a.vals = static_cast<T *>(G->nf_vals);
  a.gbar = W.nf_gbar;
  a.rows = G->n_tgt;
  a.M = G->n_tris;
  return a;
}

// The near-field product in the values' storage precision (FP32 storage in an
// FP64 context halves the bytes of the HBM-bound product; the sums stay FP64).
hipError_t near_apply(const slp_geom *G, const WorkBufs &W, const slp::BatchPtrs &ptrs, int nb,
                      hipStream_t st) {
  if (G->nf_prec == SLP_FP64)
    return slp::launch_near_apply<double>(near_args<double>(G, W), ptrs, nb, G->nf_packed, st);
  return slp::launch_near_apply<float>(near_args<float>(G, W), ptrs, nb, G->nf_packed, st);
}

template <typename T>
slp::NearArgs<T> iw_args(const slp_geom *G, const WorkBufs &W) {
  slp::NearArgs<T> a{};
  a.rowptr = G->iw_rowptr;
  a.cols = G->iw_cols;
  a.bases = G->iw_bases;
  a.offs = G->iw_offs;
  a.vals = static_cast<T *>(G->iw_vals);
  a.gbar = W.iw_gbar;
  a.rows = G->iw_rows;
  a.M = G->n_tris;
  return a;
}

template <typename T>
int run_eval(slp_geom *G, const WorkBufs &W, const slp::BatchPtrs &ptrs, int nb, hipStream_t st,
             bool tm) {
  if (G->nf_nnz > 0 && G->nf_rule != G->iw_order)
    return fail(SLP_EINVAL, "the near field was built for another gridding (set it up again)");
  if (G->iw_order > 0) {
    // integrated-window gridding: a = A gbar (the whole gridding stage; the
    // block-sum stage takes no time)
    slp::IwOut<T> o{};
    o.grid = static_cast<T *>(W.grid_a);
    o.bstride = W.elems[1];
    for (int i = 0; i < 3; ++i) { o.R[i] = G->R[i]; o.P[i] = G->P[i]; }
    const bool short_rows = !G->iw_packed && G->iw_stored < 512 * G->iw_rows;
    HIP_TRY(slp::launch_iw_apply<T>(iw_args<T>(G, W), o, ptrs, nb, G->iw_packed, short_rows, st));
    if (tm) HIP_TRY(hipEventRecord(G->evs()[1], st));
  } else {
    // spread (the charges q = w g are formed inside the gridding)
    const slp::SpreadBinsArgs<T> a = spread_args<T>(G, W);
    const slp::SpreadReduceArgs<T> r = reduce_args<T>(G, W);
    HIP_TRY(slp::launch_spread<T>(a, r, ptrs, G->n_units, G->m, nb, G->reduce_cells, st,
                                  tm ? G->evs()[1] : nullptr));
  }
  if (tm) HIP_TRY(hipEventRecord(G->evs()[2], st));
  slp::FftPass<T> ps[5];
  fft_passes<T>(G, W, ps);
  for (int k = 0; k < 5; ++k) {
    HIP_TRY(slp::launch_fft<T>(ps[k], G->N[kPassAxis[k]], nb, st));
    if (tm) HIP_TRY(hipEventRecord(G->evs()[3 + k], st));
  }

  {
    const slp::InterpArgs<T> a = interp_args<T>(G, W);
    HIP_TRY(slp::launch_interp<T>(a, ptrs, G->n_tgt_tiles, G->m, nb, st));
  }
  const bool near = G->nf_nnz > 0;
  if (tm && near) HIP_TRY(hipEventRecord(G->evs()[8], st));
  if (near) HIP_TRY(near_apply(G, W, ptrs, nb, st));
  if (tm) {
    G->with_near[G->cur] = near;
    HIP_TRY(hipEventRecord(G->evs()[slp_geom::kStages], st));
    G->used[G->cur] = true;
    G->cur = (G->cur + 1) % slp_geom::kRing;
  }
  return SLP_OK;
}

// Evaluation through a captured HIP graph: the kernel sequence of one
// evaluation with nb items is captured once per batch size on a private stream;
// a replay updates the per-item pointers of the gridding and interpolation
// launches (their other arguments are rebuilt from the context, unchanged
// since capture) and launches the graph on the caller's stream.
template <typename T>
int run_graph(slp_geom *G, const slp::BatchPtrs &ptrs, int nb, hipStream_t st) {
  slp_geom::Captured *cg = nullptr;
  for (slp_geom::Captured &c : G->graphs)
    if (c.nb == nb) cg = &c;
  if (!cg) {
    if (!G->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&G->cap_stream, hipStreamNonBlocking));
    slp_geom::Captured c;
    c.nb = nb;
    HIP_TRY(hipStreamBeginCapture(G->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = run_eval<T>(G, ctx_work(G), ptrs, nb, G->cap_stream, false);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(G->cap_stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    HIP_TRY(ec);
    c.graph = graph;
    size_t n = 0;
    HIP_TRY(hipGraphGetNodes(graph, nullptr, &n));
    std::vector<hipGraphNode_t> nodes(n);
    HIP_TRY(hipGraphGetNodes(graph, nodes.data(), &n));
    const void *fs = slp::spread_bins_kernel<T>(G->m), *fi = slp::interp_kernel<T>(G->m);
    const void *fn = G->nf_prec == SLP_FP64 ? slp::near_apply_kernel<double>(nb, G->nf_packed)
                                            : slp::near_apply_kernel<float>(nb, G->nf_packed);
    const void *fg = slp::near_gbar_kernel();
    for (hipGraphNode_t nd : nodes) {
      hipGraphNodeType ty;
      HIP_TRY(hipGraphNodeGetType(nd, &ty));
      if (ty != hipGraphNodeTypeKernel) continue;
      hipKernelNodeParams kp{};
      HIP_TRY(hipGraphKernelNodeGetParams(nd, &kp));
      if (kp.func == fs) { c.spread_node = nd; c.spread_p = kp; }
      if (kp.func == fi) { c.interp_node = nd; c.interp_p = kp; }
      if (kp.func == fn) { c.near_node = nd; c.near_p = kp; }
      if (kp.func == fg) { c.gbar_node = nd; c.gbar_p = kp; }
    }
    const bool near = G->nf_nnz > 0;
    if (!c.spread_node || !c.interp_node || near != (c.near_node != nullptr) ||
        near != (c.gbar_node != nullptr)) {
      (void)hipGraphDestroy(graph);
      return fail(SLP_EDEVICE, "captured evaluation lacks the gridding, interpolation or near-field launch");
    }
    HIP_TRY(hipGraphInstantiate(&c.exec, graph, nullptr, nullptr, 0));
    G->graphs.push_back(c);
    cg = &G->graphs.back();
  }
  slp::BatchPtrs p = ptrs;
  const WorkBufs W = ctx_work(G);
  slp::SpreadBinsArgs<T> sa = spread_args<T>(G, W);
  slp::InterpArgs<T> ia = interp_args<T>(G, W);
  void *sargs[2] = {&sa, &p};
  void *iargs[2] = {&ia, &p};
  hipKernelNodeParams kp = cg->spread_p;
  kp.kernelParams = sargs;
  kp.extra = nullptr;
  HIP_TRY(hipGraphExecKernelNodeSetParams(cg->exec, cg->spread_node, &kp));
  kp = cg->interp_p;
  kp.kernelParams = iargs;
  kp.extra = nullptr;
  HIP_TRY(hipGraphExecKernelNodeSetParams(cg->exec, cg->interp_node, &kp));
  if (cg->near_node) {
    // the two argument types differ only in the type of the value pointer
    slp::NearArgs<double> nad = near_args<double>(G, W);
    slp::NearArgs<float> naf = near_args<float>(G, W);
    int32_t nbv = nb;
    double *gbar = W.nf_gbar;
    int64_t M = G->n_tris;
    void *gargs[3] = {&p, &gbar, &M};
    kp = cg->gbar_p;
    kp.kernelParams = gargs;
    kp.extra = nullptr;
    HIP_TRY(hipGraphExecKernelNodeSetParams(cg->exec, cg->gbar_node, &kp));
    void *nargs[3] = {G->nf_prec == SLP_FP64 ? static_cast<void *>(&nad) : static_cast<void *>(&naf),
                      &p, &nbv};
    kp = cg->near_p;
    kp.kernelParams = nargs;
    kp.extra = nullptr;
    HIP_TRY(hipGraphExecKernelNodeSetParams(cg->exec, cg->near_node, &kp));
  }
  HIP_TRY(hipGraphLaunch(cg->exec, st));
  return SLP_OK;
}

int begin_timed(slp_geom *G, hipStream_t st);

// One evaluation of nb items on the context's buffers: replayed graph or
// direct launches (the latter also record the sampled stage events).
template <typename T>
int eval_items(slp_geom *G, const slp::BatchPtrs &ptrs, int nb, hipStream_t st) {
  if (G->use_graph) return run_graph<T>(G, ptrs, nb, st);
  const bool tm = G->timing && (G->evals++ % G->every == 0);
  if (tm) {
    const int rc = begin_timed(G, st);
    if (rc) return rc;
  }
  return run_eval<T>(G, ctx_work(G), ptrs, nb, st, tm);
}

int collect_one(slp_geom *G, int r) {
  if (!G->used[r]) return SLP_OK;
  HIP_TRY(hipEventSynchronize(G->ev[r][slp_geom::kStages]));
  // without a near field, event 8 is not recorded: the interpolation ends at
  // the last event and the near-field stage takes no time
  const int last = G->with_near[r] ? slp_geom::kStages : slp_geom::kStages - 1;
  for (int i = 0; i < last; ++i) {
    float ms = 0.f;
    const int to = (i + 1 == last) ? slp_geom::kStages : i + 1;
    HIP_TRY(hipEventElapsedTime(&ms, G->ev[r][i], G->ev[r][to]));
    G->acc_ms[i] += ms;
  }
  G->count += 1;
  G->used[r] = false;
  return SLP_OK;
}

// Accumulate every recorded evaluation (synchronises with the newest one).
int collect_timing(slp_geom *G) {
  for (int k = 0; k < slp_geom::kRing; ++k) {
    int rc = collect_one(G, (G->cur + k) % slp_geom::kRing);
    if (rc) return rc;
  }
  return SLP_OK;
}

int ensure_events(slp_geom *G) {
  if (G->ev_ready) return SLP_OK;
  for (auto &set : G->ev)
    for (auto &e : set) HIP_TRY(hipEventCreate(&e));
  G->ev_ready = true;
  return SLP_OK;
}

// Start the event set of the next evaluation: the oldest set in the ring is
// read back first if it is still pending (long completed in steady state).
int begin_timed(slp_geom *G, hipStream_t st) {
  int rc = ensure_events(G);
  if (!rc) rc = collect_one(G, G->cur);
  if (rc) return rc;
  HIP_TRY(hipEventRecord(G->evs()[0], st));
  return SLP_OK;
}

}  // namespace

int64_t slp::item_device_bytes(const slp_geom *G) {
  const int64_t e = (int64_t)G->esz();
  const int64_t per[5] = {e, e, 2 * e, 2 * e, e};
  int64_t b = 0;
  for (int i = 0; i < 5; ++i) b += G->item_elems[i] * per[i];
  if (G->nf_gbar) b += G->n_tris * 8;
  if (G->iw_gbar) b += G->n_tris * 8;
  return b;
}

int slp::reserve_items(slp_geom *G, int nb, hipStream_t st) {
  if (!G || nb < 1 || nb > slp::kMaxBatch) return fail(SLP_EINVAL, "reserve_items: bad arguments");
  return ensure_capacity(G, nb, st);
}

void slp::destroy_idle(slp_geom *G) { delete G; }

extern "C" {

const char *slp_last_error(void) { return g_err.c_str(); }

int slp_expsum_sinc(double h, double r_lo, double r_hi, double tol, double *omega, double *gamma,
                    int32_t cap, int32_t *count) {
  if (!(h > 0) || !(r_lo > 0) || !(r_hi > r_lo) || !(tol > 0) || !count)
    return fail(SLP_EINVAL, "expsum: need h > 0, 0 < r_lo < r_hi, tol > 0, count != NULL");
  const double sqrt_pi = std::sqrt(3.141592653589793238462643383279502884);
  const double u_hi = std::log(7.0 / r_lo);
  const double u_lo = std::log(tol * sqrt_pi / (2.0 * r_hi));
  const int32_t n = (int32_t)std::floor((u_hi - u_lo) / h) + 1;
  *count = n;
  if (n > cap || !omega || !gamma) return fail(SLP_EINVAL, "expsum: capacity %d < %d terms", cap, n);
  for (int32_t t = 0; t < n; ++t) {
    const double u = u_lo + h * t;
    omega[t] = (2.0 / sqrt_pi) * h * std::exp(u);
    gamma[t] = std::exp(2.0 * u);
  }
  return SLP_OK;
}

namespace {

// Setup phase. With dry_bytes != NULL only the host part runs and the device
// bytes the context would hold are returned (no device call is made).
int setup_impl(slp_geom **out, const double *nodes, int64_t n_nodes, const int32_t *tris,
               int64_t n_tris, const double *targets, int64_t n_tgt, const slp_params *p,
               void *stream, int64_t *dry_bytes) {
  if (!out && !dry_bytes) return fail(SLP_EINVAL, "out is NULL");
  if (out) *out = nullptr;
  int rc = validate_params(p);
  if (rc) return rc;
  if (!nodes || !tris || n_nodes < 3 || n_tris < 1)
    return fail(SLP_EINVAL, "need >= 3 nodes and >= 1 triangle");
  if (!targets) {
    targets = nodes;
    n_tgt = n_nodes;
  }
  if (n_tgt < 1) return fail(SLP_EINVAL, "need >= 1 target point");
  if (3 * n_tris > (int64_t)std::numeric_limits<int32_t>::max() ||
      n_nodes > (int64_t)std::numeric_limits<int32_t>::max() ||
      n_tgt > (int64_t)std::numeric_limits<int32_t>::max())
    return fail(SLP_EINVAL, "mesh too large for 32-bit indices");
  for (int64_t i = 0; i < 3 * n_tgt; ++i)
    if (!std::isfinite(targets[i]))
      return fail(SLP_EINVAL, "target %lld has a non-finite coordinate", (long long)(i / 3));
  hipStream_t st = static_cast<hipStream_t>(stream);

  // bounding box, scaling into (-0.2, 0.2)^3 with s_q N_q equal on every axis
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < n_nodes; ++i)
    for (int q = 0; q < 3; ++q) {
      const double v = nodes[3 * i + q];
      if (!std::isfinite(v)) return fail(SLP_EINVAL, "node %lld has a non-finite coordinate", (long long)i);
      lo[q] = std::min(lo[q], v);
      hi[q] = std::max(hi[q], v);
    }
  for (int64_t j = 0; j < 3 * n_tris; ++j)
    if (tris[j] < 0 || tris[j] >= n_nodes)
      return fail(SLP_EINVAL, "triangle %lld references node %d out of range", (long long)(j / 3), tris[j]);

  slp_geom *G = new (std::nothrow) slp_geom();
  if (!G) return fail(SLP_ENOMEM, "host allocation failed");
  struct Guard {
    slp_geom *g;
    ~Guard() { delete g; }
  } guard{G};

  G->prec = p->precision;
  G->alpha = p->alpha;
  G->m = p->m;
  {
    const double pi = 3.141592653589793238462643383279502884;
    G->window = p->window;
    if (p->window == SLP_WINDOW_GAUSS) {
      G->b = 2.0 * p->alpha * p->m / ((2.0 * p->alpha - 1.0) * pi);
    } else {
      G->b = pi * (2.0 - 1.0 / p->alpha);
      G->kb_inv_norm = p->m / std::sinh(G->b * p->m);
      G->kb_coef = kb_polynomials(p->m, G->b, G->kb_inv_norm,
                                  slp::kb_degree(p->precision == SLP_FP64, p->m));
    }
  }
  G->n_nodes = n_nodes;
  G->n_tgt = n_tgt;
  G->n_tris = n_tris;
  G->n_src = 3 * n_tris;
  double Kmin = INFINITY;
  for (int q = 0; q < 3; ++q) {
    G->N[q] = p->grid[q];
    G->n[q] = p->grid[q] / p->alpha;
    G->c[q] = 0.5 * (lo[q] + hi[q]);
    const double ext = hi[q] - lo[q];
    if (ext > 0) Kmin = std::min(Kmin, 0.4 * G->N[q] / ext);
  }
  if (!std::isfinite(Kmin)) return fail(SLP_EINVAL, "all nodes coincide");
  for (int q = 0; q < 3; ++q) G->s[q] = Kmin / G->N[q];

  // quadrature sources (k = j + s M) and grid-unit coordinates t = (x~ + 1/2) N
  const int64_t M = n_tris, Ms = G->n_src;
  std::vector<double> ts(3 * Ms), wsrc(Ms), tt(3 * n_tgt), tnrm(3 * M);
  std::vector<int32_t> tv(3 * M);
  const double bary[3][3] = {{4.0 / 6, 1.0 / 6, 1.0 / 6}, {1.0 / 6, 4.0 / 6, 1.0 / 6}, {1.0 / 6, 1.0 / 6, 4.0 / 6}};
  for (int64_t j = 0; j < M; ++j) {
    const double *P0 = nodes + 3 * (int64_t)tris[3 * j];
    const double *P1 = nodes + 3 * (int64_t)tris[3 * j + 1];
    const double *P2 = nodes + 3 * (int64_t)tris[3 * j + 2];
    double e1[3], e2[3];
    for (int q = 0; q < 3; ++q) { e1[q] = P1[q] - P0[q]; e2[q] = P2[q] - P0[q]; }
    const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double area = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    if (!(area > 0.0)) return fail(SLP_EINVAL, "triangle %lld is degenerate", (long long)j);
    for (int q = 0; q < 3; ++q) {
      tnrm[q * M + j] = cr[q] / (2.0 * area);
      tv[q * M + j] = tris[3 * j + q];
    }
    for (int s = 0; s < 3; ++s) {
      const int64_t k = j + s * M;
      wsrc[k] = area / 3.0;
      for (int q = 0; q < 3; ++q) {
        const double y = bary[s][0] * P0[q] + bary[s][1] * P1[q] + bary[s][2] * P2[q];
        ts[3 * k + q] = ((y - G->c[q]) * G->s[q] + 0.5) * G->N[q];
      }
    }
  }
  for (int64_t i = 0; i < n_tgt; ++i)
    for (int q = 0; q < 3; ++q)
      tt[3 * i + q] = ((targets[3 * i + q] - G->c[q]) * G->s[q] + 0.5) * G->N[q];

  // region touched by any stencil {floor(t) - m + 1 .. floor(t) + m}
  int64_t cmin[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, cmax[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  auto upd = [&](const std::vector<double> &t, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
      for (int q = 0; q < 3; ++q) {
        const int64_t f = (int64_t)std::floor(t[3 * i + q]);
        cmin[q] = std::min(cmin[q], f);
        cmax[q] = std::max(cmax[q], f);
      }
  };
  upd(ts, Ms);
  upd(tt, n_tgt);
  for (int q = 0; q < 3; ++q) {
    const int64_t rlo = cmin[q] - G->m + 1, rhi = cmax[q] + G->m;
    if (rlo < 0 || rhi > G->N[q] - 1)
      return fail(SLP_EINVAL, "axis %d: stencils reach [%lld, %lld] outside the grid [0, %d): "
                  "m = %d is too large for grid %d", q, (long long)rlo, (long long)rhi, G->N[q], G->m, G->N[q]);
    G->lo[q] = (int32_t)rlo;
    G->R[q] = (int32_t)(rhi - rlo + 1);
    G->tiles[q] = (G->R[q] + kTile - 1) / kTile;
    G->P[q] = G->tiles[q] * kTile;
  }
  G->K[0] = G->n[0] / 2 + 1;
  G->K[1] = G->n[1] + 1;
  G->K[2] = G->n[2] + 1;

  // exponential-sum truncation (keep the terms the grid resolves)
  std::vector<double> om, gam;
  for (int t = 0; t < p->es_terms; ++t) {
    bool keep = true;
    for (int q = 0; q < 3; ++q) {
      const double lim = std::pow(3.141592653589793238462643383279502884 * G->n[q] / 2.0, 2) / p->eta2;
      if (p->es_gamma[t] / (G->s[q] * G->s[q]) > lim) keep = false;
    }
    if (keep) { om.push_back(p->es_w[t]); gam.push_back(p->es_gamma[t]); }
  }
  if (om.empty()) return fail(SLP_EINVAL, "no exponential-sum term is resolved by the grid");
  G->terms_kept = (int32_t)om.size();
  G->kept_w = om;
  G->kept_g = gam;

  // binning: sources by (tile, cell in tile), targets by tile
  const int64_t ntiles = (int64_t)G->tiles[0] * G->tiles[1] * G->tiles[2];
  auto cell_key = [&](const double *t, int32_t *tile, int32_t *incell) {
    int32_t id[3], in[3];
    for (int q = 0; q < 3; ++q) {
      const int32_t c = (int32_t)std::floor(t[q]) - G->lo[q];
      id[q] = c / kTile;
      in[q] = c % kTile;
    }
    *tile = id[0] + G->tiles[0] * (id[1] + G->tiles[1] * id[2]);
    *incell = in[0] | (in[1] << 4) | (in[2] << 8);
  };
  std::vector<int32_t> skey(Ms), sincell(Ms), tbin(n_tgt), sorder, sstart, torder, tstart;
  for (int64_t k = 0; k < Ms; ++k) {
    int32_t tile, inc;
    cell_key(&ts[3 * k], &tile, &inc);
    sincell[k] = inc;
    skey[k] = tile * 512 + ((inc & 7) + 8 * ((inc >> 4) & 7) + 64 * (inc >> 8));
  }
  // targets by (tile, cell in tile): the targets of one cell are consecutive,
  // so that the interpolation can read their shared stencil rows once
  for (int64_t i = 0; i < n_tgt; ++i) {
    int32_t tile, inc;
    cell_key(&tt[3 * i], &tile, &inc);
    tbin[i] = tile * 512 + ((inc & 7) + 8 * ((inc >> 4) & 7) + 64 * (inc >> 8));
  }
  counting_sort(skey, ntiles * 512, sorder, sstart);
  {
    std::vector<int32_t> cstart;
    counting_sort(tbin, ntiles * 512, torder, cstart);
    tstart.resize(ntiles + 1);
    for (int64_t t = 0; t <= ntiles; ++t) tstart[t] = cstart[t * 512];
  }
  std::vector<double> wsorted(Ms);
  for (int64_t i = 0; i < Ms; ++i) wsorted[i] = wsrc[sorder[i]];

  // segments: the sources of one tile, cut into equal pieces where a tile holds
  // more than 1.5x the average share of one workgroup slot of the chip (every
  // CU holding as many gridding workgroups as its LDS allows). Each segment is
  // cut into chunks of <= spread_chunk(fp64, m) sources and runs of sources sharing one
  // cell. (At least max(64, (8 + 2m - 1)^3 / 20) sources per share, / 80 for the
  // matrix-core form, so that
  // small problems do not pay more for storing and summing blocks than for
  // gridding.)
  const int per_cu = slp::spread_units_per_cu(G->m, G->prec == SLP_FP64);
  // The matrix-core form (FP64, 2m = 16) grids a source several times faster
  // than the vector form, so its pieces pay off down to fewer sources: timed
  // splits of icospheres of 1.5e4 and 6.1e4 sources ran 19% and 9% faster at
  // about 150 sources per piece than at the vector form's floor.
  const bool mx = G->prec == SLP_FP64 && G->m == 8;
  const int64_t min_src = std::max<int64_t>(64, slp::pad_cells(G->m) / (mx ? 80 : 20));
  const int64_t max_units = std::max<int64_t>(
      1, std::min<int64_t>((int64_t)slp::kComputeUnits * per_cu, Ms / min_src));
  // (a share below ~300 sources (150 for the matrix-core form) makes storing and
  // summing the extra blocks cost more than the better balance gains, measured
  // on MI355X for m = 4..8)
  const int64_t share = p->seg_share > 0
                            ? (int64_t)p->seg_share
                            : std::max<int64_t>(mx ? 150 : 300, (Ms + max_units - 1) / max_units);
  G->share = share;
  G->reduce_cells = p->reduce_cells;
  std::vector<int4> segs, chunks;
  std::vector<int32_t> runs;
  std::vector<int64_t> seg_size;
  {
    const int CH = slp::spread_chunk(p->precision == SLP_FP64, p->m);
    // a chunk's runs longest first: the vector form processes several runs of a
    // wave side by side, for as many steps as the longest of them
    auto close_chunk = [&](const int4 &c) {
      std::stable_sort(runs.begin() + c.z, runs.begin() + c.z + c.w, [](int32_t x, int32_t y) {
        return ((x >> 19) & 2047) > ((y >> 19) & 2047);
      });
      chunks.push_back(c);
    };
    int64_t i = 0;
    while (i < Ms) {
      const int32_t tile = skey[sorder[i]] / 512;
      int64_t te = i;
      while (te < Ms && skey[sorder[te]] / 512 == tile) ++te;
      const int64_t n = te - i;
      const int64_t pieces = n * 2 > share * 3 ? (n + share - 1) / share : 1;
      for (int64_t pc = 0; pc < pieces; ++pc) {
        const int64_t pb = i + n * pc / pieces, pe = i + n * (pc + 1) / pieces;
        int4 sg = {(int)chunks.size(), 0, tile, 0};
        int4 cur = {(int)pb, 0, (int)runs.size(), 0};
        int64_t k = pb;
        while (k < pe) {
          const int32_t key = skey[sorder[k]];
          int64_t e = k;
          while (e < pe && skey[sorder[e]] == key) ++e;
          const int32_t inc = sincell[sorder[k]];
          const int32_t cell = (inc & 7) | (((inc >> 4) & 7) << 3) | ((inc >> 8) << 6);
          int64_t pos = k;
          while (pos < e) {
            if (cur.y == CH) {
              close_chunk(cur);
              cur = {(int)pos, 0, (int)runs.size(), 0};
            }
            const int take = (int)std::min<int64_t>(e - pos, CH - cur.y);
            runs.push_back(cell | (cur.y << 9) | (take << 19));
            cur.y += take;
            cur.w += 1;
            pos += take;
          }
          k = e;
        }
        close_chunk(cur);
        sg.y = (int)chunks.size();
        segs.push_back(sg);
        seg_size.push_back(pe - pb);
      }
      i = te;
    }
  }
  // one workgroup per segment, longest first: the hardware hands out
  // workgroups in launch order to whichever CU frees up, which balances the
  // actual run times better than any static packing by source count
  const int64_t n_units = (int64_t)segs.size();
  // pad cells of a tile's padded block that its sources reach: per axis from
  // the lowest source cell (in the tile) to the highest plus 2m - 1, packed
  // lo x | y << 5 | z << 10, hi << 15 | << 20 | << 25; the blocks of that tile
  // store, and the sum reads, only that box
  std::vector<int32_t> tile_box(ntiles, 0);
  {
    const int w1 = 2 * G->m - 1;
    std::vector<int4> tlo(ntiles, int4{7, 7, 7, 0}), thi(ntiles, int4{0, 0, 0, 0});
    for (const int4 &sg : segs) {
      int4 &lo = tlo[sg.z], &hi = thi[sg.z];
      for (int c = sg.x; c < sg.y; ++c)
        for (int r = 0; r < chunks[c].w; ++r) {
          const int32_t rec = runs[chunks[c].z + r];
          const int x = rec & 7, y = (rec >> 3) & 7, z = (rec >> 6) & 7;
          lo.x = std::min(lo.x, x); lo.y = std::min(lo.y, y); lo.z = std::min(lo.z, z);
          hi.x = std::max(hi.x, x); hi.y = std::max(hi.y, y); hi.z = std::max(hi.z, z);
        }
    }
    for (const int4 &sg : segs) {
      const int4 lo = tlo[sg.z], hi = thi[sg.z];
      tile_box[sg.z] = lo.x | (lo.y << 5) | (lo.z << 10) | ((hi.x + w1) << 15) |
                        ((hi.y + w1) << 20) | ((hi.z + w1) << 25);
    }
  }
  // unit u: {slot, first chunk, end chunk, tile's reach box} and the
  // first chunk's record
  std::vector<int4> units(2 * n_units);
  {
    std::vector<int32_t> order(segs.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int32_t)k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return seg_size[a] > seg_size[b]; });
    for (int64_t u = 0; u < n_units; ++u) {
      const int4 sg = segs[order[u]];
      units[2 * u] = {order[u], sg.x, sg.y, tile_box[sg.z]};
      units[2 * u + 1] = chunks[sg.x];
    }
  }
  // consistency of the tables the gridding kernel indexes with (cheap, host side)
  {
    int64_t next_src = 0;
    bool ok = true;
    std::vector<char> seen(segs.size(), 0);
    for (int64_t u = 0; ok && u < n_units; ++u) {
      const int4 un = units[2 * u], c0 = units[2 * u + 1];
      ok = un.x >= 0 && un.x < (int32_t)segs.size() && !seen[un.x] && un.y == segs[un.x].x &&
           un.z == segs[un.x].y && un.w == tile_box[segs[un.x].z] && c0.x == chunks[un.y].x &&
           c0.y == chunks[un.y].y && c0.z == chunks[un.y].z && c0.w == chunks[un.y].w;
      if (ok) seen[un.x] = 1;
    }
    for (size_t sgi = 0; ok && sgi < segs.size(); ++sgi) {
      const int4 sg = segs[sgi];
      ok = sg.x < sg.y && sg.z >= 0 && sg.z < ntiles;
      for (int c = sg.x; ok && c < sg.y; ++c) {
        const int4 ch = chunks[c];
        const int CH = slp::spread_chunk(G->prec == SLP_FP64, G->m);
        ok = ch.x == next_src && ch.y >= 1 && ch.y <= CH && ch.w >= 1 && ch.w <= CH &&
             ch.z + ch.w <= (int)runs.size();
        // the chunk's runs (in any order) cover its sources exactly once
        std::vector<std::pair<int, int>> span;
        for (int r = 0; ok && r < ch.w; ++r) {
          const int32_t rec = runs[ch.z + r];
          const int off = (rec >> 9) & 1023, cnt = (rec >> 19) & 2047;
          ok = cnt >= 1 && off + cnt <= ch.y;
          for (int k = 0; ok && k < cnt; ++k) {
            const int32_t key = skey[sorder[ch.x + off + k]];
            const int32_t cl = key % 512;
            ok = key / 512 == sg.z && (rec & 511) == cl;
          }
          span.emplace_back(off, cnt);
        }
        std::sort(span.begin(), span.end());
        int expect_off = 0;
        for (size_t r = 0; ok && r < span.size(); ++r) {
          ok = span[r].first == expect_off;
          expect_off += span[r].second;
        }
        ok = ok && expect_off == ch.y;
        next_src += ch.y;
      }
    }
    if (!ok || next_src != Ms) return fail(SLP_EDEVICE, "internal error: gridding tables inconsistent");
  }
  // the segments of one tile are consecutive (sources sorted by tile)
  std::vector<int4> tile_slots(ntiles, int4{0, 0, 0, 0});
  for (size_t sgi = 0; sgi < segs.size(); ++sgi) {
    int4 &slot = tile_slots[segs[sgi].z];
    if (slot.y == 0) slot.x = (int)sgi;
    slot.y += 1;
    slot.z = tile_box[segs[sgi].z];
  }
  G->n_units = (int32_t)n_units;
  G->n_slots = (int32_t)segs.size();
  G->unit_len.resize(n_units);
  for (int64_t u = 0; u < n_units; ++u) G->unit_len[u] = (int32_t)seg_size[units[2 * u].x];
  std::vector<int32_t> tgt_active;
  for (int64_t t = 0; t < ntiles; ++t)
    if (tstart[t + 1] > tstart[t]) tgt_active.push_back((int32_t)t);
  std::stable_sort(tgt_active.begin(), tgt_active.end(), [&](int32_t a, int32_t b) {
    return tstart[a + 1] - tstart[a] > tstart[b + 1] - tstart[b];
  });
  G->n_tgt_tiles = (int32_t)tgt_active.size();
  G->tgt_len.resize(tgt_active.size());
  for (size_t k = 0; k < tgt_active.size(); ++k)
    G->tgt_len[k] = tstart[tgt_active[k] + 1] - tstart[tgt_active[k]];
  // per tile the bounding box of its targets' cells (3 bits per bound): the
  // interpolation stages only the grid values their stencils reach
  std::vector<int32_t> tgt_box(ntiles, 0);
  {
    std::vector<int32_t> blo(3 * ntiles, 7), bhi(3 * ntiles, 0);
    for (int64_t i = 0; i < n_tgt; ++i) {
      const int64_t t = tbin[i] / 512;
      const int c = tbin[i] % 512;
      const int in[3] = {c & 7, (c >> 3) & 7, c >> 6};
      for (int q = 0; q < 3; ++q) {
        blo[3 * t + q] = std::min(blo[3 * t + q], in[q]);
        bhi[3 * t + q] = std::max(bhi[3 * t + q], in[q]);
      }
    }
    for (int64_t t = 0; t < ntiles; ++t)
      if (tstart[t + 1] > tstart[t])
        tgt_box[t] = blo[3 * t] | blo[3 * t + 1] << 3 | blo[3 * t + 2] << 6 | bhi[3 * t] << 9 |
                     bhi[3 * t + 1] << 12 | bhi[3 * t + 2] << 15;
  }
  // one record per active tile (a single load at the start of its workgroup)
  std::vector<int4> tgt_rec(tgt_active.size());
  for (size_t k = 0; k < tgt_active.size(); ++k) {
    const int32_t t = tgt_active[k];
    tgt_rec[k] = int4{t, tstart[t], tstart[t + 1], tgt_box[t]};
  }

  // device allocations
  const size_t e = G->esz();
  const int64_t Gsz = (int64_t)G->P[0] * G->P[1] * G->P[2];
  const int64_t S1n = (int64_t)G->R[2] * G->R[1] * G->K[0];
  const int64_t S2n = (int64_t)G->R[2] * G->K[1] * G->K[0];
  const int64_t gn = (int64_t)G->R[0] * G->R[1] * G->R[2];
  const int64_t mun = (int64_t)(G->n[0] / 2 + 1) * (G->n[1] / 2 + 1) * (G->n[2] / 2 + 1);
  G->item_elems[0] = (int64_t)G->n_slots * slp::pad_cells(G->m);
  G->item_elems[1] = Gsz;
  G->item_elems[2] = S1n;
  G->item_elems[3] = S2n;
  G->item_elems[4] = gn;
  struct AllocReq {
    void **dst;
    size_t bytes;
  };
  const AllocReq reqs[] = {
      {&G->src_frac, (size_t)(3 * Ms) * e},
      {reinterpret_cast<void **>(&G->src_w), (size_t)Ms * 8},
      {reinterpret_cast<void **>(&G->src_perm), (size_t)Ms * 4},
      {reinterpret_cast<void **>(&G->units), units.size() * sizeof(int4)},
      {reinterpret_cast<void **>(&G->chunks), chunks.size() * sizeof(int4)},
      {reinterpret_cast<void **>(&G->runs), runs.size() * sizeof(int32_t)},
      {reinterpret_cast<void **>(&G->tile_slots), (size_t)ntiles * sizeof(int4)},
      {&G->scratch, (size_t)G->n_slots * (size_t)slp::pad_cells(G->m) * e},
      {reinterpret_cast<void **>(&G->tgt_rec), tgt_rec.size() * sizeof(int4)},
      {&G->kb_tab, (size_t)slp::kKbCoef * e},
      {reinterpret_cast<void **>(&G->tgt_cell), (size_t)(3 * n_tgt) * 4},
      {&G->tgt_frac, (size_t)(3 * n_tgt) * e},
      {reinterpret_cast<void **>(&G->tgt_perm), (size_t)n_tgt * 4},
      {&G->grid_a, (size_t)Gsz * e},
      {&G->S1, (size_t)S1n * 2 * e},
      {&G->S2, (size_t)S2n * 2 * e},
      {&G->grid_g, (size_t)gn * e},
      {&G->mu, (size_t)mun * e},
      {&G->tw[0], (size_t)G->N[0] * 2 * e},
      {&G->tw[1], (size_t)G->N[1] * 2 * e},
      {&G->tw[2], (size_t)G->N[2] * 2 * e},
      {reinterpret_cast<void **>(&G->tri_v), (size_t)(3 * M) * 4},
      {reinterpret_cast<void **>(&G->tri_n), (size_t)(3 * M) * 8},
      {reinterpret_cast<void **>(&G->own_dens), (size_t)(3 * M) * 8},
  };
  if (dry_bytes) {
    int64_t tot = 0;
    for (const AllocReq &r : reqs) tot += (int64_t)std::max<size_t>(r.bytes, slp_geom::kMinAlloc);
    *dry_bytes = tot;
    return SLP_OK;
  }
  bool ok = true;
  for (const AllocReq &r : reqs) ok = ok && G->alloc(r.dst, r.bytes) == hipSuccess;
  if (!ok) return fail(SLP_ENOMEM, "device allocation failed (%lld bytes so far)", (long long)G->bytes);
  try {
    G->h_nodes.assign(nodes, nodes + 3 * n_nodes);
    G->h_tris.assign(tris, tris + 3 * n_tris);
    G->h_tgt.assign(targets, targets + 3 * n_tgt);
  } catch (const std::bad_alloc &) {
    return fail(SLP_ENOMEM, "host copy of the geometry failed");
  }
  {
    double blo[3], bhi[3];
    for (int q = 0; q < 3; ++q) { blo[q] = lo[q]; bhi[q] = hi[q]; }
    for (int64_t i = 0; i < n_tgt; ++i)
      for (int q = 0; q < 3; ++q) {
        blo[q] = std::min(blo[q], targets[3 * i + q]);
        bhi[q] = std::max(bhi[q], targets[3 * i + q]);
      }
    double d2 = 0.0;
    for (int q = 0; q < 3; ++q) d2 += (bhi[q] - blo[q]) * (bhi[q] - blo[q]);
    G->r_max = std::sqrt(d2);
  }

  HIP_TRY(hipMemcpyAsync(G->src_w, wsorted.data(), Ms * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->src_perm, sorder.data(), Ms * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->units, units.data(), units.size() * sizeof(int4), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->chunks, chunks.data(), chunks.size() * sizeof(int4), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->runs, runs.data(), runs.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->tile_slots, tile_slots.data(), (size_t)ntiles * sizeof(int4), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->tgt_rec, tgt_rec.data(), tgt_rec.size() * sizeof(int4), hipMemcpyHostToDevice, st));
  std::vector<float> kbt32(slp::kKbCoef);
  for (int i = 0; i < slp::kKbCoef; ++i) kbt32[i] = (float)G->kb_coef[i];
  if (G->prec == SLP_FP64)
    HIP_TRY(hipMemcpyAsync(G->kb_tab, G->kb_coef.data(), slp::kKbCoef * 8, hipMemcpyHostToDevice, st));
  else
    HIP_TRY(hipMemcpyAsync(G->kb_tab, kbt32.data(), slp::kKbCoef * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->tgt_perm, torder.data(), n_tgt * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->tri_v, tv.data(), tv.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->tri_n, tnrm.data(), tnrm.size() * 8, hipMemcpyHostToDevice, st));
  std::vector<int32_t> cs, ct;
  std::vector<double> fs64, ft64;
  std::vector<float> fs32, ft32;
  std::vector<std::vector<double>> tw64;
  std::vector<std::vector<float>> tw32;
  if (G->prec == SLP_FP64) {
    rc = upload_tables<double>(G, ts, sorder, tt, torder, st, cs, fs64, ct, ft64);
    if (!rc) rc = upload_twiddles<double>(G, st, tw64);
  } else {
    rc = upload_tables<float>(G, ts, sorder, tt, torder, st, cs, fs32, ct, ft32);
    if (!rc) rc = upload_twiddles<float>(G, st, tw32);
  }
  if (rc) return rc;

  // kernel Fourier coefficients (FP64) and the multiplier table
  {
    std::vector<double> glx, glw;
    const int order = 16;
    gauss_legendre(order, glx, glw);
    const int S = G->terms_kept;
    double *d_gl = nullptr, *d_om = nullptr, *d_gam = nullptr, *d_C[3] = {nullptr, nullptr, nullptr};
    std::vector<void *> tmps;
    auto talloc = [&](double **ptr, size_t n) {
      hipError_t er = hipMalloc((void **)ptr, n * sizeof(double));
      if (er == hipSuccess) tmps.push_back(*ptr);
      return er;
    };
    struct TmpGuard {
      std::vector<void *> &v;
      ~TmpGuard() { for (void *x : v) (void)hipFree(x); }
    } tguard{tmps};
    int L[3];
    for (int q = 0; q < 3; ++q) L[q] = G->n[q] / 2 + 1;
    if (talloc(&d_gl, 2 * order) != hipSuccess || talloc(&d_om, S) != hipSuccess ||
        talloc(&d_gam, 3 * (size_t)S) != hipSuccess || talloc(&d_C[0], (size_t)S * L[0]) != hipSuccess ||
        talloc(&d_C[1], (size_t)S * L[1]) != hipSuccess || talloc(&d_C[2], (size_t)S * L[2]) != hipSuccess)
      return fail(SLP_ENOMEM, "device allocation for kernel tables failed");
    std::vector<double> gl(2 * order), gsc(3 * (size_t)S);
    std::vector<double> dec_host[3];
    for (int j = 0; j < order; ++j) { gl[j] = glx[j]; gl[order + j] = glw[j]; }
    for (int q = 0; q < 3; ++q)
      for (int t = 0; t < S; ++t) gsc[(size_t)q * S + t] = gam[t] / (G->s[q] * G->s[q]);
    HIP_TRY(hipMemcpyAsync(d_gl, gl.data(), gl.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_om, om.data(), om.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_gam, gsc.data(), gsc.size() * 8, hipMemcpyHostToDevice, st));
    for (int q = 0; q < 3; ++q) {
      const int panels = std::max(G->n[q] / 2 + 8, 16);
      HIP_TRY(slp::launch_chat(d_C[q], d_gam + (size_t)q * S, S, L[q], d_gl, d_gl + order, order, panels, st));
    }
    // per-axis deconvolution factors 1 / u^(l / N)^2 of the window the kernels
    // evaluate (u^ its Fourier transform in grid units): Gaussian exp(-tau^2 / b)
    // -> sqrt(pi b) exp(-pi^2 b w^2); Kaiser-Bessel sinh(b s) / s * inv_norm ->
    // pi inv_norm I_0(m sqrt(b^2 - (2 pi w)^2)) (eq. cFB)
    double *d_dec[3] = {nullptr, nullptr, nullptr};
    for (int q = 0; q < 3; ++q) {
      if (talloc(&d_dec[q], L[q]) != hipSuccess)
        return fail(SLP_ENOMEM, "device allocation for kernel tables failed");
      const double pi = 3.141592653589793238462643383279502884;
      std::vector<double> &dec = dec_host[q];
      dec.resize(L[q]);
      for (int l = 0; l < L[q]; ++l) {
        const double w = (double)l / G->N[q];
        double uhat;
        if (G->window == SLP_WINDOW_GAUSS)
          uhat = std::sqrt(pi * G->b) * std::exp(-pi * pi * G->b * w * w);
        else
          uhat = pi * G->kb_inv_norm *
                 std::cyl_bessel_i(0.0, G->m * std::sqrt(G->b * G->b - 4.0 * pi * pi * w * w));
        dec[l] = 1.0 / (uhat * uhat);
      }
      HIP_TRY(hipMemcpyAsync(d_dec[q], dec.data(), dec.size() * 8, hipMemcpyHostToDevice, st));
    }
    if (G->prec == SLP_FP64)
      HIP_TRY(slp::launch_mu<double>((double *)G->mu, d_C[0], d_C[1], d_C[2], d_om, S, G->n,
                                     d_dec[0], d_dec[1], d_dec[2], st));
    else
      HIP_TRY(slp::launch_mu<float>((float *)G->mu, d_C[0], d_C[1], d_C[2], d_om, S, G->n,
                                    d_dec[0], d_dec[1], d_dec[2], st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  guard.g = nullptr;
  *out = G;
  return SLP_OK;
}

}  // namespace

int slp_setup_geometry(slp_geom **out, const double *nodes, int64_t n_nodes, const int32_t *tris,
                       int64_t n_tris, const slp_params *p, void *stream) {
  return setup_impl(out, nodes, n_nodes, tris, n_tris, nullptr, 0, p, stream, nullptr);
}

int slp_setup_geometry_targets(slp_geom **out, const double *nodes, int64_t n_nodes,
                               const int32_t *tris, int64_t n_tris, const double *targets,
                               int64_t n_targets, const slp_params *p, void *stream) {
  if (!targets) return fail(SLP_EINVAL, "targets is NULL");
  return setup_impl(out, nodes, n_nodes, tris, n_tris, targets, n_targets, p, stream, nullptr);
}

int slp_geometry_device_bytes(const double *nodes, int64_t n_nodes, const int32_t *tris,
                              int64_t n_tris, const slp_params *p, int64_t *bytes) {
  if (!bytes) return fail(SLP_EINVAL, "bytes is NULL");
  return setup_impl(nullptr, nodes, n_nodes, tris, n_tris, nullptr, 0, p, nullptr, bytes);
}

int slp_set_density(slp_geom *G, const double *dens, void *stream) {
  if (!G || !dens) return fail(SLP_EINVAL, "geometry and density must be non-NULL");
  (void)stream;
  G->dens = dens;
  return SLP_OK;
}

int slp_set_density_from_m(slp_geom *G, const double *m_nodes, const double *dphi1_dn,
                           void *stream) {
  if (!G || !m_nodes) return fail(SLP_EINVAL, "geometry and m_nodes must be non-NULL");
  HIP_TRY(slp::launch_density_from_m(G->tri_v, G->tri_n, m_nodes, dphi1_dn, G->n_tris,
                                     G->own_dens, static_cast<hipStream_t>(stream)));
  G->dens = G->own_dens;
  return SLP_OK;
}

int slp_eval_single_layer(slp_geom *G, double *phi, void *stream) {
  if (!G || !phi) return fail(SLP_EINVAL, "geometry and phi must be non-NULL");
  if (!G->dens) return fail(SLP_EINVAL, "no density set (slp_set_density)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  slp::BatchPtrs ptrs{};
  ptrs.dens[0] = G->dens;
  ptrs.phi[0] = phi;
  return G->prec == SLP_FP64 ? eval_items<double>(G, ptrs, 1, st)
                             : eval_items<float>(G, ptrs, 1, st);
}

namespace {

// Streams on which the launch groups of different geometries of one batched
// call overlap (per device, created on first use, default priority).
constexpr int kLanes = 4;
struct Lanes {
  hipStream_t s[kLanes]{};
  hipEvent_t fork{};
  hipEvent_t join[kLanes]{};
};
std::mutex g_lanes_mu;              // guards the table and every fork/join section
std::map<int, Lanes> g_lanes;

int get_lanes(Lanes **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  auto it = g_lanes.find(dev);
  if (it == g_lanes.end()) {
    Lanes L;
    for (int i = 0; i < kLanes; ++i) {
      HIP_TRY(hipStreamCreateWithFlags(&L.s[i], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&L.join[i], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&L.fork, hipEventDisableTiming));
    it = g_lanes.emplace(dev, L).first;
  }
  *out = &it->second;
  return SLP_OK;
}

// One launch group: consecutive items of one geometry (at most kMaxBatch).
int run_group(slp_geom *G, const double *const *dens, double *const *phi, int nb, hipStream_t st) {
  int rc = ensure_capacity(G, nb, st);
  if (rc) return rc;
  slp::BatchPtrs ptrs{};
  for (int i = 0; i < nb; ++i) {
    ptrs.dens[i] = dens[i];
    ptrs.phi[i] = phi[i];
  }
  return G->prec == SLP_FP64 ? eval_items<double>(G, ptrs, nb, st)
                             : eval_items<float>(G, ptrs, nb, st);
}

}  // namespace

// C++ linkage for the templates of the fused path (this part of the file is
// inside the C-linkage block of the entry points).
extern "C++" {
namespace {

// ----------------------------------------------------------- fused batches
// Items on several geometries evaluated with one launch per stage for all of
// them (gridding, block sum, each FFT pass once per line length and kernel,
// interpolation) instead of one launch sequence per geometry: small meshes
// that leave most of the chip idle on their own fill it together, and the
// gridding's longest-first order runs over the units of every item. Item i of
// a geometry that occurs k times in the batch uses that context's per-item
// buffers of slot k (the context grows them as for a batch of its own). The
// device tables of a batch composition (the per-item arguments with their
// buffers offset to the slot, the FFT pass tables, the work lists) are built
// once and cached; the density and potential pointers travel as kernel
// arguments.
struct FusedPlan {
  int dev = -1, prec = 0, m = 0;
  std::vector<uint64_t> key;            // per item: context serial, slot
  std::vector<const void *> bufs;       // per item: the five work buffers it was built for
  void *mem = nullptr;                  // device tables
  size_t off_items = 0, off_bins = 0, off_red = 0, off_interp = 0;
  int64_t n_bins = 0, n_red = 0, n_interp = 0;
  struct Fft {
    int variant, N;
    size_t off_passes, off_work;
    int64_t n;
  };
  std::vector<Fft> ffts;                // in pass order
  uint64_t last_use = 0;
};
std::mutex g_fused_mu;
std::vector<FusedPlan> g_fused;
uint64_t g_fused_clock = 0;
constexpr size_t kFusedPlans = 8;

// The work buffers of item slot `slot` of a context.
WorkBufs slot_work(const slp_geom *G, int slot) {
  WorkBufs W = ctx_work(G);
  const size_t e = G->esz();
  const size_t per[5] = {e, e, 2 * e, 2 * e, e};
  void **b[5] = {&W.scratch, &W.grid_a, &W.S1, &W.S2, &W.grid_g};
  for (int k = 0; k < 5; ++k)
    *b[k] = static_cast<char *>(*b[k]) + (size_t)slot * (size_t)W.elems[k] * per[k];
  return W;
}

template <typename T>
int build_fused(FusedPlan &P, slp_geom *const *geoms, const std::vector<int32_t> &slot) {
  const int n = (int)slot.size();
  std::vector<slp::MultiItem<T>> items(n);
  std::vector<std::array<slp::FftPass<T>, 5>> passes(n);
  for (int i = 0; i < n; ++i) {
    const slp_geom *G = geoms[i];
    const WorkBufs W = slot_work(G, slot[i]);
    items[i].sp = spread_args<T>(G, W);
    items[i].rd = reduce_args<T>(G, W);
    items[i].ip = interp_args<T>(G, W);
    slp::FftPass<T> ps[5];
    fft_passes<T>(G, W, ps);
    for (int k = 0; k < 5; ++k) passes[i][k] = ps[k];
  }
  // gridding units of every item, longest first (ties: item, then unit order)
  struct U { int32_t len, i, u; };
  std::vector<U> us;
  for (int i = 0; i < n; ++i)
    for (int32_t u = 0; u < geoms[i]->n_units; ++u) us.push_back({geoms[i]->unit_len[u], i, u});
  std::stable_sort(us.begin(), us.end(), [](const U &a, const U &b) { return a.len > b.len; });
  std::vector<int2> bins(us.size());
  for (size_t k = 0; k < us.size(); ++k) bins[k] = make_int2(us[k].i, us[k].u);
  std::vector<int2> red;
  for (int i = 0; i < n; ++i) {
    const int64_t t = (int64_t)geoms[i]->tiles[0] * geoms[i]->tiles[1] * geoms[i]->tiles[2];
    for (int64_t k = 0; k < t; ++k) red.push_back(make_int2(i, (int)k));
  }
  us.clear();
  for (int i = 0; i < n; ++i)
    for (int32_t k = 0; k < geoms[i]->n_tgt_tiles; ++k) us.push_back({geoms[i]->tgt_len[k], i, k});
  std::stable_sort(us.begin(), us.end(), [](const U &a, const U &b) { return a.len > b.len; });
  std::vector<int2> interp(us.size());
  for (size_t k = 0; k < us.size(); ++k) interp[k] = make_int2(us[k].i, us[k].u);
  // FFT launches: per pass, the items grouped by line length and kernel
  struct FftHost { int variant, N; std::vector<slp::FftPass<T>> ps; std::vector<int2> work; };
  std::vector<FftHost> fh;
  for (int k = 0; k < 5; ++k) {
    const size_t first = fh.size();
    for (int i = 0; i < n; ++i) {
      const int N = geoms[i]->N[kPassAxis[k]];
      int64_t blocks = 0;
      const int v = slp::fft_variant<T>(passes[i][k], N, &blocks);
      if (v < 0) return fail(SLP_EINVAL, "fused batch: FFT pass %d of item %d is not supported", k, i);
      size_t g = first;
      while (g < fh.size() && !(fh[g].variant == v && fh[g].N == N)) ++g;
      if (g == fh.size()) fh.push_back({v, N, {}, {}});
      const int j = (int)fh[g].ps.size();
      fh[g].ps.push_back(passes[i][k]);
      for (int64_t b = 0; b < blocks; ++b) fh[g].work.push_back(make_int2(j, (int)b));
    }
  }
  // one device allocation for every table
  size_t bytes = 0;
  auto take = [&](size_t sz) {
    const size_t at = bytes;
    bytes += (sz + 255) / 256 * 256;
    return at;
  };
  P.off_items = take(items.size() * sizeof(items[0]));
  P.off_bins = take(bins.size() * sizeof(int2));
  P.off_red = take(red.size() * sizeof(int2));
  P.off_interp = take(interp.size() * sizeof(int2));
  P.ffts.clear();
  for (const FftHost &f : fh)
    P.ffts.push_back({f.variant, f.N, take(f.ps.size() * sizeof(f.ps[0])),
                      take(f.work.size() * sizeof(int2)), (int64_t)f.work.size()});
  std::vector<char> host(bytes, 0);
  auto put = [&](size_t off, const void *src, size_t sz) {
    if (sz) std::memcpy(host.data() + off, src, sz);
  };
  put(P.off_items, items.data(), items.size() * sizeof(items[0]));
  put(P.off_bins, bins.data(), bins.size() * sizeof(int2));
  put(P.off_red, red.data(), red.size() * sizeof(int2));
  put(P.off_interp, interp.data(), interp.size() * sizeof(int2));
  for (size_t g = 0; g < fh.size(); ++g) {
    put(P.ffts[g].off_passes, fh[g].ps.data(), fh[g].ps.size() * sizeof(fh[g].ps[0]));
    put(P.ffts[g].off_work, fh[g].work.data(), fh[g].work.size() * sizeof(int2));
  }
  P.n_bins = (int64_t)bins.size();
  P.n_red = (int64_t)red.size();
  P.n_interp = (int64_t)interp.size();
  if (hipMalloc(&P.mem, bytes ? bytes : 256) != hipSuccess)
    return fail(SLP_ENOMEM, "fused batch: %zu bytes of device tables: allocation failed", bytes);
  HIP_TRY(hipMemcpy(P.mem, host.data(), bytes, hipMemcpyHostToDevice));
  return SLP_OK;
}

template <typename T>
int launch_fused(const FusedPlan &P, const slp_geom *G0, const slp::BatchPtrs &ptrs, hipStream_t st) {
  const char *b = static_cast<const char *>(P.mem);
  const auto *items = reinterpret_cast<const slp::MultiItem<T> *>(b + P.off_items);
  // the window of every item (the pointer fields are not read)
  const slp::SpreadBinsArgs<T> win = spread_args<T>(G0, ctx_work(G0));
  HIP_TRY(slp::launch_spread_multi<T>(items, reinterpret_cast<const int2 *>(b + P.off_bins), P.n_bins,
                                      reinterpret_cast<const int2 *>(b + P.off_red), P.n_red, P.m,
                                      ptrs, win, st));
  for (const FusedPlan::Fft &f : P.ffts)
    HIP_TRY(slp::launch_fft_multi<T>(f.variant, f.N,
                                     reinterpret_cast<const slp::FftPass<T> *>(b + f.off_passes),
                                     reinterpret_cast<const int2 *>(b + f.off_work), f.n, st));
  HIP_TRY(slp::launch_interp_multi<T>(items, reinterpret_cast<const int2 *>(b + P.off_interp),
                                      P.n_interp, P.m, ptrs, st));
  return SLP_OK;
}

// Whether the items can share fused launches: one precision, cut-off and
// window (kind and shape), the point-source gridding (no integrated-window
// gridding).
bool fusable(slp_geom *const *geoms, int32_t batch) {
  for (int32_t b = 0; b < batch; ++b) {
    const slp_geom *G = geoms[b], *G0 = geoms[0];
    if (G->prec != G0->prec || G->m != G0->m || G->window != G0->window || G->b != G0->b ||
        G->iw_order > 0)
      return false;
    if (G->nf_nnz > 0 && G->nf_rule != 0) return false;
  }
  return true;
}

// At most kMaxBatch items.
int run_fused(slp_geom *const *geoms, const double *const *dens, double *const *phi, int n,
              hipStream_t st) {
  std::vector<int32_t> slot(n);
  std::map<slp_geom *, int> count;
  for (int i = 0; i < n; ++i) slot[i] = count[geoms[i]]++;
  for (auto &gc : count) {
    const int rc = ensure_capacity(gc.first, gc.second, st);
    if (rc) return rc;
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::vector<uint64_t> key(2 * (size_t)n);
  std::vector<const void *> bufs(5 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    key[2 * i] = geoms[i]->serial;
    key[2 * i + 1] = (uint64_t)slot[i];
    const slp_geom *G = geoms[i];
    const void *bs[5] = {G->scratch, G->grid_a, G->S1, G->S2, G->grid_g};
    for (int k = 0; k < 5; ++k) bufs[5 * i + k] = bs[k];
  }
  const int prec = geoms[0]->prec, m = geoms[0]->m;
  std::lock_guard<std::mutex> lock(g_fused_mu);
  FusedPlan *P = nullptr;
  for (FusedPlan &q : g_fused)
    if (q.dev == dev && q.prec == prec && q.m == m && q.key == key && q.bufs == bufs) P = &q;
  if (!P) {
    if (g_fused.size() >= kFusedPlans) {
      // evict the least recently used plan; its tables may still be read by
      // launches in flight
      size_t lru = 0;
      for (size_t k = 1; k < g_fused.size(); ++k)
        if (g_fused[k].last_use < g_fused[lru].last_use) lru = k;
      HIP_TRY(hipDeviceSynchronize());
      if (g_fused[lru].mem) HIP_TRY(hipFree(g_fused[lru].mem));
      g_fused.erase(g_fused.begin() + (std::ptrdiff_t)lru);
    }
    FusedPlan q;
    q.dev = dev;
    q.prec = prec;
    q.m = m;
    q.key = key;
    q.bufs = bufs;
    const int rc = prec == SLP_FP64 ? build_fused<double>(q, geoms, slot)
                                    : build_fused<float>(q, geoms, slot);
    if (rc) {
      if (q.mem) (void)hipFree(q.mem);
      return rc;
    }
    g_fused.push_back(q);
    P = &g_fused.back();
  }
  P->last_use = ++g_fused_clock;
  slp::BatchPtrs ptrs{};
  for (int i = 0; i < n; ++i) {
    ptrs.dens[i] = dens[i];
    ptrs.phi[i] = phi[i];
  }
  int rc = prec == SLP_FP64 ? launch_fused<double>(*P, geoms[0], ptrs, st)
                            : launch_fused<float>(*P, geoms[0], ptrs, st);
  if (rc) return rc;
  // near-field corrections, per geometry for its items in slot order
  for (auto &gc : count) {
    slp_geom *G = gc.first;
    if (G->nf_nnz == 0) continue;
    slp::BatchPtrs np{};
    for (int i = 0; i < n; ++i)
      if (geoms[i] == G) {
        np.dens[slot[i]] = dens[i];
        np.phi[slot[i]] = phi[i];
      }
    HIP_TRY(near_apply(G, ctx_work(G), np, gc.second, st));
  }
  return SLP_OK;
}

}  // namespace
}  // extern "C++"

int slp_eval_single_layer_static(slp_geom *G, double *phi, void *stream) {
  if (!G || !phi) return fail(SLP_EINVAL, "geometry and phi must be non-NULL");
  if (!G->dens) return fail(SLP_EINVAL, "no density set (slp_set_density)");
  // carve the work buffers of one item out of the static workspace, each
  // 256-byte aligned
  const size_t e = G->esz();
  const size_t per[5] = {e, e, 2 * e, 2 * e, e};
  size_t off[7], need = 0;
  auto take = [&](size_t bytes) {
    const size_t at = need;
    need += (bytes + 255) / 256 * 256;
    return at;
  };
  for (int i = 0; i < 5; ++i) off[i] = take((size_t)G->item_elems[i] * per[i]);
  const bool nf = G->nf_nnz > 0, iw = G->iw_order > 0;
  off[5] = take(nf ? (size_t)G->n_tris * 8 : 0);
  off[6] = take(iw ? (size_t)G->n_tris * 8 : 0);
  if (need > slp::kStaticWorkspaceBytes)
    return fail(SLP_ENOMEM,
                "static workspace: this evaluation needs %zu bytes of work buffers, the workspace "
                "holds %zu (use slp_eval_single_layer)",
                need, slp::kStaticWorkspaceBytes);
  void *base = nullptr;
  HIP_TRY(slp::static_workspace(&base));
  char *b = static_cast<char *>(base);
  WorkBufs W;
  W.scratch = b + off[0];
  W.grid_a = b + off[1];
  W.S1 = b + off[2];
  W.S2 = b + off[3];
  W.grid_g = b + off[4];
  W.nf_gbar = nf ? reinterpret_cast<double *>(b + off[5]) : nullptr;
  W.iw_gbar = iw ? reinterpret_cast<double *>(b + off[6]) : nullptr;
  for (int i = 0; i < 5; ++i) W.elems[i] = G->item_elems[i];
  hipStream_t st = static_cast<hipStream_t>(stream);
  slp::BatchPtrs ptrs{};
  ptrs.dens[0] = G->dens;
  ptrs.phi[0] = phi;
  // direct launches (no captured graph: it would hold the context's buffers);
  // the sampled stage events are recorded as for the other evaluations
  const bool tm = G->timing && (G->evals++ % G->every == 0);
  if (tm) {
    const int rc = begin_timed(G, st);
    if (rc) return rc;
  }
  return G->prec == SLP_FP64 ? run_eval<double>(G, W, ptrs, 1, st, tm)
                             : run_eval<float>(G, W, ptrs, 1, st, tm);
}

int slp_eval_batched(slp_geom *const *geoms, const double *const *dens, double *const *phi,
                     int32_t batch, void *stream) {
  return slp_eval_batched_mode(geoms, dens, phi, batch, SLP_BATCH_AUTO, stream);
}

int slp_eval_batched_mode(slp_geom *const *geoms, const double *const *dens, double *const *phi,
                          int32_t batch, int32_t mode, void *stream) {
  if (batch < 1 || !geoms || !dens || !phi) return fail(SLP_EINVAL, "batched: batch >= 1 and non-NULL arrays");
  for (int32_t b = 0; b < batch; ++b)
    if (!geoms[b] || !dens[b] || !phi[b]) return fail(SLP_EINVAL, "batched: item %d has a NULL pointer", b);
  if (mode != SLP_BATCH_AUTO && mode != SLP_BATCH_LANES && mode != SLP_BATCH_FUSED)
    return fail(SLP_EINVAL, "batched: unknown mode %d", mode);
  hipStream_t st = static_cast<hipStream_t>(stream);
  bool fuse = mode == SLP_BATCH_FUSED;
  if (fuse && !fusable(geoms, batch))
    return fail(SLP_EINVAL, "batched: fused launches need one precision, cut-off and window and "
                            "the point-source gridding on every item");
  if (mode == SLP_BATCH_AUTO && fusable(geoms, batch))
    for (int32_t b = 1; b < batch && !fuse; ++b) fuse = geoms[b] != geoms[0];
  if (fuse) {
    for (int32_t b = 0; b < batch; b += slp::kMaxBatch) {
      const int n = std::min<int32_t>(slp::kMaxBatch, batch - b);
      const int rc = run_fused(geoms + b, dens + b, phi + b, n, st);
      if (rc) return rc;
    }
    return SLP_OK;
  }
  // launch groups: consecutive items on one geometry share every launch
  struct Group { slp_geom *G; int32_t b, e; };
  std::vector<Group> groups;
  for (int32_t b = 0; b < batch;) {
    int32_t e = b + 1;
    while (e < batch && geoms[e] == geoms[b] && e - b < slp::kMaxBatch) ++e;
    groups.push_back({geoms[b], b, e});
    b = e;
  }
  // every geometry gets one lane (its work buffers serve one group at a time)
  std::map<slp_geom *, int> lane_of;
  for (const Group &g : groups)
    if (!lane_of.count(g.G)) {
      const int l = (int)lane_of.size() % kLanes;
      lane_of[g.G] = l;
    }
  if (lane_of.size() == 1) {
    for (const Group &g : groups) {
      const int rc = run_group(g.G, dens + g.b, phi + g.b, g.e - g.b, st);
      if (rc) return rc;
    }
    return SLP_OK;
  }
  // several geometries: their groups overlap on the lanes, forked from and
  // joined back into the caller's stream
  std::lock_guard<std::mutex> lock(g_lanes_mu);
  Lanes *L = nullptr;
  int rc = get_lanes(&L);
  if (rc) return rc;
  const int used = std::min<int>(kLanes, (int)lane_of.size());
  HIP_TRY(hipEventRecord(L->fork, st));
  for (int l = 0; l < used; ++l) HIP_TRY(hipStreamWaitEvent(L->s[l], L->fork, 0));
  for (const Group &g : groups) {
    rc = run_group(g.G, dens + g.b, phi + g.b, g.e - g.b, L->s[lane_of[g.G]]);
    if (rc) break;
  }
  // join even after an error, so the caller's stream never runs ahead of work
  // already enqueued on the lanes
  for (int l = 0; l < used; ++l) {
    HIP_TRY(hipEventRecord(L->join[l], L->s[l]));
    HIP_TRY(hipStreamWaitEvent(st, L->join[l], 0));
  }
  return rc;
}

int slp_geom_get_info(const slp_geom *G, slp_geom_info *info) {
  if (!G || !info) return fail(SLP_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  for (int q = 0; q < 3; ++q) {
    info->centre[q] = G->c[q];
    info->scale[q] = G->s[q];
    info->lo[q] = G->lo[q];
    info->extent[q] = G->R[q];
    info->tiles[q] = G->tiles[q];
  }
  info->window_b = G->b;
  info->n_nodes = G->n_nodes;
  info->n_targets = G->n_tgt;
  info->n_tris = G->n_tris;
  info->n_src = G->n_src;
  info->terms_kept = G->terms_kept;
  info->device_bytes = G->bytes;
  info->seg_share = G->share;
  info->n_segments = G->n_slots;
  const int64_t ntiles = (int64_t)G->tiles[0] * G->tiles[1] * G->tiles[2];
  info->reduce_cells = G->reduce_cells ? G->reduce_cells : (ntiles >= slp::kReduceTwoCells ? 2 : 1);
  return SLP_OK;
}

int slp_choose_cutoff(double tol, int32_t precision, int32_t window_in, int32_t *window,
                      int32_t *m) {
  if (!window || !m) return fail(SLP_EINVAL, "NULL output");
  if (!(tol > 0.0)) return fail(SLP_EINVAL, "tol must be positive");
  if (precision != SLP_FP64 && precision != SLP_FP32)
    return fail(SLP_EINVAL, "precision must be SLP_FP64 or SLP_FP32");
  if (window_in < -1 || window_in > SLP_WINDOW_KB) return fail(SLP_EINVAL, "unknown window");
  const double pi = 3.141592653589793238462643383279502884;
  const double floor_err = precision == SLP_FP32 ? 2e-6 : 0.0;
  auto predicted = [&](int w, int mm) {
    const double bound = w == SLP_WINDOW_KB
        ? 4.0 * pi * (std::sqrt((double)mm) + mm) * std::pow(0.5, 0.25) *
              std::exp(-2.0 * pi * mm * std::sqrt(0.5))
        : 4.0 * std::exp(-2.0 * pi * mm / 3.0);
    return bound / 5.0 + floor_err;
  };
  int best_w = -1, best_m = 0;
  for (int w = SLP_WINDOW_GAUSS; w <= SLP_WINDOW_KB; ++w) {
    if (window_in != -1 && w != window_in) continue;
    for (int mm = 1; mm <= slp::kMaxM; ++mm)
      if (predicted(w, mm) <= tol) {
        if (best_w < 0 || mm < best_m) { best_w = w; best_m = mm; }
        break;
      }
  }
  if (best_w < 0) return fail(SLP_EINVAL, "no cut-off m <= %d reaches rel. error %g", slp::kMaxM, tol);
  *window = best_w;
  *m = best_m;
  return SLP_OK;
}

int slp_set_graph(slp_geom *G, int32_t enable) {
  if (!G) return fail(SLP_EINVAL, "NULL geometry");
  if (enable && G->iw_order > 0)
    return fail(SLP_EINVAL, "captured evaluations do not combine with integrated-window gridding");
  if (!enable && G->use_graph) {
    HIP_TRY(hipDeviceSynchronize());
    G->drop_graphs();
  }
  G->use_graph = enable != 0;
  return SLP_OK;
}

int slp_set_timing(slp_geom *G, int32_t every) {
  if (!G || every < 0) return fail(SLP_EINVAL, "NULL geometry or every < 0");
  if (every) {
    int rc = ensure_events(G);
    if (rc) return rc;
  }
  G->timing = every != 0;
  G->every = every ? every : 1;
  G->evals = 0;
  return SLP_OK;
}

int slp_stage_times(slp_geom *G, double *ms, int64_t *count, int32_t reset) {
  if (!G || !ms || !count) return fail(SLP_EINVAL, "NULL argument");
  int rc = collect_timing(G);
  if (rc) return rc;
  for (int i = 0; i < slp_geom::kStages; ++i) ms[i] = G->acc_ms[i];
  *count = G->count;
  if (reset) {
    for (double &v : G->acc_ms) v = 0.0;
    G->count = 0;
  }
  return SLP_OK;
}

int slp_debug_copy(const slp_geom *G, int32_t which, void *dst, size_t dst_bytes, void *stream) {
  if (!G || !dst) return fail(SLP_EINVAL, "NULL argument");
  const size_t e = G->esz();
  size_t need;
  const void *src;
  if (which == 0) {
    need = (size_t)G->P[0] * G->P[1] * G->P[2] * e;
    src = G->grid_a;
  } else if (which == 1) {
    need = (size_t)G->R[0] * G->R[1] * G->R[2] * e;
    src = G->grid_g;
  } else if (which == 2) {
    need = (size_t)G->n_src * sizeof(double);
    src = G->own_dens;
  } else {
    return fail(SLP_EINVAL, "debug_copy: which must be 0, 1 or 2");
  }
  if (dst_bytes < need) return fail(SLP_EINVAL, "debug_copy: dst holds %zu bytes, need %zu", dst_bytes, need);
  HIP_TRY(hipMemcpyAsync(dst, src, need, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  return SLP_OK;
}

// ------------------------------------------------------------ near field ---

namespace {
// Stored form of a near-field pattern: every row padded with column -1 to a
// multiple of the group size, or of the interleaved chunk when rows average
// 2048 pairs or more (padding then a few per cent); chunked columns packed as
// chunk base + 16-bit offsets when every chunk spans fewer than 65535.
struct NearLayout {
  bool chunked = false, packed = false;
  int64_t stored = 0;
  std::vector<int64_t> prow, counts;
  std::vector<int32_t> cols, bases;
  std::vector<uint16_t> offs;
};

bool near_layout(const std::vector<int64_t> &rowptr, const std::vector<int32_t> &cols, int64_t P,
                 NearLayout &L) {
  try {
    const int64_t nnz = rowptr[P];
    L.chunked = nnz >= (int64_t)8 * slp::kNearChunk * P;
    const int64_t grp = L.chunked ? slp::kNearChunk : slp::kNearGroup;
    L.prow.assign(P + 1, 0);
    L.counts.resize(P);
    for (int64_t i = 0; i < P; ++i) {
      L.counts[i] = rowptr[i + 1] - rowptr[i];
      L.prow[i + 1] = L.prow[i] + (L.counts[i] + grp - 1) / grp * grp;
    }
    L.stored = L.prow[P];
    L.cols.assign(L.stored, -1);
    for (int64_t i = 0; i < P; ++i) {
      const int64_t n = L.counts[i];
      if (!L.chunked) {
        std::copy(cols.begin() + rowptr[i], cols.begin() + rowptr[i + 1], L.cols.begin() + L.prow[i]);
        continue;
      }
      // entry e = c * 256 + 64 k + l of the row goes to c * 256 + 4 l + k
      for (int64_t e = 0; e < n; ++e) {
        const int64_t c = e / slp::kNearChunk, r = e % slp::kNearChunk;
        const int64_t k = r / 64, l = r % 64;
        L.cols[L.prow[i] + c * slp::kNearChunk + 4 * l + k] = cols[rowptr[i] + e];
      }
    }
    L.packed = L.chunked;
    if (L.packed) {
      const int64_t nch = L.stored / slp::kNearChunk;
      L.bases.assign(nch, 0);
      for (int64_t c = 0; c < nch && L.packed; ++c) {
        int32_t lo = std::numeric_limits<int32_t>::max(), hi = -1;
        for (int64_t e = c * slp::kNearChunk; e < (c + 1) * slp::kNearChunk; ++e)
          if (L.cols[e] >= 0) { lo = std::min(lo, L.cols[e]); hi = std::max(hi, L.cols[e]); }
        if (hi < 0) lo = hi = 0;
        if ((int64_t)hi - lo >= 65535) L.packed = false;
        L.bases[c] = lo;
      }
      if (L.packed) {
        L.offs.assign(L.stored, 0);
        for (int64_t e = 0; e < L.stored; ++e)
          if (L.cols[e] >= 0) L.offs[e] = (uint16_t)(L.cols[e] - L.bases[e / slp::kNearChunk]);
      } else {
        std::vector<int32_t>().swap(L.bases);
      }
    }
    return true;
  } catch (const std::bad_alloc &) {
    return false;
  }
}

// Device bytes of a stored near field (every buffer at least the allocation
// minimum, as the context allocates them).
int64_t near_bytes(const NearLayout &L, int64_t P, int64_t M, size_t esz, int cap) {
  auto a = [](int64_t b) { return std::max<int64_t>(b, (int64_t)slp_geom::kMinAlloc); };
  int64_t b = a((P + 1) * 8) + a(L.stored * (int64_t)esz) + a(M * 8 * cap);
  b += L.packed ? a((int64_t)L.bases.size() * 4) + a(L.stored * 2) : a(L.stored * 4);
  return b;
}

int host_threads() {
  const unsigned hw = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(16u, hw ? hw : 1u));
}

void drop_near(slp_geom *G) {
  G->release(G->nf_rowptr);
  G->release(G->nf_cols);
  G->release(G->nf_bases);
  G->release(G->nf_offs);
  G->release(G->nf_vals);
  G->release(G->nf_gbar);
  G->nf_rowptr = nullptr;
  G->nf_cols = nullptr;
  G->nf_bases = nullptr;
  G->nf_offs = nullptr;
  G->nf_packed = false;
  G->nf_chunked = false;
  std::vector<int64_t>().swap(G->nf_rows);
  G->nf_vals = nullptr;
  G->nf_gbar = nullptr;
  G->nf_nnz = 0;
  G->nf_stored = 0;
  G->nf_eps = 0.0;
}

void drop_iw(slp_geom *G) {
  for (void *q : {(void *)G->iw_rowptr, (void *)G->iw_cols, (void *)G->iw_bases, (void *)G->iw_offs,
                  G->iw_vals, (void *)G->iw_gbar})
    G->release(q);
  G->iw_rowptr = nullptr;
  G->iw_cols = nullptr;
  G->iw_bases = nullptr;
  G->iw_offs = nullptr;
  G->iw_vals = nullptr;
  G->iw_gbar = nullptr;
  G->iw_packed = false;
  G->iw_order = 0;
  G->iw_nnz = G->iw_stored = G->iw_rows = 0;
}
}  // namespace

int slp_setup_near_field(slp_geom *G, double eps, void *stream) {
  if (!G) return fail(SLP_EINVAL, "NULL geometry");
  return slp_setup_near_field_stored(G, eps, G->prec, stream);
}

int slp_setup_near_field_stored(slp_geom *G, double eps, int32_t storage, void *stream) {
  if (!G) return fail(SLP_EINVAL, "NULL geometry");
  if (!std::isfinite(eps)) return fail(SLP_EINVAL, "eps must be finite");
  if (storage != SLP_FP64 && storage != SLP_FP32)
    return fail(SLP_EINVAL, "storage must be SLP_FP64 or SLP_FP32");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipDeviceSynchronize());     // captured evaluations may still run elsewhere
  G->drop_graphs();                    // they were captured with the old near field
  drop_near(G);
  if (eps <= 0.0) return SLP_OK;

  std::vector<int64_t> rowptr;
  std::vector<int32_t> cols;
  std::string err;
  if (!slp::build_near_pattern(G->h_nodes.data(), G->n_nodes, G->h_tris.data(), G->n_tris,
                               G->h_tgt.data(), G->n_tgt, eps, host_threads(), rowptr, cols, err))
    return fail(SLP_ENOMEM, "%s", err.c_str());
  const int64_t nnz = rowptr.back();
  G->nf_eps = eps;
  G->nf_prec = storage;
  if (nnz == 0) return SLP_OK;

  const int64_t P = G->n_tgt;
  NearLayout L;
  if (!near_layout(rowptr, cols, P, L))
    return fail(SLP_ENOMEM, "host allocation for the padded near-field pattern failed");
  const bool chunked = L.chunked, packed = L.packed;
  const int64_t stored = L.stored;
  rowptr.swap(L.prow);
  cols.swap(L.cols);
  std::vector<int32_t> &bases = L.bases;
  std::vector<uint16_t> &offs = L.offs;
  std::vector<int64_t> &counts = L.counts;

  // persistent: pattern, values, element means; temporary: coordinates,
  // triangles, terms (and the int32 columns when packed)
  void *rp = nullptr, *cl = nullptr, *bs = nullptr, *of = nullptr, *vl = nullptr, *gb = nullptr;
  bool ok = G->alloc(&rp, rowptr.size() * sizeof(int64_t)) == hipSuccess &&
            G->alloc(&vl, (size_t)stored * (storage == SLP_FP64 ? 8 : 4)) == hipSuccess &&
            G->alloc(&gb, (size_t)G->n_tris * 8 * G->cap) == hipSuccess;
  if (ok && packed)
    ok = G->alloc(&bs, bases.size() * sizeof(int32_t)) == hipSuccess &&
         G->alloc(&of, offs.size() * sizeof(uint16_t)) == hipSuccess;
  else if (ok)
    ok = G->alloc(&cl, (size_t)stored * sizeof(int32_t)) == hipSuccess;
  if (!ok) {
    for (void *q : {rp, cl, bs, of, vl, gb}) G->release(q);
    G->nf_eps = 0.0;
    return fail(SLP_ENOMEM, "near field: %lld entries do not fit in device memory", (long long)nnz);
  }
  G->nf_rowptr = static_cast<int64_t *>(rp);
  G->nf_cols = static_cast<int32_t *>(cl);
  G->nf_bases = static_cast<int32_t *>(bs);
  G->nf_offs = static_cast<uint16_t *>(of);
  G->nf_packed = packed;
  G->nf_chunked = chunked;
  G->nf_rows.swap(counts);
  G->nf_vals = vl;
  G->nf_gbar = static_cast<double *>(gb);
  G->nf_nnz = nnz;
  G->nf_stored = stored;
  const int S = G->terms_kept;
  double *d_tg = nullptr, *d_nodes = nullptr, *d_terms = nullptr;
  int32_t *d_tris = nullptr, *d_cols = G->nf_cols;
  struct Temp {
    std::vector<void *> p;
    ~Temp() { for (void *q : p) (void)hipFree(q); }
  } tmp;
  auto talloc = [&](void **q, size_t bytes) {
    hipError_t e = hipMalloc(q, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) tmp.p.push_back(*q);
    return e;
  };
  // with integrated-window gridding the smooth share is the collapsed rule's
  const std::vector<double> rule = G->iw_order > 0 ? collapsed_rule(G->iw_order) : std::vector<double>();
  double *d_rule = nullptr;
  if (talloc((void **)&d_tg, G->h_tgt.size() * 8) != hipSuccess ||
      talloc((void **)&d_nodes, G->h_nodes.size() * 8) != hipSuccess ||
      talloc((void **)&d_tris, G->h_tris.size() * 4) != hipSuccess ||
      talloc((void **)&d_terms, (size_t)2 * S * 8) != hipSuccess ||
      (!rule.empty() && talloc((void **)&d_rule, rule.size() * 8) != hipSuccess) ||
      (packed && talloc((void **)&d_cols, (size_t)stored * 4) != hipSuccess)) {
    drop_near(G);
    return fail(SLP_ENOMEM, "near field: temporary device buffers failed");
  }
  HIP_TRY(hipMemcpyAsync(G->nf_rowptr, rowptr.data(), rowptr.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_cols, cols.data(), (size_t)stored * 4, hipMemcpyHostToDevice, st));
  if (packed) {
    HIP_TRY(hipMemcpyAsync(G->nf_bases, bases.data(), bases.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(G->nf_offs, offs.data(), offs.size() * 2, hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(d_tg, G->h_tgt.data(), G->h_tgt.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_nodes, G->h_nodes.data(), G->h_nodes.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_tris, G->h_tris.data(), G->h_tris.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_terms, G->kept_w.data(), (size_t)S * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_terms + S, G->kept_g.data(), (size_t)S * 8, hipMemcpyHostToDevice, st));
  if (d_rule) HIP_TRY(hipMemcpyAsync(d_rule, rule.data(), rule.size() * 8, hipMemcpyHostToDevice, st));
  const int32_t npts = (int32_t)(rule.size() / 3);
  G->nf_rule = G->iw_order;
  if (storage == SLP_FP64) {
    slp::NearArgs<double> na = near_args<double>(G, ctx_work(G));
    na.cols = d_cols;
    HIP_TRY(slp::launch_near_values<double>(na, d_tg, d_nodes, d_tris, d_terms, d_terms + S, S,
                                            d_rule, npts, st));
  } else {
    slp::NearArgs<float> na = near_args<float>(G, ctx_work(G));
    na.cols = d_cols;
    HIP_TRY(slp::launch_near_values<float>(na, d_tg, d_nodes, d_tris, d_terms, d_terms + S, S,
                                           d_rule, npts, st));
  }
  HIP_TRY(hipStreamSynchronize(st));   // host vectors and temporaries go out of scope
  return SLP_OK;
}

int slp_near_field_device_bytes(const double *nodes, int64_t n_nodes, const int32_t *tris,
                                int64_t n_tris, const double *targets, int64_t n_targets,
                                double eps, int32_t precision, int64_t *bytes) {
  if (!nodes || !tris || !bytes) return fail(SLP_EINVAL, "NULL argument");
  if (n_nodes < 3 || n_tris < 1) return fail(SLP_EINVAL, "empty mesh");
  if (!std::isfinite(eps)) return fail(SLP_EINVAL, "eps must be finite");
  if (precision != SLP_FP64 && precision != SLP_FP32)
    return fail(SLP_EINVAL, "precision must be SLP_FP64 or SLP_FP32");
  for (int64_t j = 0; j < 3 * n_tris; ++j)
    if (tris[j] < 0 || tris[j] >= n_nodes)
      return fail(SLP_EINVAL, "triangle %lld references node %d out of range", (long long)(j / 3), tris[j]);
  if (!targets) {
    targets = nodes;
    n_targets = n_nodes;
  }
  *bytes = 0;
  if (eps <= 0.0) return SLP_OK;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> cols;
  std::string err;
  if (!slp::build_near_pattern(nodes, n_nodes, tris, n_tris, targets, n_targets, eps, host_threads(),
                               rowptr, cols, err))
    return fail(SLP_ENOMEM, "%s", err.c_str());
  if (rowptr.back() == 0) return SLP_OK;
  NearLayout L;
  if (!near_layout(rowptr, cols, n_targets, L))
    return fail(SLP_ENOMEM, "host allocation for the padded near-field pattern failed");
  *bytes = near_bytes(L, n_targets, n_tris, precision == SLP_FP64 ? 8 : 4, 1);
  return SLP_OK;
}

int slp_near_radius(const slp_geom *G, double tol, double *eps) {
  if (!G || !eps) return fail(SLP_EINVAL, "NULL argument");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(SLP_EINVAL, "tol must be positive");
  const double r = slp::near_radius(G->kept_w.data(), G->kept_g.data(), G->terms_kept, G->r_max, tol);
  if (r < 0.0)
    return fail(SLP_EINVAL, "the kept exponential sum misses 1/r by more than %g at the body diameter %g",
                tol, G->r_max);
  *eps = r;
  return SLP_OK;
}


int slp_setup_integrated_gridding(slp_geom *G, int32_t order, void *stream) {
  if (!G) return fail(SLP_EINVAL, "NULL geometry");
  if (order < 0 || order > 16) return fail(SLP_EINVAL, "order must be 0 (off) or 1..16, got %d", (int)order);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (order > 0 && G->use_graph)
    return fail(SLP_EINVAL, "integrated-window gridding does not combine with captured evaluations");
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipDeviceSynchronize());
  G->drop_graphs();
  drop_iw(G);
  // a near field subtracts the smooth kernel with the gridding's quadrature:
  // rebuild its values for the new gridding
  auto rebuild_near = [&]() {
    return G->nf_eps > 0.0 ? slp_setup_near_field_stored(G, G->nf_eps, G->nf_prec, stream) : SLP_OK;
  };
  if (order == 0) return rebuild_near();

  // vertices in grid units, areas, and each triangle's index box
  // {floor(t_min) - m + 1 .. floor(t_max) + m} per axis (eq. indexset2),
  // relative to the region
  const int64_t M = G->n_tris;
  const int64_t R0 = G->R[0], R1 = G->R[1], rows = (int64_t)G->R[0] * G->R[1] * G->R[2];
  std::vector<int64_t> rowptr;
  std::vector<int32_t> cols;
  std::vector<double> tv(9 * M), area(M);
  std::vector<int32_t> box(6 * M);
  try {
    for (int64_t j = 0; j < M; ++j) {
      const double *P[3];
      for (int k = 0; k < 3; ++k) P[k] = &G->h_nodes[3 * (int64_t)G->h_tris[3 * j + k]];
      double e1[3], e2[3];
      for (int q = 0; q < 3; ++q) { e1[q] = P[1][q] - P[0][q]; e2[q] = P[2][q] - P[0][q]; }
      const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                            e1[0] * e2[1] - e1[1] * e2[0]};
      area[j] = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      for (int q = 0; q < 3; ++q) {
        double tmin = INFINITY, tmax = -INFINITY;
        for (int k = 0; k < 3; ++k) {
          const double t = ((P[k][q] - G->c[q]) * G->s[q] + 0.5) * G->N[q];
          tv[9 * j + 3 * k + q] = t;
          tmin = std::min(tmin, t);
          tmax = std::max(tmax, t);
        }
        const int64_t blo = (int64_t)std::floor(tmin) - G->m + 1 - G->lo[q];
        const int64_t bhi = (int64_t)std::floor(tmax) + G->m - G->lo[q];
        if (blo < 0 || bhi >= G->R[q])
          return fail(SLP_EINVAL, "triangle %lld: its window box leaves the region of the sources and "
                      "targets (evaluate at the nodes, or at points that include them)", (long long)j);
        box[6 * j + q] = (int32_t)blo;
        box[6 * j + 3 + q] = (int32_t)bhi;
      }
    }
    // rows = region cells, columns = triangles in ascending order
    rowptr.assign(rows + 1, 0);
    auto cells = [&](int64_t j, auto &&fn) {
      const int32_t *b = &box[6 * j];
      for (int64_t z = b[2]; z <= b[5]; ++z)
        for (int64_t y = b[1]; y <= b[4]; ++y)
          for (int64_t x = b[0]; x <= b[3]; ++x) fn(x + R0 * (y + R1 * z));
    };
    for (int64_t j = 0; j < M; ++j) cells(j, [&](int64_t r) { rowptr[r + 1] += 1; });
    for (int64_t r = 0; r < rows; ++r) rowptr[r + 1] += rowptr[r];
    cols.resize(rowptr[rows]);
    std::vector<int64_t> fill(rowptr.begin(), rowptr.end() - 1);
    for (int64_t j = 0; j < M; ++j) cells(j, [&](int64_t r) { cols[fill[r]++] = (int32_t)j; });
  } catch (const std::bad_alloc &) {
    return fail(SLP_ENOMEM, "host allocation for the integrated-window pattern failed");
  }
  const int64_t nnz = rowptr.back();
  NearLayout L;
  if (!near_layout(rowptr, cols, rows, L))
    return fail(SLP_ENOMEM, "host allocation for the padded integrated-window pattern failed");
  std::vector<int32_t>().swap(cols);

  void *rp = nullptr, *cl = nullptr, *bs = nullptr, *of = nullptr, *vl = nullptr, *gb = nullptr;
  bool ok = G->alloc(&rp, L.prow.size() * sizeof(int64_t)) == hipSuccess &&
            G->alloc(&vl, (size_t)L.stored * G->esz()) == hipSuccess &&
            G->alloc(&gb, (size_t)M * 8 * G->cap) == hipSuccess;
  if (ok && L.packed)
    ok = G->alloc(&bs, L.bases.size() * sizeof(int32_t)) == hipSuccess &&
         G->alloc(&of, L.offs.size() * sizeof(uint16_t)) == hipSuccess;
  else if (ok)
    ok = G->alloc(&cl, (size_t)L.stored * sizeof(int32_t)) == hipSuccess;
  if (!ok) {
    for (void *q : {rp, cl, bs, of, vl, gb}) G->release(q);
    return fail(SLP_ENOMEM, "integrated-window gridding: %lld entries do not fit in device memory",
                (long long)nnz);
  }
  G->iw_rowptr = static_cast<int64_t *>(rp);
  G->iw_cols = static_cast<int32_t *>(cl);
  G->iw_bases = static_cast<int32_t *>(bs);
  G->iw_offs = static_cast<uint16_t *>(of);
  G->iw_vals = vl;
  G->iw_gbar = static_cast<double *>(gb);
  G->iw_packed = L.packed;
  G->iw_nnz = nnz;
  G->iw_stored = L.stored;
  G->iw_rows = rows;

  const std::vector<double> rule = collapsed_rule(order);
  struct Temp {
    std::vector<void *> p;
    ~Temp() { for (void *q : p) (void)hipFree(q); }
  } tmp;
  auto talloc = [&](void **q, size_t bytes) {
    hipError_t e = hipMalloc(q, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) tmp.p.push_back(*q);
    return e;
  };
  double *d_tv = nullptr, *d_area = nullptr, *d_rule = nullptr;
  int32_t *d_cols = G->iw_cols;
  if (talloc((void **)&d_tv, tv.size() * 8) != hipSuccess ||
      talloc((void **)&d_area, area.size() * 8) != hipSuccess ||
      talloc((void **)&d_rule, rule.size() * 8) != hipSuccess ||
      (L.packed && talloc((void **)&d_cols, (size_t)L.stored * 4) != hipSuccess)) {
    drop_iw(G);
    return fail(SLP_ENOMEM, "integrated-window gridding: temporary device buffers failed");
  }
  HIP_TRY(hipMemcpyAsync(G->iw_rowptr, L.prow.data(), L.prow.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_cols, L.cols.data(), (size_t)L.stored * 4, hipMemcpyHostToDevice, st));
  if (L.packed) {
    HIP_TRY(hipMemcpyAsync(G->iw_bases, L.bases.data(), L.bases.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(G->iw_offs, L.offs.data(), L.offs.size() * 2, hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(d_tv, tv.data(), tv.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_area, area.data(), area.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_rule, rule.data(), rule.size() * 8, hipMemcpyHostToDevice, st));
  slp::IwGeom g{};
  g.tv = d_tv;
  g.area = d_area;
  g.rule = d_rule;
  g.npts = order * order;
  for (int q = 0; q < 3; ++q) { g.lo[q] = G->lo[q]; g.R[q] = G->R[q]; }
  g.m = G->m;
  g.window = G->window == SLP_WINDOW_KB ? 1 : 0;
  g.inv_b = 1.0 / G->b;
  g.b = G->b;
  g.kb_inv_norm = G->kb_inv_norm;
  if (G->prec == SLP_FP64) {
    slp::NearArgs<double> a = iw_args<double>(G, ctx_work(G));
    a.cols = d_cols;
    HIP_TRY(slp::launch_iw_values<double>(a, g, st));
  } else {
    slp::NearArgs<float> a = iw_args<float>(G, ctx_work(G));
    a.cols = d_cols;
    HIP_TRY(slp::launch_iw_values<float>(a, g, st));
  }
  HIP_TRY(hipStreamSynchronize(st));   // host vectors and temporaries go out of scope
  G->iw_order = order;
  return rebuild_near();
}

int slp_integrated_gridding_info(const slp_geom *G, int32_t *order, int64_t *nnz, int64_t *stored,
                                 int32_t *packed) {
  if (!G) return fail(SLP_EINVAL, "NULL geometry");
  if (order) *order = G->iw_order;
  if (nnz) *nnz = G->iw_nnz;
  if (stored) *stored = G->iw_stored;
  if (packed) *packed = G->iw_packed ? 1 : 0;
  return SLP_OK;
}

int slp_near_field_info(const slp_geom *G, double *eps, int64_t *nnz, double *r_max,
                        int64_t *stored, int32_t *packed) {
  if (!G) return fail(SLP_EINVAL, "NULL geometry");
  if (eps) *eps = G->nf_eps;
  if (nnz) *nnz = G->nf_nnz;
  if (r_max) *r_max = G->r_max;
  if (stored) *stored = G->nf_stored;
  if (packed) *packed = G->nf_packed ? 1 : 0;
  return SLP_OK;
}

int slp_debug_copy_near(const slp_geom *G, int64_t *rowptr, int32_t *cols, double *vals,
                        int64_t cap) {
  if (!G || !rowptr) return fail(SLP_EINVAL, "NULL argument");
  if (G->nf_nnz > cap) return fail(SLP_EINVAL, "debug_copy_near: %lld entries, room for %lld",
                                   (long long)G->nf_nnz, (long long)cap);
  HIP_TRY(hipDeviceSynchronize());
  if (G->nf_nnz == 0) {
    for (int64_t i = 0; i <= G->n_tgt; ++i) rowptr[i] = 0;
    return SLP_OK;
  }
  // the stored rows carry padding (column -1) at their ends: drop it
  const int64_t P = G->n_tgt, S = G->nf_stored;
  std::vector<int64_t> prow(P + 1);
  std::vector<int32_t> pc(S);
  std::vector<double> pv(vals ? S : 0);
  HIP_TRY(hipMemcpy(prow.data(), G->nf_rowptr, (size_t)(P + 1) * 8, hipMemcpyDeviceToHost));
  if (G->nf_packed) {
    // columns from chunk bases and offsets; padding from the row lengths
    std::vector<int32_t> bs((size_t)(S / slp::kNearChunk));
    std::vector<uint16_t> of((size_t)S);
    HIP_TRY(hipMemcpy(bs.data(), G->nf_bases, bs.size() * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(of.data(), G->nf_offs, of.size() * 2, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < P; ++i)
      for (int64_t p = prow[i]; p < prow[i + 1]; ++p) {
        const int64_t w = p - prow[i], c = w / slp::kNearChunk, r = w % slp::kNearChunk;
        const int64_t e = c * slp::kNearChunk + 64 * (r % 4) + r / 4;
        pc[p] = e < G->nf_rows[i] ? bs[p / slp::kNearChunk] + of[p] : -1;
      }
  } else {
    HIP_TRY(hipMemcpy(pc.data(), G->nf_cols, (size_t)S * 4, hipMemcpyDeviceToHost));
  }
  if (vals) {
    if (G->nf_prec == SLP_FP64) {
      HIP_TRY(hipMemcpy(pv.data(), G->nf_vals, (size_t)S * 8, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> f((size_t)S);
      HIP_TRY(hipMemcpy(f.data(), G->nf_vals, f.size() * 4, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < f.size(); ++i) pv[i] = f[i];
    }
  }
  // rows in increasing triangle order (long rows are stored interleaved)
  int64_t k = 0;
  rowptr[0] = 0;
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t i = 0; i < P; ++i) {
    row.clear();
    for (int64_t e = prow[i]; e < prow[i + 1]; ++e)
      if (pc[e] >= 0) row.emplace_back(pc[e], vals ? pv[e] : 0.0);
    std::sort(row.begin(), row.end(),
              [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
                return a.first < b.first;
              });
    for (const auto &ent : row) {
      if (cols) cols[k] = ent.first;
      if (vals) vals[k] = ent.second;
      ++k;
    }
    rowptr[i + 1] = k;
  }
  return SLP_OK;
}

int slp_near_pattern_host(const double *nodes, int64_t n_nodes, const int32_t *tris,
                          int64_t n_tris, const double *targets, int64_t n_targets, double eps,
                          int64_t *rowptr, int32_t *cols, int64_t cols_cap, int64_t *nnz) {
  if (!nodes || !tris || !targets || !nnz) return fail(SLP_EINVAL, "NULL argument");
  if (n_nodes < 3 || n_tris < 1 || n_targets < 1) return fail(SLP_EINVAL, "empty mesh or targets");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(SLP_EINVAL, "eps must be finite and >= 0");
  for (int64_t j = 0; j < 3 * n_tris; ++j)
    if (tris[j] < 0 || tris[j] >= n_nodes)
      return fail(SLP_EINVAL, "triangle %lld references node %d out of range", (long long)(j / 3), tris[j]);
  std::vector<int64_t> rp;
  std::vector<int32_t> cl;
  std::string err;
  if (!slp::build_near_pattern(nodes, n_nodes, tris, n_tris, targets, n_targets, eps, host_threads(),
                               rp, cl, err))
    return fail(SLP_ENOMEM, "%s", err.c_str());
  *nnz = rp.back();
  if (rowptr) std::copy(rp.begin(), rp.end(), rowptr);
  if (cols) {
    if (cols_cap < rp.back()) return fail(SLP_EINVAL, "cols holds %lld entries, need %lld",
                                          (long long)cols_cap, (long long)rp.back());
    std::copy(cl.begin(), cl.end(), cols);
  }
  return SLP_OK;
}

int slp_triangle_potential_host(const double *x, const double *a, const double *b,
                                const double *c, int64_t count, double *out) {
  if (!x || !a || !b || !c || !out || count < 0) return fail(SLP_EINVAL, "NULL argument or count < 0");
  for (int64_t i = 0; i < count; ++i)
    out[i] = slp::triangle_potential(x + 3 * i, a + 3 * i, b + 3 * i, c + 3 * i);
  return SLP_OK;
}

int slp_near_radius_host(const double *es_w, const double *es_gamma, int32_t terms, double r_max,
                         double tol, double *eps) {
  if (!es_w || !es_gamma || !eps || terms < 1) return fail(SLP_EINVAL, "NULL argument or no terms");
  if (!(tol > 0.0) || !(r_max > 0.0)) return fail(SLP_EINVAL, "tol and r_max must be positive");
  const double r = slp::near_radius(es_w, es_gamma, terms, r_max, tol);
  if (r < 0.0) return fail(SLP_EINVAL, "the sum misses 1/r by more than %g at r_max", tol);
  *eps = r;
  return SLP_OK;
}

int slp_geom_destroy(slp_geom *G) {
  if (!G) return SLP_OK;
  (void)hipDeviceSynchronize();
  delete G;
  return SLP_OK;
}

}  // extern "C"
