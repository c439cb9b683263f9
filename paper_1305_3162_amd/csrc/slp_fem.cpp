// Host side of the Dirichlet problem for phi_1 (Sec. 2.1) and of the complete
// scalar potential phi = phi_1 + phi_2 (Alg. 1): mesh analysis, the free-node
// stiffness matrix, and the orchestration of the device solve.
#include "slp.h"
#include "slp_amg.hpp"
#include "slp_fem.hpp"
#include "slp_internal.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cfloat>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>
#include <thread>
#include <vector>

namespace {

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  slp::set_error_message(buf);
  return code;
}

#define FEM_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(SLP_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                  __FILE__, __LINE__);                                                   \
  } while (0)

}  // namespace

struct slp_fem {
  int64_t n_nodes = 0, n_tets = 0, n_free = 0, n_btris = 0, nnz = 0;
  std::vector<int32_t> h_btris;   // [Mb][3] outward boundary triangles
  // device
  int32_t *tets = nullptr;        // [T][4]
  double *vol = nullptr;          // [T]
  double *grad = nullptr;         // [T][4][3]
  int32_t *inc_ptr = nullptr, *inc = nullptr;
  int32_t *free_node = nullptr;   // [Nf] node of free index f
  int32_t *node_free = nullptr;   // [N] free index or -1
  int32_t *sptr = nullptr, *ci = nullptr;   // S_ff in 64-row slices
  double *val = nullptr, *dinv = nullptr;
  int32_t *owner = nullptr;       // [Mb]
  double *nrm = nullptr;          // [Mb][3]
  double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *q = nullptr;
  double *p[2] = {nullptr, nullptr};
  double *vm = nullptr;           // [T][3] work of the load vector
  double *part = nullptr, *hist = nullptr;
  int32_t hist_cap = 0;
  double *phi1 = nullptr, *dn = nullptr;   // for slp_scalar_potential
  double *epart = nullptr;                 // [ceil(T / 256) + 1] energy partials and sum
  double *h_pin = nullptr;                 // pinned [2] for the convergence check
  int32_t nblk = 1;
  // preconditioner: SLP_PRECOND_JACOBI or SLP_PRECOND_AMG (the hierarchy below)
  int32_t precond = SLP_PRECOND_JACOBI;
  slp::HostCsr h_S;                        // S_ff on the host, for building the hierarchy
  struct DevCsr {
    int32_t *rp = nullptr, *ci = nullptr;
    double *v = nullptr;
    int64_t rows = 0, nnz = 0;
    int32_t lanes = 1;
  };
  struct DevLevel {
    DevCsr A, P, R;                        // A unused on the finest level (the sliced S_ff)
    double *w = nullptr;                   // omega / a_ii
    double *f = nullptr;                   // right-hand side (the CG residual on the finest level)
    double *x = nullptr;                   // smoothed iterate
    double *res = nullptr;                 // residual, then the level's result
    int64_t n = 0;
  };
  std::vector<DevLevel> amg;
  bool amg_built = false;
  DevCsr amg_coarse;                       // dense inverse of the coarsest operator, as CSR
  double *amg_fc = nullptr, *amg_ec = nullptr;
  int64_t bytes = 0;
  std::vector<void *> allocs;
  std::vector<int64_t> alloc_bytes;
  hipError_t alloc(void **p_, size_t n) {
    *p_ = nullptr;
    const size_t sz = std::max<size_t>(n, 256);
    hipError_t e = hipMalloc(p_, sz);
    if (e == hipSuccess) {
      allocs.push_back(*p_);
      alloc_bytes.push_back((int64_t)sz);
      bytes += (int64_t)sz;
    }
    return e;
  }
  void release(void *p_) {
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == p_) {
        (void)hipFree(p_);
        bytes -= alloc_bytes[i];
        allocs.erase(allocs.begin() + i);
        alloc_bytes.erase(alloc_bytes.begin() + i);
        return;
      }
  }
  ~slp_fem() {
    for (void *p_ : allocs) (void)hipFree(p_);
    if (h_pin) (void)hipHostFree(h_pin);
  }
};

namespace {

// Boundary faces: faces of exactly one tetrahedron, oriented away from the
// tetrahedron's fourth vertex, ordered by their sorted vertex triple.
struct Face {
  std::array<int32_t, 3> key;
  int32_t tet, local;
};

// The free-node stiffness matrix and the free nodes, for the host-only
// assembly (slp_fem_assemble_host).
struct HostAssembly {
  std::vector<int32_t> rp, ci, free_node;
  std::vector<double> val;
};

int fem_setup_impl(slp_fem **out, const double *nodes, int64_t N, const int32_t *tets, int64_t T,
                   hipStream_t st, HostAssembly *host = nullptr) {
  if (!out && !host) return fail(SLP_EINVAL, "out is NULL");
  if (out) *out = nullptr;
  if (!nodes || !tets || N < 4 || T < 1) return fail(SLP_EINVAL, "need >= 4 nodes and >= 1 tetrahedron");
  if (N > INT32_MAX || 4 * T > INT32_MAX) return fail(SLP_EINVAL, "mesh too large for 32-bit indices");
  for (int64_t i = 0; i < 4 * T; ++i)
    if (tets[i] < 0 || tets[i] >= N)
      return fail(SLP_EINVAL, "tetrahedron %lld references node %d out of range", (long long)(i / 4), tets[i]);
  for (int64_t i = 0; i < 3 * N; ++i)
    if (!std::isfinite(nodes[i])) return fail(SLP_EINVAL, "node %lld has a non-finite coordinate", (long long)(i / 3));

  slp_fem *F = new (std::nothrow) slp_fem();
  if (!F) return fail(SLP_ENOMEM, "host allocation failed");
  struct Guard {
    slp_fem *f;
    ~Guard() { delete f; }
  } guard{F};
  F->n_nodes = N;
  F->n_tets = T;
  try {
    // gradients of the barycentric coordinates: rows of J^{-1}, J = [x1-x0, x2-x0, x3-x0]
    std::vector<double> vol(T), grad(12 * T);
    for (int64_t t = 0; t < T; ++t) {
      const double *x0 = nodes + 3 * (int64_t)tets[4 * t];
      double J[3][3];
      for (int c = 0; c < 3; ++c) {
        const double *xc = nodes + 3 * (int64_t)tets[4 * t + 1 + c];
        for (int rr = 0; rr < 3; ++rr) J[rr][c] = xc[rr] - x0[rr];
      }
      const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      if (!(std::fabs(det) > 0.0)) return fail(SLP_EINVAL, "tetrahedron %lld is degenerate", (long long)t);
      double inv[3][3];
      inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
      inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
      inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
      inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
      inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
      inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
      inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
      inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
      inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
      vol[t] = std::fabs(det) / 6.0;
      for (int q = 0; q < 3; ++q) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
          grad[12 * t + 3 * (a + 1) + q] = inv[a][q];
          s += inv[a][q];
        }
        grad[12 * t + q] = -s;
      }
    }

    // boundary faces
    std::vector<Face> faces(4 * T);
    const int fl[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    for (int64_t t = 0; t < T; ++t)
      for (int f = 0; f < 4; ++f) {
        Face &fc = faces[4 * t + f];
        for (int k = 0; k < 3; ++k) fc.key[k] = tets[4 * t + fl[f][k]];
        std::sort(fc.key.begin(), fc.key.end());
        fc.tet = (int32_t)t;
        fc.local = f;
      }
    std::sort(faces.begin(), faces.end(), [](const Face &a, const Face &b) { return a.key < b.key; });
    std::vector<int32_t> btris, owner;
    std::vector<double> bn;
    std::vector<char> on_bnd(N, 0);
    for (size_t i = 0; i < faces.size();) {
      size_t j = i + 1;
      while (j < faces.size() && faces[j].key == faces[i].key) ++j;
      if (j - i > 2) return fail(SLP_EINVAL, "a face is shared by more than two tetrahedra");
      if (j - i == 1) {
        const Face &fc = faces[i];
        int32_t v[3];
        for (int k = 0; k < 3; ++k) v[k] = tets[4 * (int64_t)fc.tet + fl[fc.local][k]];
        const int32_t opp = tets[4 * (int64_t)fc.tet + fc.local];
        const double *a = nodes + 3 * (int64_t)v[0], *b = nodes + 3 * (int64_t)v[1], *c = nodes + 3 * (int64_t)v[2];
        const double *o = nodes + 3 * (int64_t)opp;
        double e1[3], e2[3], n[3];
        for (int q = 0; q < 3; ++q) { e1[q] = b[q] - a[q]; e2[q] = c[q] - a[q]; }
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double side = n[0] * (o[0] - a[0]) + n[1] * (o[1] - a[1]) + n[2] * (o[2] - a[2]);
        if (side > 0) {
          std::swap(v[1], v[2]);
          for (double &w : n) w = -w;
        }
        const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int k = 0; k < 3; ++k) {
          btris.push_back(v[k]);
          on_bnd[v[k]] = 1;
          bn.push_back(n[k] / len);
        }
        owner.push_back(fc.tet);
      }
      i = j;
    }
    std::vector<Face>().swap(faces);
    const int64_t Mb = (int64_t)owner.size();
    if (Mb == 0) return fail(SLP_EINVAL, "the mesh has no boundary");

    // free nodes, node -> (tet, local) incidence of the free nodes
    std::vector<int32_t> node_free(N, -1), free_node;
    for (int64_t k = 0; k < N; ++k)
      if (!on_bnd[k]) {
        node_free[k] = (int32_t)free_node.size();
        free_node.push_back((int32_t)k);
      }
    const int64_t Nf = (int64_t)free_node.size();
    std::vector<int32_t> inc_ptr(Nf + 1, 0), inc;
    for (int64_t i = 0; i < 4 * T; ++i)
      if (node_free[tets[i]] >= 0) inc_ptr[node_free[tets[i]] + 1] += 1;
    for (int64_t f = 0; f < Nf; ++f) inc_ptr[f + 1] += inc_ptr[f];
    inc.resize(inc_ptr[Nf]);
    {
      std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
      for (int64_t i = 0; i < 4 * T; ++i) {
        const int32_t f = node_free[tets[i]];
        if (f >= 0) inc[fill[f]++] = (int32_t)i;   // 4 t + local
      }
    }

    // S(fn, fn) by rows: row f sums |T| grad_a . grad_b over the tetrahedra
    // of its node; columns sorted; up to 16 threads over row ranges
    std::vector<int32_t> rp(Nf + 1, 0);
    std::vector<std::vector<int32_t>> pc;
    std::vector<std::vector<double>> pv;
    const int nth = (int)std::max<int64_t>(1, std::min<int64_t>(
        std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency())), Nf));
    pc.resize(nth);
    pv.resize(nth);
    std::vector<int32_t> rowlen(Nf, 0);
    auto rows = [&](int w) {
      const int64_t f0 = Nf * w / nth, f1 = Nf * (w + 1) / nth;
      std::vector<std::pair<int32_t, double>> ent;
      for (int64_t f = f0; f < f1; ++f) {
        ent.clear();
        for (int32_t e = inc_ptr[f]; e < inc_ptr[f + 1]; ++e) {
          const int64_t t = inc[e] >> 2;
          const int la = inc[e] & 3;
          for (int lb = 0; lb < 4; ++lb) {
            const int32_t g = node_free[tets[4 * t + lb]];
            if (g < 0) continue;
            const double *ga = &grad[12 * t + 3 * la], *gb = &grad[12 * t + 3 * lb];
            ent.emplace_back(g, vol[t] * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]));
          }
        }
        std::sort(ent.begin(), ent.end(),
                  [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
                    return a.first < b.first;
                  });
        // an off-diagonal entry whose contributions cancel to within the
        // rounding of their sum is zero (on lattices of Kuhn simplices half
        // of the stored pattern) and is not stored
        int32_t n = 0;
        for (size_t k = 0; k < ent.size();) {
          size_t l = k;
          double s = 0.0, sa = 0.0;
          while (l < ent.size() && ent[l].first == ent[k].first) {
            s += ent[l].second;
            sa += std::fabs(ent[l++].second);
          }
          if (ent[k].first == f || std::fabs(s) > 16.0 * DBL_EPSILON * sa) {
            pc[w].push_back(ent[k].first);
            pv[w].push_back(s);
            ++n;
          }
          k = l;
        }
        rowlen[f] = n;
      }
    };
    {
      std::vector<std::thread> pool;
      for (int w = 1; w < nth; ++w) pool.emplace_back(rows, w);
      rows(0);
      for (std::thread &t : pool) t.join();
    }
    for (int64_t f = 0; f < Nf; ++f) rp[f + 1] = rp[f] + rowlen[f];
    const int64_t nnz = rp[Nf];
    std::vector<int32_t> ci(nnz);
    std::vector<double> val(nnz), dinv(Nf, 0.0);
    for (int w = 0; w < nth; ++w) {
      const int64_t f0 = Nf * w / nth;
      std::copy(pc[w].begin(), pc[w].end(), ci.begin() + rp[f0]);
      std::copy(pv[w].begin(), pv[w].end(), val.begin() + rp[f0]);
    }
    for (int64_t f = 0; f < Nf; ++f)
      for (int32_t e = rp[f]; e < rp[f + 1]; ++e)
        if (ci[e] == f) dinv[f] = 1.0 / val[e];
    // sliced layout: 64 rows per slice, entries column by column
    const int64_t ns = (Nf + 63) / 64;
    std::vector<int32_t> sptr(ns + 1, 0);
    for (int64_t sl = 0; sl < ns; ++sl) {
      int32_t w = 0;
      for (int64_t f = 64 * sl; f < std::min<int64_t>(Nf, 64 * sl + 64); ++f) w = std::max(w, rp[f + 1] - rp[f]);
      if ((int64_t)sptr[sl] + 64 * (int64_t)w > INT32_MAX)
        return fail(SLP_EINVAL, "stiffness matrix too large for 32-bit offsets");
      sptr[sl + 1] = sptr[sl] + 64 * w;
    }
    std::vector<int32_t> sci(sptr[ns]);
    std::vector<double> sval(sptr[ns], 0.0);
    for (int64_t sl = 0; sl < ns; ++sl) {
      const int32_t w = (sptr[sl + 1] - sptr[sl]) / 64;
      for (int64_t l = 0; l < 64; ++l) {
        const int64_t f = std::min<int64_t>(64 * sl + l, Nf - 1);
        const bool real = 64 * sl + l < Nf;
        for (int32_t k = 0; k < w; ++k) {
          const int64_t e = sptr[sl] + 64 * (int64_t)k + l;
          const int32_t src = rp[f] + k;
          if (real && src < rp[f + 1]) {
            sci[e] = ci[src];
            sval[e] = val[src];
          } else {
            sci[e] = (int32_t)f;
          }
        }
      }
    }

    if (host) {
      // host-only: the assembled matrix, no device work
      host->rp = rp;
      host->ci = ci;
      host->val = val;
      host->free_node = free_node;
      return SLP_OK;
    }
    F->n_free = Nf;
    F->h_S.rows = F->h_S.cols = Nf;
    F->h_S.rp = std::move(rp);
    F->h_S.ci = std::move(ci);
    F->h_S.v = std::move(val);
    F->n_btris = Mb;
    F->nnz = nnz;
    F->nblk = (int32_t)std::max<int64_t>(1, (Nf + slp::kFemThreads - 1) / slp::kFemThreads);
    F->h_btris = btris;

    // device buffers
    struct Req { void **p; size_t n; };
    const Req reqs[] = {
        {(void **)&F->tets, (size_t)4 * T * 4}, {(void **)&F->vol, (size_t)T * 8},
        {(void **)&F->grad, (size_t)12 * T * 8}, {(void **)&F->inc_ptr, (size_t)(Nf + 1) * 4},
        {(void **)&F->inc, inc.size() * 4}, {(void **)&F->free_node, (size_t)std::max<int64_t>(Nf, 1) * 4},
        {(void **)&F->node_free, (size_t)N * 4}, {(void **)&F->sptr, sptr.size() * 4},
        {(void **)&F->ci, sci.size() * 4}, {(void **)&F->val, sval.size() * 8},
        {(void **)&F->dinv, (size_t)Nf * 8}, {(void **)&F->owner, (size_t)Mb * 4},
        {(void **)&F->nrm, (size_t)3 * Mb * 8}, {(void **)&F->b, (size_t)Nf * 8},
        {(void **)&F->x, (size_t)Nf * 8}, {(void **)&F->r, (size_t)Nf * 8},
        {(void **)&F->z, (size_t)Nf * 8}, {(void **)&F->p[0], (size_t)Nf * 8},
        {(void **)&F->p[1], (size_t)Nf * 8}, {(void **)&F->vm, (size_t)3 * T * 8},
        {(void **)&F->q, (size_t)Nf * 8}, {(void **)&F->part, (size_t)5 * F->nblk * 8},
        {(void **)&F->phi1, (size_t)N * 8}, {(void **)&F->dn, (size_t)Mb * 8},
        {(void **)&F->epart, (size_t)((T + slp::kFemThreads - 1) / slp::kFemThreads + 1) * 8},
    };
    for (const Req &rq : reqs)
      if (F->alloc(rq.p, rq.n) != hipSuccess)
        return fail(SLP_ENOMEM, "device allocation failed (%lld bytes so far)", (long long)F->bytes);
    FEM_TRY(hipHostMalloc((void **)&F->h_pin, 2 * sizeof(double), hipHostMallocDefault));
    FEM_TRY(hipMemcpyAsync(F->tets, tets, (size_t)4 * T * 4, hipMemcpyHostToDevice, st));
    FEM_TRY(hipMemcpyAsync(F->vol, vol.data(), (size_t)T * 8, hipMemcpyHostToDevice, st));
    FEM_TRY(hipMemcpyAsync(F->grad, grad.data(), (size_t)12 * T * 8, hipMemcpyHostToDevice, st));
    FEM_TRY(hipMemcpyAsync(F->inc_ptr, inc_ptr.data(), (size_t)(Nf + 1) * 4, hipMemcpyHostToDevice, st));
    FEM_TRY(hipMemcpyAsync(F->inc, inc.data(), inc.size() * 4, hipMemcpyHostToDevice, st));
    if (Nf > 0) FEM_TRY(hipMemcpyAsync(F->free_node, free_node.data(), (size_t)Nf * 4, hipMemcpyHostToDevice, st));
    FEM_TRY(hipMemcpyAsync(F->node_free, node_free.data(), (size_t)N * 4, hipMemcpyHostToDevice, st));
    FEM_TRY(hipMemcpyAsync(F->sptr, sptr.data(), sptr.size() * 4, hipMemcpyHostToDevice, st));
    if (!sci.empty()) {
      FEM_TRY(hipMemcpyAsync(F->ci, sci.data(), sci.size() * 4, hipMemcpyHostToDevice, st));
      FEM_TRY(hipMemcpyAsync(F->val, sval.data(), sval.size() * 8, hipMemcpyHostToDevice, st));
      FEM_TRY(hipMemcpyAsync(F->dinv, dinv.data(), (size_t)Nf * 8, hipMemcpyHostToDevice, st));
    }
    FEM_TRY(hipMemcpyAsync(F->owner, owner.data(), (size_t)Mb * 4, hipMemcpyHostToDevice, st));
    FEM_TRY(hipMemcpyAsync(F->nrm, bn.data(), (size_t)3 * Mb * 8, hipMemcpyHostToDevice, st));
    FEM_TRY(hipStreamSynchronize(st));
  } catch (const std::bad_alloc &) {
    return fail(SLP_ENOMEM, "host allocation failed during the mesh analysis");
  }
  guard.f = nullptr;
  *out = F;
  return SLP_OK;
}

slp::PcgArgs pcg_args(slp_fem *F, const double *x0) {
  slp::PcgArgs a{};
  a.sptr = F->sptr;
  a.ci = F->ci;
  a.val = F->val;
  a.dinv = F->dinv;
  a.b = F->b;
  a.x = F->x;
  a.r = F->r;
  a.z = F->z;
  a.p[0] = F->p[0];
  a.p[1] = F->p[1];
  a.q = F->q;
  a.part = F->part;
  a.hist = F->hist;
  a.node_free = F->node_free;
  a.x0 = x0;
  a.nf = F->n_free;
  a.n_nodes = F->n_nodes;
  a.nblk = F->nblk;
  a.jacobi = F->precond == SLP_PRECOND_AMG ? 0 : 1;
  return a;
}

// Uploads a host CSR matrix; lanes per row: the power of two nearest above
// the mean row length, from 1 to 64.
int upload_csr(slp_fem *F, const slp::HostCsr &H, slp_fem::DevCsr &D, hipStream_t st) {
  D.rows = H.rows;
  D.nnz = (int64_t)H.ci.size();
  if (F->alloc((void **)&D.rp, H.rp.size() * 4) != hipSuccess ||
      F->alloc((void **)&D.ci, H.ci.size() * 4) != hipSuccess ||
      F->alloc((void **)&D.v, H.v.size() * 8) != hipSuccess)
    return fail(SLP_ENOMEM, "device allocation of the multigrid hierarchy failed");
  FEM_TRY(hipMemcpyAsync(D.rp, H.rp.data(), H.rp.size() * 4, hipMemcpyHostToDevice, st));
  if (D.nnz > 0) {
    FEM_TRY(hipMemcpyAsync(D.ci, H.ci.data(), H.ci.size() * 4, hipMemcpyHostToDevice, st));
    FEM_TRY(hipMemcpyAsync(D.v, H.v.data(), H.v.size() * 8, hipMemcpyHostToDevice, st));
  }
  const double mean = H.rows > 0 ? (double)D.nnz / (double)H.rows : 1.0;
  D.lanes = 1;
  while (D.lanes < 64 && D.lanes < mean) D.lanes *= 2;
  return SLP_OK;
}

int upload_amg(slp_fem *F, slp::AmgHierarchy &h, hipStream_t st);

// Builds the smoothed-aggregation hierarchy of S_ff on the host and moves it
// to the device with the vectors of the cycle.
int build_amg_impl(slp_fem *F, hipStream_t st) {
  if (F->amg_built) return SLP_OK;
  slp::AmgHierarchy h;
  char err[256] = {0};
  try {
    if (!slp::build_amg(F->h_S, slp::AmgParams(), h, err, sizeof err))
      return fail(SLP_EINVAL, "multigrid setup: %s", err);
  } catch (const std::bad_alloc &) {
    return fail(SLP_ENOMEM, "host allocation failed while building the multigrid hierarchy");
  }
  const size_t first = F->allocs.size();
  int rc = upload_amg(F, h, st);
  // the copies read the host hierarchy, which goes out of scope here
  const hipError_t e = hipStreamSynchronize(st);
  if (!rc && e != hipSuccess)
    rc = fail(SLP_EDEVICE, "copying the multigrid hierarchy failed: %s", hipGetErrorString(e));
  if (rc) {
    // free what this attempt allocated (the allocations are recorded in order)
    while (F->allocs.size() > first) F->release(F->allocs.back());
    F->amg.clear();
    F->amg_coarse = slp_fem::DevCsr();
    F->amg_fc = F->amg_ec = nullptr;
    return rc;
  }
  F->amg_built = true;
  return SLP_OK;
}

int upload_amg(slp_fem *F, slp::AmgHierarchy &h, hipStream_t st) {
  const size_t nl = h.levels.size();
  F->amg.assign(nl, slp_fem::DevLevel());
  for (size_t l = 0; l < nl; ++l) {
    slp_fem::DevLevel &d = F->amg[l];
    const slp::AmgLevel &H = h.levels[l];
    d.n = H.A.rows;
    int rc;
    if (l > 0 && (rc = upload_csr(F, H.A, d.A, st)) != SLP_OK) return rc;
    if ((rc = upload_csr(F, H.P, d.P, st)) != SLP_OK) return rc;
    if ((rc = upload_csr(F, H.R, d.R, st)) != SLP_OK) return rc;
    const size_t vb = (size_t)d.n * 8;
    if (F->alloc((void **)&d.w, vb) != hipSuccess || F->alloc((void **)&d.x, vb) != hipSuccess ||
        F->alloc((void **)&d.res, vb) != hipSuccess ||
        (l > 0 && F->alloc((void **)&d.f, vb) != hipSuccess))
      return fail(SLP_ENOMEM, "device allocation of the multigrid vectors failed");
    if (l == 0) d.f = F->r;
    FEM_TRY(hipMemcpyAsync(d.w, H.w.data(), vb, hipMemcpyHostToDevice, st));
  }
  slp::HostCsr C;
  C.rows = C.cols = h.nc;
  C.rp.resize(h.nc + 1);
  C.ci.resize(h.nc * h.nc);
  for (int64_t i = 0; i <= h.nc; ++i) C.rp[i] = (int32_t)(i * h.nc);
  for (int64_t k = 0; k < h.nc * h.nc; ++k) C.ci[k] = (int32_t)(k % h.nc);
  C.v = std::move(h.coarse_inv);
  int rc = upload_csr(F, C, F->amg_coarse, st);
  if (rc != SLP_OK) return rc;
  if (nl > 0 && (F->alloc((void **)&F->amg_fc, (size_t)h.nc * 8) != hipSuccess ||
                 F->alloc((void **)&F->amg_ec, (size_t)h.nc * 8) != hipSuccess))
    return fail(SLP_ENOMEM, "device allocation of the multigrid vectors failed");
  return SLP_OK;
}

// z = B r for the V(1,1) cycle B (damped-Jacobi pre- and post-smoothing,
// R = P^T, exact coarsest solve), and the partial sums of r.z into `slot`.
int vcycle(slp_fem *F, const slp::PcgArgs &a, int32_t slot, hipStream_t st) {
  const int nl = (int)F->amg.size();
  slp::AmgOp op{};
  if (nl == 0) {   // the whole system is the coarsest: z = S_ff^-1 r
    const slp_fem::DevCsr &C = F->amg_coarse;
    op = slp::AmgOp{C.rp, C.ci, C.v, F->r, nullptr, nullptr, F->z, nullptr, C.rows};
    FEM_TRY(slp::launch_amg_csr(op, slp::kAmgRestrict, C.lanes, st));
    FEM_TRY(slp::launch_amg_dot(a, slot, st));
    return SLP_OK;
  }
  for (int l = 0; l < nl; ++l) {
    slp_fem::DevLevel &d = F->amg[l];
    op = slp::AmgOp{d.A.rp, d.A.ci, d.A.v, d.f, d.w, d.f, d.x, d.res, d.n};
    if (l == 0)
      FEM_TRY(slp::launch_amg_fine(a, op, slp::kAmgPre, slot, st));
    else
      FEM_TRY(slp::launch_amg_csr(op, slp::kAmgPre, d.A.lanes, st));
    double *fnext = l + 1 < nl ? F->amg[l + 1].f : F->amg_fc;
    op = slp::AmgOp{d.R.rp, d.R.ci, d.R.v, d.res, nullptr, nullptr, fnext, nullptr, d.R.rows};
    FEM_TRY(slp::launch_amg_csr(op, slp::kAmgRestrict, d.R.lanes, st));
  }
  const slp_fem::DevCsr &C = F->amg_coarse;
  op = slp::AmgOp{C.rp, C.ci, C.v, F->amg_fc, nullptr, nullptr, F->amg_ec, nullptr, C.rows};
  FEM_TRY(slp::launch_amg_csr(op, slp::kAmgRestrict, C.lanes, st));
  for (int l = nl - 1; l >= 0; --l) {
    slp_fem::DevLevel &d = F->amg[l];
    const double *e = l + 1 < nl ? F->amg[l + 1].res : F->amg_ec;
    op = slp::AmgOp{d.P.rp, d.P.ci, d.P.v, e, nullptr, d.x, d.x, nullptr, d.n};
    FEM_TRY(slp::launch_amg_csr(op, slp::kAmgProlong, d.P.lanes, st));
    double *out = l == 0 ? F->z : d.res;
    op = slp::AmgOp{d.A.rp, d.A.ci, d.A.v, d.x, d.w, d.f, out, nullptr, d.n};
    if (l == 0)
      FEM_TRY(slp::launch_amg_fine(a, op, slp::kAmgPost, slot, st));
    else
      FEM_TRY(slp::launch_amg_csr(op, slp::kAmgPost, d.A.lanes, st));
  }
  return SLP_OK;
}

int solve_impl(slp_fem *F, const double *m, double *phi1, double tol, int32_t max_iter,
               int32_t warm, int32_t *iters, double *rel_res, hipStream_t st) {
  if (!F || !m || !phi1) return fail(SLP_EINVAL, "NULL argument");
  if (!(tol > 0.0) || max_iter < 1) return fail(SLP_EINVAL, "tol must be positive and max_iter >= 1");
  if (F->hist_cap < max_iter + 1) {
    void *h = nullptr;
    if (F->alloc(&h, (size_t)(max_iter + 1) * 8) != hipSuccess)
      return fail(SLP_ENOMEM, "device allocation of the residual history failed");
    F->release(F->hist);
    F->hist = static_cast<double *>(h);
    F->hist_cap = max_iter + 1;
  }
  int32_t it = 0;
  double rel = 0.0;
  if (F->n_free > 0) {
    slp::FemLoadArgs la{};
    la.inc_ptr = F->inc_ptr;
    la.inc = F->inc;
    la.tets = F->tets;
    la.vol = F->vol;
    la.grad = F->grad;
    la.m = m;
    la.vm = F->vm;
    la.b = F->b;
    la.nf = F->n_free;
    la.nt = F->n_tets;
    FEM_TRY(slp::launch_fem_load(la, st));
    const bool amg = F->precond == SLP_PRECOND_AMG;
    const slp::PcgArgs a = pcg_args(F, warm ? phi1 : nullptr);
    FEM_TRY(slp::launch_pcg_start(a, F->free_node, st));
    if (amg) {
      const int rc = vcycle(F, a, 1, st);
      if (rc) return rc;
    }
    FEM_TRY(slp::launch_pcg_reduce(a, 4, 0, st));
    // the residual of the start is the first check: r.r from the start kernel
    // is not formed, so check after the first block of iterations (shorter
    // with the multigrid cycle, which converges in tens of iterations)
    const int32_t every = amg ? 4 : 16;
    // With the multigrid cycle (an iteration costs several checks), from the
    // second check on the next one is placed where the rate seen between the
    // last two checks reaches tol (at most two blocks ahead), so a solve stops
    // within about one iteration of convergence, not one block. Jacobi
    // iterations cost about as much as a check: every 16.
    int32_t block = every, it_last = 0;
    double bb = -1.0, rel_last = -1.0;
    for (it = 0; it < max_iter;) {
      const int32_t n = std::min(block, max_iter - it);
      for (int32_t k = 0; k < n; ++k, ++it) {
        FEM_TRY(slp::launch_pcg_iteration(a, it, st));
        if (amg) {
          const int rc = vcycle(F, a, 1 + ((it + 1) & 1), st);
          if (rc) return rc;
        }
      }
      FEM_TRY(slp::launch_pcg_reduce(a, 3, it, st));
      FEM_TRY(hipMemcpyAsync(F->h_pin, F->hist, 8, hipMemcpyDeviceToHost, st));
      FEM_TRY(hipMemcpyAsync(F->h_pin + 1, F->hist + it, 8, hipMemcpyDeviceToHost, st));
      FEM_TRY(hipStreamSynchronize(st));
      bb = F->h_pin[0];
      const double rr = F->h_pin[1];
      rel = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
      if (!std::isfinite(rel)) return fail(SLP_EDEVICE, "conjugate gradients broke down (residual %g)", rel);
      if (rel <= tol) break;
      block = every;
      if (amg && rel_last > 0.0 && rel > 0.0 && rel < rel_last) {
        const double per_it = std::log(rel / rel_last) / (double)(it - it_last);   // < 0
        const double need = std::ceil(std::log(tol / rel) / per_it);
        block = (int32_t)std::max(1.0, std::min(need, 2.0 * every));
      }
      rel_last = rel;
      it_last = it;
    }
  }
  FEM_TRY(slp::launch_fem_scatter(F->x, F->node_free, phi1, F->n_nodes, st));
  if (iters) *iters = it;
  if (rel_res) *rel_res = rel;
  if (rel > tol) return fail(SLP_EINVAL, "no convergence in %d iterations (relative residual %g > %g)",
                             max_iter, rel, tol);
  return SLP_OK;
}

}  // namespace

extern "C" {

int slp_fem_setup(slp_fem **out, const double *nodes, int64_t n_nodes, const int32_t *tets,
                  int64_t n_tets, void *stream) {
  return fem_setup_impl(out, nodes, n_nodes, tets, n_tets, static_cast<hipStream_t>(stream));
}

int slp_fem_info(const slp_fem *F, int64_t *n_free, int64_t *n_boundary_tris, int64_t *nnz,
                 int64_t *device_bytes) {
  if (!F) return fail(SLP_EINVAL, "NULL context");
  if (n_free) *n_free = F->n_free;
  if (n_boundary_tris) *n_boundary_tris = F->n_btris;
  if (nnz) *nnz = F->nnz;
  if (device_bytes) *device_bytes = F->bytes;
  return SLP_OK;
}

int slp_fem_boundary(const slp_fem *F, int32_t *tris, int64_t cap) {
  if (!F || !tris) return fail(SLP_EINVAL, "NULL argument");
  if (cap < F->n_btris) return fail(SLP_EINVAL, "tris holds %lld triangles, need %lld", (long long)cap,
                                    (long long)F->n_btris);
  std::copy(F->h_btris.begin(), F->h_btris.end(), tris);
  return SLP_OK;
}

int slp_fem_solve_phi1(slp_fem *F, const double *m_nodes, double *phi1, double tol,
                       int32_t max_iter, int32_t warm_start, int32_t *iters, double *rel_res,
                       void *stream) {
  return solve_impl(F, m_nodes, phi1, tol, max_iter, warm_start, iters, rel_res,
                    static_cast<hipStream_t>(stream));
}

int slp_fem_set_preconditioner(slp_fem *F, int32_t kind, void *stream) {
  if (!F) return fail(SLP_EINVAL, "NULL context");
  if (kind != SLP_PRECOND_JACOBI && kind != SLP_PRECOND_AMG)
    return fail(SLP_EINVAL, "unknown preconditioner %d", (int)kind);
  if (kind == SLP_PRECOND_AMG && F->n_free > 0) {
    const int rc = build_amg_impl(F, static_cast<hipStream_t>(stream));
    if (rc) return rc;
  }
  F->precond = kind;
  return SLP_OK;
}

int slp_fem_assemble_host(const double *nodes, int64_t n_nodes, const int32_t *tets,
                          int64_t n_tets, int64_t *n_free, int64_t *nnz, int64_t *rowptr,
                          int32_t *cols, double *vals, int32_t *free_nodes) {
  if (!n_free || !nnz) return fail(SLP_EINVAL, "n_free and nnz must be non-NULL");
  HostAssembly h;
  const int rc = fem_setup_impl(nullptr, nodes, n_nodes, tets, n_tets, nullptr, &h);
  if (rc) return rc;
  *n_free = (int64_t)h.free_node.size();
  *nnz = (int64_t)h.ci.size();
  if (rowptr)
    for (size_t i = 0; i < h.rp.size(); ++i) rowptr[i] = h.rp[i];
  if (cols) std::copy(h.ci.begin(), h.ci.end(), cols);
  if (vals) std::copy(h.val.begin(), h.val.end(), vals);
  if (free_nodes) std::copy(h.free_node.begin(), h.free_node.end(), free_nodes);
  return SLP_OK;
}

int slp_amg_apply_host(int64_t n, const int64_t *rowptr, const int32_t *cols, const double *vals,
                       const double *r, double *z, int32_t *n_levels) {
  if (n <= 0 || !rowptr || !cols || !vals || !r || !z) return fail(SLP_EINVAL, "NULL argument or n <= 0");
  if (rowptr[0] != 0 || rowptr[n] > INT32_MAX) return fail(SLP_EINVAL, "rowptr must start at 0 and fit 32 bits");
  slp::HostCsr A;
  A.rows = A.cols = n;
  A.rp.resize(n + 1);
  for (int64_t i = 0; i <= n; ++i) {
    if (i > 0 && rowptr[i] < rowptr[i - 1]) return fail(SLP_EINVAL, "rowptr decreases at %lld", (long long)i);
    A.rp[i] = (int32_t)rowptr[i];
  }
  A.ci.assign(cols, cols + rowptr[n]);
  A.v.assign(vals, vals + rowptr[n]);
  for (int32_t c : A.ci)
    if (c < 0 || c >= n) return fail(SLP_EINVAL, "column %d out of range", (int)c);
  slp::AmgHierarchy h;
  char err[256] = {0};
  try {
    if (!slp::build_amg(A, slp::AmgParams(), h, err, sizeof err))
      return fail(SLP_EINVAL, "multigrid setup: %s", err);
    slp::amg_apply_host(h, r, z);
  } catch (const std::bad_alloc &) {
    return fail(SLP_ENOMEM, "host allocation failed while building the multigrid hierarchy");
  }
  if (n_levels) *n_levels = (int32_t)h.levels.size() + 1;
  return SLP_OK;
}

int slp_fem_amg_info(const slp_fem *F, int32_t *n_levels, int64_t *rows, int64_t *nnz, int32_t cap) {
  if (!F || !n_levels) return fail(SLP_EINVAL, "NULL argument");
  if (!F->amg_built) return fail(SLP_EINVAL, "no multigrid hierarchy (select SLP_PRECOND_AMG first)");
  const int32_t nl = (int32_t)F->amg.size() + 1;
  *n_levels = nl;
  if (cap < nl && (rows || nnz)) return fail(SLP_EINVAL, "cap %d < %d levels", (int)cap, (int)nl);
  for (int32_t l = 0; l < nl; ++l) {
    const bool last = l + 1 == nl;
    if (rows) rows[l] = last ? F->amg_coarse.rows : F->amg[l].n;
    if (nnz) nnz[l] = last ? F->amg_coarse.nnz : (l == 0 ? F->nnz : F->amg[l].A.nnz);
  }
  return SLP_OK;
}

int slp_fem_dphi1_dn(slp_fem *F, const double *phi1, double *dphi1_dn, void *stream) {
  if (!F || !phi1 || !dphi1_dn) return fail(SLP_EINVAL, "NULL argument");
  FEM_TRY(slp::launch_fem_dn(F->owner, F->nrm, F->tets, F->grad, phi1, dphi1_dn, F->n_btris,
                             static_cast<hipStream_t>(stream)));
  return SLP_OK;
}

int slp_scalar_potential(slp_fem *F, slp_geom *g, const double *m_nodes, double *phi, double tol,
                         int32_t max_iter, int32_t warm_start, int32_t *iters, void *stream) {
  if (!F || !g || !m_nodes || !phi) return fail(SLP_EINVAL, "NULL argument");
  slp_geom_info gi;
  int rc = slp_geom_get_info(g, &gi);
  if (rc) return rc;
  if (gi.n_nodes != F->n_nodes || gi.n_tris != F->n_btris || gi.n_targets != F->n_nodes)
    return fail(SLP_EINVAL, "the geometry must hold the mesh's nodes (also as targets) and its "
                            "boundary triangles from slp_fem_boundary");
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = solve_impl(F, m_nodes, F->phi1, tol, max_iter, warm_start, iters, nullptr, st);
  if (rc) return rc;
  FEM_TRY(slp::launch_fem_dn(F->owner, F->nrm, F->tets, F->grad, F->phi1, F->dn, F->n_btris, st));
  rc = slp_set_density_from_m(g, m_nodes, F->dn, stream);
  if (rc) return rc;
  rc = slp_eval_single_layer(g, phi, stream);
  if (rc) return rc;
  FEM_TRY(slp::launch_fem_add(phi, F->phi1, F->n_nodes, st));
  return SLP_OK;
}

int slp_fem_energy(slp_fem *F, const double *m_nodes, const double *phi, double *energy,
                   void *stream) {
  if (!F || !m_nodes || !phi || !energy) return fail(SLP_EINVAL, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nb = (F->n_tets + slp::kFemThreads - 1) / slp::kFemThreads;
  FEM_TRY(slp::launch_fem_energy(F->tets, F->vol, F->grad, m_nodes, phi, F->epart, F->epart + nb,
                                 F->n_tets, st));
  FEM_TRY(hipMemcpyAsync(F->h_pin, F->epart + nb, 8, hipMemcpyDeviceToHost, st));
  FEM_TRY(hipStreamSynchronize(st));
  *energy = 0.5 * F->h_pin[0];
  return SLP_OK;
}

int slp_fem_destroy(slp_fem *F) {
  if (!F) return SLP_OK;
  (void)hipDeviceSynchronize();
  delete F;
  return SLP_OK;
}

}  // extern "C"
