// Smoothed-aggregation hierarchy (Vanek, Mandel and Brezina, Computing 56
// (1996)) of the free-node stiffness matrix: strength of connection,
// aggregation in three passes, tentative prolongation by the constant vector
// on each aggregate, one damped-Jacobi smoothing step of it with the l1
// weights of Baker, Falgout, Kolev and Yang (SIAM J. Sci. Comput. 33 (2011)),
// Galerkin coarse operators R A P with R = P^T, and the dense inverse of the
// coarsest operator.
#include "slp_amg.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <limits>

namespace slp {

namespace {

bool failf(char *err, size_t errlen, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  if (err && errlen) vsnprintf(err, errlen, fmt, ap);
  va_end(ap);
  return false;
}

// Diagonal of a square CSR matrix (0 where a row holds none).
std::vector<double> diagonal(const HostCsr &A) {
  std::vector<double> d(A.rows, 0.0);
  for (int64_t i = 0; i < A.rows; ++i)
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e)
      if (A.ci[e] == i) d[i] += A.v[e];
  return d;
}

// Aggregates of the strongly connected neighbourhoods: j is a strong
// neighbour of i if |a_ij| >= theta sqrt(a_ii a_jj). Pass 1 takes every node
// whose strong neighbours are all still free, together with them; pass 2 adds
// each remaining node to the pass-1 aggregate of its strongest aggregated
// neighbour; pass 3 groups what is left with its free strong neighbours
// (isolated nodes become aggregates of their own). Returns the count.
int64_t aggregate(const HostCsr &A, const std::vector<double> &d, double theta,
                  std::vector<int32_t> &agg) {
  const int64_t n = A.rows;
  std::vector<int32_t> sp(n + 1, 0), sc;
  std::vector<double> sv;
  sc.reserve(A.ci.size());
  sv.reserve(A.ci.size());
  for (int64_t i = 0; i < n; ++i) {
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int32_t j = A.ci[e];
      const double a = std::fabs(A.v[e]);
      if (j != i && a >= theta * std::sqrt(std::fabs(d[i] * d[j]))) {
        sc.push_back(j);
        sv.push_back(a);
      }
    }
    sp[i + 1] = (int32_t)sc.size();
  }
  agg.assign(n, -1);
  int32_t na = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0 || sp[i] == sp[i + 1]) continue;
    bool free_nbhd = true;
    for (int32_t e = sp[i]; e < sp[i + 1] && free_nbhd; ++e) free_nbhd = agg[sc[e]] < 0;
    if (!free_nbhd) continue;
    agg[i] = na;
    for (int32_t e = sp[i]; e < sp[i + 1]; ++e) agg[sc[e]] = na;
    ++na;
  }
  std::vector<int32_t> join(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    double best = -1.0;
    for (int32_t e = sp[i]; e < sp[i + 1]; ++e)
      if (agg[sc[e]] >= 0 && sv[e] > best) {
        best = sv[e];
        join[i] = agg[sc[e]];
      }
  }
  for (int64_t i = 0; i < n; ++i)
    if (join[i] >= 0) agg[i] = join[i];
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int32_t e = sp[i]; e < sp[i + 1]; ++e)
      if (agg[sc[e]] < 0) agg[sc[e]] = na;
    ++na;
  }
  return na;
}

// P = (I - W A) T: T the 0/1 aggregate matrix, W = diag(w).
HostCsr smoothed_prolongation(const HostCsr &A, const std::vector<double> &w,
                              const std::vector<int32_t> &agg, int64_t na) {
  HostCsr P;
  P.rows = A.rows;
  P.cols = na;
  P.rp.assign(A.rows + 1, 0);
  std::vector<int32_t> pos(na, -1);
  for (int64_t i = 0; i < A.rows; ++i) {
    const size_t start = P.ci.size();
    auto add = [&](int32_t a, double x) {
      if (pos[a] < 0) {
        pos[a] = (int32_t)P.ci.size();
        P.ci.push_back(a);
        P.v.push_back(x);
      } else {
        P.v[pos[a]] += x;
      }
    };
    add(agg[i], 1.0);
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) add(agg[A.ci[e]], -w[i] * A.v[e]);
    for (size_t k = start; k < P.ci.size(); ++k) pos[P.ci[k]] = -1;
    P.rp[i + 1] = (int32_t)P.ci.size();
  }
  return P;
}

HostCsr transpose(const HostCsr &M) {
  HostCsr T;
  T.rows = M.cols;
  T.cols = M.rows;
  T.rp.assign(M.cols + 1, 0);
  for (int32_t c : M.ci) T.rp[c + 1] += 1;
  for (int64_t c = 0; c < M.cols; ++c) T.rp[c + 1] += T.rp[c];
  T.ci.resize(M.ci.size());
  T.v.resize(M.v.size());
  std::vector<int32_t> fill(T.rp.begin(), T.rp.end() - 1);
  for (int64_t i = 0; i < M.rows; ++i)
    for (int32_t e = M.rp[i]; e < M.rp[i + 1]; ++e) {
      const int32_t k = fill[M.ci[e]]++;
      T.ci[k] = (int32_t)i;
      T.v[k] = M.v[e];
    }
  return T;
}

// C = X Y, row by row with a position marker over the columns of Y.
bool multiply(const HostCsr &X, const HostCsr &Y, HostCsr &C, char *err, size_t errlen) {
  C = HostCsr();
  C.rows = X.rows;
  C.cols = Y.cols;
  C.rp.assign(X.rows + 1, 0);
  std::vector<int64_t> pos(Y.cols, -1);
  for (int64_t i = 0; i < X.rows; ++i) {
    const size_t start = C.ci.size();
    for (int32_t e = X.rp[i]; e < X.rp[i + 1]; ++e) {
      const int32_t k = X.ci[e];
      const double x = X.v[e];
      for (int32_t f = Y.rp[k]; f < Y.rp[k + 1]; ++f) {
        const int32_t j = Y.ci[f];
        if (pos[j] < 0) {
          pos[j] = (int64_t)C.ci.size();
          C.ci.push_back(j);
          C.v.push_back(x * Y.v[f]);
        } else {
          C.v[pos[j]] += x * Y.v[f];
        }
      }
    }
    for (size_t k = start; k < C.ci.size(); ++k) pos[C.ci[k]] = -1;
    if (C.ci.size() > (size_t)std::numeric_limits<int32_t>::max())
      return failf(err, errlen, "coarse operator too large for 32-bit offsets");
    C.rp[i + 1] = (int32_t)C.ci.size();
  }
  return true;
}

// Inverse of the symmetric positive definite matrix A (symmetrised against
// rounding) through its Cholesky factor: A^-1 = L^-T L^-1.
bool dense_inverse(const HostCsr &A, std::vector<double> &inv, char *err, size_t errlen) {
  const int64_t n = A.rows;
  std::vector<double> L(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      L[i * n + A.ci[e]] += 0.5 * A.v[e];
      L[A.ci[e] * n + i] += 0.5 * A.v[e];
    }
  for (int64_t j = 0; j < n; ++j) {
    double s = L[j * n + j];
    for (int64_t k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0)) return failf(err, errlen, "coarsest operator is not positive definite (pivot %lld)", (long long)j);
    const double ljj = std::sqrt(s);
    L[j * n + j] = ljj;
    for (int64_t i = j + 1; i < n; ++i) {
      double t = L[i * n + j];
      for (int64_t k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / ljj;
    }
    for (int64_t i = 0; i < j; ++i) L[i * n + j] = 0.0;
  }
  // M = L^-1, lower triangular, column by column
  std::vector<double> M(n * n, 0.0);
  for (int64_t c = 0; c < n; ++c) {
    M[c * n + c] = 1.0 / L[c * n + c];
    for (int64_t i = c + 1; i < n; ++i) {
      double t = 0.0;
      for (int64_t k = c; k < i; ++k) t -= L[i * n + k] * M[k * n + c];
      M[i * n + c] = t / L[i * n + i];
    }
  }
  inv.assign(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      double t = 0.0;
      for (int64_t k = i; k < n; ++k) t += M[k * n + i] * M[k * n + j];
      inv[i * n + j] = t;
      inv[j * n + i] = t;
    }
  return true;
}

}  // namespace

bool build_amg(const HostCsr &A, const AmgParams &prm, AmgHierarchy &h, char *err, size_t errlen) {
  h = AmgHierarchy();
  constexpr int64_t kDenseLimit = 1024;   // coarsest size accepted when the coarsening stalls
  HostCsr cur = A;
  double theta = prm.theta;
  while (cur.rows > prm.max_coarse) {
    const std::vector<double> d = diagonal(cur);
    // l1-Jacobi weights w_i = (4/3) / sum_j |a_ij|: the spectrum of W A lies in
    // (0, 4/3], so the smoother converges, and each row is damped by its own
    // off-diagonal mass (distorted elements do not slow the others down)
    std::vector<double> w(cur.rows);
    for (int64_t i = 0; i < cur.rows; ++i) {
      if (!(d[i] > 0.0)) return failf(err, errlen, "non-positive diagonal entry in row %lld", (long long)i);
      double s = 0.0;
      for (int32_t e = cur.rp[i]; e < cur.rp[i + 1]; ++e) s += std::fabs(cur.v[e]);
      w[i] = 4.0 / (3.0 * s);
    }
    std::vector<int32_t> agg;
    const int64_t na = aggregate(cur, d, theta, agg);
    if ((int)h.levels.size() + 1 >= prm.max_levels || 10 * na > 9 * cur.rows) {
      if (cur.rows <= kDenseLimit) break;
      return failf(err, errlen, "aggregation stalled at %lld unknowns", (long long)cur.rows);
    }
    AmgLevel L;
    L.P = smoothed_prolongation(cur, w, agg, na);
    L.R = transpose(L.P);
    HostCsr AP, Ac;
    if (!multiply(cur, L.P, AP, err, errlen) || !multiply(L.R, AP, Ac, err, errlen)) return false;
    L.w = std::move(w);
    L.A = std::move(cur);
    h.levels.push_back(std::move(L));
    cur = std::move(Ac);
    theta *= 0.5;
  }
  h.nc = cur.rows;
  if (h.nc > 0 && !dense_inverse(cur, h.coarse_inv, err, errlen)) return false;
  return true;
}

namespace {

void spmv(const HostCsr &M, const double *x, double *y) {
  for (int64_t i = 0; i < M.rows; ++i) {
    double t = 0.0;
    for (int32_t e = M.rp[i]; e < M.rp[i + 1]; ++e) t += M.v[e] * x[M.ci[e]];
    y[i] = t;
  }
}

void cycle(const AmgHierarchy &h, size_t l, const double *f, double *out) {
  if (l == h.levels.size()) {
    const int64_t n = h.nc;
    for (int64_t i = 0; i < n; ++i) {
      double t = 0.0;
      for (int64_t j = 0; j < n; ++j) t += h.coarse_inv[i * n + j] * f[j];
      out[i] = t;
    }
    return;
  }
  const AmgLevel &L = h.levels[l];
  const int64_t n = L.A.rows, nc = L.P.cols;
  std::vector<double> x(n), t(n), fc(nc), e(nc);
  for (int64_t i = 0; i < n; ++i) x[i] = L.w[i] * f[i];
  spmv(L.A, x.data(), t.data());
  for (int64_t i = 0; i < n; ++i) t[i] = f[i] - t[i];
  spmv(L.R, t.data(), fc.data());
  cycle(h, l + 1, fc.data(), e.data());
  spmv(L.P, e.data(), t.data());
  for (int64_t i = 0; i < n; ++i) x[i] += t[i];
  spmv(L.A, x.data(), t.data());
  for (int64_t i = 0; i < n; ++i) out[i] = x[i] + L.w[i] * (f[i] - t[i]);
}

}  // namespace

void amg_apply_host(const AmgHierarchy &h, const double *r, double *z) { cycle(h, 0, r, z); }

}  // namespace slp
