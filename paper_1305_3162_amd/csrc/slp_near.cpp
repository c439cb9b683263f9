// Host side of the near-field correction (Sec. 3.4): index sets of eq.
// (nf_index) and the radius from which the truncated exponential sum matches
// the Newton kernel.
#include "slp_near.hpp"

#include <algorithm>
#include <cmath>
#include <new>
#include <thread>

namespace slp {

bool build_near_pattern(const double *nodes, int64_t n_nodes, const int32_t *tris, int64_t M,
                        const double *tg, int64_t P, double eps, int threads,
                        std::vector<int64_t> &rowptr, std::vector<int32_t> &cols, std::string &err) {
  (void)n_nodes;
  try {
    // centroids, radii about them, cell grid over the centroids
    std::vector<double> cen(3 * M), rad(M);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double rmax = 0.0;
    for (int64_t j = 0; j < M; ++j) {
      const double *v[3] = {nodes + 3 * (int64_t)tris[3 * j], nodes + 3 * (int64_t)tris[3 * j + 1],
                            nodes + 3 * (int64_t)tris[3 * j + 2]};
      for (int q = 0; q < 3; ++q) {
        cen[3 * j + q] = (v[0][q] + v[1][q] + v[2][q]) / 3.0;
        lo[q] = std::min(lo[q], cen[3 * j + q]);
        hi[q] = std::max(hi[q], cen[3 * j + q]);
      }
      double r2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int q = 0; q < 3; ++q) s += (v[k][q] - cen[3 * j + q]) * (v[k][q] - cen[3 * j + q]);
        r2 = std::max(r2, s);
      }
      rad[j] = std::sqrt(r2);
      rmax = std::max(rmax, rad[j]);
    }
    const double reach = eps + rmax;
    double h = 0.5 * reach;
    int64_t dims[3];
    for (;;) {
      int64_t tot = 1;
      for (int q = 0; q < 3; ++q) {
        dims[q] = std::max<int64_t>(1, (int64_t)std::floor((hi[q] - lo[q]) / h) + 1);
        tot *= dims[q];
      }
      if (tot <= (int64_t)1 << 22) break;
      h *= 1.5;
    }
    auto cell_of = [&](const double *y, int64_t *ci) {
      for (int q = 0; q < 3; ++q)
        ci[q] = std::min<int64_t>(dims[q] - 1, std::max<int64_t>(0, (int64_t)std::floor((y[q] - lo[q]) / h)));
    };
    const int64_t ncell = dims[0] * dims[1] * dims[2];
    std::vector<int64_t> start(ncell + 1, 0);
    std::vector<int32_t> member(M);
    std::vector<int64_t> key(M);
    for (int64_t j = 0; j < M; ++j) {
      int64_t ci[3];
      cell_of(&cen[3 * j], ci);
      key[j] = (ci[2] * dims[1] + ci[1]) * dims[0] + ci[0];
      start[key[j] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    {
      std::vector<int64_t> fill(start.begin(), start.end() - 1);
      for (int64_t j = 0; j < M; ++j) member[fill[key[j]]++] = (int32_t)j;
    }

    // rows, split into contiguous target ranges, one per thread
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(threads, P));
    std::vector<std::vector<int32_t>> part(T);
    std::vector<int64_t> count(P, 0);
    std::vector<std::string> perr(T);
    auto work = [&](int w) {
      try {
        const int64_t i0 = P * w / T, i1 = P * (w + 1) / T;
        std::vector<int32_t> row;
        for (int64_t i = i0; i < i1; ++i) {
          const double *x = tg + 3 * i;
          int64_t c0[3], c1[3];
          for (int q = 0; q < 3; ++q) {
            c0[q] = std::max<int64_t>(0, (int64_t)std::floor((x[q] - reach - lo[q]) / h));
            c1[q] = std::min<int64_t>(dims[q] - 1, (int64_t)std::floor((x[q] + reach - lo[q]) / h));
          }
          row.clear();
          for (int64_t cz = c0[2]; cz <= c1[2]; ++cz)
            for (int64_t cy = c0[1]; cy <= c1[1]; ++cy)
              for (int64_t cx = c0[0]; cx <= c1[0]; ++cx) {
                const int64_t c = (cz * dims[1] + cy) * dims[0] + cx;
                for (int64_t k = start[c]; k < start[c + 1]; ++k) {
                  const int32_t j = member[k];
                  const double *cj = &cen[3 * (int64_t)j];
                  const double dc = std::sqrt((x[0] - cj[0]) * (x[0] - cj[0]) + (x[1] - cj[1]) * (x[1] - cj[1]) +
                                              (x[2] - cj[2]) * (x[2] - cj[2]));
                  if (dc > eps + rad[j]) continue;
                  if (dc > eps) {
                    const double *a = nodes + 3 * (int64_t)tris[3 * (int64_t)j];
                    const double *b = nodes + 3 * (int64_t)tris[3 * (int64_t)j + 1];
                    const double *cc = nodes + 3 * (int64_t)tris[3 * (int64_t)j + 2];
                    if (point_triangle_distance(x, a, b, cc) > eps) continue;
                  }
                  row.push_back(j);
                }
              }
          std::sort(row.begin(), row.end());
          count[i] = (int64_t)row.size();
          part[w].insert(part[w].end(), row.begin(), row.end());
        }
      } catch (const std::bad_alloc &) {
        perr[w] = "host allocation failed while building the near-field pattern";
      }
    };
    std::vector<std::thread> pool;
    for (int w = 1; w < T; ++w) pool.emplace_back(work, w);
    work(0);
    for (std::thread &t : pool) t.join();
    for (const std::string &e : perr)
      if (!e.empty()) { err = e; return false; }
    rowptr.assign(P + 1, 0);
    for (int64_t i = 0; i < P; ++i) rowptr[i + 1] = rowptr[i] + count[i];
    cols.resize(rowptr[P]);
    for (int w = 0; w < T; ++w) {
      const int64_t i0 = P * w / T;
      std::copy(part[w].begin(), part[w].end(), cols.begin() + rowptr[i0]);
      std::vector<int32_t>().swap(part[w]);
    }
    return true;
  } catch (const std::bad_alloc &) {
    err = "host allocation failed while building the near-field pattern";
    return false;
  }
}

double near_radius(const double *w, const double *g, int terms, double r_max, double tol) {
  double last = -1.0;
  for (double r = r_max; r > 1e-6 * r_max; r *= 0.999) {
    double s = 0.0;
    for (int t = 0; t < terms; ++t) s += w[t] * std::exp(-g[t] * r * r);
    if (std::fabs(s * r - 1.0) <= tol)
      last = r;
    else
      break;
  }
  return last;
}

}  // namespace slp
