// The library's host-only logic, built with the address and
// undefined-behaviour sanitizers (the host sources; device code is compiled
// as usual and never launched here), run on inputs of the benchmark's sizes:
//   - the gridding and interpolation tables of slp_setup_geometry (binning,
//     segments, chunks, runs, tile boxes; its host-only dry run
//     slp_geometry_device_bytes) for the 64-cell cube at every cut-off and
//     the 1024 x 1024 x 64 film, both windows and precisions;
//   - the near-field index sets (slp_near_pattern_host) and radius scan;
//   - the FEM mesh analysis and stiffness assembly (slp_fem_assemble_host) of
//     the 32-cell tetrahedral cube, and the multigrid hierarchy built from it
//     with one cycle applied on the host (slp_amg_apply_host);
//   - the exponential sum, the window choice and the closed-form triangle
//     potential.
// Meshes are generated here (a structured box surface and its tetrahedral
// lattice). Prints "ALL OK"; exits non-zero on a failed check (the sanitizers
// abort on their own findings).
#include "slp.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "CHECK failed: %s (line %d): %s\n", #c, __LINE__, slp_last_error()); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

// Surface of the box [-e/2, e/2] with c[q] cells along axis q, two triangles
// per face cell.
static void box_surface(const double e[3], const int c[3], std::vector<double> &nodes,
                        std::vector<int32_t> &tris) {
  const int nx = c[0] + 1, ny = c[1] + 1, nz = c[2] + 1;
  std::vector<int32_t> id((size_t)nx * ny * nz, -1);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        if (!(i == 0 || j == 0 || k == 0 || i == c[0] || j == c[1] || k == c[2])) continue;
        id[((size_t)k * ny + j) * nx + i] = (int32_t)(nodes.size() / 3);
        nodes.push_back((double(i) / c[0] - 0.5) * e[0]);
        nodes.push_back((double(j) / c[1] - 0.5) * e[1]);
        nodes.push_back((double(k) / c[2] - 0.5) * e[2]);
      }
  auto at = [&](int i, int j, int k) { return id[((size_t)k * ny + j) * nx + i]; };
  for (int a = 0; a < 3; ++a) {
    const int u = (a + 1) % 3, v = (a + 2) % 3;
    for (int side = 0; side < 2; ++side)
      for (int p = 0; p < c[u]; ++p)
        for (int q = 0; q < c[v]; ++q) {
          int ijk[4][3];
          const int du[4] = {0, 1, 1, 0}, dv[4] = {0, 0, 1, 1};
          for (int t = 0; t < 4; ++t) {
            ijk[t][a] = side ? c[a] : 0;
            ijk[t][u] = p + du[t];
            ijk[t][v] = q + dv[t];
          }
          int32_t w[4];
          for (int t = 0; t < 4; ++t) w[t] = at(ijk[t][0], ijk[t][1], ijk[t][2]);
          const int32_t t1[3] = {w[0], w[1], w[2]}, t2[3] = {w[0], w[2], w[3]};
          for (int t = 0; t < 3; ++t) tris.push_back(side ? t1[t] : t1[2 - t]);
          for (int t = 0; t < 3; ++t) tris.push_back(side ? t2[t] : t2[2 - t]);
        }
  }
}

// The (c+1)^3 lattice of the unit cube, six tetrahedra per cell around the
// cell's main diagonal.
static void cube_tets(int c, std::vector<double> &nodes, std::vector<int32_t> &tets) {
  const int n = c + 1;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        nodes.push_back(double(i) / c - 0.5);
        nodes.push_back(double(j) / c - 0.5);
        nodes.push_back(double(k) / c - 0.5);
      }
  auto v = [&](int i, int j, int k) { return (int32_t)(((int64_t)k * n + j) * n + i); };
  const int path[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int k = 0; k < c; ++k)
    for (int j = 0; j < c; ++j)
      for (int i = 0; i < c; ++i)
        for (const auto &pp : path) {
          int p[3] = {i, j, k};
          int32_t t[4];
          t[0] = v(p[0], p[1], p[2]);
          for (int s = 0; s < 3; ++s) {
            p[pp[s]] += 1;
            t[s + 1] = v(p[0], p[1], p[2]);
          }
          for (int s = 0; s < 4; ++s) tets.push_back(t[s]);
        }
}

static void expsum(double r_hi, std::vector<double> &w, std::vector<double> &g) {
  int32_t n = 0;
  w.resize(1024);
  g.resize(1024);
  CHECK(slp_expsum_sinc(0.2, 1e-3 * r_hi, r_hi, 1e-12, w.data(), g.data(), 1024, &n) == SLP_OK);
  CHECK(n > 10 && n <= 1024);
  w.resize(n);
  g.resize(n);
}

static int64_t dry_bytes(const std::vector<double> &nodes, const std::vector<int32_t> &tris,
                         const int grid[3], int m, int prec, int window,
                         const std::vector<double> &w, const std::vector<double> &g) {
  slp_params p{};
  for (int q = 0; q < 3; ++q) p.grid[q] = grid[q];
  p.alpha = 2;
  p.m = m;
  p.precision = prec;
  p.es_w = w.data();
  p.es_gamma = g.data();
  p.es_terms = (int32_t)w.size();
  p.window = window;
  p.eta2 = 37.0;
  int64_t b = 0;
  CHECK(slp_geometry_device_bytes(nodes.data(), (int64_t)nodes.size() / 3, tris.data(),
                                  (int64_t)tris.size() / 3, &p, &b) == SLP_OK);
  CHECK(b > 0);
  return b;
}

int main() {
  // gridding / interpolation tables: cube64 (grid 128^3), a 512 x 512 plate
  // (grid 1024 x 1024 x 64), all cut-offs the benchmark uses
  {
    std::vector<double> nodes;
    std::vector<int32_t> tris;
    const double e[3] = {1, 1, 1};
    const int c[3] = {64, 64, 64};
    box_surface(e, c, nodes, tris);
    CHECK(tris.size() / 3 == 49152 && nodes.size() / 3 == 24578);
    std::vector<double> w, g;
    expsum(std::sqrt(3.0), w, g);
    const int grid[3] = {128, 128, 128};
    for (int m = 1; m <= 8; ++m) {
      dry_bytes(nodes, tris, grid, m, SLP_FP64, SLP_WINDOW_GAUSS, w, g);
      dry_bytes(nodes, tris, grid, m, SLP_FP32, SLP_WINDOW_KB, w, g);
    }
    std::printf("OK cube64 tables\n");
  }
  {
    std::vector<double> nodes;
    std::vector<int32_t> tris;
    const double e[3] = {1, 1, 0.02};
    const int c[3] = {512, 512, 10};
    box_surface(e, c, nodes, tris);
    CHECK(tris.size() / 3 == 1089536 && nodes.size() / 3 == 544770);
    std::vector<double> w, g;
    expsum(std::sqrt(2.0 + 0.0004), w, g);
    const int grid[3] = {1024, 1024, 64};
    dry_bytes(nodes, tris, grid, 4, SLP_FP64, SLP_WINDOW_KB, w, g);
    dry_bytes(nodes, tris, grid, 3, SLP_FP32, SLP_WINDOW_KB, w, g);
    std::printf("OK film tables\n");
  }
  // near-field index sets and radius
  {
    std::vector<double> nodes;
    std::vector<int32_t> tris;
    const double e[3] = {1, 1, 1};
    const int c[3] = {16, 16, 16};
    box_surface(e, c, nodes, tris);
    const int64_t nn = (int64_t)nodes.size() / 3, nt = (int64_t)tris.size() / 3;
    int64_t nnz = 0;
    CHECK(slp_near_pattern_host(nodes.data(), nn, tris.data(), nt, nodes.data(), nn, 0.2, nullptr,
                                nullptr, 0, &nnz) == SLP_OK && nnz > 0);
    std::vector<int64_t> rp(nn + 1);
    std::vector<int32_t> cols(nnz);
    CHECK(slp_near_pattern_host(nodes.data(), nn, tris.data(), nt, nodes.data(), nn, 0.2,
                                rp.data(), cols.data(), nnz, &nnz) == SLP_OK);
    CHECK(rp[nn] == nnz);
    for (int64_t i = 0; i < nn; ++i)
      for (int64_t k = rp[i]; k < rp[i + 1]; ++k) CHECK(cols[k] >= 0 && cols[k] < nt);
    std::vector<double> w, g;
    expsum(std::sqrt(3.0), w, g);
    double eps = 0.0;
    CHECK(slp_near_radius_host(w.data(), g.data(), (int32_t)w.size(), std::sqrt(3.0), 1e-3,
                               &eps) == SLP_OK && eps > 0.0);
    const double x[3] = {0.1, 0.2, 0.3}, a[3] = {0, 0, 0}, b[3] = {1, 0, 0}, cc[3] = {0, 1, 0};
    double v = 0.0;
    CHECK(slp_triangle_potential_host(x, a, b, cc, 1, &v) == SLP_OK && v > 0.0);
    std::printf("OK near-field host logic nnz=%lld\n", (long long)nnz);
  }
  // FEM assembly and the multigrid hierarchy with one cycle
  {
    std::vector<double> nodes;
    std::vector<int32_t> tets;
    cube_tets(32, nodes, tets);
    const int64_t nn = (int64_t)nodes.size() / 3, nt = (int64_t)tets.size() / 4;
    int64_t nf = 0, nnz = 0;
    CHECK(slp_fem_assemble_host(nodes.data(), nn, tets.data(), nt, &nf, &nnz, nullptr, nullptr,
                                nullptr, nullptr) == SLP_OK);
    CHECK(nf == 31 * 31 * 31 && nnz > 0);
    std::vector<int64_t> rp(nf + 1);
    std::vector<int32_t> ci(nnz), fn(nf);
    std::vector<double> val(nnz);
    CHECK(slp_fem_assemble_host(nodes.data(), nn, tets.data(), nt, &nf, &nnz, rp.data(), ci.data(),
                                val.data(), fn.data()) == SLP_OK);
    std::vector<double> r(nf, 1.0), z(nf, 0.0);
    int32_t levels = 0;
    CHECK(slp_amg_apply_host(nf, rp.data(), ci.data(), val.data(), r.data(), z.data(), &levels) ==
          SLP_OK);
    CHECK(levels >= 2);
    double rz = 0.0;
    for (int64_t i = 0; i < nf; ++i) rz += r[i] * z[i];
    CHECK(rz > 0.0);   // the cycle is positive definite
    std::printf("OK fem assembly and multigrid cycle (levels %d)\n", levels);
  }
  {
    int32_t win = 0, m = 0;
    CHECK(slp_choose_cutoff(1e-6, SLP_FP64, -1, &win, &m) == SLP_OK && m >= 1 && m <= 8);
    CHECK(slp_choose_cutoff(1e-4, SLP_FP32, SLP_WINDOW_GAUSS, &win, &m) == SLP_OK);
  }
  std::printf("ALL OK\n");
  return 0;
}
