// Near-field correction (Sec. 3.4): closed-form integral of the Newton kernel
// over a flat triangle (host and device), and the host-side construction of
// the index sets of eq. (nf_index). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

namespace slp {

// int_T dsigma(y) / |x - y| over the flat triangle T = (a, b, c), exact.
//
// With n the unit normal, d = n.(x - a) the signed height of x and p its foot
// point in the plane, T is the signed sum of the three triangles (p, u, v) over
// its edges (u, v). For one edge, with e the unit edge direction, t the signed
// in-plane distance of p from the edge line (> 0 when p is on the interior
// side), s the coordinate along the line measured from the foot of p and
// rho^2 = t^2 + d^2, R(s) = sqrt(s^2 + rho^2), polar coordinates about p give
//   sign(t) * [ |t| asinh(s / rho) + |d| atan(|d| s / (|t| R)) - |d| atan(s / |t|) ]
// between the edge's end points s_u < s_v. Edges whose line passes through p
// contribute nothing. The difference of the two asinh values is formed without
// cancellation when s_u and s_v have the same sign:
//   asinh(x) - asinh(y) = asinh((s_v^2 - s_u^2) / (s_v R_u + s_u R_v)).
__host__ __device__ inline double triangle_potential(const double x[3], const double a[3],
                                                     const double b[3], const double c[3]) {
  double e1[3], e2[3], n[3];
  for (int q = 0; q < 3; ++q) { e1[q] = b[q] - a[q]; e2[q] = c[q] - a[q]; }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int q = 0; q < 3; ++q) n[q] /= nn;
  const double d = (x[0] - a[0]) * n[0] + (x[1] - a[1]) * n[1] + (x[2] - a[2]) * n[2];
  const double ad = fabs(d);
  double p[3];
  for (int q = 0; q < 3; ++q) p[q] = x[q] - d * n[q];
  const double *V[4] = {a, b, c, a};
  double len[3], scale = 0.0;
  for (int k = 0; k < 3; ++k) {
    double l2 = 0.0;
    for (int q = 0; q < 3; ++q) l2 += (V[k + 1][q] - V[k][q]) * (V[k + 1][q] - V[k][q]);
    len[k] = sqrt(l2);
    scale = fmax(scale, len[k]);
  }
  double total = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double *u = V[k], *v = V[k + 1];
    double e[3];
    for (int q = 0; q < 3; ++q) e[q] = (v[q] - u[q]) / len[k];
    // outward in-plane normal of the edge: e x n
    const double o[3] = {e[1] * n[2] - e[2] * n[1], e[2] * n[0] - e[0] * n[2], e[0] * n[1] - e[1] * n[0]};
    double t = 0.0, su = 0.0, sv = 0.0;
    for (int q = 0; q < 3; ++q) {
      t += (u[q] - p[q]) * o[q];
      su += (u[q] - p[q]) * e[q];
      sv += (v[q] - p[q]) * e[q];
    }
    const double at = fabs(t);
    if (!(at > 1e-14 * scale)) continue;
    const double rho2 = at * at + d * d;
    const double rho = sqrt(rho2);
    const double Ru = sqrt(su * su + rho2), Rv = sqrt(sv * sv + rho2);
    const double das = (su * sv > 0.0) ? asinh((sv - su) * (sv + su) / (sv * Ru + su * Rv))
                                       : asinh(sv / rho) - asinh(su / rho);
    const double ang = atan2(ad * sv, at * Rv) - atan2(ad * su, at * Ru) - atan2(sv, at) + atan2(su, at);
    const double J = at * das + ad * ang;
    total += (t > 0.0) ? J : -J;
  }
  return total;
}

// Distance from x to the closest point of the triangle (a, b, c): the closest
// point is found by classifying x against the vertex, edge and face regions
// of the triangle with the dot products of x - vertex with the two edge
// vectors (the face region yields barycentric coordinates of the foot point).
// This is the published Voronoi-region test of C. Ericson, Real-Time
// Collision Detection (Morgan Kaufmann, 2005), Sec. 5.1.5, written here from
// its description.
inline double point_triangle_distance(const double x[3], const double a[3], const double b[3],
                                      const double c[3]) {
  double ab[3], ac[3], ap[3], bp[3], cp[3];
  for (int q = 0; q < 3; ++q) {
    ab[q] = b[q] - a[q]; ac[q] = c[q] - a[q];
    ap[q] = x[q] - a[q]; bp[q] = x[q] - b[q]; cp[q] = x[q] - c[q];
  }
  auto dot = [](const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
  double y[3];
  auto at = [&](const double *base, const double *dir, double f) {
    for (int q = 0; q < 3; ++q) y[q] = base[q] + f * dir[q];
  };
  const double d1 = dot(ab, ap), d2 = dot(ac, ap);
  const double d3 = dot(ab, bp), d4 = dot(ac, bp);
  const double d5 = dot(ab, cp), d6 = dot(ac, cp);
  const double vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
  if (d1 <= 0.0 && d2 <= 0.0) {
    at(a, ab, 0.0);
  } else if (d3 >= 0.0 && d4 <= d3) {
    at(b, ab, 0.0);
  } else if (d6 >= 0.0 && d5 <= d6) {
    at(c, ab, 0.0);
  } else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
    at(a, ab, d1 / (d1 - d3));
  } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
    at(a, ac, d2 / (d2 - d6));
  } else if (va <= 0.0 && d4 - d3 >= 0.0 && d5 - d6 >= 0.0) {
    const double bc[3] = {c[0] - b[0], c[1] - b[1], c[2] - b[2]};
    at(b, bc, (d4 - d3) / ((d4 - d3) + (d5 - d6)));
  } else {
    const double den = 1.0 / (va + vb + vc);
    const double v = vb * den, w = vc * den;
    for (int q = 0; q < 3; ++q) y[q] = a[q] + v * ab[q] + w * ac[q];
  }
  const double r[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
  return std::sqrt(dot(r, r));
}

// CSR pattern of the near field: row i lists, in increasing order, the
// triangles j with distance(x_i, S_j) <= eps. Candidates come from a uniform
// cell grid over the triangle centroids; a triangle is accepted at once when
// its centroid is within eps, rejected when the centroid is further than eps
// plus the triangle's radius about it, and decided by the exact distance
// otherwise. Runs on up to `threads` host threads. Returns false (with a
// message) when the host runs out of memory.
bool build_near_pattern(const double *nodes, int64_t n_nodes, const int32_t *tris, int64_t n_tris,
                        const double *targets, int64_t n_targets, double eps, int threads,
                        std::vector<int64_t> &rowptr, std::vector<int32_t> &cols, std::string &err);

// Smallest radius on the scan r_k = r_max 0.999^k (k = 0, 1, ...) from which
// up to r_max the exponential sum sum_t w_t exp(-g_t r^2) matches 1/r to
// relative accuracy tol at every scan point; -1 if r_max itself fails.
double near_radius(const double *w, const double *g, int terms, double r_max, double tol);

}  // namespace slp
