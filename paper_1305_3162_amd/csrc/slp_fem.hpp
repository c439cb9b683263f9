// Device side of the Dirichlet problem for phi_1 (Sec. 2.1) and the complete
// scalar potential of Alg. 1. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace slp {

constexpr int kFemThreads = 256;

// Load vector on the free nodes: b_f = sum over the tetrahedra T holding node
// free_node[f] (local index a) of |T| mbar_T . grad lambda_a^T.
struct FemLoadArgs {
  const int32_t *inc_ptr;   // [Nf + 1]
  const int32_t *inc;       // 4 T + a
  const int32_t *tets;      // [T][4]
  const double *vol;        // [T]
  const double *grad;       // [T][4][3]
  const double *m;          // [N][3] nodal magnetisation
  double *b;                // [Nf]
  int64_t nf;
};
hipError_t launch_fem_load(const FemLoadArgs &a, hipStream_t s);

// Preconditioned conjugate gradients (Jacobi) on S_ff x = b. Partial sums
// of the dot products are written per workgroup; every consumer sums them.
struct PcgArgs {
  const int32_t *rp, *ci;   // CSR of S_ff
  const double *val;
  const double *dinv;       // 1 / diag(S_ff)
  const double *b;
  double *x, *r, *z, *p, *q;
  double *part;             // [5][nblk]: p.q, r.z (two slots by parity), r.r, b.b
  double *hist;             // [max_iter + 1] r.r after each iteration (slot 0: b.b)
  const int32_t *node_free; // warm start: free index of each node or -1
  const double *x0;         // warm start: phi_1 of the previous solve [N], or null
  int64_t nf, n_nodes;
  int32_t nblk;
};
// x = x0 (or 0), r = b - S x, z = D^-1 r, p = z; partial r.z and b.b.
hipError_t launch_pcg_start(const PcgArgs &a, const int32_t *free_node, hipStream_t s);
// One iteration (three kernels): q = S p with p.q; x, r, z updates with r.z
// and r.r; p = z + beta p. `it` selects the parity slot of r.z.
hipError_t launch_pcg_iteration(const PcgArgs &a, int32_t it, hipStream_t s);
// hist[slot] = sum of the partial sums `which` (2: r.r, 4: b.b); one workgroup.
hipError_t launch_pcg_reduce(const PcgArgs &a, int32_t which, int32_t slot, hipStream_t s);

// phi_1 on every node: x at the free nodes, 0 on the boundary.
hipError_t launch_fem_scatter(const double *x, const int32_t *node_free, double *phi1,
                              int64_t n_nodes, hipStream_t s);
// d phi_1 / dn on each boundary triangle: grad phi_1 in the owning tetrahedron
// dotted with the unit outward normal.
hipError_t launch_fem_dn(const int32_t *owner, const double *nrm, const int32_t *tets,
                         const double *grad, const double *phi1, double *dn, int64_t mb,
                         hipStream_t s);
// phi += phi_1.
hipError_t launch_fem_add(double *phi, const double *phi1, int64_t n, hipStream_t s);

}  // namespace slp
