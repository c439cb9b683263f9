// Device side of the Dirichlet problem for phi_1 (Sec. 2.1) and the complete
// scalar potential of Alg. 1. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace slp {

constexpr int kFemThreads = 256;
constexpr int kFemLoadLanes = 8;   // lanes per free node in the load vector

// Load vector on the free nodes: b_f = sum over the tetrahedra T holding node
// free_node[f] (local index a) of |T| mbar_T . grad lambda_a^T. The products
// |T| mbar_T are formed once per tetrahedron first.
struct FemLoadArgs {
  const int32_t *inc_ptr;   // [Nf + 1]
  const int32_t *inc;       // 4 T + a
  const int32_t *tets;      // [T][4]
  const double *vol;        // [T]
  const double *grad;       // [T][4][3]
  const double *m;          // [N][3] nodal magnetisation
  double *vm;               // [T][3] work: |T| mbar_T
  double *b;                // [Nf]
  int64_t nf, nt;
};
hipError_t launch_fem_load(const FemLoadArgs &a, hipStream_t s);

// Preconditioned conjugate gradients on S_ff x = b. Partial sums
// of the dot products are written per workgroup; every consumer sums them.
// S_ff is stored sliced: rows in slices of 64, slice s holding its entries
// column by column (entry k of row 64 s + l at sptr[s] + 64 k + l), slice
// width = its longest row; padding entries point at the row itself with value 0.
struct PcgArgs {
  const int32_t *sptr;      // [n_slices + 1]
  const int32_t *ci;        // column (free index)
  const double *val;
  const double *dinv;       // 1 / diag(S_ff)
  const double *b;
  double *x, *r, *z, *q;
  double *p[2];             // search directions, iteration it writes p[it & 1]
  double *part;             // [5][nblk]: p.q, r.z (two slots by parity), r.r, b.b
  double *hist;             // [max_iter + 1] r.r after each iteration (slot 0: b.b)
  const int32_t *node_free; // warm start: free index of each node or -1
  const double *x0;         // warm start: phi_1 of the previous solve [N], or null
  int64_t nf, n_nodes;
  int32_t nblk;
  int32_t jacobi;           // 1: z = D^-1 r in the start and update kernels; 0: the
                            // multigrid cycle forms z and the partial r.z instead
};
// x = x0 (or 0), r = b - S x, z = D^-1 r; partial r.z and b.b.
hipError_t launch_pcg_start(const PcgArgs &a, const int32_t *free_node, hipStream_t s);
// One iteration, two kernels: (1) p = z + beta p (beta = 0 in iteration 0),
// formed on the fly for the neighbours and stored for the own row, q = S p
// (16 lanes per row) with p.q; (2) x, r, z updates with r.z and r.r. `it`
// selects the parity slots of r.z and of p.
hipError_t launch_pcg_iteration(const PcgArgs &a, int32_t it, hipStream_t s);
// One operator application of the multigrid cycle. Matrices above the finest
// level are CSR (rp, ci, val) with `lanes` threads per row; the finest level's
// operator is the sliced S_ff of PcgArgs, one thread per row. Modes, with
// (M v)_i = sum_j M_ij v_j:
//   pre      : o1 = w f,  o2 = f - M (w f)      (one damped-Jacobi step from 0 and
//              its residual; `in` = f)
//   post     : o1 = in + w (f - M in)           (damped-Jacobi step from `in`)
//   restrict : o1 = M in                        (also the dense coarse inverse)
//   prolong  : o1 = f + M in                    (o1 may equal f)
// On the finest level `post` also writes the per-workgroup partials of
// o1 . f into part[slot][nblk] (the r.z of the next direction).
enum AmgMode { kAmgPre = 0, kAmgPost = 1, kAmgRestrict = 2, kAmgProlong = 3 };
struct AmgOp {
  const int32_t *rp, *ci;
  const double *val;
  const double *in, *w, *f;
  double *o1, *o2;
  int64_t n;
};
hipError_t launch_amg_csr(const AmgOp &op, int mode, int lanes, hipStream_t s);
hipError_t launch_amg_fine(const PcgArgs &a, const AmgOp &op, int mode, int32_t slot,
                           hipStream_t s);
// part[slot][nblk] = per-workgroup partials of r . z (cycles without a finest smoothing level).
hipError_t launch_amg_dot(const PcgArgs &a, int32_t slot, hipStream_t s);

// hist[slot] = sum of the partial sums `which` (3: r.r, 4: b.b); one workgroup.
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
// out[0] = sum over tetrahedra of |T| mbar_T . grad phi_T (per-workgroup
// partials in part [ceil(T / kFemThreads)], then one workgroup sums them).
hipError_t launch_fem_energy(const int32_t *tets, const double *vol, const double *grad,
                             const double *m, const double *phi, double *part, double *out,
                             int64_t nt, hipStream_t s);

}  // namespace slp
