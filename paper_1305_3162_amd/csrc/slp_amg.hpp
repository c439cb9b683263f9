// Smoothed-aggregation algebraic multigrid for the free-node stiffness system
// of phi_1 (Sec. 2.1 names algebraic-multigrid preconditioned CG as one way to
// solve eq. poisson in linear time). Host side: the hierarchy of operators.
// Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace slp {

// Compressed sparse rows, 32-bit offsets.
struct HostCsr {
  int64_t rows = 0, cols = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> v;
};

// One level above the coarsest: its operator A, the smoother weights
// w_i = (4/3) / sum_j |a_ij| of l1-damped Jacobi, the prolongation P from the
// next level and the restriction R = P^T.
struct AmgLevel {
  HostCsr A, P, R;
  std::vector<double> w;
};

struct AmgHierarchy {
  std::vector<AmgLevel> levels;
  int64_t nc = 0;                 // size of the coarsest operator
  std::vector<double> coarse_inv; // its inverse, dense, row-major [nc][nc]
};

struct AmgParams {
  double theta = 0.08;            // strength threshold on the finest level, halved per level
  int64_t max_coarse = 512;       // stop coarsening at this size (dense inverse)
  int max_levels = 12;
};

// Builds the hierarchy of the symmetric positive definite matrix A (its copy
// becomes levels[0].A unless A is already small enough to be the coarsest).
// Returns false with a message in err if the coarse operator is not positive
// definite or the coarsening stalls above the dense limit.
bool build_amg(const HostCsr &A, const AmgParams &prm, AmgHierarchy &h, char *err, size_t errlen);

// z = B r for one V(1,1) cycle of the hierarchy on the host, the steps of the
// device cycle in the same order (pre-smoothing from zero, restriction, the
// coarser cycle or the dense inverse, prolongation, post-smoothing). The
// hierarchy must have been built from A; `r` and `z` hold A.rows values.
void amg_apply_host(const AmgHierarchy &h, const double *r, double *z);

}  // namespace slp
