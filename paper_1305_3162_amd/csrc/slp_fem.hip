// Device code of the Dirichlet problem for phi_1 (Sec. 2.1, eq. poisson): the
// load vector, preconditioned conjugate gradients on the free-node system
// (Jacobi, or a smoothed-aggregation multigrid V-cycle), the normal derivative
// on the boundary triangles, and the final sum phi = phi_1 + phi_2 of Alg. 1.
// FP64 throughout.
#include "slp_fem.hpp"

namespace slp {

namespace {

// Sum over the workgroup; every thread receives the total. Fixed order.
__device__ double block_sum(double v) {
  __shared__ double ws[kFemThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();                       // ws may still be read by a previous call
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kFemThreads / 64; ++i) t += ws[i];
  return t;
}

// Sum of the nblk per-workgroup partial sums of one dot product.
__device__ double sum_parts(const double *__restrict__ part, int nblk) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kFemThreads) v += part[i];
  return block_sum(v);
}

// |T| mbar_T for every tetrahedron.
__global__ __launch_bounds__(kFemThreads) void k_fem_tet_m(FemLoadArgs a) {
  const int64_t t = (int64_t)blockIdx.x * kFemThreads + threadIdx.x;
  if (t >= a.nt) return;
  double mb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t nd = a.tets[4 * t + v];
#pragma unroll
    for (int q = 0; q < 3; ++q) mb[q] += a.m[3 * nd + q];
  }
  const double f = a.vol[t] * 0.25;
#pragma unroll
  for (int q = 0; q < 3; ++q) a.vm[3 * t + q] = f * mb[q];
}

// b_f, kFemLoadLanes lanes per free node: each lane takes every
// kFemLoadLanes-th incident tetrahedron, then a fixed-order shuffle sum.
__global__ __launch_bounds__(kFemThreads) void k_fem_load(FemLoadArgs a) {
  constexpr int L = kFemLoadLanes;
  const int64_t f = ((int64_t)blockIdx.x * kFemThreads + threadIdx.x) / L;
  if (f >= a.nf) return;   // whole groups of L lanes
  const int lane = threadIdx.x & (L - 1);
  double acc = 0.0;
  for (int32_t e = a.inc_ptr[f] + lane; e < a.inc_ptr[f + 1]; e += L) {
    const int64_t t = a.inc[e] >> 2;
    const int la = a.inc[e] & 3;
    const double *g = a.grad + 12 * t + 3 * la;
    const double *vm = a.vm + 3 * t;
    acc += vm[0] * g[0] + vm[1] * g[1] + vm[2] * g[2];
  }
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, L);
  if (lane == 0) a.b[f] = acc;
}

__global__ __launch_bounds__(kFemThreads) void k_pcg_start(PcgArgs a,
                                                           const int32_t *__restrict__ free_node) {
  const int64_t i = (int64_t)blockIdx.x * kFemThreads + threadIdx.x;
  double rz = 0.0, bb = 0.0;
  if (i < a.nf) {
    double xi = 0.0, ri = a.b[i];
    if (a.x0) {
      xi = a.x0[free_node[i]];
      const int64_t sl = i >> 6;
      const int32_t w = (a.sptr[sl + 1] - a.sptr[sl]) >> 6;
      for (int32_t k = 0; k < w; ++k) {
        const int64_t e = a.sptr[sl] + 64 * k + (i & 63);
        ri -= a.val[e] * a.x0[free_node[a.ci[e]]];
      }
    }
    a.x[i] = xi;
    a.r[i] = ri;
    if (a.jacobi) {
      const double zi = a.dinv[i] * ri;
      a.z[i] = zi;
      rz = ri * zi;
    }
    bb = a.b[i] * a.b[i];
  }
  rz = block_sum(rz);
  bb = block_sum(bb);
  if (threadIdx.x == 0) {
    if (a.jacobi) a.part[1 * a.nblk + blockIdx.x] = rz;
    a.part[4 * a.nblk + blockIdx.x] = bb;
  }
}

// p = z + beta p_old (formed on the fly for every neighbour, stored for the
// own row), q = S p, partial p.q. One thread per row: a wave is one slice, so
// the column and value loads of entry k are contiguous across the wave.
__global__ __launch_bounds__(kFemThreads) void k_pcg_spmv(PcgArgs a, int32_t it) {
  double beta = 0.0;
  if (it > 0) {
    const double rzn = sum_parts(a.part + (1 + (it & 1)) * a.nblk, a.nblk);
    const double rzo = sum_parts(a.part + (1 + ((it + 1) & 1)) * a.nblk, a.nblk);
    beta = rzo != 0.0 ? rzn / rzo : 0.0;
  }
  const double *__restrict__ po = a.p[(it + 1) & 1];
  double *__restrict__ pn = a.p[it & 1];
  const int64_t i = (int64_t)blockIdx.x * kFemThreads + threadIdx.x;
  double pq = 0.0;
  if (i < a.nf) {
    const int64_t sl = i >> 6;
    const int64_t base = a.sptr[sl] + (i & 63);
    const int32_t w = (a.sptr[sl + 1] - a.sptr[sl]) >> 6;
    double s = 0.0;
    for (int32_t k = 0; k < w; ++k) {
      const int32_t j = a.ci[base + 64 * k];
      const double pj = it > 0 ? a.z[j] + beta * po[j] : a.z[j];
      s += a.val[base + 64 * k] * pj;
    }
    const double pr = it > 0 ? a.z[i] + beta * po[i] : a.z[i];
    pn[i] = pr;
    a.q[i] = s;
    pq = pr * s;
  }
  pq = block_sum(pq);
  if (threadIdx.x == 0) a.part[blockIdx.x] = pq;
}

// alpha = r.z / p.q; x += alpha p; r -= alpha q; partial r.r; with the Jacobi
// preconditioner also z = D^-1 r and partial r.z.
__global__ __launch_bounds__(kFemThreads) void k_pcg_update(PcgArgs a, int32_t it) {
  const double pq = sum_parts(a.part, a.nblk);
  const double rz = sum_parts(a.part + (1 + (it & 1)) * a.nblk, a.nblk);
  const double alpha = pq != 0.0 ? rz / pq : 0.0;
  const double *__restrict__ p = a.p[it & 1];
  const int64_t i = (int64_t)blockIdx.x * kFemThreads + threadIdx.x;
  double rzn = 0.0, rr = 0.0;
  if (i < a.nf) {
    a.x[i] += alpha * p[i];
    const double ri = a.r[i] - alpha * a.q[i];
    a.r[i] = ri;
    if (a.jacobi) {
      const double zi = a.dinv[i] * ri;
      a.z[i] = zi;
      rzn = ri * zi;
    }
    rr = ri * ri;
  }
  rzn = block_sum(rzn);
  rr = block_sum(rr);
  if (threadIdx.x == 0) {
    if (a.jacobi) a.part[(1 + ((it + 1) & 1)) * a.nblk + blockIdx.x] = rzn;
    a.part[3 * a.nblk + blockIdx.x] = rr;
  }
}

// Multigrid cycle on the finest level: the sliced S_ff, one thread per row
// (modes pre and post of AmgOp).
template <int MODE>
__global__ __launch_bounds__(kFemThreads) void k_amg_fine(PcgArgs a, AmgOp op, int32_t slot) {
  const int64_t i = (int64_t)blockIdx.x * kFemThreads + threadIdx.x;
  double rz = 0.0;
  if (i < a.nf) {
    const int64_t sl = i >> 6;
    const int64_t base = a.sptr[sl] + (i & 63);
    const int32_t w = (a.sptr[sl + 1] - a.sptr[sl]) >> 6;
    double t = 0.0;
    for (int32_t k = 0; k < w; ++k) {
      const int32_t j = a.ci[base + 64 * k];
      const double vj = MODE == kAmgPre ? op.w[j] * op.in[j] : op.in[j];
      t += a.val[base + 64 * k] * vj;
    }
    const double fi = op.f[i];
    if (MODE == kAmgPre) {
      op.o1[i] = op.w[i] * fi;
      op.o2[i] = fi - t;
    } else {
      const double zi = op.in[i] + op.w[i] * (fi - t);
      op.o1[i] = zi;
      rz = zi * fi;
    }
  }
  if (MODE == kAmgPost) {
    rz = block_sum(rz);
    if (threadIdx.x == 0) a.part[slot * a.nblk + blockIdx.x] = rz;
  }
}

// Multigrid cycle on a CSR operator: L lanes per row, a row's lanes in one
// wave, their sum by butterfly shuffles.
template <int L, int MODE>
__global__ __launch_bounds__(kFemThreads) void k_amg_csr(AmgOp op) {
  const int64_t row = ((int64_t)blockIdx.x * kFemThreads + threadIdx.x) / L;
  const int lane = threadIdx.x & (L - 1);
  double t = 0.0;
  if (row < op.n) {
    const int32_t e1 = op.rp[row + 1];
    for (int32_t e = op.rp[row] + lane; e < e1; e += L) {
      const int32_t j = op.ci[e];
      t += op.val[e] * (MODE == kAmgPre ? op.w[j] * op.in[j] : op.in[j]);
    }
  }
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) t += __shfl_xor(t, off, L);
  if (row >= op.n || lane != 0) return;
  if (MODE == kAmgPre) {
    const double fi = op.f[row];
    op.o1[row] = op.w[row] * fi;
    op.o2[row] = fi - t;
  } else if (MODE == kAmgPost) {
    const double yi = op.in[row];
    op.o1[row] = yi + op.w[row] * (op.f[row] - t);
  } else if (MODE == kAmgRestrict) {
    op.o1[row] = t;
  } else {
    op.o1[row] = op.f[row] + t;
  }
}

__global__ __launch_bounds__(kFemThreads) void k_amg_dot(PcgArgs a, int32_t slot) {
  const int64_t i = (int64_t)blockIdx.x * kFemThreads + threadIdx.x;
  double rz = i < a.nf ? a.r[i] * a.z[i] : 0.0;
  rz = block_sum(rz);
  if (threadIdx.x == 0) a.part[slot * a.nblk + blockIdx.x] = rz;
}

__global__ __launch_bounds__(kFemThreads) void k_pcg_reduce(PcgArgs a, int32_t which,
                                                            int32_t slot) {
  const double s = sum_parts(a.part + which * a.nblk, a.nblk);
  if (threadIdx.x == 0) a.hist[slot] = s;
}

__global__ __launch_bounds__(kFemThreads) void k_fem_scatter(const double *__restrict__ x,
                                                             const int32_t *__restrict__ node_free,
                                                             double *__restrict__ phi1, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kFemThreads + threadIdx.x;
  if (k >= n) return;
  const int32_t f = node_free[k];
  phi1[k] = f >= 0 ? x[f] : 0.0;
}

__global__ __launch_bounds__(kFemThreads) void k_fem_dn(const int32_t *__restrict__ owner,
                                                        const double *__restrict__ nrm,
                                                        const int32_t *__restrict__ tets,
                                                        const double *__restrict__ grad,
                                                        const double *__restrict__ phi1,
                                                        double *__restrict__ dn, int64_t mb) {
  const int64_t j = (int64_t)blockIdx.x * kFemThreads + threadIdx.x;
  if (j >= mb) return;
  const int64_t t = owner[j];
  double g[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double u = phi1[tets[4 * t + v]];
#pragma unroll
    for (int q = 0; q < 3; ++q) g[q] += u * grad[12 * t + 3 * v + q];
  }
  dn[j] = g[0] * nrm[3 * j] + g[1] * nrm[3 * j + 1] + g[2] * nrm[3 * j + 2];
}

__global__ __launch_bounds__(kFemThreads) void k_fem_add(double *__restrict__ phi,
                                                         const double *__restrict__ phi1,
                                                         int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kFemThreads + threadIdx.x;
  if (k < n) phi[k] += phi1[k];
}

__global__ __launch_bounds__(kFemThreads) void k_fem_energy(const int32_t *__restrict__ tets,
                                                            const double *__restrict__ vol,
                                                            const double *__restrict__ grad,
                                                            const double *__restrict__ m,
                                                            const double *__restrict__ phi,
                                                            double *__restrict__ part, int64_t nt) {
  const int64_t t = (int64_t)blockIdx.x * kFemThreads + threadIdx.x;
  double e = 0.0;
  if (t < nt) {
    double g[3] = {0.0, 0.0, 0.0}, mb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t nd = tets[4 * t + v];
      const double u = phi[nd];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        g[q] += u * grad[12 * t + 3 * v + q];
        mb[q] += m[3 * nd + q];
      }
    }
    e = vol[t] * 0.25 * (mb[0] * g[0] + mb[1] * g[1] + mb[2] * g[2]);
  }
  e = block_sum(e);
  if (threadIdx.x == 0) part[blockIdx.x] = e;
}

__global__ __launch_bounds__(kFemThreads) void k_fem_sum(const double *__restrict__ part, int n,
                                                         double *__restrict__ out) {
  const double s = sum_parts(part, n);
  if (threadIdx.x == 0) out[0] = s;
}

unsigned blocks(int64_t n) { return (unsigned)((n + kFemThreads - 1) / kFemThreads); }

}  // namespace

hipError_t launch_fem_load(const FemLoadArgs &a, hipStream_t s) {
  if (a.nf <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fem_tet_m, dim3(blocks(a.nt)), dim3(kFemThreads), 0, s, a);
  hipLaunchKernelGGL(k_fem_load, dim3(blocks(a.nf * kFemLoadLanes)), dim3(kFemThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pcg_start(const PcgArgs &a, const int32_t *free_node, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_start, dim3(a.nblk), dim3(kFemThreads), 0, s, a, free_node);
  return hipGetLastError();
}

hipError_t launch_pcg_iteration(const PcgArgs &a, int32_t it, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_spmv, dim3(a.nblk), dim3(kFemThreads), 0, s, a, it);
  hipLaunchKernelGGL(k_pcg_update, dim3(a.nblk), dim3(kFemThreads), 0, s, a, it);
  return hipGetLastError();
}

namespace {
template <int L>
void launch_csr_lanes(const AmgOp &op, int mode, hipStream_t s) {
  const int64_t threads = op.n * L;
  const dim3 grid((unsigned)((threads + kFemThreads - 1) / kFemThreads));
  switch (mode) {
    case kAmgPre: hipLaunchKernelGGL((k_amg_csr<L, kAmgPre>), grid, dim3(kFemThreads), 0, s, op); break;
    case kAmgPost: hipLaunchKernelGGL((k_amg_csr<L, kAmgPost>), grid, dim3(kFemThreads), 0, s, op); break;
    case kAmgRestrict:
      hipLaunchKernelGGL((k_amg_csr<L, kAmgRestrict>), grid, dim3(kFemThreads), 0, s, op);
      break;
    default: hipLaunchKernelGGL((k_amg_csr<L, kAmgProlong>), grid, dim3(kFemThreads), 0, s, op); break;
  }
}
}  // namespace

hipError_t launch_amg_csr(const AmgOp &op, int mode, int lanes, hipStream_t s) {
  if (op.n <= 0) return hipSuccess;
  switch (lanes) {
    case 1: launch_csr_lanes<1>(op, mode, s); break;
    case 2: launch_csr_lanes<2>(op, mode, s); break;
    case 4: launch_csr_lanes<4>(op, mode, s); break;
    case 8: launch_csr_lanes<8>(op, mode, s); break;
    case 16: launch_csr_lanes<16>(op, mode, s); break;
    case 32: launch_csr_lanes<32>(op, mode, s); break;
    case 64: launch_csr_lanes<64>(op, mode, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_amg_fine(const PcgArgs &a, const AmgOp &op, int mode, int32_t slot,
                           hipStream_t s) {
  if (mode == kAmgPre)
    hipLaunchKernelGGL(k_amg_fine<kAmgPre>, dim3(a.nblk), dim3(kFemThreads), 0, s, a, op, slot);
  else if (mode == kAmgPost)
    hipLaunchKernelGGL(k_amg_fine<kAmgPost>, dim3(a.nblk), dim3(kFemThreads), 0, s, a, op, slot);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_amg_dot(const PcgArgs &a, int32_t slot, hipStream_t s) {
  hipLaunchKernelGGL(k_amg_dot, dim3(a.nblk), dim3(kFemThreads), 0, s, a, slot);
  return hipGetLastError();
}

hipError_t launch_pcg_reduce(const PcgArgs &a, int32_t which, int32_t slot, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_reduce, dim3(1), dim3(kFemThreads), 0, s, a, which, slot);
  return hipGetLastError();
}

hipError_t launch_fem_scatter(const double *x, const int32_t *node_free, double *phi1,
                              int64_t n_nodes, hipStream_t s) {
  if (n_nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fem_scatter, dim3(blocks(n_nodes)), dim3(kFemThreads), 0, s, x, node_free,
                     phi1, n_nodes);
  return hipGetLastError();
}

hipError_t launch_fem_dn(const int32_t *owner, const double *nrm, const int32_t *tets,
                         const double *grad, const double *phi1, double *dn, int64_t mb,
                         hipStream_t s) {
  if (mb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fem_dn, dim3(blocks(mb)), dim3(kFemThreads), 0, s, owner, nrm, tets, grad,
                     phi1, dn, mb);
  return hipGetLastError();
}

hipError_t launch_fem_energy(const int32_t *tets, const double *vol, const double *grad,
                             const double *m, const double *phi, double *part, double *out,
                             int64_t nt, hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fem_energy, dim3(blocks(nt)), dim3(kFemThreads), 0, s, tets, vol, grad, m,
                     phi, part, nt);
  hipLaunchKernelGGL(k_fem_sum, dim3(1), dim3(kFemThreads), 0, s, part, (int)blocks(nt), out);
  return hipGetLastError();
}

hipError_t launch_fem_add(double *phi, const double *phi1, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fem_add, dim3(blocks(n)), dim3(kFemThreads), 0, s, phi, phi1, n);
  return hipGetLastError();
}

}  // namespace slp
