// Device code for the smooth-part single-layer potential (gfx950).
//
// Stages (Sec. 3, Alg. 1 computation phase, eq. BEM_NFFT_compact2):
//   spread   a_r = sum_k q_k prod_q psi(t_kq - r_q), with the charges
//            q_k = w_k g_k formed while staging          (eq. gridding, naive_gridding)
//   fft      pruned 3-D FFT, multiply by mu, inverse FFT    (eq. FFT, deconv, Alg. 1;
//            in slp_fft.hip)
//   interp   phi_i = sum_r g_r prod_q psi(t_iq - r_q)       (type-2 NFFT)
// mu folds the two window deconvolutions, c_l(N_s), the Hermitian weights of
// the asymmetric index set and 1/(4 pi) into one real factor per mode.
#include "slp_internal.hpp"
#include "slp_near.hpp"

#include <hip/hip_runtime.h>

namespace slp {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float wexp(float x) { return __expf(x); }
__device__ __forceinline__ double wexp(double x) { return exp(x); }

// A pointer read from memory (the argument tables of the fused launches)
// marked as pointing to global memory, so that accesses through it are
// global rather than flat instructions (flat accesses also count against the
// LDS wait counter, and a wait for LDS then waits for them too).
template <typename P>
__device__ __forceinline__ P *gptr(P *p) {
  return (P *)(__attribute__((address_space(1))) P *)(uintptr_t)p;
}

// Kaiser-Bessel window of eq. KBfct in grid units, scaled to 1 at tau = 0:
// sinh(b s) / s * inv_norm with s = sqrt(m^2 - tau^2) (|tau| <= m on every
// stencil point; the limit b at s = 0).
template <typename T>
__device__ __forceinline__ T kb_weight(T tau, T m, T b, T inv_norm) {
  const T s2 = m * m - tau * tau;
  const T s = s2 > T(0) ? sqrt(s2) : T(0);
  if (s < T(1e-4)) return b * inv_norm;
  const T e = wexp(b * s);
  return (e - T(1) / e) * T(0.5) / s * inv_norm;
}

// Kaiser-Bessel window at the 2m stencil points of a point with fraction f,
// u = 2 f - 1: out[j] = q * P_j(u), P_j the polynomial fitted on the host for
// the window at tau = f + m - 1 - j. The window is even, so the stencil point
// 2m - 1 - j sees P_j(-u): with P_j(u) = E_j(u^2) + u O_j(u^2) one pass over
// the even and odd coefficients of P_j gives both points (the host stores the
// mirrored polynomials exactly so). The coefficients are wave-uniform kernel
// arguments. When all pairs' coefficients take more than 48 scalar
// registers, the pairs are a loop that is not unrolled, so that only one
// pair's coefficients are held at a time (all of them at once overflow the
// scalar registers into vector-register lanes, and every use then costs a
// vector instruction).
template <typename T, int M>
__device__ __forceinline__ void kb_stencil(const T (&c)[kKbCoef], T u, T q, T *out) {
  constexpr int D = kb_degree<T, M>();
  static_assert(D % 2 == 0, "even polynomial degree");
  const T v = u * u;
  auto pair = [&](int j) {
    const T *cj = c + j * (D + 1);
    T e = cj[D], o = cj[D - 1];
#pragma unroll
    for (int d = D - 2; d >= 0; d -= 2) e = e * v + cj[d];
#pragma unroll
    for (int d = D - 3; d >= 1; d -= 2) o = o * v + cj[d];
    const T uo = u * o;
    out[j] = (e + uo) * q;
    out[2 * M - 1 - j] = (e - uo) * q;
  };
  if constexpr (M * (D + 1) * sizeof(T) / 4 > 48) {
#pragma unroll 1
    for (int j = 0; j < M; ++j) pair(j);
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) pair(j);
  }
}

// The 2m window factors of one source along one axis (fraction f of its
// coordinate), times q: Gaussian by the fast-Gaussian-gridding recurrence
// w_{j+1} = w_j r_j, r_{j+1} = r_j exp(-2/b) (two exponentials), Kaiser-Bessel
// by the fitted polynomials.
template <typename T, int M, typename A>
__device__ __forceinline__ void stencil_factors(const A &a, T f, T q, T *dst) {
  if (a.window == 0) {
    const T fm = f + T(M - 1);
    T w = wexp(-fm * fm * a.inv_b) * q;
    T rr = wexp((T(2) * fm - T(1)) * a.inv_b);
#pragma unroll
    for (int j = 0; j < 2 * M; ++j) {
      dst[j] = w;
      w *= rr;
      rr *= a.step_ratio;
    }
  } else {
    kb_stencil<T, M>(a.kb_c, T(2) * f - T(1), q, dst);
  }
}

// ----------------------------------------------------------------- spread ---
// Phase A (one workgroup of 8 waves per work unit; the setup gives every unit
// one segment, the sources of one tile or an equal piece of a crowded tile,
// longest first): the segment's sources are scattered into an FP64 LDS block
// covering the tile plus the stencil halo, (8 + 2m - 1)^3 cells, which is then
// stored to the segment's slot. The sources are staged in chunks; a chunk's
// runs (sources sharing one grid cell) are ordered longest first. A wave takes
// R runs side by side, L lanes per run: each lane keeps the 2m z-values of a
// few (dx, dy) columns of its run's stencil in registers over the whole run
// and adds them to the LDS block once per run. The 1-D window factors of SB
// sources of each of the R runs are built per step in a wave-private LDS
// slice, one (run, source, axis) per lane: Gaussian factors with the
// fast-Gaussian-gridding recurrence w_{j+1} = w_j r_j, r_{j+1} = r_j exp(-2/b)
// (two exponentials per source and axis), Kaiser-Bessel factors from the
// fitted polynomials (one pass per mirrored pair of stencil points).
// With FP64 and 2m = 16 a run is instead accumulated by the matrix cores: for
// the sources k of a run (cell fixed, so the stencil offsets are the same),
// the block update is sum_k fz_k[dz] fy_k[dy] fx_k[dx], for every dy a
// 16 x K by K x 16 product D_dy[dz][dx] += sum_k (fz_k[dz] fy_k[dy]) fx_k[dx]
// (fx carries the charge). One v_mfma_f64_16x16x4f64 takes four sources; a
// lane supplies A[dz = lane % 16][k = lane / 16] and B[k = lane / 16][dx =
// lane % 16] and holds D[dz = 4 r + lane / 16][dx = lane % 16] in its
// register r, so the sixteen dy tiles are 64 FP64 accumulators per lane, as in
// the vector form. Missing sources of the last group of four enter as zeros.
// Phase B (one workgroup per region tile): every cell sums the blocks of the
// segments of the neighbouring tiles that cover it, in a fixed order, and
// writes the grid.
//
// Blocked layout of a stored block: along each axis the padded range splits
// into the part that lands in the previous tile (m - 1 cells), in the own tile
// (8) and in the next tile (m); the 27 sub-blocks are stored one after the
// other (z part, then y part, then x part), each row-major, so the reduction
// for one tile reads every contributing sub-block as one contiguous range.
template <typename T, int M>
struct SpreadShape {
  static constexpr int W = 2 * M;
  static constexpr int PD = kTile + W - 1;
  static constexpr int P3 = PD * PD * PD;
  static constexpr int WAVES = 8;
  static constexpr int THREADS = WAVES * 64;
  static constexpr int SBW = 12;                       // sources per factor batch (matrix form)
  static constexpr int CH = spread_chunk(sizeof(T) == 8, M);   // sources staged per block chunk
  // FP64 with 2m = 16: a run's update goes to the matrix cores (see
  // k_spread_bins); the factors of a source then sit 16-byte aligned
  static constexpr bool MX = sizeof(T) == 8 && W == 16;
  // vector form: a lane holds CX x CY x CZ cells of a run's stencil (CX x CY
  // whole (dx, dy) columns, except FP64 with 2m = 8), L lanes cover one run's
  // stencil, R runs share a wave, and the factors of SB sources of each of
  // the R runs are built per batch; RP and PP are the LDS block's row and
  // plane pitch, PL its size
  // FP64 with 2m = 8: a lane holds 1 x 4 x 4 cells (x on consecutive lanes,
  // y and z 2 apart) and the LDS block has rows of 16 and planes of 264
  // doubles, so that a run's 32 lanes flushing one register hit 32 distinct
  // (double-wide) banks: x 0..7, y adds 0 or 16, z adds 0 or 8 (mod 32)
  static constexpr bool LAY8 = sizeof(T) == 8 && W == 8;
  static constexpr int CX = (W <= 4 || LAY8) ? 1 : 2;
  static constexpr int CY = LAY8 ? 4 : ((W <= 4 || (sizeof(T) == 8 && W == 6)) ? 1 : 2);
  static constexpr int CZ = LAY8 ? 4 : W;
  static constexpr int RP = LAY8 ? 16 : PD;
  static constexpr int PP = LAY8 ? 264 : PD * PD;
  static constexpr int PL = PP * PD;
  static constexpr int L = (W / CX) * (W / CY) * (W / CZ);
  static constexpr int R = 64 / L;
  static constexpr int SB0 = 64 / (3 * R);
  static constexpr int SB = LAY8 ? 10 : (SB0 > 12 ? 12 : SB0);
  static constexpr int NFAC = MX ? SBW : R * SB;       // factor slots per wave
  static constexpr int FST = MX ? 3 * W + 2 : 3 * W + 1;   // LDS stride of one source's factors
  static_assert(W % CX == 0 && W % CY == 0 && W % CZ == 0 && L <= 64 && R >= 1 && SB >= 1,
                "gridding shape");
  // the factors of a step are built one (run, source, axis) per lane
  static_assert(MX || 3 * R * SB <= 64, "factor step larger than a wave");
};

int64_t pad_cells(int m) {
  const int64_t pd = kTile + 2 * m - 1;
  return pd * pd * pd;
}

int spread_units_per_cu(int m, bool fp64) {
  auto lds = [](auto shape, size_t esz) {
    using S = decltype(shape);
    return (size_t)S::PL * 8 + (size_t)S::WAVES * S::NFAC * S::FST * esz +
           4 * (size_t)S::CH * esz + (size_t)S::CH * 4;
  };
  size_t b = 0;
  switch (m) {
#define SLP_LDS_CASE(MM)                                                            \
  case MM:                                                                          \
    b = fp64 ? lds(SpreadShape<double, MM>{}, 8) : lds(SpreadShape<float, MM>{}, 4); \
    break;
    SLP_LDS_CASE(1) SLP_LDS_CASE(2) SLP_LDS_CASE(3) SLP_LDS_CASE(4)
    SLP_LDS_CASE(5) SLP_LDS_CASE(6) SLP_LDS_CASE(7) SLP_LDS_CASE(8)
#undef SLP_LDS_CASE
    default: return 1;
  }
  const int fit = (int)((size_t)160 * 1024 / b);
  return fit < 1 ? 1 : (fit > 2 ? 2 : fit);
}

// Part of the padded range holding pad coordinate c, its first coordinate and
// its length (m - 1, 8, m).
template <int M>
__device__ __forceinline__ void pad_part(int c, int &part, int &start, int &len) {
  if (c < M - 1) { part = 0; start = 0; len = M - 1; }
  else if (c < M + kTile - 1) { part = 1; start = M - 1; len = kTile; }
  else { part = 2; start = M + kTile - 1; len = M; }
}

// Blocked index of pad cell (x, y, z).
template <int M>
__device__ __forceinline__ int pad_block_index(int x, int y, int z) {
  constexpr int PD = kTile + 2 * M - 1;
  int px, sx, lx, py, sy, ly, pz, sz, lz;
  pad_part<M>(x, px, sx, lx);
  pad_part<M>(y, py, sy, ly);
  pad_part<M>(z, pz, sz, lz);
  return sz * PD * PD + lz * sy * PD + lz * ly * sx + ((z - sz) * ly + (y - sy)) * lx + (x - sx);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One workgroup per work unit `unit` of the geometry `a` describes, for the
// density `dens` of batch item `item` (whose blocks lie item * scratch_bstride
// further); the window (window, inv_b, step_ratio, kb_c) is read from `win`.
template <typename T, int M>
__device__ __forceinline__ void spread_bins_body(const SpreadBinsArgs<T> &a,
                                                 const SpreadBinsArgs<T> &win, const double *dens,
                                                 int64_t unit, int item) {
  using S = SpreadShape<T, M>;
  constexpr int W = S::W, PD = S::PD, CH = S::CH;
  // The block is accumulated in FP64 in both precisions: LDS FP64 atomic adds
  // are native and fast on gfx950, FP32 LDS atomic adds measured several times
  // slower; the block is stored in T.
  constexpr int FST = S::FST;
  __shared__ double pad[S::PL];
  __shared__ __attribute__((aligned(16))) T wts[S::WAVES * S::NFAC * FST];
  __shared__ T src[4][CH];          // fractions x, y, z and charge of the staged chunk
  __shared__ int32_t rrec[CH];      // runs of the chunk

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  T *ww = wts + wave * S::NFAC * FST;
  const int64_t ns = a.ns;
  // {slot, first chunk, end chunk, reach of the tile's sources} and the first
  // chunk's record, side by side (one round trip)
  const int4 ui = a.units[2 * unit];

  // The global loads of a chunk are issued one chunk ahead: those of chunk
  // c + 1 fly while chunk c is gridded (and the header of chunk c + 2 with
  // them), so only the first chunk's loads are waited for in full. Thread t
  // loads source t of the chunk (its three fractions, weight and density);
  // the charge q = w g is formed when the values are stored to LDS, so that
  // no arithmetic waits on the loads in flight.
  static_assert(S::CH <= S::THREADS, "one source per thread and chunk");
  T v[3];
  double wq = 0.0, dv = 0.0;
  int32_t rv = 0;
  auto load_chunk = [&](const int4 h) {
    if (tid < h.y) {
      const int64_t si = (int64_t)h.x + tid;
      const int32_t pm = a.perm[si];
      v[0] = a.frac[si];
      v[1] = a.frac[ns + si];
      v[2] = a.frac[2 * ns + si];
      wq = a.w[si];
      dv = dens[pm];
    }
    if (tid < h.w) rv = a.runs[h.z + tid];
  };
  int4 ch = a.units[2 * unit + 1];   // {first source, count, first run, run count}
  int4 hn = ui.y + 1 < ui.z ? a.chunks[ui.y + 1] : ch;
  load_chunk(ch);
  for (int i = tid; i < S::PL; i += S::THREADS) pad[i] = 0.0;
  for (int c = ui.y; c < ui.z; ++c) {
    __syncthreads();                   // the previous chunk is done with src / rrec
    if (tid < ch.y) {
      src[0][tid] = v[0];
      src[1][tid] = v[1];
      src[2][tid] = v[2];
      src[3][tid] = (T)(wq * dv);
    }
    if (tid < ch.w) rrec[tid] = rv;
    const int nrun = ch.w;
    __syncthreads();
    if (c + 1 < ui.z) {
      ch = hn;
      load_chunk(ch);
      if (c + 2 < ui.z) {
        // a scalar load: the header is the same for the whole workgroup, and
        // the wave need not wait for the vector loads above to take it over
        const __attribute__((address_space(4))) int32_t *hp =
            (const __attribute__((address_space(4))) int32_t *)(a.chunks + c + 2);
        hn = make_int4(hp[0], hp[1], hp[2], hp[3]);
      }
    }

    if constexpr (S::MX) {
      // matrix-core form: each wave takes every WAVES-th run
      for (int r = wave; r < nrun; r += S::WAVES) {
        const int rec = rrec[r];
        const int cx = rec & 7, cy = (rec >> 3) & 7, cz = (rec >> 6) & 7;
        const int off = (rec >> 9) & 1023, cnt = (rec >> 19) & 2047;
        // macc[dy][r] for dx = lane % 16, dz = 4 r + lane / 16
        dbl4 macc[W];
#pragma unroll
        for (int t = 0; t < W; ++t) macc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
        for (int c0 = 0; c0 < cnt; c0 += S::SBW) {
          const int n = min(S::SBW, cnt - c0);
          if (lane < 3 * n) {
            const int ax = lane / n, sl = lane - ax * n;
            const int si = off + c0 + sl;
            stencil_factors<T, M>(win, src[ax][si], ax == 0 ? src[3][si] : T(1), ww + sl * FST + ax * W);
          }
          wave_sync();
          const int lk = lane >> 4, li = lane & 15;
          for (int g = 0; g < n; g += 4) {
            const int sl = g + lk;
            const bool ok = sl < n;
            // slot 0 holds this batch's factors, so the loads stay finite
            const double *f3 = reinterpret_cast<const double *>(ww) + (ok ? sl : 0) * FST;
            const double bx = ok ? f3[li] : 0.0;
            const double az = ok ? f3[2 * W + li] : 0.0;
            const dbl2 *fy2 = reinterpret_cast<const dbl2 *>(f3 + W);
#pragma unroll
            for (int t2 = 0; t2 < W / 2; ++t2) {
              const dbl2 fy = fy2[t2];
              macc[2 * t2] = __builtin_amdgcn_mfma_f64_16x16x4f64(az * fy.x, bx, macc[2 * t2], 0, 0, 0);
              macc[2 * t2 + 1] =
                  __builtin_amdgcn_mfma_f64_16x16x4f64(az * fy.y, bx, macc[2 * t2 + 1], 0, 0, 0);
            }
          }
          wave_sync();
        }
        double *base = pad + (cz + (lane >> 4)) * S::PP + cy * S::RP + cx + (lane & 15);
#pragma unroll
        for (int t = 0; t < W; ++t)
#pragma unroll
          for (int rg = 0; rg < 4; ++rg) atomicAdd(base + 4 * rg * S::PP + t * S::RP, macc[t][rg]);
      }
    } else {
      // vector form: a wave takes R runs at a time, L lanes per run; a lane
      // keeps CX x CY x CZ stencil cells of its run in registers over the run,
      // W / CX, W / CY and W / CZ apart (the factors of a source are read once
      // per CX, CY and CZ cells; neighbouring lanes hold neighbouring x, so each
      // flush instruction covers whole x rows)
      constexpr int R = S::R, L = S::L, CX = S::CX, CY = S::CY, CZ = S::CZ, SB = S::SB;
      constexpr int SX = W / CX, SY = W / CY, SZ = W / CZ;
      const int g = lane / L, lc = lane - g * L;
      const int dx0 = lc % SX, dy0 = (lc / SX) % SY, dz0 = lc / (SX * SY);
      for (int rb = wave * R; rb < nrun; rb += S::WAVES * R) {
        const int r = rb + g;
        const bool act = g < R && r < nrun;
        const int rec = act ? rrec[r] : 0;
        const int cx = rec & 7, cy = (rec >> 3) & 7, cz = (rec >> 6) & 7;
        const int cnt = act ? (rec >> 19) & 2047 : 0;
        int maxv = cnt;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) maxv = max(maxv, __shfl_xor(maxv, o));
        // the same on every lane: a scalar, so that the source loop below is
        // a scalar loop with compile-time factor offsets
        const int maxc = __builtin_amdgcn_readfirstlane(maxv);
        T acc[CX * CY][CZ];
#pragma unroll
        for (int c2 = 0; c2 < CX * CY; ++c2)
#pragma unroll
          for (int j = 0; j < CZ; ++j) acc[c2][j] = T(0);
        for (int c0 = 0; c0 < maxc; c0 += SB) {
          // factors of source c0 + b of each of the R runs: one (run, source,
          // axis) per lane; sources beyond a run's end get zero factors
          if (lane < R * SB * 3) {
            const int g2 = lane / (SB * 3), b = (lane / 3) % SB, ax = lane % 3;
            const int r2 = rb + g2;
            T *dst = ww + (g2 * SB + b) * FST + ax * W;
            const int rec2 = r2 < nrun ? rrec[r2] : 0;
            const int off2 = (rec2 >> 9) & 1023, cnt2 = r2 < nrun ? (rec2 >> 19) & 2047 : 0;
            if (c0 + b < cnt2) {
              const int si = off2 + c0 + b;
              stencil_factors<T, M>(win, src[ax][si], ax == 0 ? src[3][si] : T(1), dst);
            } else {
#pragma unroll
              for (int j = 0; j < W; ++j) dst[j] = T(0);
            }
          }
          wave_sync();
          if (g < R) {
            const int nb = min(SB, maxc - c0);
#pragma unroll
            for (int b = 0; b < SB; ++b) {
              if (b < nb) {
                const T *f3 = ww + (g * SB + b) * FST;
                T wz[CZ], fx[CX], fy[CY];
#pragma unroll
                for (int j = 0; j < CZ; ++j) wz[j] = f3[2 * W + dz0 + j * SZ];
#pragma unroll
                for (int i = 0; i < CX; ++i) fx[i] = f3[dx0 + i * SX];
#pragma unroll
                for (int i = 0; i < CY; ++i) fy[i] = f3[W + dy0 + i * SY];
#pragma unroll
                for (int iy = 0; iy < CY; ++iy)
#pragma unroll
                  for (int ix = 0; ix < CX; ++ix) {
                    const T pw = fx[ix] * fy[iy];
#pragma unroll
                    for (int j = 0; j < CZ; ++j) acc[iy * CX + ix][j] += pw * wz[j];
                  }
              }
            }
          }
          wave_sync();
        }
        if (act) {
#pragma unroll
          for (int iy = 0; iy < CY; ++iy)
#pragma unroll
            for (int ix = 0; ix < CX; ++ix) {
              double *base = pad + (cz + dz0) * S::PP + (cy + dy0 + iy * SY) * S::RP + cx + dx0 + ix * SX;
#pragma unroll
              for (int j = 0; j < CZ; ++j)
                atomicAdd(base + j * SZ * S::PP, (double)acc[iy * CX + ix][j]);
            }
        }
      }
    }
  }
  __syncthreads();
  T *dst = a.scratch + item * a.scratch_bstride + (int64_t)ui.x * S::P3;
  {
    // 32 lanes per pad row: x is fixed per thread, rows advance; only the box
    // of pad cells that the tile's sources reach is stored (and read back)
    const int x = tid & 31;
    const int bxl = ui.w & 31, byl = (ui.w >> 5) & 31, bzl = (ui.w >> 10) & 31;
    const int bxh = (ui.w >> 15) & 31, byh = (ui.w >> 20) & 31, bzh = (ui.w >> 25) & 31;
    if (x >= bxl && x <= bxh) {
      int px, sx, lx;
      pad_part<M>(x, px, sx, lx);
      for (int rw = tid >> 5; rw < PD * PD; rw += S::THREADS / 32) {
        const int y = rw % PD, z = rw / PD;
        int py, sy, ly, pz, sz, lz;
        pad_part<M>(y, py, sy, ly);
        pad_part<M>(z, pz, sz, lz);
        if (y < byl || y > byh || z < bzl || z > bzh) continue;
        dst[sz * PD * PD + lz * sy * PD + lz * ly * sx + ((z - sz) * ly + (y - sy)) * lx + (x - sx)] =
            (T)pad[z * S::PP + y * S::RP + x];
      }
    }
  }
}

template <typename T, int M>
__global__ __launch_bounds__((SpreadShape<T, M>::THREADS)) void k_spread_bins(SpreadBinsArgs<T> a,
                                                                               BatchPtrs ptrs) {
  spread_bins_body<T, M>(a, a, ptrs.dens[blockIdx.y], blockIdx.x, blockIdx.y);
}

// Several geometries in one launch: workgroup i takes unit work[i].y of item
// work[i].x (the list holds the units of every item, longest first over all).
// The window, the same for every item, comes with the launch.
template <typename T, int M>
__global__ __launch_bounds__((SpreadShape<T, M>::THREADS)) void k_spread_bins_multi(
    const MultiItem<T> *__restrict__ items, const int2 *__restrict__ work, BatchPtrs ptrs,
    SpreadBinsArgs<T> win) {
  const int2 w = work[blockIdx.x];
  const SpreadBinsArgs<T> &it = items[w.x].sp;
  SpreadBinsArgs<T> a;
  a.frac = gptr(it.frac);
  a.w = gptr(it.w);
  a.perm = gptr(it.perm);
  a.units = gptr(it.units);
  a.chunks = gptr(it.chunks);
  a.runs = gptr(it.runs);
  a.scratch = gptr(it.scratch);
  a.ns = it.ns;
  a.scratch_bstride = 0;
  spread_bins_body<T, M>(a, win, gptr(ptrs.dens[w.x]), w.y, 0);
}

// One workgroup per region tile, one or two cells per thread. For each of the
// 27 neighbouring tiles (fixed order) and each of its segments, the threads
// whose cell the block covers read the matching sub-block, which is
// contiguous in the blocked layout.
template <typename T, int M, int CPT>
__device__ __forceinline__ void spread_reduce_body(const SpreadReduceArgs<T> a, int tile, int item) {
  using S = SpreadShape<T, M>;
  constexpr int ZS = kTile / CPT;    // planes between a thread's cells
  const int tx = tile % a.tiles[0];
  const int ty = (tile / a.tiles[0]) % a.tiles[1];
  const int tz = tile / (a.tiles[0] * a.tiles[1]);
  const int64_t Px = (int64_t)a.tiles[0] * kTile, Py = (int64_t)a.tiles[1] * kTile;
  const T *scr = a.scratch + item * a.scratch_bstride;
  T *grid = a.grid + item * a.grid_bstride;
  // CPT cells per thread, planes cz, cz + ZS, ...: the neighbour's record and
  // the x, y tests are shared, the loads independent
  const int c = threadIdx.x;
  const int cx = c & 7, cy = (c >> 3) & 7, cz = c >> 6;
  // the segment ranges and reach boxes of the 27 neighbouring tiles, read
  // once per workgroup
  __shared__ int4 nts[27];
  if (c < 27) {
    const int bx = tx + c % 3 - 1, by = ty + (c / 3) % 3 - 1, bz = tz + c / 9 - 1;
    int4 ts = make_int4(0, 0, 0, 0);
    if (bx >= 0 && bx < a.tiles[0] && by >= 0 && by < a.tiles[1] && bz >= 0 && bz < a.tiles[2])
      ts = a.tile_slots[bx + a.tiles[0] * (by + a.tiles[1] * bz)];
    nts[c] = ts;
  }
  __syncthreads();
  T v[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) v[j] = T(0);
#pragma unroll
  for (int d = 0; d < 27; ++d) {
    const int4 ts = nts[d];
    if (ts.y == 0) continue;
    const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
    // pad coordinates of the cells in the neighbour's block; pad cells of
    // that tile that none of its sources reaches were not stored
    const int ix = cx - kTile * dx + M - 1, iy = cy - kTile * dy + M - 1, iz = cz - kTile * dz + M - 1;
    const int bx = ts.z;
    if (ix < (bx & 31) || ix > ((bx >> 15) & 31) || iy < ((bx >> 5) & 31) || iy > ((bx >> 20) & 31))
      continue;
    const int zl = (bx >> 10) & 31, zh = (bx >> 25) & 31;
    const T *p0 = scr + (int64_t)ts.x * S::P3;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int izj = iz + j * ZS;
      if (izj >= zl && izj <= zh) {
        const T *q = p0 + pad_block_index<M>(ix, iy, izj);
        for (int k = 0; k < ts.y; ++k) v[j] += q[(int64_t)k * S::P3];
      }
    }
  }
  T *out = grid + ((tz * kTile + cz) * Py + ty * kTile + cy) * Px + tx * kTile + cx;
#pragma unroll
  for (int j = 0; j < CPT; ++j) out[(int64_t)j * ZS * Py * Px] = v[j];
}

template <typename T, int M, int CPT>
__global__ __launch_bounds__(512 / CPT) void k_spread_reduce(SpreadReduceArgs<T> a) {
  spread_reduce_body<T, M, CPT>(a, blockIdx.x, blockIdx.y);
}

template <typename T, int M, int CPT>
__global__ __launch_bounds__(512 / CPT) void k_spread_reduce_multi(const MultiItem<T> *__restrict__ items,
                                                             const int2 *__restrict__ work) {
  const int2 w = work[blockIdx.x];
  SpreadReduceArgs<T> a = items[w.x].rd;
  a.scratch = gptr(a.scratch);
  a.tile_slots = gptr(a.tile_slots);
  a.grid = gptr(a.grid);
  spread_reduce_body<T, M, CPT>(a, w.y, 0);
}

template <typename T, int M>
static hipError_t spread_m(const SpreadBinsArgs<T> &a, const SpreadReduceArgs<T> &r,
                           const BatchPtrs &p, int n_units, int nb, int cells, hipStream_t s,
                           hipEvent_t between) {
  using S = SpreadShape<T, M>;
  if (n_units > 0)
    hipLaunchKernelGGL((k_spread_bins<T, M>), dim3((unsigned)n_units, (unsigned)nb),
                       dim3(S::THREADS), 0, s, a, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (between) {
    e = hipEventRecord(between, s);
    if (e != hipSuccess) return e;
  }
  const int64_t tiles = (int64_t)r.tiles[0] * r.tiles[1] * r.tiles[2];
  // automatic: two cells per thread where there are enough tiles to fill the
  // chip (film regions of 5,408 and 8,427 tiles: 51 -> 42 and 74 -> 59 us; at
  // the threshold the 256-thread form has 32 waves per CU); one where there
  // are few (a cube surface, 512 tiles: 16 against 22 us)
  if (cells == 2 || (cells == 0 && tiles * nb >= kReduceTwoCells))
    hipLaunchKernelGGL((k_spread_reduce<T, M, 2>), dim3((unsigned)tiles, (unsigned)nb), dim3(256), 0,
                       s, r);
  else
    hipLaunchKernelGGL((k_spread_reduce<T, M, 1>), dim3((unsigned)tiles, (unsigned)nb), dim3(512), 0,
                       s, r);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spread(const SpreadBinsArgs<T> &a, const SpreadReduceArgs<T> &r,
                         const BatchPtrs &p, int n_units, int m, int nb, int cells, hipStream_t s,
                         hipEvent_t between) {
  if (cells < 0 || cells > 2) return hipErrorInvalidValue;
  switch (m) {
    case 1: return spread_m<T, 1>(a, r, p, n_units, nb, cells, s, between);
    case 2: return spread_m<T, 2>(a, r, p, n_units, nb, cells, s, between);
    case 3: return spread_m<T, 3>(a, r, p, n_units, nb, cells, s, between);
    case 4: return spread_m<T, 4>(a, r, p, n_units, nb, cells, s, between);
    case 5: return spread_m<T, 5>(a, r, p, n_units, nb, cells, s, between);
    case 6: return spread_m<T, 6>(a, r, p, n_units, nb, cells, s, between);
    case 7: return spread_m<T, 7>(a, r, p, n_units, nb, cells, s, between);
    case 8: return spread_m<T, 8>(a, r, p, n_units, nb, cells, s, between);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int M>
static hipError_t spread_multi_m(const MultiItem<T> *items, const int2 *bins_work, int64_t n_bins,
                                 const int2 *red_work, int64_t n_red, const BatchPtrs &p,
                                 const SpreadBinsArgs<T> &win, hipStream_t s) {
  if (n_bins > 0)
    hipLaunchKernelGGL((k_spread_bins_multi<T, M>), dim3((unsigned)n_bins),
                       dim3(SpreadShape<T, M>::THREADS), 0, s, items, bins_work, p, win);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_red == 0) return e;
  if (n_red >= kReduceTwoCells)
    hipLaunchKernelGGL((k_spread_reduce_multi<T, M, 2>), dim3((unsigned)n_red), dim3(256), 0, s, items,
                       red_work);
  else
    hipLaunchKernelGGL((k_spread_reduce_multi<T, M, 1>), dim3((unsigned)n_red), dim3(512), 0, s, items,
                       red_work);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spread_multi(const MultiItem<T> *items, const int2 *bins_work, int64_t n_bins,
                               const int2 *red_work, int64_t n_red, int m, const BatchPtrs &p,
                               const SpreadBinsArgs<T> &win, hipStream_t s) {
  switch (m) {
#define SLP_CASE(MM) case MM: return spread_multi_m<T, MM>(items, bins_work, n_bins, red_work, n_red, p, win, s);
    SLP_CASE(1) SLP_CASE(2) SLP_CASE(3) SLP_CASE(4) SLP_CASE(5) SLP_CASE(6) SLP_CASE(7) SLP_CASE(8)
#undef SLP_CASE
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------------- interp ---
// One workgroup per tile holding targets (largest tiles first). The grid values
// of the bounding box of the tile's target stencils (within the tile plus its
// halo) are staged in LDS; then every wave works through its own contiguous
// share of the tile's targets, TPW = 64 / 2m at a time, with no further
// workgroup barrier. A target takes 2m lanes, lane dz summing the stencil
// plane cz + dz: sum over dy of w_y[dy] sum over dx of w_x[dx] g (the 2m values
// of a row in T, the plane in FP64), times w_z[dz]; the 2m plane sums of a
// target are added in a fixed order by one lane, so each target costs its
// (2m)^3 multiply-adds plus O(2m) work and no cross-lane reduction. The target
// data of the next group is loaded one group ahead; the 1-D window factors of
// a group are computed one mirrored pair of stencil points per lane into the
// wave's LDS slice (Gaussian: an exponential per point; Kaiser-Bessel: one
// pass over the fitted polynomial's coefficients, read as scalars). Workgroups
// are sized so that several share a CU (the staged block sets the LDS).
template <typename T, int M>
struct InterpShape {
  static constexpr int W = 2 * M;
  static constexpr int PD = kTile + W - 1;
  static constexpr int P3 = PD * PD * PD;
  static constexpr int TPW = 64 / W;                               // targets per wave pass
  // plane pitch of the staged block: in FP64 with 2m = 8 padded to 2 (mod 16)
  // doubles, so that the 8 lanes of a target, each reading two doubles of its
  // own plane, cover distinct banks (measured: 89 -> 82 us on the film; the
  // same rule at 2m = 16 was slower, 32 -> 44 us on cube64)
  static constexpr int PPL =
      (sizeof(T) == 8 && W == 8) ? PD * PD + (18 - (PD * PD) % 16) % 16 : PD * PD;
  static constexpr int GT = PD * PPL;                              // staged block size
  // LDS of one wave besides the staged block: factors, fractions, cells,
  // caller indices, plane sums
  static constexpr int WAVE_LDS = TPW * (3 * W + 3) * (int)sizeof(T) + TPW * 4 * 4 + 64 * 8;
  static constexpr int fit(int waves) {
    return (160 * 1024) / (GT * (int)sizeof(T) + waves * WAVE_LDS);
  }
  // FP64 with 2m = 8: eight waves share a tile's targets, three workgroups per
  // CU (cube64: 17 -> 14 us; the film, with fewer targets per tile, unchanged)
  static constexpr int WAVES =
      (sizeof(T) == 8 && W == 8) ? 8 : (fit(4) >= 4 ? 4 : (fit(8) >= 2 ? 8 : 16));
  static constexpr int THREADS = WAVES * 64;
  static constexpr int PERG = (P3 + THREADS - 1) / THREADS;       // staged cells per thread
  static constexpr int NLD = (7 * TPW + 63) / 64;                 // target fields per lane
};

// One workgroup for the active tile at position `slot` of a.rec, batch item
// `bitem` (grid bitem * g_bstride further), potentials into `phi`.
template <typename T, int M>
__device__ __forceinline__ void interp_body(const InterpArgs<T> a, double *phi, int64_t slot,
                                            int bitem) {
  using S = InterpShape<T, M>;
  constexpr int W = S::W, PD = S::PD, TPW = S::TPW, D = kb_degree<T, M>();
  __shared__ T gt[S::GT];
  __shared__ T wf[S::WAVES][TPW][3][W];     // window factors of each wave's group
  __shared__ T tfr[S::WAVES][TPW][3];       // fractions of each wave's group
  __shared__ int32_t tcl[S::WAVES][TPW][3]; // cells (in the tile) of each wave's group
  __shared__ int32_t tpm[S::WAVES][TPW];    // caller indices of each wave's group
  __shared__ double psum[S::WAVES][64];     // plane sums

  const int tid = threadIdx.x;
  const int4 rec = a.rec[slot];
  const int tile = rec.x;
  const int tx = tile % a.tiles[0];
  const int ty = (tile / a.tiles[0]) % a.tiles[1];
  const int tz = tile / (a.tiles[0] * a.tiles[1]);
  const int ox = tx * kTile - M + 1, oy = ty * kTile - M + 1, oz = tz * kTile - M + 1;
  const int64_t Rx = a.R[0], Ry = a.R[1];
  const T *gsrc = a.g + bitem * a.g_bstride;
  const int t0 = rec.y, t1 = rec.z;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int64_t nt = a.nt;
  // stencil box of the tile's targets in pad coordinates: cells lo..hi (in
  // the tile) per axis, stencils reaching W - 1 further
  const int32_t box = rec.w;
  const int bx0 = box & 7, by0 = (box >> 3) & 7, bz0 = (box >> 6) & 7;
  const int bx1 = ((box >> 9) & 7) + W - 1, by1 = ((box >> 12) & 7) + W - 1,
            bz1 = ((box >> 15) & 7) + W - 1;
  // this wave's contiguous share of the tile's targets, in groups of TPW
  const int ntile = t1 - t0;
  const int per = ((ntile + S::WAVES - 1) / S::WAVES + TPW - 1) / TPW * TPW;
  const int ws = t0 + wave * per, we = min(t1, ws + per);
  // target data of a group: field f = lane + 64 k (k < NLD) holds item f % TPW,
  // kind f / TPW (0..2 cell, 3..5 fraction, 6 caller index), loaded one group
  // ahead. Every lane loads unconditionally (items past the group's end read
  // its last target, an integer and a fraction per field, the kind choosing
  // only the addresses): a load under a branch leaves other lanes to set its
  // register, and a register written while its load is in flight makes the
  // wave wait for that load.
  int32_t ci[S::NLD];
  T fr[S::NLD];
  auto load_group = [&](int g0) {
#pragma unroll
    for (int k = 0; k < S::NLD; ++k) {
      const int f = lane + 64 * k, item = f % TPW, kind = f / TPW;
      const int64_t i = min(g0 + item, we - 1);
      const int32_t *ip = kind < 3 ? a.cell + kind * nt + i : a.perm + i;
      const int fk = (kind >= 3 && kind < 6) ? kind - 3 : 0;
      ci[k] = *ip;
      fr[k] = a.frac[fk * nt + i];
    }
  };
  // this lane's target in the group and stencil plane
  const int tq = lane / W, dz = lane % W;
  // the first group's target data is loaded together with the staged block
  if (ws < we) load_group(ws);
  {
    // issue every load of the box before writing LDS
    T v[S::PERG];
#pragma unroll
    for (int k = 0; k < S::PERG; ++k) {
      const int i = tid + k * S::THREADS;
      v[k] = T(0);
      if (i < S::P3) {
        const int ix = i % PD, iy = (i / PD) % PD, iz = i / (PD * PD);
        const int gx = ox + ix, gy = oy + iy, gz = oz + iz;
        if (ix >= bx0 && ix <= bx1 && iy >= by0 && iy <= by1 && iz >= bz0 && iz <= bz1 &&
            gx >= 0 && gx < a.R[0] && gy >= 0 && gy < a.R[1] && gz >= 0 && gz < a.R[2])
          v[k] = gsrc[((int64_t)gz * Ry + gy) * Rx + gx];
      }
    }
#pragma unroll
    for (int k = 0; k < S::PERG; ++k) {
      const int i = tid + k * S::THREADS;
      if (i < S::P3) gt[(i / (PD * PD)) * S::PPL + i % (PD * PD)] = v[k];
    }
  }
  __syncthreads();

  for (int g0 = ws; g0 < we; g0 += TPW) {
    const int ng = min(TPW, we - g0);
#pragma unroll
    for (int k = 0; k < S::NLD; ++k) {
      const int f = lane + 64 * k, item = f % TPW, kind = f / TPW;
      if (kind < 7 && item < ng) {
        if (kind < 3) tcl[wave][item][kind] = ci[k];
        else if (kind < 6) tfr[wave][item][kind - 3] = fr[k];
        else tpm[wave][item] = ci[k];
      }
    }
    if (g0 + TPW < we) load_group(g0 + TPW);
    wave_sync();
    // window factors of the group, one mirrored pair of stencil points (j,
    // 2m - 1 - j) per (lane, pass). Gaussian: lanes over (j, axis, target).
    // Kaiser-Bessel: P_j(u) = E_j(u^2) + u O_j(u^2) and P_j(-u) from one pass
    // over the coefficients; one pass per j with the lanes over (axis,
    // target), so that the coefficients are wave-uniform scalar loads (no LDS
    // traffic)
    if (a.window == 0) {
      for (int idx = lane; idx < ng * 3 * M; idx += 64) {
        const int j = idx % M, rest = idx / M;
        const int ax = rest % 3, it = rest / 3;
        const T f = tfr[wave][it][ax];
        const T d0 = f - T(j - M + 1), d1 = f - T(M - j);
        wf[wave][it][ax][j] = wexp(-d0 * d0 * a.inv_b);
        wf[wave][it][ax][W - 1 - j] = wexp(-d1 * d1 * a.inv_b);
      }
    } else {
      const __attribute__((address_space(4))) T *kb =
          (const __attribute__((address_space(4))) T *)a.kb_tab;
      for (int j = 0; j < M; ++j) {
        T c[D + 1];
#pragma unroll
        for (int d = 0; d <= D; ++d) c[d] = kb[j * (D + 1) + d];
        for (int idx = lane; idx < ng * 3; idx += 64) {
          const int ax = idx % 3, it = idx / 3;
          const T u = T(2) * tfr[wave][it][ax] - T(1), v = u * u;
          T e = c[D], o = c[D - 1];
#pragma unroll
          for (int d = D - 2; d >= 0; d -= 2) e = e * v + c[d];
#pragma unroll
          for (int d = D - 3; d >= 1; d -= 2) o = o * v + c[d];
          wf[wave][it][ax][j] = e + u * o;
          wf[wave][it][ax][W - 1 - j] = e - u * o;
        }
      }
    }
    wave_sync();
    if (tq < ng) {
      const int cx = tcl[wave][tq][0] - tx * kTile, cy = tcl[wave][tq][1] - ty * kTile,
                cz = tcl[wave][tq][2] - tz * kTile;
      const T *plane = gt + (cz + dz) * S::PPL + cy * PD + cx;
      T wx[W];
#pragma unroll
      for (int j = 0; j < W; ++j) wx[j] = wf[wave][tq][0][j];
      double acc = 0.0;
#pragma unroll
      for (int dy = 0; dy < W; ++dy) {
        const T *row = plane + dy * PD;
        T s0 = T(0), s1 = T(0);
#pragma unroll
        for (int j = 0; j < W; j += 2) {
          s0 += row[j] * wx[j];
          s1 += row[j + 1] * wx[j + 1];
        }
        acc += (double)(s0 + s1) * (double)wf[wave][tq][1][dy];
      }
      psum[wave][lane] = acc * (double)wf[wave][tq][2][dz];
    }
    wave_sync();
    if (lane < ng) {
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < W; ++k) sum += psum[wave][lane * W + k];
      phi[tpm[wave][lane]] = sum;
    }
    wave_sync();   // the slices are rewritten by the next group
  }
}

template <typename T, int M>
__global__ __launch_bounds__((InterpShape<T, M>::THREADS)) void k_interp(InterpArgs<T> a,
                                                                          BatchPtrs ptrs) {
  interp_body<T, M>(a, ptrs.phi[blockIdx.y], blockIdx.x, blockIdx.y);
}

// Several geometries in one launch: workgroup i takes active tile slot
// work[i].y of item work[i].x (largest tiles first over all items).
template <typename T, int M>
__global__ __launch_bounds__((InterpShape<T, M>::THREADS)) void k_interp_multi(
    const MultiItem<T> *__restrict__ items, const int2 *__restrict__ work, BatchPtrs ptrs) {
  const int2 w = work[blockIdx.x];
  InterpArgs<T> a = items[w.x].ip;
  a.cell = gptr(a.cell);
  a.frac = gptr(a.frac);
  a.perm = gptr(a.perm);
  a.rec = gptr(a.rec);
  a.g = gptr(a.g);
  a.kb_tab = gptr(a.kb_tab);
  interp_body<T, M>(a, gptr(ptrs.phi[w.x]), w.y, 0);
}

template <typename T, int M>
static hipError_t interp_m(const InterpArgs<T> &a, const BatchPtrs &p, int n_active, int nb,
                           hipStream_t s) {
  if (n_active == 0) return hipSuccess;
  hipLaunchKernelGGL((k_interp<T, M>), dim3((unsigned)n_active, (unsigned)nb),
                     dim3(InterpShape<T, M>::THREADS), 0, s, a, p);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interp(const InterpArgs<T> &a, const BatchPtrs &p, int n_active, int m, int nb,
                         hipStream_t s) {
  switch (m) {
    case 1: return interp_m<T, 1>(a, p, n_active, nb, s);
    case 2: return interp_m<T, 2>(a, p, n_active, nb, s);
    case 3: return interp_m<T, 3>(a, p, n_active, nb, s);
    case 4: return interp_m<T, 4>(a, p, n_active, nb, s);
    case 5: return interp_m<T, 5>(a, p, n_active, nb, s);
    case 6: return interp_m<T, 6>(a, p, n_active, nb, s);
    case 7: return interp_m<T, 7>(a, p, n_active, nb, s);
    case 8: return interp_m<T, 8>(a, p, n_active, nb, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int M>
static hipError_t interp_multi_m(const MultiItem<T> *items, const int2 *work, int64_t n,
                                 const BatchPtrs &p, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_interp_multi<T, M>), dim3((unsigned)n), dim3(InterpShape<T, M>::THREADS), 0,
                     s, items, work, p);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interp_multi(const MultiItem<T> *items, const int2 *work, int64_t n, int m,
                               const BatchPtrs &p, hipStream_t s) {
  switch (m) {
#define SLP_CASE(MM) case MM: return interp_multi_m<T, MM>(items, work, n, p, s);
    SLP_CASE(1) SLP_CASE(2) SLP_CASE(3) SLP_CASE(4) SLP_CASE(5) SLP_CASE(6) SLP_CASE(7) SLP_CASE(8)
#undef SLP_CASE
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- density ---
// Element-constant density of the P1 ansatz: the integral mean of the affine
// m . n over a flat triangle is its value at the centroid, i.e. the vertex mean;
// the normal derivative of phi_1 is constant per triangle and subtracted.
__global__ __launch_bounds__(256) void k_density_from_m(const int32_t *__restrict__ tri_v,
                                                        const double *__restrict__ tri_n,
                                                        const double *__restrict__ m_nodes,
                                                        const double *__restrict__ dphi1_dn,
                                                        int64_t M, double *__restrict__ dens) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int64_t a = tri_v[j], b = tri_v[M + j], c = tri_v[2 * M + j];
  double g = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q)
    g += tri_n[q * M + j] * (m_nodes[3 * a + q] + m_nodes[3 * b + q] + m_nodes[3 * c + q]);
  g *= 1.0 / 3.0;
  if (dphi1_dn) g -= dphi1_dn[j];
  dens[j] = g;
  dens[M + j] = g;
  dens[2 * M + j] = g;
}

hipError_t launch_density_from_m(const int32_t *tri_v, const double *tri_n, const double *m_nodes,
                                 const double *dphi1_dn, int64_t n_tris, double *dens,
                                 hipStream_t s) {
  if (n_tris <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_density_from_m, dim3((unsigned)((n_tris + 255) / 256)), dim3(256), 0, s,
                     tri_v, tri_n, m_nodes, dphi1_dn, (int64_t)n_tris, dens);
  return hipGetLastError();
}

// ------------------------------------------------------------ setup (FP64) ---
// c_{t,q}(l) = int_{-1/2}^{1/2} exp(-gamma xi^2) cos(2 pi l xi) dxi (eq. Fcoeff of
// one separable factor), composite Gauss-Legendre on [0, 1/2], doubled.
__global__ void k_chat(double *C, const double *__restrict__ gam, int32_t S, int32_t L,
                       const double *__restrict__ glx, const double *__restrict__ glw,
                       int32_t order, int32_t panels) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)S * L) return;
  const int t = (int)(i / L), l = (int)(i % L);
  const double g = gam[t];
  const double h = 0.5 / panels;
  double acc = 0.0;
  for (int pnl = 0; pnl < panels; ++pnl) {
    const double mid = (pnl + 0.5) * h;
    double part = 0.0;
    for (int j = 0; j < order; ++j) {
      const double xi = mid + 0.5 * h * glx[j];
      part += glw[j] * exp(-g * xi * xi) * cospi(2.0 * l * xi);
    }
    acc += 0.5 * h * part;
  }
  C[i] = 2.0 * acc;
}

hipError_t launch_chat(double *C, const double *gamma_scaled, int32_t S, int32_t L,
                       const double *gl_x, const double *gl_w, int32_t order, int32_t panels,
                       hipStream_t s) {
  const int64_t n = (int64_t)S * L;
  hipLaunchKernelGGL(k_chat, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, C, gamma_scaled,
                     S, L, gl_x, gl_w, order, panels);
  return hipGetLastError();
}

// The multiplier without its Hermitian weight, folded over the signs of ky
// and kz: F(kx, |ky|, |kz|) for kx = 0..n_x/2, |ky| = 0..n_y/2, |kz| = 0..n_z/2
// (layout [n_z/2 + 1][n_y/2 + 1][n_x/2 + 1]), a quarter of the stored half
// spectrum. The z pass multiplies by mu = h(l) F (see fft_mul_weight):
//   F = c_l prod_q exp(2 b (pi l_q / N_q)^2) / (pi b) / (4 pi)
// c_l = sum_t omega_t prod_q c_{t,q}(|l_q|) (Sec. 3.3 separable coefficients),
// exp(2 b ...) / (pi b): the two deconvolutions by the window coefficients
// (eq. deconv and the type-2 counterpart) for the unnormalised window
// exp(-tau^2 / b) (the Kaiser-Bessel window's own factors in its place).
template <typename T>
__global__ void k_mu(T *mu, const double *__restrict__ C0, const double *__restrict__ C1,
                     const double *__restrict__ C2, const double *__restrict__ omega, int32_t S,
                     int3 n, const double *__restrict__ dec0, const double *__restrict__ dec1,
                     const double *__restrict__ dec2) {
  const int Lx = n.x / 2 + 1, Ly = n.y / 2 + 1, Lz = n.z / 2 + 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)Lx * Ly * Lz;
  if (i >= tot) return;
  const int ax = (int)(i % Lx);
  const int ay = (int)((i / Lx) % Ly);
  const int az = (int)(i / ((int64_t)Lx * Ly));
  double c = 0.0;
  for (int t = 0; t < S; ++t)
    c += omega[t] * C0[(int64_t)t * Lx + ax] * C1[(int64_t)t * Ly + ay] * C2[(int64_t)t * Lz + az];
  const double pi = 3.141592653589793238462643383279502884;
  mu[i] = (T)(c * dec0[ax] * dec1[ay] * dec2[az] / (4.0 * pi));
}

template <typename T>
hipError_t launch_mu(T *mu, const double *C0, const double *C1, const double *C2,
                     const double *omega, int32_t S, const int32_t n[3], const double *dec0,
                     const double *dec1, const double *dec2, hipStream_t s) {
  const int64_t tot = (int64_t)(n[0] / 2 + 1) * (n[1] / 2 + 1) * (n[2] / 2 + 1);
  hipLaunchKernelGGL(k_mu<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, mu, C0, C1, C2,
                     omega, S, make_int3(n[0], n[1], n[2]), dec0, dec1, dec2);
  return hipGetLastError();
}

// ------------------------------------------------------------ near field ---
// One wave per target row; lanes take the row's entries in turn. Padding
// entries (column -1) get the value 0. The smooth kernel's share is taken with
// the gridding's quadrature: the three-point rule, or with integrated-window
// gridding the collapsed rule `rule` [npts][3] (xi_1, xi_2, weight).
template <typename T>
__global__ __launch_bounds__(256) void k_near_values(NearArgs<T> a, const double *__restrict__ tg,
                                                     const double *__restrict__ nodes,
                                                     const int32_t *__restrict__ tris,
                                                     const double *__restrict__ es_w,
                                                     const double *__restrict__ es_g,
                                                     int32_t terms, const double *__restrict__ rule,
                                                     int32_t npts) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= a.rows) return;
  const int lane = threadIdx.x & 63;
  const double x[3] = {tg[3 * row], tg[3 * row + 1], tg[3 * row + 2]};
  const int64_t e1 = a.rowptr[row + 1];
  for (int64_t e = a.rowptr[row] + lane; e < e1; e += 64) {
    const int64_t j = a.cols[e];
    if (j < 0) {
      a.vals[e] = (T)0;
      continue;
    }
    double v[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int64_t nd = tris[3 * j + k];
#pragma unroll
      for (int q = 0; q < 3; ++q) v[k][q] = nodes[3 * nd + q];
    }
    const double exact = triangle_potential(x, v[0], v[1], v[2]);
    double e1v[3], e2v[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) { e1v[q] = v[1][q] - v[0][q]; e2v[q] = v[2][q] - v[0][q]; }
    const double cx = e1v[1] * e2v[2] - e1v[2] * e2v[1];
    const double cy = e1v[2] * e2v[0] - e1v[0] * e2v[2];
    const double cz = e1v[0] * e2v[1] - e1v[1] * e2v[0];
    const double area = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    double smooth = 0.0;
    if (rule) {
      for (int p = 0; p < npts; ++p) {
        const double x1 = rule[3 * p], x2 = rule[3 * p + 1];
        double r2 = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const double y = v[0][q] + x1 * e1v[q] + x2 * e2v[q];
          r2 += (x[q] - y) * (x[q] - y);
        }
        double ns = 0.0;
        for (int t = 0; t < terms; ++t) ns += es_w[t] * exp(-es_g[t] * r2);
        smooth += rule[3 * p + 2] * ns;
      }
      smooth *= 2.0 * area;
    } else {
      // quadrature point s: weight 2/3 on vertex s, 1/6 on the other two
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        double r2 = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const double wq0 = (s == 0) ? 4.0 / 6 : 1.0 / 6;
          const double wq1 = (s == 1) ? 4.0 / 6 : 1.0 / 6;
          const double wq2 = (s == 2) ? 4.0 / 6 : 1.0 / 6;
          const double y = wq0 * v[0][q] + wq1 * v[1][q] + wq2 * v[2][q];
          r2 += (x[q] - y) * (x[q] - y);
        }
        for (int t = 0; t < terms; ++t) smooth += es_w[t] * exp(-es_g[t] * r2);
      }
      smooth *= area / 3.0;
    }
    a.vals[e] = (T)(exact - smooth);
  }
}

template <typename T>
hipError_t launch_near_values(const NearArgs<T> &a, const double *targets, const double *nodes,
                              const int32_t *tris, const double *es_w, const double *es_g,
                              int32_t terms, const double *rule, int32_t npts, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_near_values<T>, dim3((unsigned)((a.rows + 3) / 4)), dim3(256), 0, s, a,
                     targets, nodes, tris, es_w, es_g, terms, rule, npts);
  return hipGetLastError();
}

// gbar[item][j] = (g_j + g_{j+M} + g_{j+2M}) / 3 for item = blockIdx.y.
__global__ __launch_bounds__(256) void k_near_gbar(BatchPtrs p, double *__restrict__ gbar,
                                                   int64_t M) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= M) return;
  const double *__restrict__ g = p.dens[blockIdx.y];
  gbar[blockIdx.y * M + j] = (g[j] + g[j + M] + g[j + 2 * M]) * (1.0 / 3.0);
}

// Four entries (their triangles and values) times the element means of IB
// items. Padding entries carry value 0 and read a valid triangle.
template <int IB>
__device__ __forceinline__ void near_group(int64_t j0, int64_t j1, int64_t j2, int64_t j3,
                                           const double v[4], const double *__restrict__ gb,
                                           int64_t M, int n_it, double acc[IB]) {
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    if (i < n_it) {
      const double *__restrict__ g = gb + i * M;
      acc[i] += v[0] * g[j0] + v[1] * g[j1] + v[2] * g[j2] + v[3] * g[j3];
    }
  }
}

__device__ __forceinline__ void load_group(const double *vals, int64_t q, double v[4]) {
  const double2 a = reinterpret_cast<const double2 *>(vals)[2 * q];
  const double2 b = reinterpret_cast<const double2 *>(vals)[2 * q + 1];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void load_group(const float *vals, int64_t q, double v[4]) {
  const float4 a = reinterpret_cast<const float4 *>(vals)[q];
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// Triangles of the group at q: 16-byte column load, or packed base + four
// 16-bit offsets (the base of the chunk q / 64 is the same on every lane).
template <bool PACKED, typename A>
__device__ __forceinline__ void group_cols(const A &a, int64_t q, int64_t j[4]) {
  if constexpr (PACKED) {
    const int32_t base = a.bases[__builtin_amdgcn_readfirstlane((int)(q >> 6))];
    const uint2 o = reinterpret_cast<const uint2 *>(a.offs)[q];
    j[0] = base + (int32_t)(o.x & 0xffffu);
    j[1] = base + (int32_t)(o.x >> 16);
    j[2] = base + (int32_t)(o.y & 0xffffu);
    j[3] = base + (int32_t)(o.y >> 16);
  } else {
    const int4 c = reinterpret_cast<const int4 *>(a.cols)[q];
    j[0] = c.x < 0 ? 0 : c.x;
    j[1] = c.y < 0 ? 0 : c.y;
    j[2] = c.z < 0 ? 0 : c.z;
    j[3] = c.w < 0 ? 0 : c.w;
  }
}

// Lane partials of sum_j A_rj gbar_j for one row of a matrix in the
// near-field layout, L lanes per row: a lane takes groups of four entries, two
// groups in flight; the IB items share the matrix reads. FP64 accumulation.
// (Packed columns need L = 64: a wave reads the base of one chunk.)
template <typename T, int IB, bool PACKED, int L = 64>
__device__ __forceinline__ void row_partials(const NearArgs<T> &a, int64_t row, int lane,
                                             const double *__restrict__ gb, int n_it,
                                             double acc[IB]) {
  static_assert(L == 64 || !PACKED, "packed columns are read a wave per row");
  const int64_t M = a.M;
  const int64_t q1 = a.rowptr[row + 1] / kNearGroup;
  int64_t q = a.rowptr[row] / kNearGroup + lane;
#pragma unroll
  for (int i = 0; i < IB; ++i) acc[i] = 0.0;
  for (; q + L < q1; q += 2 * L) {
    int64_t j0[4], j1[4];
    group_cols<PACKED>(a, q, j0);
    group_cols<PACKED>(a, q + L, j1);
    double v0[4], v1[4];
    load_group(a.vals, q, v0);
    load_group(a.vals, q + L, v1);
    near_group<IB>(j0[0], j0[1], j0[2], j0[3], v0, gb, M, n_it, acc);
    near_group<IB>(j1[0], j1[1], j1[2], j1[3], v1, gb, M, n_it, acc);
  }
  if (q < q1) {
    int64_t j0[4];
    group_cols<PACKED>(a, q, j0);
    double v0[4];
    load_group(a.vals, q, v0);
    near_group<IB>(j0[0], j0[1], j0[2], j0[3], v0, gb, M, n_it, acc);
  }
}

// phi_i += sum_j C_ij gbar_j / (4 pi), one wave per target row.
template <typename T, int IB, bool PACKED>
__global__ __launch_bounds__(256) void k_near_apply(NearArgs<T> a, BatchPtrs p, int32_t nb) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= a.rows) return;
  const int lane = threadIdx.x & 63;
  const int item0 = blockIdx.y * IB;
  const int n_it = nb - item0 < IB ? nb - item0 : IB;
  double acc[IB];
  row_partials<T, IB, PACKED>(a, row, lane, a.gbar + (int64_t)item0 * a.M, n_it, acc);
  const double inv4pi = 1.0 / (4.0 * 3.141592653589793238462643383279502884);
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    double s = acc[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0 && i < n_it) p.phi[item0 + i][row] += s * inv4pi;
  }
}

// ------------------------------------------ integrated-window gridding ---
// A_rj = int_{S_j} prod_q psi(r_q - t_q(y)) [-m < r_q - t_q(y) <= m] dsigma(y)
// for the stored entries (row r = cell of the region, column j = triangle),
// by the collapsed Gauss rule: t(xi) = t_0 + xi_1 (t_1 - t_0) + xi_2 (t_2 - t_0)
// in grid units, dsigma = 2 |S_j| dxi; psi the gridding's window factor.
// One wave per row; padding entries (column -1) get 0.
template <typename T>
__global__ __launch_bounds__(256) void k_iw_values(NearArgs<T> a, IwGeom g) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= a.rows) return;
  const int lane = threadIdx.x & 63;
  const double r[3] = {(double)(g.lo[0] + row % g.R[0]), (double)(g.lo[1] + (row / g.R[0]) % g.R[1]),
                       (double)(g.lo[2] + row / ((int64_t)g.R[0] * g.R[1]))};
  const double m = (double)g.m;
  const int64_t e1 = a.rowptr[row + 1];
  for (int64_t e = a.rowptr[row] + lane; e < e1; e += 64) {
    const int64_t j = a.cols[e];
    if (j < 0) {
      a.vals[e] = (T)0;
      continue;
    }
    const double *tv = g.tv + 9 * j;     // three vertices, grid units
    double acc = 0.0;
    for (int p = 0; p < g.npts; ++p) {
      const double x1 = g.rule[3 * p], x2 = g.rule[3 * p + 1];
      double w = g.rule[3 * p + 2];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double t = tv[q] + x1 * (tv[3 + q] - tv[q]) + x2 * (tv[6 + q] - tv[q]);
        const double tau = r[q] - t;
        if (!(tau > -m && tau <= m)) w = 0.0;
        else if (g.window == 0) w *= exp(-tau * tau * g.inv_b);
        else w *= kb_weight<double>(tau, m, g.b, g.kb_inv_norm);
      }
      acc += w;
    }
    a.vals[e] = (T)(2.0 * g.area[j] * acc);
  }
}

template <typename T>
hipError_t launch_iw_values(const NearArgs<T> &a, const IwGeom &g, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iw_values<T>, dim3((unsigned)((a.rows + 3) / 4)), dim3(256), 0, s, a, g);
  return hipGetLastError();
}

// a_r = sum_j A_rj gbar_j into the region grid of every item, L lanes per
// cell of the region (row = x + R_x (y + R_y z), stored at (z P_y + y) P_x + x):
// a wave per cell for long rows, four cells per wave for short ones.
template <typename T, int IB, bool PACKED, int L>
__global__ __launch_bounds__(256) void k_iw_apply(NearArgs<T> a, IwOut<T> o, int32_t nb) {
  const int64_t row = (int64_t)blockIdx.x * (256 / L) + threadIdx.x / L;
  if (row >= a.rows) return;   // whole groups of L lanes: a row's lanes stay together
  const int lane = threadIdx.x & (L - 1);
  const int item0 = blockIdx.y * IB;
  const int n_it = nb - item0 < IB ? nb - item0 : IB;
  double acc[IB];
  row_partials<T, IB, PACKED, L>(a, row, lane, a.gbar + (int64_t)item0 * a.M, n_it, acc);
  const int64_t x = row % o.R[0], y = (row / o.R[0]) % o.R[1], z = row / ((int64_t)o.R[0] * o.R[1]);
  const int64_t at = (z * o.P[1] + y) * o.P[0] + x;
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    double s = acc[i];
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
    if (lane == 0 && i < n_it) o.grid[(int64_t)(item0 + i) * o.bstride + at] = (T)s;
  }
}

template <typename T, bool PACKED, int L>
void launch_iw_apply_p(const NearArgs<T> &a, const IwOut<T> &o, int nb, hipStream_t s) {
  const int ib = nb >= 8 ? 8 : nb >= 4 ? 4 : nb >= 2 ? 2 : 1;
  constexpr int RPB = 256 / L;
  const dim3 grid((unsigned)((a.rows + RPB - 1) / RPB), (unsigned)((nb + ib - 1) / ib));
  switch (ib) {
    case 8: hipLaunchKernelGGL((k_iw_apply<T, 8, PACKED, L>), grid, dim3(256), 0, s, a, o, nb); break;
    case 4: hipLaunchKernelGGL((k_iw_apply<T, 4, PACKED, L>), grid, dim3(256), 0, s, a, o, nb); break;
    case 2: hipLaunchKernelGGL((k_iw_apply<T, 2, PACKED, L>), grid, dim3(256), 0, s, a, o, nb); break;
    default: hipLaunchKernelGGL((k_iw_apply<T, 1, PACKED, L>), grid, dim3(256), 0, s, a, o, nb); break;
  }
}

template <typename T>
hipError_t launch_iw_apply(const NearArgs<T> &a, const IwOut<T> &o, const BatchPtrs &p, int nb,
                           bool packed, bool short_rows, hipStream_t s) {
  if (a.rows <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_near_gbar, dim3((unsigned)((a.M + 255) / 256), (unsigned)nb), dim3(256), 0,
                     s, p, a.gbar, a.M);
  if (packed)
    launch_iw_apply_p<T, true, 64>(a, o, nb, s);
  else if (short_rows)
    launch_iw_apply_p<T, false, 16>(a, o, nb, s);
  else
    launch_iw_apply_p<T, false, 64>(a, o, nb, s);
  return hipGetLastError();
}

template <typename T, bool PACKED>
const void *near_apply_kernel_p(int nb) {
  if (nb >= 8) return reinterpret_cast<const void *>(&k_near_apply<T, 8, PACKED>);
  if (nb >= 4) return reinterpret_cast<const void *>(&k_near_apply<T, 4, PACKED>);
  if (nb >= 2) return reinterpret_cast<const void *>(&k_near_apply<T, 2, PACKED>);
  return reinterpret_cast<const void *>(&k_near_apply<T, 1, PACKED>);
}

template <typename T>
const void *near_apply_kernel(int nb, bool packed) {
  return packed ? near_apply_kernel_p<T, true>(nb) : near_apply_kernel_p<T, false>(nb);
}

const void *near_gbar_kernel() { return reinterpret_cast<const void *>(&k_near_gbar); }

template <typename T, bool PACKED>
void launch_near_apply_p(const NearArgs<T> &a, const BatchPtrs &p, int nb, hipStream_t s) {
  const int ib = nb >= 8 ? 8 : nb >= 4 ? 4 : nb >= 2 ? 2 : 1;
  const dim3 grid((unsigned)((a.rows + 3) / 4), (unsigned)((nb + ib - 1) / ib));
  switch (ib) {
    case 8: hipLaunchKernelGGL((k_near_apply<T, 8, PACKED>), grid, dim3(256), 0, s, a, p, nb); break;
    case 4: hipLaunchKernelGGL((k_near_apply<T, 4, PACKED>), grid, dim3(256), 0, s, a, p, nb); break;
    case 2: hipLaunchKernelGGL((k_near_apply<T, 2, PACKED>), grid, dim3(256), 0, s, a, p, nb); break;
    default: hipLaunchKernelGGL((k_near_apply<T, 1, PACKED>), grid, dim3(256), 0, s, a, p, nb); break;
  }
}

template <typename T>
hipError_t launch_near_apply(const NearArgs<T> &a, const BatchPtrs &p, int nb, bool packed,
                             hipStream_t s) {
  if (a.rows <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_near_gbar, dim3((unsigned)((a.M + 255) / 256), (unsigned)nb), dim3(256), 0,
                     s, p, a.gbar, a.M);
  if (packed)
    launch_near_apply_p<T, true>(a, p, nb, s);
  else
    launch_near_apply_p<T, false>(a, p, nb, s);
  return hipGetLastError();
}

template <typename T>
const void *spread_bins_kernel(int m) {
  switch (m) {
    case 1: return reinterpret_cast<const void *>(&k_spread_bins<T, 1>);
    case 2: return reinterpret_cast<const void *>(&k_spread_bins<T, 2>);
    case 3: return reinterpret_cast<const void *>(&k_spread_bins<T, 3>);
    case 4: return reinterpret_cast<const void *>(&k_spread_bins<T, 4>);
    case 5: return reinterpret_cast<const void *>(&k_spread_bins<T, 5>);
    case 6: return reinterpret_cast<const void *>(&k_spread_bins<T, 6>);
    case 7: return reinterpret_cast<const void *>(&k_spread_bins<T, 7>);
    case 8: return reinterpret_cast<const void *>(&k_spread_bins<T, 8>);
    default: return nullptr;
  }
}

template <typename T>
const void *interp_kernel(int m) {
  switch (m) {
    case 1: return reinterpret_cast<const void *>(&k_interp<T, 1>);
    case 2: return reinterpret_cast<const void *>(&k_interp<T, 2>);
    case 3: return reinterpret_cast<const void *>(&k_interp<T, 3>);
    case 4: return reinterpret_cast<const void *>(&k_interp<T, 4>);
    case 5: return reinterpret_cast<const void *>(&k_interp<T, 5>);
    case 6: return reinterpret_cast<const void *>(&k_interp<T, 6>);
    case 7: return reinterpret_cast<const void *>(&k_interp<T, 7>);
    case 8: return reinterpret_cast<const void *>(&k_interp<T, 8>);
    default: return nullptr;
  }
}

// explicit instantiations
template const void *spread_bins_kernel<float>(int);
template const void *spread_bins_kernel<double>(int);
template const void *interp_kernel<float>(int);
template const void *interp_kernel<double>(int);
template hipError_t launch_spread<float>(const SpreadBinsArgs<float> &,
                                         const SpreadReduceArgs<float> &, const BatchPtrs &, int,
                                         int, int, int, hipStream_t, hipEvent_t);
template hipError_t launch_spread<double>(const SpreadBinsArgs<double> &,
                                          const SpreadReduceArgs<double> &, const BatchPtrs &,
                                          int, int, int, int, hipStream_t, hipEvent_t);
template hipError_t launch_spread_multi<float>(const MultiItem<float> *, const int2 *, int64_t,
                                               const int2 *, int64_t, int, const BatchPtrs &,
                                               const SpreadBinsArgs<float> &, hipStream_t);
template hipError_t launch_spread_multi<double>(const MultiItem<double> *, const int2 *, int64_t,
                                                const int2 *, int64_t, int, const BatchPtrs &,
                                                const SpreadBinsArgs<double> &, hipStream_t);
template hipError_t launch_interp_multi<float>(const MultiItem<float> *, const int2 *, int64_t, int,
                                               const BatchPtrs &, hipStream_t);
template hipError_t launch_interp_multi<double>(const MultiItem<double> *, const int2 *, int64_t,
                                                int, const BatchPtrs &, hipStream_t);
template hipError_t launch_interp<float>(const InterpArgs<float> &, const BatchPtrs &, int, int,
                                         int, hipStream_t);
template hipError_t launch_interp<double>(const InterpArgs<double> &, const BatchPtrs &, int, int,
                                          int, hipStream_t);
template hipError_t launch_near_values<float>(const NearArgs<float> &, const double *,
                                              const double *, const int32_t *, const double *,
                                              const double *, int32_t, const double *, int32_t,
                                              hipStream_t);
template hipError_t launch_near_values<double>(const NearArgs<double> &, const double *,
                                               const double *, const int32_t *, const double *,
                                               const double *, int32_t, const double *, int32_t,
                                               hipStream_t);
template hipError_t launch_near_apply<float>(const NearArgs<float> &, const BatchPtrs &, int,
                                             bool, hipStream_t);
template hipError_t launch_near_apply<double>(const NearArgs<double> &, const BatchPtrs &, int,
                                              bool, hipStream_t);
template const void *near_apply_kernel<float>(int, bool);
template const void *near_apply_kernel<double>(int, bool);
template hipError_t launch_iw_values<float>(const NearArgs<float> &, const IwGeom &, hipStream_t);
template hipError_t launch_iw_values<double>(const NearArgs<double> &, const IwGeom &, hipStream_t);
template hipError_t launch_iw_apply<float>(const NearArgs<float> &, const IwOut<float> &,
                                           const BatchPtrs &, int, bool, bool, hipStream_t);
template hipError_t launch_iw_apply<double>(const NearArgs<double> &, const IwOut<double> &,
                                            const BatchPtrs &, int, bool, bool, hipStream_t);
template hipError_t launch_mu<float>(float *, const double *, const double *, const double *,
                                     const double *, int32_t, const int32_t[3], const double *,
                                     const double *, const double *, hipStream_t);
template hipError_t launch_mu<double>(double *, const double *, const double *, const double *,
                                      const double *, int32_t, const int32_t[3], const double *,
                                      const double *, const double *, hipStream_t);

}  // namespace slp
