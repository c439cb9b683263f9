// Batched 1-D FFT passes of the pruned 3-D transform (eq. FFT and the
// inverse transform of the type-2 step; the multiplier of eq. deconv and
// Alg. 1 fused into the z pass).
//
// A pass transforms "lines" of a 3-D array along one axis (FftPass). Each
// line of length N is held by TL = N / E threads, E complex elements per
// thread in registers; thread t always holds the positions t + TL i,
// i = 0 .. E-1. The transform is a Stockham autosort FFT whose stages have
// radix E (the last one radix N / E^(s-1)): a stage's butterflies are DFTs of
// size R evaluated in registers, and between stages the line goes once
// through LDS (write in Stockham order, read back positions t + TL i). The
// first stage reads its inputs straight from global memory and the last one
// leaves its outputs in the registers whose positions they belong to, so a
// 1024-point line costs three LDS round trips at E = 8 (radices 8, 8, 8, 2)
// instead of nine radix-2 or five radix-4 passes.
//
// Two lane maps:
//  * contiguous lines (element stride 1, the x passes): the TL threads of a
//    line are consecutive lanes, so a wave reads consecutive elements;
//  * strided lines (y and z passes, element stride > 1, consecutive lines
//    adjacent in memory): consecutive lanes take G consecutive lines at the
//    same element, so a wave reads runs of G adjacent complex values (at least
//    64 bytes) instead of one value per cache line. The LDS copy of the lines
//    is then stored element-major ([position][line]).
// LDS positions are padded by one slot per R0 (the first radix), which keeps
// the strided writes of the first exchange free of bank conflicts.
//
// Workgroups are renumbered so that each of the eight XCDs (which receive
// consecutive workgroups round robin and have their own L2) processes a
// contiguous range of line groups: neighbouring groups share cache lines.
#include "slp_internal.hpp"

#include <hip/hip_runtime.h>

namespace slp {

namespace {

template <typename T>
struct Cx;
template <>
struct Cx<float> { using type = float2; };
template <>
struct Cx<double> { using type = double2; };

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }

// cos(2 pi k / 16) for k = 0..4
constexpr double kCos16[5] = {1.0, 0.92387953251128675612818318939678829,
                              0.70710678118654752440084436210484904,
                              0.38268343236508977172845998403039886, 0.0};

// b * exp(sign 2 pi i q / 16), q = 0..7 (compile-time q)
template <int SIGN, int Q, typename C>
__device__ __forceinline__ C rot16(C b) {
  using T = decltype(b.x);
  static_assert(Q >= 0 && Q < 8, "rotation index");
  if constexpr (Q == 0) {
    return b;
  } else if constexpr (Q == 4) {
    C r;   // multiply by sign * i
    r.x = SIGN > 0 ? -b.y : b.y;
    r.y = SIGN > 0 ? b.x : -b.x;
    return r;
  } else {
    constexpr double c = Q < 4 ? kCos16[Q] : -kCos16[8 - Q];
    constexpr double s0 = Q < 4 ? kCos16[4 - Q] : kCos16[Q - 4];
    constexpr double s = SIGN > 0 ? s0 : -s0;
    C r;
    r.x = b.x * (T)c - b.y * (T)s;
    r.y = b.x * (T)s + b.y * (T)c;
    return r;
  }
}

constexpr int bitrev(int i, int R) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r <<= 1;
    if (i & b) r |= 1;
  }
  return r;
}

// One radix-2 butterfly group of the in-register DFT: for the block starting
// at I of length LEN, pair K with K + LEN/2.
template <int SIGN, int R, int LEN, int I, int K, typename C>
__device__ __forceinline__ void dft_bf(C (&y)[R]) {
  if constexpr (K < LEN / 2) {
    const C a = y[I + K];
    const C b = rot16<SIGN, K * (16 / LEN)>(y[I + K + LEN / 2]);
    y[I + K] = cadd(a, b);
    y[I + K + LEN / 2] = csub(a, b);
    dft_bf<SIGN, R, LEN, I, K + 1>(y);
  }
}
template <int SIGN, int R, int LEN, int I, typename C>
__device__ __forceinline__ void dft_blocks(C (&y)[R]) {
  if constexpr (I < R) {
    dft_bf<SIGN, R, LEN, I, 0>(y);
    dft_blocks<SIGN, R, LEN, I + LEN>(y);
  }
}
template <int SIGN, int R, int LEN, typename C>
__device__ __forceinline__ void dft_levels(C (&y)[R]) {
  if constexpr (LEN <= R) {
    dft_blocks<SIGN, R, LEN, 0>(y);
    dft_levels<SIGN, R, LEN * 2>(y);
  }
}

// In-place DFT of size R (2, 4, 8 or 16) in registers:
// x_k <- sum_j x_j exp(sign 2 pi i j k / R) (radix-2 decimation in time).
template <int SIGN, int R, typename C>
__device__ __forceinline__ void dft(C (&x)[R]) {
  static_assert(R == 2 || R == 4 || R == 8 || R == 16, "radix");
  C y[R];
#pragma unroll
  for (int i = 0; i < R; ++i) y[bitrev(i, R)] = x[i];
  dft_levels<SIGN, R, 2>(y);
#pragma unroll
  for (int i = 0; i < R; ++i) x[i] = y[i];
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

template <typename T, int N, bool STRIDED>
struct FftCfg {
  using C = typename Cx<T>::type;
  static constexpr int NL = N;                       // line length
  static constexpr bool STR = STRIDED;
  // elements per thread: 8 (radix-8 stages) for lines of 64 and more, 16
  // below: 16 complex values and the radix-16 temporaries take 200+ VGPRs in
  // FP64 (two waves per SIMD) and 155+ in FP32; at 8 the kernels fit 128
  // VGPRs, four waves per SIMD (MINW), for one more LDS round trip per line
  static constexpr int E = N < 16 ? N : (N >= 64 ? 8 : 16);
  static constexpr int MINW = N >= 64 ? 4 : 1;
  static constexpr int TL = N / E;                   // threads per line
  static constexpr int STAGES = (ilog2(N) + ilog2(E) - 1) / ilog2(E);
  static constexpr int R0 = E;                       // first radix
  static constexpr int NPAD = N + N / R0;            // padded LDS positions per line
  static constexpr int GMIN = STRIDED ? (64 / (int)sizeof(C) > 1 ? 64 / (int)sizeof(C) : 1) : 1;
  static constexpr int G0 = 256 / TL > GMIN ? 256 / TL : GMIN;
  static constexpr int LDS_CAP = 80 * 1024;
  static constexpr int G1 = G0 * NPAD * (int)sizeof(C) > LDS_CAP
                                ? (LDS_CAP / (NPAD * (int)sizeof(C)) > 0 ? LDS_CAP / (NPAD * (int)sizeof(C)) : 1)
                                : G0;
  static constexpr int G = STAGES > 1 ? G1 : G0;     // lines per workgroup
  static constexpr int THREADS = G * TL;
  static constexpr int LDS = STAGES > 1 ? G * NPAD : 1;
  // radix of stage s and the product of the radices before it
  static constexpr int radix(int s) {
    return s < STAGES - 1 ? E : N / ipow(E, STAGES - 1);
  }
  static constexpr int span(int s) { return ipow(E, s); }
  static constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
  // LDS slot of (padded) position pp of a line: line-major for contiguous
  // lines, position-major for strided ones
  static __device__ __forceinline__ int slot(int pos, int line) {
    const int pp = pos + pos / R0;
    return STRIDED ? pp * G + line : line * NPAD + pp;
  }
};

// Logical workgroup index: the hardware hands consecutive workgroups to the
// eight XCDs in turn; give each XCD a contiguous range instead.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblk) {
  constexpr int64_t kXcd = 8;
  const int64_t q = nblk / kXcd, r = nblk % kXcd;
  const int64_t x = b % kXcd, i = b / kXcd;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// One Stockham stage for the thread's E registers. Butterfly j = t + b TL
// (b < E / R) takes positions j + r N / R = t + TL (b + r E / R), i.e.
// registers b + r E / R; with k = j mod Ns, input r is twiddled by
// w^(r k), w = exp(sign 2 pi i / (R Ns)), and output r belongs at position
// (j - k) R + k + r Ns. The last stage (R Ns = N) keeps each output in the
// register it came from; others write it to LDS.
template <typename F, int S, int SIGN, bool LAST, int TWS>
__device__ __forceinline__ void fft_stage(typename F::C (&v)[F::E], int t, int line,
                                          const typename F::C *__restrict__ tw,
                                          typename F::C *lds) {
  using C = typename F::C;
  constexpr int R = F::radix(S);
  constexpr int NS = F::span(S);
  constexpr int NB = F::E / R;                         // butterflies per thread
  static_assert(F::TL * F::E == F::NL && NB * R == F::E, "plan");
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + b * F::TL;
    const int k = j & (NS - 1);
    C x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = v[b + r * NB];
    if constexpr (NS > 1) {
      constexpr int step = F::NL / (R * NS);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C w = tw[r * k * step * TWS];
        if (SIGN > 0) w.y = -w.y;
        x[r] = cmul(x[r], w);
      }
    }
    dft<SIGN, R>(x);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + r * NB] = x[r];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        lds[F::slot((j - k) * R + k + r * NS, line)] = x[r];
      }
    }
  }
}

// Read positions t + TL i of the line back from LDS.
template <typename F>
__device__ __forceinline__ void lds_gather(typename F::C (&v)[F::E], int t, int line,
                                           const typename F::C *lds) {
#pragma unroll
  for (int i = 0; i < F::E; ++i) v[i] = lds[F::slot(t + F::TL * i, line)];
}

// All stages of one transform direction, from registers to registers. The
// twiddle table holds exp(-2 pi i k / (TWS N)) (a table of a TWS times longer
// transform, read with stride TWS).
template <typename F, int SIGN, int TWS = 1, int S = 0>
__device__ __forceinline__ void fft_all(typename F::C (&v)[F::E], int t, int line,
                                        const typename F::C *__restrict__ tw,
                                        typename F::C *lds) {
  if constexpr (S < F::STAGES) {
    constexpr bool last = S == F::STAGES - 1;
    fft_stage<F, S, SIGN, last, TWS>(v, t, line, tw, lds);
    if constexpr (!last) {
      __syncthreads();
      lds_gather<F>(v, t, line, lds);
      __syncthreads();
    }
    fft_all<F, SIGN, TWS, S + 1>(v, t, line, tw, lds);
  }
}

template <typename F>
__device__ __forceinline__ void fft_dir(typename F::C (&v)[F::E], int sign, int t, int line,
                                        const typename F::C *__restrict__ tw,
                                        typename F::C *lds) {
  if (sign < 0) fft_all<F, -1>(v, t, line, tw, lds);
  else fft_all<F, +1>(v, t, line, tw, lds);
}

// The multiplier at mode (kx, ky, kz) of a z-pass line (kx, ky index) and
// element kz index em: h(l) F(kx, |ky|, |kz|), with the weight
// h(l) = ([l in I_n] + [-l in I_n]) / 2 of the asymmetric index set I_n
// (1 inside, 1/2 or 0 on its boundary planes; exact in T).
template <typename T>
__device__ __forceinline__ T mu_at(const FftPass<T> &p, int2 line, int em) {
  const int hx = p.mu_n[0] / 2, hy = p.mu_n[1] / 2, hz = p.mu_n[2] / 2;
  const int kx = line.x, ky = line.y - hy, kz = em - hz;
  const bool in_i = kx <= hx - 1 && ky >= -hy && ky <= hy - 1 && kz >= -hz && kz <= hz - 1;
  const bool in_mi = kx >= -hx + 1 && ky >= -hy + 1 && ky <= hy && kz >= -hz + 1 && kz <= hz;
  const int ay = ky < 0 ? -ky : ky, az = kz < 0 ? -kz : kz;
  const T f = p.mu[((int64_t)az * (hy + 1) + ay) * (hx + 1) + kx];
  return (in_i && in_mi) ? f : ((in_i || in_mi) ? T(0.5) * f : T(0));
}

// A pass read from a table in memory, its pointers marked as pointing to
// global memory (so that accesses through them are global rather than flat
// instructions).
template <typename P>
__device__ __forceinline__ P *gptr(P *p) {
  return (P *)(__attribute__((address_space(1))) P *)(uintptr_t)p;
}
template <typename T>
__device__ __forceinline__ FftPass<T> global_pass(const FftPass<T> &q) {
  FftPass<T> p = q;
  p.in = gptr(p.in);
  p.out = gptr(p.out);
  p.tw = gptr(p.tw);
  p.mu = gptr(p.mu);
  return p;
}

// Lines blk G .. blk G + G - 1 of pass p for batch item `item`.
template <typename T, int N, bool STRIDED, bool MULINV>
__device__ __forceinline__ void fft_body(const FftPass<T> p, int64_t item, int64_t blk) {
  using F = FftCfg<T, N, STRIDED>;
  using C = typename F::C;
  constexpr int E = F::E, TL = F::TL, G = F::G;
  __shared__ C lds[F::LDS];
  const C *tw = reinterpret_cast<const C *>(p.tw);
  const int tid = threadIdx.x;
  const int line = STRIDED ? tid % G : tid / TL;
  const int t = STRIDED ? tid / G : tid % TL;
  const int64_t L = blk * G + line;
  const bool live = L < p.n_lines;
  int64_t ibase = 0, obase = 0;
  int2 mline = make_int2(0, 0);   // (kx, ky index) of a z-pass line
  if (live) {
    const int64_t l1i = L % p.l1, l2i = L / p.l1;
    mline = make_int2((int)l1i, (int)l2i);
    ibase = l1i * p.in_s1 + l2i * p.in_s2 + item * p.in_bstride;
    obase = l1i * p.out_s1 + l2i * p.out_s2 + item * p.out_bstride;
  }
  // gather: position pos holds element (pos - in_shift) mod N if that is
  // below in_cnt; a Hermitian input also fills position pos with
  // conj(element N - pos); every other position is zero
  C v[E];
  T mu[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int pos = t + TL * i;
    const int e = (pos - p.in_shift) & (N - 1);
    v[i].x = T(0);
    v[i].y = T(0);
    if (live) {
      if (e < p.in_cnt) {
        const int64_t off = ibase + (int64_t)e * p.in_es;
        if (p.in_real) v[i].x = reinterpret_cast<const T *>(p.in)[off];
        else v[i] = reinterpret_cast<const C *>(p.in)[off];
      } else if (p.in_hermitian && pos > 0 && N - pos < p.in_cnt) {
        const C c = reinterpret_cast<const C *>(p.in)[ibase + (int64_t)(N - pos) * p.in_es];
        v[i].x = c.x;
        v[i].y = -c.y;
      }
    }
    mu[i] = T(0);
    if (MULINV && live) {
      const int em = (pos - p.mu_shift) & (N - 1);
      if (em < p.mu_cnt) mu[i] = mu_at(p, mline, em);
    }
  }
  fft_dir<F>(v, p.sign, t, line, tw, lds);
  if constexpr (MULINV) {
    // registers hold positions t + TL i again: multiply and transform back
#pragma unroll
    for (int i = 0; i < E; ++i) {
      v[i].x *= mu[i];
      v[i].y *= mu[i];
    }
    fft_dir<F>(v, -p.sign, t, line, tw, lds);
  }
  if (!live) return;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int pos = t + TL * i;
    const int e = (pos - p.out_shift) & (N - 1);
    if (e < p.out_cnt) {
      const int64_t off = obase + (int64_t)e * p.out_es;
      if (p.out_real) reinterpret_cast<T *>(p.out)[off] = v[i].x;
      else reinterpret_cast<C *>(p.out)[off] = v[i];
    }
  }
}

template <typename T, int N, bool STRIDED, bool MULINV>
__global__ __launch_bounds__((FftCfg<T, N, STRIDED>::THREADS), (FftCfg<T, N, STRIDED>::MINW)) void k_fft(FftPass<T> p) {
  const int64_t nblk = (int64_t)gridDim.x * gridDim.y;
  const int64_t lb = xcd_block((int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x, nblk);
  fft_body<T, N, STRIDED, MULINV>(p, lb / gridDim.x, lb % gridDim.x);
}

// Several passes (one per geometry of a batch) in one launch: logical
// workgroup i takes block work[i].y of pass work[i].x.
template <typename T, int N, bool STRIDED, bool MULINV>
__global__ __launch_bounds__((FftCfg<T, N, STRIDED>::THREADS), (FftCfg<T, N, STRIDED>::MINW)) void k_fft_multi(
    const FftPass<T> *__restrict__ passes, const int2 *__restrict__ work) {
  const int2 w = work[xcd_block(blockIdx.x, gridDim.x)];
  fft_body<T, N, STRIDED, MULINV>(global_pass(passes[w.x]), 0, w.y);
}

// Real lines of length N (contiguous lines only) through a complex transform
// of length N / 2, which halves the butterflies, the registers and the LDS
// per line. Forward (real in, half spectrum out): the line is packed as
// z[k] = a[2k] + i a[2k+1]; with Z = FFT(z), E[l] = (Z[l] + conj Z[N/2 - l]) / 2
// and O[l] = -i (Z[l] - conj Z[N/2 - l]) / 2 are the transforms of the even and
// odd samples, and X[l] = E[l] + w^l O[l], w = exp(sign 2 pi i / N), for
// l = 0 .. N/2 (X[N/2] = E[0] - O[0]). Inverse (half spectrum X[0 .. N/2] in,
// Hermitian, real out): Z[l] = (X[l] + conj X[N/2 - l]) + i (X[l] - conj
// X[N/2 - l]) w^l, and z = FFT(Z) holds a[2k] + i a[2k+1]. The pairing of l
// with N/2 - l goes through LDS (forward) or is read from global memory
// (inverse).
template <typename T, int N>
__device__ __forceinline__ void fft_real_body(const FftPass<T> p, int64_t item, int64_t blk) {
  constexpr int NH = N / 2;
  using F = FftCfg<T, NH, false>;
  using C = typename F::C;
  constexpr int E = F::E, TL = F::TL, G = F::G;
  static_assert(F::STAGES > 1, "the pairing exchange uses the stages' LDS");
  __shared__ C lds[G * F::NPAD];
  const C *tw = reinterpret_cast<const C *>(p.tw);
  const int tid = threadIdx.x;
  const int line = tid / TL, t = tid % TL;
  const int64_t L = blk * G + line;
  const bool live = L < p.n_lines;
  int64_t ibase = 0, obase = 0;
  if (live) {
    const int64_t l1i = L % p.l1, l2i = L / p.l1;
    ibase = l1i * p.in_s1 + l2i * p.in_s2 + item * p.in_bstride;
    obase = l1i * p.out_s1 + l2i * p.out_s2 + item * p.out_bstride;
  }
  const bool fwd = !p.out_real;
  // w^l = exp(sign 2 pi i l / N) from the table of exp(-2 pi i k / N)
  auto wl = [&](int l) {
    C w = tw[l];
    if (p.sign > 0) w.y = -w.y;
    return w;
  };
  C v[E];
  if (fwd) {
    const T *in = reinterpret_cast<const T *>(p.in);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int k = t + TL * i;
      const int e0 = (2 * k - p.in_shift) & (N - 1), e1 = (2 * k + 1 - p.in_shift) & (N - 1);
      v[i].x = live && e0 < p.in_cnt ? in[ibase + e0] : T(0);
      v[i].y = live && e1 < p.in_cnt ? in[ibase + e1] : T(0);
    }
    if (p.sign < 0) fft_all<F, -1, 2>(v, t, line, tw, lds);
    else fft_all<F, +1, 2>(v, t, line, tw, lds);
#pragma unroll
    for (int i = 0; i < E; ++i) lds[F::slot(t + TL * i, line)] = v[i];
    __syncthreads();
    if (!live) return;
    C *out = reinterpret_cast<C *>(p.out);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int l = t + TL * i;
      if (l >= p.out_cnt) continue;
      const C zl = v[i], zm = lds[F::slot((NH - l) & (NH - 1), line)];
      C ev, od;
      ev.x = T(0.5) * (zl.x + zm.x);
      ev.y = T(0.5) * (zl.y - zm.y);
      od.x = T(0.5) * (zl.y + zm.y);
      od.y = T(-0.5) * (zl.x - zm.x);
      out[obase + l] = cadd(ev, cmul(wl(l), od));
    }
    if (t == 0 && NH < p.out_cnt) {
      C x;
      x.x = v[0].x - v[0].y;
      x.y = T(0);
      out[obase + NH] = x;
    }
  } else {
    const C *in = reinterpret_cast<const C *>(p.in);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int l = t + TL * i, j = NH - l;
      C xl, xm;
      xl.x = xl.y = xm.x = xm.y = T(0);
      if (live && l < p.in_cnt) xl = in[ibase + l];
      if (live && j < p.in_cnt) xm = in[ibase + j];
      C a, b;
      a.x = xl.x + xm.x;
      a.y = xl.y - xm.y;
      b.x = xl.x - xm.x;
      b.y = xl.y + xm.y;
      const C bw = cmul(b, wl(l));
      v[i].x = a.x - bw.y;
      v[i].y = a.y + bw.x;
    }
    if (p.sign < 0) fft_all<F, -1, 2>(v, t, line, tw, lds);
    else fft_all<F, +1, 2>(v, t, line, tw, lds);
    if (!live) return;
    T *out = reinterpret_cast<T *>(p.out);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int k = t + TL * i;
      const int e0 = (2 * k - p.out_shift) & (N - 1), e1 = (2 * k + 1 - p.out_shift) & (N - 1);
      if (e0 < p.out_cnt) out[obase + e0] = v[i].x;
      if (e1 < p.out_cnt) out[obase + e1] = v[i].y;
    }
  }
}

template <typename T, int N>
__global__ __launch_bounds__((FftCfg<T, N / 2, false>::THREADS), (FftCfg<T, N / 2, false>::MINW)) void k_fft_real(FftPass<T> p) {
  const int64_t nblk = (int64_t)gridDim.x * gridDim.y;
  const int64_t lb = xcd_block((int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x, nblk);
  fft_real_body<T, N>(p, lb / gridDim.x, lb % gridDim.x);
}

template <typename T, int N>
__global__ __launch_bounds__((FftCfg<T, N / 2, false>::THREADS), (FftCfg<T, N / 2, false>::MINW)) void k_fft_real_multi(
    const FftPass<T> *__restrict__ passes, const int2 *__restrict__ work) {
  const int2 w = work[xcd_block(blockIdx.x, gridDim.x)];
  fft_real_body<T, N>(global_pass(passes[w.x]), 0, w.y);
}

// Which kernel takes pass p of length N: 0 / 1 contiguous lines without /
// with the fused multiply-and-inverse, 2 / 3 the same on strided lines, 4 real
// contiguous lines through the half-length transform; -1 if unsupported.
template <typename T, int N>
int fft_kind(const FftPass<T> &p) {
  // both sides of a pass use the same lane map
  if ((p.in_es == 1) != (p.out_es == 1)) return -1;
  if (p.in_hermitian && p.in_shift != 0) return -1;
  if constexpr (N >= 64) {
    // real contiguous lines: half-length complex transform
    const bool r2c = p.in_real && !p.in_hermitian && !p.out_real && p.out_shift == 0 &&
                     p.out_cnt <= N / 2 + 1;
    const bool c2r = p.in_hermitian && !p.in_real && p.out_real && p.in_shift == 0 &&
                     p.in_cnt <= N / 2 + 1;
    if (p.in_es == 1 && !p.mul_inv && (r2c || c2r)) return 4;
  }
  return (p.in_es == 1 ? 0 : 2) + (p.mul_inv ? 1 : 0);
}

// Lines per workgroup of kernel `kind`.
template <typename T, int N>
int fft_lines(int kind) {
  if (kind == 4) return FftCfg<T, N / 2, false>::G;
  return kind >= 2 ? FftCfg<T, N, true>::G : FftCfg<T, N, false>::G;
}

template <typename T, int N>
int fft_threads(int kind) {
  if (kind == 4) return FftCfg<T, N / 2, false>::THREADS;
  return kind >= 2 ? FftCfg<T, N, true>::THREADS : FftCfg<T, N, false>::THREADS;
}

template <typename T, int N>
hipError_t fft_map(const FftPass<T> &p, int nb, hipStream_t s) {
  const int kind = fft_kind<T, N>(p);
  if (kind < 0) return hipErrorInvalidValue;
  if (p.n_lines == 0) return hipSuccess;
  const int G = fft_lines<T, N>(kind);
  const dim3 grid((unsigned)((p.n_lines + G - 1) / G), (unsigned)nb), block(fft_threads<T, N>(kind));
  // the fused multiply-and-inverse form (the z pass) is a kernel of its own,
  // so that the other passes do not hold its registers
  switch (kind) {
    case 0: hipLaunchKernelGGL((k_fft<T, N, false, false>), grid, block, 0, s, p); break;
    case 1: hipLaunchKernelGGL((k_fft<T, N, false, true>), grid, block, 0, s, p); break;
    case 2: hipLaunchKernelGGL((k_fft<T, N, true, false>), grid, block, 0, s, p); break;
    case 3: hipLaunchKernelGGL((k_fft<T, N, true, true>), grid, block, 0, s, p); break;
    default:
      if constexpr (N >= 64) hipLaunchKernelGGL((k_fft_real<T, N>), grid, block, 0, s, p);
      else return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int N>
hipError_t fft_map_multi(int kind, const FftPass<T> *passes, const int2 *work, int64_t n,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)n), block(fft_threads<T, N>(kind));
  switch (kind) {
    case 0: hipLaunchKernelGGL((k_fft_multi<T, N, false, false>), grid, block, 0, s, passes, work); break;
    case 1: hipLaunchKernelGGL((k_fft_multi<T, N, false, true>), grid, block, 0, s, passes, work); break;
    case 2: hipLaunchKernelGGL((k_fft_multi<T, N, true, false>), grid, block, 0, s, passes, work); break;
    case 3: hipLaunchKernelGGL((k_fft_multi<T, N, true, true>), grid, block, 0, s, passes, work); break;
    case 4:
      if constexpr (N >= 64) {
        hipLaunchKernelGGL((k_fft_real_multi<T, N>), grid, block, 0, s, passes, work);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int N>
int fft_variant_n(const FftPass<T> &p, int64_t *blocks) {
  const int kind = fft_kind<T, N>(p);
  if (kind >= 0) {
    const int G = fft_lines<T, N>(kind);
    *blocks = (p.n_lines + G - 1) / G;
  }
  return kind;
}

}  // namespace

#define SLP_FFT_SIZES(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048)

template <typename T>
hipError_t launch_fft(const FftPass<T> &p, int N, int nb, hipStream_t s) {
  switch (N) {
#define SLP_CASE(SZ) case SZ: return fft_map<T, SZ>(p, nb, s);
    SLP_FFT_SIZES(SLP_CASE)
#undef SLP_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
int fft_variant(const FftPass<T> &p, int N, int64_t *blocks) {
  *blocks = 0;
  switch (N) {
#define SLP_CASE(SZ) case SZ: return fft_variant_n<T, SZ>(p, blocks);
    SLP_FFT_SIZES(SLP_CASE)
#undef SLP_CASE
    default: return -1;
  }
}

template <typename T>
hipError_t launch_fft_multi(int variant, int N, const FftPass<T> *passes, const int2 *work,
                            int64_t n, hipStream_t s) {
  switch (N) {
#define SLP_CASE(SZ) case SZ: return fft_map_multi<T, SZ>(variant, passes, work, n, s);
    SLP_FFT_SIZES(SLP_CASE)
#undef SLP_CASE
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_fft<float>(const FftPass<float> &, int, int, hipStream_t);
template hipError_t launch_fft<double>(const FftPass<double> &, int, int, hipStream_t);
template int fft_variant<float>(const FftPass<float> &, int, int64_t *);
template int fft_variant<double>(const FftPass<double> &, int, int64_t *);
template hipError_t launch_fft_multi<float>(int, int, const FftPass<float> *, const int2 *,
                                            int64_t, hipStream_t);
template hipError_t launch_fft_multi<double>(int, int, const FftPass<double> *, const int2 *,
                                             int64_t, hipStream_t);

}  // namespace slp
