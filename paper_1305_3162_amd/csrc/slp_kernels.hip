// Device code for the smooth-part single-layer potential (gfx950).
//
// Stages (Sec. 3, Alg. 1 computation phase, eq. BEM_NFFT_compact2):
//   charges  q = w * g gathered into tile order             (eq. naive_gridding)
//   spread   a_r = sum_k q_k prod_q psi(t_kq - r_q)         (eq. gridding)
//   fft      pruned 3-D FFT, multiply by mu, inverse FFT    (eq. FFT, deconv, Alg. 1)
//   interp   phi_i = sum_r g_r prod_q psi(t_iq - r_q)       (type-2 NFFT)
// mu folds the two window deconvolutions, c_l(N_s), the Hermitian weights of
// the asymmetric index set and 1/(4 pi) into one real factor per mode.
#include "slp_internal.hpp"

#include <hip/hip_runtime.h>

namespace slp {

template <typename T>
struct Cplx;
template <>
struct Cplx<float> { using type = float2; };
template <>
struct Cplx<double> { using type = double2; };

__device__ __forceinline__ float wexp(float x) { return __expf(x); }
__device__ __forceinline__ double wexp(double x) { return exp(x); }

// ---------------------------------------------------------------- charges ---
template <typename T>
__global__ void k_charges(const double *__restrict__ dens, const double *__restrict__ w,
                          const int32_t *__restrict__ perm, T *__restrict__ q, int64_t ns) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) q[i] = (T)(w[i] * dens[perm[i]]);
}

template <typename T>
hipError_t launch_charges(const double *dens, const double *w, const int32_t *perm, T *q,
                          int64_t ns, hipStream_t s) {
  if (ns == 0) return hipSuccess;
  int64_t blocks = (ns + 255) / 256;
  hipLaunchKernelGGL(k_charges<T>, dim3((unsigned)blocks), dim3(256), 0, s, dens, w, perm, q, ns);
  return hipGetLastError();
}

// ----------------------------------------------------------------- spread ---
// One 64-lane workgroup owns one 8x8x8 output tile: lane (x, y) keeps the 8
// z-cells of its column in registers. Sources whose stencil can reach the tile
// are read from the neighbouring bins; per source the lanes first build the
// tile-restricted 1-D window factors in LDS, then every lane accumulates
// q wx(x) wy(y) wz(z). Each output cell is written once, without atomics.
template <typename T, int M>
__global__ __launch_bounds__(64) void k_spread(SpreadArgs<T> a) {
  constexpr int TL = kTile;
  constexpr int RLO = (M + TL - 1) / TL;       // bins below that can reach the tile
  constexpr int RHI = (TL + M - 2) / TL;       // bins above
  __shared__ T W[64][3 * TL + 1];

  const int tile = blockIdx.x;
  const int tx = tile % a.tiles[0];
  const int ty = (tile / a.tiles[0]) % a.tiles[1];
  const int tz = tile / (a.tiles[0] * a.tiles[1]);
  const int X0 = tx * TL, Y0 = ty * TL, Z0 = tz * TL;
  const int lane = threadIdx.x;
  const int x = lane & 7, y = lane >> 3;
  const int64_t ns = a.ns;

  T acc[TL];
#pragma unroll
  for (int z = 0; z < TL; ++z) acc[z] = T(0);

  for (int dz = -RLO; dz <= RHI; ++dz) {
    const int bz = tz + dz;
    if (bz < 0 || bz >= a.tiles[2]) continue;
    for (int dy = -RLO; dy <= RHI; ++dy) {
      const int by = ty + dy;
      if (by < 0 || by >= a.tiles[1]) continue;
      for (int dx = -RLO; dx <= RHI; ++dx) {
        const int bx = tx + dx;
        if (bx < 0 || bx >= a.tiles[0]) continue;
        const int bin = bx + a.tiles[0] * (by + a.tiles[1] * bz);
        const int s0 = a.bin_start[bin], s1 = a.bin_start[bin + 1];
        for (int c = s0; c < s1; c += 64) {
          const int s = c + lane;
          if (s < s1) {
            const int cx = a.cell[s], cy = a.cell[ns + s], cz = a.cell[2 * ns + s];
            const T fx = a.frac[s], fy = a.frac[ns + s], fz = a.frac[2 * ns + s];
            const T qv = a.q[s];
#pragma unroll
            for (int j = 0; j < TL; ++j) {
              const int kx = X0 + j - cx, ky = Y0 + j - cy, kz = Z0 + j - cz;
              const T ddx = fx - (T)kx, ddy = fy - (T)ky, ddz = fz - (T)kz;
              W[lane][j] = (kx > -M && kx <= M) ? qv * wexp(-ddx * ddx * a.inv_b) : T(0);
              W[lane][TL + j] = (ky > -M && ky <= M) ? wexp(-ddy * ddy * a.inv_b) : T(0);
              W[lane][2 * TL + j] = (kz > -M && kz <= M) ? wexp(-ddz * ddz * a.inv_b) : T(0);
            }
          }
          __syncthreads();
          const int cnt = min(64, s1 - c);
          for (int si = 0; si < cnt; ++si) {
            const T p = W[si][x] * W[si][TL + y];
#pragma unroll
            for (int z = 0; z < TL; ++z) acc[z] += p * W[si][2 * TL + z];
          }
          __syncthreads();
        }
      }
    }
  }
  const int64_t Px = (int64_t)a.tiles[0] * TL, Py = (int64_t)a.tiles[1] * TL;
#pragma unroll
  for (int z = 0; z < TL; ++z)
    a.grid[((int64_t)(Z0 + z) * Py + (Y0 + y)) * Px + (X0 + x)] = acc[z];
}

template <typename T, int M>
static hipError_t spread_m(const SpreadArgs<T> &a, hipStream_t s) {
  const int64_t tiles = (int64_t)a.tiles[0] * a.tiles[1] * a.tiles[2];
  hipLaunchKernelGGL((k_spread<T, M>), dim3((unsigned)tiles), dim3(64), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spread(const SpreadArgs<T> &a, int m, hipStream_t s) {
  switch (m) {
    case 1: return spread_m<T, 1>(a, s);
    case 2: return spread_m<T, 2>(a, s);
    case 3: return spread_m<T, 3>(a, s);
    case 4: return spread_m<T, 4>(a, s);
    case 5: return spread_m<T, 5>(a, s);
    case 6: return spread_m<T, 6>(a, s);
    case 7: return spread_m<T, 7>(a, s);
    case 8: return spread_m<T, 8>(a, s);
    case 9: return spread_m<T, 9>(a, s);
    case 10: return spread_m<T, 10>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------------- interp ---
// One thread per target: the 2m x 2m x 2m stencil gather with separable
// Gaussian factors. Rows along x are summed in T, the row contributions are
// accumulated in FP64 (the per-node sum), result written in caller order.
template <typename T, int M>
__global__ __launch_bounds__(256) void k_interp(InterpArgs<T> a) {
  constexpr int W2 = 2 * M;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nt) return;
  const int64_t nt = a.nt;
  const int cx = a.cell[i], cy = a.cell[nt + i], cz = a.cell[2 * nt + i];
  const T fx = a.frac[i], fy = a.frac[nt + i], fz = a.frac[2 * nt + i];
  T wx[W2], wy[W2], wz[W2];
#pragma unroll
  for (int j = 0; j < W2; ++j) {
    const T k = (T)(j - M + 1);
    wx[j] = wexp(-(fx - k) * (fx - k) * a.inv_b);
    wy[j] = wexp(-(fy - k) * (fy - k) * a.inv_b);
    wz[j] = wexp(-(fz - k) * (fz - k) * a.inv_b);
  }
  const int64_t Rx = a.R[0], Ry = a.R[1];
  double acc = 0.0;
  for (int jz = 0; jz < W2; ++jz) {
    for (int jy = 0; jy < W2; ++jy) {
      const T *row = a.g + ((int64_t)(cz + jz - M + 1) * Ry + (cy + jy - M + 1)) * Rx + (cx - M + 1);
      T r = T(0);
#pragma unroll
      for (int jx = 0; jx < W2; ++jx) r += row[jx] * wx[jx];
      acc += (double)(r * (wy[jy] * wz[jz]));
    }
  }
  a.phi[a.perm[i]] = acc;
}

template <typename T, int M>
static hipError_t interp_m(const InterpArgs<T> &a, hipStream_t s) {
  if (a.nt == 0) return hipSuccess;
  const int64_t blocks = (a.nt + 255) / 256;
  hipLaunchKernelGGL((k_interp<T, M>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interp(const InterpArgs<T> &a, int m, hipStream_t s) {
  switch (m) {
    case 1: return interp_m<T, 1>(a, s);
    case 2: return interp_m<T, 2>(a, s);
    case 3: return interp_m<T, 3>(a, s);
    case 4: return interp_m<T, 4>(a, s);
    case 5: return interp_m<T, 5>(a, s);
    case 6: return interp_m<T, 6>(a, s);
    case 7: return interp_m<T, 7>(a, s);
    case 8: return interp_m<T, 8>(a, s);
    case 9: return interp_m<T, 9>(a, s);
    case 10: return interp_m<T, 10>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// -------------------------------------------------------------------- fft ---
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
// multiply by sign * i
template <typename C>
__device__ __forceinline__ C cmul_si(C a, int sign) {
  C r;
  r.x = sign > 0 ? -a.y : a.y;
  r.y = sign > 0 ? a.x : -a.x;
  return r;
}

// Stockham autosort FFT of B lines of length N held in LDS (radix 4, one
// radix-2 stage when log2 N is odd). Returns the buffer holding the result.
template <typename T, int N>
__device__ typename Cplx<T>::type *lds_fft(typename Cplx<T>::type *src,
                                           typename Cplx<T>::type *dst, int B, int sign,
                                           const typename Cplx<T>::type *__restrict__ tw) {
  using C = typename Cplx<T>::type;
  for (int Ns = 1; Ns < N; ) {
    if (N / Ns >= 4) {
      constexpr int Q = N / 4;
      for (int j = threadIdx.x; j < B * Q; j += blockDim.x) {
        const int b = j / Q, jj = j % Q;
        const int k = jj & (Ns - 1);
        const C *s = src + b * N;
        C v0 = s[jj], v1 = s[jj + Q], v2 = s[jj + 2 * Q], v3 = s[jj + 3 * Q];
        const int st = N / (4 * Ns);
        if (Ns > 1) {
          C w1 = tw[k * st], w2 = tw[2 * k * st], w3 = tw[3 * k * st];
          if (sign > 0) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
          v1 = cmul(v1, w1); v2 = cmul(v2, w2); v3 = cmul(v3, w3);
        }
        const C a0 = cadd(v0, v2), a1 = csub(v0, v2);
        const C b0 = cadd(v1, v3), b1 = cmul_si(csub(v1, v3), sign);
        C *d = dst + b * N + (jj - k) * 4 + k;
        d[0] = cadd(a0, b0);
        d[Ns] = cadd(a1, b1);
        d[2 * Ns] = csub(a0, b0);
        d[3 * Ns] = csub(a1, b1);
      }
      Ns *= 4;
    } else {
      constexpr int H = N / 2;
      for (int j = threadIdx.x; j < B * H; j += blockDim.x) {
        const int b = j / H, jj = j % H;
        const int k = jj & (Ns - 1);
        const C *s = src + b * N;
        C v0 = s[jj], v1 = s[jj + H];
        C w = tw[k * (N / (2 * Ns))];
        if (sign > 0) w.y = -w.y;
        v1 = cmul(v1, w);
        C *d = dst + b * N + (jj - k) * 2 + k;
        d[0] = cadd(v0, v1);
        d[Ns] = csub(v0, v1);
      }
      Ns *= 2;
    }
    __syncthreads();
    C *t = src; src = dst; dst = t;
  }
  return src;
}

__device__ __forceinline__ int wrap_pos(int e, int shift, int N) {
  int p = (e + shift) % N;
  return p < 0 ? p + N : p;
}

template <typename T, int N>
__global__ __launch_bounds__(256) void k_fft(FftPass<T> p, int B) {
  using C = typename Cplx<T>::type;
  extern __shared__ unsigned char smem_raw[];
  C *buf0 = reinterpret_cast<C *>(smem_raw);
  C *buf1 = buf0 + (size_t)B * N;
  const C *tw = reinterpret_cast<const C *>(p.tw);
  const int64_t L0 = (int64_t)blockIdx.x * B;
  const int nb = (int)min((int64_t)B, p.n_lines - L0);

  for (int j = threadIdx.x; j < B * N; j += blockDim.x) { buf0[j].x = T(0); buf0[j].y = T(0); }
  __syncthreads();

  // load (coalesced along e when the element stride is 1, along lines otherwise)
  const int total_in = nb * p.in_cnt;
  for (int idx = threadIdx.x; idx < total_in; idx += blockDim.x) {
    int b, e;
    if (p.in_es == 1) { e = idx % p.in_cnt; b = idx / p.in_cnt; }
    else { b = idx % nb; e = idx / nb; }
    const int64_t L = L0 + b;
    const int64_t off = (L % p.l1) * p.in_s1 + (L / p.l1) * p.in_s2 + (int64_t)e * p.in_es;
    C v;
    if (p.in_real) { v.x = reinterpret_cast<const T *>(p.in)[off]; v.y = T(0); }
    else { v = reinterpret_cast<const C *>(p.in)[off]; }
    const int pos = wrap_pos(e, p.in_shift, N);
    buf0[b * N + pos] = v;
    if (p.in_hermitian && e > 0) { C c = v; c.y = -c.y; buf0[b * N + (N - pos)] = c; }
  }
  __syncthreads();

  C *res = lds_fft<T, N>(buf0, buf1, B, p.sign, tw);

  if (p.mul_inv) {
    C *oth = (res == buf0) ? buf1 : buf0;
    for (int j = threadIdx.x; j < B * N; j += blockDim.x) { oth[j].x = T(0); oth[j].y = T(0); }
    __syncthreads();
    const int total_mu = nb * p.mu_cnt;
    for (int idx = threadIdx.x; idx < total_mu; idx += blockDim.x) {
      const int b = idx % nb, e = idx / nb;
      const int64_t L = L0 + b;
      const int64_t off = (L % p.l1) * p.in_s1 + (L / p.l1) * p.in_s2 + (int64_t)e * p.in_es;
      const T mu = p.mu[off];
      const int pos = wrap_pos(e, p.mu_shift, N);
      C v = res[b * N + pos];
      v.x *= mu; v.y *= mu;
      oth[b * N + pos] = v;
    }
    __syncthreads();
    C *spare = (oth == buf0) ? buf1 : buf0;
    res = lds_fft<T, N>(oth, spare, B, -p.sign, tw);
  }

  const int total_out = nb * p.out_cnt;
  for (int idx = threadIdx.x; idx < total_out; idx += blockDim.x) {
    int b, e;
    if (p.out_es == 1) { e = idx % p.out_cnt; b = idx / p.out_cnt; }
    else { b = idx % nb; e = idx / nb; }
    const int64_t L = L0 + b;
    const int64_t off = (L % p.l1) * p.out_s1 + (L / p.l1) * p.out_s2 + (int64_t)e * p.out_es;
    const C v = res[b * N + wrap_pos(e, p.out_shift, N)];
    if (p.out_real) reinterpret_cast<T *>(p.out)[off] = v.x;
    else reinterpret_cast<C *>(p.out)[off] = v;
  }
}

template <typename T, int N>
static hipError_t fft_n(const FftPass<T> &p, hipStream_t s) {
  using C = typename Cplx<T>::type;
  constexpr int kElems = (sizeof(T) == 8) ? 2048 : 4096;   // 64 KiB of LDS per workgroup
  constexpr int B = (kElems / N) > 0 ? (kElems / N) : 1;
  if (p.n_lines == 0) return hipSuccess;
  const int64_t blocks = (p.n_lines + B - 1) / B;
  const size_t shmem = 2 * (size_t)B * N * sizeof(C);
  hipLaunchKernelGGL((k_fft<T, N>), dim3((unsigned)blocks), dim3(256), shmem, s, p, B);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft(const FftPass<T> &p, int N, hipStream_t s) {
  switch (N) {
    case 8: return fft_n<T, 8>(p, s);
    case 16: return fft_n<T, 16>(p, s);
    case 32: return fft_n<T, 32>(p, s);
    case 64: return fft_n<T, 64>(p, s);
    case 128: return fft_n<T, 128>(p, s);
    case 256: return fft_n<T, 256>(p, s);
    case 512: return fft_n<T, 512>(p, s);
    case 1024: return fft_n<T, 1024>(p, s);
    case 2048: return fft_n<T, 2048>(p, s);
    default: return hipErrorInvalidValue;
  }
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

// mu over the stored half spectrum kx = 0..n_x/2, ky = -n_y/2..n_y/2,
// kz = -n_z/2..n_z/2 (layout [K_z][K_y][K_x]):
//   mu = h(l) c_l prod_q exp(2 b (pi l_q / N_q)^2) / (pi b) / (4 pi)
// c_l = sum_t omega_t prod_q c_{t,q}(|l_q|) (Sec. 3.3 separable coefficients),
// exp(2 b ...) / (pi b): the two deconvolutions by the window coefficients
// (eq. deconv and the type-2 counterpart) for the unnormalised window
// exp(-tau^2 / b); h(l) = ([l in I_n] + [-l in I_n]) / 2 is the real part of
// the sum over the asymmetric index set.
template <typename T>
__global__ void k_mu(T *mu, const double *__restrict__ C0, const double *__restrict__ C1,
                     const double *__restrict__ C2, const double *__restrict__ omega, int32_t S,
                     int3 n, int3 N, int3 K, double b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)K.x * K.y * K.z;
  if (i >= tot) return;
  const int kx = (int)(i % K.x);
  const int ky = (int)((i / K.x) % K.y) - n.y / 2;
  const int kz = (int)(i / ((int64_t)K.x * K.y)) - n.z / 2;
  const bool inI = (kx <= n.x / 2 - 1) && (ky >= -n.y / 2) && (ky <= n.y / 2 - 1) &&
                   (kz >= -n.z / 2) && (kz <= n.z / 2 - 1);
  const bool inmI = (kx >= -n.x / 2 + 1) && (ky >= -n.y / 2 + 1) && (ky <= n.y / 2) &&
                    (kz >= -n.z / 2 + 1) && (kz <= n.z / 2);
  const double h = 0.5 * ((inI ? 1.0 : 0.0) + (inmI ? 1.0 : 0.0));
  double v = 0.0;
  if (h > 0.0) {
    const int ax = kx, ay = ky < 0 ? -ky : ky, az = kz < 0 ? -kz : kz;
    const int Lx = n.x / 2 + 1, Ly = n.y / 2 + 1, Lz = n.z / 2 + 1;
    double c = 0.0;
    for (int t = 0; t < S; ++t)
      c += omega[t] * C0[(int64_t)t * Lx + ax] * C1[(int64_t)t * Ly + ay] * C2[(int64_t)t * Lz + az];
    const double pi = 3.141592653589793238462643383279502884;
    const double ex = (double)kx / N.x, ey = (double)ky / N.y, ez = (double)kz / N.z;
    const double dec = exp(2.0 * b * pi * pi * (ex * ex + ey * ey + ez * ez));
    v = h * c * dec / (pi * b * pi * b * pi * b) / (4.0 * pi);
  }
  mu[i] = (T)v;
}

template <typename T>
hipError_t launch_mu(T *mu, const double *C0, const double *C1, const double *C2,
                     const double *omega, int32_t S, const int32_t n[3], const int32_t N[3],
                     const int32_t K[3], double b, hipStream_t s) {
  const int64_t tot = (int64_t)K[0] * K[1] * K[2];
  hipLaunchKernelGGL(k_mu<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, mu, C0, C1, C2,
                     omega, S, make_int3(n[0], n[1], n[2]), make_int3(N[0], N[1], N[2]),
                     make_int3(K[0], K[1], K[2]), b);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_charges<float>(const double *, const double *, const int32_t *, float *,
                                          int64_t, hipStream_t);
template hipError_t launch_charges<double>(const double *, const double *, const int32_t *,
                                           double *, int64_t, hipStream_t);
template hipError_t launch_spread<float>(const SpreadArgs<float> &, int, hipStream_t);
template hipError_t launch_spread<double>(const SpreadArgs<double> &, int, hipStream_t);
template hipError_t launch_interp<float>(const InterpArgs<float> &, int, hipStream_t);
template hipError_t launch_interp<double>(const InterpArgs<double> &, int, hipStream_t);
template hipError_t launch_fft<float>(const FftPass<float> &, int, hipStream_t);
template hipError_t launch_fft<double>(const FftPass<double> &, int, hipStream_t);
template hipError_t launch_mu<float>(float *, const double *, const double *, const double *,
                                     const double *, int32_t, const int32_t *, const int32_t *,
                                     const int32_t *, double, hipStream_t);
template hipError_t launch_mu<double>(double *, const double *, const double *, const double *,
                                      const double *, int32_t, const int32_t *, const int32_t *,
                                      const int32_t *, double, hipStream_t);

}  // namespace slp
