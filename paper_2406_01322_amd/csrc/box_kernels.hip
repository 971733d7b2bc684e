// HIP kernels of the periodic-box Navier-Stokes + Cahn-Hilliard step (gfx950).
//
// The step of Sec. 2.2 (steps ii-v) is executed as four kernels per time step,
// all on the caller's stream:
//   k_lines  <inverse, y>  : y-inverse of u, v, w, phi, d_z phi, plus i k_y phi
//   k_xstep                : x-inverse (7 fields) -> pointwise products
//                            (Sec. 3.2.2, Hadamard products) -> x-forward (8)
//   k_lines  <forward, y>  : y-forward with 2/3 truncation
//   k_zstep                : z-forward, spectral RHS assembly, Leray projection,
//                            CN/AB2 (NS) and IE/AB2 (CH) updates, then the
//                            z-inverse of the new state for the next step.
// Spectral data is stored only inside the retained band |k_i| <= K =
// floor((N-1)/3), so the pruned transforms never touch discarded modes.
//
// Layouts (complex values interleaved re, im):
//   state, history : [4][C kz][C ky][H kx] double   (C = 2K+1, H = K+1)
//   G (z-inverse)  : [5][N z][C ky][H kx]           (u, v, w, phi, d_z phi)
//   Y (y-inverse)  : [6][N z][N y][H kx]            (u, v, w, phi, d_y phi, d_z phi)
//   X (x-forward)  : [8][N z][N y][H kx]            (T_xx T_yy T_zz T_xy T_xz T_yz, a, c)
//   W (y-forward)  : [8][N z][C ky][H kx]
#include <hip/hip_runtime.h>

#include "box_kernels.hpp"
#include "fft_core.hpp"

namespace psms {

template <typename T>
__device__ __forceinline__ cpx<T> to_cpx(cpx<double> v) { return {T(v.re), T(v.im)}; }
template <typename T>
__device__ __forceinline__ cpx<double> to_dbl(cpx<T> v) { return {double(v.re), double(v.im)}; }

// ---------------------------------------------------------------------------
// batched transforms along a strided axis (y or z)
//   element (line l = o * inner + i, position a) at ((o * cnt + a) * inner + i)
//   S = -1: forward, output band of n_out slots; S = +1: inverse, input band
//   of n_in slots zero-padded to n.  Output field f = blockIdx.y reads input
//   field (fmap >> 4f) & 15; bit f of dmask multiplies by i k along the axis.
// ---------------------------------------------------------------------------
template <typename T, int E, int S>
__global__ void __launch_bounds__(512) k_lines(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                                               const cpx<T>* __restrict__ tw_g, LineArgs a) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  const int n = a.pl.n;
  cpx<T>* buf = tw + n;
  const int tpl = a.pl.tpl;
  const int L = blockDim.x / tpl;
  const int lp = L + 1;
  const int tid = threadIdx.x;
  const int line = tid % L, lane = tid / L;
  for (int i = tid; i < n; i += blockDim.x) tw[i] = tw_g[i];

  const int fo = blockIdx.y;
  const cpx<T>* src = in + (long long)((a.fmap >> (4 * fo)) & 15) * a.in_fstride;
  cpx<T>* dst = out + (long long)fo * a.out_fstride;
  const bool deriv = (a.dmask >> fo) & 1;
  const long long l0 = (long long)blockIdx.x * L;

  for (int idx = tid; idx < n * L; idx += blockDim.x) {
    const int p = idx / L, l = idx % L;
    const long long gl = l0 + l;
    cpx<T> v = {T(0), T(0)};
    const int slot = band_slot(p, a.n_in, n);
    if (gl < a.nlines && slot >= 0) {
      const long long o = gl / a.inner, i = gl % a.inner;
      v = src[(o * a.n_in + slot) * a.inner + i];
      if (S > 0 && deriv) {
        const T k = T(signed_k(p, n));
        v = cpx<T>{-k * v.im, k * v.re};
      }
    }
    buf[p * lp + l] = v;
  }
  __syncthreads();
  fft_tile<E, S>(buf, lp, line, lane, true, a.pl, tw);
  const T sc = T(a.scale);
  for (int idx = tid; idx < a.n_out * L; idx += blockDim.x) {
    const int slot = idx / L, l = idx % L;
    const long long gl = l0 + l;
    if (gl >= a.nlines) continue;
    const int p = full_pos(slot, a.n_out, n);
    cpx<T> v = buf[p * lp + l];
    if (S < 0 && deriv) {
      const T k = T(signed_k(p, n));
      v = cpx<T>{-k * v.im, k * v.re};
    }
    v.re *= sc;
    v.im *= sc;
    const long long o = gl / a.inner, i = gl % a.inner;
    dst[(o * a.n_out + slot) * a.inner + i] = v;
  }
}

// ---------------------------------------------------------------------------
// real transforms along x (contiguous rows), two rows packed per complex FFT
// ---------------------------------------------------------------------------
template <typename T, int E>
__global__ void __launch_bounds__(512) k_rows_fwd(const T* __restrict__ in, cpx<T>* __restrict__ out,
                                                  const cpx<T>* __restrict__ tw_g, RowArgs a) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  const int n = a.pl.n;
  cpx<T>* buf = tw + n;
  const int tpl = a.pl.tpl;
  const int P = blockDim.x / tpl;
  const int lp = P + 1;
  const int tid = threadIdx.x;
  const int line = tid % P, lane = tid / P;
  for (int i = tid; i < n; i += blockDim.x) tw[i] = tw_g[i];
  const T* src = in + (long long)blockIdx.y * a.in_fstride;
  cpx<T>* dst = out + (long long)blockIdx.y * a.out_fstride;
  const long long r0 = (long long)blockIdx.x * 2 * P;
  for (int idx = tid; idx < n * P; idx += blockDim.x) {
    const int p = idx % n, pr = idx / n;
    const long long r = r0 + 2 * pr;
    cpx<T> v = {T(0), T(0)};
    if (r < a.nrows) {
      v.re = src[r * n + p];
      v.im = (r + 1 < a.nrows) ? src[(r + 1) * n + p] : T(0);
    }
    buf[p * lp + pr] = v;
  }
  __syncthreads();
  fft_tile<E, -1>(buf, lp, line, lane, true, a.pl, tw);
  const T h = T(0.5) * T(a.scale);
  for (int idx = tid; idx < a.n_out * P; idx += blockDim.x) {
    const int k = idx % a.n_out, pr = idx / a.n_out;
    const long long r = r0 + 2 * pr;
    if (r >= a.nrows) continue;
    const cpx<T> zk = buf[k * lp + pr];
    const cpx<T> zm = buf[((n - k) % n) * lp + pr];
    dst[r * a.n_out + k] = cpx<T>{h * (zk.re + zm.re), h * (zk.im - zm.im)};
    if (r + 1 < a.nrows) dst[(r + 1) * a.n_out + k] = cpx<T>{h * (zk.im + zm.im), h * (zm.re - zk.re)};
  }
}

template <typename T, int E>
__global__ void __launch_bounds__(512) k_rows_inv(const cpx<T>* __restrict__ in, T* __restrict__ out,
                                                  const cpx<T>* __restrict__ tw_g, RowArgs a) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  const int n = a.pl.n;
  cpx<T>* buf = tw + n;
  const int tpl = a.pl.tpl;
  const int P = blockDim.x / tpl;
  const int lp = P + 1;
  const int tid = threadIdx.x;
  const int line = tid % P, lane = tid / P;
  for (int i = tid; i < n; i += blockDim.x) tw[i] = tw_g[i];
  const cpx<T>* src = in + (long long)blockIdx.y * a.in_fstride;
  T* dst = out + (long long)blockIdx.y * a.out_fstride;
  const long long r0 = (long long)blockIdx.x * 2 * P;
  const int half = n / 2;
  for (int idx = tid; idx < n * P; idx += blockDim.x) {
    const int p = idx % n, pr = idx / n;
    const long long r = r0 + 2 * pr;
    const int k = (p <= half) ? p : n - p;  // source wavenumber
    cpx<T> A = {T(0), T(0)}, B = {T(0), T(0)};
    if (r < a.nrows && k < a.n_in) {
      A = src[r * a.n_in + k];
      if (r + 1 < a.nrows) B = src[(r + 1) * a.n_in + k];
      if (k == 0 || 2 * k == n) {  // real-valued entries of a real signal's spectrum
        A.im = T(0);
        B.im = T(0);
      }
    }
    cpx<T> z;
    if (p <= half) z = cpx<T>{A.re - B.im, A.im + B.re};   // A + i B
    else z = cpx<T>{A.re + B.im, B.re - A.im};              // conj(A) + i conj(B)
    buf[p * lp + pr] = z;
  }
  __syncthreads();
  fft_tile<E, +1>(buf, lp, line, lane, true, a.pl, tw);
  const T sc = T(a.scale);
  for (int idx = tid; idx < n * P; idx += blockDim.x) {
    const int p = idx % n, pr = idx / n;
    const long long r = r0 + 2 * pr;
    if (r >= a.nrows) continue;
    const cpx<T> z = buf[p * lp + pr];
    dst[r * n + p] = sc * z.re;
    if (r + 1 < a.nrows) dst[(r + 1) * n + p] = sc * z.im;
  }
}

// ---------------------------------------------------------------------------
// fused x stage of the step: x-inverse of 7 fields, products, x-forward of 8
// Block: 2P consecutive rows (row = z N + y); LDS holds [8 fields][n][P pairs].
// ---------------------------------------------------------------------------
template <typename T, int E>
__global__ void __launch_bounds__(512) k_xstep(const cpx<T>* __restrict__ yin, cpx<T>* __restrict__ xout,
                                               const cpx<T>* __restrict__ tw_g, FftPlan pl, BoxGeom g,
                                               double csig_d, int P) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  const int n = pl.n;
  cpx<T>* buf = tw + n;
  const int lp = P + 1;
  const int tid = threadIdx.x;
  const int nl = 8 * P;
  const int lid = tid % nl, lane = tid / nl;
  const int f = lid / P, pair = lid % P;
  const int H = g.H;
  const long long rows = (long long)n * n;
  const long long r0 = (long long)blockIdx.x * 2 * P;
  for (int i = tid; i < n; i += blockDim.x) tw[i] = tw_g[i];

  // 1) pack the 7 physical inputs: u v w phi dx_phi dy_phi dz_phi
  for (int idx = tid; idx < 7 * P * H; idx += blockDim.x) {
    const int k = idx % H;
    const int rest = idx / H;
    const int pr = rest % P, vf = rest / P;
    const int fin = (vf <= 3) ? vf : vf - 1;   // vf 4 reads phi and multiplies by i kx
    const long long r = r0 + 2 * pr;
    const cpx<T>* src = yin + (long long)fin * rows * H;
    cpx<T> A = src[r * H + k];
    cpx<T> B = src[(r + 1) * H + k];
    if (vf == 4) {
      const T kx = T(k);
      A = cpx<T>{-kx * A.im, kx * A.re};
      B = cpx<T>{-kx * B.im, kx * B.re};
    }
    if (k == 0) {
      A.im = T(0);
      B.im = T(0);
    }
    cpx<T>* b = buf + (long long)vf * n * lp;
    b[k * lp + pr] = cpx<T>{A.re - B.im, A.im + B.re};
    if (k > 0) b[(n - k) * lp + pr] = cpx<T>{A.re + B.im, B.re - A.im};
  }
  const int nz = n - 2 * H + 1;  // positions H .. n-H hold zeros
  for (int idx = tid; idx < 7 * P * nz; idx += blockDim.x) {
    const int p = H + idx % nz;
    const int rest = idx / nz;
    const int pr = rest % P, vf = rest / P;
    buf[((long long)vf * n + p) * lp + pr] = cpx<T>{T(0), T(0)};
  }
  __syncthreads();
  fft_tile<E, +1>(buf + (long long)f * n * lp, lp, pair, lane, f < 7, pl, tw);

  // 2) products at every point of the 2P rows (re: even row, im: odd row)
  const T cs = T(csig_d);
  for (int idx = tid; idx < n * P; idx += blockDim.x) {
    const int p = idx / P, pr = idx % P;
    cpx<T> q[7];
#pragma unroll
    for (int v = 0; v < 7; ++v) q[v] = buf[((long long)v * n + p) * lp + pr];
    cpx<T> o[8];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const T u = c ? q[0].im : q[0].re, vv = c ? q[1].im : q[1].re, w = c ? q[2].im : q[2].re;
      const T ph = c ? q[3].im : q[3].re;
      const T gx = c ? q[4].im : q[4].re, gy = c ? q[5].im : q[5].re, gz = c ? q[6].im : q[6].re;
      const T g2 = gx * gx + gy * gy + gz * gz;
      T r[8];
      r[0] = -u * u + cs * (g2 - gx * gx);
      r[1] = -vv * vv + cs * (g2 - gy * gy);
      r[2] = -w * w + cs * (g2 - gz * gz);
      r[3] = -u * vv - cs * gx * gy;
      r[4] = -u * w - cs * gx * gz;
      r[5] = -vv * w - cs * gy * gz;
      r[6] = u * gx + vv * gy + w * gz;
      r[7] = ph * ph * ph;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        if (c) o[v].im = r[v];
        else o[v].re = r[v];
      }
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) buf[((long long)v * n + p) * lp + pr] = o[v];
  }
  __syncthreads();
  fft_tile<E, -1>(buf + (long long)f * n * lp, lp, pair, lane, true, pl, tw);

  // 3) unpack the retained kx = 0..K of both rows and store
  const T h = T(0.5);
  for (int idx = tid; idx < 8 * P * H; idx += blockDim.x) {
    const int k = idx % H;
    const int rest = idx / H;
    const int pr = rest % P, vf = rest / P;
    const long long r = r0 + 2 * pr;
    const cpx<T>* b = buf + (long long)vf * n * lp;
    const cpx<T> zk = b[k * lp + pr];
    const cpx<T> zm = b[((n - k) % n) * lp + pr];
    cpx<T>* dst = xout + (long long)vf * rows * H;
    dst[r * H + k] = cpx<T>{h * (zk.re + zm.re), h * (zk.im - zm.im)};
    dst[(r + 1) * H + k] = cpx<T>{h * (zk.im + zm.im), h * (zm.re - zk.re)};
  }
}

// ---------------------------------------------------------------------------
// fused z stage: z-forward of the 8 products, RHS, projection, update, and the
// z-inverse of the new state.  One line per (ky, kx) retained pair q.
// do_update = 0 only loads the state and performs the z-inverse (prologue).
// ---------------------------------------------------------------------------
template <typename T, int E>
__global__ void __launch_bounds__(512) k_zstep(const cpx<T>* __restrict__ rhs, cpx<double>* __restrict__ state,
                                               cpx<double>* __restrict__ hist, cpx<T>* __restrict__ gout,
                                               const cpx<T>* __restrict__ tw_g, FftPlan pl, BoxGeom g,
                                               StepCoef sc, int do_update) {
  constexpr int J = (2 * E + 2) / 3;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  const int n = pl.n;
  cpx<T>* buf = tw + n;
  const int tpl = pl.tpl;
  const int L = blockDim.x / tpl;
  const int lp = L + 1;
  const int tid = threadIdx.x;
  const int line = tid % L, lane = tid / L;
  for (int i = tid; i < n; i += blockDim.x) tw[i] = tw_g[i];

  const int K = g.K, C = g.C, H = g.H;
  const long long Q = g.Q, M = g.M;
  const long long q0 = (long long)blockIdx.x * L;
  const long long q = q0 + line;
  const bool valid = q < Q;
  const int iy = valid ? int(q / H) : 0, ix = valid ? int(q % H) : 0;
  const double kx = double(ix);
  const double ky = double(iy <= K ? iy : iy - C);

  cpx<double> acc[4][J];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int j = 0; j < J; ++j) acc[c][j] = cpx<double>{0.0, 0.0};

  if (do_update) {
    for (int f = 0; f < 8; ++f) {
      const cpx<T>* src = rhs + (long long)f * n * Q;
      for (int idx = tid; idx < n * L; idx += blockDim.x) {
        const int p = idx / L, l = idx % L;
        const long long qq = q0 + l;
        buf[p * lp + l] = (qq < Q) ? src[(long long)p * Q + qq] : cpx<T>{T(0), T(0)};
      }
      __syncthreads();
      fft_tile<E, -1>(buf, lp, line, lane, true, pl, tw);
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int m = lane + tpl * j;
        if (m < C && valid) {
          const cpx<T> t = buf[full_pos(m, C, n) * lp + line];
          const cpx<double> v = {double(t.re) * sc.inv_n3, double(t.im) * sc.inv_n3};
          const double kz = double(m <= K ? m : m - C);
          // i k v
          const cpx<double> ikx = {-kx * v.im, kx * v.re};
          const cpx<double> iky = {-ky * v.im, ky * v.re};
          const cpx<double> ikz = {-kz * v.im, kz * v.re};
          if (f == 0) acc[0][j] = cadd(acc[0][j], ikx);                 // d_x T_xx
          else if (f == 1) acc[1][j] = cadd(acc[1][j], iky);            // d_y T_yy
          else if (f == 2) acc[2][j] = cadd(acc[2][j], ikz);            // d_z T_zz
          else if (f == 3) {                                             // T_xy
            acc[0][j] = cadd(acc[0][j], iky);
            acc[1][j] = cadd(acc[1][j], ikx);
          } else if (f == 4) {                                           // T_xz
            acc[0][j] = cadd(acc[0][j], ikz);
            acc[2][j] = cadd(acc[2][j], ikx);
          } else if (f == 5) {                                           // T_yz
            acc[1][j] = cadd(acc[1][j], ikz);
            acc[2][j] = cadd(acc[2][j], iky);
          } else if (f == 6) {                                           // -u.grad(phi)
            acc[3][j] = csub(acc[3][j], v);
          } else {                                                       // lap(phi^3) / Pe
            const double k2 = kx * kx + ky * ky + kz * kz;
            acc[3][j].re -= k2 * sc.inv_pe * v.re;
            acc[3][j].im -= k2 * sc.inv_pe * v.im;
          }
        }
      }
      __syncthreads();
    }
    // spectral update of the owned modes
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int m = lane + tpl * j;
      if (m < C && valid) {
        const double kz = double(m <= K ? m : m - C);
        const double k2 = kx * kx + ky * ky + kz * kz;
        const long long id = (long long)m * Q + q;
        cpx<double> Sx = acc[0][j], Sy = acc[1][j], Sz = acc[2][j], Sp = acc[3][j];
        const cpx<double> ph = state[3 * M + id];
        Sp.re += sc.e_coef * k2 * ph.re;
        Sp.im += sc.e_coef * k2 * ph.im;
        if (k2 == 0.0) {
          Sx = Sy = Sz = Sp = cpx<double>{0.0, 0.0};
        } else {  // Leray projection, FP64
          const double ir = 1.0 / k2;
          const cpx<double> kd = {kx * Sx.re + ky * Sy.re + kz * Sz.re, kx * Sx.im + ky * Sy.im + kz * Sz.im};
          Sx.re -= kx * kd.re * ir; Sx.im -= kx * kd.im * ir;
          Sy.re -= ky * kd.re * ir; Sy.im -= ky * kd.im * ir;
          Sz.re -= kz * kd.re * ir; Sz.im -= kz * kd.im * ir;
        }
        cpx<double> ex[4] = {Sx, Sy, Sz, Sp};
        if (!sc.ab1) {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const cpx<double> hp = hist[c * M + id];
            ex[c].re = 1.5 * ex[c].re - 0.5 * hp.re;
            ex[c].im = 1.5 * ex[c].im - 0.5 * hp.im;
          }
        }
        hist[0 * M + id] = Sx;
        hist[1 * M + id] = Sy;
        hist[2 * M + id] = Sz;
        hist[3 * M + id] = Sp;
        const double a = 0.5 * sc.dt * sc.nu * k2;
        const double ia = 1.0 / (1.0 + a);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const cpx<double> u = state[c * M + id];
          const cpx<double> un = {((1.0 - a) * u.re + sc.dt * ex[c].re) * ia, ((1.0 - a) * u.im + sc.dt * ex[c].im) * ia};
          state[c * M + id] = un;
          acc[c][j] = un;
        }
        const double den = 1.0 / (1.0 + sc.dt * sc.ch2_pe * (k2 * k2 + sc.s * k2));
        const cpx<double> pn = {(ph.re + sc.dt * ex[3].re) * den, (ph.im + sc.dt * ex[3].im) * den};
        state[3 * M + id] = pn;
        acc[3][j] = pn;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int m = lane + tpl * j;
      if (m < C && valid) {
        const long long id = (long long)m * Q + q;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c][j] = state[c * M + id];
      }
    }
  }

  // z-inverse of u, v, w, phi and i kz phi
  const int nz = n - C;
  for (int gf = 0; gf < 5; ++gf) {
    for (int idx = tid; idx < nz * L; idx += blockDim.x) {
      const int p = K + 1 + idx / L, l = idx % L;
      buf[p * lp + l] = cpx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int m = lane + tpl * j;
      if (m < C) {
        cpx<double> v = {0.0, 0.0};
        if (valid) {
          if (gf == 0) v = acc[0][j];
          else if (gf == 1) v = acc[1][j];
          else if (gf == 2) v = acc[2][j];
          else if (gf == 3) v = acc[3][j];
          else {
            const double kz = double(m <= K ? m : m - C);
            v = cpx<double>{-kz * acc[3][j].im, kz * acc[3][j].re};
          }
        }
        buf[full_pos(m, C, n) * lp + line] = to_cpx<T>(v);
      }
    }
    __syncthreads();
    fft_tile<E, +1>(buf, lp, line, lane, true, pl, tw);
    cpx<T>* dst = gout + (long long)gf * n * Q;
    for (int idx = tid; idx < n * L; idx += blockDim.x) {
      const int p = idx / L, l = idx % L;
      const long long qq = q0 + l;
      if (qq < Q) dst[(long long)p * Q + qq] = buf[p * lp + l];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// small per-mode kernels
// ---------------------------------------------------------------------------

// compact band [nf][C][C][H] <-> full half spectrum [nf][n][n][n/2+1]
template <typename T>
__global__ void k_expand(const cpx<T>* __restrict__ cmp, cpx<T>* __restrict__ full, BoxGeom g, int nf) {
  const int n = g.n, nh = n / 2 + 1;
  const long long per = (long long)n * n * nh;
  const long long tot = per * nf;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < tot;
       id += (long long)gridDim.x * blockDim.x) {
    const long long f = id / per, r = id % per;
    const int kxp = int(r % nh);
    const int kyp = int((r / nh) % n);
    const int kzp = int(r / ((long long)nh * n));
    const int sy = band_slot(kyp, g.C, n), sz = band_slot(kzp, g.C, n);
    cpx<T> v = {T(0), T(0)};
    if (kxp < g.H && sy >= 0 && sz >= 0) v = cmp[f * g.M + ((long long)sz * g.C + sy) * g.H + kxp];
    full[id] = v;
  }
}

template <typename T>
__global__ void k_compact(const cpx<T>* __restrict__ full, cpx<T>* __restrict__ cmp, BoxGeom g, int nf) {
  const int n = g.n, nh = n / 2 + 1;
  const long long tot = g.M * nf;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < tot;
       id += (long long)gridDim.x * blockDim.x) {
    const long long f = id / g.M, r = id % g.M;
    const int ix = int(r % g.H);
    const int iy = int((r / g.H) % g.C);
    const int iz = int(r / ((long long)g.H * g.C));
    const int py = full_pos(iy, g.C, n), pz = full_pos(iz, g.C, n);
    cmp[id] = full[f * (long long)n * n * nh + ((long long)pz * n + py) * nh + ix];
  }
}

// Leray projection of the compact velocity [3][M] in place (k = 0 -> 0).
__global__ void k_project(cpx<double>* __restrict__ u, BoxGeom g) {
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < g.M;
       id += (long long)gridDim.x * blockDim.x) {
    const int ix = int(id % g.H);
    const int iy = int((id / g.H) % g.C);
    const int iz = int(id / ((long long)g.H * g.C));
    const double kx = ix, ky = (iy <= g.K) ? iy : iy - g.C, kz = (iz <= g.K) ? iz : iz - g.C;
    const double k2 = kx * kx + ky * ky + kz * kz;
    cpx<double> a = u[id], b = u[g.M + id], c = u[2 * g.M + id];
    if (k2 == 0.0) {
      a = b = c = cpx<double>{0.0, 0.0};
    } else {
      const double ir = 1.0 / k2;
      const double dre = kx * a.re + ky * b.re + kz * c.re, dim = kx * a.im + ky * b.im + kz * c.im;
      a.re -= kx * dre * ir; a.im -= kx * dim * ir;
      b.re -= ky * dre * ir; b.im -= ky * dim * ir;
      c.re -= kz * dre * ir; c.im -= kz * dim * ir;
    }
    u[id] = a;
    u[g.M + id] = b;
    u[2 * g.M + id] = c;
  }
}

// Full half spectrum: optional 2/3 mask and i k_axis factor, scale.
template <typename T>
__global__ void k_spec_finish(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, BoxGeom g, int nf,
                              int dealias, int axis, double scale) {
  const int n = g.n, nh = n / 2 + 1;
  const long long per = (long long)n * n * nh;
  const long long tot = per * nf;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < tot;
       id += (long long)gridDim.x * blockDim.x) {
    const long long r = id % per;
    const int kxp = int(r % nh);
    const int kyp = int((r / nh) % n);
    const int kzp = int(r / ((long long)nh * n));
    cpx<T> v = in[id];
    if (dealias && (kxp > g.K || band_slot(kyp, g.C, n) < 0 || band_slot(kzp, g.C, n) < 0)) v = cpx<T>{T(0), T(0)};
    if (axis >= 0) {
      const int k = (axis == 0) ? kxp : signed_k(axis == 1 ? kyp : kzp, n);
      v = cpx<T>{-T(k) * v.im, T(k) * v.re};
    }
    out[id] = cpx<T>{T(scale) * v.re, T(scale) * v.im};
  }
}

// Helmholtz (lap - lambda_f) f = g per mode: f = -g / (k^2 + lambda_f).
__global__ void k_helmholtz_box(const cpx<double>* __restrict__ rhs, cpx<double>* __restrict__ out, BoxGeom g,
                                int nf, double lam) {
  const int n = g.n, nh = n / 2 + 1;
  const long long per = (long long)n * n * nh;
  const long long tot = per * nf;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < tot;
       id += (long long)gridDim.x * blockDim.x) {
    const long long r = id % per;
    const int kxp = int(r % nh);
    const int ky = signed_k(int((r / nh) % n), n);
    const int kz = signed_k(int(r / ((long long)nh * n)), n);
    const double den = double(kxp) * kxp + double(ky) * ky + double(kz) * kz + lam;
    const cpx<double> v = rhs[id];
    out[id] = (den != 0.0) ? cpx<double>{-v.re / den, -v.im / den} : cpx<double>{0.0, 0.0};
  }
}

// Index maps of the compact band as used by every kernel: for slot (f=0) id,
// writes kz, ky, kx and the offset into the full half spectrum.
__global__ void k_index_maps(int* __restrict__ out, BoxGeom g) {
  const int n = g.n, nh = n / 2 + 1;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < g.M;
       id += (long long)gridDim.x * blockDim.x) {
    const int ix = int(id % g.H);
    const int iy = int((id / g.H) % g.C);
    const int iz = int(id / ((long long)g.H * g.C));
    const int py = full_pos(iy, g.C, n), pz = full_pos(iz, g.C, n);
    out[4 * id + 0] = signed_k(pz, n);
    out[4 * id + 1] = signed_k(py, n);
    out[4 * id + 2] = ix;
    out[4 * id + 3] = int(((long long)pz * n + py) * nh + ix);
  }
}

// Diagnostics over the compact state, two-pass deterministic reduction.
// part[b] = {ke, grad2, max_div, nonfinite}
__global__ void k_diag_partial(const cpx<double>* __restrict__ st, BoxGeom g, double* __restrict__ part) {
  __shared__ double sh[4][256];
  double ke = 0.0, gr = 0.0, md = 0.0, nf = 0.0;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < g.M;
       id += (long long)gridDim.x * blockDim.x) {
    const int ix = int(id % g.H);
    const int iy = int((id / g.H) % g.C);
    const int iz = int(id / ((long long)g.H * g.C));
    const double kx = ix, ky = (iy <= g.K) ? iy : iy - g.C, kz = (iz <= g.K) ? iz : iz - g.C;
    const double w = (ix == 0) ? 1.0 : 2.0;
    const cpx<double> a = st[id], b = st[g.M + id], c = st[2 * g.M + id], p = st[3 * g.M + id];
    const double e = a.re * a.re + a.im * a.im + b.re * b.re + b.im * b.im + c.re * c.re + c.im * c.im;
    ke += 0.5 * w * e;
    gr += w * (kx * kx + ky * ky + kz * kz) * (p.re * p.re + p.im * p.im);
    const double dre = kx * a.re + ky * b.re + kz * c.re, dim = kx * a.im + ky * b.im + kz * c.im;
    const double d = sqrt(dre * dre + dim * dim);
    md = fmax(md, d);
    const double s = e + p.re * p.re + p.im * p.im;
    if (!isfinite(s)) nf += 1.0;
  }
  const int t = threadIdx.x;
  sh[0][t] = ke; sh[1][t] = gr; sh[2][t] = md; sh[3][t] = nf;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) {
      sh[0][t] += sh[0][t + s];
      sh[1][t] += sh[1][t + s];
      sh[2][t] = fmax(sh[2][t], sh[2][t + s]);
      sh[3][t] += sh[3][t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[4 * blockIdx.x + 0] = sh[0][0];
    part[4 * blockIdx.x + 1] = sh[1][0];
    part[4 * blockIdx.x + 2] = sh[2][0];
    part[4 * blockIdx.x + 3] = sh[3][0];
  }
}

__global__ void k_diag_final(const double* __restrict__ part, int nb, const cpx<double>* __restrict__ st, BoxGeom g,
                             double* __restrict__ out) {
  __shared__ double sh[4][256];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int i = t; i < nb; i += blockDim.x) {
    a += part[4 * i];
    b += part[4 * i + 1];
    c = fmax(c, part[4 * i + 2]);
    d += part[4 * i + 3];
  }
  sh[0][t] = a; sh[1][t] = b; sh[2][t] = c; sh[3][t] = d;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) {
      sh[0][t] += sh[0][t + s];
      sh[1][t] += sh[1][t + s];
      sh[2][t] = fmax(sh[2][t], sh[2][t + s]);
      sh[3][t] += sh[3][t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = st[3 * g.M].re;  // mean phi = phi_hat(0)
    out[1] = sh[0][0];
    out[2] = sh[1][0];
    out[3] = sh[2][0];
    out[4] = sh[3][0];
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
namespace {
template <typename K>
void set_lds(K kern, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}
}  // namespace

template <typename T>
hipError_t launch_lines(int E, int dir, const cpx<T>* in, cpx<T>* out, const cpx<T>* tw, const LineArgs& a,
                        int nfield, hipStream_t st) {
  const int L = line_tile(a.pl.tpl);
  const dim3 grid(unsigned((a.nlines + L - 1) / L), unsigned(nfield));
  const dim3 block(unsigned(L * a.pl.tpl));
  const size_t lds = sizeof(cpx<T>) * (size_t(a.pl.n) + size_t(a.pl.n) * (L + 1));
  if (E == 8) {
    if (dir < 0) { set_lds(k_lines<T, 8, -1>, lds); k_lines<T, 8, -1><<<grid, block, lds, st>>>(in, out, tw, a); }
    else { set_lds(k_lines<T, 8, 1>, lds); k_lines<T, 8, 1><<<grid, block, lds, st>>>(in, out, tw, a); }
  } else {
    if (dir < 0) { set_lds(k_lines<T, 12, -1>, lds); k_lines<T, 12, -1><<<grid, block, lds, st>>>(in, out, tw, a); }
    else { set_lds(k_lines<T, 12, 1>, lds); k_lines<T, 12, 1><<<grid, block, lds, st>>>(in, out, tw, a); }
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rows(int E, int dir, const void* in, void* out, const cpx<T>* tw, const RowArgs& a, int nfield,
                       hipStream_t st) {
  const int P = row_pairs(a.pl.tpl);
  const dim3 grid(unsigned((a.nrows + 2 * P - 1) / (2 * P)), unsigned(nfield));
  const dim3 block(unsigned(P * a.pl.tpl));
  const size_t lds = sizeof(cpx<T>) * (size_t(a.pl.n) + size_t(a.pl.n) * (P + 1));
  if (dir < 0) {
    const T* src = static_cast<const T*>(in);
    cpx<T>* dst = static_cast<cpx<T>*>(out);
    if (E == 8) { set_lds(k_rows_fwd<T, 8>, lds); k_rows_fwd<T, 8><<<grid, block, lds, st>>>(src, dst, tw, a); }
    else { set_lds(k_rows_fwd<T, 12>, lds); k_rows_fwd<T, 12><<<grid, block, lds, st>>>(src, dst, tw, a); }
  } else {
    const cpx<T>* src = static_cast<const cpx<T>*>(in);
    T* dst = static_cast<T*>(out);
    if (E == 8) { set_lds(k_rows_inv<T, 8>, lds); k_rows_inv<T, 8><<<grid, block, lds, st>>>(src, dst, tw, a); }
    else { set_lds(k_rows_inv<T, 12>, lds); k_rows_inv<T, 12><<<grid, block, lds, st>>>(src, dst, tw, a); }
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xstep(int E, const cpx<T>* yin, cpx<T>* xout, const cpx<T>* tw, const FftPlan& pl,
                        const BoxGeom& g, double csig, int P, hipStream_t st) {
  const long long rows = (long long)pl.n * pl.n;
  const dim3 grid(unsigned(rows / (2 * P)));
  const dim3 block(unsigned(8 * P * pl.tpl));
  const size_t lds = sizeof(cpx<T>) * (size_t(pl.n) + 8 * size_t(pl.n) * (P + 1));
  if (E == 8) { set_lds(k_xstep<T, 8>, lds); k_xstep<T, 8><<<grid, block, lds, st>>>(yin, xout, tw, pl, g, csig, P); }
  else { set_lds(k_xstep<T, 12>, lds); k_xstep<T, 12><<<grid, block, lds, st>>>(yin, xout, tw, pl, g, csig, P); }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zstep(int E, const cpx<T>* rhs, cpx<double>* state, cpx<double>* hist, cpx<T>* gout,
                        const cpx<T>* tw, const FftPlan& pl, const BoxGeom& g, const StepCoef& sc, int do_update,
                        hipStream_t st) {
  const int L = line_tile(pl.tpl);
  const dim3 grid(unsigned((g.Q + L - 1) / L));
  const dim3 block(unsigned(L * pl.tpl));
  const size_t lds = sizeof(cpx<T>) * (size_t(pl.n) + size_t(pl.n) * (L + 1));
  if (E == 8) {
    set_lds(k_zstep<T, 8>, lds);
    k_zstep<T, 8><<<grid, block, lds, st>>>(rhs, state, hist, gout, tw, pl, g, sc, do_update);
  } else {
    set_lds(k_zstep<T, 12>, lds);
    k_zstep<T, 12><<<grid, block, lds, st>>>(rhs, state, hist, gout, tw, pl, g, sc, do_update);
  }
  return hipGetLastError();
}

static unsigned grid_for(long long tot) {
  long long b = (tot + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return unsigned(b);
}

template <typename T>
hipError_t launch_expand(const cpx<T>* cmp, cpx<T>* full, const BoxGeom& g, int nf, hipStream_t st) {
  const long long tot = (long long)g.n * g.n * (g.n / 2 + 1) * nf;
  k_expand<T><<<grid_for(tot), 256, 0, st>>>(cmp, full, g, nf);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_compact(const cpx<T>* full, cpx<T>* cmp, const BoxGeom& g, int nf, hipStream_t st) {
  k_compact<T><<<grid_for(g.M * nf), 256, 0, st>>>(full, cmp, g, nf);
  return hipGetLastError();
}
hipError_t launch_project(cpx<double>* u, const BoxGeom& g, hipStream_t st) {
  k_project<<<grid_for(g.M), 256, 0, st>>>(u, g);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_spec_finish(const cpx<T>* in, cpx<T>* out, const BoxGeom& g, int nf, int dealias, int axis,
                              double scale, hipStream_t st) {
  const long long tot = (long long)g.n * g.n * (g.n / 2 + 1) * nf;
  k_spec_finish<T><<<grid_for(tot), 256, 0, st>>>(in, out, g, nf, dealias, axis, scale);
  return hipGetLastError();
}
hipError_t launch_helmholtz_box(const cpx<double>* rhs, cpx<double>* out, const BoxGeom& g, double lam,
                                hipStream_t st) {
  const long long tot = (long long)g.n * g.n * (g.n / 2 + 1);
  k_helmholtz_box<<<grid_for(tot), 256, 0, st>>>(rhs, out, g, 1, lam);
  return hipGetLastError();
}
hipError_t launch_index_maps(int* out, const BoxGeom& g, hipStream_t st) {
  k_index_maps<<<grid_for(g.M), 256, 0, st>>>(out, g);
  return hipGetLastError();
}
hipError_t launch_diag(const cpx<double>* state, const BoxGeom& g, double* part, int max_blocks, double* out,
                       hipStream_t st) {
  long long nb = (g.M + 255) / 256;
  if (nb > max_blocks) nb = max_blocks;
  k_diag_partial<<<unsigned(nb), 256, 0, st>>>(state, g, part);
  k_diag_final<<<1, 256, 0, st>>>(part, int(nb), state, g, out);
  return hipGetLastError();
}

template hipError_t launch_lines<double>(int, int, const cpx<double>*, cpx<double>*, const cpx<double>*,
                                         const LineArgs&, int, hipStream_t);
template hipError_t launch_lines<float>(int, int, const cpx<float>*, cpx<float>*, const cpx<float>*,
                                        const LineArgs&, int, hipStream_t);
template hipError_t launch_rows<double>(int, int, const void*, void*, const cpx<double>*, const RowArgs&, int,
                                        hipStream_t);
template hipError_t launch_rows<float>(int, int, const void*, void*, const cpx<float>*, const RowArgs&, int,
                                       hipStream_t);
template hipError_t launch_xstep<double>(int, const cpx<double>*, cpx<double>*, const cpx<double>*, const FftPlan&,
                                         const BoxGeom&, double, int, hipStream_t);
template hipError_t launch_xstep<float>(int, const cpx<float>*, cpx<float>*, const cpx<float>*, const FftPlan&,
                                        const BoxGeom&, double, int, hipStream_t);
template hipError_t launch_zstep<double>(int, const cpx<double>*, cpx<double>*, cpx<double>*, cpx<double>*,
                                         const cpx<double>*, const FftPlan&, const BoxGeom&, const StepCoef&, int,
                                         hipStream_t);
template hipError_t launch_zstep<float>(int, const cpx<float>*, cpx<double>*, cpx<double>*, cpx<float>*,
                                        const cpx<float>*, const FftPlan&, const BoxGeom&, const StepCoef&, int,
                                        hipStream_t);
template hipError_t launch_expand<double>(const cpx<double>*, cpx<double>*, const BoxGeom&, int, hipStream_t);
template hipError_t launch_compact<double>(const cpx<double>*, cpx<double>*, const BoxGeom&, int, hipStream_t);
template hipError_t launch_spec_finish<double>(const cpx<double>*, cpx<double>*, const BoxGeom&, int, int, int,
                                               double, hipStream_t);
template hipError_t launch_spec_finish<float>(const cpx<float>*, cpx<float>*, const BoxGeom&, int, int, int, double,
                                              hipStream_t);

}  // namespace psms
