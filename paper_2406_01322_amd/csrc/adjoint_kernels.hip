// Discrete adjoint of the periodic-box step (FP64).
//
// The step maps (x^n, h^n) to x^{n+1} = A x^n + B (alpha S^n + beta h^n),
// h^{n+1} = S^n with S^n = R(x^n; We) the projected nonlinear terms.  Its
// transpose, given lam = dJ/dx^{n+1} and mu = dJ/dh^{n+1}, is
//   Sbar = alpha B lam + mu,  mu^n = beta B lam,
//   lam^n = A lam + (dR/dx)^T Sbar,  dJ/dWe += (dR/dWe)^T Sbar,
// under the half-spectrum inner product sum_k w_k Re(conj(a_k) b_k)
// (w = 1 at kx = 0, 2 otherwise), for which per-mode real factors are
// self-adjoint, (i k)^T = -i k, and the transforms are transposes of each
// other up to n^3.  R in the divergence form of the forward kernels:
//   S_i = P sum_j i k_j F(T_ij), T_ij = -u_i u_j + c (|g|^2 d_ij - g_i g_j),
//   S_phi = -F(u.g) - (k^2/Pe) F(phi^3) + E k^2 phi_hat, g = grad phi.
// Kernels (one adjoint step = z_in, y-inverse, x, y-forward, z_out):
//   k_zadj_in   per mode: Sbar, mu^n, A lam + E k^2 Sbar_phi, and the spectral
//               cotangents of the 8 transformed products, z-inverted;
//   k_xadj      per row pair: the physical forward fields (x-inverse of the
//               forward step's y-inverse output), the transposed products and
//               the We term, x-forward of the 7 field cotangents;
//   k_zadj_out  per line: z-forward of the 7 cotangents, added into lam^n.
#include <hip/hip_runtime.h>

#include "adjoint_kernels.hpp"
#include "fft_engine.hpp"

namespace psms {

// -------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(256) k_zadj_in(cpx<double>* __restrict__ lam, cpx<double>* __restrict__ mu,
                                                 cpx<double>* __restrict__ gout, const cpx<double>* __restrict__ tw_g,
                                                 AdjCoef ac) {
  using P = Plan<N>;
  using G = Tile<P>;
  constexpr int E = G::E, L = G::L, LP = L + 1, K = G::K, C = G::C, H = G::H;
  constexpr int Q = C * H;
  constexpr long long M = (long long)C * Q;
  constexpr int RI = first_radix<P, 1>(), RO = last_radix<P, 1>();
  __shared__ cpx<double> tw[N];
  __shared__ cpx<double> lds[2][N * LP];
  const int tid = threadIdx.x;
  const int line = tid % L, t = tid / L;
  for (int i = tid; i < N; i += blockDim.x) tw[i] = tw_g[i];
  const int q = blockIdx.x * L + line;
  const bool valid = q < Q;
  const int iy = valid ? q / H : 0, ix = valid ? q % H : 0;
  const double kx = double(ix), ky = double(iy <= K ? iy : iy - C);
  const IdxPosMajor idx{LP, line};
  int par = 0;

  cpx<double> sb[4][E];  // projected Sbar_u (3) and Sbar_phi at the owned modes
  double kz[E];
  bool inb[E];
#pragma unroll
  for (int b = 0; b < E / RI; ++b)
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int e = b * RI + r;
      const int p = slot_pos<P, RI>(t, b, r);
      const int s = band_slot(p, C, N);
      inb[e] = valid && s >= 0;
      kz[e] = double(signed_k(p, N));
#pragma unroll
      for (int c = 0; c < 4; ++c) sb[c][e] = cpx<double>{0.0, 0.0};
      if (inb[e]) {
        const long long id = (long long)s * Q + q;
        const double k2 = kx * kx + ky * ky + kz[e] * kz[e];
        const double a = 0.5 * ac.dt * ac.nu * k2;
        const double Au = (1.0 - a) / (1.0 + a), Bu = ac.dt / (1.0 + a);
        const double Bp = ac.dt / (1.0 + ac.dt * ac.ch2_pe * (k2 * k2 + ac.s * k2));
        const double Ap = Bp / ac.dt;
        cpx<double> S[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double A = (c < 3) ? Au : Ap, B = (c < 3) ? Bu : Bp;
          const cpx<double> l = lam[c * M + id], m = mu[c * M + id];
          S[c] = cpx<double>{ac.alpha * B * l.re + m.re, ac.alpha * B * l.im + m.im};
          mu[c * M + id] = cpx<double>{ac.beta * B * l.re, ac.beta * B * l.im};
          lam[c * M + id] = cpx<double>{A * l.re, A * l.im};
        }
        if (k2 == 0.0) {
          S[0] = S[1] = S[2] = S[3] = cpx<double>{0.0, 0.0};
        } else {
          const double ir = 1.0 / k2, kze = kz[e];
          const cpx<double> kd = {kx * S[0].re + ky * S[1].re + kze * S[2].re,
                                  kx * S[0].im + ky * S[1].im + kze * S[2].im};
          S[0].re -= kx * kd.re * ir; S[0].im -= kx * kd.im * ir;
          S[1].re -= ky * kd.re * ir; S[1].im -= ky * kd.im * ir;
          S[2].re -= kze * kd.re * ir; S[2].im -= kze * kd.im * ir;
          // direct dependence of S_phi on phi_hat
          const cpx<double> lp = lam[3 * M + id];
          lam[3 * M + id] = cpx<double>{lp.re + ac.e_coef * k2 * S[3].re, lp.im + ac.e_coef * k2 * S[3].im};
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) sb[c][e] = S[c];
      }
    }
  __syncthreads();

  // cotangents of F(T_xx), F(T_yy), F(T_zz), F(T_xy), F(T_xz), F(T_yz), F(a), F(c);
  // the field index is a compile-time constant in each body
  static_for<0, 8>([&](auto fc) {
    constexpr int f = decltype(fc)::value;
    cpx<double> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      // -i k s  ->  (k s.im, -k s.re)
      const double kze = kz[e];
      cpx<double> x;
      if constexpr (f == 0) x = {kx * sb[0][e].im, -kx * sb[0][e].re};
      else if constexpr (f == 1) x = {ky * sb[1][e].im, -ky * sb[1][e].re};
      else if constexpr (f == 2) x = {kze * sb[2][e].im, -kze * sb[2][e].re};
      else if constexpr (f == 3) x = {ky * sb[0][e].im + kx * sb[1][e].im, -ky * sb[0][e].re - kx * sb[1][e].re};
      else if constexpr (f == 4) x = {kze * sb[0][e].im + kx * sb[2][e].im, -kze * sb[0][e].re - kx * sb[2][e].re};
      else if constexpr (f == 5) x = {kze * sb[1][e].im + ky * sb[2][e].im, -kze * sb[1][e].re - ky * sb[2][e].re};
      else if constexpr (f == 6) x = {-sb[3][e].re, -sb[3][e].im};
      else {
        const double k2 = kx * kx + ky * ky + kze * kze;
        x = {-k2 * ac.inv_pe * sb[3][e].re, -k2 * ac.inv_pe * sb[3][e].im};
      }
      v[e] = x;
    }
    fft_line<double, P, 1>(v, lds[0], lds[1], par, t, idx, tw);
    cpx<double>* dst = gout + (long long)f * N * Q;
    if (valid) {
#pragma unroll
      for (int b = 0; b < E / RO; ++b)
#pragma unroll
        for (int r = 0; r < RO; ++r) dst[(long long)slot_pos<P, RO>(t, b, r) * Q + q] = v[b * RO + r];
    }
  });
}

// -------------------------------------------------------------------------
// x stage of the adjoint.  yf: the forward step's y-inverse output
// [6][N][N][H] (u v w phi dy_phi dz_phi), yb: the product cotangents after
// the y-inverse [8][N][N][H]; out: [7][N][N][H] x-forward of the cotangents
// of u v w phi gx gy gz.  part[blockIdx.x]: this block's share of
// sum_x sum_f Tbar_f dT_f/dc (the We term before the factor -c/(We n^3)).
template <int N>
__global__ void __launch_bounds__(256) k_xadj(const cpx<double>* __restrict__ yf, const cpx<double>* __restrict__ yb,
                                              cpx<double>* __restrict__ out, const cpx<double>* __restrict__ tw_g,
                                              double csig, double* __restrict__ part) {
  using P = Plan<N>;
  using G = Tile<P>;
  constexpr int E = G::E, TT = G::TT, L = G::L, LP = kRowStride<N>, K = G::K, H = G::H;
  constexpr int RI = first_radix<P, 1>(), RP = last_radix<P, 1>(), RO = last_radix<P, -1>();
  static_assert(RP == first_radix<P, -1>(), "mirrored radix order");
  constexpr long long ROWS = (long long)N * N;
  __shared__ cpx<double> twf[tw_size<P, -1>()];
  __shared__ cpx<double> twi[tw_size<P, 1>()];
  __shared__ cpx<double> lds[2][L * LP];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int t = tid % TT, line = tid / TT;
  build_twiddles<double, P, -1>(twf, [&](int m) { return tw_g[m]; }, tid, int(blockDim.x));
  build_twiddles<double, P, 1>(twi, [&](int m) { return tw_g[m]; }, tid, int(blockDim.x));
  const long long r0 = ((long long)blockIdx.x * L + line) * 2;
  const bool valid = r0 < ROWS;
  const IdxLineMajor<N, TT> idx{line * LP};
  int par = 0;
  __syncthreads();

  // x-inverse of one field of a [*][N][N][H] array into register slots (re: row r0, im: row r0+1)
  auto xinv = [&](const cpx<double>* src, bool dx, cpx<double>* v) {
#pragma unroll
    for (int b = 0; b < E / RI; ++b)
#pragma unroll
      for (int r = 0; r < RI; ++r) {
        const int p = slot_pos<P, RI>(t, b, r);
        const int k = (p <= N / 2) ? p : N - p;
        cpx<double> z = {0.0, 0.0};
        if (valid && k <= K) {
          cpx<double> A = src[r0 * H + k], B = src[(r0 + 1) * H + k];
          if (dx) {
            const double kk = double(k);
            A = cpx<double>{-kk * A.im, kk * A.re};
            B = cpx<double>{-kk * B.im, kk * B.re};
          }
          if (k == 0) {
            A.im = 0.0;
            B.im = 0.0;
          }
          z = (p <= N / 2) ? cpx<double>{A.re - B.im, A.im + B.re} : cpx<double>{A.re + B.im, B.re - A.im};
        }
        v[b * RI + r] = z;
      }
    fft_line<double, P, 1>(v, lds[0], lds[1], par, t, idx, twi);
  };
  // x-forward of register slots and store of the retained kx of both rows
  auto xfwd = [&](cpx<double>* v, cpx<double>* dst) {
    fft_line<double, P, -1>(v, lds[0], lds[1], par, t, idx, twf);
    cpx<double>* Lb = par ? lds[1] : lds[0];
    par ^= 1;
#pragma unroll
    for (int b = 0; b < E / RO; ++b)
#pragma unroll
      for (int r = 0; r < RO; ++r) Lb[idx(slot_pos<P, RO>(t, b, r))] = v[b * RO + r];
    wave_lds_sync();  // the line's threads are one wavefront's lanes
    for (int k = t; valid && k < H; k += TT) {
      const cpx<double> zk = Lb[idx(k)], zm = Lb[idx((N - k) % N)];
      dst[r0 * H + k] = cpx<double>{0.5 * (zk.re + zm.re), 0.5 * (zk.im - zm.im)};
      dst[(r0 + 1) * H + k] = cpx<double>{0.5 * (zk.im + zm.im), 0.5 * (zm.re - zk.re)};
    }
  };
  const long long FS = ROWS * H;

  // phi: phi_bar = 3 phi^2 c_bar
  {
    cpx<double> ph[E], cb[E];
    xinv(yf + 3 * FS, false, ph);
    xinv(yb + 7 * FS, false, cb);
#pragma unroll
    for (int e = 0; e < E; ++e) cb[e] = cpx<double>{3.0 * ph[e].re * ph[e].re * cb[e].re, 3.0 * ph[e].im * ph[e].im * cb[e].im};
    xfwd(cb, out + 3 * FS);
  }
  // forward fields u v w gx gy gz
  cpx<double> fw[6][E];
  xinv(yf + 0 * FS, false, fw[0]);
  xinv(yf + 1 * FS, false, fw[1]);
  xinv(yf + 2 * FS, false, fw[2]);
  xinv(yf + 3 * FS, true, fw[3]);
  xinv(yf + 4 * FS, false, fw[4]);
  xinv(yf + 5 * FS, false, fw[5]);
  cpx<double> acc[6][E];
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[c][e] = cpx<double>{0.0, 0.0};
  double dwe = 0.0;
  const double c2 = 2.0 * csig;
  static_for<0, 7>([&](auto fc) {
    constexpr int f = decltype(fc)::value;
    cpx<double> tb[E];
    xinv(yb + f * FS, false, tb);
#pragma unroll
    for (int e = 0; e < E; ++e) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double u = h ? fw[0][e].im : fw[0][e].re, v = h ? fw[1][e].im : fw[1][e].re;
        const double w = h ? fw[2][e].im : fw[2][e].re, gx = h ? fw[3][e].im : fw[3][e].re;
        const double gy = h ? fw[4][e].im : fw[4][e].re, gz = h ? fw[5][e].im : fw[5][e].re;
        const double x = h ? tb[e].im : tb[e].re;
        double du = 0, dv = 0, dw = 0, dgx = 0, dgy = 0, dgz = 0;
        if constexpr (f == 0) { du = -2.0 * u * x; dgy = c2 * gy * x; dgz = c2 * gz * x; dwe += x * (gy * gy + gz * gz); }
        else if constexpr (f == 1) { dv = -2.0 * v * x; dgx = c2 * gx * x; dgz = c2 * gz * x; dwe += x * (gx * gx + gz * gz); }
        else if constexpr (f == 2) { dw = -2.0 * w * x; dgx = c2 * gx * x; dgy = c2 * gy * x; dwe += x * (gx * gx + gy * gy); }
        else if constexpr (f == 3) { du = -v * x; dv = -u * x; dgx = -csig * gy * x; dgy = -csig * gx * x; dwe -= x * gx * gy; }
        else if constexpr (f == 4) { du = -w * x; dw = -u * x; dgx = -csig * gz * x; dgz = -csig * gx * x; dwe -= x * gx * gz; }
        else if constexpr (f == 5) { dv = -w * x; dw = -v * x; dgy = -csig * gz * x; dgz = -csig * gy * x; dwe -= x * gy * gz; }
        else { du = gx * x; dv = gy * x; dw = gz * x; dgx = u * x; dgy = v * x; dgz = w * x; }
        if (h) {
          acc[0][e].im += du; acc[1][e].im += dv; acc[2][e].im += dw;
          acc[3][e].im += dgx; acc[4][e].im += dgy; acc[5][e].im += dgz;
        } else {
          acc[0][e].re += du; acc[1][e].re += dv; acc[2][e].re += dw;
          acc[3][e].re += dgx; acc[4][e].re += dgy; acc[5][e].re += dgz;
        }
      }
    }
  });
  if (!valid) dwe = 0.0;
  xfwd(acc[0], out + 0 * FS);
  xfwd(acc[1], out + 1 * FS);
  xfwd(acc[2], out + 2 * FS);
  xfwd(acc[3], out + 4 * FS);
  xfwd(acc[4], out + 5 * FS);
  xfwd(acc[5], out + 6 * FS);
  // block reduction of the We term (fixed order: deterministic)
  red[tid] = dwe;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) part[blockIdx.x] = red[0];
}

// -------------------------------------------------------------------------
// z-forward of the 7 field cotangents [7][N][C][H] and accumulation into lam:
// lam_u += F(ubar), lam_phi += F(phibar) - sum_j i k_j F(gbar_j).
template <int N>
__global__ void __launch_bounds__(256) k_zadj_out(const cpx<double>* __restrict__ zin, cpx<double>* __restrict__ lam,
                                                  const cpx<double>* __restrict__ tw_g, double inv_n3) {
  using P = Plan<N>;
  using G = Tile<P>;
  constexpr int E = G::E, L = G::L, LP = L + 1, K = G::K, C = G::C, H = G::H;
  constexpr int Q = C * H;
  constexpr long long M = (long long)C * Q;
  constexpr int RF = first_radix<P, -1>(), RL = last_radix<P, -1>();
  __shared__ cpx<double> tw[N];
  __shared__ cpx<double> lds[2][N * LP];
  const int tid = threadIdx.x;
  const int line = tid % L, t = tid / L;
  for (int i = tid; i < N; i += blockDim.x) tw[i] = tw_g[i];
  const int q = blockIdx.x * L + line;
  const bool valid = q < Q;
  const int iy = valid ? q / H : 0, ix = valid ? q % H : 0;
  const double kx = double(ix), ky = double(iy <= K ? iy : iy - C);
  const IdxPosMajor idx{LP, line};
  int par = 0;
  cpx<double> acc[4][E];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[c][e] = cpx<double>{0.0, 0.0};
  __syncthreads();
#pragma unroll 1
  for (int f = 0; f < 7; ++f) {
    cpx<double> v[E];
    const cpx<double>* src = zin + (long long)f * N * Q;
#pragma unroll
    for (int b = 0; b < E / RF; ++b)
#pragma unroll
      for (int r = 0; r < RF; ++r)
        v[b * RF + r] = valid ? src[(long long)slot_pos<P, RF>(t, b, r) * Q + q] : cpx<double>{0.0, 0.0};
    fft_line<double, P, -1>(v, lds[0], lds[1], par, t, idx, tw);
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int e = b * RL + r;
        const cpx<double> w = {v[e].re * inv_n3, v[e].im * inv_n3};
        const double kz = double(signed_k(slot_pos<P, RL>(t, b, r), N));
        if (f == 0) acc[0][e] = cadd(acc[0][e], w);
        else if (f == 1) acc[1][e] = cadd(acc[1][e], w);
        else if (f == 2) acc[2][e] = cadd(acc[2][e], w);
        else if (f == 3) acc[3][e] = cadd(acc[3][e], w);
        else {
          const double k = (f == 4) ? kx : (f == 5) ? ky : kz;   // -i k w
          acc[3][e].re += k * w.im;
          acc[3][e].im -= k * w.re;
        }
      }
  }
  if (valid) {
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int e = b * RL + r;
        const int s = band_slot(slot_pos<P, RL>(t, b, r), C, N);
        if (s >= 0) {
          const long long id = (long long)s * Q + q;
#pragma unroll
          for (int c = 0; c < 4; ++c) lam[c * M + id] = cadd(lam[c * M + id], acc[c][e]);
        }
      }
  }
}

// Terminal cotangent of J = V (<|grad phi|^2> + 1/2 <|u|^2>):
// lam_u = V u_hat, lam_phi = 2 V k^2 phi_hat, mu = 0 (compact band, per mode).
__global__ void k_adj_terminal(const cpx<double>* __restrict__ st, cpx<double>* __restrict__ lam,
                               cpx<double>* __restrict__ mu, int K, int C, int H, long long M, double vol) {
  for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < M;
       id += (long long)gridDim.x * blockDim.x) {
    const int ix = int(id % H);
    const int iy = int((id / H) % C);
    const int iz = int(id / ((long long)H * C));
    const double kx = ix, ky = (iy <= K) ? iy : iy - C, kz = (iz <= K) ? iz : iz - C;
    const double k2 = kx * kx + ky * ky + kz * kz;
    for (int c = 0; c < 3; ++c) {
      const cpx<double> a = st[c * M + id];
      lam[c * M + id] = cpx<double>{vol * a.re, vol * a.im};
    }
    const cpx<double> p = st[3 * M + id];
    lam[3 * M + id] = cpx<double>{2.0 * vol * k2 * p.re, 2.0 * vol * k2 * p.im};
    for (int c = 0; c < 4; ++c) mu[c * M + id] = cpx<double>{0.0, 0.0};
  }
}

// acc[0] += scale * sum(part[0..n-1]) in a fixed order (one block).
__global__ void k_adj_sum(const double* __restrict__ part, int n, double scale, double* __restrict__ acc) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[0] += scale * red[0];
}

// -------------------------------------------------------------------------
#define PSMS_FOR_EACH_N(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256)

namespace {
template <int N>
hipError_t adj_n(int stage, cpx<double>* lam, cpx<double>* mu, const cpx<double>* a, const cpx<double>* b,
                 cpx<double>* out, const cpx<double>* tw, const AdjCoef& ac, double csig, double* part,
                 hipStream_t st) {
  using P = Plan<N>;
  using G = Tile<P>;
  const int Q = G::C * G::H;
  const unsigned threads = unsigned(G::L * G::TT);
  if (stage == 0) {
    k_zadj_in<N><<<unsigned((Q + G::L - 1) / G::L), threads, 0, st>>>(lam, mu, out, tw, ac);
  } else if (stage == 1) {
    const long long pairs = (long long)N * N / 2;
    k_xadj<N><<<unsigned((pairs + G::L - 1) / G::L), threads, 0, st>>>(a, b, out, tw, csig, part);
  } else {
    k_zadj_out<N><<<unsigned((Q + G::L - 1) / G::L), threads, 0, st>>>(a, lam, tw, ac.inv_n3);
  }
  return hipGetLastError();
}
}  // namespace

int adj_xblocks(int n) {
  switch (n) {
#define PSMS_CASE(NN) \
  case NN: return int(((long long)NN * NN / 2 + Tile<Plan<NN>>::L - 1) / Tile<Plan<NN>>::L);
    PSMS_FOR_EACH_N(PSMS_CASE)
#undef PSMS_CASE
  }
  return 0;
}

hipError_t launch_adj_stage(int n, int stage, cpx<double>* lam, cpx<double>* mu, const cpx<double>* a,
                            const cpx<double>* b, cpx<double>* out, const cpx<double>* tw, const AdjCoef& ac,
                            double csig, double* part, hipStream_t st) {
  switch (n) {
#define PSMS_CASE(NN) case NN: return adj_n<NN>(stage, lam, mu, a, b, out, tw, ac, csig, part, st);
    PSMS_FOR_EACH_N(PSMS_CASE)
#undef PSMS_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adj_terminal(const cpx<double>* state, cpx<double>* lam, cpx<double>* mu, int K, int C, int H,
                               long long M, double vol, hipStream_t st) {
  long long b = (M + 255) / 256;
  if (b > 65536) b = 65536;
  k_adj_terminal<<<unsigned(b), 256, 0, st>>>(state, lam, mu, K, C, H, M, vol);
  return hipGetLastError();
}

hipError_t launch_adj_sum(const double* part, int n, double scale, double* acc, hipStream_t st) {
  k_adj_sum<<<1, 256, 0, st>>>(part, n, scale, acc);
  return hipGetLastError();
}

}  // namespace psms
