// Wall-normal (Chebyshev) kernels of the channel: Sec. 2.2 and Sec. 3.2.
//
//  * k_dct: the Chebyshev transform as a DCT-I obtained from the FFT of the
//    2 nc-point even extension of each line (Sec. 3.2.1), applied to the real
//    and imaginary parts at once; k_dct_half the same through one nc-point
//    FFT.  Lines are (kx, ky) pairs, stored position-major ([n][line]), so the
//    lanes of a wavefront read consecutive lines and no transpose is needed.
//    Both read through a source: an array, or the channel step's fields formed
//    from the state as they are loaded.
//  * k_cheb_seg, k_cheb_seg_q: derivative (and D^2 - k^2) in coefficient
//    space, the backward recurrence c_{n-1} b_{n-1} = b_{n+1} + 2 n a_n summed
//    piecewise along each parity chain.
//  * k_helm: the Chebyshev-tau Helmholtz problem (D^2 - beta) f = g with two
//    Dirichlet or Neumann boundary rows, in FP64.  Rewriting the tau rows with
//    the integration recurrence turns each parity (even / odd n) into a
//    tridiagonal system plus one boundary row; it is solved by one downward
//    elimination sweep and two upward sweeps, one thread per (line, parity)
//    (the banded wall-normal solves of Sec. 3.2.2).  k_helm_batch_reg keeps a
//    chain on chip; k_helm_factors stores a context's elimination factors,
//    from which k_helm_pieces solves each chain in 8 pieces (affine-map scans).
//  * k_influence, k_uv: the influence-matrix combination that enforces
//    w' = 0 at the walls, and u, v from continuity and eq. omegadef.
#include <hip/hip_runtime.h>

#include "channel_kernels.hpp"
#include "fft_engine.hpp"

namespace psms {

namespace {

// 16 lines per workgroup (8 for the 512-point extension, nc = 256): the lanes
// of a position read 16 consecutive lines (128 bytes in FP32), and the LDS
// tile stays within 160 KB in FP64.
template <class P>
struct CTile {
  static constexpr int N = P::N;
  static constexpr int E = P::E;
  static constexpr int TT = N / E;
  static constexpr int L = (16 * TT <= 1024) ? 16 : 1024 / TT;
  static_assert(L * TT <= 1024, "workgroup size");
  static_assert(2 * N * (L + 1) * 16 + N * 16 <= 160 * 1024, "LDS tile");
};

}  // namespace

// dir = +1: values at the CGL points -> Chebyshev coefficients,
//   a_n = G_n / (nc cbar_n),  G = FFT of the even extension of f;
// dir = -1: coefficients -> values, f_j = FFT of the even extension of b with
//   b_0 = a_0, b_nc = a_nc, b_n = a_n / 2.
// out64 (forward only, if not NULL): the coefficients are written in FP64
// instead, those with n > kz as zero (the products' Chebyshev truncation),
// so the step needs no separate promotion pass.
// Where the DCT kernels read their input value of field f, coefficient j, line
// l: an array [field][n][line] (ArraySrc), or the channel step's fields formed
// from the FP64 state as they are loaded (ChanFieldSrc: u, v by continuity and
// the definition of omega_z, w, phi, i ky phi, D phi).
template <typename T>
struct ArraySrc {
  const cpx<T>* in;
  long long fstride, nlines;
  __device__ __forceinline__ cpx<T> operator()(int f, long long j, long long l) const {
    return in[f * fstride + j * nlines + l];
  }
};
template <typename T>
struct ChanFieldSrcT {
  ChanFieldSrc s;
  __device__ __forceinline__ cpx<T> operator()(int f, long long j, long long l) const {
    const long long id = j * s.nlines + l;
    cpx<double> x;
    if (f <= 1) {
      if (l == 0) {                          // the mean line carries U, V
        x = s.mean[2 * j + f];
      } else {
        const double kx = s.kx[l], ky = s.ky[l];
        const double ik2 = 1.0 / (kx * kx + ky * ky);
        const cpx<double> o = s.om[id], d = s.dw[id];
        const cpx<double> a = (f == 0) ? cpx<double>{kx * d.re + ky * o.re, kx * d.im + ky * o.im}
                                       : cpx<double>{ky * d.re - kx * o.re, ky * d.im - kx * o.im};
        x = cpx<double>{ik2 * (-1.0 * a.im), ik2 * (1.0 * a.re)};   // i a / k^2
      }
    } else if (f == 2) {
      x = s.w[id];
    } else if (f == 3) {
      x = s.phi[id];
    } else if (f == 4) {
      const double ky = s.ky[l];
      const cpx<double> p = s.phi[id];
      x = cpx<double>{-ky * p.im, ky * p.re};
    } else {
      x = s.dphi[id];
    }
    return cpx<T>{T(x.re), T(x.im)};
  }
};

template <typename T, int N, class Src>
__global__ void __launch_bounds__(1024) k_dct(Src src, cpx<T>* __restrict__ out,
                                             long long nlines, int dir, long long fstride,
                                             const cpx<T>* __restrict__ tw_g, cpx<double>* __restrict__ out64,
                                             int kz) {
  using P = Plan<N>;
  using G = CTile<P>;
  constexpr int E = G::E, L = G::L, LP = L + 1, NC = N / 2;
  constexpr int RI = first_radix<P, -1>(), RO = last_radix<P, -1>();
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> lds[2][N * LP];
  const int tid = threadIdx.x;
  const int line = tid % L, t = tid / L;
  out += (long long)blockIdx.y * fstride;   // field blockIdx.y
  if (out64) out64 += (long long)blockIdx.y * fstride;
  if (tw_g) {
    for (int i = tid; i < N; i += blockDim.x) tw[i] = tw_g[i];
  } else {
    for (int i = tid; i < N; i += blockDim.x) {
      double s, c;
      sincospi(-2.0 * double(i) / double(N), &s, &c);
      tw[i] = cpx<T>{T(c), T(s)};
    }
  }
  const long long l = (long long)blockIdx.x * L + line;
  const bool valid = l < nlines;
  cpx<T> v[E];
#pragma unroll
  for (int b = 0; b < E / RI; ++b)
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int p = slot_pos<P, RI>(t, b, r);
      const int j = (p <= NC) ? p : N - p;
      cpx<T> x = {T(0), T(0)};
      if (valid) {
        x = src(int(blockIdx.y), j, l);
        if (dir < 0 && j != 0 && j != NC) {
          x.re *= T(0.5);
          x.im *= T(0.5);
        }
      }
      v[b * RI + r] = x;
    }
  __syncthreads();
  int par = 0;
  fft_line<T, P, -1>(v, lds[0], lds[1], par, t, IdxPosMajor{LP, line}, tw);
  if (valid) {
#pragma unroll
    for (int b = 0; b < E / RO; ++b)
#pragma unroll
      for (int r = 0; r < RO; ++r) {
        const int p = slot_pos<P, RO>(t, b, r);
        if (p <= NC) {
          cpx<T> x = v[b * RO + r];
          if (dir > 0) {
            const T sc = T(1.0 / (double(NC) * ((p == 0 || p == NC) ? 2.0 : 1.0)));
            x.re *= sc;
            x.im *= sc;
          }
          if (out64)
            out64[(long long)p * nlines + l] = (p > kz) ? cpx<double>{0.0, 0.0} : cpx<double>{double(x.re), double(x.im)};
          else
            out[(long long)p * nlines + l] = x;
        }
      }
  }
}

// The same transform through one FFT of nc points instead of 2 nc (the
// half-length route to the DCT-I; Sec. 3.2.1 names it as the next step).  With
// the end points halved, C_k = sum_j w_j x_j cos(pi j k / nc) (w_0 = w_nc = 1/2)
// is obtained from Z = FFT_nc(y),
//   y_0 = (x_0 + x_nc) / 2,  y_j = (x_j + x_{nc-j}) / 2 - sin(pi j / nc) (x_j - x_{nc-j}):
// the even part of y carries the cosines of even order and the odd part, with
// the sine, the differences of neighbouring odd orders, so
//   C_{2k} = (Z_k + Z_{nc-k}) / 2,
//   C_{2k+1} = C_{2k-1} + (i / 2) (Z_k - Z_{nc-k}),  C_1 = sum_j w_j x_j cos(pi j / nc)
// (complex x: the real and imaginary parts go through the one FFT together).
// The odd orders are a running sum over k, formed in FP64: each thread of a
// line sums a contiguous run of k, and the runs' totals give every thread its
// starting value.  dir = +1: x = f, a_n = 2 C_n / (nc cbar_n); dir = -1:
// x = cbar a, f_j = C_j.  tw_g: exp(-i pi m / nc), m < 2 nc (or NULL).
template <typename T, int NC, class Src>
__global__ void __launch_bounds__(1024) k_dct_half(Src src, cpx<T>* __restrict__ out,
                                                  long long nlines, int dir, long long fstride,
                                                  const cpx<T>* __restrict__ tw_g, cpx<double>* __restrict__ out64,
                                                  int kz) {
  using P = Plan<NC>;
  using G = CTile<P>;
  constexpr int E = G::E, L = G::L, LP = L + 1, TT = G::TT;
  constexpr int RI = first_radix<P, -1>(), RO = last_radix<P, -1>();
  constexpr int NK = NC / 2 - 1;                 // increments of the odd orders, k = 1 .. NC/2 - 1
  constexpr int CS = (NK + TT - 1) / TT;         // a thread's run of k
  static_assert(2 * NC * LP * int(sizeof(cpx<T>)) + 3 * NC * int(sizeof(cpx<T>)) <= 160 * 1024, "LDS");
  static_assert(TT * L * 2 * 16 <= NC * LP * int(sizeof(cpx<T>)), "partial sums fit one exchange buffer");
  __shared__ cpx<T> tw2[2 * NC];                 // exp(-i pi m / NC)
  __shared__ cpx<T> tw[NC];                      // exp(-2 pi i m / NC)
  __shared__ cpx<T> lds[2][NC * LP];
  const int tid = threadIdx.x;
  const int line = tid % L, t = tid / L;
  out += (long long)blockIdx.y * fstride;
  if (out64) out64 += (long long)blockIdx.y * fstride;
  for (int i = tid; i < 2 * NC; i += blockDim.x) {
    cpx<T> w;
    if (tw_g) {
      w = tw_g[i];
    } else {
      double s, c;
      sincospi(-double(i) / double(NC), &s, &c);
      w = cpx<T>{T(c), T(s)};
    }
    tw2[i] = w;
    if (!(i & 1)) tw[i >> 1] = w;
  }
  const long long l = (long long)blockIdx.x * L + line;
  const bool valid = l < nlines;
  __syncthreads();
  // y at the positions the FFT starts from, and this thread's share of C_1
  cpx<T> v[E];
  double c1r = 0.0, c1i = 0.0;
#pragma unroll
  for (int b = 0; b < E / RI; ++b)
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int j = slot_pos<P, RI>(t, b, r);    // 0 .. NC-1
      cpx<T> y = {T(0), T(0)};
      if (valid) {
        cpx<T> xa = src(int(blockIdx.y), j, l);
        cpx<T> xb = src(int(blockIdx.y), NC - j, l);   // x_{NC-j} (x_NC for j = 0)
        if (dir < 0 && j == 0) {                 // x = cbar a: the end points doubled
          xa = cpx<T>{T(2) * xa.re, T(2) * xa.im};
          xb = cpx<T>{T(2) * xb.re, T(2) * xb.im};
        }
        const T cj = tw2[j].re, sj = -tw2[j].im;   // cos, sin (pi j / NC)
        if (j == 0) {
          y = cpx<T>{T(0.5) * (xa.re + xb.re), T(0.5) * (xa.im + xb.im)};
          c1r += 0.5 * double(xa.re) - 0.5 * double(xb.re);   // w_0 x_0 cos 0 + w_NC x_NC cos pi
          c1i += 0.5 * double(xa.im) - 0.5 * double(xb.im);
        } else {
          const cpx<T> sm = {T(0.5) * (xa.re + xb.re), T(0.5) * (xa.im + xb.im)};
          const cpx<T> df = {xa.re - xb.re, xa.im - xb.im};
          y = cpx<T>{sm.re - sj * df.re, sm.im - sj * df.im};
          c1r += double(cj) * double(xa.re);
          c1i += double(cj) * double(xa.im);
        }
      }
      v[b * RI + r] = y;
    }
  int par = 0;
  fft_line<T, P, -1>(v, lds[0], lds[1], par, t, IdxPosMajor{LP, line}, tw);
  // Z in natural order in lds[0]; the partial sums in lds[1] (as doubles)
  __syncthreads();
  const IdxPosMajor idx{LP, line};
#pragma unroll
  for (int b = 0; b < E / RO; ++b)
#pragma unroll
    for (int r = 0; r < RO; ++r) lds[0][idx(slot_pos<P, RO>(t, b, r))] = v[b * RO + r];
  double* ps = reinterpret_cast<double*>(lds[1]);     // [2][TT][L] pairs (re, im)
  ps[2 * (t * L + line)] = c1r;
  ps[2 * (t * L + line) + 1] = c1i;
  __syncthreads();
  double s1r = 0.0, s1i = 0.0;                         // C_1 of the line
#pragma unroll 4
  for (int u = 0; u < TT; ++u) {
    s1r += ps[2 * (u * L + line)];
    s1i += ps[2 * (u * L + line) + 1];
  }
  // this thread's run of increments (i/2)(Z_k - Z_{NC-k}), k in [k0, k1)
  const int k0 = 1 + t * CS, k1 = (k0 + CS <= NK + 1) ? k0 + CS : NK + 1;
  double rr = 0.0, ri = 0.0;
#pragma unroll 2
  for (int k = k0; k < k1; ++k) {
    const cpx<T> a = lds[0][idx(k)], c = lds[0][idx(NC - k)];
    rr += -0.5 * (double(a.im) - double(c.im));
    ri += 0.5 * (double(a.re) - double(c.re));
  }
  ps[2 * TT * L + 2 * (t * L + line)] = rr;
  ps[2 * TT * L + 2 * (t * L + line) + 1] = ri;
  __syncthreads();
  if (!valid) return;
  auto put = [&](int n, double re, double im) {
    if (dir > 0) {
      const double sc = 2.0 / (double(NC) * ((n == 0 || n == NC) ? 2.0 : 1.0));
      re *= sc;
      im *= sc;
    }
    if (out64)
      out64[(long long)n * nlines + l] = (n > kz) ? cpx<double>{0.0, 0.0} : cpx<double>{re, im};
    else
      out[(long long)n * nlines + l] = cpx<T>{T(re), T(im)};
  };
  // even orders
#pragma unroll 1
  for (int k = t; k <= NC / 2; k += TT) {
    const cpx<T> a = lds[0][idx(k)], c = lds[0][idx((NC - k) % NC)];
    put(2 * k, 0.5 * (double(a.re) + double(c.re)), 0.5 * (double(a.im) + double(c.im)));
  }
  // odd orders: C_1 plus the runs before this thread's, then its own run
  double ar = s1r, ai = s1i;
#pragma unroll 4
  for (int u = 0; u < t; ++u) {
    ar += ps[2 * TT * L + 2 * (u * L + line)];
    ai += ps[2 * TT * L + 2 * (u * L + line) + 1];
  }
  if (t == 0) put(1, ar, ai);
#pragma unroll 1
  for (int k = k0; k < k1; ++k) {
    const cpx<T> a = lds[0][idx(k)], c = lds[0][idx(NC - k)];
    ar += -0.5 * (double(a.im) - double(c.im));
    ai += 0.5 * (double(a.re) - double(c.re));
    put(2 * k + 1, ar, ai);
  }
}

// Coefficients of d/dz: b_nc = 0, c_{m} b_{m} = b_{m+2} + 2 (m+1) a_{m+1} for
// m = nc-1 .. 0 (c_0 = 2, else 1); and of D^2 - k^2 through c = D b with
// b = D a.  Both recurrences link m to m+2 only, so the outputs of each parity
// form a chain, and along a chain they are suffix sums:
//   D:       c_m b_m = B_m = sum_{j >= m, j = m mod 2} 2 (j+1) a_{j+1}
//   D^2:     b_{m+1} = sum_{p >= m+2, p = m mod 2} 2 p a_p,
//            c_m (D^2 a)_m = sum_{j >= m, j = m mod 2} 2 (j+1) b_{j+1}.
// A chain of cnt terms (m = top, top-2, ..) is cut into PC pieces (8, or 16
// for the longest chains) of at most LEN terms; each lane sums its piece, and
// the pieces' totals are combined by a scan across the lanes.  A wavefront
// holds the chains of one parity of 64 / PC consecutive lines: lane =
// (64 / PC) piece + line, so that for one term the lanes of a piece read
// consecutive lines (128 or 64 contiguous bytes), and each lane issues its
// piece's loads at once.  (One lane per chain would leave a 256 x 129 line set
// with fewer wavefronts than SIMDs, each waiting on one load per term.)
namespace {

// exclusive scan over the PC pieces of a chain (lanes 64 / PC apart), piece
// `pc` of this lane
template <int PC>
__device__ __forceinline__ cpx<double> piece_carry(cpx<double> tot, int pc) {
  constexpr int LPW = 64 / PC;
  auto up = [](cpx<double> v, int d) { return cpx<double>{__shfl_up(v.re, LPW * d), __shfl_up(v.im, LPW * d)}; };
  cpx<double> inc = tot;
#pragma unroll
  for (int d = 1; d < PC; d <<= 1) {
    const cpx<double> o = up(inc, d);
    if (pc >= d) inc = cadd(inc, o);
  }
  const cpx<double> ex = up(inc, 1);
  return pc == 0 ? cpx<double>{0.0, 0.0} : ex;
}

template <int LEN, int PC>
__global__ void __launch_bounds__(256) k_cheb_seg(ChebBatch bt, int nc, long long nlines,
                                                  const double* __restrict__ kx, const double* __restrict__ ky,
                                                  int lapmask) {
  constexpr int LPW = 64 / PC;   // lines per wavefront
  const int lap = (lapmask >> blockIdx.y) & 1;   // uniform in the workgroup
  if (bt.nl[blockIdx.y]) nlines = bt.nl[blockIdx.y];
  if ((bt.nok >> blockIdx.y) & 1) kx = nullptr;
  const int lane = threadIdx.x & 63;
  const int pc = lane / LPW;
  const long long groups = (nlines + LPW - 1) / LPW;
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wave >= 2 * groups) return;   // whole wavefronts
  const int q = int(wave / groups);
  const long long l = (wave % groups) * LPW + (lane % LPW);
  const bool valid = l < nlines;
  const cpx<double>* __restrict__ a = bt.in[blockIdx.y];
  cpx<double>* __restrict__ out = bt.out[blockIdx.y];
  const int top = ((nc - q) & 1) ? nc - 1 : nc;   // largest m <= nc of parity q
  const int cnt = top / 2 + 1;                     // terms m = top, top - 2, .., q
  const int i0 = pc * LEN;
  const cpx<double> zero = {0.0, 0.0};
  if (!lap) {
    cpx<double> x[LEN];
#pragma unroll
    for (int k = 0; k < LEN; ++k) {
      const int m = top - 2 * (i0 + k);
      x[k] = zero;
      if (valid && i0 + k < cnt && m + 1 <= nc) {
        const cpx<double> v = a[(long long)(m + 1) * nlines + l];
        x[k] = cpx<double>{2.0 * (m + 1) * v.re, 2.0 * (m + 1) * v.im};
      }
    }
#pragma unroll
    for (int k = 1; k < LEN; ++k) x[k] = cadd(x[k - 1], x[k]);
    const cpx<double> c = piece_carry<PC>(x[LEN - 1], pc);
#pragma unroll
    for (int k = 0; k < LEN; ++k) {
      const int m = top - 2 * (i0 + k);
      if (valid && i0 + k < cnt) {
        const double s = (m == 0) ? 0.5 : 1.0;
        const cpx<double> bm = cadd(c, x[k]);
        out[(long long)m * nlines + l] = cpx<double>{s * bm.re, s * bm.im};
      }
    }
    return;
  }
  const double k2 = (kx && valid) ? kx[l] * kx[l] + ky[l] * ky[l] : 0.0;
  // one D^2 - k^2 pass over the piece's terms in[k] (zero past the chain)
  auto lap_pass = [&](const cpx<double>* in, cpx<double>* res) {
    cpx<double> x[LEN];
    // b_{m+1} = sum of 2 p a_p over the chain's earlier terms (p > m): exclusive sums
    cpx<double> run = zero;
#pragma unroll
    for (int k = 0; k < LEN; ++k) {
      const int m = top - 2 * (i0 + k);
      x[k] = run;
      run = cadd(run, cpx<double>{2.0 * m * in[k].re, 2.0 * m * in[k].im});
    }
    const cpx<double> c1 = piece_carry<PC>(run, pc);
    // c_m = sum of 2 (j+1) b_{j+1} over j >= m: inclusive sums
    run = zero;
#pragma unroll
    for (int k = 0; k < LEN; ++k) {
      const int m = top - 2 * (i0 + k);
      const cpx<double> bm1 = cadd(c1, x[k]);
      run = cadd(run, cpx<double>{2.0 * (m + 1) * bm1.re, 2.0 * (m + 1) * bm1.im});
      x[k] = run;
    }
    const cpx<double> c2 = piece_carry<PC>(run, pc);
#pragma unroll
    for (int k = 0; k < LEN; ++k) {
      const int m = top - 2 * (i0 + k);
      const double s = (m == 0) ? 0.5 : 1.0;
      const cpx<double> cm = cadd(c2, x[k]);
      res[k] = (i0 + k < cnt) ? cpx<double>{s * cm.re - k2 * in[k].re, s * cm.im - k2 * in[k].im} : zero;
    }
  };
  const cpx<double>* __restrict__ a2 = bt.in2[blockIdx.y];
  const double w1 = bt.w1[blockIdx.y], w2 = bt.w2[blockIdx.y];
  const double ab = bt.addb[blockIdx.y], ab2 = bt.addb2[blockIdx.y];
  cpx<double> av[LEN], r1[LEN];
#pragma unroll
  for (int k = 0; k < LEN; ++k) {
    const int m = top - 2 * (i0 + k);
    av[k] = zero;
    if (valid && i0 + k < cnt) {
      av[k] = a[(long long)m * nlines + l];
      if (a2) {
        const cpx<double> b = a2[(long long)m * nlines + l];
        av[k] = cpx<double>{w1 * av[k].re + w2 * b.re, w1 * av[k].im + w2 * b.im};
      }
    }
  }
  lap_pass(av, r1);
  if (out) {
#pragma unroll
    for (int k = 0; k < LEN; ++k) {
      const int m = top - 2 * (i0 + k);
      if (valid && i0 + k < cnt)
        out[(long long)m * nlines + l] = cpx<double>{r1[k].re + ab * av[k].re, r1[k].im + ab * av[k].im};
    }
  }
  // optionally (D^2 - k^2)^2 as well: the chain of the result is in this wavefront
  cpx<double>* __restrict__ out2 = bt.out2[blockIdx.y];
  if (out2) {
    lap_pass(r1, av);
#pragma unroll
    for (int k = 0; k < LEN; ++k) {
      const int m = top - 2 * (i0 + k);
      if (valid && i0 + k < cnt)
        out2[(long long)m * nlines + l] = cpx<double>{av[k].re + ab2 * r1[k].re, av[k].im + ab2 * r1[k].im};
    }
  }
}


// D Q of Q = i kx S_x + i ky S_y, S_x = i kx T_xx + i ky T_xy + D T_xz,
// S_y = i kx T_xy + i ky T_yy + D T_yz (the horizontal divergence of the
// stress divergence), with Q formed term by term from its five arrays as it
// is loaded: the pieced D recurrence of k_cheb_seg.
template <int LEN, int PC>
__global__ void __launch_bounds__(256) k_cheb_seg_q(ChebQ in, int nc, long long nlines,
                                                    const double* __restrict__ kxl, const double* __restrict__ kyl,
                                                    cpx<double>* __restrict__ out) {
  constexpr int LPW = 64 / PC;   // lines per wavefront
  const int lane = threadIdx.x & 63;
  const int pc = lane / LPW;
  const long long groups = (nlines + LPW - 1) / LPW;
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wave >= 2 * groups) return;   // whole wavefronts
  const int q = int(wave / groups);
  const long long l = (wave % groups) * LPW + (lane % LPW);
  const bool valid = l < nlines;
  const double kx = valid ? kxl[l] : 0.0, ky = valid ? kyl[l] : 0.0;
  auto ti = [](double k, cpx<double> a) { return cpx<double>{-k * a.im, k * a.re}; };
  const int top = ((nc - q) & 1) ? nc - 1 : nc;
  const int cnt = top / 2 + 1;
  const int i0 = pc * LEN;
  cpx<double> x[LEN];
#pragma unroll
  for (int k = 0; k < LEN; ++k) {
    const int m = top - 2 * (i0 + k);
    x[k] = cpx<double>{0.0, 0.0};
    if (valid && i0 + k < cnt && m + 1 <= nc) {
      const long long id = (long long)(m + 1) * nlines + l;
      const cpx<double> txx = in.txx[id], tyy = in.tyy[id], txy = in.txy[id];
      const cpx<double> sx = cadd(cadd(ti(kx, txx), ti(ky, txy)), in.dxz[id]);
      const cpx<double> sy = cadd(cadd(ti(kx, txy), ti(ky, tyy)), in.dyz[id]);
      const cpx<double> v = cadd(ti(kx, sx), ti(ky, sy));
      x[k] = cpx<double>{2.0 * (m + 1) * v.re, 2.0 * (m + 1) * v.im};
    }
  }
#pragma unroll
  for (int k = 1; k < LEN; ++k) x[k] = cadd(x[k - 1], x[k]);
  const cpx<double> c = piece_carry<PC>(x[LEN - 1], pc);
#pragma unroll
  for (int k = 0; k < LEN; ++k) {
    const int m = top - 2 * (i0 + k);
    if (valid && i0 + k < cnt) {
      const double sm = (m == 0) ? 0.5 : 1.0;
      const cpx<double> bm = cadd(c, x[k]);
      out[(long long)m * nlines + l] = cpx<double>{sm * bm.re, sm * bm.im};
    }
  }
}
}  // namespace

// Chebyshev-tau Helmholtz solve (D^2 - beta) f = g, one thread per (line,
// parity).  For n >= 2 the tau rows are equivalent to
//   A_n a_{n-2} + B_n a_n + C_n a_{n+2} = R_n,
//   A_n = c_{n-2} beta / (4 n (n-1)),  B_n = -(1 + e_n beta / (2 (n^2 - 1))),
//   C_n = e_{n+2} beta / (4 n (n+1)),
//   R_n = -c_{n-2} g_{n-2} / (4 n (n-1)) + e_n g_n / (2 (n^2 - 1)) - e_{n+2} g_{n+2} / (4 n (n+1)),
// e_m = 1 if m <= nc-2 else 0: a tridiagonal chain per parity.  The boundary
// rows evaluate f (Dirichlet) or f' (Neumann) at each wall: bit 0 of bc makes
// the top wall (z = +1) Neumann, bit 1 the bottom wall.  With the same
// condition at both walls the rows split into one row per parity; with
// different conditions (a no-slip and a free-slip wall) they couple the two
// parities, and the thread of parity 0 solves both chains and the 2 x 2
// system for their first coefficients.
// beta = beta_line[l] (if given) + beta_add + (kx_l^2 + ky_l^2 if kx given).
// Boundary values: bcv[2l], bcv[2l+1] (top z=+1, bottom z=-1; if given)
// plus the constants top_c, bot_c.  g may be NULL (zero).  xw: nc+1 doubles
// per line of scratch.

// The coefficients of the tau rows that depend only on the index n:
// q1 = 1 / (4 n (n - 1)), q2 = 1 / (2 (n^2 - 1)), q3 = 1 / (4 n (n + 1)), n >= 2,
// evaluated at compile time (correctly rounded, as the run-time division would
// be) and read with wave-uniform addresses, so no recurrence step divides by them.
struct TauQ {
  double q[3][kTauQMax + 1];
};
constexpr int kHelmPieces = 8;   // pieces per chain in k_helm_pieces
constexpr TauQ make_tau_q() {
  TauQ t{};
  for (int n = 2; n <= kTauQMax; ++n) {
    const double dn = double(n);
    t.q[0][n] = 1.0 / (4.0 * dn * (dn - 1.0));
    t.q[1][n] = 1.0 / (2.0 * (dn * dn - 1.0));
    t.q[2][n] = 1.0 / (4.0 * dn * (dn + 1.0));
  }
  return t;
}
__constant__ TauQ kTauQ = make_tau_q();

// downward sweep of parity p: a_i = X_i a_{i-1} + Y_i for the indices
// n = p + 2 i, i = m..1 (X in xw, Y in f)
__device__ __forceinline__ void helm_down(const cpx<double>* __restrict__ g, cpx<double>* __restrict__ f,
                                          double* __restrict__ xw, int nc, long long nlines, double be, int p,
                                          long long l) {
  const int m = (nc - p) / 2;
  auto G = [&](int n) -> cpx<double> {
    if (!g || n > nc - 2 || n < 0) return cpx<double>{0.0, 0.0};
    return g[(long long)n * nlines + l];
  };
  double Xn = 0.0;
  cpx<double> Yn = {0.0, 0.0};
  cpx<double> gm = G(p + 2 * m - 2), g0 = G(p + 2 * m), g2 = G(p + 2 * m + 2);
#pragma unroll 4
  for (int i = m; i >= 1; --i) {
    const int n = p + 2 * i;
    const double dn = double(n);
    const double cm2 = (n - 2 == 0) ? 2.0 : 1.0;
    const double en = (n <= nc - 2) ? 1.0 : 0.0;
    const double en2 = (n + 2 <= nc - 2) ? 1.0 : 0.0;
    const double q1 = kTauQ.q[0][n], q2 = kTauQ.q[1][n], q3 = kTauQ.q[2][n];
    const double A = cm2 * be * q1;
    const double B = -(1.0 + en * be * q2);
    const double C = en2 * be * q3;
    const cpx<double> R = {-cm2 * gm.re * q1 + en * g0.re * q2 - en2 * g2.re * q3,
                           -cm2 * gm.im * q1 + en * g0.im * q2 - en2 * g2.im * q3};
    const double den = 1.0 / (B + C * Xn);
    const double X = -A * den;
    const cpx<double> Y = {(R.re - C * Yn.re) * den, (R.im - C * Yn.im) * den};
    xw[(long long)n * nlines + l] = X;
    f[(long long)n * nlines + l] = Y;
    Xn = X;
    Yn = Y;
    g2 = g0;
    g0 = gm;
    gm = G(n - 4);
  }
}

// wall weights of coefficient n: f(+1), f'(+1), f(-1), f'(-1)
__device__ __forceinline__ double helm_top_w(int n, bool neu) { return neu ? double(n) * double(n) : 1.0; }
__device__ __forceinline__ double helm_bot_w(int n, bool neu) {
  const double s = (n & 1) ? -1.0 : 1.0;   // (-1)^n
  return neu ? -s * double(n) * double(n) : s;
}

// upward sweep 1 of parity p: a_i = P_i a_p + Q_i; sums of the top and bottom
// rows over the chain
__device__ __forceinline__ void helm_up1(const cpx<double>* __restrict__ f, const double* __restrict__ xw, int nc,
                                         long long nlines, int p, long long l, bool ntop, bool nbot, double& SPt,
                                         cpx<double>& SQt, double& SPb, cpx<double>& SQb) {
  const int m = (nc - p) / 2;
  double P = 1.0;
  cpx<double> Qv = {0.0, 0.0};
  SPt = SPb = 0.0;
  SQt = SQb = cpx<double>{0.0, 0.0};
#pragma unroll 4
  for (int i = 0; i <= m; ++i) {
    const int n = p + 2 * i;
    if (i > 0) {
      const double X = xw[(long long)n * nlines + l];
      const cpx<double> Y = f[(long long)n * nlines + l];
      P = X * P;
      Qv = cpx<double>{X * Qv.re + Y.re, X * Qv.im + Y.im};
    }
    const double wt = helm_top_w(n, ntop), wb = helm_bot_w(n, nbot);
    SPt += wt * P;
    SQt.re += wt * Qv.re;
    SQt.im += wt * Qv.im;
    SPb += wb * P;
    SQb.re += wb * Qv.re;
    SQb.im += wb * Qv.im;
  }
}

// upward sweep 2 of parity p from its first coefficient a
__device__ __forceinline__ void helm_up2(cpx<double>* __restrict__ f, const double* __restrict__ xw, int nc,
                                         long long nlines, int p, long long l, cpx<double> a) {
  const int m = (nc - p) / 2;
  f[(long long)p * nlines + l] = a;
#pragma unroll 4
  for (int i = 1; i <= m; ++i) {
    const int n = p + 2 * i;
    const double X = xw[(long long)n * nlines + l];
    const cpx<double> Y = f[(long long)n * nlines + l];
    a = cpx<double>{X * a.re + Y.re, X * a.im + Y.im};
    f[(long long)n * nlines + l] = a;
  }
}

__device__ __forceinline__ void helm_line(const cpx<double>* __restrict__ g, cpx<double>* __restrict__ f,
                                          double* __restrict__ xw, int nc, long long nlines,
                                          const double* __restrict__ beta_line, double beta_add,
                                          const double* __restrict__ kx, const double* __restrict__ ky, int bc,
                                          const cpx<double>* __restrict__ bcv, cpx<double> top_c, cpx<double> bot_c,
                                          long long id) {
  const long long l = id % nlines;
  const int p = int(id / nlines);             // parity
  const bool ntop = bc & 1, nbot = (bc >> 1) & 1;
  if (ntop != nbot && p == 1) return;         // both chains on the thread of parity 0
  double be = beta_add;
  if (beta_line) be += beta_line[l];
  if (kx) be += kx[l] * kx[l] + ky[l] * ky[l];
  cpx<double> top = top_c, bot = bot_c;
  if (bcv) {
    top = cadd(top, bcv[2 * l]);
    bot = cadd(bot, bcv[2 * l + 1]);
  }
  if (ntop == nbot) {
    // the rows (top +- bottom)/2 restricted to this parity: sum_i w_i a_i = s
    cpx<double> s;
    const bool plus = (p == 0) != ntop;       // Dirichlet even, Neumann odd: (top + bottom) / 2
    s = plus ? cpx<double>{0.5 * (top.re + bot.re), 0.5 * (top.im + bot.im)}
             : cpx<double>{0.5 * (top.re - bot.re), 0.5 * (top.im - bot.im)};
    helm_down(g, f, xw, nc, nlines, be, p, l);
    double SPt, SPb;
    cpx<double> SQt, SQb;
    helm_up1(f, xw, nc, nlines, p, l, ntop, nbot, SPt, SQt, SPb, SQb);
    helm_up2(f, xw, nc, nlines, p, l, cpx<double>{(s.re - SQt.re) / SPt, (s.im - SQt.im) / SPt});
    return;
  }
  // different conditions at the two walls: both parities, then
  //   SPt0 a_0 + SPt1 a_1 = top - SQt0 - SQt1,  SPb0 a_0 + SPb1 a_1 = bot - SQb0 - SQb1
  double SPt[2], SPb[2];
  cpx<double> SQt[2], SQb[2];
  for (int q = 0; q < 2; ++q) {
    helm_down(g, f, xw, nc, nlines, be, q, l);
    helm_up1(f, xw, nc, nlines, q, l, ntop, nbot, SPt[q], SQt[q], SPb[q], SQb[q]);
  }
  const cpx<double> rt = {top.re - SQt[0].re - SQt[1].re, top.im - SQt[0].im - SQt[1].im};
  const cpx<double> rb = {bot.re - SQb[0].re - SQb[1].re, bot.im - SQb[0].im - SQb[1].im};
  const double det = SPt[0] * SPb[1] - SPt[1] * SPb[0];
  const cpx<double> a0 = {(rt.re * SPb[1] - SPt[1] * rb.re) / det, (rt.im * SPb[1] - SPt[1] * rb.im) / det};
  const cpx<double> a1 = {(SPt[0] * rb.re - SPb[0] * rt.re) / det, (SPt[0] * rb.im - SPb[0] * rt.im) / det};
  helm_up2(f, xw, nc, nlines, 0, l, a0);
  helm_up2(f, xw, nc, nlines, 1, l, a1);
}

__global__ void k_helm(const cpx<double>* __restrict__ g, cpx<double>* __restrict__ f, double* __restrict__ xw,
                       int nc, long long nlines, const double* __restrict__ beta_line, double beta_add,
                       const double* __restrict__ kx, const double* __restrict__ ky, int neumann,
                       const cpx<double>* __restrict__ bcv, cpx<double> top_c, cpx<double> bot_c) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 2 * nlines) return;
  helm_line(g, f, xw, nc, nlines, beta_line, beta_add, kx, ky, neumann ? 3 : 0, bcv, top_c, bot_c, id);
}

// Several independent problems in one launch (blockIdx.y selects the problem):
// each thread's elimination is a sequential chain, so more chains per launch
// hide more of their memory latency.
__global__ void k_helm_batch(HelmBatch b, int nc) {
  const HelmProblem& P = b.p[blockIdx.y];
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 2 * P.nlines) return;
  helm_line(P.g, P.f, P.xw, nc, P.nlines, nullptr, P.beta_add, P.kx, P.ky, P.bc, nullptr, P.top_c, P.bot_c, id);
}

// The same problems with the elimination held on chip: one workgroup of 64
// lines per (problem, parity) (blockIdx.z = parity, uniform in the
// workgroup), X_i of each chain in registers and Y_i in LDS, so that HBM sees
// only the right-hand side read and the solution written (32 bytes per
// coefficient instead of 104 through the scratch chains).  The loops over i
// are unrolled for the compile-time NC (i > m is skipped uniformly), and the
// tau-row coefficients come from the compile-time table kTauQ, which leaves one
// FP64 division per step of the recurrence.  The chain's right-hand side entries are first
// copied into the LDS rows by 16-byte global_load_lds copies, all in flight at
// once: each chain is one thread's sequential recurrence and a workgroup is
// one wavefront, so loads issued inside the recurrence would leave their
// latency exposed.  Same condition at both walls only (bc 0 or 3); the
// arithmetic is that of helm_line, in the same order.  With P.wh the w
// problem's influence correction follows in the second upward sweep
// (HelmProblem).
// MODE 2 stores the elimination factors of each chain instead of solving
// (see k_helm_pieces): fac [2 parities][NC/2 + 1][nlines] pairs of doubles,
// row i >= 1 (X_i, 1 / (B_i + C_i X_{i+1})), row 0 (sum w_n P_n, sum n^2 P_n).
template <int NC, int MODE>
__device__ __forceinline__ void helm_reg_chain(const HelmProblem& P, cpx<double> (*Ys)[64], int tid, long long l,
                                               int p, double* fac_out = nullptr) {
  constexpr int MM = NC / 2;                 // longest chain: parity 0, i = 0..MM
  const int m = (NC - p) / 2;
  const long long nl = P.nlines;
  const cpx<double>* __restrict__ g = (MODE == 2) ? nullptr : P.g;
  if (g) {
    // entries n = p + 2 i <= NC - 2 of this parity into row i (lane tid's
    // 16 bytes at &Ys[i][tid]); lanes past the last line copy nothing
    if (l < nl) {
#pragma unroll
      for (int i = 0; i <= MM; ++i) {
        if (i <= m && p + 2 * i <= NC - 2)
          __builtin_amdgcn_global_load_lds(
              (const __attribute__((address_space(1))) void*)(g + (long long)(p + 2 * i) * nl + l),
              (__attribute__((address_space(3))) void*)(&Ys[i][0]), 16, 0, 0);
      }
    }
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x0F70);      // vmcnt(0): the copies have landed in LDS
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
  }
  if (l >= nl) return;                       // no barrier below: each chain is one thread's
  const bool neu = P.bc == 3;
  double be = P.beta_add;
  if (P.kx) be += P.kx[l] * P.kx[l] + P.ky[l] * P.ky[l];
  const cpx<double> top = P.top_c, bot = P.bot_c;
  const bool plus = (p == 0) != neu;
  const cpx<double> s = plus ? cpx<double>{0.5 * (top.re + bot.re), 0.5 * (top.im + bot.im)}
                             : cpx<double>{0.5 * (top.re - bot.re), 0.5 * (top.im - bot.im)};
  const long long frow = (long long)p * (MM + 1);   // factor row i of this chain at ((frow + i) nl + l) 2
  // entry n of g (zero outside the tau rows); row (n - p) / 2 of Ys until the
  // downward sweep overwrites it with Y (after its last use: the sweep keeps
  // the three entries it needs in registers)
  auto G = [&](int n) -> cpx<double> {
    if (!g || n > NC - 2 || n < 0) return cpx<double>{0.0, 0.0};
    return Ys[(n - p) >> 1][tid];
  };
  // downward sweep: a_i = X_i a_{i-1} + Y_i
  double X[MM + 1];
  double Xn = 0.0;
  cpx<double> Yn = {0.0, 0.0};
  cpx<double> gm = G(p + 2 * m - 2), g0 = G(p + 2 * m), g2 = G(p + 2 * m + 2);
#pragma unroll
  for (int i = MM; i >= 1; --i) {
    if (i > m) continue;                     // uniform: the odd chain is one shorter
    const int n = p + 2 * i;
    const double cm2 = (n - 2 == 0) ? 2.0 : 1.0;
    const double en = (n <= NC - 2) ? 1.0 : 0.0;
    const double en2 = (n + 2 <= NC - 2) ? 1.0 : 0.0;
    const double q1 = kTauQ.q[0][n], q2 = kTauQ.q[1][n], q3 = kTauQ.q[2][n];
    const double A = cm2 * be * q1;
    const double B = -(1.0 + en * be * q2);
    const double C = en2 * be * q3;
    const cpx<double> R = {-cm2 * gm.re * q1 + en * g0.re * q2 - en2 * g2.re * q3,
                           -cm2 * gm.im * q1 + en * g0.im * q2 - en2 * g2.im * q3};
    const double den = 1.0 / (B + C * Xn);
    const double Xv = -A * den;
    if constexpr (MODE == 2) {
      fac_out[((frow + i) * nl + l) * 2] = Xv;
      fac_out[((frow + i) * nl + l) * 2 + 1] = den;
    } else {
      const cpx<double> Y = {(R.re - C * Yn.re) * den, (R.im - C * Yn.im) * den};
      g2 = g0;
      g0 = gm;
      gm = G(n - 4);
      Ys[i][tid] = Y;
      Yn = Y;
    }
    X[i] = Xv;
    Xn = Xv;
  }
  // upward sweep 1: a_i = P_i a_0 + Q_i and the boundary row of this parity;
  // with the influence correction also sum n^2 P_i and sum n^2 Q_i
  const bool infl = P.wh != nullptr;
  double Pc = 1.0, SP = 0.0, SPn = 0.0;
  cpx<double> Qv = {0.0, 0.0}, SQ = {0.0, 0.0}, SQn = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i <= MM; ++i) {
    if (i > m) continue;
    const int n = p + 2 * i;
    if constexpr (MODE == 2) {
      if (i > 0) Pc = X[i] * Pc;
      const double n2 = double(n) * double(n);
      SP += (neu ? n2 : 1.0) * Pc;
      SPn += n2 * Pc;
    } else {
      if (i > 0) {
        const cpx<double> Y = Ys[i][tid];
        Pc = X[i] * Pc;
        Qv = cpx<double>{X[i] * Qv.re + Y.re, X[i] * Qv.im + Y.im};
      }
      const double n2 = double(n) * double(n);
      const double w = neu ? n2 : 1.0;
      SP += w * Pc;
      SQ.re += w * Qv.re;
      SQ.im += w * Qv.im;
      if (infl) {
        SPn += n2 * Pc;
        SQn.re += n2 * Qv.re;
        SQn.im += n2 * Qv.im;
      }
    }
  }
  if constexpr (MODE == 2) {
    fac_out[(frow * nl + l) * 2] = SP;
    fac_out[(frow * nl + l) * 2 + 1] = SPn;
    return;
  }
  // a_0, the influence coefficient, then upward sweep 2
  cpx<double> a = {(s.re - SQ.re) / SP, (s.im - SQ.im) / SP};
  cpx<double>* __restrict__ f = P.f;
  cpx<double> c = {0.0, 0.0};
  if (infl) {
    if (P.kx[l] == 0.0 && P.ky[l] == 0.0) {  // no wall-normal velocity on the mean line
#pragma unroll
      for (int i = 0; i <= MM; ++i)
        if (i <= m) f[(long long)(p + 2 * i) * nl + l] = cpx<double>{0.0, 0.0};
      return;
    }
    // sum n^2 (a_n + c wh_n) = 0 with sum n^2 a_n = a_0 SPn + SQn
    const double r = -1.0 / P.mh[(long long)p * nl + l];
    c = cpx<double>{r * (a.re * SPn + SQn.re), r * (a.im * SPn + SQn.im)};
  }
  const double* __restrict__ wh = P.wh;
  auto put = [&](int n, cpx<double> v) {
    if (infl) {
      const double h = wh[(long long)n * nl + l];
      v = cpx<double>{v.re + c.re * h, v.im + c.im * h};
    }
    f[(long long)n * nl + l] = v;
  };
  put(p, a);
#pragma unroll
  for (int i = 1; i <= MM; ++i) {
    if (i > m) continue;
    const cpx<double> Y = Ys[i][tid];
    a = cpx<double>{X[i] * a.re + Y.re, X[i] * a.im + Y.im};
    put(p + 2 * i, a);
  }
}

template <int NC>
__global__ void __launch_bounds__(64) k_helm_batch_reg(HelmBatch b) {
  __shared__ cpx<double> Ys[NC / 2 + 1][64];
  const HelmProblem& P = b.p[blockIdx.y];
  const long long l = (long long)blockIdx.x * 64 + threadIdx.x;
  helm_reg_chain<NC, 0>(P, Ys, threadIdx.x, l, int(blockIdx.z));
}

// the factors of one problem (helm_reg_chain, MODE 2)
template <int NC>
__global__ void __launch_bounds__(64) k_helm_factors(HelmProblem P, double* fac) {
  const long long l = (long long)blockIdx.x * 64 + threadIdx.x;
  helm_reg_chain<NC, 2>(P, nullptr, threadIdx.x, l, int(blockIdx.z), fac);
}


// The tau solves of a batch whose problems carry their elimination factors
// (P.fac, from helm_reg_chain MODE 2: beta + k^2 and the wall conditions of
// a context do not change between steps).  With X_i and d_i = 1 / (B_i + C_i
// X_{i+1}) given, the three sweeps of a chain are first-order linear
// recurrences:
//   Y_i = d_i R_i - d_i C_i Y_{i+1}   (i = m .. 1, Y_{m+1} = 0)
//   Q_i = X_i Q_{i-1} + Y_i           (i = 1 .. m, Q_0 = 0), P_i = X_i P_{i-1}
//   a_i = P_i a_0 + Q_i,  a_0 = (s - sum w_i Q_i) / sum w_i P_i,
// so a chain of m + 1 terms is cut into 8 pieces of at most LEN terms: the
// wavefronts of a workgroup are the pieces of the chains of 64 lines of one
// parity (lane = line, so each term's load is 1 KB of consecutive lines, and
// a piece's term indices are the same in every lane), each lane forms its
// piece's affine maps and its part of the boundary-row sums, the pieces'
// maps pass through LDS, and each lane composes those of the pieces before
// its own.  The serial chain of the on-chip kernel (one lane per chain, its
// loads and divisions in sequence) becomes 8 short ones with every load
// issued at once.
template <int NC, int PAR>
__device__ __forceinline__ void helm_pieces_chain(const HelmProblem& P, double (*sh)[kHelmPieces][64], int pc,
                                                  int ln, long long l) {
  constexpr int MM = NC / 2;
  constexpr int LEN = (MM + 1 + kHelmPieces - 1) / kHelmPieces;
  constexpr int m = (NC - PAR) / 2;          // chain i = 0..m, n = PAR + 2 i
  const long long nl = P.nlines;
  const bool valid = l < nl;
  const long long lc = valid ? l : 0;         // lanes past the last line read line 0 and store nothing
  const int i0 = pc * LEN;                    // uniform in the wavefront
  const bool neu = P.bc == 3;
  double be = P.beta_add;
  if (P.kx) be += P.kx[lc] * P.kx[lc] + P.ky[lc] * P.ky[lc];
  const cpx<double> top = P.top_c, bot = P.bot_c;
  const bool plus = (PAR == 0) != neu;
  const cpx<double> s = plus ? cpx<double>{0.5 * (top.re + bot.re), 0.5 * (top.im + bot.im)}
                             : cpx<double>{0.5 * (top.re - bot.re), 0.5 * (top.im - bot.im)};
  const double* __restrict__ fac = P.fac + ((long long)PAR * (MM + 1) * nl + lc) * 2;   // row i at 2 i nl
  const cpx<double>* __restrict__ g = P.g;
  // the piece's loads, all issued before any use
  cpx<double> gv[LEN + 2];
  double Xv[LEN], dv[LEN];
#pragma unroll
  for (int k = 0; k < LEN + 2; ++k) {
    const int i = i0 - 1 + k, n = PAR + 2 * i;
    gv[k] = (g && i >= 0 && n <= NC - 2) ? g[(long long)n * nl + lc] : cpx<double>{0.0, 0.0};
  }
#pragma unroll
  for (int k = 0; k < LEN; ++k) {
    const int i = i0 + k;
    const bool in = i >= 1 && i <= m;
    Xv[k] = in ? fac[2 * (long long)i * nl] : 0.0;
    dv[k] = in ? fac[2 * (long long)i * nl + 1] : 0.0;
  }
  // 1. Y, downward: Y_i = ay_i Y_in + Y_i(local), Y_in = Y at the first term of the piece above
  double ay[LEN];
  cpx<double> Y[LEN];
  double A = 1.0;
  cpx<double> B = {0.0, 0.0};
#pragma unroll
  for (int k = LEN - 1; k >= 0; --k) {
    const int i = i0 + k, n = PAR + 2 * i;
    if (i >= 1 && i <= m) {
      const double cm2 = (n - 2 == 0) ? 2.0 : 1.0;
      const double en = (n <= NC - 2) ? 1.0 : 0.0;
      const double en2 = (n + 2 <= NC - 2) ? 1.0 : 0.0;
      const double q1 = kTauQ.q[0][n], q2 = kTauQ.q[1][n], q3 = kTauQ.q[2][n];
      const double C = en2 * be * q3;
      const cpx<double> gm = gv[k], g0 = gv[k + 1], g2 = gv[k + 2];
      const cpx<double> R = {-cm2 * gm.re * q1 + en * g0.re * q2 - en2 * g2.re * q3,
                             -cm2 * gm.im * q1 + en * g0.im * q2 - en2 * g2.im * q3};
      const double al = -C * dv[k];
      A = al * A;
      B = cpx<double>{dv[k] * R.re + al * B.re, dv[k] * R.im + al * B.im};
    }
    ay[k] = A;
    Y[k] = B;
  }
  sh[0][pc][ln] = A;
  sh[1][pc][ln] = B.re;
  sh[2][pc][ln] = B.im;
  __syncthreads();
  cpx<double> yin = {0.0, 0.0};               // the pieces above, applied to Y_{m+1} = 0
  for (int j = kHelmPieces - 1; j > pc; --j) {
    const double a = sh[0][j][ln];
    yin = cpx<double>{a * yin.re + sh[1][j][ln], a * yin.im + sh[2][j][ln]};
  }
#pragma unroll
  for (int k = 0; k < LEN; ++k) Y[k] = cpx<double>{ay[k] * yin.re + Y[k].re, ay[k] * yin.im + Y[k].im};
  // 2. Q, upward: the piece's map Q_out = aq Q_in + bq, its product of X, and
  // its parts of sum w_i Q_i and sum n^2 Q_i as linear functions of Q_in
  double aq = 1.0, pp = 1.0, swa = 0.0, sna = 0.0;
  cpx<double> bq = {0.0, 0.0}, swb = {0.0, 0.0}, snb = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < LEN; ++k) {
    const int i = i0 + k, n = PAR + 2 * i;
    if (i == 0) {
      aq = 0.0;                               // Q_0 = 0 whatever comes in
    } else if (i <= m) {
      const double n2 = double(n) * double(n);
      const double w = neu ? n2 : 1.0;
      aq = Xv[k] * aq;
      bq = cpx<double>{Xv[k] * bq.re + Y[k].re, Xv[k] * bq.im + Y[k].im};
      pp = Xv[k] * pp;
      swa += w * aq;
      swb = cpx<double>{swb.re + w * bq.re, swb.im + w * bq.im};
      sna += n2 * aq;
      snb = cpx<double>{snb.re + n2 * bq.re, snb.im + n2 * bq.im};
    }
  }
  __syncthreads();                            // the Y maps have been read
  const double mine[10] = {aq, bq.re, bq.im, pp, swa, swb.re, swb.im, sna, snb.re, snb.im};
#pragma unroll
  for (int v = 0; v < 10; ++v) sh[v][pc][ln] = mine[v];
  __syncthreads();
  // Q_in and the product of X of the pieces below, and the sums over all pieces
  cpx<double> qv = {0.0, 0.0}, qin = {0.0, 0.0}, SQ = {0.0, 0.0}, SQn = {0.0, 0.0};
  double pin = 1.0;
  for (int j = 0; j < kHelmPieces; ++j) {
    if (j == pc) {
      qin = qv;
    }
    SQ = cpx<double>{SQ.re + sh[4][j][ln] * qv.re + sh[5][j][ln], SQ.im + sh[4][j][ln] * qv.im + sh[6][j][ln]};
    SQn = cpx<double>{SQn.re + sh[7][j][ln] * qv.re + sh[8][j][ln], SQn.im + sh[7][j][ln] * qv.im + sh[9][j][ln]};
    const double a = sh[0][j][ln];
    qv = cpx<double>{a * qv.re + sh[1][j][ln], a * qv.im + sh[2][j][ln]};
    if (j < pc) pin *= sh[3][j][ln];
  }
  // 3. a_0 and the influence coefficient
  const double SP = fac[0], SPn = fac[1];
  const cpx<double> a0 = {(s.re - SQ.re) / SP, (s.im - SQ.im) / SP};
  const bool infl = P.wh != nullptr;
  cpx<double>* __restrict__ f = P.f;
  cpx<double> c = {0.0, 0.0};
  bool zero = false;
  if (infl) {
    if (P.kx[lc] == 0.0 && P.ky[lc] == 0.0) {
      zero = true;                            // no wall-normal velocity on the mean line
    } else {
      const double r = -1.0 / P.mh[(long long)PAR * nl + lc];
      c = cpx<double>{r * (a0.re * SPn + SQn.re), r * (a0.im * SPn + SQn.im)};
    }
  }
  // 4. the piece's coefficients a_i = P_i a_0 + Q_i
  if (!valid) return;
  cpx<double> q = qin;
  double pr = pin;
#pragma unroll
  for (int k = 0; k < LEN; ++k) {
    const int i = i0 + k, n = PAR + 2 * i;
    if (i > m) continue;
    if (i == 0) {
      q = cpx<double>{0.0, 0.0};
      pr = 1.0;
    } else {
      q = cpx<double>{Xv[k] * q.re + Y[k].re, Xv[k] * q.im + Y[k].im};
      pr = Xv[k] * pr;
    }
    cpx<double> v = {pr * a0.re + q.re, pr * a0.im + q.im};
    if (infl) {
      const double h = P.wh[(long long)n * nl + l];
      v = zero ? cpx<double>{0.0, 0.0} : cpx<double>{v.re + c.re * h, v.im + c.im * h};
    }
    f[(long long)n * nl + l] = v;
  }
}

template <int NC>
__global__ void __launch_bounds__(64 * kHelmPieces) k_helm_pieces(HelmBatch bt) {
  __shared__ double sh[10][kHelmPieces][64];
  const HelmProblem& P = bt.p[blockIdx.y];
  const int pc = int(threadIdx.x >> 6), ln = int(threadIdx.x & 63);
  const long long l = (long long)blockIdx.x * 64 + ln;
  if ((long long)blockIdx.x * 64 >= P.nlines) return;   // the whole workgroup (problems of fewer lines)
  if (blockIdx.z == 0) helm_pieces_chain<NC, 0>(P, sh, pc, ln, l);
  else helm_pieces_chain<NC, 1>(P, sh, pc, ln, l);
}

// wh_n = (w_t + w_b)_n (even n) or (w_t - w_b)_n (odd n): the homogeneous
// solutions with psi = 1 at both walls (even) and psi = +-1 (odd); mh[p][l] =
// sum over the parity of n^2 wh_n (w'(+1) = +-w'(-1) splits by parity)
__global__ void k_influence_parity_pre(const cpx<double>* __restrict__ wt, const cpx<double>* __restrict__ wb, int nc,
                                       long long nlines, double* __restrict__ wh, double* __restrict__ mh) {
  const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlines) return;
  double s[2] = {0.0, 0.0};
  for (int n = 0; n <= nc; ++n) {
    const long long o = (long long)n * nlines + l;
    const double h = (n & 1) ? wt[o].re - wb[o].re : wt[o].re + wb[o].re;
    wh[o] = h;
    s[n & 1] += double(n) * double(n) * h;
  }
  mh[l] = s[0];
  mh[nlines + l] = s[1];
}

// w = w_p + c_t w_t + c_b w_b with (c_t, c_b) making w'(+1) = w'(-1) = 0;
// w = 0 where kx = ky = 0.  Written over w_p.
__global__ void k_influence(cpx<double>* __restrict__ wp, const cpx<double>* __restrict__ wt,
                            const cpx<double>* __restrict__ wb, int nc, long long nlines,
                            const double* __restrict__ kx, const double* __restrict__ ky) {
  const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlines) return;
  const bool mean = (kx[l] == 0.0 && ky[l] == 0.0);
  cpx<double> dpt = {0, 0}, dpb = {0, 0};
  double dtt = 0, dtb = 0, dbt = 0, dbb = 0;
#pragma unroll 4
  for (int n = 0; n <= nc; ++n) {
    const double w2 = double(n) * double(n);
    const double sg = (n & 1) ? w2 : -w2;  // (-1)^(n+1) n^2
    const long long o = (long long)n * nlines + l;
    const cpx<double> a = wp[o];
    dpt.re += w2 * a.re; dpt.im += w2 * a.im;
    dpb.re += sg * a.re; dpb.im += sg * a.im;
    dtt += w2 * wt[o].re; dtb += sg * wt[o].re;
    dbt += w2 * wb[o].re; dbb += sg * wb[o].re;
  }
  // [dtt dbt; dtb dbb] (c_t, c_b) = -(dpt, dpb)
  const double det = dtt * dbb - dbt * dtb;
  const cpx<double> ct = {(-dpt.re * dbb + dbt * dpb.re) / det, (-dpt.im * dbb + dbt * dpb.im) / det};
  const cpx<double> cb = {(-dtt * dpb.re + dtb * dpt.re) / det, (-dtt * dpb.im + dtb * dpt.im) / det};
#pragma unroll 4
  for (int n = 0; n <= nc; ++n) {
    const long long o = (long long)n * nlines + l;
    cpx<double> w = {0.0, 0.0};
    if (!mean) {
      const cpx<double> a = wp[o];
      const double t = wt[o].re, b = wb[o].re;
      w = cpx<double>{a.re + ct.re * t + cb.re * b, a.im + ct.im * t + cb.im * b};
    }
    wp[o] = w;
  }
}

// The influence matrix of the clamped w problem when the homogeneous solutions
// w_t, w_b are fixed (they depend only on k^2 and beta): M = (w_t'(+1),
// w_t'(-1), w_b'(+1), w_b'(-1)) per line, M [4][nlines].
__global__ void k_influence_pre(const cpx<double>* __restrict__ wt, const cpx<double>* __restrict__ wb, int nc,
                                long long nlines, double* __restrict__ M, int free_slip) {
  const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlines) return;
  double dtt = 0, dtb = 0, dbt = 0, dbb = 0;
  for (int n = 0; n <= nc; ++n) {
    const double w2 = double(n) * double(n);
    const double sg = (n & 1) ? w2 : -w2;  // (-1)^(n+1) n^2
    const long long o = (long long)n * nlines + l;
    dtt += w2 * wt[o].re;
    dtb += sg * wt[o].re;
    dbt += w2 * wb[o].re;
    dbb += sg * wb[o].re;
  }
  if (free_slip & 1) {   // top row: c_t = 0
    dtt = 1.0;
    dbt = 0.0;
  }
  if (free_slip & 2) {   // bottom row: c_b = 0
    dtb = 0.0;
    dbb = 1.0;
  }
  M[l] = dtt;
  M[nlines + l] = dtb;
  M[2 * nlines + l] = dbt;
  M[3 * nlines + l] = dbb;
}

// w = w_p + c_t w_t + c_b w_b with M from k_influence_pre (written over w_p;
// w = 0 where kx = ky = 0).  64 lines per workgroup, 4 threads per line share
// the sums over n through LDS.
__global__ void __launch_bounds__(256) k_influence_apply(cpx<double>* __restrict__ wp,
                                                         const cpx<double>* __restrict__ wt,
                                                         const cpx<double>* __restrict__ wb,
                                                         const double* __restrict__ M, int nc, long long nlines,
                                                         const double* __restrict__ kx,
                                                         const double* __restrict__ ky, int free_slip) {
  __shared__ cpx<double> part[2][4][64];
  const int li = threadIdx.x % 64, ch = threadIdx.x / 64;
  const long long l = (long long)blockIdx.x * 64 + li;
  const bool ok = l < nlines;
  cpx<double> dpt = {0.0, 0.0}, dpb = {0.0, 0.0};
  if (ok) {
#pragma unroll 4
    for (int n = ch; n <= nc; n += 4) {
      const double w2 = double(n) * double(n);
      const double sg = (n & 1) ? w2 : -w2;
      const cpx<double> a = wp[(long long)n * nlines + l];
      dpt.re += w2 * a.re; dpt.im += w2 * a.im;
      dpb.re += sg * a.re; dpb.im += sg * a.im;
    }
  }
  part[0][ch][li] = dpt;
  part[1][ch][li] = dpb;
  __syncthreads();
  if (!ok) return;
  dpt = cpx<double>{0.0, 0.0};
  dpb = cpx<double>{0.0, 0.0};
  for (int c = 0; c < 4; ++c) {
    dpt = cadd(dpt, part[0][c][li]);
    dpb = cadd(dpb, part[1][c][li]);
  }
  if (free_slip & 1) dpt = cpx<double>{0.0, 0.0};
  if (free_slip & 2) dpb = cpx<double>{0.0, 0.0};
  const double dtt = M[l], dtb = M[nlines + l], dbt = M[2 * nlines + l], dbb = M[3 * nlines + l];
  const bool mean = (kx[l] == 0.0 && ky[l] == 0.0);
  const double det = dtt * dbb - dbt * dtb;
  const cpx<double> ct = {(-dpt.re * dbb + dbt * dpb.re) / det, (-dpt.im * dbb + dbt * dpb.im) / det};
  const cpx<double> cb = {(-dtt * dpb.re + dtb * dpt.re) / det, (-dtt * dpb.im + dtb * dpt.im) / det};
#pragma unroll 4
  for (int n = ch; n <= nc; n += 4) {
    const long long o = (long long)n * nlines + l;
    cpx<double> w = {0.0, 0.0};
    if (!mean) {
      const cpx<double> a = wp[o];
      const double t = wt[o].re, b = wb[o].re;
      w = cpx<double>{a.re + ct.re * t + cb.re * b, a.im + ct.im * t + cb.im * b};
    }
    wp[o] = w;
  }
}

// u = i (kx w' + ky omega) / k^2, v = i (ky w' - kx omega) / k^2 (0 where k = 0).
__global__ void k_uv(const cpx<double>* __restrict__ om, const cpx<double>* __restrict__ dw, cpx<double>* __restrict__ u,
                     cpx<double>* __restrict__ v, int nc, long long nlines, const double* __restrict__ kx,
                     const double* __restrict__ ky) {
  const long long tot = (long long)(nc + 1) * nlines;
  for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < tot;
       id += (long long)gridDim.x * blockDim.x) {
    const long long l = id % nlines;
    const double a = kx[l], b = ky[l];
    const double k2 = a * a + b * b;
    cpx<double> uu = {0.0, 0.0}, vv = {0.0, 0.0};
    if (k2 != 0.0) {
      const double ik = 1.0 / k2;
      const cpx<double> o = om[id], d = dw[id];
      const cpx<double> su = {a * d.re + b * o.re, a * d.im + b * o.im};
      const cpx<double> sv = {b * d.re - a * o.re, b * d.im - a * o.im};
      uu = cpx<double>{-su.im * ik, su.re * ik};
      vv = cpx<double>{-sv.im * ik, sv.re * ik};
    }
    u[id] = uu;
    v[id] = vv;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define PSMS_FOR_EACH_2NC(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(512)

bool supported_nc(int nc) {
  switch (2 * nc) {
#define PSMS_CASE(NN) case NN:
    PSMS_FOR_EACH_2NC(PSMS_CASE)
#undef PSMS_CASE
    return true;
    default:
      return false;
  }
}

namespace {
template <typename T, int N, class Src>
hipError_t dct_n(const Src& in, cpx<T>* out, long long nlines, int dir, long long fstride, int nfield,
                 const cpx<T>* tw, cpx<double>* out64, int kz, hipStream_t st) {
  // FP64 lines take the nc-point route (measured at nc = 128 on the channel
  // workload: 56.7 us per launch against 72.1 us for the 2 nc-point FFT); FP32
  // lines keep the 2 nc-point even extension (40.3 us against 43.4 us: the
  // FP32 transform is cheaper than the nc-point route's extra loads and
  // running-sum passes through LDS)
  if constexpr (N >= 16 && sizeof(T) == 8) {   // nc = N / 2 >= 8
    using G = CTile<Plan<N / 2>>;
    const dim3 grid(unsigned((nlines + G::L - 1) / G::L), unsigned(nfield));
    k_dct_half<T, N / 2, Src><<<grid, unsigned(G::L * G::TT), 0, st>>>(in, out, nlines, dir, fstride, tw, out64, kz);
  } else {
    using G = CTile<Plan<N>>;
    const dim3 grid(unsigned((nlines + G::L - 1) / G::L), unsigned(nfield));
    k_dct<T, N, Src><<<grid, unsigned(G::L * G::TT), 0, st>>>(in, out, nlines, dir, fstride, tw, out64, kz);
  }
  return hipGetLastError();
}
unsigned blocks(long long n, int bs) {
  long long b = (n + bs - 1) / bs;
  return unsigned(b < 1 ? 1 : b);
}
}  // namespace

template <typename T>
hipError_t launch_dct(int nc, const cpx<T>* in, cpx<T>* out, long long nlines, int dir, hipStream_t st) {
  return launch_dct_fields<T>(nc, in, out, nlines, 0, 1, nullptr, dir, st);
}

template <typename T>
hipError_t launch_dct_fields(int nc, const cpx<T>* in, cpx<T>* out, long long nlines, long long fstride, int nfield,
                             const cpx<T>* tw, int dir, hipStream_t st, cpx<double>* out64, int kz) {
  if (nfield < 1 || nlines == 0) return hipSuccess;
  if (out64 && dir < 0) return hipErrorInvalidValue;
  const ArraySrc<T> src{in, fstride, nlines};
  switch (2 * nc) {
#define PSMS_CASE(NN) case NN: return dct_n<T, NN>(src, out, nlines, dir, fstride, nfield, tw, out64, kz, st);
    PSMS_FOR_EACH_2NC(PSMS_CASE)
#undef PSMS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_dct_chfields(int nc, const ChanFieldSrc& fs, cpx<T>* out, long long fstride, const cpx<T>* tw,
                               hipStream_t st) {
  if (fs.nlines == 0) return hipSuccess;
  const ChanFieldSrcT<T> src{fs};
  switch (2 * nc) {
#define PSMS_CASE(NN) case NN: return dct_n<T, NN>(src, out, fs.nlines, -1, fstride, 6, tw, nullptr, 0, st);
    PSMS_FOR_EACH_2NC(PSMS_CASE)
#undef PSMS_CASE
  }
  return hipErrorInvalidValue;
}
template hipError_t launch_dct_chfields<float>(int, const ChanFieldSrc&, cpx<float>*, long long, const cpx<float>*,
                                               hipStream_t);
template hipError_t launch_dct_chfields<double>(int, const ChanFieldSrc&, cpx<double>*, long long,
                                                const cpx<double>*, hipStream_t);

hipError_t launch_cheb_batch(const ChebBatch& b, int nc, long long nlines, const double* kx, const double* ky,
                             int lapmask, hipStream_t st) {
  if (b.n < 0 || b.n > kChebBatchMax || nlines < 0 || nc < 1) return hipErrorInvalidValue;
  for (int j = 0; j < b.n; ++j)
    if (b.nl[j] < 0 || b.nl[j] > nlines) return hipErrorInvalidValue;
  if (b.n == 0 || nlines == 0) return hipSuccess;
  // 8 pieces per chain (8 lines a wavefront) up to 9 terms a piece, else 16
  // pieces (4 lines a wavefront), which keeps the longest chains (nc = 256) at
  // 9 terms a piece and off the register limit
  const int need = (nc / 2 + 1 + 7) / 8;
  const int pcs = need <= 9 ? 8 : 16;
  const dim3 grid(blocks(2 * ((nlines + 64 / pcs - 1) / (64 / pcs)) * 64, 256), unsigned(b.n));
#define PSMS_SEG(LEN, PCS) \
  if (pcs == PCS && (nc / 2 + PCS) / PCS <= LEN) { \
    k_cheb_seg<LEN, PCS><<<grid, 256, 0, st>>>(b, nc, nlines, kx, ky, lapmask); \
    return hipGetLastError(); \
  }
  PSMS_SEG(1, 8) PSMS_SEG(2, 8) PSMS_SEG(3, 8) PSMS_SEG(5, 8) PSMS_SEG(9, 8) PSMS_SEG(9, 16)
#undef PSMS_SEG
  return hipErrorInvalidValue;   // nc > 287
}

hipError_t launch_chebd_q(const ChebQ& in, int nc, long long nlines, const double* kx, const double* ky,
                          cpx<double>* out, hipStream_t st) {
  if (nlines < 0 || nc < 1) return hipErrorInvalidValue;
  if (nlines == 0) return hipSuccess;
  const int need = (nc / 2 + 1 + 7) / 8;
  const int pcs = need <= 9 ? 8 : 16;   // as in launch_cheb_batch
  const dim3 grid(blocks(2 * ((nlines + 64 / pcs - 1) / (64 / pcs)) * 64, 256));
#define PSMS_SEG(LEN, PCS) \
  if (pcs == PCS && (nc / 2 + PCS) / PCS <= LEN) { \
    k_cheb_seg_q<LEN, PCS><<<grid, 256, 0, st>>>(in, nc, nlines, kx, ky, out); \
    return hipGetLastError(); \
  }
  PSMS_SEG(1, 8) PSMS_SEG(2, 8) PSMS_SEG(3, 8) PSMS_SEG(5, 8) PSMS_SEG(9, 8) PSMS_SEG(9, 16)
#undef PSMS_SEG
  return hipErrorInvalidValue;
}

hipError_t launch_chebd(const cpx<double>* a, cpx<double>* d, int nc, long long nlines, hipStream_t st) {
  ChebBatch b{};
  b.n = 1;
  b.in[0] = a;
  b.out[0] = d;
  return launch_cheb_batch(b, nc, nlines, nullptr, nullptr, 0, st);
}

hipError_t launch_cheb_lap(const cpx<double>* a, cpx<double>* out, int nc, long long nlines, const double* kx,
                           const double* ky, hipStream_t st) {
  ChebBatch b{};
  b.n = 1;
  b.in[0] = a;
  b.out[0] = out;
  return launch_cheb_batch(b, nc, nlines, kx, ky, 1, st);
}

hipError_t launch_helm(const cpx<double>* g, cpx<double>* f, double* xw, int nc, long long nlines,
                       const double* beta_line, double beta_add, const double* kx, const double* ky, int neumann,
                       const cpx<double>* bcv, cpx<double> top_c, cpx<double> bot_c, hipStream_t st) {
  k_helm<<<blocks(2 * nlines, 64), 64, 0, st>>>(g, f, xw, nc, nlines, beta_line, beta_add, kx, ky, neumann, bcv,
                                                   top_c, bot_c);
  return hipGetLastError();
}

hipError_t launch_helm_batch(const HelmBatch& b, int nc, hipStream_t st) {
  if (b.np < 0 || b.np > kHelmBatchMax) return hipErrorInvalidValue;
  long long most = 0;
  bool same_walls = true;
  for (int i = 0; i < b.np; ++i) {
    if (b.p[i].nlines < 0) return hipErrorInvalidValue;
    most = most > b.p[i].nlines ? most : b.p[i].nlines;
    same_walls = same_walls && (b.p[i].bc == 0 || b.p[i].bc == 3);
  }
  if (b.np == 0 || most == 0) return hipSuccess;
  const bool reg = same_walls && helm_fuses_influence(nc);
  for (int i = 0; i < b.np; ++i)
    if (b.p[i].wh && (!reg || !b.p[i].kx || !b.p[i].mh)) return hipErrorInvalidValue;
  // factors: given for every problem of the batch or for none
  int nfac = 0;
  for (int i = 0; i < b.np; ++i) nfac += b.p[i].fac ? 1 : 0;
  if (nfac && (nfac != b.np || !reg)) return hipErrorInvalidValue;
  if (nfac) {
    const dim3 grid(blocks(most, 64), unsigned(b.np), 2);
    switch (nc) {
#define PSMS_CASE(NC) \
  case NC: k_helm_pieces<NC><<<grid, 64 * kHelmPieces, 0, st>>>(b); return hipGetLastError();
      PSMS_CASE(4) PSMS_CASE(6) PSMS_CASE(8) PSMS_CASE(12) PSMS_CASE(16) PSMS_CASE(24) PSMS_CASE(32)
      PSMS_CASE(48) PSMS_CASE(64) PSMS_CASE(96) PSMS_CASE(128)
#undef PSMS_CASE
      default: return hipErrorInvalidValue;
    }
  }
  if (same_walls) {
    const dim3 grid(blocks(most, 64), unsigned(b.np), 2);
    switch (nc) {
#define PSMS_CASE(NC) \
  case NC: k_helm_batch_reg<NC><<<grid, 64, 0, st>>>(b); return hipGetLastError();
      PSMS_CASE(4) PSMS_CASE(6) PSMS_CASE(8) PSMS_CASE(12) PSMS_CASE(16) PSMS_CASE(24) PSMS_CASE(32)
      PSMS_CASE(48) PSMS_CASE(64) PSMS_CASE(96) PSMS_CASE(128)
#undef PSMS_CASE
      default: break;   // longer chains (nc = 256) through the scratch path
    }
  }
  k_helm_batch<<<dim3(blocks(2 * most, 64), unsigned(b.np)), 64, 0, st>>>(b, nc);
  return hipGetLastError();
}

hipError_t launch_helm_factors(const HelmProblem& P, int nc, double* fac, hipStream_t st) {
  if (!fac || P.nlines < 0 || !(P.bc == 0 || P.bc == 3) || !helm_fuses_influence(nc)) return hipErrorInvalidValue;
  if (P.nlines == 0) return hipSuccess;
  const dim3 grid(blocks(P.nlines, 64), 1, 2);
  switch (nc) {
#define PSMS_CASE(NC) \
  case NC: k_helm_factors<NC><<<grid, 64, 0, st>>>(P, fac); return hipGetLastError();
    PSMS_CASE(4) PSMS_CASE(6) PSMS_CASE(8) PSMS_CASE(12) PSMS_CASE(16) PSMS_CASE(24) PSMS_CASE(32)
    PSMS_CASE(48) PSMS_CASE(64) PSMS_CASE(96) PSMS_CASE(128)
#undef PSMS_CASE
    default: break;
  }
  return hipErrorInvalidValue;
}

size_t helm_factor_doubles(int nc, long long nlines) { return size_t(2) * size_t(nc / 2 + 1) * size_t(nlines) * 2; }

bool helm_fuses_influence(int nc) {
  switch (nc) {
    case 4: case 6: case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96: case 128: return true;
    default: return false;
  }
}

hipError_t launch_influence_parity_pre(const cpx<double>* wt, const cpx<double>* wb, int nc, long long nlines,
                                       double* wh, double* mh, hipStream_t st) {
  if (nlines <= 0) return hipSuccess;
  k_influence_parity_pre<<<blocks(nlines, 64), 64, 0, st>>>(wt, wb, nc, nlines, wh, mh);
  return hipGetLastError();
}

hipError_t launch_influence(cpx<double>* wp, const cpx<double>* wt, const cpx<double>* wb, int nc, long long nlines,
                            const double* kx, const double* ky, hipStream_t st) {
  k_influence<<<blocks(nlines, 64), 64, 0, st>>>(wp, wt, wb, nc, nlines, kx, ky);
  return hipGetLastError();
}

hipError_t launch_influence_pre(const cpx<double>* wt, const cpx<double>* wb, int nc, long long nlines, double* M,
                                int free_slip, hipStream_t st) {
  k_influence_pre<<<blocks(nlines, 64), 64, 0, st>>>(wt, wb, nc, nlines, M, free_slip);
  return hipGetLastError();
}

hipError_t launch_influence_apply(cpx<double>* wp, const cpx<double>* wt, const cpx<double>* wb, const double* M,
                                  int nc, long long nlines, const double* kx, const double* ky, int free_slip,
                                  hipStream_t st) {
  k_influence_apply<<<blocks(nlines, 64), 256, 0, st>>>(wp, wt, wb, M, nc, nlines, kx, ky, free_slip);
  return hipGetLastError();
}

hipError_t launch_uv(const cpx<double>* om, const cpx<double>* dw, cpx<double>* u, cpx<double>* v, int nc,
                     long long nlines, const double* kx, const double* ky, hipStream_t st) {
  long long b = ((long long)(nc + 1) * nlines + 255) / 256;
  if (b > 65536) b = 65536;
  k_uv<<<unsigned(b < 1 ? 1 : b), 256, 0, st>>>(om, dw, u, v, nc, nlines, kx, ky);
  return hipGetLastError();
}

template hipError_t launch_dct<double>(int, const cpx<double>*, cpx<double>*, long long, int, hipStream_t);
template hipError_t launch_dct_fields<double>(int, const cpx<double>*, cpx<double>*, long long, long long, int,
                                              const cpx<double>*, int, hipStream_t, cpx<double>*, int);
template hipError_t launch_dct_fields<float>(int, const cpx<float>*, cpx<float>*, long long, long long, int,
                                             const cpx<float>*, int, hipStream_t, cpx<double>*, int);
template hipError_t launch_dct<float>(int, const cpx<float>*, cpx<float>*, long long, int, hipStream_t);

}  // namespace psms
