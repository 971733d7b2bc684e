// Register/LDS FFT engine with compile-time length for gfx950.
//
// The transforms of Sec. 3.2.1 are batched 1-D FFTs along one axis.  Here a
// line of N points is transformed by TT = N/E threads that each own E complex
// values.  The algorithm is a Stockham autosort FFT whose stages run on
// registers; consecutive stages exchange data through LDS (ping-pong
// buffers, one barrier per exchange).  Two properties make fusion cheap:
//
//  * the first stage reads positions  t + TT*b + r*N/R_first  and the last
//    stage leaves positions            t + TT*b + r*N/R_last
//    in registers, so loads feed the first stage and stores drain the last
//    one directly;
//  * the inverse uses the radix sequence of the forward transform reversed, so
//    a thread's output positions after a forward FFT are its input positions
//    for the following inverse FFT and vice versa.  Pointwise work between two
//    transforms (the products, the spectral update) then needs no exchange.
//
// Radix plans: N = 2^m uses E = 4 (radix 4 stages, one radix-2 stage when m
// is odd); N = 3*2^m uses E = 6 (one radix-3 stage, radix-2 stages).
// Twiddles exp(-2 pi i m / N) come from a table computed in FP64 on the host.
#pragma once

#include <hip/hip_runtime.h>

namespace psms {

template <typename T>
struct cpx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// a * (S i)
template <int S, typename T>
__device__ __forceinline__ cpx<T> mul_si(cpx<T> a) {
  return (S > 0) ? cpx<T>{-a.im, a.re} : cpx<T>{a.im, -a.re};
}

// ---------------------------------------------------------------------------
// compile-time plans
// ---------------------------------------------------------------------------
template <int N>
struct Plan;
template <> struct Plan<8>   { static constexpr int E = 4, NST = 2; static constexpr int R[8] = {4, 2}; };
template <> struct Plan<16>  { static constexpr int E = 4, NST = 2; static constexpr int R[8] = {4, 4}; };
template <> struct Plan<32>  { static constexpr int E = 4, NST = 3; static constexpr int R[8] = {4, 4, 2}; };
template <> struct Plan<64>  { static constexpr int E = 4, NST = 3; static constexpr int R[8] = {4, 4, 4}; };
template <> struct Plan<128> { static constexpr int E = 4, NST = 4; static constexpr int R[8] = {4, 4, 4, 2}; };
template <> struct Plan<256> { static constexpr int E = 4, NST = 4; static constexpr int R[8] = {4, 4, 4, 4}; };
template <> struct Plan<12>  { static constexpr int E = 6, NST = 3; static constexpr int R[8] = {3, 2, 2}; };
template <> struct Plan<24>  { static constexpr int E = 6, NST = 4; static constexpr int R[8] = {3, 2, 2, 2}; };
template <> struct Plan<48>  { static constexpr int E = 6, NST = 5; static constexpr int R[8] = {3, 2, 2, 2, 2}; };
template <> struct Plan<96>  { static constexpr int E = 6, NST = 6; static constexpr int R[8] = {3, 2, 2, 2, 2, 2}; };
template <> struct Plan<192> { static constexpr int E = 6, NST = 7; static constexpr int R[8] = {3, 2, 2, 2, 2, 2, 2}; };

// Radix of stage s when running in direction S (S < 0: forward order,
// S > 0: reversed order).
template <int N, int S, int s>
__host__ __device__ constexpr int radix_at() {
  return (S < 0) ? Plan<N>::R[s] : Plan<N>::R[Plan<N>::NST - 1 - s];
}
// Radix of the first / last stage in direction S.
template <int N, int S>
__host__ __device__ constexpr int first_radix() { return radix_at<N, S, 0>(); }
template <int N, int S>
__host__ __device__ constexpr int last_radix() { return radix_at<N, S, Plan<N>::NST - 1>(); }

// Position of register slot (b, r) for a stage of radix R: t + TT*b + r*N/R.
template <int N, int R>
__device__ __forceinline__ int slot_pos(int t, int b, int r) {
  constexpr int TT = N / Plan<N>::E;
  return t + TT * b + r * (N / R);
}

// ---------------------------------------------------------------------------
// in-register DFTs, roots exp(S 2 pi i / R)
// ---------------------------------------------------------------------------
template <int R, int S, typename T>
__device__ __forceinline__ void dft(cpx<T>* v) {
  if constexpr (R == 2) {
    const cpx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    const T c1 = T(-0.5);
    const T c2 = T(S) * T(0.86602540378443864676372317075294);
    const cpx<T> s = cadd(v[1], v[2]);
    const cpx<T> d = csub(v[1], v[2]);
    const cpx<T> m = {v[0].re + c1 * s.re, v[0].im + c1 * s.im};
    const cpx<T> r = {-c2 * d.im, c2 * d.re};
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  } else {
    static_assert(R == 4, "radix");
    const cpx<T> t0 = cadd(v[0], v[2]);
    const cpx<T> t1 = csub(v[0], v[2]);
    const cpx<T> t2 = cadd(v[1], v[3]);
    const cpx<T> t3 = mul_si<S>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
}

// One Stockham stage on registers.  Input  v[b*R + r] = x[j_b + r N/R],
// output v[b*R + r] = y[d_b + r NS], j_b = t + TT b, k = j_b mod NS,
// d_b = (j_b / NS) NS R + k, with the twiddle exp(S 2 pi i r k / (NS R)).
template <typename T, int N, int R, int NS, int S>
__device__ __forceinline__ void stage_regs(cpx<T>* v, int t, const cpx<T>* tw) {
  constexpr int E = Plan<N>::E;
  constexpr int TT = N / E;
  constexpr int NB = E / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + TT * b;
    if constexpr (NS > 1) {
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cpx<T> w = tw[r * k * (N / (NS * R))];
        v[b * R + r] = (S < 0) ? cmul(v[b * R + r], w) : cmulc(v[b * R + r], w);
      }
    }
    dft<R, S>(&v[b * R]);
  }
}

// LDS index functors.  Strided tiles: element (pos, line) at pos*LP + line.
// Row tiles: element (line, pos) at line*LP + pos.
struct IdxPosMajor {
  int lp, line;
  __device__ __forceinline__ int operator()(int pos) const { return pos * lp + line; }
};
struct IdxLineMajor {
  int base;  // line * LP
  __device__ __forceinline__ int operator()(int pos) const { return base + pos; }
};

// Stages s .. NST-1 of a transform in direction S, starting from registers
// holding the input of stage s.  The exchange buffer alternates between b0 and
// b1 (selected by par); one barrier per exchange.  All threads of the block
// must call it.
template <typename T, int N, int S, int s, int NS, class Idx>
__device__ __forceinline__ void fft_stages(cpx<T>* v, cpx<T>* b0, cpx<T>* b1, int& par, int t, const Idx& idx,
                                           const cpx<T>* tw) {
  constexpr int R = radix_at<N, S, s>();
  stage_regs<T, N, R, NS, S>(v, t, tw);
  if constexpr (s + 1 < Plan<N>::NST) {
    constexpr int E = Plan<N>::E;
    constexpr int TT = N / E;
    constexpr int R2 = radix_at<N, S, s + 1>();
    cpx<T>* L = par ? b1 : b0;
    par ^= 1;
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
      const int j = t + TT * b;
      const int d = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) L[idx(d + r * NS)] = v[b * R + r];
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < E / R2; ++b) {
#pragma unroll
      for (int r = 0; r < R2; ++r) v[b * R2 + r] = L[idx(slot_pos<N, R2>(t, b, r))];
    }
    fft_stages<T, N, S, s + 1, NS * R>(v, b0, b1, par, t, idx, tw);
  }
}

// Whole transform.  On entry v[b*R + r] holds x at slot_pos<N, first_radix>;
// on exit it holds X at slot_pos<N, last_radix>.  S = -1 forward, +1 inverse
// (unnormalised).
template <typename T, int N, int S, class Idx>
__device__ __forceinline__ void fft_line(cpx<T>* v, cpx<T>* b0, cpx<T>* b1, int& par, int t, const Idx& idx,
                                         const cpx<T>* tw) {
  fft_stages<T, N, S, 0, 1>(v, b0, b1, par, t, idx, tw);
}

// Tiling of a batch of lines of length N: E values per thread, TT threads per
// line, L lines per workgroup of THREADS = 64 << V threads (V is the
// workgroup-size variant the autotuner chooses between; V = 2 is 256).
template <int N, int V = 2>
struct Tile {
  static constexpr int E = Plan<N>::E;
  static constexpr int TT = N / E;
  static constexpr int THREADS = 64 << V;
  static constexpr int L = (THREADS / TT) > 0 ? THREADS / TT : 1;
  static constexpr int K = (N - 1) / 3;
  static constexpr int C = 2 * K + 1;
  static constexpr int H = K + 1;
};

// XCD-aware tile index.  Workgroups are dealt round-robin to the 8 XCDs of
// the MI355X, each with its own L2; this bijection gives every XCD a
// contiguous range of tiles, so neighbouring tiles (which share cache lines
// of the strided-axis layouts) are served by the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  constexpr int X = 8;
  const int q = nb / X, r = nb % X;
  const int x = b % X, i = b / X;
  return x * q + (x < r ? x : r) + i;
}

// ---------------------------------------------------------------------------
// index maps of the retained band and of FFT order
// ---------------------------------------------------------------------------
// A band of `cnt` slots along an axis of length n stores wavenumbers 0..h and
// -h..-1 (h = (cnt-1)/2); cnt = n is the full FFT order.
__host__ __device__ __forceinline__ int full_pos(int i, int cnt, int n) {
  return (i <= (cnt - 1) / 2) ? i : i + (n - cnt);
}
__host__ __device__ __forceinline__ int band_slot(int p, int cnt, int n) {
  const int h = (cnt - 1) / 2;
  if (p <= h) return p;
  const int q = p - (n - cnt);
  return (q > h) ? q : -1;
}
// Signed wavenumber at FFT-order position p (numpy fftfreq convention).
__host__ __device__ __forceinline__ int signed_k(int p, int n) { return (p < (n + 1) / 2) ? p : p - n; }

}  // namespace psms
