// Batched 1-D complex FFT engine for gfx950, used by every transform stage.
//
// The transforms of Sec. 3.2.1 (batched Fourier transforms along one axis at a
// time) are written here as a Stockham autosort FFT executed by a workgroup on
// a tile of lines held in LDS.  A line of length n is processed by n/E
// threads; every thread owns E complex values per stage and performs E/R
// radix-R butterflies, R in {2, 3, 4, 8}.  E = 8 serves n = 2^m, E = 12
// serves n = 3 * 2^m.  The radix sequence is a runtime plan so that one
// kernel binary serves every supported length.
//
// LDS layout: element (pos, line) lives at buf[pos * lp + line].  Threads are
// mapped line-fastest, so the 64 lanes of a wavefront touch consecutive LDS
// words and, on strided axes, consecutive global addresses.
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
// a * (S i), S = +1 or -1
template <int S, typename T>
__device__ __forceinline__ cpx<T> mul_si(cpx<T> a) {
  return (S > 0) ? cpx<T>{-a.im, a.re} : cpx<T>{a.im, -a.re};
}

// Runtime FFT plan: length, radix sequence, threads per line.
struct FftPlan {
  int n;
  int nstage;
  int tpl;          // threads per line = n / E
  int radix[8];
};

// ---------------------------------------------------------------------------
// in-register DFTs of size 2, 3, 4, 8 with exp(S 2 pi i / R) roots
// ---------------------------------------------------------------------------

template <int S, typename T>
__device__ __forceinline__ void dft2(cpx<T>* v) {
  cpx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <int S, typename T>
__device__ __forceinline__ void dft3(cpx<T>* v) {
  const T c1 = T(-0.5);
  const T c2 = T(S) * T(0.86602540378443864676372317075294);  // S sqrt(3)/2
  cpx<T> t = cadd(v[1], v[2]);
  cpx<T> d = csub(v[1], v[2]);
  cpx<T> m = {v[0].re + c1 * t.re, v[0].im + c1 * t.im};
  cpx<T> r = {-c2 * d.im, c2 * d.re};  // i c2 d
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, r);
  v[2] = csub(m, r);
}

template <int S, typename T>
__device__ __forceinline__ void dft4(cpx<T>* v) {
  cpx<T> t0 = cadd(v[0], v[2]);
  cpx<T> t1 = csub(v[0], v[2]);
  cpx<T> t2 = cadd(v[1], v[3]);
  cpx<T> t3 = mul_si<S>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <int S, typename T>
__device__ __forceinline__ void dft8(cpx<T>* v) {
  const T h = T(0.70710678118654752440084436210485);
  cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<S>(e);
  dft4<S>(o);
  // o[k] *= w8^k, w8 = exp(S i pi / 4)
  cpx<T> o1 = {h * (o[1].re - T(S) * o[1].im), h * (o[1].im + T(S) * o[1].re)};
  cpx<T> o2 = mul_si<S>(o[2]);
  cpx<T> o3 = {h * (-o[3].re - T(S) * o[3].im), h * (-o[3].im + T(S) * o[3].re)};
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <int R, int S, typename T>
__device__ __forceinline__ void dft(cpx<T>* v) {
  if constexpr (R == 2) dft2<S>(v);
  else if constexpr (R == 3) dft3<S>(v);
  else if constexpr (R == 4) dft4<S>(v);
  else dft8<S>(v);
}

// One Stockham stage of radix R on the lines of a tile.
//   input position  j + r n/R, twiddle exp(S 2 pi i r (j mod ns) / (ns R))
//   output position (j / ns) ns R + (j mod ns) + r ns
// Every thread owns E/R butterflies j = lane + tpl * b.
template <int R, int E, int S, typename T>
__device__ __forceinline__ void stockham_stage(cpx<T>* buf, int lp, int line, int lane, bool active,
                                               int n, int tpl, int ns, const cpx<T>* tw) {
  constexpr int NB = E / R;
  cpx<T> v[E];
  const int stride = n / R;
  if (active) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = lane + tpl * b;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b * R + r] = buf[(j + r * stride) * lp + line];
    }
  }
  __syncthreads();
  if (active) {
    const int tstep = n / (ns * R);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = lane + tpl * b;
      const int k = j % ns;
      if (ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cpx<T> w = tw[r * k * tstep];  // exp(-2 pi i r k / (ns R))
          v[b * R + r] = (S < 0) ? cmul(v[b * R + r], w) : cmulc(v[b * R + r], w);
        }
      }
      dft<R, S>(&v[b * R]);
      const int d = (j / ns) * ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(d + r * ns) * lp + line] = v[b * R + r];
    }
  }
  __syncthreads();
}

// Full FFT of every line of the tile, in place in LDS.  S = -1: forward
// (exp(-i...)), S = +1: inverse (unnormalised).  tw[m] = exp(-2 pi i m / n).
// All threads of the block must call this (it contains barriers).
template <int E, int S, typename T>
__device__ void fft_tile(cpx<T>* buf, int lp, int line, int lane, bool active, const FftPlan& pl,
                         const cpx<T>* tw) {
  int ns = 1;
  for (int s = 0; s < pl.nstage; ++s) {
    const int R = pl.radix[s];
    if constexpr (E % 8 == 0) {
      if (R == 8) stockham_stage<8, E, S>(buf, lp, line, lane, active, pl.n, pl.tpl, ns, tw);
      else if (R == 4) stockham_stage<4, E, S>(buf, lp, line, lane, active, pl.n, pl.tpl, ns, tw);
      else stockham_stage<2, E, S>(buf, lp, line, lane, active, pl.n, pl.tpl, ns, tw);
    } else {
      if (R == 3) stockham_stage<3, E, S>(buf, lp, line, lane, active, pl.n, pl.tpl, ns, tw);
      else if (R == 4) stockham_stage<4, E, S>(buf, lp, line, lane, active, pl.n, pl.tpl, ns, tw);
      else stockham_stage<2, E, S>(buf, lp, line, lane, active, pl.n, pl.tpl, ns, tw);
    }
    ns *= R;
  }
}

// Spectral index maps shared by all kernels.  A band of `cnt` entries along
// a periodic axis of length n stores wavenumbers 0..h then -h..-1 with
// h = (cnt - 1) / 2 (cnt = n: the full FFT order).  full_pos maps a band slot
// to its FFT-order position; band_slot is the inverse (-1 if not stored).
__device__ __forceinline__ int full_pos(int i, int cnt, int n) {
  return (i <= (cnt - 1) / 2) ? i : i + (n - cnt);
}
__device__ __forceinline__ int band_slot(int p, int cnt, int n) {
  const int h = (cnt - 1) / 2;
  if (p <= h) return p;
  const int q = p - (n - cnt);
  return (q > h) ? q : -1;
}
// Signed wavenumber at FFT-order position p (numpy fftfreq convention).
__device__ __forceinline__ int signed_k(int p, int n) { return (p < (n + 1) / 2) ? p : p - n; }

}  // namespace psms
