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
// Twiddles exp(-2 pi i m / N) come from a table computed in FP64 on the host,
// regrouped per stage in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

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

// Global-memory access through an explicit global address space.  Pointers
// read from a descriptor table in memory are generic (flat) to the compiler,
// and flat accesses also count against the LDS wait counter, so every LDS
// wait of a transform would drain them; these helpers issue global loads and
// stores instead.  p must point to device global memory, 2 * sizeof(T)
// aligned.
// f(std::integral_constant<int, I>{}) for I = 0 .. COUNT-1, in order: the
// body sees its index as a compile-time constant.
template <int I, int COUNT, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < COUNT) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, COUNT>(f);
  }
}

template <typename T>
__device__ __forceinline__ cpx<T> ld_global(const cpx<T>* p) {
  typedef T T2 __attribute__((ext_vector_type(2)));
  const T2 v = *(const __attribute__((address_space(1))) T2*)(const void*)p;
  return cpx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void st_global(cpx<T>* p, cpx<T> v) {
  typedef T T2 __attribute__((ext_vector_type(2)));
  T2 w;
  w.x = v.re;
  w.y = v.im;
  *(__attribute__((address_space(1))) T2*)(void*)p = w;
}

// ---------------------------------------------------------------------------
// compile-time plans: transform length N, values per thread E, radix sequence
// ---------------------------------------------------------------------------
template <int N_, int E_, int R0, int R1 = 0, int R2 = 0, int R3 = 0, int R4 = 0, int R5 = 0, int R6 = 0>
struct PlanT {
  static constexpr int N = N_;
  static constexpr int E = E_;
  static constexpr int NST = (R0 > 0) + (R1 > 0) + (R2 > 0) + (R3 > 0) + (R4 > 0) + (R5 > 0) + (R6 > 0);
  static constexpr int R[8] = {R0, R1, R2, R3, R4, R5, R6, 0};
};

// Default plans: N = 2^m with E = 4 (radix-4 stages, one radix-2 stage when m
// is odd); N = 3*2^m with E = 6 (one radix-3 stage, radix-2 stages).
template <int N> struct PlanSel;
template <> struct PlanSel<8>   { using type = PlanT<8, 4, 4, 2>; };
template <> struct PlanSel<16>  { using type = PlanT<16, 4, 4, 4>; };
template <> struct PlanSel<32>  { using type = PlanT<32, 4, 4, 4, 2>; };
template <> struct PlanSel<64>  { using type = PlanT<64, 4, 4, 4, 4>; };
template <> struct PlanSel<128> { using type = PlanT<128, 4, 4, 4, 4, 2>; };
template <> struct PlanSel<256> { using type = PlanT<256, 4, 4, 4, 4, 4>; };
template <> struct PlanSel<512> { using type = PlanT<512, 4, 4, 4, 4, 4, 2>; };
template <> struct PlanSel<12>  { using type = PlanT<12, 6, 3, 2, 2>; };
template <> struct PlanSel<24>  { using type = PlanT<24, 6, 3, 2, 2, 2>; };
template <> struct PlanSel<48>  { using type = PlanT<48, 6, 3, 2, 2, 2, 2>; };
template <> struct PlanSel<96>  { using type = PlanT<96, 6, 3, 2, 2, 2, 2, 2>; };
template <> struct PlanSel<192> { using type = PlanT<192, 6, 3, 2, 2, 2, 2, 2, 2>; };
template <int N>
using Plan = typename PlanSel<N>::type;

// Radix of stage s when running in direction S (S < 0: forward order,
// S > 0: reversed order).
template <class P, int S, int s>
__host__ __device__ constexpr int radix_at() {
  return (S < 0) ? P::R[s] : P::R[P::NST - 1 - s];
}
// Radix of the first / last stage in direction S.
template <class P, int S>
__host__ __device__ constexpr int first_radix() { return radix_at<P, S, 0>(); }
template <class P, int S>
__host__ __device__ constexpr int last_radix() { return radix_at<P, S, P::NST - 1>(); }

// Position of register slot (b, r) for a stage of radix R: t + TT*b + r*N/R.
template <class P, int R>
__device__ __forceinline__ int slot_pos(int t, int b, int r) {
  constexpr int TT = P::N / P::E;
  return t + TT * b + r * (P::N / R);
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
    static_assert(R == 4, "radix 2, 3 or 4");
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

// Twiddles.  Stage s of direction S (radix R, stride NS > 1) needs
// w(r, k) = exp(-2 pi i r k / (NS R)) for r = 1..R-1, k = 0..NS-1; the inverse
// applies the conjugates.  Two LDS layouts:
//  * the plain table exp(-2 pi i m / N), m < N, read at m = r k N / (NS R):
//    used by strided tiles, whose lanes run over lines and so read the same
//    entry (a broadcast);
//  * per-stage tables [r-1][k] at the stage's offset (build_twiddles): used by
//    row tiles, whose lanes run over positions (k), so that they read
//    consecutive entries instead of entries r N / (NS R) apart.
template <class P, int S, int s, int NS = 1>
__host__ __device__ constexpr int tw_span() {
  if constexpr (s >= P::NST) {
    return 0;
  } else {
    constexpr int R = radix_at<P, S, s>();
    return (NS > 1 ? (R - 1) * NS : 0) + tw_span<P, S, s + 1, NS * R>();
  }
}
// Entries of the whole table of direction S.
template <class P, int S>
__host__ __device__ constexpr int tw_size() { return tw_span<P, S, 0>(); }

// Fill the table of direction S from base(m) = exp(-2 pi i m / N), with the
// nthr threads of the block (tid = 0..nthr-1).  The caller synchronises.
template <typename T, class P, int S, int s = 0, int NS = 1, int OFF = 0, class Base>
__device__ __forceinline__ void build_twiddles(cpx<T>* dst, const Base& base, int tid, int nthr) {
  if constexpr (s < P::NST) {
    constexpr int R = radix_at<P, S, s>();
    if constexpr (NS > 1) {
      for (int e = tid; e < (R - 1) * NS; e += nthr) {
        const int r = 1 + e / NS, k = e % NS;
        dst[OFF + e] = base(r * k * (P::N / (NS * R)));
      }
    }
    build_twiddles<T, P, S, s + 1, NS * R, OFF + (NS > 1 ? (R - 1) * NS : 0)>(dst, base, tid, nthr);
  }
}

// One Stockham stage on registers.  Input  v[b*R + r] = x[j_b + r N/R],
// output v[b*R + r] = y[d_b + r NS], j_b = t + TT b, k = j_b mod NS,
// d_b = (j_b / NS) NS R + k, with the twiddle exp(S 2 pi i r k / (NS R)),
// read from the stage table at OFF (ST) or from the plain table.
template <typename T, class P, int R, int NS, int S, int OFF, bool ST>
__device__ __forceinline__ void stage_regs(cpx<T>* v, int t, const cpx<T>* tw) {
  constexpr int N = P::N;
  constexpr int E = P::E;
  constexpr int TT = N / E;
  constexpr int NB = E / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + TT * b;
    if constexpr (NS > 1) {
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cpx<T> w = ST ? tw[OFF + (r - 1) * NS + k] : tw[r * k * (N / (NS * R))];
        v[b * R + r] = (S < 0) ? cmul(v[b * R + r], w) : cmulc(v[b * R + r], w);
      }
    }
    dft<R, S>(&v[b * R]);
  }
}

// LDS index functors.  kWaveLocal also selects the twiddle layout (per-stage
// tables for row tiles, the plain table for strided tiles).
//  * strided tiles (lanes run over lines first): element (pos, line) at
//    pos * (L + 1) + line (IdxPosMajor), or at swz(pos) * L + line
//    (IdxPosSwz), swz(p) = p ^ (((p >> 2) ^ (p >> 4) ^ (p >> 6) ^ (p >> 8)) & 3),
//    a bijection on any multiple of 4 positions: a half wavefront's lanes
//    touch 4 positions of the L lines, at position strides 1, R, R^2, ...
//    depending on the stage, and the XOR sends each such set of positions to
//    4 different groups of banks, where the padding of one line per position
//    lets the bank groups of stride-4 positions overlap pairwise.  Measured:
//    the swizzle pays in the z stage and for N = 256 lines, the padding is
//    as fast or faster elsewhere.  A line's threads span the workgroup, so
//    the exchanges synchronise the workgroup;
//  * row tiles (lanes run over positions first): element (line, pos) at
//    line * kRowStride<N> + pos + 3 (pos >> 4), the padding spreading the
//    stride-R writes of the early stages over the banks; a line's TT <= 64
//    threads are consecutive lanes of one wavefront, so the exchanges only
//    need the wavefront's own ordering.
template <int N>
constexpr int kRowStride = N + 3 * ((N - 1) >> 4) + 2;
struct IdxPosMajor {
  static constexpr bool kWaveLocal = false;
  int lp, line;  // lp = L + 1
  __device__ __forceinline__ int operator()(int pos) const { return pos * lp + line; }
};
struct IdxPosSwz {
  static constexpr bool kWaveLocal = false;
  int l, line;  // l = L
  __device__ __forceinline__ int operator()(int pos) const {
    return (pos ^ (((pos >> 2) ^ (pos >> 4) ^ (pos >> 6) ^ (pos >> 8)) & 3)) * l + line;
  }
};
template <int N, int TT = N>
struct IdxLineMajor {
  static_assert(TT <= 64 && 64 % TT == 0, "a row line must lie within one wavefront");
  static constexpr bool kWaveLocal = true;
  int base;  // line * kRowStride<N>
  __device__ __forceinline__ int operator()(int pos) const { return base + pos + 3 * (pos >> 4); }
};

// Row tiles with an XOR swizzle in place of the padding: element (line, pos)
// at line * kRowStrideSwz<N> + (pos ^ ((pos >> 3) & 15)).  The XOR changes
// only the low 4 bits, with bits that it leaves unchanged or can be undone
// from (bit 3 is XORed with bit 6, bits 0-2 with bits 3-5), so it permutes
// every block of 16 positions; N must be a multiple of 16.
template <int N>
constexpr int kRowStrideSwz = N + 1;
template <int N, int TT = N>
struct IdxLineSwz {
  static_assert(TT <= 64 && 64 % TT == 0, "a row line must lie within one wavefront");
  static_assert(N % 16 == 0, "the swizzle permutes blocks of 16 positions");
  static constexpr bool kWaveLocal = true;
  int base;  // line * kRowStrideSwz<N>
  __device__ __forceinline__ int operator()(int pos) const { return base + (pos ^ ((pos >> 3) & 15)); }
};

// Orders the LDS accesses of one wavefront: the LDS executes a wavefront's
// instructions in issue order, so only the compiler must not move memory
// operations across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <class Idx>
__device__ __forceinline__ void exchange_sync() {
  if constexpr (Idx::kWaveLocal) {
    wave_lds_sync();
  } else {
    __syncthreads();
  }
}

// Stages s .. NST-1 of NF independent transforms in direction S, starting
// from registers holding the input of stage s (v[f] holds line f).  Line f
// exchanges through the LDS buffer base + f * fstride + par * pstride, par
// alternating between exchanges; one synchronisation per exchange (of the
// workgroup or, for row tiles, of the wavefront) serves all NF lines, and
// their independent butterflies fill each other's LDS latency.  A row tile may
// use a single buffer per line (pstride = 0): a wavefront's LDS accesses
// complete in order, and each exchange's writes depend on the previous one's
// reads.  All threads of the block must call it.
template <typename T, class P, int S, int s, int NS, int OFF, int NF, class Idx>
__device__ __forceinline__ void fft_stages(cpx<T> (*v)[P::E], cpx<T>* base, int fstride, int pstride, int& par,
                                           int t, const Idx& idx, const cpx<T>* tw) {
  constexpr int R = radix_at<P, S, s>();
#pragma unroll
  for (int f = 0; f < NF; ++f) stage_regs<T, P, R, NS, S, OFF, Idx::kWaveLocal>(v[f], t, tw);
  if constexpr (s + 1 < P::NST) {
    constexpr int E = P::E;
    constexpr int TT = P::N / E;
    constexpr int R2 = radix_at<P, S, s + 1>();
    cpx<T>* L = base + par * pstride;
    par ^= 1;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int b = 0; b < E / R; ++b) {
        const int j = t + TT * b;
        const int d = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) L[f * fstride + idx(d + r * NS)] = v[f][b * R + r];
      }
    exchange_sync<Idx>();
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int b = 0; b < E / R2; ++b)
#pragma unroll
        for (int r = 0; r < R2; ++r) v[f][b * R2 + r] = L[f * fstride + idx(slot_pos<P, R2>(t, b, r))];
    fft_stages<T, P, S, s + 1, NS * R, OFF + (NS > 1 ? (R - 1) * NS : 0), NF>(v, base, fstride, pstride, par, t,
                                                                              idx, tw);
  }
}

// Whole transform.  On entry v[b*R + r] holds x at slot_pos<P, first_radix>;
// on exit it holds X at slot_pos<P, last_radix>.  S = -1 forward, +1 inverse
// (unnormalised); tw is the twiddle table of direction S for the tile kind.
// Exchanges alternate between the buffers b0 and b1.
template <typename T, class P, int S, class Idx>
__device__ __forceinline__ void fft_line(cpx<T>* v, cpx<T>* b0, cpx<T>* b1, int& par, int t, const Idx& idx,
                                         const cpx<T>* tw) {
  fft_stages<T, P, S, 0, 1, 0, 1>(reinterpret_cast<cpx<T>(*)[P::E]>(v), b0, 0, int(b1 - b0), par, t, idx, tw);
}

// NF transforms at once (see fft_stages): line f exchanges through
// base + f * fstride (+ pstride on alternate exchanges).
template <typename T, class P, int S, int NF, class Idx>
__device__ __forceinline__ void fft_lines(cpx<T> (*v)[P::E], cpx<T>* base, int fstride, int pstride, int& par, int t,
                                          const Idx& idx, const cpx<T>* tw) {
  fft_stages<T, P, S, 0, 1, 0, NF>(v, base, fstride, pstride, par, t, idx, tw);
}

// Tiling of a batch of lines of length N: E values per thread, TT threads per
// line, L lines per workgroup of THREADS = 64 << V threads (V is the
// workgroup-size variant the autotuner chooses between; V = 2 is 256).
template <class P, int V = 2>
struct Tile {
  static constexpr int N = P::N;
  static constexpr int E = P::E;
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
