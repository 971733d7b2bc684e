// HIP kernels of the periodic-box Navier-Stokes + Cahn-Hilliard step (gfx950).
//
// The step of Sec. 2.2 (steps ii-v) is executed as four kernels per time step,
// all on the caller's stream:
//   k_ystep<+1>  y-inverse of u, v, w, phi, d_z phi, plus i k_y phi
//   k_xstep      x-inverse (7 fields), the pointwise products (Sec. 3.2.2,
//                Hadamard products) and the x-forward of the 8 products
//   k_ystep<-1>  y-forward with 2/3 truncation
//   k_zstep      z-forward, spectral RHS assembly, Leray projection, CN/AB2
//                (NS) and IE/AB2 (CH) updates, then the z-inverse of the new
//                state for the next step.
// Spectral data is stored only inside the retained band |k_i| <= K =
// floor((N-1)/3), so the transforms never read or write discarded modes.
//
// Layouts (complex values interleaved re, im):
//   state, history : [4][C kz][C ky][H kx] double   (C = 2K+1, H = K+1)
//   G (z-inverse)  : [5][N z][C ky][H kx]           (u, v, w, phi, d_z phi)
//   Y (y-inverse)  : [6][N z][N y][H kx]            (u, v, w, phi, d_y phi, d_z phi)
//   X (x-forward)  : [8][N z][N y][H kx]            (T_xx T_yy T_zz T_xy T_xz T_yz, a, c)
//   W (y-forward)  : [8][N z][C ky][H kx]
//
// Every kernel is instantiated per transform length N (compile time) so that
// all index arithmetic folds to constants.  The step kernels read their
// pointers and coefficients from a device table of boxes (BoxDev) indexed by
// blockIdx.z, so one launch advances every box of a given size.
#include <hip/hip_runtime.h>

#include <type_traits>


#include "box_kernels.hpp"
#include "fft_engine.hpp"

namespace psms {

template <typename T>
__device__ __forceinline__ cpx<T> to_cpx(cpx<double> v) { return {T(v.re), T(v.im)}; }


// ---------------------------------------------------------------------------
// batched transforms along a strided axis (y or z): L lines per workgroup,
// lanes line-fastest, LDS element (pos, line) at pos * (L+1) + line.
// S = -1 forward (output band of n_out slots), S = +1 inverse (input band of
// n_in slots, zero-padded).  Output field f reads input field (fmap >> 4f)&15;
// bit f of dmask multiplies by i k along the axis.
// ---------------------------------------------------------------------------
template <typename T, class P, int S, int V>
__device__ __forceinline__ void lines_body(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                           const cpx<T>* __restrict__ tw_g, const LineArgs& a, bool deriv) {
  using G = Tile<P, V>;
  constexpr int N = P::N;
  constexpr bool SWZ = N >= 256;   // see the LDS index functors
  constexpr int E = G::E, L = G::L, LP = SWZ ? L : L + 1;
  constexpr int RI = first_radix<P, S>(), RO = last_radix<P, S>();
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> lds[2][N * LP];
  const int tid = threadIdx.x;
  const int line = tid % L, t = tid / L;
  for (int i = tid; i < N; i += blockDim.x) tw[i] = tw_g[i];
  const long long gl = (long long)xcd_tile(blockIdx.x, gridDim.x) * L + line;
  const bool valid = gl < a.nlines;
  const long long o = valid ? gl / a.inner : 0, i = valid ? gl % a.inner : 0;

  cpx<T> v[E];
#pragma unroll
  for (int b = 0; b < E / RI; ++b) {
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int p = slot_pos<P, RI>(t, b, r);
      const int s = band_slot(p, a.n_in, N);
      cpx<T> x = {T(0), T(0)};
      if (valid && s >= 0) {
        x = ld_global(src + (o * a.n_in + s) * a.inner + i);
        if (S > 0 && deriv) {
          const T k = T(signed_k(p, N));
          x = cpx<T>{-k * x.im, k * x.re};
        }
      }
      v[b * RI + r] = x;
    }
  }
  __syncthreads();
  int par = 0;
  if constexpr (SWZ)
    fft_line<T, P, S>(v, lds[0], lds[1], par, t, IdxPosSwz{LP, line}, tw);
  else
    fft_line<T, P, S>(v, lds[0], lds[1], par, t, IdxPosMajor{LP, line}, tw);
  const T sc = T(a.scale);
#pragma unroll
  for (int b = 0; b < E / RO; ++b) {
#pragma unroll
    for (int r = 0; r < RO; ++r) {
      const int p = slot_pos<P, RO>(t, b, r);
      const int s = band_slot(p, a.n_out, N);
      if (valid && s >= 0) {
        cpx<T> x = v[b * RO + r];
        if (S < 0 && deriv) {
          const T k = T(signed_k(p, N));
          x = cpx<T>{-k * x.im, k * x.re};
        }
        st_global(dst + (o * a.n_out + s) * a.inner + i, cpx<T>{sc * x.re, sc * x.im});
      }
    }
  }
}

template <typename T, int N, int S>
__global__ void __launch_bounds__(256) k_lines(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                                               const cpx<T>* __restrict__ tw_g, LineArgs a) {
  const int fo = blockIdx.y;
  lines_body<T, Plan<N>, S, 2>(in + (long long)((a.fmap >> (4 * fo)) & 15) * a.in_fstride,
                         out + (long long)fo * a.out_fstride, tw_g, a, (a.dmask >> fo) & 1);
}

// y stages of the step for box box0 + blockIdx.z.
//   S = +1: G [5][N][C][H] (bufb) -> Y [6][N][N][H] (bufa); output 4 is i ky phi.
//   S = -1: X [8][N][N][H] (bufb) -> W [8][N][C][H] (bufa), truncated to the band.
template <typename T, int N, int S, int V>
__global__ void __launch_bounds__(64 << V) k_ystep(const BoxDev* __restrict__ boxes, int box0,
                                                   const cpx<T>* __restrict__ tw_g) {
  using P = Plan<N>;
  using G = Tile<P, V>;
  const BoxDev& bx = boxes[box0 + blockIdx.z];
  const int fo = blockIdx.y;
  LineArgs a;
  a.inner = G::H;
  a.nlines = (long long)N * G::H;
  a.scale = 1.0;
  const long long nq = (long long)N * G::C * G::H, nnh = (long long)N * N * G::H;
  if (S > 0) {
    a.n_in = G::C;
    a.n_out = N;
    const int fin = (fo <= 3) ? fo : fo - 1;
    lines_body<T, P, S, V>(static_cast<const cpx<T>*>(bx.bufb) + fin * nq,
                           static_cast<cpx<T>*>(bx.bufa) + fo * nnh,
                           tw_g, a, fo == 4);
  } else {
    a.n_in = N;
    a.n_out = G::C;
    lines_body<T, P, S, V>(static_cast<const cpx<T>*>(bx.bufb) + fo * nnh,
                           static_cast<cpx<T>*>(bx.bufa) + fo * nq,
                           tw_g, a, false);
  }
}

// ---------------------------------------------------------------------------
// real transforms along x (contiguous rows), two rows packed per complex FFT
// (z = a + i b).  L row pairs per workgroup, lanes position-fastest, LDS
// element (pos, pair) at pair * (N+1) + pos.
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(256) k_rows_fwd(const T* __restrict__ in, cpx<T>* __restrict__ out,
                                                  const cpx<T>* __restrict__ tw_g, RowArgs a) {
  using P = Plan<N>;
  using G = Tile<P>;
  constexpr int E = G::E, TT = G::TT, L = G::L, LP = kRowStride<N>;
  constexpr int RI = first_radix<P, -1>(), RO = last_radix<P, -1>();
  __shared__ cpx<T> tw[tw_size<P, -1>()];
  __shared__ cpx<T> lds[2][L * LP];
  const int tid = threadIdx.x;
  const int t = tid % TT, line = tid / TT;
  build_twiddles<T, P, -1>(tw, [&](int m) { return tw_g[m]; }, tid, int(blockDim.x));
  const T* src = in + (long long)blockIdx.y * a.in_fstride;
  cpx<T>* dst = out + (long long)blockIdx.y * a.out_fstride;
  const long long r0 = ((long long)blockIdx.x * L + line) * 2;
  const bool v0 = r0 < a.nrows, v1 = r0 + 1 < a.nrows;
  cpx<T> v[E];
#pragma unroll
  for (int b = 0; b < E / RI; ++b)
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int p = slot_pos<P, RI>(t, b, r);
      v[b * RI + r] = cpx<T>{v0 ? src[r0 * N + p] : T(0), v1 ? src[(r0 + 1) * N + p] : T(0)};
    }
  __syncthreads();
  int par = 0;
  const IdxLineMajor<N, TT> idx{line * LP};
  fft_line<T, P, -1>(v, lds[0], lds[1], par, t, idx, tw);
  cpx<T>* Lb = par ? lds[1] : lds[0];
#pragma unroll
  for (int b = 0; b < E / RO; ++b)
#pragma unroll
    for (int r = 0; r < RO; ++r) Lb[idx(slot_pos<P, RO>(t, b, r))] = v[b * RO + r];
  wave_lds_sync();  // the line's threads are one wavefront's lanes
  const T h = T(0.5) * T(a.scale);
  for (int k = t; k < a.n_out; k += TT) {
    const cpx<T> zk = Lb[idx(k)];
    const cpx<T> zm = Lb[idx((N - k) % N)];
    if (v0) dst[r0 * a.n_out + k] = cpx<T>{h * (zk.re + zm.re), h * (zk.im - zm.im)};
    if (v1) dst[(r0 + 1) * a.n_out + k] = cpx<T>{h * (zk.im + zm.im), h * (zm.re - zk.re)};
  }
}

template <typename T, int N>
__global__ void __launch_bounds__(256) k_rows_inv(const cpx<T>* __restrict__ in, T* __restrict__ out,
                                                  const cpx<T>* __restrict__ tw_g, RowArgs a) {
  using P = Plan<N>;
  using G = Tile<P>;
  constexpr int E = G::E, TT = G::TT, L = G::L, LP = kRowStride<N>;
  constexpr int RI = first_radix<P, 1>(), RO = last_radix<P, 1>();
  __shared__ cpx<T> tw[tw_size<P, 1>()];
  __shared__ cpx<T> lds[2][L * LP];
  const int tid = threadIdx.x;
  const int t = tid % TT, line = tid / TT;
  build_twiddles<T, P, 1>(tw, [&](int m) { return tw_g[m]; }, tid, int(blockDim.x));
  const cpx<T>* src = in + (long long)blockIdx.y * a.in_fstride;
  T* dst = out + (long long)blockIdx.y * a.out_fstride;
  const long long r0 = ((long long)blockIdx.x * L + line) * 2;
  const bool v0 = r0 < a.nrows, v1 = r0 + 1 < a.nrows;
  cpx<T> v[E];
#pragma unroll
  for (int b = 0; b < E / RI; ++b)
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int p = slot_pos<P, RI>(t, b, r);
      const int k = (p <= N / 2) ? p : N - p;
      cpx<T> A = {T(0), T(0)}, B = {T(0), T(0)};
      if (k < a.n_in) {
        if (v0) A = src[r0 * a.n_in + k];
        if (v1) B = src[(r0 + 1) * a.n_in + k];
        if (k == 0 || 2 * k == N) {  // entries that are real for a real signal
          A.im = T(0);
          B.im = T(0);
        }
      }
      v[b * RI + r] = (p <= N / 2) ? cpx<T>{A.re - B.im, A.im + B.re}   // A + i B
                                   : cpx<T>{A.re + B.im, B.re - A.im};  // conj(A) + i conj(B)
    }
  __syncthreads();
  int par = 0;
  fft_line<T, P, 1>(v, lds[0], lds[1], par, t, IdxLineMajor<N, TT>{line * LP}, tw);
  const T sc = T(a.scale);
#pragma unroll
  for (int b = 0; b < E / RO; ++b)
#pragma unroll
    for (int r = 0; r < RO; ++r) {
      const int p = slot_pos<P, RO>(t, b, r);
      if (v0) dst[r0 * N + p] = sc * v[b * RO + r].re;
      if (v1) dst[(r0 + 1) * N + p] = sc * v[b * RO + r].im;
    }
}

// ---------------------------------------------------------------------------
// fused x stage of the step.  Each row pair (rows 2l, 2l+1 of the N^2 rows
// z N + y) is one complex line.  The 7 physical fields stay in registers at
// the positions the inverse leaves them, which are the positions the forward
// transform starts from, so the products need no data exchange.
// ---------------------------------------------------------------------------
// In FP32 the power-of-two plans up to 128 fit 128 VGPRs without spilling, so
// the compiler is asked for four waves per SIMD.
template <typename T, int N>
constexpr int kXstepWaves = (sizeof(T) == 4 && N <= 128 && (N & (N - 1)) == 0) ? 4 : 1;
// For those plans the fields are transformed four at a time (one LDS round
// trip per exchange for four lines; the inverse as fields 0-3, then 4-6) and
// the exchanges use the XOR-swizzled row layout; measured faster at N = 128
// (products in fours and the swizzle: 30.5 -> 28.8 us; the inverse in fours
// as well: a further 0.6 us).
template <typename T, int N>
constexpr bool kXstepWide = kXstepWaves<T, N> == 4 && N >= 64;
// the swizzled layout alone (FP64 at N = 64, 128)
template <typename T, int N>
constexpr bool kXstepSwz = kXstepWide<T, N> || (sizeof(T) == 8 && (N == 64 || N == 128));

// Staging of the x stage's inputs through LDS by direct global->LDS copies.
// A wavefront transforms LPW = 64 / TT consecutive row pairs, i.e. 2 LPW
// consecutive rows of H retained complex values each: one contiguous run of
// BYTES bytes per field, copied in 16-byte pieces (lane l of copy i moves
// piece 64 i + l to byte 16 (64 i + l) of the staging area).
template <typename T, int N, int TT, int H>
struct XStage {
  static_assert(TT <= 64 && 64 % TT == 0, "a wavefront holds whole lines");
  static constexpr int LPW = 64 / TT;
  static constexpr int BYTES = LPW * 2 * H * int(sizeof(cpx<T>));
  static_assert(BYTES % 16 == 0, "16-byte pieces");
  static constexpr int PIECES = BYTES / 16;
  static constexpr int NI = (PIECES + 63) / 64;
};
// Used where one wavefront holds one line (N = 256): measured faster there,
// and slower than register loads for the shorter lines.
template <typename T, int N>
constexpr bool kXstepDma = (N >= 256);

// Copy the pieces of one field that lie within `left` bytes of src.  dst is
// the wavefront's staging area (wave-uniform); each active lane's 16 bytes
// land at dst + 1024 i + 16 lane.
template <class XS>
__device__ __forceinline__ void xstage_copy(const char* src, char* dst, int lane, long long left) {
#pragma unroll
  for (int i = 0; i < XS::NI; ++i) {
    const int j = i * 64 + lane;
    if (j < XS::PIECES && (long long)(j + 1) * 16 <= left)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + 16 * j),
                                       (__attribute__((address_space(3))) void*)(dst + 1024 * i), 16, 0, 0);
  }
}
// the copies issued by this wavefront have landed in LDS (vmcnt = 0)
__device__ __forceinline__ void xstage_wait() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt unconstrained
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}
// this wavefront's reads of the staging area have completed (lgkmcnt = 0), so
// the next copies may overwrite it
__device__ __forceinline__ void xstage_release() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// Product F of the x stage (divergence form, eqs. NSE, kort, CHE) at slot e,
// component c (0: row 2l, 1: row 2l + 1) of the 7 physical fields u, v, w,
// phi, dx phi, dy phi, dz phi.
template <int F, typename T, int E>
__device__ __forceinline__ T xproduct(const cpx<T> (&ph)[7][E], int e, int c, T cs) {
  const T u = c ? ph[0][e].im : ph[0][e].re;
  const T vv = c ? ph[1][e].im : ph[1][e].re;
  const T w = c ? ph[2][e].im : ph[2][e].re;
  const T p3 = c ? ph[3][e].im : ph[3][e].re;
  const T gx = c ? ph[4][e].im : ph[4][e].re;
  const T gy = c ? ph[5][e].im : ph[5][e].re;
  const T gz = c ? ph[6][e].im : ph[6][e].re;
  if constexpr (F == 0) return -u * u + cs * (gy * gy + gz * gz);      // T_xx
  else if constexpr (F == 1) return -vv * vv + cs * (gx * gx + gz * gz);  // T_yy
  else if constexpr (F == 2) return -w * w + cs * (gx * gx + gy * gy);    // T_zz
  else if constexpr (F == 3) return -u * vv - cs * gx * gy;               // T_xy
  else if constexpr (F == 4) return -u * w - cs * gx * gz;                // T_xz
  else if constexpr (F == 5) return -vv * w - cs * gy * gz;               // T_yz
  else if constexpr (F == 6) return u * gx + vv * gy + w * gz;            // u . grad phi
  else return p3 * p3 * p3;                                               // phi^3
}

// order in which the x stage forms and transforms the 8 products
constexpr int kXstepFwdOrder[8] = {7, 6, 0, 1, 2, 3, 4, 5};

// CH: the same stage on rows of any count (the plane channel's x stage:
// xrows = (nc + 1) ny rows of the y-inverse, kx = kxs k for x periods other
// than 2 pi); the box passes xrows = N^2 and kxs = 1 implicitly.
template <typename T, int N, int V, bool CH = false>
__global__ void __launch_bounds__(64 << V) __attribute__((amdgpu_waves_per_eu(kXstepWaves<T, N>)))
k_xstep(const BoxDev* __restrict__ boxes, int box0, const cpx<T>* __restrict__ tw_g, long long xrows, double kxs) {
  using P = Plan<N>;
  using G = Tile<P, V>;
  const BoxDev& bx = boxes[box0 + blockIdx.z];
  const cpx<T>* __restrict__ yin = static_cast<const cpx<T>*>(bx.bufa);
  cpx<T>* __restrict__ xout = static_cast<cpx<T>*>(bx.bufb);
  const double csig_d = bx.csig;
  constexpr bool WIDE = kXstepWide<T, N>;
  constexpr bool SWZ = kXstepSwz<T, N>;
  constexpr int E = G::E, TT = G::TT, L = G::L, LP = SWZ ? kRowStrideSwz<N> : kRowStride<N>, K = G::K, H = G::H;
  constexpr int NFF = WIDE ? 4 : 2;   // products per forward group
  constexpr int RI = first_radix<P, 1>();   // inverse starts with R[NST-1]
  constexpr int RP = last_radix<P, 1>();    // inverse ends / forward starts with R[0]
  constexpr int RO = last_radix<P, -1>();   // forward ends with R[NST-1]
  const long long ROWS = CH ? xrows : (long long)N * N;
  constexpr bool XDMA = kXstepDma<T, N>;
  __shared__ cpx<T> twf[tw_size<P, -1>()];
  __shared__ cpx<T> twi[tw_size<P, 1>()];
  __shared__ cpx<T> lds[NFF][L * LP];
  __shared__ __attribute__((aligned(16))) char xstage_lds[XDMA ? (64 << V) / 64 * 2 * XStage<T, N, TT, H>::BYTES : 16];
  const int tid = threadIdx.x;
  const int t = tid % TT, line = tid / TT;
  build_twiddles<T, P, -1>(twf, [&](int m) { return tw_g[m]; }, tid, int(blockDim.x));
  build_twiddles<T, P, 1>(twi, [&](int m) { return tw_g[m]; }, tid, int(blockDim.x));
  const long long r0 = ((long long)xcd_tile(blockIdx.x, gridDim.x) * L + line) * 2;
  const bool valid = r0 < ROWS;  // ROWS is even: both rows exist
  using Idx = std::conditional_t<SWZ, IdxLineSwz<N, TT>, IdxLineMajor<N, TT>>;
  const Idx idx{line * LP};
  int par = 0;
  __syncthreads();

  // x-inverse of u v w phi dx_phi dy_phi dz_phi, two fields at a time; each of
  // the pair exchanges through its own buffer lds[g] (wavefront-local).  Where
  // registers allow (PF), the loads of the next pair are issued before the
  // current pair is transformed, so that their latency overlaps the transforms;
  // under the four-wavefront register budget they would spill.
  cpx<T> ph[7][E];
  // raw retained kx of both rows of field vf at slot e (= b RI + r) of the
  // positions the inverse starts from
  auto load_raw_slot = [&](int vf, int e, cpx<T>& A, cpx<T>& B) {
    const int fin = (vf <= 3) ? vf : vf - 1;   // vf 4 is i kx times phi
    const cpx<T>* src = yin + (long long)fin * ROWS * H;
    const int p = slot_pos<P, RI>(t, e / RI, e % RI);
    const int k = (p <= N / 2) ? p : N - p;
    A = cpx<T>{T(0), T(0)};
    B = cpx<T>{T(0), T(0)};
    if (valid && k <= K) {
      A = ld_global(src + r0 * H + k);
      B = ld_global(src + (r0 + 1) * H + k);
    }
  };
  // the packed complex line z = row0 + i row1 in Hermitian-extended FFT order
  auto pack_slot = [&](int vf, int e, cpx<T> A, cpx<T> B, cpx<T>& z) {
    const int p = slot_pos<P, RI>(t, e / RI, e % RI);
    const int k = (p <= N / 2) ? p : N - p;
    if (vf == 4) {
      const T kx = CH ? T(double(k) * kxs) : T(k);
      A = cpx<T>{-kx * A.im, kx * A.re};
      B = cpx<T>{-kx * B.im, kx * B.re};
    }
    if (k == 0) {
      A.im = T(0);
      B.im = T(0);
    }
    z = (p <= N / 2) ? cpx<T>{A.re - B.im, A.im + B.re} : cpx<T>{A.re + B.im, B.re - A.im};
  };
  auto load_raw = [&](int vf, cpx<T>* a, cpx<T>* bb) {
#pragma unroll
    for (int e = 0; e < E; ++e) load_raw_slot(vf, e, a[e], bb[e]);
  };
  auto pack = [&](int vf, const cpx<T>* a, const cpx<T>* bb, cpx<T>* v) {
#pragma unroll
    for (int e = 0; e < E; ++e) pack_slot(vf, e, a[e], bb[e], v[e]);
  };
  constexpr int FS = L * LP;  // buffer of the second transform of a pair
  constexpr bool PF = kXstepWaves<T, N> == 1;  // registers to spare for prefetching
  // Direct-to-LDS staging: the rows of one field that a wavefront transforms
  // are one contiguous run of XS::BYTES bytes, copied by a few 16-byte
  // global_load_lds instructions into the wavefront's staging area while the
  // previous pair is transformed (no registers held in flight).
  using XS = XStage<T, N, TT, H>;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  char* stg = xstage_lds + wv * 2 * XS::BYTES;
  // first row of the wavefront (uniform across it)
  const int wrow0 = __builtin_amdgcn_readfirstlane(int(r0) - 2 * ((tid & 63) / TT));
  auto dma_pair = [&](int vf0) {
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int vf = vf0 + g;
      if (vf >= 7) continue;
      const int fin = (vf <= 3) ? vf : vf - 1;
      const char* src = reinterpret_cast<const char*>(yin + (long long)fin * ROWS * H + (long long)wrow0 * H);
      const long long left = (ROWS - wrow0) * H * (long long)sizeof(cpx<T>);   // bytes of the field from here
      xstage_copy<XS>(src, stg + g * XS::BYTES, lane, left);
    }
  };
  cpx<T> ra[2][E], rb[2][E];
  if (XDMA) {
    dma_pair(0);
  } else if (PF) {
    load_raw(0, ra[0], rb[0]);
    load_raw(1, ra[1], rb[1]);
  }
  if constexpr (WIDE) {
    // four inverse transforms per LDS round trip: fields 0-3, then 4-6
    static_for<0, 2>([&](auto gi) {
      constexpr int f0 = decltype(gi)::value * 4;
      constexpr int nf = f0 == 0 ? 4 : 3;
      cpx<T> v[nf][E];
#pragma unroll
      for (int g = 0; g < nf; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          cpx<T> A, B;
          load_raw_slot(f0 + g, e, A, B);
          pack_slot(f0 + g, e, A, B, v[g][e]);
        }
      fft_lines<T, P, 1, nf>(v, lds[0], FS, 0, par, t, idx, twi);
#pragma unroll
      for (int g = 0; g < nf; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e) ph[f0 + g][e] = v[g][e];
    });
  } else
#pragma unroll
  for (int vf = 0; vf < 7; vf += 2) {
    const int nf = (vf + 1 < 7) ? 2 : 1;
    cpx<T> v[2][E];
    if (XDMA) {
      xstage_wait();
#pragma unroll
      for (int g = 0; g < 2; ++g)
        if (g < nf) {
          const cpx<T>* sg = reinterpret_cast<const cpx<T>*>(stg + g * XS::BYTES) + ((tid & 63) / TT) * 2 * H;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int p = slot_pos<P, RI>(t, e / RI, e % RI);
            const int k = (p <= N / 2) ? p : N - p;
            cpx<T> A = {T(0), T(0)}, B = {T(0), T(0)};
            if (valid && k <= K) {
              A = sg[k];
              B = sg[H + k];
            }
            pack_slot(vf + g, e, A, B, v[g][e]);
          }
        }
      xstage_release();
      if (vf + 2 < 7) dma_pair(vf + 2);
    } else if (PF) {
#pragma unroll
      for (int g = 0; g < 2; ++g)
        if (g < nf) pack(vf + g, ra[g], rb[g], v[g]);
#pragma unroll
      for (int g = 0; g < 2; ++g)
        if (vf + 2 + g < 7) load_raw(vf + 2 + g, ra[g], rb[g]);
    } else {
      // load and pack slot by slot, so that few raw values are live at once
#pragma unroll
      for (int g = 0; g < 2; ++g)
        if (g < nf) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            cpx<T> A, B;
            load_raw_slot(vf + g, e, A, B);
            pack_slot(vf + g, e, A, B, v[g][e]);
          }
        }
    }
    if (nf == 2) {
      fft_lines<T, P, 1, 2>(v, lds[0], FS, 0, par, t, idx, twi);
    } else {
      fft_lines<T, P, 1, 1>(v, lds[0], FS, 0, par, t, idx, twi);
    }
#pragma unroll
    for (int g = 0; g < 2; ++g)
      if (g < nf)
#pragma unroll
        for (int e = 0; e < E; ++e) ph[vf + g][e] = v[g][e];
  }

  // products and x-forward, NFF fields at a time in the order phi^3, u . grad
  // phi, T_xx .. T_yz (phi is then dead after the first group, and this order
  // fits the four-wavefront register budget without spills); the field indices
  // are compile-time constants, so the products are straight-line code with
  // no per-element branching
  const T cs = T(csig_d);
  const T h = T(0.5);
  static_assert(RP == first_radix<P, -1>(), "mirrored radix order");
  static_for<0, 8 / NFF>([&](auto gi) {
    constexpr int f0 = decltype(gi)::value * NFF;
    cpx<T> v[NFF][E];
    static_for<0, NFF>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      constexpr int F = kXstepFwdOrder[f0 + g];
#pragma unroll
      for (int e = 0; e < E; ++e) v[g][e] = cpx<T>{xproduct<F>(ph, e, 0, cs), xproduct<F>(ph, e, 1, cs)};
    });
    fft_lines<T, P, -1, NFF>(v, lds[0], FS, 0, par, t, idx, twf);
    // natural order through the group's buffers, then the retained kx of both rows
#pragma unroll
    for (int g = 0; g < NFF; ++g)
#pragma unroll
      for (int b = 0; b < E / RO; ++b)
#pragma unroll
        for (int r = 0; r < RO; ++r) lds[g][idx(slot_pos<P, RO>(t, b, r))] = v[g][b * RO + r];
    wave_lds_sync();  // the line's threads are one wavefront's lanes
    static_for<0, NFF>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      cpx<T>* dst = xout + (long long)kXstepFwdOrder[f0 + g] * ROWS * H;
      for (int k = t; valid && k < H; k += TT) {
        const cpx<T> zk = lds[g][idx(k)];
        const cpx<T> zm = lds[g][idx((N - k) % N)];
        st_global(dst + r0 * H + k, cpx<T>{h * (zk.re + zm.re), h * (zk.im - zm.im)});
        st_global(dst + (r0 + 1) * H + k, cpx<T>{h * (zk.im + zm.im), h * (zm.re - zk.re)});
      }
    });
  });
}

// ---------------------------------------------------------------------------
// fused z stage: z-forward of the 8 products, RHS, projection, update, and the
// z-inverse of the new state.  One line per retained (ky, kx) pair q; each
// thread keeps the modes its forward transform leaves in registers, which are
// the inputs its inverse transform starts from.
// do_update = 0 only loads the state and performs the z-inverse (prologue).
// ---------------------------------------------------------------------------
template <typename T, int N, int V>
__global__ void __launch_bounds__(64 << V) k_zstep(const BoxDev* __restrict__ boxes, int box0,
                                                   const cpx<T>* __restrict__ tw_g, int do_update) {
  using P = Plan<N>;
  using G = Tile<P, V>;
  const BoxDev& bx = boxes[box0 + blockIdx.z];
  const cpx<T>* __restrict__ rhs = static_cast<const cpx<T>*>(bx.bufa);
  cpx<double>* __restrict__ state = bx.state;
  cpx<double>* __restrict__ hist = bx.hist;
  cpx<T>* __restrict__ gout = static_cast<cpx<T>*>(bx.bufb);
  const StepCoef sc = bx.sc;
  constexpr int E = G::E, L = G::L, LP = L, K = G::K, C = G::C, H = G::H;   // swizzled tile
  constexpr int Q = C * H;
  constexpr long long M = (long long)C * Q;
  constexpr int RF = first_radix<P, -1>();   // forward starts with R[0]
  constexpr int RL = last_radix<P, -1>();    // forward ends / inverse starts with R[NST-1]
  static_assert(RL == first_radix<P, 1>(), "mirrored radix order");
  __shared__ cpx<T> tw[N];
  // two lines per exchange (one per field of a pair), each with its two
  // ping-pong buffers: line f, parity par at lds[2 f + par]
  __shared__ cpx<T> lds[4][N * LP];
  const int tid = threadIdx.x;
  const int line = tid % L, t = tid / L;
  for (int i = tid; i < N; i += blockDim.x) tw[i] = tw_g[i];
  const int q = xcd_tile(blockIdx.x, gridDim.x) * L + line;
  const bool valid = q < Q;
  const int iy = valid ? q / H : 0, ix = valid ? q % H : 0;
  const double kx = double(ix);
  const double ky = double(iy <= K ? iy : iy - C);
  const IdxPosSwz idx{LP, line};
  int par = 0;

  // band membership and wavenumber of the slots the forward leaves in registers
  bool inb[E];
  int slot[E];
  double kz[E];
#pragma unroll
  for (int b = 0; b < E / RL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int p = slot_pos<P, RL>(t, b, r);
      const int s = band_slot(p, C, N);
      inb[b * RL + r] = valid && s >= 0;
      slot[b * RL + r] = s;
      kz[b * RL + r] = double(signed_k(p, N));
    }

  cpx<double> acc[4][E];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[c][e] = cpx<double>{0.0, 0.0};

  __syncthreads();
  if (do_update) {
    // the forward transforms two products at a time (one barrier per exchange
    // for both), the next pair's loads in flight while a pair is transformed
    cpx<T> nx[2][E];
    auto load_pair = [&](int f0) {
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const cpx<T>* src = rhs + (long long)(f0 + g) * N * Q;
#pragma unroll
        for (int b = 0; b < E / RF; ++b)
#pragma unroll
          for (int r = 0; r < RF; ++r)
            nx[g][b * RF + r] = valid ? ld_global(src + (long long)slot_pos<P, RF>(t, b, r) * Q + q) : cpx<T>{T(0), T(0)};
      }
    };
    load_pair(0);
    // product f's contribution to the accumulators; f is a compile-time
    // constant in each call, so the accumulation is straight-line code
    auto accumulate = [&](auto fc, const cpx<T>* v) {
      constexpr int f = decltype(fc)::value;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (inb[e]) {
          const cpx<double> w = {double(v[e].re) * sc.inv_n3, double(v[e].im) * sc.inv_n3};
          const cpx<double> ikx = {-kx * w.im, kx * w.re};
          const cpx<double> iky = {-ky * w.im, ky * w.re};
          const cpx<double> ikz = {-kz[e] * w.im, kz[e] * w.re};
          if constexpr (f == 0) acc[0][e] = cadd(acc[0][e], ikx);                 // d_x T_xx
          else if constexpr (f == 1) acc[1][e] = cadd(acc[1][e], iky);            // d_y T_yy
          else if constexpr (f == 2) acc[2][e] = cadd(acc[2][e], ikz);            // d_z T_zz
          else if constexpr (f == 3) {                                             // T_xy
            acc[0][e] = cadd(acc[0][e], iky);
            acc[1][e] = cadd(acc[1][e], ikx);
          } else if constexpr (f == 4) {                                           // T_xz
            acc[0][e] = cadd(acc[0][e], ikz);
            acc[2][e] = cadd(acc[2][e], ikx);
          } else if constexpr (f == 5) {                                           // T_yz
            acc[1][e] = cadd(acc[1][e], ikz);
            acc[2][e] = cadd(acc[2][e], iky);
          } else if constexpr (f == 6) {                                           // -u.grad(phi)
            acc[3][e] = csub(acc[3][e], w);
          } else {                                                                 // lap(phi^3) / Pe
            const double k2 = kx * kx + ky * ky + kz[e] * kz[e];
            acc[3][e].re -= k2 * sc.inv_pe * w.re;
            acc[3][e].im -= k2 * sc.inv_pe * w.im;
          }
        }
      }
    };
    static_for<0, 4>([&](auto pc) {
      constexpr int f0 = decltype(pc)::value * 2;
      cpx<T> v[2][E];
#pragma unroll
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e) v[g][e] = nx[g][e];
      if constexpr (f0 + 2 < 8) load_pair(f0 + 2);
      fft_lines<T, P, -1, 2>(v, lds[0], 2 * N * LP, N * LP, par, t, idx, tw);
      accumulate(std::integral_constant<int, f0>(), v[0]);
      accumulate(std::integral_constant<int, f0 + 1>(), v[1]);
    });
    // spectral update of the owned modes (FP64)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (inb[e]) {
        const double k2 = kx * kx + ky * ky + kz[e] * kz[e];
        const long long id = (long long)slot[e] * Q + q;
        cpx<double> Sx = acc[0][e], Sy = acc[1][e], Sz = acc[2][e], Sp = acc[3][e];
        const cpx<double> ph = ld_global(state + 3 * M + id);
        Sp.re += sc.e_coef * k2 * ph.re;
        Sp.im += sc.e_coef * k2 * ph.im;
        if (k2 == 0.0) {
          if (bx.sphi0) st_global(bx.sphi0, Sp);   // the mean of S_phi, a divergence: rounding level
          Sx = Sy = Sz = Sp = cpx<double>{0.0, 0.0};
        } else {  // Leray projection
          const double ir = 1.0 / k2;
          const double kze = kz[e];
          const cpx<double> kd = {kx * Sx.re + ky * Sy.re + kze * Sz.re, kx * Sx.im + ky * Sy.im + kze * Sz.im};
          Sx.re -= kx * kd.re * ir; Sx.im -= kx * kd.im * ir;
          Sy.re -= ky * kd.re * ir; Sy.im -= ky * kd.im * ir;
          Sz.re -= kze * kd.re * ir; Sz.im -= kze * kd.im * ir;
        }
        cpx<double> ex[4] = {Sx, Sy, Sz, Sp};
        if (!sc.ab1) {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const cpx<double> hp = ld_global(hist + c * M + id);
            ex[c].re = 1.5 * ex[c].re - 0.5 * hp.re;
            ex[c].im = 1.5 * ex[c].im - 0.5 * hp.im;
          }
        }
        st_global(hist + 0 * M + id, Sx);
        st_global(hist + 1 * M + id, Sy);
        st_global(hist + 2 * M + id, Sz);
        st_global(hist + 3 * M + id, Sp);
        const double a = 0.5 * sc.dt * sc.nu * k2;
        const double ia = 1.0 / (1.0 + a);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const cpx<double> u = ld_global(state + c * M + id);
          const cpx<double> un = {((1.0 - a) * u.re + sc.dt * ex[c].re) * ia,
                                  ((1.0 - a) * u.im + sc.dt * ex[c].im) * ia};
          st_global(state + c * M + id, un);
          acc[c][e] = un;
        }
        const double den = 1.0 / (1.0 + sc.dt * sc.ch2_pe * (k2 * k2 + sc.s * k2));
        const cpx<double> pn = {(ph.re + sc.dt * ex[3].re) * den, (ph.im + sc.dt * ex[3].im) * den};
        st_global(state + 3 * M + id, pn);
        acc[3][e] = pn;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (inb[e]) {
        const long long id = (long long)slot[e] * Q + q;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c][e] = ld_global(state + c * M + id);
      }
    }
  }

  // z-inverse of u, v, w, phi and i kz phi, two fields at a time
  auto inv_fields = [&](auto gc, auto nc) {
    constexpr int g0 = decltype(gc)::value, nf = decltype(nc)::value;
    cpx<T> v[nf][E];
#pragma unroll
    for (int g = 0; g < nf; ++g)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        cpx<double> x = {0.0, 0.0};
        if (inb[e]) {
          if (g0 + g < 4) x = acc[g0 + g][e];
          else x = cpx<double>{-kz[e] * acc[3][e].im, kz[e] * acc[3][e].re};
        }
        v[g][e] = to_cpx<T>(x);
      }
    fft_lines<T, P, 1, nf>(v, lds[0], 2 * N * LP, N * LP, par, t, idx, tw);
    if (valid) {
#pragma unroll
      for (int g = 0; g < nf; ++g) {
        cpx<T>* dst = gout + (long long)(g0 + g) * N * Q;
#pragma unroll
        for (int b = 0; b < E / RF; ++b)
#pragma unroll
          for (int r = 0; r < RF; ++r) st_global(dst + (long long)slot_pos<P, RF>(t, b, r) * Q + q, v[g][b * RF + r]);
      }
    }
  };
  using std::integral_constant;
  inv_fields(integral_constant<int, 0>(), integral_constant<int, 2>());
  inv_fields(integral_constant<int, 2>(), integral_constant<int, 2>());
  inv_fields(integral_constant<int, 4>(), integral_constant<int, 1>());
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

// a compact FP64 band converted to precision T (n entries)
template <typename T>
__global__ void k_band_to(const cpx<double>* __restrict__ a, cpx<T>* __restrict__ out, long long n) {
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n;
       id += (long long)gridDim.x * blockDim.x) {
    const cpx<double> v = a[id];
    out[id] = cpx<T>{T(v.re), T(v.im)};
  }
}

// f <- f^3 over n values
template <typename T>
__global__ void k_cube(T* __restrict__ f, long long n) {
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n;
       id += (long long)gridDim.x * blockDim.x) {
    const T a = f[id];
    f[id] = a * a * a;
  }
}

// The pressure that the projection removes, from the compact spectra of the six
// products T_ij (order xx, yy, zz, xy, xz, yz; [6][M], precision T): with
// S_i = i k_j T_ij and lap p = div S, p_hat = k_i k_j T_ij / k^2 (FP64; k = 0 -> 0).
template <typename T>
__global__ void k_pressure_band(const cpx<T>* __restrict__ t6, BoxGeom g, cpx<double>* __restrict__ p) {
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < g.M;
       id += (long long)gridDim.x * blockDim.x) {
    const int ix = int(id % g.H);
    const int iy = int((id / g.H) % g.C);
    const int iz = int(id / ((long long)g.H * g.C));
    const double kx = ix, ky = (iy <= g.K) ? iy : iy - g.C, kz = (iz <= g.K) ? iz : iz - g.C;
    const double k2 = kx * kx + ky * ky + kz * kz;
    const double w[6] = {kx * kx, ky * ky, kz * kz, 2.0 * kx * ky, 2.0 * kx * kz, 2.0 * ky * kz};
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const cpx<T> a = t6[f * g.M + id];
      re += w[f] * double(a.re);
      im += w[f] * double(a.im);
    }
    p[id] = (k2 == 0.0) ? cpx<double>{0.0, 0.0} : cpx<double>{re / k2, im / k2};
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

// CFL number dt max_x sum_i |u_i| / dx (dx = 2 pi / n) from the physical
// velocity components, accumulated one component at a time:
// acc = (first ? 0 : acc) + scale |f|, then a two-pass maximum.
__global__ void k_abs_accum(const double* __restrict__ f, double* __restrict__ acc, long long n, double scale,
                            int first) {
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n; id += (long long)gridDim.x * blockDim.x)
    acc[id] = (first ? 0.0 : acc[id]) + scale * fabs(f[id]);
}

__global__ void k_max_partial(const double* __restrict__ a, long long n, double* __restrict__ part) {
  __shared__ double sh[256];
  double m = 0.0;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n; id += (long long)gridDim.x * blockDim.x)
    m = fmax(m, a[id]);
  const int t = threadIdx.x;
  sh[t] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_max_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, part[i]);
  const int t = threadIdx.x;
  sh[t] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  if (t == 0) out[0] = sh[0];
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
// host-side launchers (dispatch on the transform length)
// ---------------------------------------------------------------------------
#define PSMS_FOR_EACH_N(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256)

bool supported_n(int n) {
  switch (n) {
#define PSMS_CASE(NN) case NN:
    PSMS_FOR_EACH_N(PSMS_CASE)
#undef PSMS_CASE
    return true;
    default:
      return false;
  }
}

namespace {

template <typename T, int N>
hipError_t lines_n(int dir, const cpx<T>* in, cpx<T>* out, const cpx<T>* tw, const LineArgs& a, int nfield,
                   hipStream_t st) {
  using P = Plan<N>;
  using G = Tile<P>;
  const dim3 grid(unsigned((a.nlines + G::L - 1) / G::L), unsigned(nfield));
  const dim3 block(unsigned(G::L * G::TT));
  if (dir < 0) k_lines<T, N, -1><<<grid, block, 0, st>>>(in, out, tw, a);
  else k_lines<T, N, 1><<<grid, block, 0, st>>>(in, out, tw, a);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t rows_n(int dir, const void* in, void* out, const cpx<T>* tw, const RowArgs& a, int nfield,
                  hipStream_t st) {
  using P = Plan<N>;
  using G = Tile<P>;
  const long long pairs = (a.nrows + 1) / 2;
  const dim3 grid(unsigned((pairs + G::L - 1) / G::L), unsigned(nfield));
  const dim3 block(unsigned(G::L * G::TT));
  if (dir < 0)
    k_rows_fwd<T, N><<<grid, block, 0, st>>>(static_cast<const T*>(in), static_cast<cpx<T>*>(out), tw, a);
  else
    k_rows_inv<T, N><<<grid, block, 0, st>>>(static_cast<const cpx<T>*>(in), static_cast<T*>(out), tw, a);
  return hipGetLastError();
}

// The y stages' largest variant: 512 threads in FP32 (twice the lines per
// workgroup, so each position's row segment is 128 bytes, a whole cache line;
// measured faster), 256 in FP64 (measured slower at 512).
template <typename T, int V>
constexpr int kYVariant = (V == 2 && sizeof(T) == 4) ? 3 : V;

template <typename T, int N, int V>
hipError_t step_nv(int stage, const BoxDev* boxes, int box0, int nbox, const cpx<T>* tw, int do_update,
                   hipStream_t st) {
  using P = Plan<N>;
  using G = Tile<P, V>;
  const unsigned threads = unsigned(G::L * G::TT);
  switch (stage) {
    case 0: {  // y-inverse, 6 output fields
      using GY = Tile<P, kYVariant<T, V>>;
      const dim3 grid(unsigned(((long long)N * GY::H + GY::L - 1) / GY::L), 6, unsigned(nbox));
      k_ystep<T, N, 1, kYVariant<T, V>><<<grid, unsigned(GY::L * GY::TT), 0, st>>>(boxes, box0, tw);
      break;
    }
    case 1: {  // x stage with products
      const long long pairs = (long long)N * N / 2;
      const dim3 grid(unsigned((pairs + G::L - 1) / G::L), 1, unsigned(nbox));
      k_xstep<T, N, V><<<grid, threads, 0, st>>>(boxes, box0, tw, 0, 1.0);
      break;
    }
    case 2: {  // y-forward, 8 fields
      using GY = Tile<P, kYVariant<T, V>>;
      const dim3 grid(unsigned(((long long)N * GY::H + GY::L - 1) / GY::L), 8, unsigned(nbox));
      k_ystep<T, N, -1, kYVariant<T, V>><<<grid, unsigned(GY::L * GY::TT), 0, st>>>(boxes, box0, tw);
      break;
    }
    default: {  // z stage with the update
      const int Q = G::C * G::H;
      const dim3 grid(unsigned((Q + G::L - 1) / G::L), 1, unsigned(nbox));
      k_zstep<T, N, V><<<grid, threads, 0, st>>>(boxes, box0, tw, do_update);
      break;
    }
  }
  return hipGetLastError();
}

template <typename T, int N>
hipError_t step_n(int stage, int variant, const BoxDev* boxes, int box0, int nbox, const cpx<T>* tw, int do_update,
                  hipStream_t st) {
  switch (variant) {
    case 0: return step_nv<T, N, 0>(stage, boxes, box0, nbox, tw, do_update, st);
    case 1: return step_nv<T, N, 1>(stage, boxes, box0, nbox, tw, do_update, st);
    default: return step_nv<T, N, 2>(stage, boxes, box0, nbox, tw, do_update, st);
  }
}

}  // namespace

template <typename T, int N>
hipError_t xstage_rows_n(const BoxDev* dev, const cpx<T>* tw, long long rows, double kxs, hipStream_t st) {
  using G = Tile<Plan<N>, 2>;
  const long long pairs = rows / 2;
  const dim3 grid(unsigned((pairs + G::L - 1) / G::L), 1, 1);
  k_xstep<T, N, 2, true><<<grid, unsigned(G::L * G::TT), 0, st>>>(dev, 0, tw, rows, kxs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xstage_rows(int n, const BoxDev* dev, const cpx<T>* tw, long long rows, double kxs,
                              hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  if (rows % 2) return hipErrorInvalidValue;   // rows are transformed in pairs
  switch (n) {
#define PSMS_CASE(NN) case NN: return xstage_rows_n<T, NN>(dev, tw, rows, kxs, st);
    PSMS_FOR_EACH_N(PSMS_CASE)
#undef PSMS_CASE
  }
  return hipErrorInvalidValue;
}
template hipError_t launch_xstage_rows<float>(int, const BoxDev*, const cpx<float>*, long long, double, hipStream_t);
template hipError_t launch_xstage_rows<double>(int, const BoxDev*, const cpx<double>*, long long, double,
                                               hipStream_t);

template <typename T>
hipError_t launch_lines(int n, int dir, const cpx<T>* in, cpx<T>* out, const cpx<T>* tw, const LineArgs& a,
                        int nfield, hipStream_t st) {
  switch (n) {
#define PSMS_CASE(NN) case NN: return lines_n<T, NN>(dir, in, out, tw, a, nfield, st);
    PSMS_FOR_EACH_N(PSMS_CASE)
#undef PSMS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_rows(int n, int dir, const void* in, void* out, const cpx<T>* tw, const RowArgs& a, int nfield,
                       hipStream_t st) {
  switch (n) {
#define PSMS_CASE(NN) case NN: return rows_n<T, NN>(dir, in, out, tw, a, nfield, st);
    PSMS_FOR_EACH_N(PSMS_CASE)
#undef PSMS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_step_stage(int n, int stage, int variant, const BoxDev* boxes, int box0, int nbox,
                             const cpx<T>* tw, int do_update, hipStream_t st) {
  if (nbox < 1) return hipSuccess;
  switch (n) {
#define PSMS_CASE(NN) case NN: return step_n<T, NN>(stage, variant, boxes, box0, nbox, tw, do_update, st);
    PSMS_FOR_EACH_N(PSMS_CASE)
#undef PSMS_CASE
  }
  return hipErrorInvalidValue;
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
hipError_t launch_band_to(const cpx<double>* a, cpx<T>* out, long long n, hipStream_t st) {
  k_band_to<T><<<grid_for(n), 256, 0, st>>>(a, out, n);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_cube(T* f, long long n, hipStream_t st) {
  k_cube<T><<<grid_for(n), 256, 0, st>>>(f, n);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_pressure_band(const cpx<T>* t6, const BoxGeom& g, cpx<double>* p, hipStream_t st) {
  k_pressure_band<T><<<grid_for(g.M), 256, 0, st>>>(t6, g, p);
  return hipGetLastError();
}
template hipError_t launch_band_to<float>(const cpx<double>*, cpx<float>*, long long, hipStream_t);
template hipError_t launch_cube<float>(float*, long long, hipStream_t);
template hipError_t launch_cube<double>(double*, long long, hipStream_t);
template hipError_t launch_pressure_band<float>(const cpx<float>*, const BoxGeom&, cpx<double>*, hipStream_t);
template hipError_t launch_pressure_band<double>(const cpx<double>*, const BoxGeom&, cpx<double>*, hipStream_t);
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
hipError_t launch_abs_accum(const double* f, double* acc, long long n, double scale, int first, hipStream_t st) {
  long long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  k_abs_accum<<<unsigned(b < 1 ? 1 : b), 256, 0, st>>>(f, acc, n, scale, first);
  return hipGetLastError();
}

hipError_t launch_max(const double* a, long long n, double* part, int max_blocks, double* out, hipStream_t st) {
  long long b = (n + 255) / 256;
  if (b > max_blocks) b = max_blocks;
  if (b < 1) b = 1;
  k_max_partial<<<unsigned(b), 256, 0, st>>>(a, n, part);
  k_max_final<<<1, 256, 0, st>>>(part, int(b), out);
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
template hipError_t launch_step_stage<double>(int, int, int, const BoxDev*, int, int, const cpx<double>*, int,
                                              hipStream_t);
template hipError_t launch_step_stage<float>(int, int, int, const BoxDev*, int, int, const cpx<float>*, int,
                                             hipStream_t);
template hipError_t launch_expand<double>(const cpx<double>*, cpx<double>*, const BoxGeom&, int, hipStream_t);
template hipError_t launch_compact<double>(const cpx<double>*, cpx<double>*, const BoxGeom&, int, hipStream_t);
template hipError_t launch_spec_finish<double>(const cpx<double>*, cpx<double>*, const BoxGeom&, int, int, int,
                                               double, hipStream_t);
template hipError_t launch_spec_finish<float>(const cpx<float>*, cpx<float>*, const BoxGeom&, int, int, int, double,
                                              hipStream_t);

}  // namespace psms
