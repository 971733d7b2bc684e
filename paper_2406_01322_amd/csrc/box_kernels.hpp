// Kernel argument blocks and host launchers for the periodic-box step.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_engine.hpp"

namespace psms {

// Geometry of the retained band on an n^3 box: K = floor((n-1)/3),
// C = 2K+1 slots along y and z, H = K+1 along x, Q = C*H lines along z,
// M = C*Q modes per field.
struct BoxGeom {
  int n, K, C, H;
  long long Q, M;
};

// Coefficients of the IMEX update (Sec. 2.2).
struct StepCoef {
  double dt;       // time step
  double nu;       // 1 / Re
  double ch2_pe;   // Ch^2 / Pe
  double s;        // CH splitting coefficient
  double inv_pe;   // 1 / Pe
  double e_coef;   // (1 + s Ch^2) / Pe
  double inv_n3;   // forward normalisation 1 / n^3
  int ab1;         // 1: Adams-Bashforth order 1 (first step)
};

// Per-box device descriptor read by the step kernels (box = table[box0 + blockIdx.z]).
// bufa / bufb hold the step's intermediates (G and X in bufb, Y and W in bufa).
struct BoxDev {
  void* bufa;
  void* bufb;
  cpx<double>* state;
  cpx<double>* hist;
  StepCoef sc;
  double csig;     // (3 / sqrt 8) Ch / We
  cpx<double>* sphi0 = nullptr;   // if set, the z stage stores S_phi(0) here before zeroing it
};

// Batched transform along a strided axis: line l = o * inner + i holds
// element a at ((o * cnt + a) * inner + i), cnt = n_in on input, n_out on
// output (n: the full axis, 2K+1: the retained band).
struct LineArgs {
  int n_in, n_out;
  long long inner, nlines;
  long long in_fstride, out_fstride;
  unsigned fmap;   // input field of output field f in bits 4f..4f+3
  int dmask;       // bit f: multiply output field f by i k along the axis
  double scale;
};

// Real transforms along x: rows of n reals <-> rows of `cnt` complex
// (cnt = n/2+1 for the full half spectrum, K+1 for the band).
struct RowArgs {
  long long nrows;
  int n_in, n_out;
  long long in_fstride, out_fstride;
  double scale;
};

bool supported_n(int n);

template <typename T>
hipError_t launch_lines(int n, int dir, const cpx<T>* in, cpx<T>* out, const cpx<T>* tw, const LineArgs& a,
                        int nfield, hipStream_t st);
template <typename T>
hipError_t launch_rows(int n, int dir, const void* in, void* out, const cpx<T>* tw, const RowArgs& a, int nfield,
                       hipStream_t st);
// One stage of the step for boxes table[box0 .. box0+nbox-1], all of size n:
// stage 0 y-inverse, 1 x stage with products, 2 y-forward, 3 z stage with the
// update (do_update = 0: z-inverse of the state only).  variant selects the
// workgroup size 64 << variant.
constexpr int kStepVariants = 3;
template <typename T>
hipError_t launch_step_stage(int n, int stage, int variant, const BoxDev* table, int box0, int nbox,
                             const cpx<T>* tw, int do_update, hipStream_t st);
// The x stage of the step (x-inverse of u, v, w, phi, i kx phi (formed on
// load from phi), dy phi, dz phi; the 8 products; x-forward) on `rows` rows
// of length n (rows even): dev->bufa holds the 6 input fields [6][rows][n/2+1
// band entries K+1], dev->bufb receives the 8 products [8][rows][K+1]; kx =
// kxs k; dev->csig the capillary coefficient.  One descriptor (box0 = 0).
template <typename T>
hipError_t launch_xstage_rows(int n, const BoxDev* dev, const cpx<T>* tw, long long rows, double kxs,
                              hipStream_t st);
template <typename T>
hipError_t launch_expand(const cpx<T>* cmp, cpx<T>* full, const BoxGeom& g, int nf, hipStream_t st);
template <typename T>
hipError_t launch_compact(const cpx<T>* full, cpx<T>* cmp, const BoxGeom& g, int nf, hipStream_t st);
hipError_t launch_project(cpx<double>* u, const BoxGeom& g, hipStream_t st);
// exact cube of phi: a compact FP64 band converted to T (n entries); the
// pointwise cube of n values in place
template <typename T>
hipError_t launch_band_to(const cpx<double>* a, cpx<T>* out, long long n, hipStream_t st);
template <typename T>
hipError_t launch_cube(T* f, long long n, hipStream_t st);
// p_hat = k_i k_j T_ij / k^2 from the compact spectra [6][M] of the products
// (xx, yy, zz, xy, xz, yz), into p [M] (FP64)
template <typename T>
hipError_t launch_pressure_band(const cpx<T>* t6, const BoxGeom& g, cpx<double>* p, hipStream_t st);
template <typename T>
hipError_t launch_spec_finish(const cpx<T>* in, cpx<T>* out, const BoxGeom& g, int nf, int dealias, int axis,
                              double scale, hipStream_t st);
hipError_t launch_helmholtz_box(const cpx<double>* rhs, cpx<double>* out, const BoxGeom& g, double lam,
                                hipStream_t st);
hipError_t launch_index_maps(int* out, const BoxGeom& g, hipStream_t st);
// acc = (first ? 0 : acc) + scale |f| over n values
hipError_t launch_abs_accum(const double* f, double* acc, long long n, double scale, int first, hipStream_t st);
// out[0] = max of a[0..n) (a >= 0), two passes through part[max_blocks]
hipError_t launch_max(const double* a, long long n, double* part, int max_blocks, double* out, hipStream_t st);
hipError_t launch_diag(const cpx<double>* state, const BoxGeom& g, double* part, int max_blocks, double* out,
                       hipStream_t st);

}  // namespace psms
