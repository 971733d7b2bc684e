// Launchers of the pointwise and per-mode kernels of the channel step (Sec. 2.2).
// Spectral arrays are [field][n][line], line = iy * Hx + ix over the 2/3 band
// (ky = 0..Ky, -Ky..-1; kx = 0..Kx), n the Chebyshev index 0..nc; physical
// arrays are [field][z][y][x] at the Chebyshev-Gauss-Lobatto points in z.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_engine.hpp"

namespace psms {

// Geometry and coefficients of one channel step.
struct ChanGeom {
  int nx, ny, nc;
  int Kx, Hx, Ky, Cy, Kz;  // band cut-offs; Kz: Chebyshev modes kept in the products
  long long NL;            // lines Cy * Hx
  long long NZL;           // (nc + 1) * NL
  long long P;             // (nc + 1) * ny * nx physical points
  int sp;                  // single phase: phi = 0, no Korteweg stress, no CH terms
  int nf_in, nf_out;       // fields transformed to physical space / back (7, 8; 3, 6 single phase)
};

struct ChanCoef {
  double re, beta;     // Re_tau and 2 Re / dt
  double inv_pe, e_coef, g_phi_scale, dt, forcing;
  double csig;
  int ab1;
};

// the 7 spectral fields u, v, w, phi, i kx phi, i ky phi, D phi (precision T);
// with six, the 6 fields u, v, w, phi, i ky phi, D phi (the fused x stage
// forms i kx phi itself); u, v, w only in single phase
template <typename T>
hipError_t launch_ch_fields(const ChanGeom& g, const cpx<double>* om, const cpx<double>* w, const cpx<double>* phi,
                            const cpx<double>* dw, const cpx<double>* dphi, const cpx<double>* mean, const double* kx,
                            const double* ky, cpx<T>* out, hipStream_t st, int six = 0);
// pointwise products, 7 physical fields in, 8 out (in place, [8][P]); single
// phase 3 in, the 6 components of -u_i u_j out
template <typename T>
hipError_t launch_ch_products(const ChanGeom& g, T* f, double csig, hipStream_t st);
// H_omega, H_w, S_phi; Adams-Bashforth with the history (then overwritten);
// the right-hand sides g_om, g_w, g_phi of the wall-normal solves; the mean
// lines' H and right-hand sides.
struct ChanAssembleArgs {
  const cpx<double>* d3;      // [3][NZL] D T_xz, D T_yz, D T_zz (S = div T is formed from them and R)
  const cpx<double>* dq;      // D Q, Q = i kx S_x + i ky S_y
  const cpx<double>* R;       // products T_xx T_yy T_zz T_xy T_xz T_yz, field 6 = a, 7 = c
  const cpx<double>* lsphi;   // lap (c / Pe - (1 + s Ch^2) / Pe phi^n)
  const cpx<double>* phi;     // phi^n
  const cpx<double>* lom;     // lap omega^n + beta omega^n
  const cpx<double>* lpsi;    // lap psi + beta psi, psi = lap w^n
  const double* kx;
  const double* ky;
  cpx<double>* hist;          // [3][NZL] H_omega, H_w, S_phi of the previous step (in/out)
  cpx<double>* g;             // [3][NZL] g_om, g_w, g_phi
  const cpx<double>* mean;    // [nc+1][2] U, V
  const cpx<double>* d2mean;  // [nc+1][2]
  cpx<double>* hmean;         // [nc+1][2] (in/out)
  cpx<double>* gmean;         // [nc+1][2]
};
hipError_t launch_ch_assemble(const ChanGeom& g, const ChanCoef& c, const ChanAssembleArgs& a, hipStream_t st);
// initial state from the 4 transformed physical fields u, v, w, phi ([4][NZL], FP64;
// 3 in single phase, phi set to zero)
hipError_t launch_ch_init(const ChanGeom& g, const cpx<double>* U4, const double* kx, const double* ky,
                          cpx<double>* om, cpx<double>* w, cpx<double>* phi, cpx<double>* mean, hipStream_t st);
// diagnostics of the state (volume averages; eqs. cont and CHE): per-line partial
// sums (at most max_blocks blocks of 256 lines' worth of work, part[4 * block]),
// the CFL maxima of physical FP64 u, v, w [3][P] (part[4 * block + 2]), and the
// final reduction out[0..5] = mean phi, kinetic energy, <|grad phi|^2>,
// max |i kx u + i ky v + D w|, non-finite entries, CFL
hipError_t launch_ch_diag_lines(const ChanGeom& g, const cpx<double>* om, const cpx<double>* w, const cpx<double>* phi,
                                const cpx<double>* dw, const cpx<double>* dphi, const cpx<double>* mean,
                                const double* kx, const double* ky, double* part, int max_blocks, hipStream_t st);
hipError_t launch_ch_cfl(const ChanGeom& g, const double* f, double inv_dx, double inv_dy, double dt, double* part,
                         int max_blocks, hipStream_t st);
hipError_t launch_ch_diag_final(const ChanGeom& g, const double* part, int nb1, const double* part2, int nb2,
                                const cpx<double>* phi, double* out, hipStream_t st);
// mean lines: [2][nc+1] (caller) <-> [nc+1][2] (internal); dir > 0 copies into internal
hipError_t launch_ch_mean_io(const ChanGeom& g, const cpx<double>* in, cpx<double>* out, int dir, hipStream_t st);

}  // namespace psms
