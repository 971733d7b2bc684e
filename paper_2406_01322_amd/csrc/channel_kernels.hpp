// Launchers of the wall-normal (Chebyshev) kernels.  Lines are stored
// position-major: coefficient / point n of line l at n * nlines + l.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_engine.hpp"

namespace psms {

bool supported_nc(int nc);
constexpr int kTauQMax = 256;   // largest nc of the tau solves

template <typename T>
hipError_t launch_dct(int nc, const cpx<T>* in, cpx<T>* out, long long nlines, int dir, hipStream_t st);
// nfield fields fstride elements apart in one launch; tw: exp(-2 pi i m / (2 nc)),
// m < 2 nc, or NULL (computed in the kernel).  out64 (forward only): write the
// coefficients to it in FP64 instead of to out, those with n > kz as zero.
template <typename T>
hipError_t launch_dct_fields(int nc, const cpx<T>* in, cpx<T>* out, long long nlines, long long fstride, int nfield,
                             const cpx<T>* tw, int dir, hipStream_t st, cpx<double>* out64 = nullptr, int kz = 0);
// The inverse transform of the channel step's six fields u, v, w, phi, i ky phi,
// D phi ([6][n][line] out, fstride apart), each value formed from the FP64
// state as it is loaded (u, v by continuity and the definition of omega_z;
// the mean line, l = 0, carries U, V from mean [n][2]).
struct ChanFieldSrc {
  const cpx<double>* om;
  const cpx<double>* w;
  const cpx<double>* phi;
  const cpx<double>* dw;
  const cpx<double>* dphi;
  const cpx<double>* mean;
  const double* kx;
  const double* ky;
  long long nlines;
};
template <typename T>
hipError_t launch_dct_chfields(int nc, const ChanFieldSrc& fs, cpx<T>* out, long long fstride, const cpx<T>* tw,
                               hipStream_t st);
hipError_t launch_chebd(const cpx<double>* a, cpx<double>* d, int nc, long long nlines, hipStream_t st);
// up to kChebBatchMax arrays of the same lines per launch: out[j] = D in[j]
// (bit j of lapmask clear) or D^2 in[j] - k^2 in[j] (bit j set)
constexpr int kChebBatchMax = 8;
struct ChebBatch {
  const cpx<double>* in[kChebBatchMax];
  cpx<double>* out[kChebBatchMax];
  cpx<double>* out2[kChebBatchMax];   // D^2 - k^2 arrays: (D^2 - k^2)^2 in[j] as well where non-NULL
  long long nl[kChebBatchMax];        // lines of array j if nonzero (at most the launch's nlines), else nlines
  int nok;                            // bit j: k^2 = 0 for array j (lines that are not (kx, ky) pairs)
  // D^2 - k^2 arrays only: the input is w1 in + w2 in2 where in2[j] is non-NULL,
  // out[j] (if non-NULL) receives (D^2 - k^2) x + addb x, out2[j] (D^2 - k^2)^2 x
  // + addb2 (D^2 - k^2) x
  const cpx<double>* in2[kChebBatchMax];
  double w1[kChebBatchMax], w2[kChebBatchMax], addb[kChebBatchMax], addb2[kChebBatchMax];
  int n;
};
hipError_t launch_cheb_batch(const ChebBatch& b, int nc, long long nlines, const double* kx, const double* ky,
                             int lapmask, hipStream_t st);
// out = D Q, Q = i kx S_x + i ky S_y formed from T_xx, T_yy, T_xy, D T_xz, D T_yz
// (S_x = i kx T_xx + i ky T_xy + D T_xz, S_y = i kx T_xy + i ky T_yy + D T_yz)
struct ChebQ {
  const cpx<double>* txx;
  const cpx<double>* tyy;
  const cpx<double>* txy;
  const cpx<double>* dxz;
  const cpx<double>* dyz;
};
hipError_t launch_chebd_q(const ChebQ& in, int nc, long long nlines, const double* kx, const double* ky,
                          cpx<double>* out, hipStream_t st);
// out = D^2 a - (kx^2 + ky^2) a per line (k^2 = 0 if kx is NULL)
hipError_t launch_cheb_lap(const cpx<double>* a, cpx<double>* out, int nc, long long nlines, const double* kx,
                           const double* ky, hipStream_t st);
hipError_t launch_helm(const cpx<double>* g, cpx<double>* f, double* xw, int nc, long long nlines,
                       const double* beta_line, double beta_add, const double* kx, const double* ky, int neumann,
                       const cpx<double>* bcv, cpx<double> top_c, cpx<double> bot_c, hipStream_t st);
// independent tau problems (D^2 - (beta_add + kx^2 + ky^2)) f = g of one launch;
// kx = NULL means k^2 = 0, g = NULL a zero right-hand side; xw: (nc+1) nlines
// doubles of scratch per problem
constexpr int kHelmBatchMax = 4;
struct HelmProblem {
  const cpx<double>* g;
  cpx<double>* f;
  double* xw;
  long long nlines;
  double beta_add;
  const double* kx;
  const double* ky;
  int bc;   // bit 0: Neumann at the top wall (z = +1), bit 1: at the bottom wall; else Dirichlet
  cpx<double> top_c, bot_c;
  // optional (on-chip path only, see helm_fuses_influence): the clamped-wall
  // influence correction of the w problem between two no-slip walls, f + c_p wh
  // per parity p with c_p making sum_{n = p mod 2} n^2 f_n = 0 (f' = 0 at both
  // walls); wh [nc+1][nlines] the parity-split homogeneous solutions, mh [2][nlines]
  // their sums sum n^2 wh_n; f = 0 on the line kx = ky = 0
  const double* wh = nullptr;
  const double* mh = nullptr;
  // optional (nc with helm_fuses_influence(nc), bc 0 or 3): the elimination
  // factors of the problem's beta_add + k^2 and wall conditions, from
  // launch_helm_factors (helm_factor_doubles(nc, nlines) doubles); the
  // problem's beta_add, kx, ky, bc and nlines must be those the factors were
  // made with.  Given for all problems of a batch or for none; then the batch
  // is solved in pieces (k_helm_pieces).
  const double* fac = nullptr;
};
struct HelmBatch {
  HelmProblem p[kHelmBatchMax];
  int np;
};
hipError_t launch_helm_batch(const HelmBatch& b, int nc, hipStream_t st);
// whether launch_helm_batch keeps the chains on chip for this nc (same condition
// at both walls), the only path that applies HelmProblem::wh
bool helm_fuses_influence(int nc);
// the factors of problem P (its g, f, top_c, bot_c and influence fields are
// not used) for nc with helm_fuses_influence(nc) and the same condition at
// both walls (bc 0 or 3)
hipError_t launch_helm_factors(const HelmProblem& P, int nc, double* fac, hipStream_t st);
size_t helm_factor_doubles(int nc, long long nlines);
// the parity-split homogeneous solutions of the clamped w problem between two
// no-slip walls: wh_n = (w_t + w_b)_n for even n, (w_t - w_b)_n for odd n (real),
// and mh[p][l] = sum_{n = p mod 2} n^2 wh_n
hipError_t launch_influence_parity_pre(const cpx<double>* wt, const cpx<double>* wb, int nc, long long nlines,
                                       double* wh, double* mh, hipStream_t st);
hipError_t launch_influence(cpx<double>* wp, const cpx<double>* wt, const cpx<double>* wb, int nc, long long nlines,
                            const double* kx, const double* ky, hipStream_t st);
// influence matrix with fixed homogeneous solutions: M [4][nlines] once, then
// the combination per solve.  free_slip bit 0 (top wall) / bit 1 (bottom wall):
// that wall imposes w'' = 0 through psi = 0 instead of w' = 0, so its
// homogeneous solution takes no part (its row of M is the identity).
hipError_t launch_influence_pre(const cpx<double>* wt, const cpx<double>* wb, int nc, long long nlines, double* M,
                                int free_slip, hipStream_t st);
hipError_t launch_influence_apply(cpx<double>* wp, const cpx<double>* wt, const cpx<double>* wb, const double* M,
                                  int nc, long long nlines, const double* kx, const double* ky, int free_slip,
                                  hipStream_t st);
hipError_t launch_uv(const cpx<double>* om, const cpx<double>* dw, cpx<double>* u, cpx<double>* v, int nc,
                     long long nlines, const double* kx, const double* ky, hipStream_t st);

}  // namespace psms
