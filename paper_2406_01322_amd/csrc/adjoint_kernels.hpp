// Launchers of the discrete-adjoint kernels of the box step (FP64).
#pragma once

#include <hip/hip_runtime.h>

#include "fft_engine.hpp"

namespace psms {

// Coefficients of one adjoint step.  alpha, beta: the Adams-Bashforth weights
// of the forward step being transposed (1, 0 for the first step; 1.5, -0.5).
struct AdjCoef {
  double dt, nu, ch2_pe, s, inv_pe, e_coef, inv_n3;
  double alpha, beta;
};

// stage 0: k_zadj_in (lam, mu updated; out = [8][n][C][H] cotangents z-inverted)
// stage 1: k_xadj    (a = forward y-inverse [6][n][n][H], b = cotangents [8][n][n][H],
//                     out = [7][n][n][H], part[adj_xblocks(n)] We-term partial sums)
// stage 2: k_zadj_out (a = [7][n][C][H]; lam += ...)
hipError_t launch_adj_stage(int n, int stage, cpx<double>* lam, cpx<double>* mu, const cpx<double>* a,
                            const cpx<double>* b, cpx<double>* out, const cpx<double>* tw, const AdjCoef& ac,
                            double csig, double* part, hipStream_t st);
int adj_xblocks(int n);
hipError_t launch_adj_terminal(const cpx<double>* state, cpx<double>* lam, cpx<double>* mu, int K, int C, int H,
                               long long M, double vol, hipStream_t st);
hipError_t launch_adj_sum(const double* part, int n, double scale, double* acc, hipStream_t st);

}  // namespace psms
