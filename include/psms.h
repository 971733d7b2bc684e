/*
 * psms: pseudo-spectral multiphase step for one AMD MI355X (gfx950).
 *
 * C ABI of one coupled Navier-Stokes + Cahn-Hilliard timestep of the method
 * of Roccon, "A GPU-ready pseudo-spectral method for direct numerical
 * simulations of multiphase turbulence" (arXiv 2406.01322), on the triply
 * periodic box [0, 2 pi)^3 (the Fourier x Fourier x Fourier reduction of the
 * paper's Fourier x Fourier x Chebyshev channel).
 *
 * Equations (Sec. 2.1): Cahn-Hilliard (eq. CHE) with the chemical potential
 * mu = phi^3 - phi - Ch^2 lap(phi); continuity (eq. cont) and Navier-Stokes
 * (eq. NSE) with the Korteweg surface force (3/sqrt 8)(Ch/We) div(|grad phi|^2 I
 * - grad phi (x) grad phi) (eq. kort).  Scheme (Sec. 2.2): pseudo-spectral in
 * space, nonlinear terms formed in physical space, IMEX in time with
 * Adams-Bashforth for the nonlinear terms, Crank-Nicolson for the viscous
 * term, implicit Euler for the split CH operator (eq. phisplit).
 *
 * Conventions shared by every call:
 *  - Physical fields are real arrays [z][y][x] (x fastest) of n^3 points,
 *    x_j = 2 pi j / n.
 *  - Spectral fields are the half spectrum [kz][ky][kx], kz, ky in FFT order
 *    (0..n/2-1, -n/2..-1), kx = 0..n/2, complex values interleaved (re, im):
 *    u(x) = sum_k u_k exp(i k.x); the forward transform carries 1/n^3 and a
 *    derivative d/dx_j is multiplication by i k_j.
 *  - The state is kept only on the 2/3-rule band |kx|,|ky|,|kz| <= K with
 *    K = floor((n-1)/3); entries outside the band are zero on output and
 *    ignored on input.
 *  - All pointers prefixed d_ are device pointers on the current HIP device,
 *    256-byte aligned, owned by the caller and required to stay valid while
 *    the context uses them.  h_ pointers are host memory.
 *  - Every call is asynchronous on the context's stream unless stated.  The
 *    library never allocates device memory and never synchronises inside
 *    psms_step.
 *  - Functions return PSMS_OK (0) or a negative error code; psms_last_error()
 *    returns the calling thread's last message.  Kernel faults surface at the
 *    next synchronising call.
 */
#ifndef PSMS_H
#define PSMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PSMS_OK = 0,
  PSMS_E_INVAL = -1,      /* invalid argument or parameter */
  PSMS_E_WORKSPACE = -2,  /* workspace too small or misaligned */
  PSMS_E_DEVICE = -3,     /* no usable gfx950 device */
  PSMS_E_NOTSUP = -4,     /* valid but unsupported configuration */
  PSMS_E_NONFINITE = -5,  /* non-finite value detected */
  PSMS_E_STATE = -6,      /* call out of order (e.g. step before init) */
  PSMS_E_LAUNCH = -7      /* a HIP call or kernel launch failed */
};

enum { PSMS_BOX = 0, PSMS_CHANNEL = 1 };
enum { PSMS_FP64 = 0, PSMS_MIXED = 1 };

/* psms_transform flags */
enum {
  PSMS_DEALIAS = 1u, /* zero every mode outside the 2/3 band */
  PSMS_DERIV_X = 2u, /* multiply the spectrum by i kx */
  PSMS_DERIV_Y = 4u, /* multiply the spectrum by i ky */
  PSMS_DERIV_Z = 8u  /* multiply the spectrum by i kz */
};

/* Problem parameters (Sec. 2.1 dimensionless numbers and the time step). */
typedef struct psms_params {
  int32_t geometry;  /* PSMS_BOX (PSMS_CHANNEL returns PSMS_E_NOTSUP) */
  int32_t n;         /* grid points per axis: 8,12,16,24,32,48,64,96,128,192,256,384,512 */
  int32_t precision; /* PSMS_FP64, or PSMS_MIXED: FP32 transforms and products,
                        FP64 state, RHS assembly, projection and update */
  int32_t reserved;  /* must be 0 */
  double re;         /* Reynolds number Re (eq. Re) > 0 */
  double we;         /* Weber number We (eq. We) > 0 */
  double ch;         /* Cahn number Ch > 0 */
  double pe;         /* Peclet number Pe > 0 */
  double dt;         /* time step > 0 */
  double s;          /* CH splitting coefficient of eq. phisplit; <= 0 selects
                        sqrt(4 Pe / (Ch^2 dt)), the smallest s for which the
                        implicit CH operator factors into two real Helmholtz
                        operators */
} psms_params;

/* Volume-averaged diagnostics of the current state. */
typedef struct psms_diag {
  double mean_phi;   /* <phi> = phi_hat(0) */
  double ke;         /* 1/2 <|u|^2> */
  double grad2;      /* <|grad phi|^2> */
  double max_div;    /* max_k |k . u_hat(k)| (continuity, eq. cont) */
  int32_t nonfinite; /* number of modes holding a non-finite value */
  int32_t nstep;     /* steps taken since init_state / set_state(nstep) */
} psms_diag;

typedef struct psms_ctx psms_ctx;

/* Device workspace size for the parameters, in bytes.  Host only. */
int psms_workspace_bytes(const psms_params* p, size_t* bytes);

/* Create a context.  Validates p, checks that the current device is gfx950,
 * carves the caller's workspace (d_workspace, `bytes` >= psms_workspace_bytes)
 * and uploads the FFT twiddle tables (computed in FP64 on the host).
 * `stream` is a hipStream_t (NULL: the default stream).  The context owns
 * only its host-side struct; free it with psms_destroy. */
int psms_create(psms_ctx** out, const psms_params* p, void* d_workspace, size_t bytes, void* stream);

/* Step (i) of Sec. 2.2: forward-transform the physical fields d_u
 * [3][n][n][n] (u, v, w) and d_phi [n][n][n] (double), truncate to the 2/3
 * band and project the velocity onto divergence-free fields.  The history is
 * cleared, so the next step uses Adams-Bashforth order 1.  Returns
 * PSMS_E_NONFINITE (synchronising) if an input value is not finite. */
int psms_init_state(psms_ctx* c, const double* d_u, const double* d_phi);

/* Load a spectral state: d_uhat [3][n][n][n/2+1] and d_phihat [n][n][n/2+1]
 * complex double (interleaved).  d_hist [4][n][n][n/2+1] holds the projected
 * NS right-hand side and S_phi of the previous step (may be NULL when
 * nstep == 0).  nstep = 0 makes the next step Adams-Bashforth order 1. */
int psms_set_state(psms_ctx* c, const double* d_uhat, const double* d_phihat, const double* d_hist, int32_t nstep);

/* Steps (ii)-(v) of Sec. 2.2, `nsteps` times: nonlinear terms in physical
 * space, Leray projection (the periodic form of the velocity-vorticity
 * system), CN + AB2 for u, IE + AB2 for phi.  Asynchronous, no allocation. */
int psms_step(psms_ctx* c, int32_t nsteps);

/* Copy the state out in the layouts of psms_set_state; d_hist may be NULL. */
int psms_get_state(psms_ctx* c, double* d_uhat, double* d_phihat, double* d_hist);

/* Batched 3-D transforms of Sec. 3.2.1.  dir = +1: physical -> spectral,
 * d_in [nfield][n][n][n] real, d_out [nfield][n][n][n/2+1] complex, with
 * 1/n^3.  dir = -1: spectral -> physical, unnormalised, the kx = 0 and
 * kx = n/2 entries taken as real.  Element type: double for PSMS_FP64
 * contexts, float for PSMS_MIXED.  flags: PSMS_DEALIAS and at most one
 * PSMS_DERIV_*, applied to the spectrum.  Uses the context's scratch. */
int psms_transform(psms_ctx* c, int32_t dir, int32_t nfield, const void* d_in, void* d_out, uint32_t flags);

/* Helmholtz problems of Sec. 2.2: solve (lap - lambda_f) f = g_f for
 * nfield fields given their spectra d_rhs [nfield][n][n][n/2+1] (complex
 * double).  On the box: f_hat = -g_hat / (k^2 + lambda_f); the mode with
 * k^2 + lambda_f = 0 is set to zero.  h_lambda[nfield] >= 0 (host). */
int psms_solve_helmholtz(psms_ctx* c, int32_t nfield, const double* h_lambda, const double* d_rhs, double* d_out);

/* Diagnostics of the current state into *h_out (synchronises the stream). */
int psms_diagnostics(psms_ctx* c, psms_diag* h_out);

/* The device-side index maps of the retained band, as the kernels use them:
 * for each band mode m (ordered [kz slot][ky slot][kx]), d_out[4m..4m+3] =
 * (kz, ky, kx, offset into the [n][n][n/2+1] half spectrum).  int32. */
int psms_index_maps(psms_ctx* c, int32_t* d_out);

/* Stage timing (the NVTX-range profiling of Sec. 3.3, with HIP events):
 * runs `nsteps` steps like psms_step, recording a HIP event on the
 * context's stream around each of the step's kernels, synchronises, and
 * writes the average duration in milliseconds of each stage to h_ms[0..3]:
 * y-inverse, x stage with products, y-forward, z stage with the update. */
int psms_stage_times(psms_ctx* c, int32_t nsteps, double* h_ms);

/* Number of retained modes per field, (2K+1)^2 (K+1). */
int64_t psms_band_modes(const psms_ctx* c);

int psms_destroy(psms_ctx* c);
const char* psms_last_error(void);
const char* psms_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSMS_H */
