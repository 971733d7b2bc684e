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
  int32_t n;         /* grid points per axis: 8,12,16,24,32,48,64,96,128,192,256 */
  int32_t precision; /* PSMS_FP64, or PSMS_MIXED: FP32 transforms and products,
                        FP64 state, RHS assembly, projection and update */
  int32_t cube;      /* phi^3 in the chemical potential (Sec. 2.1.1): 0 = the pointwise
                        cube on the n grid, then truncated to the 2/3 band (it aliases:
                        a cube is not dealiased by the 2/3 rule); 1 = the band of the
                        exact cube, formed on a padded grid m > 4K (the smallest
                        supported size; n <= 192; not for batches or the adjoint) */
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
  double cfl;        /* dt max_x (|u| + |v| + |w|) / dx, dx = 2 pi / n (physical grid) */
  double sphi0_re;   /* box: S_phi(k = 0) of the last step before it was set to zero (Sec. 2.2 */
  double sphi0_im;   /* step ii): every CH term is a divergence, so rounding level; 0 before a step */
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
 * system), CN + AB2 for u, IE + AB2 for phi.  Asynchronous, no allocation.
 * With graph replay enabled (psms_set_graphs) and a non-NULL stream, every
 * step after the first (Adams-Bashforth 1) one replays a captured hipGraph of
 * the step's four kernels; by default the kernels are launched directly. */
int psms_step(psms_ctx* c, int32_t nsteps);

/* Enable or disable (default) the graph replay of psms_step.  The replay saves
 * host launch work but not GPU time: on gfx950 with ROCm 7 the directly
 * launched step measured 5 to 6 percent faster at 128^3 (the replayed one
 * leaves longer gaps between the kernels). */
int psms_set_graphs(psms_ctx* c, int32_t enable);

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

/* The pressure of the current state (eq. cont): the field that the projection
 * of Sec. 2.2 removes from the nonlinear term S = div T of eqs. NSE and kort,
 * lap p = div S, i.e. p_hat = k_i k_j T_ij_hat / k^2 with p_hat(0) = 0, into
 * d_p [n][n][n/2+1] complex double (zero outside the band).  Products and
 * transforms in the context's precision, the division in FP64.  Asynchronous;
 * uses the step's scratch (the next step rebuilds its input).  For a resting
 * drop of radius R the jump between inside and outside is the Laplace
 * pressure 2 / (We R) (surface tension 1/We of the Korteweg force). */
int psms_pressure(psms_ctx* c, double* d_p);

/* The device-side index maps of the retained band, as the kernels use them:
 * for each band mode m (ordered [kz slot][ky slot][kx]), d_out[4m..4m+3] =
 * (kz, ky, kx, offset into the [n][n][n/2+1] half spectrum).  int32. */
int psms_index_maps(psms_ctx* c, int32_t* d_out);

/* Stage timing (the NVTX-range profiling of Sec. 3.3, with HIP events):
 * runs `nsteps` steps like psms_step, recording a HIP event on the
 * context's stream around each of the step's kernels, synchronises, and
 * writes the average duration in milliseconds of each stage to h_ms[0..3]:
 * y-inverse, x stage with products, y-forward, z stage with the update.
 * The steps are launched directly (events between kernels), never from a
 * graph: the kernels are the ones psms_step launches. */
int psms_stage_times(psms_ctx* c, int32_t nsteps, double* h_ms);

/* ---------------------------------------------------------------------------
 * Wall-normal (Chebyshev) operations of the channel, Sec. 2.2 and Sec. 3.2.
 * z in [-1, 1] is sampled at the Chebyshev-Gauss-Lobatto points
 * z_j = cos(pi j / nc), j = 0..nc (z_0 = +1), and f(z) = sum_n a_n T_n(z).
 * Data are nlines complex lines (one per Fourier pair (kx, ky)), stored
 * position-major: entry n of line l at [n][l] (nc+1 entries per line),
 * complex interleaved.  nc must make 2 nc a supported FFT length
 * (nc in {4,6,8,12,16,24,32,48,64,96,128,256}).  These calls are stateless:
 * they run on `stream` (a hipStream_t, NULL for the default stream) and
 * allocate nothing.
 * ------------------------------------------------------------------------- */
enum { PSMS_DIRICHLET = 1, PSMS_NEUMANN = 2 };

/* Chebyshev transform as a DCT-I through the FFT of the 2 nc-point even
 * extension (Sec. 3.2.1), applied to real and imaginary parts together.
 * dir = +1: values f_j -> coefficients a_n = 2/(nc cbar_n) sum_j f_j
 * cos(pi n j / nc) / cbar_j (cbar_0 = cbar_nc = 2, else 1); dir = -1:
 * coefficients -> values f_j = sum_n a_n cos(pi n j / nc).
 * precision PSMS_FP64: complex double data; PSMS_MIXED: complex float. */
int psms_cheb_transform(int32_t nc, int64_t nlines, int32_t dir, int32_t precision, const void* d_in, void* d_out,
                        void* stream);

/* Coefficients of df/dz (FP64), by c_{n-1} b_{n-1} = b_{n+1} + 2 n a_n,
 * b_nc = 0 (c_0 = 2).  d_in and d_out must not overlap. */
int psms_cheb_deriv(int32_t nc, int64_t nlines, const double* d_in, double* d_out, void* stream);

/* The wall-normal Helmholtz problems of Sec. 2.2 (one independent 1-D problem
 * per Fourier pair (kx, ky)): (D^2 - beta_l) f = g on each line by the Chebyshev-tau method in FP64,
 * rows n = 0..nc-2 of the equation (g entries n > nc-2 are ignored) and two
 * boundary rows: bc = PSMS_DIRICHLET: f(+1), f(-1); PSMS_NEUMANN: f'(+1),
 * f'(-1), given by d_bcval [nlines][2] complex (top, bottom), or zero if
 * NULL.  d_beta [nlines] >= 0 (a Neumann problem needs beta > 0).  d_work:
 * (nc+1) * nlines doubles of scratch.  d_rhs and d_out must not overlap. */
int psms_cheb_helmholtz(int32_t nc, int64_t nlines, const double* d_beta, int32_t bc, const double* d_bcval,
                        const double* d_rhs, double* d_out, double* d_work, void* stream);

/* For callers that cannot allocate device memory or hand over a workspace
 * (work recorded under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): psms_cheb_helmholtz without d_work.  The elimination
 * scratch is a device array owned by the library, PSMS_NOALLOC_SCRATCH_DOUBLES
 * doubles (8 MiB) on each GPU the call runs on, held until the process ends;
 * (nc+1) * nlines larger than that returns PSMS_E_WORKSPACE.  Nothing is
 * allocated and nothing needs clearing between calls.  Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (other streams or
 * threads) race: the caller must order them.  Other arguments, results and
 * errors as psms_cheb_helmholtz. */
#define PSMS_NOALLOC_SCRATCH_DOUBLES ((size_t)1 << 20)
int psms_cheb_helmholtz_noalloc(int32_t nc, int64_t nlines, const double* d_beta, int32_t bc, const double* d_bcval,
                                const double* d_rhs, double* d_out, void* stream);

/* The implicit wall-normal solves of one channel time step for every
 * (kx, ky) line (Sec. 2.2, items iv and v; eqs. omegaz, ww, omegadef,
 * phisplit), k^2 = kx^2 + ky^2:
 *   omega_z: (D^2 - (k^2 + beta_ns)) omega = g_om, omega(+-1) = 0;
 *   w:       (D^2 - (k^2 + beta_ns)) psi = g_w, (D^2 - k^2) w = psi with
 *            w(+-1) = w'(+-1) = 0, by the influence-matrix method (psi takes
 *            the two homogeneous solutions with unit value at one wall);
 *            w = 0 for k = 0;
 *   phi:     (D^2 - (k^2 + beta_a)) xi = g_phi, (D^2 - (k^2 + beta_b)) phi = xi,
 *            both with zero normal derivative at the walls (no-flux);
 *   u, v:    u = i (kx w' + ky omega)/k^2, v = i (ky w' - kx omega)/k^2
 *            (zero for k = 0: the mean flow is a separate Dirichlet problem).
 * All arrays [nc+1][nlines] complex double except d_kx, d_ky [nlines].
 * d_work: psms_wall_workspace_bytes bytes, 256-byte aligned. */
typedef struct psms_wall_args {
  int32_t nc;
  int32_t reserved;
  int64_t nlines;
  const double* d_kx;
  const double* d_ky;
  double beta_ns; /* 2 Re / dt for Crank-Nicolson */
  double beta_a;  /* the two factors of the implicit CH operator */
  double beta_b;
  const double* d_g_om;
  const double* d_g_w;
  const double* d_g_phi;
  double* d_om;
  double* d_w;
  double* d_phi;
  double* d_u;
  double* d_v;
} psms_wall_args;

int psms_wall_workspace_bytes(int32_t nc, int64_t nlines, size_t* bytes);
int psms_wall_solve(const psms_wall_args* a, void* d_work, size_t bytes, void* stream);

/* ---------------------------------------------------------------------------
 * The channel step (Sec. 2.1-2.2): x, y periodic (lengths lx, ly; Fourier, nx
 * and ny points), z in [-1, 1] between no-slip walls, or free-slip ones (see
 * free_slip) (Chebyshev-Gauss-Lobatto
 * points z_j = cos(pi j / nc), j = 0..nc).  The velocity is carried as the
 * wall-normal vorticity omega_z and velocity w (eqs. omegaz, ww, omegadef)
 * plus the mean velocities U(z), V(z); phi obeys the split CH equation
 * (eq. phisplit) with no flux through the walls.  One step: u, v from
 * continuity and eq. omegadef; u, v, w, phi, grad phi to physical space; the
 * products of eqs. NSE, kort, CHE (divergence form) at the collocation points;
 * back to spectral space with the 2/3 rule in x, y and in the Chebyshev index
 * (n <= floor((2 nc - 1)/3)); H_omega = (curl S)_z, H_w = lap_h S_z - D div_h S;
 * Adams-Bashforth (order 1 on the first step) with Crank-Nicolson viscous terms
 * and implicit Euler for the split CH operator, i.e. the wall-normal solves of
 * psms_wall_solve with beta_ns = 2 re / dt and the two CH factors, and the
 * Dirichlet (Neumann at a free-slip wall) mean-flow problem driven by
 * -dP/dx = forcing.  re is Re_tau = 1/nu.  In single phase, phi and its
 * history read back as zero.
 *
 * Spectral arrays are complex double [field][n][ky][kx] over the band
 * kx = 0..Kx, ky = 0..Ky, -Ky..-1 (Kx = floor((nx-1)/3), Ky = floor((ny-1)/3)),
 * n = 0..nc: the state is [3] = (omega_z, w, phi), the history (the previous
 * step's H_omega, H_w, S_phi) likewise; the mean lines are [2][nc+1] complex
 * (U, V) and their history (mean S_x, S_y).  Physical fields are real double
 * [z][y][x], x_i = lx i / nx, y_j = ly j / ny.
 * Transforms and products run in FP32 for PSMS_MIXED; the state, the
 * right-hand sides and every solve are FP64.
 * ------------------------------------------------------------------------- */
typedef struct psms_channel_params {
  int32_t nx, ny, nc; /* nx, ny as for psms_params.n; nc in {4 6 8 12 16 24 32 48 64 96 128 256} */
  int32_t precision;  /* PSMS_FP64 or PSMS_MIXED */
  double lx, ly;      /* periods in x and y */
  double re, we, ch, pe, dt;
  double s;           /* CH splitting coefficient; 0 selects sqrt(4 Pe / (Ch^2 dt)) */
  double forcing;     /* mean pressure gradient -dP/dx (1 in wall units) */
  int32_t single_phase; /* nonzero: Navier-Stokes only (the single-phase channel
                           timed in Sec. 3.4): phi is identically zero, the Korteweg stress and
                           the CH solves are left out, we, ch, pe, s are not used and
                           init_state accepts d_phi = NULL */
  int32_t free_slip;    /* bit 0: the top wall (z = +1), bit 1: the bottom wall
                           (z = -1) is free-slip (Sec. 2.1: w = 0, du/dz = dv/dz = 0,
                           hence omega_z' = 0, w'' = 0 and U' = V' = 0 there)
                           instead of no-slip; 0 is the no-slip channel */
} psms_channel_params;
typedef struct psms_channel psms_channel;

/* Device workspace of a context (owned by the caller, at least the bytes
 * reported, kept until psms_channel_destroy): the state, history and the
 * step's intermediates, and what create precomputes once because k^2 and the
 * time step are fixed: the homogeneous w solutions and their influence data
 * and, for nc <= 128 with the same condition at both walls, the elimination
 * factors of the six wall-normal problems (16 (nc/2 + 1) bytes per line and
 * parity each).  create runs on `stream` and synchronises. */
int psms_channel_workspace_bytes(const psms_channel_params* p, size_t* bytes);
int psms_channel_create(psms_channel** out, const psms_channel_params* p, void* d_workspace, size_t bytes,
                        void* stream);
/* State from physical u, v, w, phi ([nc+1][ny][nx] each, on the collocation
 * grid); the next step is Adams-Bashforth 1.  Synchronises; PSMS_E_NONFINITE if
 * an input value is not finite. */
int psms_channel_init_state(psms_channel* c, const double* d_u, const double* d_v, const double* d_w,
                            const double* d_phi);
/* State, mean lines and (for nstep > 0) history in the layouts above (in
 * single phase the phi parts are ignored and set to zero). */
int psms_channel_set_state(psms_channel* c, const double* d_state, const double* d_mean, const double* d_hist,
                           const double* d_hmean, int32_t nstep);
/* Advance nsteps steps (asynchronous).  With graph replay enabled
 * (psms_channel_set_graphs) and a non-NULL stream, every step after the first
 * (Adams-Bashforth 1) one replays a captured hipGraph of the step's launches;
 * by default they are launched directly. */
int psms_channel_step(psms_channel* c, int32_t nsteps);
/* Enable or disable (default) the graph replay of psms_channel_step (see
 * psms_set_graphs). */
int psms_channel_set_graphs(psms_channel* c, int32_t enable);
/* Diagnostics of the channel state into *h_out (synchronises the stream),
 * volume averages over [0, lx) x [0, ly) x [-1, 1] (eqs. cont and CHE):
 * mean_phi = <phi>; ke = 1/2 <|u|^2>; grad2 = <|grad phi|^2> (Parseval in x and
 * y, the exact Chebyshev integral in z); max_div = max |i kx u + i ky v + D w|
 * over the band (continuity); nonfinite = number of non-finite entries of the
 * state and mean lines; cfl = dt max (|u| / dx + |v| / dy + |w| / dz_j) over the
 * collocation grid, dx = lx / nx, dy = ly / ny, dz_j the local spacing of the
 * points ((z_{j-1} - z_{j+1}) / 2, one-sided at the walls).  Uses the step's
 * scratch (the next step rebuilds it).  psms_channel_init_state runs it and
 * returns PSMS_E_NONFINITE if an input value is not finite. */
int psms_channel_diagnostics(psms_channel* c, psms_diag* h_out);
/* d_hist and d_hmean may be NULL. */
int psms_channel_get_state(psms_channel* c, double* d_state, double* d_mean, double* d_hist, double* d_hmean);
int psms_channel_destroy(psms_channel* c);

/* ---------------------------------------------------------------------------
 * Batches of independent boxes of uneven size (each with its own N, Re, We,
 * Ch, Pe, dt, s; one precision for the whole batch).  Boxes of equal N form a
 * group; each stage kernel is launched once per group and advances all its
 * boxes (blockIdx.z indexes a device table of box descriptors).  On request
 * (psms_batch_step's use_graph), after the first (Adams-Bashforth 1) step one
 * step of all groups is captured in a hipGraph and replayed, so a step costs
 * one graph launch.
 * ------------------------------------------------------------------------- */
typedef struct psms_batch psms_batch;

/* Workspace for nbox boxes with parameters p[0..nbox-1] (host only). */
int psms_batch_workspace_bytes(int32_t nbox, const psms_params* p, size_t* bytes);
/* Create: validates every p[i], checks the device, carves the workspace.
 * Graph replay needs a non-NULL stream (a stream that can be captured). */
int psms_batch_create(psms_batch** out, int32_t nbox, const psms_params* p, void* d_workspace, size_t bytes,
                      void* stream);
/* psms_init_state / psms_get_state / psms_diagnostics of box `box`. */
int psms_batch_init_state(psms_batch* b, int32_t box, const double* d_u, const double* d_phi);
int psms_batch_get_state(psms_batch* b, int32_t box, double* d_uhat, double* d_phihat);
int psms_batch_diagnostics(psms_batch* b, int32_t box, psms_diag* h_out);
/* Advance every box by nsteps.  use_graph != 0 replays a captured graph for
 * every step after the first (needs a non-NULL stream). */
int psms_batch_step(psms_batch* b, int32_t nsteps, int32_t use_graph);
/* Groups in ascending N: *h_ngroups, and per group its N and box count
 * (h_n, h_count may be NULL; otherwise they hold *h_ngroups entries). */
int psms_batch_groups(const psms_batch* b, int32_t* h_ngroups, int32_t* h_n, int32_t* h_count);
/* Workgroup-size variant (0, 1, 2: 64, 128, 256 threads) of each stage of each
 * group, h_variants[4 * group + stage]. */
int psms_batch_set_variants(psms_batch* b, const int32_t* h_variants);
/* Autotuner: times every variant of every stage of every group (reps
 * launches each, HIP events on the batch stream) and keeps the fastest.
 * Must run before any init_state (it zeroes the boxes' state and
 * intermediates).  h_variants [4 * ngroups] (nullable) receives the choice,
 * h_ms [4 * ngroups * 3] (nullable) the average ms of every variant. */
int psms_batch_autotune(psms_batch* b, int32_t reps, int32_t* h_variants, double* h_ms);
int psms_batch_destroy(psms_batch* b);

/* ---------------------------------------------------------------------------
 * Discrete adjoint (discretise-then-differentiate) of the box step, for the
 * objective J = int |grad phi|^2 dV + 1/2 int |u|^2 dV at the final step:
 * gradients with respect to the initial phase field (a grid array) and the
 * Weber number (eq. We).  The primal run (precision of p) stores the FP64
 * state and history every seg_len steps; the backward sweep recomputes each
 * segment in FP64 and applies the transposed step
 *   Sbar = alpha B lam + mu, mu <- beta B lam, lam <- A lam + (dR/dx)^T Sbar,
 *   dJ/dWe += (dR/dWe)^T Sbar
 * (A, B the per-mode implicit factors, alpha, beta the Adams-Bashforth
 * weights, R the projected nonlinear terms) under the half-spectrum inner
 * product sum_k w_k Re(conj a_k b_k), w = 1 at kx = 0 and 2 otherwise.
 * ------------------------------------------------------------------------- */
typedef struct psms_adjoint psms_adjoint;

int psms_adjoint_workspace_bytes(const psms_params* p, int32_t max_steps, int32_t seg_len, size_t* bytes);
int psms_adjoint_create(psms_adjoint** out, const psms_params* p, int32_t max_steps, int32_t seg_len,
                        void* d_workspace, size_t bytes, void* stream);
/* Primal run from the physical fields d_u [3][n][n][n], d_phi [n][n][n]
 * (double) for nsteps <= max_steps; writes J to *h_J (synchronises). */
int psms_adjoint_forward(psms_adjoint* a, const double* d_u0, const double* d_phi0, int32_t nsteps, double* h_J);
/* Backward sweep of the last forward run: d_dphi0 [n][n][n] receives dJ/dphi0
 * on the grid, *h_dwe dJ/dWe (synchronises). */
int psms_adjoint_backward(psms_adjoint* a, double* d_dphi0, double* h_dwe);
int psms_adjoint_destroy(psms_adjoint* a);

/* Number of retained modes per field, (2K+1)^2 (K+1). */
int64_t psms_band_modes(const psms_ctx* c);

int psms_destroy(psms_ctx* c);
const char* psms_last_error(void);
const char* psms_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSMS_H */
