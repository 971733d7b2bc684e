// Pointwise and per-mode kernels of the channel step (Sec. 2.2): the fields to
// transform, the products, and the assembly of the wall-normal right-hand
// sides.  The transforms themselves (Fourier lines and rows, the DCT-I) and
// the wall-normal solves are the kernels of box_kernels.hip and
// channel_kernels.hip; every kernel here is one grid-stride pass over
// contiguous arrays (HBM-bound).
#include <hip/hip_runtime.h>

#include "channel_step_kernels.hpp"

namespace psms {

namespace {

constexpr int kThreads = 256;

unsigned blocks_for(long long n) {
  long long b = (n + kThreads - 1) / kThreads;
  if (b > 65536) b = 65536;
  return unsigned(b < 1 ? 1 : b);
}

__device__ __forceinline__ cpx<double> ti(double k, cpx<double> a) { return {-k * a.im, k * a.re}; }  // i k a
__device__ __forceinline__ cpx<double> add(cpx<double> a, cpx<double> b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cpx<double> sub(cpx<double> a, cpx<double> b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cpx<double> scl(double s, cpx<double> a) { return {s * a.re, s * a.im}; }

#define PSMS_GRID_LOOP(id, n) \
  for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < (n); id += (long long)gridDim.x * blockDim.x)

template <typename T>
__global__ void k_ch_fields(ChanGeom g, const cpx<double>* __restrict__ om, const cpx<double>* __restrict__ w,
                            const cpx<double>* __restrict__ phi, const cpx<double>* __restrict__ dw,
                            const cpx<double>* __restrict__ dphi, const cpx<double>* __restrict__ mean,
                            const double* __restrict__ kxl, const double* __restrict__ kyl, cpx<T>* __restrict__ out,
                            int six) {
  PSMS_GRID_LOOP(id, g.NZL) {
    const long long l = id % g.NL, n = id / g.NL;
    const double kx = kxl[l], ky = kyl[l];
    cpx<double> u, v;
    if (l == 0) {  // the mean line carries U, V
      u = mean[2 * n];
      v = mean[2 * n + 1];
    } else {       // continuity and the definition of omega_z (eq. omegadef)
      const double ik2 = 1.0 / (kx * kx + ky * ky);
      const cpx<double> o = om[id], d = dw[id];
      u = scl(ik2, ti(1.0, add(scl(kx, d), scl(ky, o))));
      v = scl(ik2, ti(1.0, sub(scl(ky, d), scl(kx, o))));
    }
    const cpx<double> ww = w[id];
    out[id] = cpx<T>{T(u.re), T(u.im)};
    out[g.NZL + id] = cpx<T>{T(v.re), T(v.im)};
    out[2 * g.NZL + id] = cpx<T>{T(ww.re), T(ww.im)};
    if (!g.sp) {
      const cpx<double> p = phi[id];
      if (six) {   // dx phi is formed by the x stage
        const cpx<double> f[3] = {p, ti(ky, p), dphi[id]};
#pragma unroll
        for (int k = 0; k < 3; ++k) out[(k + 3) * g.NZL + id] = cpx<T>{T(f[k].re), T(f[k].im)};
      } else {
        const cpx<double> f[4] = {p, ti(kx, p), ti(ky, p), dphi[id]};
#pragma unroll
        for (int k = 0; k < 4; ++k) out[(k + 3) * g.NZL + id] = cpx<T>{T(f[k].re), T(f[k].im)};
      }
    }
  }
}

template <typename T>
__global__ void k_ch_products(ChanGeom g, T* __restrict__ f, T cs) {
  if (g.sp) {
    PSMS_GRID_LOOP(id, g.P) {
      const T u = f[id], v = f[g.P + id], w = f[2 * g.P + id];
      f[id] = -u * u;
      f[g.P + id] = -v * v;
      f[2 * g.P + id] = -w * w;
      f[3 * g.P + id] = -u * v;
      f[4 * g.P + id] = -u * w;
      f[5 * g.P + id] = -v * w;
    }
    return;
  }
  PSMS_GRID_LOOP(id, g.P) {
    const T u = f[id], v = f[g.P + id], w = f[2 * g.P + id], p = f[3 * g.P + id];
    const T gx = f[4 * g.P + id], gy = f[5 * g.P + id], gz = f[6 * g.P + id];
    f[id] = -u * u + cs * (gy * gy + gz * gz);          // T_xx
    f[g.P + id] = -v * v + cs * (gx * gx + gz * gz);    // T_yy
    f[2 * g.P + id] = -w * w + cs * (gx * gx + gy * gy);  // T_zz
    f[3 * g.P + id] = -u * v - cs * gx * gy;            // T_xy
    f[4 * g.P + id] = -u * w - cs * gx * gz;            // T_xz
    f[5 * g.P + id] = -v * w - cs * gy * gz;            // T_yz
    f[6 * g.P + id] = u * gx + v * gy + w * gz;         // u . grad phi
    f[7 * g.P + id] = p * p * p;                        // phi^3
  }
}

__device__ __forceinline__ cpx<double> ab(cpx<double> h, cpx<double> hp, int ab1) {
  return ab1 ? h : cpx<double>{1.5 * h.re - 0.5 * hp.re, 1.5 * h.im - 0.5 * hp.im};
}

__global__ void k_ch_assemble(ChanGeom g, ChanCoef c, ChanAssembleArgs a) {
  PSMS_GRID_LOOP(id, g.NZL) {
    const long long l = id % g.NL, n = id / g.NL;
    const double kx = a.kx[l], ky = a.ky[l];
    const double k2 = kx * kx + ky * ky;
    // S = div T: S_x = i kx T_xx + i ky T_xy + D T_xz, and likewise
    const cpx<double> txx = a.R[id], tyy = a.R[g.NZL + id], txy = a.R[3 * g.NZL + id];
    const cpx<double> txz = a.R[4 * g.NZL + id], tyz = a.R[5 * g.NZL + id];
    const cpx<double> sx = add(add(ti(kx, txx), ti(ky, txy)), a.d3[id]);
    const cpx<double> sy = add(add(ti(kx, txy), ti(ky, tyy)), a.d3[g.NZL + id]);
    const cpx<double> sz = add(add(ti(kx, txz), ti(ky, tyz)), a.d3[2 * g.NZL + id]);
    const cpx<double> h_om = sub(ti(kx, sy), ti(ky, sx));                    // (curl S)_z
    const cpx<double> h_w = sub(scl(-k2, sz), a.dq[id]);                     // lap_h S_z - D(div_h S)
    const cpx<double> e_om = ab(h_om, a.hist[id], c.ab1);
    const cpx<double> e_w = ab(h_w, a.hist[g.NZL + id], c.ab1);
    a.hist[id] = h_om;
    a.hist[g.NZL + id] = h_w;
    const double r2 = 2.0 * c.re;
    a.g[id] = sub(scl(-1.0, a.lom[id]), scl(r2, e_om));        // -(lap + beta) omega - 2 Re E
    a.g[g.NZL + id] = sub(scl(-1.0, a.lpsi[id]), scl(r2, e_w));
    if (!g.sp) {
      const cpx<double> s_phi = sub(a.lsphi[id], a.R[6 * g.NZL + id]);  // -a + lap c / Pe - (1 + s Ch^2)/Pe lap phi
      const cpx<double> e_phi = ab(s_phi, a.hist[2 * g.NZL + id], c.ab1);
      a.hist[2 * g.NZL + id] = s_phi;
      a.g[2 * g.NZL + id] = scl(c.g_phi_scale, add(a.phi[id], scl(c.dt, e_phi)));
    }
    if (l == 0) {  // mean flow: S_x, S_y of the mean line, driving -dP/dx = forcing on T_0
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const cpx<double> h = k ? sy : sx;
        cpx<double> e = ab(h, a.hmean[2 * n + k], c.ab1);
        a.hmean[2 * n + k] = h;
        if (k == 0 && n == 0) e.re += c.forcing;
        const cpx<double> U = a.mean[2 * n + k];
        a.gmean[2 * n + k] = sub(scl(-1.0, add(a.d2mean[2 * n + k], scl(c.beta, U))), scl(r2, e));
      }
    }
  }
}

__global__ void k_ch_init(ChanGeom g, const cpx<double>* __restrict__ U4, const double* __restrict__ kxl,
                          const double* __restrict__ kyl, cpx<double>* __restrict__ om, cpx<double>* __restrict__ w,
                          cpx<double>* __restrict__ phi, cpx<double>* __restrict__ mean) {
  PSMS_GRID_LOOP(id, g.NZL) {
    const long long l = id % g.NL, n = id / g.NL;
    const cpx<double> u = U4[id], v = U4[g.NZL + id];
    if (l == 0) {
      om[id] = cpx<double>{0.0, 0.0};
      w[id] = cpx<double>{0.0, 0.0};
      mean[2 * n] = u;
      mean[2 * n + 1] = v;
    } else {
      om[id] = sub(ti(kxl[l], v), ti(kyl[l], u));
      w[id] = U4[2 * g.NZL + id];
    }
    phi[id] = g.sp ? cpx<double>{0.0, 0.0} : U4[3 * g.NZL + id];
  }
}

__global__ void k_ch_mean_io(int nz, const cpx<double>* __restrict__ in, cpx<double>* __restrict__ out, int dir) {
  PSMS_GRID_LOOP(id, 2LL * nz) {
    const long long k = id / nz, n = id % nz;   // caller layout [2][nz]
    if (dir > 0) out[2 * n + k] = in[id];
    else out[id] = in[2 * n + k];
  }
}

// ---------------------------------------------------------------------------
// diagnostics: volume averages over the channel (x, y by Parseval with
// half-spectrum weights, z exactly: int T_m T_n dz = (I(m+n) + I(|m-n|)) / 2,
// I(k) = int T_k dz = 2 / (1 - k^2) for even k, 0 for odd k)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double cheb_int(int k) { return (k & 1) ? 0.0 : 2.0 / (1.0 - double(k) * double(k)); }

// u, v of coefficient n on line l: continuity and eq. omegadef (the mean line: U, V)
__device__ __forceinline__ void diag_uv(const ChanGeom& g, long long l, long long n, double kx, double ky,
                                        const cpx<double>* om, const cpx<double>* dw, const cpx<double>* mean,
                                        cpx<double>& u, cpx<double>& v) {
  if (l == 0) {
    u = mean[2 * n];
    v = mean[2 * n + 1];
    return;
  }
  const long long id = n * g.NL + l;
  const double ik2 = 1.0 / (kx * kx + ky * ky);
  const cpx<double> o = om[id], d = dw[id];
  u = scl(ik2, ti(1.0, add(scl(kx, d), scl(ky, o))));
  v = scl(ik2, ti(1.0, sub(scl(ky, d), scl(kx, o))));
}

__device__ __forceinline__ double rdot(cpx<double> a, cpx<double> b) { return a.re * b.re + a.im * b.im; }
__device__ __forceinline__ bool bad(cpx<double> a) { return !isfinite(a.re) || !isfinite(a.im); }

// Four (kx, ky) lines per workgroup of 256 threads, one wavefront per line;
// part[4 b + (0..3)] = block sums of the kinetic energy and <|grad phi|^2>,
// the block max of |i kx u + i ky v + D w|, and the number of non-finite state
// entries.  Each field of a line (u, v, w, phi, D phi) is staged in LDS and its
// quadratic form sum_{m,n} G_mn Re(conj f_m f_n) is split over the lanes by m
// (G_mn = 0 unless m and n have one parity).
constexpr int kDiagNC = 256;   // largest nc
__global__ void __launch_bounds__(256) k_ch_diag_lines(ChanGeom g, const cpx<double>* __restrict__ om,
                                                       const cpx<double>* __restrict__ w,
                                                       const cpx<double>* __restrict__ phi,
                                                       const cpx<double>* __restrict__ dw,
                                                       const cpx<double>* __restrict__ dphi,
                                                       const cpx<double>* __restrict__ mean,
                                                       const double* __restrict__ kxl, const double* __restrict__ kyl,
                                                       double* __restrict__ part) {
  __shared__ double It[2 * kDiagNC + 1];
  __shared__ cpx<double> F[4][kDiagNC + 1];
  __shared__ double sh[4][4];
  const int nc = g.nc;
  const int tid = threadIdx.x, lb = tid >> 6, lane = tid & 63;
  for (int k2 = tid; k2 <= 2 * nc; k2 += blockDim.x) It[k2] = cheb_int(k2);
  double ke = 0.0, gr = 0.0, md = 0.0, nf = 0.0;   // this wavefront's line sums (lane 0 keeps them)
  const long long groups = (g.NL + 3) / 4;
  for (long long grp = blockIdx.x; grp < groups; grp += gridDim.x) {
    const long long l = grp * 4 + lb;
    const bool ok = l < g.NL;                      // uniform within the wavefront
    const double kx = ok ? kxl[l] : 0.0, ky = ok ? kyl[l] : 0.0;
    double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int nfld = g.sp ? 3 : 5;
    for (int fld = 0; fld < nfld; ++fld) {
      __syncthreads();                             // It ready / the previous field's reads done
      if (ok) {
        for (int n = lane; n <= nc; n += 64) {
          const long long id = (long long)n * g.NL + l;
          cpx<double> v;
          if (fld < 2) {
            cpx<double> uu, vv;
            diag_uv(g, l, n, kx, ky, om, dw, mean, uu, vv);
            v = fld ? vv : uu;
          } else {
            v = (fld == 2) ? w[id] : (fld == 3) ? phi[id] : dphi[id];
          }
          F[lb][n] = v;
        }
      }
      __syncthreads();
      double acc = 0.0;
      if (ok) {
        for (int m = lane; m <= nc; m += 64) {
          const cpx<double> fm = F[lb][m];
          double br = 0.0, bi = 0.0;               // (G f)_m
          for (int n = m & 1; n <= nc; n += 2) {
            const double gmn = 0.5 * (It[m + n] + It[m > n ? m - n : n - m]);
            br += gmn * F[lb][n].re;
            bi += gmn * F[lb][n].im;
          }
          acc += fm.re * br + fm.im * bi;
        }
      }
#pragma unroll
      for (int s = 32; s > 0; s >>= 1) acc += __shfl_xor(acc, s);
      q[fld] = acc;
    }
    if (ok) {
      // continuity and the non-finite entries, coefficient by coefficient
      for (int n = lane; n <= nc; n += 64) {
        const long long id = (long long)n * g.NL + l;
        cpx<double> uu, vv;
        diag_uv(g, l, n, kx, ky, om, dw, mean, uu, vv);
        const cpx<double> dv = add(add(ti(kx, uu), ti(ky, vv)), dw[id]);
        md = fmax(md, sqrt(dv.re * dv.re + dv.im * dv.im));
        nf += (bad(om[id]) ? 1.0 : 0.0) + (bad(w[id]) ? 1.0 : 0.0) + ((!g.sp && bad(phi[id])) ? 1.0 : 0.0);
        if (l == 0) nf += (bad(mean[2 * n]) ? 1.0 : 0.0) + (bad(mean[2 * n + 1]) ? 1.0 : 0.0);
      }
      const double wx = (kx == 0.0) ? 1.0 : 2.0;  // half spectrum: kx > 0 stands for +-kx
      ke += 0.25 * wx * (q[0] + q[1] + q[2]);     // 1/2 <|u|^2>, <.> in z = (1/2) int dz
      gr += 0.5 * wx * ((kx * kx + ky * ky) * q[3] + q[4]);
    }
  }
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    md = fmax(md, __shfl_xor(md, s));
    nf += __shfl_xor(nf, s);
  }
  if (lane == 0) {
    sh[lb][0] = ke;
    sh[lb][1] = gr;
    sh[lb][2] = md;
    sh[lb][3] = nf;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
    for (int i = 0; i < 4; ++i) {
      a += sh[i][0];
      b += sh[i][1];
      c = fmax(c, sh[i][2]);
      d += sh[i][3];
    }
    part[4 * blockIdx.x + 0] = a;
    part[4 * blockIdx.x + 1] = b;
    part[4 * blockIdx.x + 2] = c;
    part[4 * blockIdx.x + 3] = d;
  }
}

// Block maxima of dt (|u| / dx + |v| / dy + |w| / dz_j) over the collocation
// grid (u, v, w physical FP64 [3][P]; dz_j the local spacing of the CGL points,
// (z_{j-1} - z_{j+1}) / 2 inside, one-sided at the walls) into part[4 b + 2].
__global__ void k_ch_cfl(ChanGeom g, const double* __restrict__ f, double inv_dx, double inv_dy, double dt,
                         double* __restrict__ part) {
  __shared__ double sh[kThreads];
  double mx = 0.0;
  const long long plane = (long long)g.ny * g.nx;
  PSMS_GRID_LOOP(id, g.P) {
    const int j = int(id / plane);
    const double h = M_PI / double(g.nc);
    double dz;
    if (j == 0) dz = cos(0.0) - cos(h);
    else if (j == g.nc) dz = cos(h * double(g.nc - 1)) - cos(h * double(g.nc));
    else dz = 0.5 * (cos(h * double(j - 1)) - cos(h * double(j + 1)));
    const double s = fabs(f[id]) * inv_dx + fabs(f[g.P + id]) * inv_dy + fabs(f[2 * g.P + id]) / dz;
    mx = fmax(mx, dt * s);
  }
  const int t = threadIdx.x;
  sh[t] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  if (t == 0) part[4 * blockIdx.x + 2] = sh[0];
}

// out[0..5] = mean phi, ke, grad2, max div, non-finite count, CFL from the
// partials of k_ch_diag_lines (nb1 blocks, part) and k_ch_cfl (nb2 blocks, part2)
__global__ void k_ch_diag_final(ChanGeom g, const double* __restrict__ part, int nb1, const double* __restrict__ part2,
                                int nb2, const cpx<double>* __restrict__ phi, double* __restrict__ out) {
  __shared__ double sh[5][kThreads];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0, e = 0.0;
  for (int i = t; i < nb1; i += blockDim.x) {
    a += part[4 * i];
    b += part[4 * i + 1];
    c = fmax(c, part[4 * i + 2]);
    d += part[4 * i + 3];
  }
  for (int i = t; i < nb2; i += blockDim.x) e = fmax(e, part2[4 * i + 2]);
  sh[0][t] = a; sh[1][t] = b; sh[2][t] = c; sh[3][t] = d; sh[4][t] = e;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) {
      sh[0][t] += sh[0][t + s];
      sh[1][t] += sh[1][t + s];
      sh[2][t] = fmax(sh[2][t], sh[2][t + s]);
      sh[3][t] += sh[3][t + s];
      sh[4][t] = fmax(sh[4][t], sh[4][t + s]);
    }
    __syncthreads();
  }
  if (t == 0) {
    double mp = 0.0;   // <phi> = (1/2) int phi_00 dz, the mean line (l = 0)
    if (!g.sp)
      for (int n = 0; n <= g.nc; n += 2) mp += 0.5 * cheb_int(n) * phi[(long long)n * g.NL].re;
    out[0] = mp;
    out[1] = sh[0][0];
    out[2] = sh[1][0];
    out[3] = sh[2][0];
    out[4] = sh[3][0];
    out[5] = sh[4][0];
  }
}

}  // namespace

hipError_t launch_ch_diag_lines(const ChanGeom& g, const cpx<double>* om, const cpx<double>* w, const cpx<double>* phi,
                                const cpx<double>* dw, const cpx<double>* dphi, const cpx<double>* mean,
                                const double* kx, const double* ky, double* part, int max_blocks, hipStream_t st) {
  if (g.nc > kDiagNC) return hipErrorInvalidValue;
  long long b = (g.NL + 3) / 4;
  if (b > max_blocks) b = max_blocks;
  k_ch_diag_lines<<<unsigned(b < 1 ? 1 : b), 256, 0, st>>>(g, om, w, phi, dw, dphi, mean, kx, ky, part);
  return hipGetLastError();
}

hipError_t launch_ch_cfl(const ChanGeom& g, const double* f, double inv_dx, double inv_dy, double dt, double* part,
                         int max_blocks, hipStream_t st) {
  long long b = (g.P + kThreads - 1) / kThreads;
  if (b > max_blocks) b = max_blocks;
  k_ch_cfl<<<unsigned(b < 1 ? 1 : b), kThreads, 0, st>>>(g, f, inv_dx, inv_dy, dt, part);
  return hipGetLastError();
}

hipError_t launch_ch_diag_final(const ChanGeom& g, const double* part, int nb1, const double* part2, int nb2,
                                const cpx<double>* phi, double* out, hipStream_t st) {
  k_ch_diag_final<<<1, kThreads, 0, st>>>(g, part, nb1, part2, nb2, phi, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ch_fields(const ChanGeom& g, const cpx<double>* om, const cpx<double>* w, const cpx<double>* phi,
                            const cpx<double>* dw, const cpx<double>* dphi, const cpx<double>* mean, const double* kx,
                            const double* ky, cpx<T>* out, hipStream_t st, int six) {
  k_ch_fields<T><<<blocks_for(g.NZL), kThreads, 0, st>>>(g, om, w, phi, dw, dphi, mean, kx, ky, out, six);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_ch_products(const ChanGeom& g, T* f, double csig, hipStream_t st) {
  k_ch_products<T><<<blocks_for(g.P), kThreads, 0, st>>>(g, f, T(csig));
  return hipGetLastError();
}
hipError_t launch_ch_assemble(const ChanGeom& g, const ChanCoef& c, const ChanAssembleArgs& a, hipStream_t st) {
  k_ch_assemble<<<blocks_for(g.NZL), kThreads, 0, st>>>(g, c, a);
  return hipGetLastError();
}
hipError_t launch_ch_init(const ChanGeom& g, const cpx<double>* U4, const double* kx, const double* ky,
                          cpx<double>* om, cpx<double>* w, cpx<double>* phi, cpx<double>* mean, hipStream_t st) {
  k_ch_init<<<blocks_for(g.NZL), kThreads, 0, st>>>(g, U4, kx, ky, om, w, phi, mean);
  return hipGetLastError();
}
hipError_t launch_ch_mean_io(const ChanGeom& g, const cpx<double>* in, cpx<double>* out, int dir, hipStream_t st) {
  k_ch_mean_io<<<blocks_for(2LL * (g.nc + 1)), kThreads, 0, st>>>(g.nc + 1, in, out, dir);
  return hipGetLastError();
}

template hipError_t launch_ch_fields<float>(const ChanGeom&, const cpx<double>*, const cpx<double>*,
                                            const cpx<double>*, const cpx<double>*, const cpx<double>*,
                                            const cpx<double>*, const double*, const double*, cpx<float>*,
                                            hipStream_t, int);
template hipError_t launch_ch_fields<double>(const ChanGeom&, const cpx<double>*, const cpx<double>*,
                                             const cpx<double>*, const cpx<double>*, const cpx<double>*,
                                             const cpx<double>*, const double*, const double*, cpx<double>*,
                                             hipStream_t, int);
template hipError_t launch_ch_products<float>(const ChanGeom&, float*, double, hipStream_t);
template hipError_t launch_ch_products<double>(const ChanGeom&, double*, double, hipStream_t);

}  // namespace psms
