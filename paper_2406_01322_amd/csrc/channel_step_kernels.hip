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
                            const double* __restrict__ kxl, const double* __restrict__ kyl, cpx<T>* __restrict__ out) {
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
      const cpx<double> f[4] = {p, ti(kx, p), ti(ky, p), dphi[id]};
#pragma unroll
      for (int k = 0; k < 4; ++k) out[(k + 3) * g.NZL + id] = cpx<T>{T(f[k].re), T(f[k].im)};
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

__global__ void k_ch_s(ChanGeom g, const cpx<double>* __restrict__ R, const cpx<double>* __restrict__ dxz,
                       const cpx<double>* __restrict__ dyz, const cpx<double>* __restrict__ dzz,
                       const double* __restrict__ kxl, const double* __restrict__ kyl, cpx<double>* __restrict__ s3,
                       cpx<double>* __restrict__ q) {
  PSMS_GRID_LOOP(id, g.NZL) {
    const long long l = id % g.NL;
    const double kx = kxl[l], ky = kyl[l];
    const cpx<double> txx = R[id], tyy = R[g.NZL + id], txy = R[3 * g.NZL + id];
    const cpx<double> txz = R[4 * g.NZL + id], tyz = R[5 * g.NZL + id];
    const cpx<double> sx = add(add(ti(kx, txx), ti(ky, txy)), dxz[id]);
    const cpx<double> sy = add(add(ti(kx, txy), ti(ky, tyy)), dyz[id]);
    const cpx<double> sz = add(add(ti(kx, txz), ti(ky, tyz)), dzz[id]);
    s3[id] = sx;
    s3[g.NZL + id] = sy;
    s3[2 * g.NZL + id] = sz;
    q[id] = add(ti(kx, sx), ti(ky, sy));
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
    const cpx<double> sx = a.s3[id], sy = a.s3[g.NZL + id], sz = a.s3[2 * g.NZL + id];
    const cpx<double> h_om = sub(ti(kx, sy), ti(ky, sx));                    // (curl S)_z
    const cpx<double> h_w = sub(scl(-k2, sz), a.dq[id]);                     // lap_h S_z - D(div_h S)
    const cpx<double> e_om = ab(h_om, a.hist[id], c.ab1);
    const cpx<double> e_w = ab(h_w, a.hist[g.NZL + id], c.ab1);
    a.hist[id] = h_om;
    a.hist[g.NZL + id] = h_w;
    const double r2 = 2.0 * c.re;
    const cpx<double> om = a.om[id], psi = a.psi[id];
    a.g[id] = sub(scl(-1.0, add(a.lapom[id], scl(c.beta, om))), scl(r2, e_om));
    a.g[g.NZL + id] = sub(scl(-1.0, add(a.lappsi[id], scl(c.beta, psi))), scl(r2, e_w));
    if (!g.sp) {
      const cpx<double> s_phi = add(sub(scl(c.inv_pe, a.lapc[id]), a.R[6 * g.NZL + id]),
                                    scl(-c.e_coef, a.lapphi[id]));  // -a + lap c / Pe - (1 + s Ch^2)/Pe lap phi
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

}  // namespace

template <typename T>
hipError_t launch_ch_fields(const ChanGeom& g, const cpx<double>* om, const cpx<double>* w, const cpx<double>* phi,
                            const cpx<double>* dw, const cpx<double>* dphi, const cpx<double>* mean, const double* kx,
                            const double* ky, cpx<T>* out, hipStream_t st) {
  k_ch_fields<T><<<blocks_for(g.NZL), kThreads, 0, st>>>(g, om, w, phi, dw, dphi, mean, kx, ky, out);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_ch_products(const ChanGeom& g, T* f, double csig, hipStream_t st) {
  k_ch_products<T><<<blocks_for(g.P), kThreads, 0, st>>>(g, f, T(csig));
  return hipGetLastError();
}
hipError_t launch_ch_s(const ChanGeom& g, const cpx<double>* R, const cpx<double>* dxz, const cpx<double>* dyz,
                       const cpx<double>* dzz, const double* kx, const double* ky, cpx<double>* s3, cpx<double>* q,
                       hipStream_t st) {
  k_ch_s<<<blocks_for(g.NZL), kThreads, 0, st>>>(g, R, dxz, dyz, dzz, kx, ky, s3, q);
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
                                            hipStream_t);
template hipError_t launch_ch_fields<double>(const ChanGeom&, const cpx<double>*, const cpx<double>*,
                                             const cpx<double>*, const cpx<double>*, const cpx<double>*,
                                             const cpx<double>*, const double*, const double*, cpx<double>*,
                                             hipStream_t);
template hipError_t launch_ch_products<float>(const ChanGeom&, float*, double, hipStream_t);
template hipError_t launch_ch_products<double>(const ChanGeom&, double*, double, hipStream_t);

}  // namespace psms
