// Host side of the psms C ABI: parameter validation, workspace carving, FFT
// plans and twiddle tables, and the sequencing of the step's kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/psms.h"
#include "box_kernels.hpp"
#include "channel_kernels.hpp"
#include "adjoint_kernels.hpp"
#include "channel_step_kernels.hpp"

using psms::BoxGeom;
using psms::cpx;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(PSMS_E_LAUNCH, std::string(where) + ": " + hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t state, hist, bufa, bufb, tw64, tw32, diag, diag_out, box, phys, acc, total;
  size_t bufa_bytes, bufb_bytes;
  // exact cube of phi (cube = 1): the padded grid m, two spectral buffers of
  // [m][m][K+1], the m^3 physical field, the m-point twiddles
  int m;
  size_t pad_s1, pad_s2, pad_phys, pad_tw64, pad_tw32;
};

constexpr int kDiagBlocks = 1024;

BoxGeom make_geom(int n) {
  BoxGeom g;
  g.n = n;
  g.K = (n - 1) / 3;
  g.C = 2 * g.K + 1;
  g.H = g.K + 1;
  g.Q = (long long)g.C * g.H;
  g.M = g.Q * g.C;
  return g;
}

// Smallest supported grid m > 4K: the cube of modes |k| <= K reaches 3K, and
// on an m grid its aliases miss the band |k| <= K exactly when m > 4K.  0 if
// none is supported.
int pad_size(int n) {
  const int K = (n - 1) / 3;
  const int sizes[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256};
  for (int m : sizes)
    if (m > 4 * K) return m;
  return 0;
}

Layout make_layout(const psms_params& p) {
  const BoxGeom g = make_geom(p.n);
  const size_t n = size_t(p.n), nh = n / 2 + 1;
  const size_t tp = (p.precision == PSMS_MIXED) ? sizeof(cpx<float>) : sizeof(cpx<double>);
  const size_t full64 = n * n * nh * sizeof(cpx<double>);
  const size_t y = 6 * n * n * size_t(g.H) * tp, w = 8 * n * size_t(g.Q) * tp;
  const size_t x = 8 * n * n * size_t(g.H) * tp, gz = 5 * n * size_t(g.Q) * tp;
  Layout L{};
  L.bufa_bytes = std::max(std::max(y, w), full64);
  L.bufb_bytes = std::max(std::max(x, gz), full64);
  size_t off = 0;
  L.state = off; off = align256(off + 4 * size_t(g.M) * sizeof(cpx<double>));
  L.hist = off; off = align256(off + 4 * size_t(g.M) * sizeof(cpx<double>));
  L.bufa = off; off = align256(off + L.bufa_bytes);
  L.bufb = off; off = align256(off + L.bufb_bytes);
  L.tw64 = off; off = align256(off + n * sizeof(cpx<double>));
  L.tw32 = off; off = align256(off + n * sizeof(cpx<float>));
  L.diag = off; off = align256(off + 4 * kDiagBlocks * sizeof(double));
  L.diag_out = off; off = align256(off + 8 * sizeof(double));
  L.box = off; off = align256(off + sizeof(psms::BoxDev));
  L.phys = off; off = align256(off + n * n * n * sizeof(double));   // CFL: one physical component
  L.acc = off; off = align256(off + n * n * n * sizeof(double));    // CFL: sum_i |u_i| / dx
  L.m = 0;
  if (p.cube == 1) {
    const size_t m = size_t(pad_size(p.n));
    L.m = int(m);
    L.pad_s1 = off; off = align256(off + m * m * size_t(g.H) * tp);
    L.pad_s2 = off; off = align256(off + m * m * size_t(g.H) * tp);
    L.pad_phys = off; off = align256(off + m * m * m * tp / 2);
    L.pad_tw64 = off; off = align256(off + m * sizeof(cpx<double>));
    L.pad_tw32 = off; off = align256(off + m * sizeof(cpx<float>));
  }
  L.total = off;
  return L;
}

int validate(const psms_params* p) {
  if (!p) return fail(PSMS_E_INVAL, "params is NULL");
  if (p->geometry == PSMS_CHANNEL) return fail(PSMS_E_NOTSUP, "channel geometry is not implemented by this library");
  if (p->geometry != PSMS_BOX) return fail(PSMS_E_INVAL, "geometry must be PSMS_BOX");
  if (!psms::supported_n(p->n))
    return fail(PSMS_E_INVAL, "n must be one of 8,12,16,24,32,48,64,96,128,192,256");
  if (p->precision != PSMS_FP64 && p->precision != PSMS_MIXED) return fail(PSMS_E_INVAL, "precision must be FP64 or MIXED");
  if (p->cube != 0 && p->cube != 1) return fail(PSMS_E_INVAL, "cube must be 0 (grid) or 1 (exact)");
  if (p->cube == 1 && pad_size(p->n) == 0)
    return fail(PSMS_E_NOTSUP, "the exact cube needs a supported grid larger than 4K (n <= 192)");
  const double v[5] = {p->re, p->we, p->ch, p->pe, p->dt};
  const char* nm[5] = {"re", "we", "ch", "pe", "dt"};
  for (int i = 0; i < 5; ++i)
    if (!(v[i] > 0.0) || !std::isfinite(v[i])) return fail(PSMS_E_INVAL, std::string(nm[i]) + " must be finite and > 0");
  if (!std::isfinite(p->s)) return fail(PSMS_E_INVAL, "s must be finite");
  return PSMS_OK;
}

}  // namespace

struct psms_ctx {
  psms_params p;
  BoxGeom g;
  double s;
  hipStream_t stream;
  Layout lay;
  char* ws;
  cpx<double>* state;
  cpx<double>* hist;
  void* bufa;
  void* bufb;
  cpx<double>* tw64;
  cpx<float>* tw32;
  double* diag;
  double* diag_out;
  int m;                 // padded grid of the exact cube (0: the grid cube)
  psms::BoxDev* d_box;   // one-entry device descriptor table
  psms::BoxDev h_box;    // its host copy
  int box_ab1;           // ab1 value last written to d_box (-1: never)
  int variant[4];        // workgroup-size variant per stage
  int use_graph;         // replay a captured step graph (needs a non-NULL stream)
  int graph_ok;
  hipGraph_t graph;
  hipGraphExec_t gexec;
  int have_state;
  int g_valid;  // the z-inverse of the current state sits in bufb
  int nstep;
};

namespace {

psms::StepCoef step_coef(const psms_ctx* c) {
  psms::StepCoef sc;
  const psms_params& p = c->p;
  sc.dt = p.dt;
  sc.nu = 1.0 / p.re;
  sc.ch2_pe = p.ch * p.ch / p.pe;
  sc.s = c->s;
  sc.inv_pe = 1.0 / p.pe;
  sc.e_coef = (1.0 + c->s * p.ch * p.ch) / p.pe;
  const double n = double(p.n);
  sc.inv_n3 = 1.0 / (n * n * n);
  sc.ab1 = (c->nstep == 0) ? 1 : 0;
  return sc;
}

template <typename T>
const cpx<T>* twiddles(const psms_ctx* c) {
  return std::is_same<T, double>::value ? reinterpret_cast<const cpx<T>*>(c->tw64)
                                        : reinterpret_cast<const cpx<T>*>(c->tw32);
}

// Make the device descriptor's Adams-Bashforth flag match the step count.
hipError_t sync_box(psms_ctx* c) {
  const int ab1 = (c->nstep == 0) ? 1 : 0;
  if (c->box_ab1 == ab1) return hipSuccess;
  c->h_box.sc = step_coef(c);
  c->box_ab1 = ab1;
  return hipMemcpyAsync(c->d_box, &c->h_box, sizeof(psms::BoxDev), hipMemcpyHostToDevice, c->stream);
}

// z-inverse of the current state into bufb (the input of the next step).
template <typename T>
hipError_t prologue(psms_ctx* c) {
  hipError_t e = sync_box(c);
  if (e != hipSuccess) return e;
  return psms::launch_step_stage<T>(c->g.n, 3, c->variant[3], c->d_box, 0, 1, twiddles<T>(c), 0, c->stream);
}

// The exact cube of phi (cube = 1), replacing the grid cube among the y-forward
// products: phi's band on the padded m^3 grid (z, y inverse from the band, x
// rows), cubed there, back to the band (x rows to K+1 entries, y and z to the
// 2K+1 band slots, 1/m^3), then z-inverse on the n grid times n^2 into product
// field 7 of the y-forward output, where the z stage's forward transform (with
// its 1/n^3) recovers the band.  Every buffer is written before it is read.
template <typename T>
hipError_t exact_cube(psms_ctx* c) {
  const BoxGeom& g = c->g;
  const int n = g.n, m = c->m;
  hipStream_t st = c->stream;
  const Layout& L = c->lay;
  cpx<T>* S1 = reinterpret_cast<cpx<T>*>(c->ws + L.pad_s1);
  cpx<T>* S2 = reinterpret_cast<cpx<T>*>(c->ws + L.pad_s2);
  T* Pm = reinterpret_cast<T*>(c->ws + L.pad_phys);
  const cpx<T>* twm = reinterpret_cast<const cpx<T>*>(c->ws + (std::is_same<T, double>::value ? L.pad_tw64
                                                                                             : L.pad_tw32));
  const cpx<double>* phi = c->state + 3 * g.M;
  const cpx<T>* band;
  hipError_t e = hipSuccess;
  if (std::is_same<T, double>::value) {
    band = reinterpret_cast<const cpx<T>*>(phi);
  } else {
    e = psms::launch_band_to<T>(phi, S2, g.M, st);
    band = S2;
  }
  psms::LineArgs lz{};
  lz.n_in = g.C;
  lz.n_out = m;
  lz.inner = g.Q;
  lz.nlines = g.Q;
  lz.fmap = 0;
  lz.scale = 1.0;
  if (e == hipSuccess) e = psms::launch_lines<T>(m, +1, band, S1, twm, lz, 1, st);   // [m][C][H]
  psms::LineArgs ly{};
  ly.n_in = g.C;
  ly.n_out = m;
  ly.inner = g.H;
  ly.nlines = (long long)m * g.H;
  ly.fmap = 0;
  ly.scale = 1.0;
  if (e == hipSuccess) e = psms::launch_lines<T>(m, +1, S1, S2, twm, ly, 1, st);     // [m][m][H]
  psms::RowArgs ra{};
  ra.nrows = (long long)m * m;
  ra.n_in = g.H;
  ra.n_out = m;
  ra.scale = 1.0;
  if (e == hipSuccess) e = psms::launch_rows<T>(m, +1, S2, Pm, twm, ra, 1, st);        // [m][m][m]
  if (e == hipSuccess) e = psms::launch_cube<T>(Pm, (long long)m * m * m, st);
  ra.n_in = m;
  ra.n_out = g.H;
  if (e == hipSuccess) e = psms::launch_rows<T>(m, -1, Pm, S1, twm, ra, 1, st);        // [m][m][H]
  ly.n_in = m;
  ly.n_out = g.C;
  if (e == hipSuccess) e = psms::launch_lines<T>(m, -1, S1, S2, twm, ly, 1, st);     // [m][C][H]
  lz.n_in = m;
  lz.n_out = g.C;
  lz.scale = 1.0 / (double(m) * m * m);
  if (e == hipSuccess) e = psms::launch_lines<T>(m, -1, S2, S1, twm, lz, 1, st);     // [C][C][H] band
  psms::LineArgs li{};
  li.n_in = g.C;
  li.n_out = n;
  li.inner = g.Q;
  li.nlines = g.Q;
  li.fmap = 0;
  li.scale = double(n) * n;
  cpx<T>* w7 = static_cast<cpx<T>*>(c->bufa) + 7LL * n * g.Q;                      // [n][C][H]
  if (e == hipSuccess) e = psms::launch_lines<T>(n, +1, S1, w7, twiddles<T>(c), li, 1, st);
  return e;
}

// One time step: y-inverse, x stage with products, y-forward, z stage with the
// update.  `ev` (optional) receives an event before each stage and after the last.
template <typename T>
hipError_t one_step(psms_ctx* c, hipEvent_t* ev = nullptr) {
  hipError_t e = sync_box(c);
  if (e != hipSuccess) return e;
  for (int stage = 0; stage < 4; ++stage) {
    if (ev && (e = hipEventRecord(ev[stage], c->stream)) != hipSuccess) return e;
    if (stage == 3 && c->m && (e = exact_cube<T>(c)) != hipSuccess) return e;
    e = psms::launch_step_stage<T>(c->g.n, stage, c->variant[stage], c->d_box, 0, 1, twiddles<T>(c), 1, c->stream);
    if (e != hipSuccess) return e;
  }
  if (ev) e = hipEventRecord(ev[4], c->stream);
  return e;
}

// Forward transform of nf real FP64 fields into the compact band (state layout).
hipError_t forward_to_band(psms_ctx* c, const double* d_in, cpx<double>* d_out, int nf) {
  const BoxGeom& g = c->g;
  const int n = g.n;
  hipError_t e;
  for (int f = 0; f < nf; ++f) {
    psms::RowArgs ra{};
    ra.nrows = (long long)n * n;
    ra.n_in = n;
    ra.n_out = g.H;
    ra.in_fstride = 0;
    ra.out_fstride = 0;
    ra.scale = 1.0;
    e = psms::launch_rows<double>(n, -1, d_in + (size_t)f * n * n * n, c->bufa, c->tw64, ra, 1, c->stream);
    if (e != hipSuccess) return e;
    psms::LineArgs ly{};
    ly.n_in = n;
    ly.n_out = g.C;
    ly.inner = g.H;
    ly.nlines = (long long)n * g.H;
    ly.fmap = 0;
    ly.scale = 1.0;
    e = psms::launch_lines<double>(n, -1, static_cast<const cpx<double>*>(c->bufa),
                                   static_cast<cpx<double>*>(c->bufb), c->tw64, ly, 1, c->stream);
    if (e != hipSuccess) return e;
    psms::LineArgs lz{};
    lz.n_in = n;
    lz.n_out = g.C;
    lz.inner = g.Q;
    lz.nlines = g.Q;
    lz.fmap = 0;
    lz.scale = 1.0 / (double(n) * n * n);
    e = psms::launch_lines<double>(n, -1, static_cast<const cpx<double>*>(c->bufb), d_out + (size_t)f * g.M,
                                   c->tw64, lz, 1, c->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t transform_fields(psms_ctx* c, int dir, int nf, const void* d_in, void* d_out, uint32_t flags) {
  const cpx<T>* tw = std::is_same<T, double>::value ? reinterpret_cast<const cpx<T>*>(c->tw64)
                                                     : reinterpret_cast<const cpx<T>*>(c->tw32);
  const BoxGeom& g = c->g;
  const int n = g.n, nh = n / 2 + 1;
  const size_t nfull = size_t(n) * n * nh, nphys = size_t(n) * n * n;
  const int dealias = (flags & PSMS_DEALIAS) ? 1 : 0;
  const int axis = (flags & PSMS_DERIV_X) ? 0 : (flags & PSMS_DERIV_Y) ? 1 : (flags & PSMS_DERIV_Z) ? 2 : -1;
  cpx<T>* A = static_cast<cpx<T>*>(c->bufa);
  cpx<T>* B = static_cast<cpx<T>*>(c->bufb);
  psms::LineArgs ly{};
  ly.n_in = n;
  ly.n_out = n;
  ly.inner = nh;
  ly.nlines = (long long)n * nh;
  ly.scale = 1.0;
  psms::LineArgs lz = ly;
  lz.inner = (long long)n * nh;
  lz.nlines = (long long)n * nh;
  psms::RowArgs ra{};
  ra.nrows = (long long)n * n;
  ra.n_in = nh;
  ra.n_out = nh;
  ra.scale = 1.0;
  hipError_t e;
  for (int f = 0; f < nf; ++f) {
    if (dir > 0) {
      const T* src = static_cast<const T*>(d_in) + f * nphys;
      cpx<T>* dst = static_cast<cpx<T>*>(d_out) + f * nfull;
      ra.n_in = n;
      if ((e = psms::launch_rows<T>(n, -1, src, A, tw, ra, 1, c->stream)) != hipSuccess) return e;
      if ((e = psms::launch_lines<T>(n, -1, A, B, tw, ly, 1, c->stream)) != hipSuccess) return e;
      if ((e = psms::launch_lines<T>(n, -1, B, A, tw, lz, 1, c->stream)) != hipSuccess) return e;
      if ((e = psms::launch_spec_finish<T>(A, dst, g, 1, dealias, axis, 1.0 / (double(n) * n * n), c->stream)) !=
          hipSuccess)
        return e;
    } else {
      const cpx<T>* src = static_cast<const cpx<T>*>(d_in) + f * nfull;
      T* dst = static_cast<T*>(d_out) + f * nphys;
      if ((e = psms::launch_spec_finish<T>(src, A, g, 1, dealias, axis, 1.0, c->stream)) != hipSuccess) return e;
      if ((e = psms::launch_lines<T>(n, +1, A, B, tw, lz, 1, c->stream)) != hipSuccess) return e;
      if ((e = psms::launch_lines<T>(n, +1, B, A, tw, ly, 1, c->stream)) != hipSuccess) return e;
      ra.n_in = nh;
      ra.n_out = n;
      if ((e = psms::launch_rows<T>(n, +1, A, dst, tw, ra, 1, c->stream)) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

}  // namespace

extern "C" {

const char* psms_last_error(void) { return g_err.c_str(); }
const char* psms_version(void) { return "psms 0.1 (gfx950)"; }

int psms_workspace_bytes(const psms_params* p, size_t* bytes) {
  int r = validate(p);
  if (r) return r;
  if (!bytes) return fail(PSMS_E_INVAL, "bytes is NULL");
  *bytes = make_layout(*p).total;
  return PSMS_OK;
}

int psms_create(psms_ctx** out, const psms_params* p, void* d_workspace, size_t bytes, void* stream) {
  if (!out) return fail(PSMS_E_INVAL, "out is NULL");
  *out = nullptr;
  int r = validate(p);
  if (r) return r;
  const Layout lay = make_layout(*p);
  if (!d_workspace) return fail(PSMS_E_WORKSPACE, "workspace is NULL");
  if (!aligned(d_workspace)) return fail(PSMS_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < lay.total)
    return fail(PSMS_E_WORKSPACE, "workspace too small: need " + std::to_string(lay.total) + " bytes, got " +
                                      std::to_string(bytes));
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(PSMS_E_DEVICE, "no HIP device available");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(PSMS_E_DEVICE, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(PSMS_E_DEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(PSMS_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");

  psms_ctx* c = new psms_ctx();
  c->p = *p;
  c->g = make_geom(p->n);
  c->s = (p->s > 0.0) ? p->s : std::sqrt(4.0 * p->pe / (p->ch * p->ch * p->dt));
  c->stream = static_cast<hipStream_t>(stream);
  c->lay = lay;
  c->ws = static_cast<char*>(d_workspace);
  c->state = reinterpret_cast<cpx<double>*>(c->ws + lay.state);
  c->hist = reinterpret_cast<cpx<double>*>(c->ws + lay.hist);
  c->bufa = c->ws + lay.bufa;
  c->bufb = c->ws + lay.bufb;
  c->tw64 = reinterpret_cast<cpx<double>*>(c->ws + lay.tw64);
  c->tw32 = reinterpret_cast<cpx<float>*>(c->ws + lay.tw32);
  c->diag = reinterpret_cast<double*>(c->ws + lay.diag);
  c->diag_out = reinterpret_cast<double*>(c->ws + lay.diag_out);
  c->d_box = reinterpret_cast<psms::BoxDev*>(c->ws + lay.box);
  c->h_box.bufa = c->bufa;
  c->h_box.bufb = c->bufb;
  c->h_box.state = c->state;
  c->h_box.hist = c->hist;
  c->h_box.sc = step_coef(c);
  c->h_box.csig = 3.0 / std::sqrt(8.0) * p->ch / p->we;
  c->h_box.sphi0 = reinterpret_cast<cpx<double>*>(c->diag_out + 6);
  c->box_ab1 = -1;
  for (int i = 0; i < 4; ++i) c->variant[i] = 2;
  c->use_graph = 0;      // eager launches unless psms_set_graphs enables the replay
  c->graph_ok = 0;

  // Twiddles exp(-2 pi i m / n) in FP64, rounded once to FP32 for MIXED.
  const int n = p->n;
  std::vector<cpx<double>> t64(n);
  std::vector<cpx<float>> t32(n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * double(m) / double(n);
    t64[m] = cpx<double>{std::cos(a), std::sin(a)};
    t32[m] = cpx<float>{float(t64[m].re), float(t64[m].im)};
  }
  hipError_t e = hipMemsetAsync(c->diag_out, 0, 8 * sizeof(double), c->stream);   // S_phi(0) before a step: 0
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->tw64, t64.data(), n * sizeof(cpx<double>), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->tw32, t32.data(), n * sizeof(cpx<float>), hipMemcpyHostToDevice, c->stream);
  c->m = lay.m;
  std::vector<cpx<double>> m64(lay.m);
  std::vector<cpx<float>> m32(lay.m);
  for (int k = 0; k < lay.m; ++k) {
    const double a = -2.0 * M_PI * double(k) / double(lay.m);
    m64[k] = cpx<double>{std::cos(a), std::sin(a)};
    m32[k] = cpx<float>{float(m64[k].re), float(m64[k].im)};
  }
  if (e == hipSuccess && lay.m)
    e = hipMemcpyAsync(c->ws + lay.pad_tw64, m64.data(), lay.m * sizeof(cpx<double>), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && lay.m)
    e = hipMemcpyAsync(c->ws + lay.pad_tw32, m32.data(), lay.m * sizeof(cpx<float>), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = sync_box(c);  // the device descriptor is valid from creation on
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "twiddle upload");
  }
  *out = c;
  return PSMS_OK;
}

int psms_destroy(psms_ctx* c) {
  if (c && c->graph_ok) {
    (void)hipGraphExecDestroy(c->gexec);
    (void)hipGraphDestroy(c->graph);
  }
  delete c;
  return PSMS_OK;
}

int psms_set_graphs(psms_ctx* c, int32_t enable) {
  if (!c) return fail(PSMS_E_INVAL, "NULL context");
  c->use_graph = enable ? 1 : 0;
  return PSMS_OK;
}

int64_t psms_band_modes(const psms_ctx* c) { return c ? int64_t(c->g.M) : 0; }

int psms_init_state(psms_ctx* c, const double* d_u, const double* d_phi) {
  if (!c || !d_u || !d_phi) return fail(PSMS_E_INVAL, "NULL argument");
  hipError_t e = forward_to_band(c, d_u, c->state, 3);
  if (e == hipSuccess) e = forward_to_band(c, d_phi, c->state + 3 * c->g.M, 1);
  if (e == hipSuccess) e = psms::launch_project(c->state, c->g, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->hist, 0, 4 * size_t(c->g.M) * sizeof(cpx<double>), c->stream);
  if (e != hipSuccess) return hip_fail(e, "init_state");
  c->nstep = 0;
  c->have_state = 1;
  c->g_valid = 0;
  psms_diag d;
  int r = psms_diagnostics(c, &d);
  if (r) return r;
  if (d.nonfinite) {
    c->have_state = 0;
    return fail(PSMS_E_NONFINITE, "non-finite value in the initial fields");
  }
  return PSMS_OK;
}

int psms_set_state(psms_ctx* c, const double* d_uhat, const double* d_phihat, const double* d_hist, int32_t nstep) {
  if (!c || !d_uhat || !d_phihat) return fail(PSMS_E_INVAL, "NULL argument");
  if (nstep < 0) return fail(PSMS_E_INVAL, "nstep must be >= 0");
  if (nstep > 0 && !d_hist) return fail(PSMS_E_INVAL, "nstep > 0 needs the history");
  const BoxGeom& g = c->g;
  hipError_t e = psms::launch_compact<double>(reinterpret_cast<const cpx<double>*>(d_uhat), c->state, g, 3, c->stream);
  if (e == hipSuccess)
    e = psms::launch_compact<double>(reinterpret_cast<const cpx<double>*>(d_phihat), c->state + 3 * g.M, g, 1,
                                     c->stream);
  if (e == hipSuccess) {
    if (d_hist) e = psms::launch_compact<double>(reinterpret_cast<const cpx<double>*>(d_hist), c->hist, g, 4, c->stream);
    else e = hipMemsetAsync(c->hist, 0, 4 * size_t(g.M) * sizeof(cpx<double>), c->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "set_state");
  c->nstep = nstep;
  c->have_state = 1;
  c->g_valid = 0;
  return PSMS_OK;
}

int psms_get_state(psms_ctx* c, double* d_uhat, double* d_phihat, double* d_hist) {
  if (!c || !d_uhat || !d_phihat) return fail(PSMS_E_INVAL, "NULL argument");
  if (!c->have_state) return fail(PSMS_E_STATE, "no state: call psms_init_state or psms_set_state first");
  const BoxGeom& g = c->g;
  hipError_t e = psms::launch_expand<double>(c->state, reinterpret_cast<cpx<double>*>(d_uhat), g, 3, c->stream);
  if (e == hipSuccess)
    e = psms::launch_expand<double>(c->state + 3 * g.M, reinterpret_cast<cpx<double>*>(d_phihat), g, 1, c->stream);
  if (e == hipSuccess && d_hist)
    e = psms::launch_expand<double>(c->hist, reinterpret_cast<cpx<double>*>(d_hist), g, 4, c->stream);
  if (e != hipSuccess) return hip_fail(e, "get_state");
  return PSMS_OK;
}

int psms_step(psms_ctx* c, int32_t nsteps) {
  if (!c) return fail(PSMS_E_INVAL, "NULL context");
  if (nsteps < 0) return fail(PSMS_E_INVAL, "nsteps must be >= 0");
  if (!c->have_state) return fail(PSMS_E_STATE, "step before init_state / set_state");
  const bool mixed = c->p.precision == PSMS_MIXED;
  hipError_t e = hipSuccess;
  if (!c->g_valid && nsteps > 0) {
    e = mixed ? prologue<float>(c) : prologue<double>(c);
    if (e != hipSuccess) return hip_fail(e, "step prologue");
    c->g_valid = 1;
  }
  for (int i = 0; i < nsteps; ++i) {
    // after the Adams-Bashforth 1 step every step is the same launch sequence:
    // capture it once and replay it
    const bool graph = c->use_graph && c->stream != nullptr && c->nstep > 0;
    if (graph) {
      e = sync_box(c);
      if (e == hipSuccess && !c->graph_ok) {
        e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          hipError_t e2 = mixed ? one_step<float>(c) : one_step<double>(c);
          e = hipStreamEndCapture(c->stream, &c->graph);
          if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0);
        if (e == hipSuccess) c->graph_ok = 1;
      }
      if (e == hipSuccess) e = hipGraphLaunch(c->gexec, c->stream);
    } else {
      e = mixed ? one_step<float>(c) : one_step<double>(c);
    }
    if (e != hipSuccess) {
      c->g_valid = 0;
      return hip_fail(e, "step");
    }
    c->nstep += 1;
  }
  return PSMS_OK;
}

int psms_stage_times(psms_ctx* c, int32_t nsteps, double* h_ms) {
  if (!c || !h_ms) return fail(PSMS_E_INVAL, "NULL argument");
  if (nsteps < 1) return fail(PSMS_E_INVAL, "nsteps must be >= 1");
  if (!c->have_state) return fail(PSMS_E_STATE, "step before init_state / set_state");
  const bool mixed = c->p.precision == PSMS_MIXED;
  hipError_t e = hipSuccess;
  if (!c->g_valid) {
    e = mixed ? prologue<float>(c) : prologue<double>(c);
    if (e != hipSuccess) return hip_fail(e, "step prologue");
    c->g_valid = 1;
  }
  // eager launches with an event between consecutive kernels (events recorded
  // inside a captured graph cannot be timed)
  std::vector<hipEvent_t> ev(5 * size_t(nsteps));
  size_t made = 0;
  for (; made < ev.size(); ++made)
    if ((e = hipEventCreate(&ev[made])) != hipSuccess) break;
  double acc[4] = {0, 0, 0, 0};
  for (int i = 0; e == hipSuccess && i < nsteps; ++i) {
    e = mixed ? one_step<float>(c, &ev[5 * i]) : one_step<double>(c, &ev[5 * i]);
    if (e == hipSuccess) c->nstep += 1;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  for (int i = 0; e == hipSuccess && i < nsteps; ++i) {
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev[5 * i + k], ev[5 * i + k + 1]);
      acc[k] += ms;
    }
  }
  for (size_t i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
  if (e != hipSuccess) {
    c->g_valid = 0;
    return hip_fail(e, "stage_times");
  }
  for (int k = 0; k < 4; ++k) h_ms[k] = acc[k] / nsteps;
  return PSMS_OK;
}

int psms_transform(psms_ctx* c, int32_t dir, int32_t nfield, const void* d_in, void* d_out, uint32_t flags) {
  if (!c) return fail(PSMS_E_INVAL, "NULL context");
  if (nfield == 0) return PSMS_OK;
  if (!d_in || !d_out) return fail(PSMS_E_INVAL, "NULL argument");
  if (dir != 1 && dir != -1) return fail(PSMS_E_INVAL, "dir must be +1 or -1");
  if (nfield < 0) return fail(PSMS_E_INVAL, "nfield must be >= 0");
  if (flags & ~uint32_t(15)) return fail(PSMS_E_INVAL, "unknown flag");
  const uint32_t d = flags & 14u;
  if (d && (d & (d - 1))) return fail(PSMS_E_INVAL, "at most one derivative flag");
  c->g_valid = 0;  // the scratch holding the next step's input is reused
  hipError_t e = (c->p.precision == PSMS_MIXED) ? transform_fields<float>(c, dir, nfield, d_in, d_out, flags)
                                                : transform_fields<double>(c, dir, nfield, d_in, d_out, flags);
  if (e != hipSuccess) return hip_fail(e, "transform");
  return PSMS_OK;
}

int psms_solve_helmholtz(psms_ctx* c, int32_t nfield, const double* h_lambda, const double* d_rhs, double* d_out) {
  if (!c || !h_lambda || !d_rhs || !d_out) return fail(PSMS_E_INVAL, "NULL argument");
  if (nfield < 0) return fail(PSMS_E_INVAL, "nfield must be >= 0");
  const BoxGeom& g = c->g;
  const size_t per = size_t(g.n) * g.n * (g.n / 2 + 1);
  for (int f = 0; f < nfield; ++f) {
    if (!(h_lambda[f] >= 0.0) || !std::isfinite(h_lambda[f])) return fail(PSMS_E_INVAL, "lambda must be finite and >= 0");
  }
  for (int f = 0; f < nfield; ++f) {
    hipError_t e = psms::launch_helmholtz_box(reinterpret_cast<const cpx<double>*>(d_rhs) + f * per,
                                              reinterpret_cast<cpx<double>*>(d_out) + f * per, g, h_lambda[f],
                                              c->stream);
    if (e != hipSuccess) return hip_fail(e, "solve_helmholtz");
  }
  return PSMS_OK;
}

int psms_diagnostics(psms_ctx* c, psms_diag* h_out) {
  if (!c || !h_out) return fail(PSMS_E_INVAL, "NULL argument");
  if (!c->have_state) return fail(PSMS_E_STATE, "no state");
  hipError_t e = psms::launch_diag(c->state, c->g, c->diag, kDiagBlocks, c->diag_out, c->stream);
  // CFL = dt max_x sum_i |u_i| / dx: each component to physical space (FP64,
  // through the step's scratch, so the next step re-runs its prologue)
  const BoxGeom& g = c->g;
  const int n = g.n, nh = n / 2 + 1;
  const long long np = (long long)n * n * n;
  double* phys = reinterpret_cast<double*>(c->ws + c->lay.phys);
  double* acc = reinterpret_cast<double*>(c->ws + c->lay.acc);
  cpx<double>* A = static_cast<cpx<double>*>(c->bufa);
  cpx<double>* B = static_cast<cpx<double>*>(c->bufb);
  psms::LineArgs ly{};
  ly.n_in = n;
  ly.n_out = n;
  ly.inner = nh;
  ly.nlines = (long long)n * nh;
  ly.scale = 1.0;
  psms::LineArgs lz = ly;
  lz.inner = (long long)n * nh;
  psms::RowArgs ra{};
  ra.nrows = (long long)n * n;
  ra.n_in = nh;
  ra.n_out = n;
  ra.scale = 1.0;
  c->g_valid = 0;
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    e = psms::launch_expand<double>(c->state + k * g.M, B, g, 1, c->stream);
    if (e == hipSuccess) e = psms::launch_spec_finish<double>(B, A, g, 1, 0, -1, 1.0, c->stream);
    if (e == hipSuccess) e = psms::launch_lines<double>(n, +1, A, B, c->tw64, lz, 1, c->stream);
    if (e == hipSuccess) e = psms::launch_lines<double>(n, +1, B, A, c->tw64, ly, 1, c->stream);
    if (e == hipSuccess) e = psms::launch_rows<double>(n, +1, A, phys, c->tw64, ra, 1, c->stream);
    if (e == hipSuccess) e = psms::launch_abs_accum(phys, acc, np, c->p.dt * n / (2.0 * M_PI), k == 0, c->stream);
  }
  if (e == hipSuccess) e = psms::launch_max(acc, np, c->diag, kDiagBlocks, c->diag_out + 5, c->stream);
  double h[8];
  if (e == hipSuccess) e = hipMemcpyAsync(h, c->diag_out, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics");
  h_out->mean_phi = h[0];
  h_out->ke = h[1];
  h_out->grad2 = h[2];
  h_out->max_div = h[3];
  h_out->nonfinite = int32_t(h[4]);
  h_out->nstep = c->nstep;
  h_out->cfl = h[5];
  h_out->sphi0_re = h[6];
  h_out->sphi0_im = h[7];
  return PSMS_OK;
}

}  // extern "C"

namespace {
// The pressure of the current state: the step's y-inverse, x (products) and
// y-forward stages, the z-forward of the six T_ij into the compact band, then
// p_hat = k_i k_j T_ij / k^2 and its full half spectrum.  The stages overwrite
// the z-inverse of the state that the next step starts from.
template <typename T>
hipError_t pressure_impl(psms_ctx* c, double* d_p) {
  const BoxGeom& g = c->g;
  const int n = g.n;
  hipError_t e = hipSuccess;
  if (!c->g_valid) e = prologue<T>(c);
  if (e == hipSuccess) e = sync_box(c);
  for (int stage = 0; stage < 3 && e == hipSuccess; ++stage)
    e = psms::launch_step_stage<T>(n, stage, c->variant[stage], c->d_box, 0, 1, twiddles<T>(c), 1, c->stream);
  c->g_valid = 0;
  psms::LineArgs lz{};
  lz.n_in = n;
  lz.n_out = g.C;
  lz.inner = g.Q;
  lz.nlines = g.Q;
  lz.in_fstride = (long long)n * g.Q;
  lz.out_fstride = g.M;
  lz.fmap = 0x543210u;
  lz.scale = 1.0 / (double(n) * n * n);
  cpx<T>* t6 = static_cast<cpx<T>*>(c->bufb);
  if (e == hipSuccess)
    e = psms::launch_lines<T>(n, -1, static_cast<const cpx<T>*>(c->bufa), t6, twiddles<T>(c), lz, 6, c->stream);
  cpx<double>* pb = reinterpret_cast<cpx<double>*>(c->ws + c->lay.phys);
  if (e == hipSuccess) e = psms::launch_pressure_band<T>(t6, g, pb, c->stream);
  if (e == hipSuccess) e = psms::launch_expand<double>(pb, reinterpret_cast<cpx<double>*>(d_p), g, 1, c->stream);
  return e;
}
}  // namespace

extern "C" {

int psms_pressure(psms_ctx* c, double* d_p) {
  if (!c || !d_p) return fail(PSMS_E_INVAL, "NULL argument");
  if (!c->have_state) return fail(PSMS_E_STATE, "no state");
  const hipError_t e = (c->p.precision == PSMS_MIXED) ? pressure_impl<float>(c, d_p) : pressure_impl<double>(c, d_p);
  if (e != hipSuccess) return hip_fail(e, "pressure");
  return PSMS_OK;
}

int psms_index_maps(psms_ctx* c, int32_t* d_out) {
  if (!c || !d_out) return fail(PSMS_E_INVAL, "NULL argument");
  hipError_t e = psms::launch_index_maps(d_out, c->g, c->stream);
  if (e != hipSuccess) return hip_fail(e, "index_maps");
  return PSMS_OK;
}

// ---------------------------------------------------------------------------
// wall-normal (Chebyshev) operations
// ---------------------------------------------------------------------------

int psms_cheb_transform(int32_t nc, int64_t nlines, int32_t dir, int32_t precision, const void* d_in, void* d_out,
                        void* stream) {
  if (!psms::supported_nc(nc)) return fail(PSMS_E_INVAL, "nc must be one of 4,6,8,12,16,24,32,48,64,96,128,256");
  if (nlines < 0 || (dir != 1 && dir != -1)) return fail(PSMS_E_INVAL, "bad nlines or dir");
  if (precision != PSMS_FP64 && precision != PSMS_MIXED) return fail(PSMS_E_INVAL, "bad precision");
  if (nlines == 0) return PSMS_OK;
  if (!d_in || !d_out) return fail(PSMS_E_INVAL, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = (precision == PSMS_FP64)
                     ? psms::launch_dct<double>(nc, static_cast<const cpx<double>*>(d_in),
                                                static_cast<cpx<double>*>(d_out), nlines, dir, st)
                     : psms::launch_dct<float>(nc, static_cast<const cpx<float>*>(d_in),
                                               static_cast<cpx<float>*>(d_out), nlines, dir, st);
  if (e != hipSuccess) return hip_fail(e, "cheb_transform");
  return PSMS_OK;
}

int psms_cheb_deriv(int32_t nc, int64_t nlines, const double* d_in, double* d_out, void* stream) {
  if (nc < 2 || nlines < 0) return fail(PSMS_E_INVAL, "bad nc or nlines");
  if (nlines == 0) return PSMS_OK;
  if (!d_in || !d_out) return fail(PSMS_E_INVAL, "NULL argument");
  if (d_in == d_out) return fail(PSMS_E_INVAL, "d_in and d_out must not overlap");
  hipError_t e = psms::launch_chebd(reinterpret_cast<const cpx<double>*>(d_in), reinterpret_cast<cpx<double>*>(d_out),
                                    nc, nlines, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "cheb_deriv");
  return PSMS_OK;
}

int psms_cheb_helmholtz(int32_t nc, int64_t nlines, const double* d_beta, int32_t bc, const double* d_bcval,
                        const double* d_rhs, double* d_out, double* d_work, void* stream) {
  if (nc < 4 || nlines < 0) return fail(PSMS_E_INVAL, "bad nc or nlines");
  if (bc != PSMS_DIRICHLET && bc != PSMS_NEUMANN) return fail(PSMS_E_INVAL, "bc must be DIRICHLET or NEUMANN");
  if (nlines == 0) return PSMS_OK;
  if (!d_beta || !d_rhs || !d_out || !d_work) return fail(PSMS_E_INVAL, "NULL argument");
  if (d_rhs == d_out) return fail(PSMS_E_INVAL, "d_rhs and d_out must not overlap");
  hipError_t e = psms::launch_helm(reinterpret_cast<const cpx<double>*>(d_rhs), reinterpret_cast<cpx<double>*>(d_out),
                                   d_work, nc, nlines, d_beta, 0.0, nullptr, nullptr, bc == PSMS_NEUMANN ? 1 : 0,
                                   reinterpret_cast<const cpx<double>*>(d_bcval), cpx<double>{0.0, 0.0},
                                   cpx<double>{0.0, 0.0}, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "cheb_helmholtz");
  return PSMS_OK;
}

// ---------------------------------------------------------------------------
// psms_cheb_helmholtz_noalloc: the elimination scratch in a library-owned
// device array instead of a caller workspace.  The array exists once per GPU
// (each device holds its own copy at its own address); host code never passes
// its name to a kernel, only the address hipGetSymbolAddress returns for the
// device that is current.
// ---------------------------------------------------------------------------

static __device__ __align__(256) double scratch[PSMS_NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch`, looked up (once per
// device, with that device current) on the first call.
hipError_t device_scratch(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

int psms_cheb_helmholtz_noalloc(int32_t nc, int64_t nlines, const double* d_beta, int32_t bc, const double* d_bcval,
                                const double* d_rhs, double* d_out, void* stream) {
  if (nc < 4 || nlines < 0) return fail(PSMS_E_INVAL, "bad nc or nlines");
  if (bc != PSMS_DIRICHLET && bc != PSMS_NEUMANN) return fail(PSMS_E_INVAL, "bc must be DIRICHLET or NEUMANN");
  if (nlines == 0) return PSMS_OK;
  if (!d_beta || !d_rhs || !d_out) return fail(PSMS_E_INVAL, "NULL argument");
  if (d_rhs == d_out) return fail(PSMS_E_INVAL, "d_rhs and d_out must not overlap");
  if (nlines > (long long)(PSMS_NOALLOC_SCRATCH_DOUBLES / size_t(nc + 1)))
    return fail(PSMS_E_WORKSPACE, "(nc + 1) * nlines exceeds the " + std::to_string(PSMS_NOALLOC_SCRATCH_DOUBLES) +
                                      " doubles of the library's scratch; use psms_cheb_helmholtz");
  double* work = nullptr;
  hipError_t e = device_scratch(&work);
  if (e != hipSuccess) return hip_fail(e, "cheb_helmholtz_noalloc: scratch address");
  // the same kernel as psms_cheb_helmholtz; the scratch needs no clearing (every
  // entry a line reads was written earlier by the same thread)
  e = psms::launch_helm(reinterpret_cast<const cpx<double>*>(d_rhs), reinterpret_cast<cpx<double>*>(d_out), work, nc,
                        nlines, d_beta, 0.0, nullptr, nullptr, bc == PSMS_NEUMANN ? 1 : 0,
                        reinterpret_cast<const cpx<double>*>(d_bcval), cpx<double>{0.0, 0.0}, cpx<double>{0.0, 0.0},
                        static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "cheb_helmholtz_noalloc");
  return PSMS_OK;
}

namespace {
struct WallLayout {
  size_t line, psi, wt, psit, wb, psib, xi, dw, xw, total;
};
WallLayout wall_layout(int nc, long long nlines) {
  WallLayout L{};
  const size_t arr = align256(size_t(nc + 1) * size_t(nlines) * sizeof(cpx<double>));
  size_t off = 0;
  L.psi = off; off += arr;
  L.wt = off; off += arr;
  L.psit = off; off += arr;
  L.wb = off; off += arr;
  L.psib = off; off += arr;
  L.xi = off; off += arr;
  L.dw = off; off += arr;
  // elimination scratch of up to four problems solved in one launch
  L.xw = off; off += 4 * align256(size_t(nc + 1) * size_t(nlines) * sizeof(double));
  L.total = off;
  return L;
}
}  // namespace

int psms_wall_workspace_bytes(int32_t nc, int64_t nlines, size_t* bytes) {
  if (nc < 4 || nlines < 0 || !bytes) return fail(PSMS_E_INVAL, "bad argument");
  *bytes = wall_layout(nc, nlines).total;
  return PSMS_OK;
}

int psms_wall_solve(const psms_wall_args* a, void* d_work, size_t bytes, void* stream) {
  if (!a) return fail(PSMS_E_INVAL, "NULL args");
  const int nc = a->nc;
  const long long nl = a->nlines;
  if (nc < 4 || nl < 0 || a->reserved != 0) return fail(PSMS_E_INVAL, "bad nc, nlines or reserved");
  if (!(a->beta_ns >= 0.0) || !(a->beta_a > 0.0) || !(a->beta_b > 0.0))
    return fail(PSMS_E_INVAL, "beta_ns must be >= 0 and beta_a, beta_b > 0");
  if (nl == 0) return PSMS_OK;
  if (!a->d_kx || !a->d_ky || !a->d_g_om || !a->d_g_w || !a->d_g_phi || !a->d_om || !a->d_w || !a->d_phi ||
      !a->d_u || !a->d_v)
    return fail(PSMS_E_INVAL, "NULL argument");
  const WallLayout L = wall_layout(nc, nl);
  if (!d_work || !aligned(d_work)) return fail(PSMS_E_WORKSPACE, "workspace NULL or misaligned");
  if (bytes < L.total) return fail(PSMS_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
  char* w = static_cast<char*>(d_work);
  auto C = [&](size_t off) { return reinterpret_cast<cpx<double>*>(w + off); };
  auto CC = [](const double* p) { return reinterpret_cast<const cpx<double>*>(p); };
  auto CM = [](double* p) { return reinterpret_cast<cpx<double>*>(p); };
  double* xw = reinterpret_cast<double*>(w + L.xw);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const cpx<double> z0 = {0.0, 0.0}, one = {1.0, 0.0};
  hipError_t e;
#define PSMS_TRY(x) \
  if ((e = (x)) != hipSuccess) return hip_fail(e, "wall_solve")
  // the independent problems share a launch: omega_z and the three psi
  // problems of w (particular, unit value at the top, at the bottom); then w
  // from each psi and the first CH factor; then phi; then the influence-matrix
  // combination
  const long long xs = (long long)(align256(size_t(nc + 1) * size_t(nl) * sizeof(double)) / sizeof(double));
  psms::HelmBatch b{};
  b.np = 4;
  b.p[0] = psms::HelmProblem{CC(a->d_g_om), CM(a->d_om), xw, nl, a->beta_ns, a->d_kx, a->d_ky, 0, z0, z0};
  b.p[1] = psms::HelmProblem{CC(a->d_g_w), C(L.psi), xw + xs, nl, a->beta_ns, a->d_kx, a->d_ky, 0, z0, z0};
  b.p[2] = psms::HelmProblem{nullptr, C(L.psit), xw + 2 * xs, nl, a->beta_ns, a->d_kx, a->d_ky, 0, one, z0};
  b.p[3] = psms::HelmProblem{nullptr, C(L.psib), xw + 3 * xs, nl, a->beta_ns, a->d_kx, a->d_ky, 0, z0, one};
  PSMS_TRY(psms::launch_helm_batch(b, nc, st));
  b.p[0] = psms::HelmProblem{C(L.psi), CM(a->d_w), xw, nl, 0.0, a->d_kx, a->d_ky, 0, z0, z0};
  b.p[1] = psms::HelmProblem{C(L.psit), C(L.wt), xw + xs, nl, 0.0, a->d_kx, a->d_ky, 0, z0, z0};
  b.p[2] = psms::HelmProblem{C(L.psib), C(L.wb), xw + 2 * xs, nl, 0.0, a->d_kx, a->d_ky, 0, z0, z0};
  b.p[3] = psms::HelmProblem{CC(a->d_g_phi), C(L.xi), xw + 3 * xs, nl, a->beta_a, a->d_kx, a->d_ky, 3, z0, z0};
  PSMS_TRY(psms::launch_helm_batch(b, nc, st));
  b.np = 1;
  b.p[0] = psms::HelmProblem{C(L.xi), CM(a->d_phi), xw, nl, a->beta_b, a->d_kx, a->d_ky, 3, z0, z0};
  PSMS_TRY(psms::launch_helm_batch(b, nc, st));
  PSMS_TRY(psms::launch_influence(CM(a->d_w), C(L.wt), C(L.wb), nc, nl, a->d_kx, a->d_ky, st));
  // u, v
  PSMS_TRY(psms::launch_chebd(CM(a->d_w), C(L.dw), nc, nl, st));
  PSMS_TRY(psms::launch_uv(CM(a->d_om), C(L.dw), CM(a->d_u), CM(a->d_v), nc, nl, a->d_kx, a->d_ky, st));
#undef PSMS_TRY
  return PSMS_OK;
}

// ---------------------------------------------------------------------------
// batches of independent boxes
// ---------------------------------------------------------------------------
}  // extern "C"

struct psms_batch {
  struct Group {
    int n;
    std::vector<int> members;
    psms::BoxDev* d_table;
    std::vector<psms::BoxDev> h_table;
    int variant[4];
  };
  int nbox;
  int prec;
  hipStream_t stream;
  std::vector<psms_ctx*> box;
  std::vector<Group> groups;
  std::vector<int> table_ab1;  // per box, value last written (-1: never)
  hipGraph_t graph;
  hipGraphExec_t exec;
  int graph_valid;
};

namespace {

struct BatchLayout {
  std::vector<size_t> box_off;
  std::vector<size_t> box_bytes;
  size_t tables;
  size_t total;
};

int batch_layout(int32_t nbox, const psms_params* p, BatchLayout* L) {
  if (nbox < 1 || !p) return fail(PSMS_E_INVAL, "nbox must be >= 1 and params non-NULL");
  size_t off = 0;
  L->box_off.assign(nbox, 0);
  L->box_bytes.assign(nbox, 0);
  for (int i = 0; i < nbox; ++i) {
    int r = validate(&p[i]);
    if (r) return r;
    if (p[i].precision != p[0].precision) return fail(PSMS_E_INVAL, "all boxes of a batch share one precision");
    if (p[i].cube != 0) return fail(PSMS_E_NOTSUP, "batched boxes take the grid cube (cube = 0)");
    L->box_off[i] = off;
    L->box_bytes[i] = make_layout(p[i]).total;
    off = align256(off + L->box_bytes[i]);
  }
  L->tables = off;
  off = align256(off + size_t(nbox) * sizeof(psms::BoxDev));
  L->total = off;
  return PSMS_OK;
}

void batch_drop_graph(psms_batch* b) {
  if (b->graph_valid) {
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
    b->graph_valid = 0;
  }
}

// Write each group's descriptor table where a box's Adams-Bashforth flag changed.
hipError_t batch_sync_tables(psms_batch* b) {
  for (auto& g : b->groups) {
    bool dirty = false;
    for (size_t j = 0; j < g.members.size(); ++j) {
      psms_ctx* c = b->box[g.members[j]];
      const int ab1 = (c->nstep == 0) ? 1 : 0;
      if (b->table_ab1[g.members[j]] != ab1) {
        g.h_table[j].sc = step_coef(c);
        b->table_ab1[g.members[j]] = ab1;
        dirty = true;
      }
    }
    if (dirty) {
      hipError_t e = hipMemcpyAsync(g.d_table, g.h_table.data(), g.h_table.size() * sizeof(psms::BoxDev),
                                    hipMemcpyHostToDevice, b->stream);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

template <typename T>
hipError_t batch_stage(psms_batch* b, int stage, int do_update) {
  for (auto& g : b->groups) {
    const psms_ctx* c0 = b->box[g.members[0]];
    hipError_t e = psms::launch_step_stage<T>(g.n, stage, g.variant[stage], g.d_table, 0, int(g.members.size()),
                                              twiddles<T>(c0), do_update, b->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t batch_one_step(psms_batch* b) {
  for (int stage = 0; stage < 4; ++stage) {
    hipError_t e = batch_stage<T>(b, stage, 1);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

int psms_batch_workspace_bytes(int32_t nbox, const psms_params* p, size_t* bytes) {
  if (!bytes) return fail(PSMS_E_INVAL, "bytes is NULL");
  BatchLayout L;
  int r = batch_layout(nbox, p, &L);
  if (r) return r;
  *bytes = L.total;
  return PSMS_OK;
}

int psms_batch_create(psms_batch** out, int32_t nbox, const psms_params* p, void* d_workspace, size_t bytes,
                      void* stream) {
  if (!out) return fail(PSMS_E_INVAL, "out is NULL");
  *out = nullptr;
  BatchLayout L;
  int r = batch_layout(nbox, p, &L);
  if (r) return r;
  if (!d_workspace || !aligned(d_workspace)) return fail(PSMS_E_WORKSPACE, "workspace NULL or misaligned");
  if (bytes < L.total) return fail(PSMS_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
  psms_batch* b = new psms_batch();
  b->nbox = nbox;
  b->prec = p[0].precision;
  b->stream = static_cast<hipStream_t>(stream);
  b->graph_valid = 0;
  char* ws = static_cast<char*>(d_workspace);
  for (int i = 0; i < nbox; ++i) {
    psms_ctx* c = nullptr;
    r = psms_create(&c, &p[i], ws + L.box_off[i], L.box_bytes[i], stream);
    if (r) {
      for (psms_ctx* q : b->box) psms_destroy(q);
      delete b;
      return r;
    }
    b->box.push_back(c);
  }
  b->table_ab1.assign(nbox, -1);
  // group by size, tables laid out contiguously per group
  std::vector<int> order(nbox);
  for (int i = 0; i < nbox; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return p[x].n < p[y].n; });
  psms::BoxDev* table = reinterpret_cast<psms::BoxDev*>(ws + L.tables);
  size_t used = 0;
  for (int idx : order) {
    if (b->groups.empty() || b->groups.back().n != p[idx].n) {
      psms_batch::Group g;
      g.n = p[idx].n;
      g.d_table = table + used;
      for (int s = 0; s < 4; ++s) g.variant[s] = 2;
      b->groups.push_back(g);
    }
    psms_batch::Group& g = b->groups.back();
    g.members.push_back(idx);
    g.h_table.push_back(b->box[idx]->h_box);
    ++used;
  }
  hipError_t e = batch_sync_tables(b);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    for (psms_ctx* q : b->box) psms_destroy(q);
    delete b;
    return hip_fail(e, "batch_create");
  }
  *out = b;
  return PSMS_OK;
}

int psms_batch_destroy(psms_batch* b) {
  if (!b) return PSMS_OK;
  batch_drop_graph(b);
  for (psms_ctx* c : b->box) psms_destroy(c);
  delete b;
  return PSMS_OK;
}

int psms_batch_init_state(psms_batch* b, int32_t box, const double* d_u, const double* d_phi) {
  if (!b || box < 0 || box >= b->nbox) return fail(PSMS_E_INVAL, "bad batch or box index");
  return psms_init_state(b->box[box], d_u, d_phi);
}

int psms_batch_get_state(psms_batch* b, int32_t box, double* d_uhat, double* d_phihat) {
  if (!b || box < 0 || box >= b->nbox) return fail(PSMS_E_INVAL, "bad batch or box index");
  return psms_get_state(b->box[box], d_uhat, d_phihat, nullptr);
}

int psms_batch_diagnostics(psms_batch* b, int32_t box, psms_diag* h_out) {
  if (!b || box < 0 || box >= b->nbox) return fail(PSMS_E_INVAL, "bad batch or box index");
  return psms_diagnostics(b->box[box], h_out);
}

int psms_batch_step(psms_batch* b, int32_t nsteps, int32_t use_graph) {
  if (!b || nsteps < 0) return fail(PSMS_E_INVAL, "bad batch or nsteps");
  bool need_prologue = false;
  for (psms_ctx* c : b->box) {
    if (!c->have_state) return fail(PSMS_E_STATE, "a box of the batch has no state");
    if (!c->g_valid) need_prologue = true;
  }
  if (nsteps == 0) return PSMS_OK;
  const bool mixed = b->prec == PSMS_MIXED;
  hipError_t e = batch_sync_tables(b);
  if (e == hipSuccess && need_prologue) e = mixed ? batch_stage<float>(b, 3, 0) : batch_stage<double>(b, 3, 0);
  if (e != hipSuccess) return hip_fail(e, "batch prologue");
  for (psms_ctx* c : b->box) c->g_valid = 1;
  for (int s = 0; s < nsteps; ++s) {
    e = batch_sync_tables(b);
    bool any_ab1 = false;
    for (psms_ctx* c : b->box) any_ab1 |= (c->nstep == 0);
    const bool graph = use_graph && b->stream != nullptr && !any_ab1;
    if (e == hipSuccess && graph && !b->graph_valid) {
      e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t e2 = mixed ? batch_one_step<float>(b) : batch_one_step<double>(b);
        e = hipStreamEndCapture(b->stream, &b->graph);
        if (e2 != hipSuccess) e = e2;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
      if (e == hipSuccess) b->graph_valid = 1;
    }
    if (e == hipSuccess) {
      if (graph) e = hipGraphLaunch(b->exec, b->stream);
      else e = mixed ? batch_one_step<float>(b) : batch_one_step<double>(b);
    }
    if (e != hipSuccess) {
      for (psms_ctx* c : b->box) c->g_valid = 0;
      return hip_fail(e, "batch_step");
    }
    for (psms_ctx* c : b->box) c->nstep += 1;
  }
  return PSMS_OK;
}

int psms_batch_groups(const psms_batch* b, int32_t* h_ngroups, int32_t* h_n, int32_t* h_count) {
  if (!b || !h_ngroups) return fail(PSMS_E_INVAL, "NULL argument");
  *h_ngroups = int32_t(b->groups.size());
  for (size_t i = 0; i < b->groups.size(); ++i) {
    if (h_n) h_n[i] = b->groups[i].n;
    if (h_count) h_count[i] = int32_t(b->groups[i].members.size());
  }
  return PSMS_OK;
}

int psms_batch_set_variants(psms_batch* b, const int32_t* h_variants) {
  if (!b || !h_variants) return fail(PSMS_E_INVAL, "NULL argument");
  for (size_t i = 0; i < 4 * b->groups.size(); ++i)
    if (h_variants[i] < 0 || h_variants[i] >= psms::kStepVariants) return fail(PSMS_E_INVAL, "variant out of range");
  for (size_t i = 0; i < b->groups.size(); ++i)
    for (int s = 0; s < 4; ++s) b->groups[i].variant[s] = h_variants[4 * i + s];
  batch_drop_graph(b);
  return PSMS_OK;
}

int psms_batch_autotune(psms_batch* b, int32_t reps, int32_t* h_variants, double* h_ms) {
  if (!b || reps < 1) return fail(PSMS_E_INVAL, "bad batch or reps");
  for (psms_ctx* c : b->box)
    if (c->have_state) return fail(PSMS_E_STATE, "autotune runs on an empty batch: call it before init_state");
  const bool mixed = b->prec == PSMS_MIXED;
  hipError_t e = hipSuccess;
  // zero every box's workspace so the timed kernels see finite data
  for (psms_ctx* c : b->box)
    if (e == hipSuccess) e = hipMemsetAsync(c->state, 0, c->lay.tw64 - c->lay.state, b->stream);  // state..bufb
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = batch_sync_tables(b);
  for (size_t gi = 0; e == hipSuccess && gi < b->groups.size(); ++gi) {
    psms_batch::Group& g = b->groups[gi];
    const psms_ctx* c0 = b->box[g.members[0]];
    for (int stage = 0; e == hipSuccess && stage < 4; ++stage) {
      double best = 1e300;
      int arg = 2;
      for (int v = 0; e == hipSuccess && v < psms::kStepVariants; ++v) {
        auto run = [&]() {
          return mixed ? psms::launch_step_stage<float>(g.n, stage, v, g.d_table, 0, int(g.members.size()),
                                                        twiddles<float>(c0), 1, b->stream)
                       : psms::launch_step_stage<double>(g.n, stage, v, g.d_table, 0, int(g.members.size()),
                                                         twiddles<double>(c0), 1, b->stream);
        };
        e = run();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        for (int r = 0; e == hipSuccess && r < reps; ++r) e = run();
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        const double avg = double(ms) / reps;
        if (h_ms) h_ms[(gi * 4 + stage) * psms::kStepVariants + v] = avg;
        if (avg < best) {
          best = avg;
          arg = v;
        }
      }
      g.variant[stage] = arg;
      if (h_variants) h_variants[gi * 4 + stage] = arg;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  batch_drop_graph(b);
  for (psms_ctx* c : b->box) c->g_valid = 0;
  if (e != hipSuccess) return hip_fail(e, "batch_autotune");
  return PSMS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// discrete adjoint with segment checkpointing
// ---------------------------------------------------------------------------
struct psms_adjoint {
  psms_params p;
  int max_steps, seg_len, nckpt;
  hipStream_t stream;
  psms_ctx* prim;  // primal run, in the requested precision
  psms_ctx* rec;   // FP64 recompute inside a segment
  cpx<double>* lam;
  cpx<double>* mu;
  cpx<double>* seg;    // seg_len states (4 M each)
  cpx<double>* ckpt;   // nckpt (state, history) pairs (8 M each)
  cpx<double>* adja;   // [8][n][C][H]
  cpx<double>* adjb;   // [8][n][n][H]
  double* part;
  double* acc;         // dJ/dWe accumulator
  int nsteps;          // steps of the last forward run (-1: none)
};

namespace {
struct AdjLayout {
  size_t prim, prim_bytes, rec, rec_bytes, lam, mu, seg, ckpt, adja, adjb, part, acc, total;
  int nckpt;
};
int adjoint_layout(const psms_params* p, int32_t max_steps, int32_t seg_len, AdjLayout* L) {
  int r = validate(p);
  if (r) return r;
  if (p->cube != 0) return fail(PSMS_E_NOTSUP, "the adjoint differentiates the grid cube (cube = 0)");
  if (max_steps < 1 || seg_len < 1) return fail(PSMS_E_INVAL, "max_steps and seg_len must be >= 1");
  psms_params p64 = *p;
  p64.precision = PSMS_FP64;
  const BoxGeom g = make_geom(p->n);
  const size_t n = size_t(p->n);
  const size_t st = 4 * size_t(g.M) * sizeof(cpx<double>);
  size_t off = 0;
  L->prim = off; L->prim_bytes = make_layout(*p).total; off = align256(off + L->prim_bytes);
  L->rec = off; L->rec_bytes = make_layout(p64).total; off = align256(off + L->rec_bytes);
  L->lam = off; off = align256(off + st);
  L->mu = off; off = align256(off + st);
  L->seg = off; off = align256(off + size_t(seg_len) * st);
  L->nckpt = (max_steps + seg_len - 1) / seg_len;
  L->ckpt = off; off = align256(off + size_t(L->nckpt) * 2 * st);
  L->adja = off; off = align256(off + 8 * n * size_t(g.Q) * sizeof(cpx<double>));
  L->adjb = off; off = align256(off + std::max(8 * n * n * size_t(g.H), n * n * (n / 2 + 1)) * sizeof(cpx<double>));
  L->part = off; off = align256(off + size_t(psms::adj_xblocks(p->n)) * sizeof(double));
  L->acc = off; off = align256(off + 8 * sizeof(double));
  L->total = off;
  return PSMS_OK;
}

// y-direction transform of nf fields between band (C) and full (n) layouts, FP64.
hipError_t y_lines64(psms_ctx* c, int dir, const cpx<double>* in, cpx<double>* out, int nf) {
  const BoxGeom& g = c->g;
  const int n = g.n;
  psms::LineArgs la{};
  la.n_in = dir > 0 ? g.C : n;
  la.n_out = dir > 0 ? n : g.C;
  la.inner = g.H;
  la.nlines = (long long)n * g.H;
  la.in_fstride = dir > 0 ? (long long)n * g.Q : (long long)n * n * g.H;
  la.out_fstride = dir > 0 ? (long long)n * n * g.H : (long long)n * g.Q;
  la.fmap = 0;
  for (unsigned i = 0; i < 8; ++i) la.fmap |= i << (4 * i);
  la.scale = 1.0;
  return psms::launch_lines<double>(n, dir, in, out, c->tw64, la, nf, c->stream);
}
}  // namespace

extern "C" {

int psms_adjoint_workspace_bytes(const psms_params* p, int32_t max_steps, int32_t seg_len, size_t* bytes) {
  if (!bytes) return fail(PSMS_E_INVAL, "bytes is NULL");
  AdjLayout L;
  int r = adjoint_layout(p, max_steps, seg_len, &L);
  if (r) return r;
  *bytes = L.total;
  return PSMS_OK;
}

int psms_adjoint_create(psms_adjoint** out, const psms_params* p, int32_t max_steps, int32_t seg_len,
                        void* d_workspace, size_t bytes, void* stream) {
  if (!out) return fail(PSMS_E_INVAL, "out is NULL");
  *out = nullptr;
  AdjLayout L;
  int r = adjoint_layout(p, max_steps, seg_len, &L);
  if (r) return r;
  if (!d_workspace || !aligned(d_workspace)) return fail(PSMS_E_WORKSPACE, "workspace NULL or misaligned");
  if (bytes < L.total) return fail(PSMS_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
  char* ws = static_cast<char*>(d_workspace);
  psms_adjoint* a = new psms_adjoint();
  a->p = *p;
  a->max_steps = max_steps;
  a->seg_len = seg_len;
  a->nckpt = L.nckpt;
  a->stream = static_cast<hipStream_t>(stream);
  psms_params p64 = *p;
  p64.precision = PSMS_FP64;
  r = psms_create(&a->prim, p, ws + L.prim, L.prim_bytes, stream);
  if (!r) r = psms_create(&a->rec, &p64, ws + L.rec, L.rec_bytes, stream);
  if (r) {
    psms_destroy(a->prim);
    delete a;
    return r;
  }
  a->lam = reinterpret_cast<cpx<double>*>(ws + L.lam);
  a->mu = reinterpret_cast<cpx<double>*>(ws + L.mu);
  a->seg = reinterpret_cast<cpx<double>*>(ws + L.seg);
  a->ckpt = reinterpret_cast<cpx<double>*>(ws + L.ckpt);
  a->adja = reinterpret_cast<cpx<double>*>(ws + L.adja);
  a->adjb = reinterpret_cast<cpx<double>*>(ws + L.adjb);
  a->part = reinterpret_cast<double*>(ws + L.part);
  a->acc = reinterpret_cast<double*>(ws + L.acc);
  a->nsteps = -1;
  *out = a;
  return PSMS_OK;
}

int psms_adjoint_destroy(psms_adjoint* a) {
  if (!a) return PSMS_OK;
  psms_destroy(a->prim);
  psms_destroy(a->rec);
  delete a;
  return PSMS_OK;
}

int psms_adjoint_forward(psms_adjoint* a, const double* d_u0, const double* d_phi0, int32_t nsteps, double* h_J) {
  if (!a || !d_u0 || !d_phi0 || !h_J) return fail(PSMS_E_INVAL, "NULL argument");
  if (nsteps < 1 || nsteps > a->max_steps) return fail(PSMS_E_INVAL, "nsteps must be in 1..max_steps");
  int r = psms_init_state(a->prim, d_u0, d_phi0);
  if (r) return r;
  psms_ctx* c = a->prim;
  const size_t st = 4 * size_t(c->g.M) * sizeof(cpx<double>);
  const long long M4 = 4 * c->g.M;
  for (int s = 0; s * a->seg_len < nsteps; ++s) {
    hipError_t e = hipMemcpyAsync(a->ckpt + 2 * s * M4, c->state, st, hipMemcpyDeviceToDevice, a->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(a->ckpt + (2 * s + 1) * M4, c->hist, st, hipMemcpyDeviceToDevice, a->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint checkpoint");
    const int k = std::min(a->seg_len, nsteps - s * a->seg_len);
    r = psms_step(c, k);
    if (r) return r;
  }
  psms_diag d;
  r = psms_diagnostics(c, &d);
  if (r) return r;
  if (d.nonfinite) return fail(PSMS_E_NONFINITE, "non-finite state in the forward run");
  const double vol = 8.0 * M_PI * M_PI * M_PI;
  *h_J = vol * (d.grad2 + d.ke);
  a->nsteps = nsteps;
  return PSMS_OK;
}

int psms_adjoint_backward(psms_adjoint* a, double* d_dphi0, double* h_dwe) {
  if (!a || !d_dphi0 || !h_dwe) return fail(PSMS_E_INVAL, "NULL argument");
  if (a->nsteps < 1) return fail(PSMS_E_STATE, "backward before forward");
  psms_ctx* c = a->rec;
  const BoxGeom& g = c->g;
  const int n = g.n;
  const size_t st = 4 * size_t(g.M) * sizeof(cpx<double>);
  const long long M4 = 4 * g.M;
  hipStream_t S = a->stream;
  const double vol = 8.0 * M_PI * M_PI * M_PI;
  const double csig = 3.0 / std::sqrt(8.0) * a->p.ch / a->p.we;
  const double n3 = double(n) * n * n;
  hipError_t e;
#define PSMS_TRY(x) \
  if ((e = (x)) != hipSuccess) return hip_fail(e, "adjoint_backward")
  PSMS_TRY(psms::launch_adj_terminal(a->prim->state, a->lam, a->mu, g.K, g.C, g.H, g.M, vol, S));
  PSMS_TRY(hipMemsetAsync(a->acc, 0, sizeof(double), S));
  const int nseg = (a->nsteps + a->seg_len - 1) / a->seg_len;
  psms::AdjCoef ac;
  ac.dt = a->p.dt;
  ac.nu = 1.0 / a->p.re;
  ac.ch2_pe = a->p.ch * a->p.ch / a->p.pe;
  ac.s = c->s;
  ac.inv_pe = 1.0 / a->p.pe;
  ac.e_coef = (1.0 + c->s * a->p.ch * a->p.ch) / a->p.pe;
  ac.inv_n3 = 1.0 / n3;
  for (int s = nseg - 1; s >= 0; --s) {
    const int n0 = s * a->seg_len;
    const int n1 = std::min(n0 + a->seg_len, a->nsteps);
    // states x^n0 .. x^(n1-1) of the segment, recomputed in FP64 from the checkpoint
    PSMS_TRY(hipMemcpyAsync(c->state, a->ckpt + 2 * s * M4, st, hipMemcpyDeviceToDevice, S));
    PSMS_TRY(hipMemcpyAsync(c->hist, a->ckpt + (2 * s + 1) * M4, st, hipMemcpyDeviceToDevice, S));
    c->nstep = n0;
    c->have_state = 1;
    c->g_valid = 0;
    PSMS_TRY(hipMemcpyAsync(a->seg, c->state, st, hipMemcpyDeviceToDevice, S));
    for (int m = n0; m < n1 - 1; ++m) {
      int r = psms_step(c, 1);
      if (r) return r;
      PSMS_TRY(hipMemcpyAsync(a->seg + size_t(m - n0 + 1) * M4, c->state, st, hipMemcpyDeviceToDevice, S));
    }
    for (int m = n1 - 1; m >= n0; --m) {
      // forward fields of x^m: z-inverse and y-inverse into the recompute context
      PSMS_TRY(hipMemcpyAsync(c->state, a->seg + size_t(m - n0) * M4, st, hipMemcpyDeviceToDevice, S));
      PSMS_TRY(psms::launch_step_stage<double>(n, 3, 2, c->d_box, 0, 1, c->tw64, 0, S));
      PSMS_TRY(psms::launch_step_stage<double>(n, 0, 2, c->d_box, 0, 1, c->tw64, 1, S));
      ac.alpha = (m == 0) ? 1.0 : 1.5;
      ac.beta = (m == 0) ? 0.0 : -0.5;
      PSMS_TRY(psms::launch_adj_stage(n, 0, a->lam, a->mu, nullptr, nullptr, a->adja, c->tw64, ac, csig, nullptr, S));
      PSMS_TRY(y_lines64(c, +1, a->adja, a->adjb, 8));
      PSMS_TRY(psms::launch_adj_stage(n, 1, a->lam, a->mu, static_cast<const cpx<double>*>(c->bufa), a->adjb,
                                      static_cast<cpx<double>*>(c->bufb), c->tw64, ac, csig, a->part, S));
      PSMS_TRY(psms::launch_adj_sum(a->part, psms::adj_xblocks(n), -csig / (a->p.we * n3), a->acc, S));
      PSMS_TRY(y_lines64(c, -1, static_cast<const cpx<double>*>(c->bufb), a->adja, 7));
      PSMS_TRY(psms::launch_adj_stage(n, 2, a->lam, a->mu, a->adja, nullptr, nullptr, c->tw64, ac, csig, nullptr, S));
    }
  }
  // dJ/dphi0 on the grid: inv(D lam_phi) / n^3
  PSMS_TRY(psms::launch_expand<double>(a->lam + 3 * g.M, a->adjb, g, 1, S));
  PSMS_TRY(psms::launch_spec_finish<double>(a->adjb, a->adjb, g, 1, 0, -1, 1.0 / n3, S));
  c->g_valid = 0;
  PSMS_TRY(transform_fields<double>(c, -1, 1, a->adjb, d_dphi0, 0));
  PSMS_TRY(hipMemcpyAsync(h_dwe, a->acc, sizeof(double), hipMemcpyDeviceToHost, S));
  PSMS_TRY(hipStreamSynchronize(S));
#undef PSMS_TRY
  return PSMS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// the channel step (Sec. 2.2): Fourier in x and y, Chebyshev in z
// ---------------------------------------------------------------------------
namespace {

struct ChanLayout {
  size_t kx, ky, twx64, twx32, twy64, twy32, twz64, twz32;
  size_t state, mean, hist, hmean;
  size_t dw, dphi, A, A2, B, C, R, D3, DQ, lapc, lapom, lappsi, G;
  size_t d2mean, gmean, wt, wb, M, whp, mhp, psip, xi, xw, diag, xdev, fac, total;
  bool has_fac;   // the step's tau problems read precomputed elimination factors
};

// the step's six tau problems (omega_z, psi_p, the mean line, xi, w_p, phi)
// each keep a table of elimination factors, in this order
enum { kChanFacOm, kChanFacPsi, kChanFacMean, kChanFacXi, kChanFacW, kChanFacPhi, kChanFacCount };

constexpr int kChanDiagBlocks = 1024;   // partial sums of the diagnostics

psms::ChanGeom chan_geom(const psms_channel_params& p) {
  psms::ChanGeom g{};
  g.nx = p.nx;
  g.ny = p.ny;
  g.nc = p.nc;
  g.Kx = (p.nx - 1) / 3;
  g.Hx = g.Kx + 1;
  g.Ky = (p.ny - 1) / 3;
  g.Cy = 2 * g.Ky + 1;
  g.Kz = (2 * p.nc - 1) / 3;
  g.NL = (long long)g.Cy * g.Hx;
  g.NZL = (long long)(p.nc + 1) * g.NL;
  g.P = (long long)(p.nc + 1) * p.ny * p.nx;
  g.sp = p.single_phase ? 1 : 0;
  g.nf_in = g.sp ? 3 : 7;
  g.nf_out = g.sp ? 6 : 8;
  return g;
}

ChanLayout chan_layout(const psms_channel_params& p) {
  const psms::ChanGeom g = chan_geom(p);
  const size_t t = (p.precision == PSMS_MIXED) ? sizeof(cpx<float>) : sizeof(cpx<double>);
  const size_t tr = t / 2;
  const size_t nz = size_t(p.nc) + 1;
  const size_t c64 = sizeof(cpx<double>);
  const size_t arr = align256(size_t(g.NZL) * c64);
  ChanLayout L{};
  size_t off = 0;
  auto take = [&](size_t& field, size_t bytes) {
    field = off;
    off += align256(bytes);
  };
  take(L.kx, size_t(g.NL) * sizeof(double));
  take(L.ky, size_t(g.NL) * sizeof(double));
  take(L.twx64, size_t(p.nx) * c64);
  take(L.twx32, size_t(p.nx) * sizeof(cpx<float>));
  take(L.twy64, size_t(p.ny) * c64);
  take(L.twy32, size_t(p.ny) * sizeof(cpx<float>));
  take(L.twz64, size_t(2 * p.nc) * c64);
  take(L.twz32, size_t(2 * p.nc) * sizeof(cpx<float>));
  take(L.state, 3 * arr);
  take(L.mean, 2 * nz * c64);
  take(L.hist, 3 * arr);
  take(L.hmean, 2 * nz * c64);
  take(L.dw, arr);
  take(L.dphi, arr);
  take(L.A, 8 * size_t(g.NZL) * t);
  take(L.A2, 8 * size_t(g.NZL) * t);
  take(L.B, 8 * nz * size_t(p.ny) * size_t(g.Hx) * t);
  take(L.C, 8 * size_t(g.P) * tr);
  take(L.R, 8 * arr);
  take(L.D3, 3 * arr);
  take(L.DQ, arr);
  take(L.lapc, arr);
  take(L.lapom, arr);
  take(L.lappsi, arr);
  take(L.G, 3 * arr);
  take(L.d2mean, 2 * nz * c64);
  take(L.gmean, 2 * nz * c64);
  take(L.wt, arr);
  take(L.wb, arr);
  take(L.M, 4 * size_t(g.NL) * sizeof(double));
  take(L.whp, nz * size_t(g.NL) * sizeof(double));
  take(L.mhp, 2 * size_t(g.NL) * sizeof(double));
  take(L.psip, arr);
  take(L.xi, arr);
  // elimination factors of the tau problems: kept where the solves stay on
  // chip (same condition at both walls and a chain length the kernels unroll)
  const int fsw = p.free_slip & 3;
  L.has_fac = (fsw == 0 || fsw == 3) && psms::helm_fuses_influence(p.nc);
  take(L.fac, L.has_fac ? kChanFacCount * psms::helm_factor_doubles(p.nc, g.NL) * sizeof(double) : 0);
  take(L.xw, 4 * nz * size_t(g.NL) * sizeof(double));   // one elimination scratch per batched problem
  take(L.diag, (8 * size_t(kChanDiagBlocks) + 8) * sizeof(double));
  take(L.xdev, sizeof(psms::BoxDev));   // descriptor of the fused x stage
  L.total = off;
  return L;
}

int chan_validate(const psms_channel_params* p) {
  if (!p) return fail(PSMS_E_INVAL, "params is NULL");
  if (p->precision != PSMS_FP64 && p->precision != PSMS_MIXED) return fail(PSMS_E_INVAL, "precision");
  if (!psms::supported_n(p->nx) || !psms::supported_n(p->ny))
    return fail(PSMS_E_NOTSUP, "nx, ny must be one of 8 12 16 24 32 48 64 96 128 192 256");
  if (!psms::supported_nc(p->nc)) return fail(PSMS_E_NOTSUP, "nc must be one of 4 6 8 12 16 24 32 48 64 96 128 256");
  if (!(p->lx > 0) || !(p->ly > 0) || !(p->re > 0) || !(p->dt > 0) || !std::isfinite(p->forcing))
    return fail(PSMS_E_INVAL, "lx, ly, re, dt must be > 0, forcing finite");
  if (p->free_slip < 0 || p->free_slip > 3) return fail(PSMS_E_INVAL, "free_slip must be 0..3 (bit 0 top, bit 1 bottom)");
  if (p->single_phase) return PSMS_OK;   // we, ch, pe, s are not used
  if (!(p->we > 0) || !(p->ch > 0) || !(p->pe > 0) || !(p->s >= 0))
    return fail(PSMS_E_INVAL, "we, ch, pe must be > 0, s >= 0");
  const double s = (p->s > 0.0) ? p->s : std::sqrt(4.0 * p->pe / (p->ch * p->ch * p->dt));
  if (s * s < 4.0 * p->pe / (p->ch * p->ch * p->dt) * (1.0 - 1e-12))
    return fail(PSMS_E_INVAL, "s^2 < 4 Pe / (Ch^2 dt): the CH operator has no real factors");
  return PSMS_OK;
}

}  // namespace

struct psms_channel {
  psms_channel_params p;
  psms::ChanGeom g;
  psms::ChanCoef coef;
  ChanLayout lay;
  psms::BoxDev h_xdev;   // host copy of the x-stage descriptor (source of its upload)
  int use_graph = 0;     // replay a captured step after the first (psms_channel_set_graphs; needs a non-NULL stream)
  int graph_ok = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  char* ws;
  hipStream_t stream;
  double a_fac, b_fac;
  int nstep;
  int have_state;
  template <typename X>
  X* at(size_t off) const {
    return reinterpret_cast<X*>(ws + off);
  }
};

namespace {

template <typename T>
const cpx<T>* chan_tw(const psms_channel* c, bool x) {
  if (std::is_same<T, double>::value)
    return reinterpret_cast<const cpx<T>*>(c->ws + (x ? c->lay.twx64 : c->lay.twy64));
  return reinterpret_cast<const cpx<T>*>(c->ws + (x ? c->lay.twx32 : c->lay.twy32));
}
template <typename T>
const cpx<T>* chan_twz(const psms_channel* c) {
  return reinterpret_cast<const cpx<T>*>(c->ws + (std::is_same<T, double>::value ? c->lay.twz64 : c->lay.twz32));
}

// x-spectral [nf][z][y][kx band] (T) -> band [nf][n][line] (T): y lines (1/(nx ny)),
// DCT-I; with band64, the DCT-I writes FP64 coefficients there instead, n > Kz zeroed
template <typename T>
hipError_t chan_forward_yz(psms_channel* c, const cpx<T>* xs, cpx<T>* band, int nf, cpx<double>* band64) {
  const psms::ChanGeom& g = c->g;
  const long long nz = g.nc + 1;
  cpx<T>* A2 = c->at<cpx<T>>(c->lay.A2);
  hipError_t e;
  psms::LineArgs la{};
  la.n_in = g.ny;
  la.n_out = g.Cy;
  la.inner = g.Hx;
  la.nlines = nz * g.Hx;
  la.in_fstride = nz * g.ny * g.Hx;
  la.out_fstride = g.NZL;
  la.fmap = 0x76543210u;
  la.dmask = 0;
  la.scale = 1.0 / (double(g.nx) * double(g.ny));
  e = psms::launch_lines<T>(g.ny, -1, xs, A2, chan_tw<T>(c, false), la, nf, c->stream);
  if (e == hipSuccess)
    e = psms::launch_dct_fields<T>(g.nc, A2, band, g.NL, g.NZL, nf, chan_twz<T>(c), +1, c->stream, band64, g.Kz);
  return e;
}

// physical [nf][z][y][x] (T) -> band [nf][n][line] (T): x rows, then chan_forward_yz
template <typename T>
hipError_t chan_forward(psms_channel* c, const T* phys, cpx<T>* band, int nf, cpx<double>* band64 = nullptr) {
  const psms::ChanGeom& g = c->g;
  const long long nz = g.nc + 1;
  cpx<T>* B = c->at<cpx<T>>(c->lay.B);
  psms::RowArgs ra{};
  ra.nrows = nz * g.ny;
  ra.n_in = g.nx;
  ra.n_out = g.Hx;
  ra.in_fstride = g.P;
  ra.out_fstride = nz * g.ny * g.Hx;
  ra.scale = 1.0;
  hipError_t e = psms::launch_rows<T>(g.nx, -1, phys, B, chan_tw<T>(c, true), ra, nf, c->stream);
  if (e != hipSuccess) return e;
  return chan_forward_yz<T>(c, B, band, nf, band64);
}

// band [nf][n][line] (T) -> x-spectral [nf][z][y][kx band] (T) in the buffer B:
// DCT-I, y lines
// band [nf][n][line] (T; or, with fs, the step's six fields formed from the
// state as the transform loads them) -> y-expanded [nf][z][y][x-band] (T)
template <typename T>
hipError_t chan_inverse_yz(psms_channel* c, const cpx<T>* band, int nf, const psms::ChanFieldSrc* fs = nullptr) {
  const psms::ChanGeom& g = c->g;
  const long long nz = g.nc + 1;
  cpx<T>* B = c->at<cpx<T>>(c->lay.B);
  cpx<T>* A2 = c->at<cpx<T>>(c->lay.A2);
  hipError_t e = fs ? psms::launch_dct_chfields<T>(g.nc, *fs, A2, g.NZL, chan_twz<T>(c), c->stream)
                    : psms::launch_dct_fields<T>(g.nc, band, A2, g.NL, g.NZL, nf, chan_twz<T>(c), -1, c->stream);
  if (e != hipSuccess) return e;
  psms::LineArgs la{};
  la.n_in = g.Cy;
  la.n_out = g.ny;
  la.inner = g.Hx;
  la.nlines = nz * g.Hx;
  la.in_fstride = g.NZL;
  la.out_fstride = nz * g.ny * g.Hx;
  la.fmap = 0x76543210u;
  la.dmask = 0;
  la.scale = 1.0;
  return psms::launch_lines<T>(g.ny, +1, A2, B, chan_tw<T>(c, false), la, nf, c->stream);
}

// band [nf][n][line] (T) -> physical [nf][z][y][x] (T)
template <typename T>
hipError_t chan_inverse(psms_channel* c, const cpx<T>* band, T* phys, int nf) {
  const psms::ChanGeom& g = c->g;
  const long long nz = g.nc + 1;
  cpx<T>* B = c->at<cpx<T>>(c->lay.B);
  hipError_t e = chan_inverse_yz<T>(c, band, nf);
  if (e != hipSuccess) return e;
  psms::RowArgs ra{};
  ra.nrows = nz * g.ny;
  ra.n_in = g.Hx;
  ra.n_out = g.nx;
  ra.in_fstride = nz * g.ny * g.Hx;
  ra.out_fstride = g.P;
  ra.scale = 1.0;
  return psms::launch_rows<T>(g.nx, +1, B, phys, chan_tw<T>(c, true), ra, nf, c->stream);
}

template <typename T>
hipError_t chan_step_once(psms_channel* c) {
  const psms::ChanGeom& g = c->g;
  const ChanLayout& L = c->lay;
  hipStream_t st = c->stream;
  const int nc = g.nc;
  const long long nl = g.NL;
  auto C64 = [&](size_t off) { return c->at<cpx<double>>(off); };
  cpx<double>* om = C64(L.state);
  cpx<double>* w = om + g.NZL;
  cpx<double>* phi = w + g.NZL;
  const double* kx = c->at<double>(L.kx);
  const double* ky = c->at<double>(L.ky);
  cpx<double>* R = C64(L.R);
  hipError_t e;
#define PSMS_TRY(x) \
  if ((e = (x)) != hipSuccess) return e
  // 1-2. fields and the inverse transforms
  psms::ChebBatch cb{};
  cb.n = g.sp ? 1 : 2;
  cb.in[0] = w;
  cb.out[0] = C64(L.dw);
  cb.in[1] = phi;
  cb.out[1] = C64(L.dphi);
  PSMS_TRY(psms::launch_cheb_batch(cb, nc, nl, kx, ky, 0, st));
  if (g.sp) {
    PSMS_TRY(psms::launch_ch_fields<T>(g, om, w, phi, C64(L.dw), C64(L.dphi), C64(L.mean), kx, ky,
                                       c->at<cpx<T>>(L.A), st));
    PSMS_TRY(chan_inverse<T>(c, c->at<cpx<T>>(L.A), c->at<T>(L.C), g.nf_in));
    // 3-4. products and the forward transforms, 2/3 rule in x, y and z
    PSMS_TRY(psms::launch_ch_products<T>(g, c->at<T>(L.C), c->coef.csig, st));
    PSMS_TRY(chan_forward<T>(c, c->at<T>(L.C), c->at<cpx<T>>(L.A), g.nf_out, R));   // FP64, Chebyshev cut
  } else {
    // two-phase: u, v, w, phi, dy phi, dz phi through the DCT-I (each formed from
    // the state as the transform loads it) and y lines; the x-inverse, the 8
    // products and the x-forward in one pass (the box's x stage on (nc + 1) ny
    // rows; dx phi formed on load), so that no physical field is stored; then y
    // lines and the DCT-I with the Chebyshev cut (FP64)
    const psms::ChanFieldSrc fs{om, w, phi, C64(L.dw), C64(L.dphi), C64(L.mean), kx, ky, nl};
    PSMS_TRY(chan_inverse_yz<T>(c, nullptr, 6, &fs));
    PSMS_TRY(psms::launch_xstage_rows<T>(g.nx, c->at<psms::BoxDev>(L.xdev), chan_tw<T>(c, true),
                                         (long long)(nc + 1) * g.ny, 2.0 * M_PI / c->p.lx, st));
    PSMS_TRY(chan_forward_yz<T>(c, c->at<cpx<T>>(L.C), c->at<cpx<T>>(L.A), 8, R));
  }
  // 5. the wall-normal derivatives the right-hand sides need, in one launch:
  // D T_xz, D T_yz, D T_zz; (D^2 - k^2 + beta) omega_z; (D^2 - k^2 + beta) psi,
  // psi = (D^2 - k^2) w (its chain is in the same wavefront); D^2 - k^2 of
  // c / Pe - (1 + s Ch^2) / Pe phi; D^2 of the mean lines; then D Q (Q =
  // div_h S, S = div T, formed on the fly)
  cpx<double>* D3 = C64(L.D3);
  cb.n = g.sp ? 6 : 7;
  cb.in[0] = R + 4 * g.NZL;
  cb.out[0] = D3;
  cb.in[1] = R + 5 * g.NZL;
  cb.out[1] = D3 + g.NZL;
  cb.in[2] = R + 2 * g.NZL;
  cb.out[2] = D3 + 2 * g.NZL;
  cb.in[3] = om;
  cb.out[3] = C64(L.lapom);
  cb.addb[3] = c->coef.beta;
  cb.in[4] = w;
  cb.out[4] = nullptr;            // psi itself is not needed
  cb.out2[4] = C64(L.lappsi);
  cb.addb2[4] = c->coef.beta;
  if (!g.sp) {
    cb.in[5] = R + 7 * g.NZL;
    cb.in2[5] = phi;
    cb.w1[5] = c->coef.inv_pe;
    cb.w2[5] = -c->coef.e_coef;
    cb.out[5] = C64(L.lapc);
  }
  const int mj = g.sp ? 5 : 6;   // the mean lines U, V ([nc+1][2], k = 0): D^2
  cb.in[mj] = C64(L.mean);
  cb.out[mj] = C64(L.d2mean);
  cb.nl[mj] = 2;
  cb.nok = 1 << mj;
  PSMS_TRY(psms::launch_cheb_batch(cb, nc, nl, kx, ky, 0xF8, st));   // arrays 3.. : D^2 - k^2
  psms::ChebQ cq{R, R + g.NZL, R + 3 * g.NZL, D3, D3 + g.NZL};
  PSMS_TRY(psms::launch_chebd_q(cq, nc, nl, kx, ky, C64(L.DQ), st));
  // 6. Adams-Bashforth, Crank-Nicolson / implicit Euler right-hand sides
  c->coef.ab1 = (c->nstep == 0) ? 1 : 0;
  psms::ChanAssembleArgs aa{};
  aa.d3 = D3;
  aa.dq = C64(L.DQ);
  aa.R = R;
  aa.lsphi = C64(L.lapc);
  aa.phi = phi;
  aa.lom = C64(L.lapom);
  aa.lpsi = C64(L.lappsi);
  aa.kx = kx;
  aa.ky = ky;
  aa.hist = C64(L.hist);
  aa.g = C64(L.G);
  aa.mean = C64(L.mean);
  aa.d2mean = C64(L.d2mean);
  aa.hmean = C64(L.hmean);
  aa.gmean = C64(L.gmean);
  PSMS_TRY(psms::launch_ch_assemble(g, c->coef, aa, st));
  // the wall-normal solves of every (kx, ky) pair (psms_wall_solve's sequence with
  // the homogeneous w solutions and their influence matrix precomputed at
  // creation), and the mean flow; independent problems share a launch
  const cpx<double> z0 = {0.0, 0.0};
  double* xw = c->at<double>(L.xw);
  const long long xws = (long long)(nc + 1) * nl;
  psms::HelmBatch b1{};
  b1.np = g.sp ? 3 : 4;
  const int fs = c->p.free_slip & 3;   // omega_z and U, V: Neumann at a free-slip wall
  b1.p[0] = psms::HelmProblem{C64(L.G), om, xw, nl, c->coef.beta, kx, ky, fs, z0, z0};                     // omega_z
  b1.p[1] = psms::HelmProblem{C64(L.G) + g.NZL, C64(L.psip), xw + xws, nl, c->coef.beta, kx, ky, 0, z0, z0};  // psi_p
  b1.p[2] = psms::HelmProblem{C64(L.gmean), C64(L.mean), xw + 2 * xws, 2, c->coef.beta, nullptr, nullptr, fs, z0,
                              z0};                                                                        // U, V
  b1.p[3] = psms::HelmProblem{C64(L.G) + 2 * g.NZL, C64(L.xi), xw + 3 * xws, nl, c->a_fac, kx, ky, 3, z0, z0};  // xi
  const size_t fd = psms::helm_factor_doubles(nc, nl);
  const double* fac = L.has_fac ? c->at<double>(L.fac) : nullptr;
  if (fac) {
    b1.p[0].fac = fac + kChanFacOm * fd;
    b1.p[1].fac = fac + kChanFacPsi * fd;
    b1.p[2].fac = fac + kChanFacMean * fd;
    b1.p[3].fac = fac + kChanFacXi * fd;   // (not among the np problems in single phase)
  }
  PSMS_TRY(psms::launch_helm_batch(b1, nc, st));
  psms::HelmBatch b2{};
  b2.np = g.sp ? 1 : 2;
  b2.p[0] = psms::HelmProblem{C64(L.psip), w, xw, nl, 0.0, kx, ky, 0, z0, z0};             // w_p
  b2.p[1] = psms::HelmProblem{C64(L.xi), phi, xw + xws, nl, c->b_fac, kx, ky, 3, z0, z0};  // phi
  // between two no-slip walls the influence correction is applied by the w
  // chains themselves (the two wall conditions split by parity)
  const bool fused = (fs == 0) && psms::helm_fuses_influence(nc);
  if (fused) {
    b2.p[0].wh = c->at<double>(L.whp);
    b2.p[0].mh = c->at<double>(L.mhp);
  }
  if (fac) {
    b2.p[0].fac = fac + kChanFacW * fd;
    b2.p[1].fac = fac + kChanFacPhi * fd;   // (not among the np problems in single phase)
  }
  PSMS_TRY(psms::launch_helm_batch(b2, nc, st));
  if (!fused)
    PSMS_TRY(psms::launch_influence_apply(w, C64(L.wt), C64(L.wb), c->at<double>(L.M), nc, nl, kx, ky, fs, st));
#undef PSMS_TRY
  return hipSuccess;
}

}  // namespace

extern "C" {

int psms_channel_workspace_bytes(const psms_channel_params* p, size_t* bytes) {
  if (!bytes) return fail(PSMS_E_INVAL, "bytes is NULL");
  const int r = chan_validate(p);
  if (r) return r;
  *bytes = chan_layout(*p).total;
  return PSMS_OK;
}

int psms_channel_create(psms_channel** out, const psms_channel_params* p, void* d_workspace, size_t bytes,
                        void* stream) {
  if (!out) return fail(PSMS_E_INVAL, "out is NULL");
  *out = nullptr;
  int r = chan_validate(p);
  if (r) return r;
  const ChanLayout lay = chan_layout(*p);
  if (!d_workspace || !aligned(d_workspace)) return fail(PSMS_E_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (bytes < lay.total) return fail(PSMS_E_WORKSPACE, "workspace too small: need " + std::to_string(lay.total));
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(PSMS_E_DEVICE, "no HIP device available");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(PSMS_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  psms_channel* c = new psms_channel();
  c->p = *p;
  c->g = chan_geom(*p);
  c->lay = lay;
  c->ws = static_cast<char*>(d_workspace);
  c->stream = static_cast<hipStream_t>(stream);
  c->coef = psms::ChanCoef{};
  if (!p->single_phase) {
    const double s = (p->s > 0.0) ? p->s : std::sqrt(4.0 * p->pe / (p->ch * p->ch * p->dt));
    const double ab = p->pe / (p->dt * p->ch * p->ch);
    const double d = std::sqrt(std::max(s * s - 4.0 * ab, 0.0));
    c->a_fac = 0.5 * (s - d);
    c->b_fac = 0.5 * (s + d);
    c->coef.inv_pe = 1.0 / p->pe;
    c->coef.e_coef = (1.0 + s * p->ch * p->ch) / p->pe;
    c->coef.g_phi_scale = ab;
    c->coef.csig = 3.0 / std::sqrt(8.0) * p->ch / p->we;
  }
  c->coef.re = p->re;
  c->coef.beta = 2.0 * p->re / p->dt;
  c->coef.dt = p->dt;
  c->coef.forcing = p->forcing;
  c->coef.ab1 = 1;
  c->nstep = 0;
  c->have_state = 0;
  // line wavenumbers (kx = 2 pi m / lx, ky = 2 pi m / ly over the band) and twiddles
  const psms::ChanGeom& g = c->g;
  std::vector<double> hkx(g.NL), hky(g.NL);
  for (int iy = 0; iy < g.Cy; ++iy)
    for (int ix = 0; ix < g.Hx; ++ix) {
      const int my = (iy <= g.Ky) ? iy : iy - g.Cy;
      hkx[size_t(iy) * g.Hx + ix] = 2.0 * M_PI / p->lx * ix;
      hky[size_t(iy) * g.Hx + ix] = 2.0 * M_PI / p->ly * my;
    }
  auto tws = [](int n, std::vector<cpx<double>>& t64, std::vector<cpx<float>>& t32) {
    t64.resize(n);
    t32.resize(n);
    for (int m = 0; m < n; ++m) {
      const double a = -2.0 * M_PI * double(m) / double(n);
      t64[m] = cpx<double>{std::cos(a), std::sin(a)};
      t32[m] = cpx<float>{float(t64[m].re), float(t64[m].im)};
    }
  };
  std::vector<cpx<double>> x64, y64, z64;
  std::vector<cpx<float>> x32, y32, z32;
  tws(p->nx, x64, x32);
  tws(p->ny, y64, y32);
  tws(2 * p->nc, z64, z32);
  hipStream_t st = c->stream;
  // descriptor of the fused x stage: y-inverse output B in, the products'
  // x-spectra into C (8 fields of (nc + 1) ny rows of Hx entries fit there)
  psms::BoxDev xd{};
  xd.bufa = c->ws + lay.B;
  xd.bufb = c->ws + lay.C;
  xd.csig = c->coef.csig;
  c->h_xdev = xd;
  hipError_t e = hipMemcpyAsync(c->ws + lay.xdev, &c->h_xdev, sizeof(psms::BoxDev), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + lay.kx, hkx.data(), g.NL * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->ws + lay.ky, hky.data(), g.NL * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->ws + lay.twx64, x64.data(), x64.size() * sizeof(cpx<double>), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->ws + lay.twx32, x32.data(), x32.size() * sizeof(cpx<float>), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->ws + lay.twy64, y64.data(), y64.size() * sizeof(cpx<double>), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->ws + lay.twy32, y32.data(), y32.size() * sizeof(cpx<float>), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->ws + lay.twz64, z64.data(), z64.size() * sizeof(cpx<double>), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->ws + lay.twz32, z32.data(), z32.size() * sizeof(cpx<float>), hipMemcpyHostToDevice, st);
  // homogeneous solutions of the clamped w problem (unit psi at one wall) and
  // their influence matrix: fixed for the context (k^2 and beta are)
  if (e == hipSuccess) {
    const cpx<double> z0 = {0.0, 0.0}, one = {1.0, 0.0};
    const double* kx = c->at<double>(lay.kx);
    const double* ky = c->at<double>(lay.ky);
    cpx<double>* pt = c->at<cpx<double>>(lay.psip);
    cpx<double>* pb = c->at<cpx<double>>(lay.xi);
    double* xw = c->at<double>(lay.xw);
    const long long xws = (long long)(p->nc + 1) * g.NL;
    psms::HelmBatch b{};
    b.np = 2;
    b.p[0] = psms::HelmProblem{nullptr, pt, xw, g.NL, c->coef.beta, kx, ky, 0, one, z0};
    b.p[1] = psms::HelmProblem{nullptr, pb, xw + xws, g.NL, c->coef.beta, kx, ky, 0, z0, one};
    e = psms::launch_helm_batch(b, p->nc, st);
    if (e == hipSuccess) {
      b.p[0] = psms::HelmProblem{pt, c->at<cpx<double>>(lay.wt), xw, g.NL, 0.0, kx, ky, 0, z0, z0};
      b.p[1] = psms::HelmProblem{pb, c->at<cpx<double>>(lay.wb), xw + xws, g.NL, 0.0, kx, ky, 0, z0, z0};
      e = psms::launch_helm_batch(b, p->nc, st);
    }
    if (e == hipSuccess)
      e = psms::launch_influence_pre(c->at<cpx<double>>(lay.wt), c->at<cpx<double>>(lay.wb), p->nc, g.NL,
                                     c->at<double>(lay.M), p->free_slip & 3, st);
    if (e == hipSuccess)
      e = psms::launch_influence_parity_pre(c->at<cpx<double>>(lay.wt), c->at<cpx<double>>(lay.wb), p->nc, g.NL,
                                            c->at<double>(lay.whp), c->at<double>(lay.mhp), st);
    // elimination factors of the step's tau problems (their beta + k^2 and
    // wall conditions are fixed for the context)
    if (e == hipSuccess && lay.has_fac) {
      const int fs = p->free_slip & 3;
      const size_t fd = psms::helm_factor_doubles(p->nc, g.NL);
      double* fac = c->at<double>(lay.fac);
      auto prob = [&](double beta, bool lines, int bc) {
        psms::HelmProblem h{};
        h.nlines = lines ? g.NL : 2;
        h.beta_add = beta;
        h.kx = lines ? kx : nullptr;
        h.ky = lines ? ky : nullptr;
        h.bc = bc;
        return h;
      };
      const psms::HelmProblem probs[kChanFacCount] = {prob(c->coef.beta, true, fs), prob(c->coef.beta, true, 0),
                                                     prob(c->coef.beta, false, fs), prob(c->a_fac, true, 3),
                                                     prob(0.0, true, 0), prob(c->b_fac, true, 3)};
      for (int k = 0; k < kChanFacCount && e == hipSuccess; ++k) {
        if (g.sp && (k == kChanFacXi || k == kChanFacPhi)) continue;   // no phi equation
        e = psms::launch_helm_factors(probs[k], p->nc, fac + k * fd, st);
      }
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "channel_create");
  }
  *out = c;
  return PSMS_OK;
}

int psms_channel_init_state(psms_channel* c, const double* d_u, const double* d_v, const double* d_w,
                            const double* d_phi) {
  if (!c || !d_u || !d_v || !d_w || (!d_phi && !c->g.sp)) return fail(PSMS_E_INVAL, "NULL argument");
  const psms::ChanGeom& g = c->g;
  const ChanLayout& L = c->lay;
  // FP64 forward chain of the 4 fields (3 in single phase) through the step's
  // buffers: in MIXED the physical, y-expanded and band buffers hold 8 FP32
  // fields, i.e. 4 FP64 ones
  double* C = c->at<double>(L.C);
  cpx<double>* A = c->at<cpx<double>>(L.R);
  hipError_t e = hipSuccess;
  const double* src[4] = {d_u, d_v, d_w, d_phi};
  const int nf = g.sp ? 3 : 4;
  for (int f = 0; f < nf && e == hipSuccess; ++f)
    e = hipMemcpyAsync(C + f * g.P, src[f], size_t(g.P) * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = chan_forward<double>(c, C, A, nf);
  if (e == hipSuccess)
    e = psms::launch_ch_init(g, A, c->at<double>(L.kx), c->at<double>(L.ky), c->at<cpx<double>>(L.state),
                             c->at<cpx<double>>(L.state) + g.NZL, c->at<cpx<double>>(L.state) + 2 * g.NZL,
                             c->at<cpx<double>>(L.mean), c->stream);
  if (e == hipSuccess)
    e = hipMemsetAsync(c->ws + L.hist, 0, size_t(3 * g.NZL) * sizeof(cpx<double>), c->stream);
  if (e == hipSuccess)
    e = hipMemsetAsync(c->ws + L.hmean, 0, size_t(2 * (g.nc + 1)) * sizeof(cpx<double>), c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "channel_init_state");
  c->nstep = 0;
  c->have_state = 1;
  // a non-finite input value reaches every coefficient of its line through the
  // transforms: the diagnostics' count finds it
  psms_diag d;
  const int r = psms_channel_diagnostics(c, &d);
  if (r) return r;
  if (d.nonfinite) {
    c->have_state = 0;
    return fail(PSMS_E_NONFINITE, "non-finite value in the initial fields");
  }
  return PSMS_OK;
}

int psms_channel_diagnostics(psms_channel* c, psms_diag* h_out) {
  if (!c || !h_out) return fail(PSMS_E_INVAL, "NULL argument");
  if (!c->have_state) return fail(PSMS_E_STATE, "channel_diagnostics before init_state / set_state");
  const psms::ChanGeom& g = c->g;
  const ChanLayout& L = c->lay;
  hipStream_t st = c->stream;
  auto C64 = [&](size_t off) { return c->at<cpx<double>>(off); };
  cpx<double>* om = C64(L.state);
  cpx<double>* w = om + g.NZL;
  cpx<double>* phi = w + g.NZL;
  const double* kx = c->at<double>(L.kx);
  const double* ky = c->at<double>(L.ky);
  double* part = c->at<double>(L.diag);
  double* part2 = part + 4 * kChanDiagBlocks;
  double* out = part2 + 4 * kChanDiagBlocks;
  const int nb1 = int(std::min<long long>(kChanDiagBlocks, (g.NL + 3) / 4));
  const int nb2 = int(std::min<long long>(kChanDiagBlocks, (g.P + 255) / 256));
  // D w and D phi (the step's scratch: the next step recomputes them), the
  // per-line sums, then u, v, w in FP64 on the collocation grid for the CFL
  // number (through the step's transform buffers, which hold 4 FP64 fields in
  // MIXED)
  psms::ChebBatch cb{};
  cb.n = g.sp ? 1 : 2;
  cb.in[0] = w;
  cb.out[0] = C64(L.dw);
  cb.in[1] = phi;
  cb.out[1] = C64(L.dphi);
  hipError_t e = psms::launch_cheb_batch(cb, g.nc, g.NL, kx, ky, 0, st);
  if (e == hipSuccess)
    e = psms::launch_ch_diag_lines(g, om, w, phi, C64(L.dw), C64(L.dphi), C64(L.mean), kx, ky, part, nb1, st);
  if (e == hipSuccess)
    e = psms::launch_ch_fields<double>(g, om, w, phi, C64(L.dw), C64(L.dphi), C64(L.mean), kx, ky, C64(L.R), st);
  if (e == hipSuccess) e = chan_inverse<double>(c, C64(L.R), c->at<double>(L.C), 3);
  if (e == hipSuccess)
    e = psms::launch_ch_cfl(g, c->at<double>(L.C), g.nx / c->p.lx, g.ny / c->p.ly, c->p.dt, part2, nb2, st);
  if (e == hipSuccess) e = psms::launch_ch_diag_final(g, part, nb1, part2, nb2, phi, out, st);
  double h[6];
  if (e == hipSuccess) e = hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "channel_diagnostics");
  h_out->mean_phi = h[0];
  h_out->ke = h[1];
  h_out->grad2 = h[2];
  h_out->max_div = h[3];
  h_out->nonfinite = int32_t(h[4]);
  h_out->nstep = c->nstep;
  h_out->cfl = h[5];
  h_out->sphi0_re = 0.0;   // the channel zeroes no mode of S_phi
  h_out->sphi0_im = 0.0;
  return PSMS_OK;
}

int psms_channel_set_state(psms_channel* c, const double* d_state, const double* d_mean, const double* d_hist,
                           const double* d_hmean, int32_t nstep) {
  if (!c || !d_state || !d_mean) return fail(PSMS_E_INVAL, "NULL argument");
  if (nstep < 0) return fail(PSMS_E_INVAL, "nstep must be >= 0");
  if (nstep > 0 && (!d_hist || !d_hmean)) return fail(PSMS_E_INVAL, "nstep > 0 needs the history");
  const psms::ChanGeom& g = c->g;
  const ChanLayout& L = c->lay;
  const size_t sz = size_t(3 * g.NZL) * sizeof(cpx<double>);
  hipError_t e = hipMemcpyAsync(c->ws + L.state, d_state, sz, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = psms::launch_ch_mean_io(g, reinterpret_cast<const cpx<double>*>(d_mean), c->at<cpx<double>>(L.mean), +1,
                                c->stream);
  if (e == hipSuccess) {
    if (nstep > 0) {
      e = hipMemcpyAsync(c->ws + L.hist, d_hist, sz, hipMemcpyDeviceToDevice, c->stream);
      if (e == hipSuccess)
        e = psms::launch_ch_mean_io(g, reinterpret_cast<const cpx<double>*>(d_hmean), c->at<cpx<double>>(L.hmean),
                                    +1, c->stream);
    } else {
      e = hipMemsetAsync(c->ws + L.hist, 0, sz, c->stream);
      if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.hmean, 0, 2 * size_t(g.nc + 1) * sizeof(cpx<double>), c->stream);
    }
  }
  if (e == hipSuccess && g.sp) {   // phi and its history are identically zero
    e = hipMemsetAsync(c->ws + L.state + size_t(2 * g.NZL) * sizeof(cpx<double>), 0,
                       size_t(g.NZL) * sizeof(cpx<double>), c->stream);
    if (e == hipSuccess)
      e = hipMemsetAsync(c->ws + L.hist + size_t(2 * g.NZL) * sizeof(cpx<double>), 0,
                         size_t(g.NZL) * sizeof(cpx<double>), c->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "channel_set_state");
  c->nstep = nstep;
  c->have_state = 1;
  return PSMS_OK;
}

int psms_channel_step(psms_channel* c, int32_t nsteps) {
  if (!c) return fail(PSMS_E_INVAL, "NULL context");
  if (nsteps < 0) return fail(PSMS_E_INVAL, "nsteps must be >= 0");
  if (!c->have_state) return fail(PSMS_E_STATE, "step before init_state / set_state");
  const bool mixed = c->p.precision == PSMS_MIXED;
  for (int i = 0; i < nsteps; ++i) {
    // after the Adams-Bashforth 1 step every step is the same launch sequence
    // with the same arguments: capture it once and replay it
    const bool graph = c->use_graph && c->stream != nullptr && c->nstep > 0;
    hipError_t e = hipSuccess;
    if (graph) {
      if (!c->graph_ok) {
        e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          const hipError_t e2 = mixed ? chan_step_once<float>(c) : chan_step_once<double>(c);
          e = hipStreamEndCapture(c->stream, &c->graph);
          if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0);
        if (e == hipSuccess) c->graph_ok = 1;
      }
      if (e == hipSuccess) e = hipGraphLaunch(c->gexec, c->stream);
    } else {
      e = mixed ? chan_step_once<float>(c) : chan_step_once<double>(c);
    }
    if (e != hipSuccess) return hip_fail(e, "channel_step");
    ++c->nstep;
  }
  return PSMS_OK;
}

int psms_channel_set_graphs(psms_channel* c, int32_t enable) {
  if (!c) return fail(PSMS_E_INVAL, "NULL context");
  c->use_graph = enable ? 1 : 0;
  return PSMS_OK;
}

int psms_channel_get_state(psms_channel* c, double* d_state, double* d_mean, double* d_hist, double* d_hmean) {
  if (!c || !d_state || !d_mean) return fail(PSMS_E_INVAL, "NULL argument");
  if (!c->have_state) return fail(PSMS_E_STATE, "no state");
  const psms::ChanGeom& g = c->g;
  const ChanLayout& L = c->lay;
  const size_t sz = size_t(3 * g.NZL) * sizeof(cpx<double>);
  hipError_t e = hipMemcpyAsync(d_state, c->ws + L.state, sz, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = psms::launch_ch_mean_io(g, c->at<cpx<double>>(L.mean), reinterpret_cast<cpx<double>*>(d_mean), -1,
                                c->stream);
  if (e == hipSuccess && d_hist) e = hipMemcpyAsync(d_hist, c->ws + L.hist, sz, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && d_hmean)
    e = psms::launch_ch_mean_io(g, c->at<cpx<double>>(L.hmean), reinterpret_cast<cpx<double>*>(d_hmean), -1,
                                c->stream);
  if (e != hipSuccess) return hip_fail(e, "channel_get_state");
  return PSMS_OK;
}

int psms_channel_destroy(psms_channel* c) {
  if (c && c->graph_ok) {
    hipGraphExecDestroy(c->gexec);
    hipGraphDestroy(c->graph);
  }
  delete c;
  return PSMS_OK;
}

}  // extern "C"
