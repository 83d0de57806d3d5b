// Host runtime of the fuzzy-web likelihood library: plans, workspace, spectral
// tables, the stage schedule of the forward model and of its adjoint, the
// leapfrog trajectory (captured as a HIP graph) and the C ABI of fzw.h.
#include <hip/hip_runtime.h>
#include <cstdlib>
#include <mutex>
#include <functional>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fzw.h"
#include "fzw_internal.hpp"
#include "fzw_ops.hpp"

namespace fzw {

static thread_local std::string g_last_error;

struct Error : std::runtime_error {
  fzw_status code;
  Error(fzw_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(expr)                                                                             \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) {                                                                      \
      (void)hipGetLastError();                                                                   \
      throw Error(e_ == hipErrorOutOfMemory ? FZW_E_OOM : FZW_E_HIP,                            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                           \
    }                                                                                            \
  } while (0)

// radial tables
// radial tables; the last four are products of two others, formed in FP64 so
// that a multiplier needs one gather instead of two
enum {
  TAB_H = 0, TAB_INVK2 = 1, TAB_K = 2, TAB_1MK = 3, TAB_WEB0 = 4, TAB_WEB1 = 5,
  TAB_K_INVK2 = 6, TAB_1MK_INVK2 = 7, TAB_H_INVK2 = 8, TAB_H_K = 9, NTAB = 10
};
static_assert(NTAB == kRadialTables, "one closed form per table");
// stage scratch spectra
constexpr int kNSpec = 13;

// ------------------------------------------------------------ power spectrum
// Linear matter power spectrum with the BBKS transfer function (Bardeen, Bond,
// Kaiser & Szalay 1986), shape Gamma = Omega_m h, tilt n_s, normalised to
// sigma8 with a top-hat of 8 Mpc/h (composite Simpson in ln k, 1e-5..1e2 h/Mpc).
static double bbks(double k, double om, double h) {
  if (k <= 0) return 1.0;
  const double q = k / (om * h);
  const double a = std::log1p(2.34 * q) / (2.34 * q);
  const double b = 1.0 + 3.89 * q + std::pow(16.1 * q, 2) + std::pow(5.46 * q, 3) + std::pow(6.71 * q, 4);
  return a * std::pow(b, -0.25);
}
static double tophat(double x) {
  if (std::fabs(x) < 1e-4) return 1.0 - x * x / 10.0;
  return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}
static double power_amplitude(const fzw_cosmo& c) {
  const int n = 400000;  // even number of intervals
  const double a = std::log(1e-5), b = std::log(1e2), dh = (b - a) / n;
  double s = 0.0;
  for (int i = 0; i <= n; ++i) {
    const double lk = a + i * dh, k = std::exp(lk);
    const double t = bbks(k, c.omega_m, c.h);
    const double f = k * k * k * std::pow(k, c.n_s) * t * t * std::pow(tophat(8.0 * k), 2);
    const double w = (i == 0 || i == n) ? 1.0 : (i % 2 ? 4.0 : 2.0);
    s += w * f;
  }
  s *= dh / 3.0 / (2.0 * M_PI * M_PI);
  return c.sigma8 * c.sigma8 / s;
}

struct Group {
  int n = 0;
  double box = 0;
  int c0 = 0, nc = 0;
  long long nv = 0;          // n^3
  int P = 0;                 // spectrum row pitch
  long long ns = 0;          // spectrum elements per chain
  int nblk = 0;              // blocks of the per-voxel kernels
  double* partial = nullptr; // FP64 block partials of this group's reductions
  hipStream_t gstream = nullptr;   // this group's stream when groups run side by side
  hipEvent_t gdone = nullptr;
  float* tabs = nullptr;
  int tab_stride = 0;
  RadialForms rf{};          // closed forms of the tables (all but h(k))
  RadialForms* rf_dev = nullptr;   // device copy read by the passes
  float2* tw_full = nullptr;
  float2* tw_half = nullptr;
  // real fields [nc][nv]
  float* phi[6] = {};
  float* s2 = nullptr;
  float* dsc = nullptr;
  float* psi[3] = {};
  float* rho = nullptr;
  float* tens[12] = {};
  float* logf = nullptr;
  float* beta = nullptr;
  float* ghat = nullptr;     // backward inputs formed by the likelihood pass
  float* nbv = nullptr;
  float* dbeta = nullptr;
  float* drho_dir = nullptr;
  float* drho = nullptr;
  float2* spec[kNSpec] = {};
  int* count = nullptr;
  int* offset = nullptr;
  int* bsum = nullptr;
  float4* sorted = nullptr;
  unsigned long long* acc = nullptr;
};

}  // namespace fzw

using namespace fzw;

struct fzw_plan {
  int n_chains = 0;
  int device = 0;                     // the device current at fzw_plan_create
  // FZW_PLAN_CHECKPOINT: phi_ij is not kept between the forward model and the
  // adjoint, which recomputes it from nu (no phi buffers in the workspace)
  bool checkpoint = false;
  int W = 1, R = 4;
  fzw_cosmo cosmo{};
  fzw_web web{};
  hipStream_t stream = nullptr;       // work is enqueued here
  hipStream_t user_stream = nullptr;  // the caller's stream
  hipStream_t cap_stream = nullptr;   // private stream for graph capture and replay
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipEvent_t ev_fork = nullptr;       // groups of different meshes fork from here
  double amp = 0;
  std::vector<Group> groups;
  std::vector<long long> chain_off;   // voxel offset per chain
  std::vector<int> chain_group;
  std::vector<bool> counts_set;
  long long total_vox = 0;
  uint16_t* counts = nullptr;
  double* scal = nullptr;             // [n_chains][kScalStride]
  int* flags = nullptr;               // [n_chains] non-finite flags (FZW_NF_*) of the last evaluation call
  // fields fzw_get_field may return (bit = field id): what the last
  // evaluation left in the buffers
  unsigned long long field_valid = 0;
  double* partial = nullptr;
  size_t partial_elems = 0;
  float* dnu_tmp = nullptr;           // leapfrog gradient
  float* table_tmp = nullptr;         // leapfrog bias tables
  float* dtable_tmp = nullptr;
  double* epartial = nullptr;         // leapfrog energy partials [n_chains][kEBlk]
  int* tie = nullptr;
  float* fsign = nullptr;             // sign of every free parameter (+1 unless set)
  double* mu = nullptr;
  double* sigma = nullptr;
  int nfree = -1;
  int cic_method = FZW_CIC_SORTED;
  std::vector<void*> allocs;
  size_t ws_bytes = 0;
  struct GraphEntry {
    hipGraph_t g;
    hipGraphExec_t e;
  };
  std::map<std::vector<uintptr_t>, GraphEntry> graphs;
  // per-kernel-class timing with HIP events (off unless enabled)
  bool timing = false;
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  struct TimingRec {
    int klass;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<TimingRec> recs;
  // no-U-turn state, allocated at the first transition and grown with the
  // tree depth or the number of free parameters
  float* nuts_vec = nullptr;          // (13 + 2 max_depth) state vectors of nuts_tv floats
  long long nuts_tv = 0;
  int nuts_md = 0;
  NutsChain* nuts_st = nullptr;
  double* nuts_partial = nullptr;
  int* nuts_any = nullptr;
  int* nuts_any_host = nullptr;       // pinned
  double* stats_buf = nullptr;        // partials and scalars of the validation statistics
  int integrator = FZW_INT_LEAPFROG;  // splitting scheme of fzw_leapfrog
  // likelihood pass in float64 per voxel instead of the float32 pass (float64
  // for the terms of lnP shared by many voxels)
  // (FZW_LIKELIHOOD_FP64=1; both sum in float64)
  bool like_fp64 = false;
};

namespace {

constexpr int kEBlk = 256;

template <class T>
T* dalloc(fzw_plan* p, size_t count) {
  void* ptr = nullptr;
  const size_t bytes = count * sizeof(T);
  hipError_t e = hipMalloc(&ptr, bytes > 0 ? bytes : 16);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(FZW_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  p->allocs.push_back(ptr);
  p->ws_bytes += bytes;
  return static_cast<T*>(ptr);
}

// Records HIP events around a launch of kernel class `klass` on the plan's
// stream when timing is enabled; `bytes` is the launch's algorithmic traffic.
struct Timed {
  fzw_plan* p;
  int idx = -1;
  hipStream_t st = nullptr;
  Timed(fzw_plan* pl, int klass, double bytes) : p(pl) {
    if (!p || !p->timing) return;
    st = p->stream;
    while (p->evpool.size() < p->evused + 2) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      p->evpool.push_back(e);
    }
    fzw_plan::TimingRec r{klass, bytes, p->evpool[p->evused], p->evpool[p->evused + 1]};
    p->evused += 2;
    HIPCHK(hipEventRecord(r.a, st));
    p->recs.push_back(r);
    idx = (int)p->recs.size() - 1;
  }
  ~Timed() {
    if (idx >= 0) (void)hipEventRecord(p->recs[idx].b, st);
  }
};

double spec_bytes(const Group& g) { return (double)g.nc * g.n * g.n * (g.n / 2 + 1) * 8.0; }
double field_bytes(const Group& g) { return (double)g.nc * g.nv * 4.0; }

// Displacement-to-cell scaling and redshift-space geometry of the CIC stage
// (Section 2.9, b_v = 1): plane-parallel RSD scales the line-of-sight axis by
// 1 + f; radial RSD shifts along the ray from the box centre in the kernels.
void set_rsd(CicArgs& ca, const fzw_cosmo& c, const Group& g) {
  for (int d = 0; d < 3; ++d) {
    const double f = (c.rsd_axis == d) ? (1.0 + c.f_growth) : 1.0;
    ca.scale[d] = (float)(f * g.n / g.box);
  }
  ca.radial = c.rsd_axis == FZW_RSD_RADIAL ? 1 : 0;
  ca.f_los = (float)c.f_growth;
}

bool supported_n(int n) {
  return n == 16 || n == 32 || n == 64 || n == 96 || n == 128 || n == 256 || n == 512;
}

void build_tables(fzw_plan* p, Group& g) {
  const int n = g.n;
  const int half = n / 2;
  const int n2max = 3 * half * half;
  g.tab_stride = n2max + 1;
  std::vector<float> tab((size_t)NTAB * g.tab_stride, 0.f);
  const double kf = 2.0 * M_PI / g.box;
  const double dx = g.box / n;
  for (int q = 0; q <= n2max; ++q) {
    const double k2 = kf * kf * q;
    const double k = std::sqrt(k2);
    double h = 0, ik2 = 0;
    if (q > 0) {
      const double t = bbks(k, p->cosmo.omega_m, p->cosmo.h);
      const double pk = p->amp * std::pow(k, p->cosmo.n_s) * t * t;
      h = std::sqrt(pk / (dx * dx * dx));
      ik2 = 1.0 / k2;
    }
    const double kern = std::exp(-0.5 * k2 * p->cosmo.r_s * p->cosmo.r_s);
    tab[(size_t)TAB_H * g.tab_stride + q] = (float)h;
    tab[(size_t)TAB_INVK2 * g.tab_stride + q] = (float)ik2;
    tab[(size_t)TAB_K * g.tab_stride + q] = (float)kern;
    tab[(size_t)TAB_1MK * g.tab_stride + q] = (float)(1.0 - kern);
    tab[(size_t)TAB_K_INVK2 * g.tab_stride + q] = (float)(kern * ik2);
    tab[(size_t)TAB_1MK_INVK2 * g.tab_stride + q] = (float)((1.0 - kern) * ik2);
    tab[(size_t)TAB_H_INVK2 * g.tab_stride + q] = (float)(h * ik2);
    tab[(size_t)TAB_H_K * g.tab_stride + q] = (float)(h * kern);
    for (int w = 0; w < p->W; ++w) {
      const double r = p->web.smooth_r[w];
      const double wg = std::exp(-0.5 * k2 * r * r);
      double m;
      if (p->web.kind[w] == FZW_WEB_PHI) m = wg * ik2;
      else m = p->web.ell[w] * p->web.ell[w] * wg;
      tab[(size_t)(TAB_WEB0 + w) * g.tab_stride + q] = (float)m;
    }
  }
  // closed forms of every table but h(k) (BBKS), evaluated in FP32 in the
  // passes; FZW_RADIAL_FORMS=0 keeps every table a lookup
  const char* env = std::getenv("FZW_RADIAL_FORMS");
  const bool forms = !(env && env[0] == '0');
  g.rf = RadialForms{};
  g.rf.inv_kf2 = (float)(1.0 / (kf * kf));
  if (forms) {
    // coefficients of exp(-k^2 r^2 / 2) written as 2^(-c q), q = |n|^2
    const double cs = 0.5 * kf * kf * p->cosmo.r_s * p->cosmo.r_s / std::log(2.0);
    g.rf.kind[TAB_INVK2] = 1;
    g.rf.kind[TAB_K] = 2;
    g.rf.c[TAB_K] = (float)cs;
    g.rf.kind[TAB_1MK] = 3;
    g.rf.c[TAB_1MK] = (float)cs;
    g.rf.kind[TAB_K_INVK2] = 4;
    g.rf.c[TAB_K_INVK2] = (float)cs;
    for (int w = 0; w < p->W; ++w) {
      const double r = p->web.smooth_r[w];
      g.rf.c[TAB_WEB0 + w] = (float)(0.5 * kf * kf * r * r / std::log(2.0));
      if (p->web.kind[w] == FZW_WEB_PHI) {
        g.rf.kind[TAB_WEB0 + w] = 4;
      } else {
        g.rf.kind[TAB_WEB0 + w] = 5;
        g.rf.l[TAB_WEB0 + w] = (float)(p->web.ell[w] * p->web.ell[w]);
      }
    }
  }
  g.rf_dev = dalloc<RadialForms>(p, 1);
  HIPCHK(hipMemcpy(g.rf_dev, &g.rf, sizeof(RadialForms), hipMemcpyHostToDevice));
  g.tabs = dalloc<float>(p, tab.size());
  HIPCHK(hipMemcpy(g.tabs, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice));
  std::vector<float2> tf(n), th(half);
  for (int k = 0; k < n; ++k) {
    const double a = -2.0 * M_PI * k / n;
    tf[k] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  for (int k = 0; k < half; ++k) {
    const double a = -2.0 * M_PI * k / half;
    th[k] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  g.tw_full = dalloc<float2>(p, n);
  g.tw_half = dalloc<float2>(p, half);
  HIPCHK(hipMemcpy(g.tw_full, tf.data(), n * sizeof(float2), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(g.tw_half, th.data(), half * sizeof(float2), hipMemcpyHostToDevice));
}

void alloc_group(fzw_plan* p, Group& g) {
  const size_t nf = (size_t)g.nc * g.nv;
  const size_t nsp = (size_t)g.nc * g.ns;
  if (!p->checkpoint)
    for (auto& f : g.phi) f = dalloc<float>(p, nf);
  // S2 and d_SC exist in real space only where the LPT step is not fused
  // with its z transforms
  if (!p->checkpoint || !has_four_step_z(g.n)) {
    g.s2 = dalloc<float>(p, nf);
    g.dsc = dalloc<float>(p, nf);
  }
  for (auto& f : g.psi) f = dalloc<float>(p, nf);
  g.rho = dalloc<float>(p, nf);
  for (int k = 0; k < 6 * p->W; ++k) g.tens[k] = dalloc<float>(p, nf);
  g.logf = dalloc<float>(p, nf);
  g.beta = dalloc<float>(p, nf);
  g.ghat = dalloc<float>(p, nf);
  g.nbv = dalloc<float>(p, nf);
  g.dbeta = dalloc<float>(p, nf);
  g.drho_dir = dalloc<float>(p, nf);
  g.drho = dalloc<float>(p, nf);
  for (auto& s : g.spec) s = dalloc<float2>(p, nsp);
  const size_t ncol = (size_t)g.n * g.n;
  g.count = dalloc<int>(p, (size_t)g.nc * ncol);
  g.offset = dalloc<int>(p, (size_t)g.nc * (ncol + 1));
  g.bsum = dalloc<int>(p, (size_t)g.nc * ((ncol + 4095) / 4096));
  g.sorted = dalloc<float4>(p, nf);
  g.acc = dalloc<unsigned long long>(p, nf);
  HIPCHK(hipMemset(g.acc, 0, nf * sizeof(unsigned long long)));
}

// ------------------------------------------------------------- pass helpers
struct Pass {
  PassArgs a{};
  Pass() {
    for (auto& r : a.A)
      for (auto& o : r) o = spec_zero();
    for (auto& r : a.B)
      for (auto& o : r) o = spec_zero();
  }
  Pass& in(const float2* p, bool fft) {
    a.in_fft |= fft ? (1u << a.nin) : 0u;
    a.in[a.nin++] = p;
    return *this;
  }
  Pass& out(float2* p, bool fft) {
    a.out_fft |= fft ? (1u << a.nout) : 0u;
    a.out[a.nout++] = p;
    return *this;
  }
};

thread_local fzw_plan* t_plan = nullptr;   // plan whose stages are being enqueued

void run_pass(const Group& g, int axis, Pass& ps, int nmid, hipStream_t s) {
  // single- and multi-input passes run different kernels: separate classes
  const int klass = ps.a.nin > 1 ? (axis == 0 ? FZW_K_XMIX_MULTI : FZW_K_YMIX_MULTI) : (axis == 0 ? FZW_K_XMIX : FZW_K_YMIX);
  Timed tm(t_plan, klass, (ps.a.nin + ps.a.nout) * spec_bytes(g));
  ps.a.nmid = nmid;
  ps.a.chain_stride = g.ns;
  ps.a.tabs = g.tabs;
  ps.a.tab_stride = g.tab_stride;
  ps.a.kf = (float)(2.0 * M_PI / g.box);
  ps.a.rf = g.rf_dev;
  launch_xy_pass(g.n, axis, ps.a, g.nc, g.tw_full, s);
}

// Pure forward or inverse transforms along an axis: out[i] = F(in[i]) (in
// place when out[i] == in[i]; no other aliasing).  One persistent launch for
// all arrays where the mesh has the four-step kernels, else one mixing pass
// per array.
void pure_xy(const Group& g, int axis, bool inverse, float2* const* in, float2* const* out, int k, hipStream_t s) {
  if (k <= 8) {
    PureArgs pa{};
    for (int i = 0; i < k; ++i) {
      pa.in[i] = in[i];
      pa.out[i] = out[i];
    }
    pa.narr = k;
    pa.chains = g.nc;
    pa.chain_stride = g.ns;
    if (has_pure_pass(g.n)) {
      Timed tm(t_plan, axis == 0 ? FZW_K_XPURE : FZW_K_YPURE, 2.0 * k * spec_bytes(g));
      if (launch_pure_pass(g.n, axis, inverse, pa, g.tw_full, s)) return;
    }
  }
  for (int i = 0; i < k; ++i) {
    Pass ps;
    ps.in(in[i], !inverse).out(out[i], inverse);
    ps.a.A[0][0] = spec_const(1.f);
    ps.a.B[0][0] = spec_const(1.f);
    run_pass(g, axis, ps, 1, s);
  }
}

// pure forward or inverse transform of k arrays along an axis, in place
void pure_pass(const Group& g, int axis, bool inverse, float2* const* arr, int k, hipStream_t s) {
  pure_xy(g, axis, inverse, arr, arr, k, s);
}

// Inverse y pass from the three x-pass outputs (factors k_x^2, k_x, 1 of a
// Hessian k_i k_j m(k)) to the six tensor components xx, yy, zz, xy, xz, yz.
void hessian_yi(const Group& g, float2* a2, float2* a1, float2* a0, float2* const* out6, hipStream_t s) {
  {
    float2* i2[1] = {a2};
    float2* o2[1] = {out6[0]};
    pure_xy(g, 1, true, i2, o2, 1, s);
  }
  {
    Pass p1;
    p1.in(a1, false).out(out6[3], true).out(out6[4], true);
    p1.a.A[0][0] = spec_const(1.f);
    p1.a.B[0][0] = spec(1.f, 0.f, 1, -1, -1, -1);   // k_y  -> xy
    p1.a.B[1][0] = spec(1.f, 0.f, 2, -1, -1, -1);   // k_z  -> xz
    run_pass(g, 1, p1, 1, s);
  }
  {
    Pass p0;
    p0.in(a0, false).out(out6[1], true).out(out6[2], true).out(out6[5], true);
    p0.a.A[0][0] = spec_const(1.f);
    p0.a.B[0][0] = spec(1.f, 0.f, 1, 1, -1, -1);    // k_y^2 -> yy
    p0.a.B[1][0] = spec(1.f, 0.f, 2, 2, -1, -1);    // k_z^2 -> zz
    p0.a.B[2][0] = spec(1.f, 0.f, 1, 2, -1, -1);    // k_y k_z -> yz
    run_pass(g, 1, p0, 1, s);
  }
}

// Adjoint of hessian_yi: forward y pass of the six cotangent components
// (xx, yy, zz, xy, xz, yz) grouped by their x factor into three arrays.
void hessian_yf(const Group& g, float2* const* in6, float2* g2, float2* g1, float2* g0, hipStream_t s) {
  // Order matters when the outputs reuse the input arrays (g2, g1, g0 may be
  // in6[0], in6[1], in6[2]): each launch only overwrites arrays already read.
  {
    Pass p0;
    p0.in(in6[1], true).in(in6[2], true).in(in6[5], true).out(g0, false);
    p0.a.A[0][0] = spec(1.f, 0.f, 1, 1, -1, -1);
    p0.a.A[0][1] = spec(1.f, 0.f, 2, 2, -1, -1);
    p0.a.A[0][2] = spec(1.f, 0.f, 1, 2, -1, -1);
    p0.a.B[0][0] = spec_const(1.f);
    run_pass(g, 1, p0, 1, s);
  }
  {
    Pass p1;
    p1.in(in6[3], true).in(in6[4], true).out(g1, false);
    p1.a.A[0][0] = spec(1.f, 0.f, 1, -1, -1, -1);
    p1.a.A[0][1] = spec(1.f, 0.f, 2, -1, -1, -1);
    p1.a.B[0][0] = spec_const(1.f);
    run_pass(g, 1, p1, 1, s);
  }
  {
    float2* i2[1] = {in6[0]};
    float2* o2[1] = {g2};
    pure_xy(g, 1, false, i2, o2, 1, s);
  }
}

// The z transforms around the LPT pointwise step, fused with it.  Forward:
// six phi_ij spectra `in` -> phi (stored) -> S2, d_SC spectra `out`[0..1].
// Adjoint: dS2, dd_SC spectra `in`[0..1] and phi -> six d phi_ij spectra
// `out`.  Returns false where the mesh has no fused kernel.
// `field` are the phi_ij buffers (null in the forward model of a checkpointed
// plan: phi is not stored); `out` null in the forward: phi only (the adjoint's
// recompute of a checkpointed plan).
bool lpt_z(fzw_plan* p, const Group& g, bool fwd, float2* const* in, float2* const* out, float* const* field,
           hipStream_t s) {
  LptZArgs a{};
  const int nin = fwd ? 6 : 2, nout = fwd ? (out ? 2 : 0) : 6;
  for (int c = 0; c < nin; ++c) a.sin[c] = in[c];
  for (int c = 0; c < 6; ++c) a.field[c] = field ? field[c] : nullptr;
  for (int c = 0; c < nout; ++c) a.sout[c] = out[c];
  a.spec_chain_stride = g.ns;
  a.field_chain_stride = g.nv;
  a.d1 = (float)p->cosmo.d1;
  a.tau = (float)p->cosmo.tau_sc;
  if (!has_four_step_z(g.n)) return false;
  Timed tm(p, fwd ? FZW_K_LPT_FWD : FZW_K_LPT_BWD, (nin + nout) * spec_bytes(g) + (field ? 6 : 0) * field_bytes(g));
  return launch_lpt_z(g.n, fwd, a, g.nc, g.tw_half, g.tw_full, s);
}

void zf(const Group& g, float* const* in, float2* const* out, int k, hipStream_t s) {
  Timed tm(t_plan, FZW_K_ZR2C, k * (field_bytes(g) + spec_bytes(g)));
  launch_zpass_r2c(g.n, (const float* const*)in, out, k, g.nc, g.nv, g.ns, g.tw_half, g.tw_full, s);
}
void zi(const Group& g, float2* const* in, float* const* out, int k, hipStream_t s) {
  Timed tm(t_plan, FZW_K_ZC2R, k * (field_bytes(g) + spec_bytes(g)));
  launch_zpass_c2r(g.n, (const float2* const*)in, out, k, g.nc, g.ns, g.nv, g.tw_half, g.tw_full, s);
}

// axis ids for SpecOp
constexpr int X = 0, Y = 1, Z = 2, NONE = -1;

// ------------------------------------------------------------- forward model
// Appendix A and Section 2.3: the delta_L spectrum h(k) rfftn(nu) (into
// sp[1], kept in k space) and the spectra of the six first-order Hessian
// components phi_ij = k_i k_j / k^2 delta_L (into sp[5..10]), through one x
// pass.  The forward model starts with it; a checkpointed plan's adjoint runs
// it again to recompute phi, with the same kernels on the same input.
void lpt_hessian_spectra(const Group& g, const float* nu, hipStream_t s) {
  const float invn3 = (float)(1.0 / ((double)g.nv));
  float2* const* sp = g.spec;
  {
    float* src[1] = {const_cast<float*>(nu)};
    zf(g, src, &sp[0], 1, s);
    pure_pass(g, Y, false, &sp[0], 1, s);
  }
  Pass ps;
  ps.in(sp[0], true).out(sp[1], false).out(sp[2], true).out(sp[3], true).out(sp[4], true);
  ps.a.A[0][0] = spec(1.f, 0.f, NONE, NONE, TAB_H, NONE);
  ps.a.B[0][0] = spec_const(1.f);
  ps.a.B[1][0] = spec(invn3, 0.f, X, X, TAB_INVK2, NONE);
  ps.a.B[2][0] = spec(invn3, 0.f, X, NONE, TAB_INVK2, NONE);
  ps.a.B[3][0] = spec(invn3, 0.f, NONE, NONE, TAB_INVK2, NONE);
  run_pass(g, X, ps, 1, s);
  hessian_yi(g, sp[2], sp[3], sp[4], &sp[5], s);
}

// The phi_ij buffers of a plan: its own, or for a checkpointed plan the first
// six web-tensor buffers, which are free while phi is needed (before the
// tensors are formed in the forward model, after their cotangents have been
// transformed in the adjoint).
float* const* phi_buffers(const fzw_plan* p, const Group& g) { return p->checkpoint ? g.tens : g.phi; }

void forward_group(fzw_plan* p, Group& g, const float* nu, const float* bias, float* nbar, double* logl,
                   bool grad) {
  hipStream_t s = p->stream;
  const float invn3 = (float)(1.0 / ((double)g.nv));
  const float d1 = (float)p->cosmo.d1;
  float2** sp = g.spec;
  lpt_hessian_spectra(g, nu, s);
  // phi_ij to real space (stored for the adjoint unless checkpointed), 2LPT
  // source and spherical-collapse divergence, and their spectra (one fused
  // launch where the mesh has the four-step z pass)
  if (!lpt_z(p, g, true, &sp[5], &sp[2], p->checkpoint ? nullptr : g.phi, s)) {
    float* const* phi = phi_buffers(p, g);
    zi(g, &sp[5], phi, 6, s);
    LptArgs la{};
    for (int c = 0; c < 6; ++c) la.phi[c] = phi[c];
    la.s2 = g.s2;
    la.dsc = g.dsc;
    la.d1 = d1;
    la.tau = (float)p->cosmo.tau_sc;
    la.n = (long long)g.nc * g.nv;
    {
      Timed tm(p, FZW_K_LPT_FWD, 8 * field_bytes(g));
      launch_lpt_fwd(la, s);
    }
    float* src[2] = {g.s2, g.dsc};
    zf(g, src, &sp[2], 2, s);
  }
  // ALPT blend -> Psi (Section 2.3)
  {
    pure_pass(g, Y, false, &sp[2], 2, s);
    Pass ps;
    ps.in(sp[2], true).in(sp[3], true).in(sp[1], false);
    ps.a.A[0][0] = spec((float)(3.0 / 7.0) * d1 * d1 * invn3, 0.f, NONE, NONE, TAB_K_INVK2, NONE);
    ps.a.A[0][1] = spec(-invn3, 0.f, NONE, NONE, TAB_1MK_INVK2, NONE);
    ps.a.A[0][2] = spec(d1 * invn3, 0.f, NONE, NONE, TAB_K_INVK2, NONE);
    ps.out(sp[4], true).out(sp[5], true);
    ps.a.B[0][0] = spec(0.f, 1.f, X, NONE, NONE, NONE);  // i k_x
    ps.a.B[1][0] = spec_const(1.f);
    run_pass(g, X, ps, 1, s);
    {
      Pass px;
      px.in(sp[4], false).out(sp[6], true);
      px.a.A[0][0] = spec_const(1.f);
      px.a.B[0][0] = spec_const(1.f);
      run_pass(g, Y, px, 1, s);
      Pass pyz;
      pyz.in(sp[5], false).out(sp[7], true).out(sp[8], true);
      pyz.a.A[0][0] = spec_const(1.f);
      pyz.a.B[0][0] = spec(0.f, 1.f, Y, NONE, NONE, NONE);
      pyz.a.B[1][0] = spec(0.f, 1.f, Z, NONE, NONE, NONE);
      run_pass(g, Y, pyz, 1, s);
    }
    zi(g, &sp[6], g.psi, 3, s);
  }
  // CIC deposit (with plane-parallel or radial RSD, Section 2.9)
  {
    CicArgs ca{};
    set_rsd(ca, p->cosmo, g);
    for (int d = 0; d < 3; ++d) ca.psi[d] = g.psi[d];
    ca.n = g.n;
    ca.nv = g.nv;
    ca.count = g.count;
    ca.offset = g.offset;
    ca.bsum = g.bsum;
    ca.sorted = g.sorted;
    ca.rho = g.rho;
    ca.acc = g.acc;
    ca.flags = p->flags + g.c0;
    Timed tm(p, FZW_K_CIC_DEP, 4 * field_bytes(g));
    if (p->cic_method == FZW_CIC_ATOMIC) launch_cic_deposit_atomic(ca, g.nc, s);
    else launch_cic_deposit(ca, g.nc, s);
  }
  // Web tensors (Section 2.8): T^w_ij = k_i k_j m_w(k) rho_k
  {
    float* src[1] = {g.rho};
    zf(g, src, &sp[0], 1, s);
    pure_pass(g, Y, false, &sp[0], 1, s);
    Pass ps;
    ps.in(sp[0], true);
    ps.a.A[0][0] = spec_const(1.f);
    for (int w = 0; w < p->W; ++w) {
      ps.out(sp[1 + 3 * w], true).out(sp[2 + 3 * w], true).out(sp[3 + 3 * w], true);
      ps.a.B[3 * w + 0][0] = spec(invn3, 0.f, X, X, TAB_WEB0 + w, NONE);
      ps.a.B[3 * w + 1][0] = spec(invn3, 0.f, X, NONE, TAB_WEB0 + w, NONE);
      ps.a.B[3 * w + 2][0] = spec(invn3, 0.f, NONE, NONE, TAB_WEB0 + w, NONE);
    }
    run_pass(g, X, ps, 1, s);
    for (int w = 0; w < p->W; ++w) {
      hessian_yi(g, sp[1 + 3 * w], sp[2 + 3 * w], sp[3 + 3 * w], &sp[7], s);
      zi(g, &sp[7], &g.tens[6 * w], 6, s);
    }
  }
  // Fused per-voxel web / bias forward, then normalisation and likelihood
  {
    VoxelArgs va{};
    for (int k = 0; k < 6 * p->W; ++k) va.tens[k] = g.tens[k];
    va.rho = g.rho;
    va.table = bias + (size_t)g.c0 * p->R * 4;
    va.logf = g.logf;
    va.beta = g.beta;
    va.partial = g.partial;
    va.x_floor = (float)p->cosmo.x_floor;
    va.steep = (float)p->web.steepness;
    va.lam_th = (float)p->web.lambda_th;
    va.nv = g.nv;
    {
      Timed tm(p, FZW_K_VOXEL_FWD, (3 + 6 * p->W) * field_bytes(g));
      launch_voxel_fwd(p->W, va, g.nc, g.nblk, s);
    }
    FinalArgs fa{};
    fa.mode = 0;
    fa.partial = g.partial;
    fa.nblk = g.nblk;
    fa.scal = p->scal + (size_t)g.c0 * kScalStride;
    fa.flags = p->flags + g.c0;
    launch_finalize(fa, g.nc, s);
    LikeArgs la{};
    la.logf = g.logf;
    la.beta = g.beta;
    la.counts = p->counts + p->chain_off[g.c0];
    la.scal = p->scal + (size_t)g.c0 * kScalStride;
    la.partial = g.partial;
    la.nbar = nbar ? nbar + p->chain_off[g.c0] : nullptr;
    if (grad) {
      la.ghat = g.ghat;
      la.nbv = g.nbv;
      la.dbeta = g.dbeta;
    }
    la.nv = g.nv;
    {
      Timed tm(p, FZW_K_LIKE, (2.5 + (nbar ? 1 : 0)) * field_bytes(g));
      launch_likelihood(la, g.nc, g.nblk, p->like_fp64, s);
    }
    fa.mode = 1;
    fa.logl = logl ? logl + g.c0 : nullptr;
    launch_finalize(fa, g.nc, s);
  }
}

// ------------------------------------------------------------------ adjoint
void adjoint_group(fzw_plan* p, Group& g, const float* nu, const float* bias, float* dnu, float* dbias) {
  hipStream_t s = p->stream;
  const float invn3 = (float)(1.0 / ((double)g.nv));
  const float d1 = (float)p->cosmo.d1;
  const int W = p->W;
  float2** sp = g.spec;
  // per-voxel backward: d rho (direct), d T (in place over T), table gradient
  {
    VoxelArgs va{};
    for (int k = 0; k < 6 * W; ++k) {
      va.tens[k] = g.tens[k];
      va.dtens[k] = g.tens[k];
    }
    va.rho = g.rho;
    va.table = bias + (size_t)g.c0 * p->R * 4;
    va.counts = p->counts + p->chain_off[g.c0];
    va.scal = p->scal + (size_t)g.c0 * kScalStride;
    va.drho = g.drho_dir;
    va.ghat = g.ghat;
    va.nbv = g.nbv;
    va.dbeta = g.dbeta;
    va.partial = g.partial;
    va.x_floor = (float)p->cosmo.x_floor;
    va.steep = (float)p->web.steepness;
    va.lam_th = (float)p->web.lambda_th;
    va.nv = g.nv;
    {
      Timed tm(p, FZW_K_VOXEL_BWD, (2.5 + 12 * W) * field_bytes(g));
      launch_voxel_bwd(W, va, g.nc, g.nblk, s);
    }
    FinalArgs fa{};
    fa.mode = 2;
    fa.partial = g.partial;
    fa.nblk = g.nblk;
    fa.scal = p->scal + (size_t)g.c0 * kScalStride;
    fa.dtable = dbias + (size_t)g.c0 * p->R * 4;
    fa.ne = p->R * 4;
    fa.flags = p->flags + g.c0;
    launch_finalize(fa, g.nc, s);
  }
  // web adjoint: d rho_k = sum_w m_w sum_ij k_i k_j rfft(dT_ij) + rfft(d rho_direct)
  {
    zf(g, g.tens, &sp[0], 6 * W, s);
    float* dd[1] = {g.drho_dir};
    zf(g, dd, &sp[12], 1, s);
    for (int w = 0; w < W; ++w) hessian_yf(g, &sp[6 * w], sp[6 * w + 0], sp[6 * w + 1], sp[6 * w + 2], s);
    pure_pass(g, Y, false, &sp[12], 1, s);
    Pass ps;
    for (int w = 0; w < W; ++w) {
      ps.in(sp[6 * w + 0], true).in(sp[6 * w + 1], true).in(sp[6 * w + 2], true);
      ps.a.A[0][3 * w + 0] = spec(invn3, 0.f, X, X, TAB_WEB0 + w, NONE);
      ps.a.A[0][3 * w + 1] = spec(invn3, 0.f, X, NONE, TAB_WEB0 + w, NONE);
      ps.a.A[0][3 * w + 2] = spec(invn3, 0.f, NONE, NONE, TAB_WEB0 + w, NONE);
    }
    ps.in(sp[12], true);
    ps.a.A[0][3 * W] = spec_const(invn3);
    ps.out(sp[0], true);
    ps.a.B[0][0] = spec_const(1.f);
    run_pass(g, X, ps, 1, s);
    pure_pass(g, Y, true, &sp[0], 1, s);
    zi(g, &sp[0], &g.drho, 1, s);
  }
  // checkpointed plan: phi_ij again from nu, into the tensor buffers (free
  // now), with the forward model's own kernels, so it equals the forward's
  // phi bit for bit
  if (p->checkpoint) {
    lpt_hessian_spectra(g, nu, s);
    if (!lpt_z(p, g, true, &sp[5], nullptr, g.tens, s)) zi(g, &sp[5], g.tens, 6, s);
  }
  // CIC adjoint -> d Psi (in place over Psi)
  {
    CicArgs ca{};
    set_rsd(ca, p->cosmo, g);
    for (int d = 0; d < 3; ++d) {
      ca.psi[d] = g.psi[d];
      ca.dpsi[d] = g.psi[d];
    }
    ca.n = g.n;
    ca.nv = g.nv;
    ca.drho = g.drho;
    Timed tm(p, FZW_K_CIC_ADJ, 7 * field_bytes(g));
    launch_cic_adjoint(ca, g.nc, s);
  }
  // ALPT adjoint: D = sum_j (-i k_j / k^2) rfft(dPsi_j)
  {
    zf(g, g.psi, &sp[0], 3, s);
    pure_pass(g, Y, false, &sp[0], 1, s);
    {
      Pass pyz;
      pyz.in(sp[1], true).in(sp[2], true).out(sp[1], false);
      pyz.a.A[0][0] = spec(0.f, -1.f, Y, NONE, NONE, NONE);
      pyz.a.A[0][1] = spec(0.f, -1.f, Z, NONE, NONE, NONE);
      pyz.a.B[0][0] = spec_const(1.f);
      run_pass(g, Y, pyz, 1, s);
    }
    Pass ps;
    ps.in(sp[0], true).in(sp[1], true);
    ps.a.A[0][0] = spec(0.f, -1.f, X, NONE, TAB_INVK2, NONE);
    ps.a.A[0][1] = spec(1.f, 0.f, NONE, NONE, TAB_INVK2, NONE);
    ps.out(sp[2], true).out(sp[3], true).out(sp[4], false);
    ps.a.B[0][0] = spec((float)(3.0 / 7.0) * d1 * d1 * invn3, 0.f, NONE, NONE, TAB_K, NONE);
    ps.a.B[1][0] = spec(-invn3, 0.f, NONE, NONE, TAB_1MK, NONE);
    ps.a.B[2][0] = spec(d1, 0.f, NONE, NONE, TAB_H_K, NONE);   // direct d nu_k (times N^3)
    run_pass(g, X, ps, 1, s);
    pure_pass(g, Y, true, &sp[2], 2, s);
  }
  // LPT pointwise adjoint and the spectra of the phi cotangents (one fused
  // launch where the mesh has the four-step z pass; otherwise d phi is formed
  // in place over phi)
  float* const* phi = phi_buffers(p, g);
  if (!lpt_z(p, g, false, &sp[2], &sp[5], phi, s)) {
    float* dst[2] = {g.s2, g.dsc};
    zi(g, &sp[2], dst, 2, s);
    LptArgs la{};
    for (int c = 0; c < 6; ++c) {
      la.phi[c] = phi[c];
      la.dphi[c] = phi[c];
    }
    la.s2 = g.s2;
    la.dsc = g.dsc;
    la.d1 = d1;
    la.tau = (float)p->cosmo.tau_sc;
    la.n = (long long)g.nc * g.nv;
    {
      Timed tm(p, FZW_K_LPT_BWD, 14 * field_bytes(g));
      launch_lpt_bwd(la, s);
    }
    zf(g, phi, &sp[5], 6, s);
  }
  // d nu_k = h / k^2 sum_ij k_i k_j rfft(d phi_ij) + direct ALPT term
  {
    hessian_yf(g, &sp[5], sp[5], sp[6], sp[7], s);
    Pass ps;
    ps.in(sp[5], true).in(sp[6], true).in(sp[7], true).in(sp[4], false);
    ps.a.A[0][0] = spec(invn3, 0.f, X, X, TAB_H_INVK2, NONE);
    ps.a.A[0][1] = spec(invn3, 0.f, X, NONE, TAB_H_INVK2, NONE);
    ps.a.A[0][2] = spec(invn3, 0.f, NONE, NONE, TAB_H_INVK2, NONE);
    ps.a.A[0][3] = spec_const(invn3);
    ps.out(sp[0], true);
    ps.a.B[0][0] = spec_const(1.f);
    run_pass(g, X, ps, 1, s);
    pure_pass(g, Y, true, &sp[0], 1, s);
    float* dst[1] = {dnu};
    zi(g, &sp[0], dst, 1, s);
  }
}

// ------------------------------------------------------------ FFT tuner
// Times the two kernel families of each FFT pass type on this group's own
// buffers (contents irrelevant: zeroed first) and records the faster in the
// process-wide schedule of the mesh size.  The register four-step kernels are
// the default; an alternative replaces them only when it is at least 10%
// faster, so choices do not flip on timing noise.  Runs once per mesh size
// and process, at plan creation (never inside a stream capture).  Setting
// FZW_FFT_TUNE=0 keeps the defaults.
double time_launch_us(hipStream_t s, const std::function<void()>& f) {
  constexpr int kReps = 4;
  f();
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  HIPCHK(hipEventRecord(a, s));
  for (int r = 0; r < kReps; ++r) f();
  HIPCHK(hipEventRecord(b, s));
  HIPCHK(hipEventSynchronize(b));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return 1e3 * ms / kReps;
}

std::mutex g_tune_mu;

void tune_fft(fzw_plan* p, Group& g) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FftSchedule& sc = fft_schedule(g.n);
  if (sc.tuned) return;
  sc.tuned = true;
  const char* env = std::getenv("FZW_FFT_TUNE");
  if (env && env[0] == '0') return;
  hipStream_t s = p->stream;
  HIPCHK(hipMemsetAsync(g.rho, 0, (size_t)g.nc * g.nv * sizeof(float), s));
  for (int k = 0; k < 2; ++k) HIPCHK(hipMemsetAsync(g.spec[k], 0, (size_t)g.nc * g.ns * sizeof(float2), s));
  float* fin[1] = {g.rho};
  float2* sp0[1] = {g.spec[0]};
  auto pick = [&](int& choice, double* us, const std::function<void()>& f) {
    choice = kSchedFourStep;
    us[0] = time_launch_us(s, f);
    choice = kSchedStockham;
    us[1] = time_launch_us(s, f);
    choice = us[1] < 0.9 * us[0] ? kSchedStockham : kSchedFourStep;
  };
  if (has_four_step_z(g.n)) {
    pick(sc.z, sc.us[0], [&] {
      zf(g, fin, sp0, 1, s);
      zi(g, sp0, fin, 1, s);
    });
  }
  // a mixing pass with an axis factor and a radial table (the general path)
  pick(sc.xy, sc.us[1], [&] {
    Pass ps;
    ps.in(g.spec[0], true).out(g.spec[1], true);
    ps.a.A[0][0] = spec(0.f, 1.f, Y, NONE, TAB_INVK2, NONE);
    ps.a.B[0][0] = spec_const(1.f);
    run_pass(g, Y, ps, 1, s);
  });
  if (has_pure_pass(g.n)) pick(sc.pure, sc.us[2], [&] { pure_xy(g, Y, false, sp0, sp0, 1, s); });
  HIPCHK(hipStreamSynchronize(s));
}

void check_ready(fzw_plan* p) {
  for (int c = 0; c < p->n_chains; ++c)
    if (!p->counts_set[c]) throw Error(FZW_E_STATE, "counts of chain " + std::to_string(c) + " not set");
}

// Runs f(g) for every group.  Groups of different meshes share no buffer, so
// with more than one they run side by side: each on its own stream, forked
// from and joined back into the plan's stream with events (inside a stream
// capture this becomes a fork / join of the graph).
template <class F>
void for_groups(fzw_plan* p, F&& f) {
  if (p->groups.size() == 1) {
    f(p->groups[0]);
    return;
  }
  hipStream_t s0 = p->stream;
  HIPCHK(hipEventRecord(p->ev_fork, s0));
  for (auto& g : p->groups) {
    HIPCHK(hipStreamWaitEvent(g.gstream, p->ev_fork, 0));
    p->stream = g.gstream;
    try {
      f(g);
    } catch (...) {
      p->stream = s0;
      throw;
    }
    p->stream = s0;
    HIPCHK(hipEventRecord(g.gdone, g.gstream));
  }
  for (auto& g : p->groups) HIPCHK(hipStreamWaitEvent(s0, g.gdone, 0));
}

// Fields fzw_get_field may return after a forward model or a gradient.
// (delta_L is the trace of the stored phi_ij: a checkpointed plan keeps none)
unsigned long long forward_fields(const fzw_plan* p) {
  return ((1ull << (6 + 6 * p->W)) - 1ull) & (p->checkpoint ? ~1ull : ~0ull);
}
unsigned long long gradient_fields(const fzw_plan* p) {
  unsigned long long m = (1ull << 4) | (1ull << 5) | (1ull << FZW_FIELD_DRHO);
  for (int j = 0; j < 3; ++j) m |= 1ull << (FZW_FIELD_DPSI + j);
  // delta_L is the trace of the stored phi_ij, which the adjoint overwrites
  // where the LPT step is not fused with its z transforms
  bool fused = true;
  for (const auto& g : p->groups) fused = fused && has_four_step_z(g.n);
  if (fused && !p->checkpoint) m |= 1ull;
  return m;
}

void clear_flags(fzw_plan* p) { launch_fill_i32(p->flags, p->n_chains, 0, p->stream); }

void forward_all(fzw_plan* p, const float* nu, const float* bias, float* nbar, double* logl) {
  t_plan = p;
  for_groups(p, [&](Group& g) { forward_group(p, g, nu + p->chain_off[g.c0], bias, nbar, logl, false); });
  p->field_valid = forward_fields(p);
}

void value_and_grad_all(fzw_plan* p, const float* nu, const float* bias, double* logl, float* dnu, float* dbias) {
  t_plan = p;
  for_groups(p, [&](Group& g) {
    forward_group(p, g, nu + p->chain_off[g.c0], bias, nullptr, logl, true);
    adjoint_group(p, g, nu + p->chain_off[g.c0], bias, dnu + p->chain_off[g.c0], dbias);
  });
  p->field_valid = gradient_fields(p);
}

template <class F>
fzw_status guarded(F&& f) {
  try {
    f();
    return FZW_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return FZW_E_HIP;
  } catch (...) {
    g_last_error = "unknown error";
    return FZW_E_HIP;
  }
}

void free_plan(fzw_plan* p) {
  for (auto& kv : p->graphs) {
    (void)hipGraphExecDestroy(kv.second.e);
    (void)hipGraphDestroy(kv.second.g);
  }
  if (p->ev_in) (void)hipEventDestroy(p->ev_in);
  if (p->ev_out) (void)hipEventDestroy(p->ev_out);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  for (auto& g : p->groups) {
    if (g.gdone) (void)hipEventDestroy(g.gdone);
    if (g.gstream) (void)hipStreamDestroy(g.gstream);
  }
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (void* a : p->allocs) (void)hipFree(a);
  if (p->nuts_vec) (void)hipFree(p->nuts_vec);
  if (p->nuts_st) (void)hipFree(p->nuts_st);
  if (p->nuts_partial) (void)hipFree(p->nuts_partial);
  if (p->nuts_any) (void)hipFree(p->nuts_any);
  if (p->nuts_any_host) (void)hipHostFree(p->nuts_any_host);
  if (p->stats_buf) (void)hipFree(p->stats_buf);
  for (auto e : p->evpool) (void)hipEventDestroy(e);
  delete p;
}

}  // namespace

// Splitting schemes of one integration step, K(a_0) D(b_1) K(a_1) ... D(b_m)
// K(a_m), the gradient evaluated after every drift (Section 2.2 names
// second- and fourth-order HMC and the variant of Blanes, Casas & Sanz-Serna
// 2014): kick-drift-kick; the two-stage splitting with b = 0.21178; three
// leapfrog steps of w1, w0, w1 with w1 = 1/(2 - 2^(1/3)), w0 = 1 - 2 w1
// (Yoshida 1990), adjacent kicks merged.
struct Scheme {
  int stages;
  double kick[4];
  double drift[3];
};

static const Scheme& scheme_of(int kind) {
  static const Scheme lf = {1, {0.5, 0.5}, {1.0}};
  static const double b = 0.21178;
  static const Scheme bl = {2, {b, 1.0 - 2.0 * b, b}, {0.5, 0.5}};
  static const double w1 = 1.0 / (2.0 - std::cbrt(2.0)), w0 = 1.0 - 2.0 * w1;
  static const Scheme y4 = {3, {0.5 * w1, 0.5 * (w1 + w0), 0.5 * (w0 + w1), 0.5 * w1}, {w1, w0, w1}};
  return kind == FZW_INT_BLANES2 ? bl : kind == FZW_INT_YOSHIDA4 ? y4 : lf;
}

// ------------------------------------------------------------------ NUTS
namespace {

constexpr int kNutsVecs = 13;   // W(q,p,g), L(q,p,g), R(q,p,g), candidates (2), momentum sums (2)

void nuts_reserve(fzw_plan* p, int md) {
  const long long tv = p->total_vox + (long long)p->n_chains * p->nfree;
  if (p->nuts_vec && p->nuts_tv == tv && p->nuts_md >= md) return;
  HIPCHK(hipStreamSynchronize(p->stream));
  if (p->nuts_vec) HIPCHK(hipFree(p->nuts_vec));
  p->nuts_vec = nullptr;
  const size_t n = (size_t)(kNutsVecs + 2 * md) * (size_t)tv;
  if (hipMalloc(&p->nuts_vec, n * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    p->nuts_vec = nullptr;
    throw Error(FZW_E_OOM, "hipMalloc of the NUTS state (" + std::to_string(n * 4) + " bytes) failed");
  }
  p->nuts_tv = tv;
  p->nuts_md = md;
  if (!p->nuts_st) {
    const size_t pe = (size_t)p->n_chains * (kNutsBlk + 1) * (2 * 12);
    HIPCHK(hipMalloc(&p->nuts_st, sizeof(NutsChain) * p->n_chains));
    HIPCHK(hipMalloc(&p->nuts_partial, sizeof(double) * pe));
    HIPCHK(hipMalloc(&p->nuts_any, sizeof(int)));
    HIPCHK(hipHostMalloc(&p->nuts_any_host, sizeof(int), hipHostMallocDefault));
  }
}

// Aligned blocks of the subtree that the leaf k closes (k odd) or opens (k even).
NutsLeafPlan leaf_plan(int k) {
  NutsLeafPlan lp{};
  lp.store = -1;
  if ((k & 1) == 0) {
    lp.store = __builtin_popcount((unsigned)k);
    return lp;
  }
  for (int m = 1; ((k + 1) & ((1 << m) - 1)) == 0 && lp.nchk < 12; ++m)
    lp.slot[lp.nchk++] = __builtin_popcount((unsigned)(k + 1 - (1 << m)));
  return lp;
}

bool nuts_any(fzw_plan* p, const NutsVec& a, NutsScalarArgs& sa, int mode) {
  launch_nuts_scalar(a, sa, p->n_chains, mode, 0, 0, 0, p->stream);
  HIPCHK(hipMemcpyAsync(p->nuts_any_host, sa.any, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return *p->nuts_any_host != 0;
}

void run_nuts(fzw_plan* p, float* nu, float* u, const float* z_nu, const float* z_u, const float* base,
              const float* minv_nu, const float* minv_u, const float* step, const float* uniforms, int md,
              double* potential, double* accept_stat, int* stats) {
  nuts_reserve(p, md);
  hipStream_t s = p->stream;
  const int C = p->n_chains;
  const long long tv = p->nuts_tv, tvox = p->total_vox;
  float* v = p->nuts_vec;
  NutsVec a{};
  float** slots[kNutsVecs] = {&a.wq, &a.wp, &a.wg, &a.lq, &a.lp, &a.lg, &a.rq, &a.rp, &a.rg,
                              &a.cq, &a.sq, &a.rho_t, &a.rho_s};
  for (int i = 0; i < kNutsVecs; ++i) *slots[i] = v + (size_t)i * tv;
  a.ckp = v + (size_t)kNutsVecs * tv;
  a.ckr = a.ckp + (size_t)md * tv;
  a.tv = tv;
  a.st = p->nuts_st;
  a.partial = p->nuts_partial;
  a.nval = 2 * 12;
  a.has_u = p->nfree > 0 ? 1 : 0;
  std::vector<NutsSeg> segs;
  for (auto& g : p->groups) {
    const long long o = p->chain_off[g.c0];
    segs.push_back(NutsSeg{o, g.nv, g.c0, g.nc, 0, minv_nu + o, z_nu + o});
  }
  if (p->nfree > 0) segs.push_back(NutsSeg{tvox, p->nfree, 0, C, 1, minv_u, z_u});
  NutsScalarArgs sa{};
  sa.step = step;
  sa.uniforms = uniforms;
  sa.max_depth = md;
  sa.n_uniforms = 2 * md + (1 << md) - 1;
  sa.scal = p->scal;
  sa.any = p->nuts_any;
  sa.potential = potential;
  sa.accept_stat = accept_stat;
  sa.stats = stats;
  ParamArgs pa{};
  pa.u = a.wq + tvox;
  pa.mu = p->mu;
  pa.sigma = p->sigma;
  pa.tie = p->tie;
  pa.sign = p->fsign;
  pa.base = base;
  pa.table = p->table_tmp;
  pa.dtable = p->dtable_tmp;
  pa.ne = p->R * 4;
  pa.nfree = p->nfree;
  pa.flags = p->flags;
  auto vec = [&](int op, float frac = 1.f) {
    for (auto& g : segs) launch_nuts_vec(a, g, op, frac, s);
  };
  const Scheme& sc = scheme_of(p->integrator);
  auto scalar = [&](int mode, int j, int k, int nchk) { launch_nuts_scalar(a, sa, C, mode, j, k, nchk, s); };
  auto gradient = [&] {
    launch_params(pa, C, 0, 0.f, kEBlk, nullptr, s);
    value_and_grad_all(p, a.wq, p->table_tmp, nullptr, a.wg, p->dtable_tmp);
    launch_nuts_ugrad(a, pa, tvox, C, s);
  };
  // start: gradient at the current state, momentum from the draws, H0
  clear_flags(p);
  HIPCHK(hipMemcpyAsync(a.wq, nu, sizeof(float) * tvox, hipMemcpyDeviceToDevice, s));
  if (p->nfree > 0)
    HIPCHK(hipMemcpyAsync(a.wq + tvox, u, sizeof(float) * C * p->nfree, hipMemcpyDeviceToDevice, s));
  gradient();
  vec(kNutsOpInit);
  vec(kNutsOpEnergy);
  scalar(kNutsInit, 0, 0, 0);
  vec(kNutsOpStart);
  for (int j = 0; j < md; ++j) {
    scalar(kNutsBegin, j, 0, 0);
    vec(kNutsOpBegin);
    const int nleaf = 1 << j;
    for (int k = 0; k < nleaf; ++k) {
      for (int st = 0; st < sc.stages; ++st) {
        vec(kNutsOpKick, (float)sc.kick[st]);
        vec(kNutsOpDrift, (float)sc.drift[st]);
        gradient();
      }
      vec(kNutsOpKick, (float)sc.kick[sc.stages]);
      vec(kNutsOpEnergy);
      scalar(kNutsLeaf, j, k, 0);
      const NutsLeafPlan lp = leaf_plan(k);
      for (auto& g : segs) launch_nuts_leaf(a, g, lp, s);
      if (lp.nchk > 0) scalar(kNutsChecks, j, k, lp.nchk);
      // every chain's subtree may have ended early (turn or divergence)
      if (k + 1 < nleaf && k >= 7 && ((k + 1) & k) == 0 && !nuts_any(p, a, sa, kNutsAnySub)) break;
    }
    scalar(kNutsJoin, j, 0, 0);
    vec(kNutsOpMerge);
    scalar(kNutsTree, j, 0, 0);
    if (!nuts_any(p, a, sa, kNutsAnyTree)) break;
  }
  scalar(kNutsOut, 0, 0, 0);
  HIPCHK(hipMemcpyAsync(nu, a.cq, sizeof(float) * tvox, hipMemcpyDeviceToDevice, s));
  if (p->nfree > 0)
    HIPCHK(hipMemcpyAsync(u, a.cq + tvox, sizeof(float) * C * p->nfree, hipMemcpyDeviceToDevice, s));
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* fzw_last_error(void) { return g_last_error.c_str(); }

fzw_status fzw_plan_create(fzw_plan** out, int n_chains, const int* mesh_n, const double* box_l,
                           const fzw_cosmo* cosmo, const fzw_web* web, void* stream) {
  return fzw_plan_create_ex(out, n_chains, mesh_n, box_l, cosmo, web, stream, 0u);
}

fzw_status fzw_plan_create_ex(fzw_plan** out, int n_chains, const int* mesh_n, const double* box_l,
                              const fzw_cosmo* cosmo, const fzw_web* web, void* stream, unsigned flags) {
  if (!out || !mesh_n || !box_l || !cosmo || !web || n_chains <= 0 || (flags & ~(unsigned)FZW_PLAN_CHECKPOINT)) {
    g_last_error = "fzw_plan_create: null argument, n_chains <= 0 or unknown flag";
    return FZW_E_ARG;
  }
  *out = nullptr;
  auto* p = new fzw_plan();
  p->checkpoint = (flags & FZW_PLAN_CHECKPOINT) != 0;
  {
    const char* e = std::getenv("FZW_LIKELIHOOD_FP64");
    p->like_fp64 = e && e[0] == '1';
  }
  fzw_status st = guarded([&] {
    if (web->n_webs < 1 || web->n_webs > 2) throw Error(FZW_E_ARG, "n_webs must be 1 or 2");
    if (cosmo->rsd_axis < -1 || cosmo->rsd_axis > FZW_RSD_RADIAL)
      throw Error(FZW_E_ARG, "rsd_axis must be -1 (none), 0..2 (plane-parallel) or 3 (radial)");
    if (!(cosmo->x_floor > 0)) throw Error(FZW_E_ARG, "x_floor must be > 0");
    p->n_chains = n_chains;
    p->cosmo = *cosmo;
    p->web = *web;
    p->W = web->n_webs;
    p->R = p->W == 1 ? 4 : 16;
    p->stream = static_cast<hipStream_t>(stream);
    p->user_stream = p->stream;
    p->amp = power_amplitude(*cosmo);
    long long off = 0;
    for (int c = 0; c < n_chains; ++c) {
      if (!supported_n(mesh_n[c]))
        throw Error(FZW_E_SIZE, "unsupported mesh size " + std::to_string(mesh_n[c]) +
                                    " (supported: 16, 32, 64, 96, 128, 256, 512)");
      if (!(box_l[c] > 0)) throw Error(FZW_E_ARG, "box_l must be > 0");
      p->chain_off.push_back(off);
      const long long nv = (long long)mesh_n[c] * mesh_n[c] * mesh_n[c];
      off += nv;
      if (!p->groups.empty() && p->groups.back().n == mesh_n[c] && p->groups.back().box == box_l[c]) {
        p->groups.back().nc++;
      } else {
        Group g;
        g.n = mesh_n[c];
        g.box = box_l[c];
        g.c0 = c;
        g.nc = 1;
        g.nv = nv;
        g.P = spectrum_pitch(g.n);
        g.ns = (long long)g.n * g.n * g.P;
        g.nblk = (int)std::min<long long>((nv + 255) / 256, 16384);
        p->groups.push_back(g);
      }
      p->chain_group.push_back((int)p->groups.size() - 1);
    }
    p->total_vox = off;
    p->counts_set.assign(n_chains, false);
    // (arguments are validated above, before any device call)
    HIPCHK(hipGetDevice(&p->device));
    // the fixed partials array of fzw_power_multipoles_noalloc on this device
    HIPCHK(scratch_setup(p->device));
    size_t part = 0;
    for (auto& g : p->groups) {
      build_tables(p, g);
      alloc_group(p, g);
      prime_launch_config(g.n);
      tune_fft(p, g);
      g.partial = dalloc<double>(p, std::max<size_t>((size_t)g.nc * g.nblk * (size_t)std::max(2, p->R * 4), 512));
      if (p->groups.size() > 1) {
        // default priority, non-blocking
        HIPCHK(hipStreamCreateWithFlags(&g.gstream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&g.gdone, hipEventDisableTiming));
      }
    }
    part = std::max<size_t>(part, 512);
    p->partial_elems = part;
    p->partial = dalloc<double>(p, part);
    p->counts = dalloc<uint16_t>(p, (size_t)off);
    p->scal = dalloc<double>(p, (size_t)n_chains * kScalStride);
    HIPCHK(hipMemset(p->scal, 0, (size_t)n_chains * kScalStride * sizeof(double)));
    p->flags = dalloc<int>(p, (size_t)n_chains);
    HIPCHK(hipMemset(p->flags, 0, (size_t)n_chains * sizeof(int)));
    p->dnu_tmp = dalloc<float>(p, (size_t)off);
    p->table_tmp = dalloc<float>(p, (size_t)n_chains * p->R * 4);
    p->dtable_tmp = dalloc<float>(p, (size_t)n_chains * p->R * 4);
    p->epartial = dalloc<double>(p, (size_t)n_chains * kEBlk);
    p->tie = dalloc<int>(p, (size_t)p->R * 4);
    p->fsign = dalloc<float>(p, 64);
    p->mu = dalloc<double>(p, 64);
    p->sigma = dalloc<double>(p, 64);
    // default priority, non-blocking: the caller's stream may be the legacy
    // default stream, which cannot be captured
    HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    HIPCHK(hipDeviceSynchronize());
  });
  if (st != FZW_OK) {
    free_plan(p);
    return st;
  }
  *out = p;
  return FZW_OK;
}

void fzw_plan_destroy(fzw_plan* plan) {
  if (!plan) return;
  (void)hipStreamSynchronize(plan->stream);
  free_plan(plan);
}

fzw_status fzw_set_counts(fzw_plan* p, int chain, const uint16_t* counts) {
  if (!p || !counts || chain < 0 || chain >= p->n_chains) {
    g_last_error = "fzw_set_counts: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    const Group& g = p->groups[p->chain_group[chain]];
    uint16_t* dst = p->counts + p->chain_off[chain];
    HIPCHK(hipMemcpyAsync(dst, counts, g.nv * sizeof(uint16_t), hipMemcpyDeviceToDevice, p->stream));
    launch_count_consts(dst, g.nv, p->partial, 256, p->scal + (size_t)chain * kScalStride, p->stream);
    HIPCHK(hipStreamSynchronize(p->stream));
    double ntr = 0;
    HIPCHK(hipMemcpy(&ntr, p->scal + (size_t)chain * kScalStride + kScalNtr, sizeof(double), hipMemcpyDeviceToHost));
    if (!(ntr > 0)) throw Error(FZW_E_ARG, "counts of chain " + std::to_string(chain) + " sum to zero");
    p->counts_set[chain] = true;
  });
}

fzw_status fzw_forward(fzw_plan* p, const float* nu, const float* bias, float* nbar, double* logl) {
  if (!p || !nu || !bias || !logl) {
    g_last_error = "fzw_forward: null argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    check_ready(p);
    clear_flags(p);
    forward_all(p, nu, bias, nbar, logl);
    HIPCHK(hipGetLastError());
  });
}

fzw_status fzw_value_and_grad(fzw_plan* p, const float* nu, const float* bias, double* logl, float* dnu,
                              float* dbias) {
  if (!p || !nu || !bias || !logl || !dnu || !dbias) {
    g_last_error = "fzw_value_and_grad: null argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    check_ready(p);
    clear_flags(p);
    value_and_grad_all(p, nu, bias, logl, dnu, dbias);
    HIPCHK(hipGetLastError());
  });
}

fzw_status fzw_set_sampling(fzw_plan* p, const int* tie, int n_free, const double* prior_mu,
                            const double* prior_sigma) {
  if (!p || !tie || n_free < 0 || n_free > 64 || (n_free > 0 && (!prior_mu || !prior_sigma))) {
    g_last_error = "fzw_set_sampling: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    for (int e = 0; e < p->R * 4; ++e)
      if (tie[e] < -1 || tie[e] >= n_free) throw Error(FZW_E_ARG, "tie entry out of range");
    for (int f = 0; f < n_free; ++f)
      if (!(prior_sigma[f] > 0)) throw Error(FZW_E_ARG, "prior_sigma must be > 0");
    HIPCHK(hipMemcpy(p->tie, tie, sizeof(int) * p->R * 4, hipMemcpyHostToDevice));
    if (n_free > 0) {
      HIPCHK(hipMemcpy(p->mu, prior_mu, sizeof(double) * n_free, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(p->sigma, prior_sigma, sizeof(double) * n_free, hipMemcpyHostToDevice));
    }
    {
      std::vector<float> ones(64, 1.f);
      HIPCHK(hipMemcpy(p->fsign, ones.data(), sizeof(float) * 64, hipMemcpyHostToDevice));
    }
    p->nfree = n_free;
    for (auto& kv : p->graphs) {
      (void)hipGraphExecDestroy(kv.second.e);
      (void)hipGraphDestroy(kv.second.g);
    }
    p->graphs.clear();
  });
}

static void enqueue_trajectory(fzw_plan* p, float* nu, float* u, float* p_nu, float* p_u, const float* base,
                               const float* minv_nu, const float* minv_u, const float* step, int n_steps,
                               double* h_start, double* h_end) {
  hipStream_t s = p->stream;
  ParamArgs pa{};
  pa.u = u;
  pa.pu = p_u;
  pa.minv_u = minv_u;
  pa.mu = p->mu;
  pa.sigma = p->sigma;
  pa.tie = p->tie;
  pa.sign = p->fsign;
  pa.base = base;
  pa.table = p->table_tmp;
  pa.dtable = p->dtable_tmp;
  pa.step = step;
  pa.scal = p->scal;
  pa.epartial = p->epartial;
  pa.ne = p->R * 4;
  pa.nfree = p->nfree;
  pa.flags = p->flags;
  const int C = p->n_chains;
  auto grad = [&] {
    launch_params(pa, C, 0, 0.f, kEBlk, nullptr, s);
    value_and_grad_all(p, nu, p->table_tmp, nullptr, p->dnu_tmp, p->dtable_tmp);
  };
  auto leap = [&](const Group& g) {
    LeapArgs la{};
    la.q = nu + p->chain_off[g.c0];
    la.p = p_nu + p->chain_off[g.c0];
    la.g = p->dnu_tmp + p->chain_off[g.c0];
    la.minv = minv_nu + p->chain_off[g.c0];
    la.step = step;
    la.chain0 = g.c0;
    la.nv = g.nv;
    la.partial = p->epartial + (size_t)g.c0 * kEBlk;
    return la;
  };
  auto hamiltonian = [&](double* h) {
    for (auto& g : p->groups) launch_energy(leap(g), g.nc, kEBlk, s);
    launch_params(pa, C, 3, 0.f, kEBlk, h, s);
  };
  const Scheme& sc = scheme_of(p->integrator);
  clear_flags(p);   // a fill kernel, not a memset node, inside the captured graph
  auto kick = [&](double a) {
    for (auto& g : p->groups) launch_kick(leap(g), g.nc, (float)a, s);
    launch_params(pa, C, 1, (float)a, kEBlk, nullptr, s);
  };
  grad();
  hamiltonian(h_start);
  for (int it = 0; it < n_steps; ++it) {
    for (int i = 0; i < sc.stages; ++i) {
      kick(sc.kick[i]);
      for (auto& g : p->groups) launch_drift(leap(g), g.nc, (float)sc.drift[i], s);
      launch_params(pa, C, 2, (float)sc.drift[i], kEBlk, nullptr, s);
      grad();
    }
    kick(sc.kick[sc.stages]);
  }
  hamiltonian(h_end);
}

fzw_status fzw_leapfrog(fzw_plan* p, float* nu, float* u, float* p_nu, float* p_u, const float* bias_base,
                        const float* minv_nu, const float* minv_u, const float* step, int n_steps,
                        double* h_start, double* h_end) {
  if (!p || !nu || !p_nu || !bias_base || !minv_nu || !step || !h_start || !h_end || n_steps < 0) {
    g_last_error = "fzw_leapfrog: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    check_ready(p);
    if (p->nfree < 0) throw Error(FZW_E_STATE, "fzw_set_sampling not called");
    if (p->nfree > 0 && (!u || !p_u || !minv_u)) throw Error(FZW_E_ARG, "u, p_u, minv_u required");
    std::vector<uintptr_t> key = {(uintptr_t)nu, (uintptr_t)u, (uintptr_t)p_nu, (uintptr_t)p_u,
                                  (uintptr_t)bias_base, (uintptr_t)minv_nu, (uintptr_t)minv_u,
                                  (uintptr_t)step, (uintptr_t)n_steps, (uintptr_t)h_start, (uintptr_t)h_end,
                                  (uintptr_t)p->integrator};
    auto it = p->graphs.find(key);
    // order the private stream after the caller's work
    HIPCHK(hipEventRecord(p->ev_in, p->user_stream));
    HIPCHK(hipStreamWaitEvent(p->cap_stream, p->ev_in, 0));
    if (it == p->graphs.end()) {
      fzw_plan::GraphEntry ge{};
      HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
      p->stream = p->cap_stream;
      const bool timing = p->timing;   // no event records inside the graph
      p->timing = false;
      try {
        enqueue_trajectory(p, nu, u, p_nu, p_u, bias_base, minv_nu, minv_u, step, n_steps, h_start, h_end);
      } catch (...) {
        p->stream = p->user_stream;
        p->timing = timing;
        hipGraph_t dummy;
        (void)hipStreamEndCapture(p->cap_stream, &dummy);
        (void)hipGetLastError();
        throw;
      }
      p->stream = p->user_stream;
      p->timing = timing;
      HIPCHK(hipStreamEndCapture(p->cap_stream, &ge.g));
      HIPCHK(hipGraphInstantiate(&ge.e, ge.g, nullptr, nullptr, 0));
      it = p->graphs.emplace(key, ge).first;
    }
    HIPCHK(hipGraphLaunch(it->second.e, p->cap_stream));
    // and the caller's stream after the trajectory
    HIPCHK(hipEventRecord(p->ev_out, p->cap_stream));
    HIPCHK(hipStreamWaitEvent(p->user_stream, p->ev_out, 0));
  });
}

fzw_status fzw_nuts(fzw_plan* p, float* nu, float* u, const float* z_nu, const float* z_u, const float* bias_base,
                    const float* minv_nu, const float* minv_u, const float* step, const float* uniforms,
                    int max_depth, double* potential, double* accept_stat, int* stats) {
  if (!p || !nu || !z_nu || !bias_base || !minv_nu || !step || !uniforms || !potential || !accept_stat || !stats ||
      max_depth < 1 || max_depth > FZW_NUTS_MAX_DEPTH) {
    g_last_error = "fzw_nuts: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    check_ready(p);
    if (p->nfree < 0) throw Error(FZW_E_STATE, "fzw_set_sampling not called");
    if (p->nfree > 0 && (!u || !z_u || !minv_u)) throw Error(FZW_E_ARG, "u, z_u, minv_u required");
    run_nuts(p, nu, u, z_nu, z_u, bias_base, minv_nu, minv_u, step, uniforms, max_depth, potential, accept_stat,
             stats);
  });
}

fzw_status fzw_welford(fzw_plan* p, const float* x, float* mean, float* m2, long long n, int count) {
  if (!p || !x || !mean || !m2 || n < 0 || count < 1) {
    g_last_error = "fzw_welford: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    if (n > 0) launch_welford(x, mean, m2, n, count, p->stream);
  });
}

fzw_status fzw_inverse_mass(fzw_plan* p, const float* m2, float* minv, long long n, int count) {
  if (!p || !m2 || !minv || n < 0 || count < 2) {
    g_last_error = "fzw_inverse_mass: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    if (n > 0) launch_inv_mass(m2, minv, n, count, p->stream);
  });
}

void fzw_dual_avg_init(fzw_dual_avg* s, double eps0, double target) {
  s->mu = std::log(10.0 * eps0);
  s->target = target;
  s->gamma = 0.05;
  s->t0 = 10.0;
  s->kappa = 0.75;
  s->t = 0;
  s->h_bar = 0.0;
  s->log_eps_bar = 0.0;
}

double fzw_dual_avg_update(fzw_dual_avg* s, double accept_stat) {
  s->t += 1;
  const double t = (double)s->t;
  const double w = 1.0 / (t + s->t0);
  s->h_bar = (1.0 - w) * s->h_bar + w * (s->target - accept_stat);
  const double log_eps = s->mu - std::sqrt(t) / s->gamma * s->h_bar;
  const double eta = std::pow(t, -s->kappa);
  s->log_eps_bar = eta * log_eps + (1.0 - eta) * s->log_eps_bar;
  return std::exp(log_eps);
}

double fzw_dual_avg_final(const fzw_dual_avg* s) { return std::exp(s->log_eps_bar); }

// ------------------------------------------------------ validation statistics
constexpr int kStatsMaxBins = 256;
constexpr int kStatsMaxTheta = 256;

static double* stats_buffer(fzw_plan* p) {
  if (!p->stats_buf) {
    const size_t n = (size_t)stats_blocks() * kStatsMaxBins * 4 + 4 * kStatsMaxTheta + 4 + kStatsMaxTheta;
    HIPCHK(hipMalloc(&p->stats_buf, n * sizeof(double)));
  }
  return p->stats_buf;
}

static Group stats_group(fzw_plan* p, int n) {
  for (auto& g : p->groups)
    if (g.n == n) {
      Group one = g;
      one.nc = 1;
      return one;
    }
  throw Error(FZW_E_SIZE, "mesh size not in plan");
}

static void forward_spectrum(const Group& g, const float* x, float2* out, hipStream_t s) {
  float* src[1] = {const_cast<float*>(x)};
  float2* dst[1] = {out};
  zf(g, src, dst, 1, s);
  pure_pass(g, Y, false, dst, 1, s);
  pure_pass(g, X, false, dst, 1, s);
}

fzw_status fzw_power_multipoles(fzw_plan* p, int mesh_n, const float* a, const float* b, double k_lo, double dk,
                                int nbins, double* out) {
  if (!p || !a || !out || !(dk > 0) || nbins < 1 || nbins > kStatsMaxBins) {
    g_last_error = "fzw_power_multipoles: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    t_plan = p;
    Group g = stats_group(p, mesh_n);
    hipStream_t s = p->stream;
    double* buf = stats_buffer(p);
    forward_spectrum(g, a, g.spec[0], s);
    if (b) forward_spectrum(g, b, g.spec[1], s);
    const double dx = g.box / g.n;
    const double pnorm = dx * dx * dx / ((double)g.n * g.n * g.n);
    launch_multipoles(g.spec[0], b ? g.spec[1] : g.spec[0], g.n, g.P, 2.0 * M_PI / g.box, k_lo, dk, nbins, pnorm,
                      buf, out, s);
    HIPCHK(hipGetLastError());
  });
}

fzw_status fzw_power_multipoles_noalloc(fzw_plan* p, int mesh_n, const float* a, const float* b, double k_lo,
                                        double dk, int nbins, double* out) {
  if (!p || !a || !out || !(dk > 0) || nbins < 1) {
    g_last_error = "fzw_power_multipoles_noalloc: bad argument";
    return FZW_E_ARG;
  }
  if (nbins > scratch_max_bins()) {
    g_last_error = "fzw_power_multipoles_noalloc: nbins " + std::to_string(nbins) + " exceeds the fixed partials " +
                   "array (at most " + std::to_string(scratch_max_bins()) + " bins)";
    return FZW_E_ARG;
  }
  return guarded([&] {
    double* buf = scratch_ptr(p->device);
    if (!buf) throw Error(FZW_E_STATE, "fzw_power_multipoles_noalloc: partials array not set up on this device");
    // no timing records: they would create events
    t_plan = nullptr;
    Group g = stats_group(p, mesh_n);
    hipStream_t s = p->stream;
    forward_spectrum(g, a, g.spec[0], s);
    if (b) forward_spectrum(g, b, g.spec[1], s);
    const double dx = g.box / g.n;
    const double pnorm = dx * dx * dx / ((double)g.n * g.n * g.n);
    launch_multipoles(g.spec[0], b ? g.spec[1] : g.spec[0], g.n, g.P, 2.0 * M_PI / g.box, k_lo, dk, nbins, pnorm,
                      buf, out, s);
    HIPCHK(hipGetLastError());
  });
}

fzw_status fzw_bispectrum(fzw_plan* p, int mesh_n, const float* delta, double k1, double k2, double dk, int ntheta,
                          const double* theta, double* out) {
  if (!p || !delta || !theta || !out || !(dk > 0) || !(k1 > 0) || !(k2 > 0) || ntheta < 1 ||
      ntheta > kStatsMaxTheta) {
    g_last_error = "fzw_bispectrum: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    t_plan = p;
    Group g = stats_group(p, mesh_n);
    hipStream_t s = p->stream;
    double* buf = stats_buffer(p);
    double* partial = buf;
    double* sc = buf + (size_t)stats_blocks() * kStatsMaxBins * 4;   // [ntheta][4]
    double* p12 = sc + 4 * kStatsMaxTheta;                            // [4]
    double* k3d = p12 + 4;                                            // [ntheta]
    const double kf = 2.0 * M_PI / g.box;
    std::vector<double> k3(ntheta);
    for (int t = 0; t < ntheta; ++t) k3[t] = std::sqrt(k1 * k1 + k2 * k2 + 2.0 * k1 * k2 * std::cos(theta[t]));
    HIPCHK(hipMemcpyAsync(k3d, k3.data(), sizeof(double) * ntheta, hipMemcpyHostToDevice, s));
    forward_spectrum(g, delta, g.spec[0], s);
    auto shell_field = [&](double kc, bool indicator, float* dst) {
      launch_shell(indicator ? nullptr : g.spec[0], g.spec[1], g.n, g.P, kf, kc - 0.5 * dk, kc + 0.5 * dk, s);
      float2* sp[1] = {g.spec[1]};
      pure_pass(g, X, true, sp, 1, s);
      pure_pass(g, Y, true, sp, 1, s);
      float* d[1] = {dst};
      zi(g, sp, d, 1, s);
    };
    // six real scratch fields: the phi buffers, or the tensor buffers of a
    // checkpointed plan
    float* const* f6 = phi_buffers(p, g);
    float *i1 = f6[0], *j1 = f6[1], *i2 = f6[2], *j2 = f6[3], *i3 = f6[4], *j3 = f6[5];
    shell_field(k1, false, i1);
    shell_field(k1, true, j1);
    shell_field(k2, false, i2);
    shell_field(k2, true, j2);
    launch_shell_power(g.spec[0], g.n, g.P, kf, k1 - 0.5 * dk, k1 + 0.5 * dk, partial, p12, s);
    launch_shell_power(g.spec[0], g.n, g.P, kf, k2 - 0.5 * dk, k2 + 0.5 * dk, partial, p12 + 2, s);
    for (int t = 0; t < ntheta; ++t) {
      shell_field(k3[t], false, i3);
      shell_field(k3[t], true, j3);
      launch_triple_sum(i1, i2, i3, g.nv, partial, sc + 4 * t, s);
      launch_triple_sum(j1, j2, j3, g.nv, partial, sc + 4 * t + 1, s);
      launch_shell_power(g.spec[0], g.n, g.P, kf, k3[t] - 0.5 * dk, k3[t] + 0.5 * dk, partial, sc + 4 * t + 2, s);
    }
    launch_bispectrum_final(sc, p12, k3d, ntheta, g.n, g.box / g.n, out, s);
    // the fields those buffers held
    p->field_valid &= p->checkpoint ? ~(((1ull << (6 * p->W)) - 1ull) << 6) : ~1ull;
    HIPCHK(hipStreamSynchronize(s));   // k3 lives on the host stack
  });
}

fzw_status fzw_wiener_start(fzw_plan* p, float* nu) {
  if (!p || !nu) {
    g_last_error = "fzw_wiener_start: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    check_ready(p);
    t_plan = p;
    hipStream_t s = p->stream;
    for (auto& g : p->groups) {
      float* out = nu + p->chain_off[g.c0];
      launch_wiener_contrast(p->counts + p->chain_off[g.c0], p->scal, g.c0, g.nc, g.nv, out, s);
      float* io[1] = {out};
      zf(g, io, &g.spec[0], 1, s);
      pure_pass(g, Y, false, &g.spec[0], 1, s);
      pure_pass(g, X, false, &g.spec[0], 1, s);
      launch_wiener_filter(g.spec[0], g.tabs + (size_t)TAB_H * g.tab_stride, g.n, g.P, p->scal, g.c0, g.nc, g.ns, s);
      pure_pass(g, X, true, &g.spec[0], 1, s);
      pure_pass(g, Y, true, &g.spec[0], 1, s);
      zi(g, &g.spec[0], io, 1, s);
    }
    HIPCHK(hipGetLastError());
  });
}

fzw_status fzw_set_sampling_signs(fzw_plan* p, const int* sign, int n_free) {
  if (!p || !sign || n_free < 0 || n_free > 64) {
    g_last_error = "fzw_set_sampling_signs: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    if (n_free != p->nfree) throw Error(FZW_E_STATE, "n_free differs from the one given to fzw_set_sampling");
    std::vector<float> sg(64, 1.f);
    for (int f = 0; f < n_free; ++f) {
      if (sign[f] != 1 && sign[f] != -1) throw Error(FZW_E_ARG, "signs must be +1 or -1");
      sg[f] = (float)sign[f];
    }
    HIPCHK(hipMemcpy(p->fsign, sg.data(), sizeof(float) * 64, hipMemcpyHostToDevice));
  });
}

fzw_status fzw_set_integrator(fzw_plan* p, int kind) {
  if (!p || kind < FZW_INT_LEAPFROG || kind > FZW_INT_YOSHIDA4) {
    g_last_error = "fzw_set_integrator: bad argument";
    return FZW_E_ARG;
  }
  p->integrator = kind;
  return FZW_OK;
}

fzw_status fzw_get_field(fzw_plan* p, int chain, int field, float* out) {
  const bool known = field >= 0 && (field < 6 + 6 * (p ? p->W : 0) ||
                                    (field >= FZW_FIELD_DRHO && field < FZW_FIELD_DPSI + 3));
  if (!p || !out || chain < 0 || chain >= p->n_chains || !known) {
    g_last_error = "fzw_get_field: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    if (!((p->field_valid >> field) & 1ull))
      throw Error(FZW_E_STATE, "fzw_get_field: field " + std::to_string(field) +
                                   " was not left by the last evaluation (see fzw.h)");
    const Group& g = p->groups[p->chain_group[chain]];
    const long long o = (long long)(chain - g.c0) * g.nv;
    const size_t bytes = g.nv * sizeof(float);
    const float* src = nullptr;
    if (field == 0) {
      // delta_L is the trace of the first-order Hessian
      launch_trace3(g.phi[0] + o, g.phi[1] + o, g.phi[2] + o, out, g.nv, p->stream);
      return;
    }
    if (field == FZW_FIELD_DRHO) src = g.drho + o;
    else if (field >= FZW_FIELD_DPSI) src = g.psi[field - FZW_FIELD_DPSI] + o;   // d Psi in place over Psi
    else if (field <= 3) src = g.psi[field - 1] + o;
    else if (field == 4) src = g.rho + o;
    else if (field == 5) src = g.logf + o;
    else src = g.tens[field - 6] + o;
    HIPCHK(hipMemcpyAsync(out, src, bytes, hipMemcpyDeviceToDevice, p->stream));
  });
}

fzw_status fzw_nonfinite_flags(fzw_plan* p, int* flags) {
  if (!p || !flags) {
    g_last_error = "fzw_nonfinite_flags: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    HIPCHK(hipMemcpyAsync(flags, p->flags, sizeof(int) * p->n_chains, hipMemcpyDeviceToDevice, p->stream));
  });
}

fzw_status fzw_check_finite(fzw_plan* p, int* flags_host) {
  if (!p) {
    g_last_error = "fzw_check_finite: null plan";
    return FZW_E_ARG;
  }
  int any = 0;
  const fzw_status st = guarded([&] {
    std::vector<int> f(p->n_chains, 0);
    HIPCHK(hipStreamSynchronize(p->stream));
    HIPCHK(hipMemcpy(f.data(), p->flags, sizeof(int) * p->n_chains, hipMemcpyDeviceToHost));
    for (int c = 0; c < p->n_chains; ++c) {
      any |= f[c];
      if (flags_host) flags_host[c] = f[c];
    }
  });
  if (st != FZW_OK) return st;
  return any ? FZW_W_NONFINITE : FZW_OK;
}

static fzw_status fft_common(fzw_plan* p, int n, int batch, const void* in, void* out, bool r2c) {
  if (!p || !in || !out || batch <= 0) {
    g_last_error = "fzw_fft: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    const Group* gp = nullptr;
    for (auto& g : p->groups)
      if (g.n == n) gp = &g;
    if (!gp) throw Error(FZW_E_SIZE, "mesh size not in plan");
    Group g = *gp;
    g.nc = 1;
    t_plan = p;
    const long long m1 = n / 2 + 1;
    for (int b = 0; b < batch; ++b) {
      if (r2c) {
        float* src[1] = {const_cast<float*>(static_cast<const float*>(in)) + (size_t)b * g.nv};
        zf(g, src, &g.spec[0], 1, p->stream);
        pure_pass(g, Y, false, &g.spec[0], 1, p->stream);
        pure_pass(g, X, false, &g.spec[0], 1, p->stream);
        launch_spec_repack(g.spec[0], static_cast<float2*>(out) + (size_t)b * n * n * m1, n, g.P, (int)m1,
                           (long long)n * n, p->stream);
      } else {
        launch_spec_repack(static_cast<const float2*>(in) + (size_t)b * n * n * m1, g.spec[0], n, (int)m1, g.P,
                           (long long)n * n, p->stream);
        pure_pass(g, X, true, &g.spec[0], 1, p->stream);
        pure_pass(g, Y, true, &g.spec[0], 1, p->stream);
        float* dst[1] = {static_cast<float*>(out) + (size_t)b * g.nv};
        zi(g, &g.spec[0], dst, 1, p->stream);
      }
    }
    HIPCHK(hipGetLastError());
  });
}

fzw_status fzw_fft_r2c(fzw_plan* p, int n, int batch, const float* in, void* out_complex) {
  return fft_common(p, n, batch, in, out_complex, true);
}
fzw_status fzw_fft_c2r(fzw_plan* p, int n, int batch, const void* in_complex, float* out) {
  return fft_common(p, n, batch, in_complex, out, false);
}

fzw_status fzw_set_cic_method(fzw_plan* p, int method) {
  if (!p || (method != FZW_CIC_SORTED && method != FZW_CIC_ATOMIC)) {
    g_last_error = "fzw_set_cic_method: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    for (auto& kv : p->graphs) {
      (void)hipGraphExecDestroy(kv.second.e);
      (void)hipGraphDestroy(kv.second.g);
    }
    p->graphs.clear();
    p->cic_method = method;
  });
}

fzw_status fzw_timing_enable(fzw_plan* p, int on) {
  if (!p) {
    g_last_error = "fzw_timing_enable: null plan";
    return FZW_E_ARG;
  }
  return guarded([&] {
    HIPCHK(hipStreamSynchronize(p->stream));
    p->timing = on != 0;
    p->recs.clear();
    p->evused = 0;
  });
}

fzw_status fzw_timing_read(fzw_plan* p, int klass, double* total_ms, long long* launches, double* bytes) {
  if (!p || klass < 0 || klass >= FZW_K_COUNT || !total_ms || !launches || !bytes) {
    g_last_error = "fzw_timing_read: bad argument";
    return FZW_E_ARG;
  }
  return guarded([&] {
    HIPCHK(hipStreamSynchronize(p->stream));
    double ms = 0, b = 0;
    long long n = 0;
    for (auto& r : p->recs) {
      if (r.klass != klass) continue;
      float e = 0;
      HIPCHK(hipEventElapsedTime(&e, r.a, r.b));
      ms += e;
      b += r.bytes;
      ++n;
    }
    *total_ms = ms;
    *launches = n;
    *bytes = b;
  });
}

size_t fzw_chain_offset(const fzw_plan* p, int chain) {
  if (!p || chain < 0 || chain >= p->n_chains) return 0;
  return (size_t)p->chain_off[chain];
}
int fzw_n_regions(const fzw_plan* p) { return p ? p->R : 0; }
size_t fzw_workspace_bytes(const fzw_plan* p) { return p ? p->ws_bytes : 0; }

fzw_status fzw_set_fft_schedule(int mesh_n, int z, int xy, int pure) {
  auto ok = [](int v) { return v == kSchedFourStep || v == kSchedStockham; };
  if (!supported_n(mesh_n) || !ok(z) || !ok(xy) || !ok(pure)) {
    g_last_error = "fzw_set_fft_schedule: bad argument";
    return FZW_E_ARG;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FftSchedule& sc = fft_schedule(mesh_n);
  sc.z = z;
  sc.xy = xy;
  sc.pure = pure;
  sc.tuned = true;
  return FZW_OK;
}

fzw_status fzw_fft_schedule(int mesh_n, int* z, int* xy, int* pure, double* us6) {
  if (!supported_n(mesh_n) || !z || !xy || !pure) {
    g_last_error = "fzw_fft_schedule: bad argument";
    return FZW_E_ARG;
  }
  const FftSchedule& sc = fft_schedule(mesh_n);
  *z = sc.z;
  *xy = sc.xy;
  *pure = sc.pure;
  if (us6)
    for (int k = 0; k < 6; ++k) us6[k] = sc.us[k / 2][k % 2];
  return sc.tuned ? FZW_OK : FZW_E_STATE;
}

}  // extern "C"
