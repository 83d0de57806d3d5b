// Argument blocks and launchers of the non-FFT kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fzw.h"

namespace fzw {

// per-chain float64 scalars kept on the device
enum { kScalNtr = 0, kScalLgConst = 1, kScalSumF = 2, kScalLnC = 3, kScalLogL = 4, kScalG = 5, kScalStride = 8 };

struct LptArgs {
  const float* phi[6];
  float* s2;     // forward: output S2; backward: input cotangent of S2
  float* dsc;    // forward: output d_SC; backward: input cotangent of d_SC
  float* dphi[6];
  float d1, tau;
  long long n;
};

// Division by a fixed divisor d > 0 of dividends below 2^31, as a multiply
// and a shift: s = ceil(log2 d), m = floor(2^(32+s) / d) + 1.  The rounding
// error of m stays below 1/(2d) of a unit, so the quotient is exact.
struct FastDiv {
  unsigned d = 1, s = 0;
  unsigned long long m = 0x100000001ull;
};
inline FastDiv make_fastdiv(unsigned d) {
  FastDiv f;
  f.d = d;
  unsigned s = 0;
  while ((1ull << s) < d) ++s;
  f.s = s;
  f.m = (unsigned long long)((((unsigned __int128)1) << (32 + s)) / d) + 1ull;
  return f;
}
__device__ __forceinline__ unsigned fast_div(unsigned x, const FastDiv& f) {
  return (unsigned)(((unsigned long long)x * f.m) >> (32 + f.s));
}

struct CicArgs {
  const float* psi[3];
  float scale[3];        // displacement -> cell units per axis (plane-parallel RSD factor included)
  int radial;            // 1: radial RSD about the box centre (scale is then 1/dx on every axis)
  float f_los;           // growth rate of the radial shift
  int n;
  FastDiv dn;            // division by n (set by the launchers)
  long long nv;
  int* count;            // [chains][n*n] particles per column, then the scatter cursor
  int* offset;           // [chains][n*n+1] column starts in the sorted array
  int* bsum;             // [chains][n*n/4096 rounded up]
  float4* sorted;        // [chains][nv] (tx, ty, tz, bits of (by << 16 | bz)) in column order
  unsigned long long* acc;  // [chains][nv] fixed-point accumulator (atomic deposit), kept zero
  float* rho;            // [chains][nv]
  int* flags;            // [chains] non-finite flags (FZW_NF_*), set by the deposit
  const float* drho;     // adjoint input
  float* dpsi[3];        // adjoint output
};

struct VoxelArgs {
  const float* tens[12];
  float* dtens[12];
  const float* rho;
  const float* table;    // [chains][R*4]
  const uint16_t* counts;
  const double* scal;
  float* logf;
  float* beta;
  float* drho;
  const float* ghat;     // backward inputs from the likelihood pass (see LikeArgs)
  const float* nbv;
  const float* dbeta;
  double* partial;
  float x_floor, steep, lam_th;
  long long nv;
};

struct LikeArgs {
  const float* logf;
  const float* beta;
  const uint16_t* counts;
  const double* scal;
  double* partial;
  float* nbar;
  // gradient precursors, written when ghat is set: g-hat = beta (n - nbar) /
  // (beta + nbar), nbar, and d lnP / d beta, all formed in float64
  float* ghat;
  float* nbv;
  float* dbeta;
  long long nv;
};

struct FinalArgs {
  int mode;
  const double* partial;
  int nblk;
  double* scal;
  double* logl;
  float* dtable;
  int ne;
  int* flags;            // [chains] non-finite flags (FZW_NF_*)
};

struct LeapArgs {
  float* q;
  float* p;
  const float* g;
  const float* minv;
  const float* step;
  int chain0;
  long long nv;
  double* partial;
};

struct ParamArgs {
  float* u;
  float* pu;
  const float* minv_u;
  const double* mu;
  const double* sigma;
  const int* tie;
  const float* sign;        // [n_free] +1 or -1: a free parameter is sign * exp(u)
  const float* base;
  float* table;
  const float* dtable;
  const float* step;
  const double* scal;
  const double* epartial;
  int ne, nfree;
  int* flags;               // [chains] non-finite flags (FZW_NF_*)
};

// ---------------------------------------------------------------- NUTS
// Per-chain scalar state of a no-U-turn transition (device).
struct NutsChain {
  double h0;        // Hamiltonian at the start
  double log_w;     // log weight of the tree, relative to exp(-h0)
  double log_ws;    // log weight of the subtree being built
  double acc_sum;   // sum over leaves of min(1, exp(h0 - H))
  double u_cand;    // potential at the tree's candidate
  double u_sub;     // potential at the subtree's candidate
  double u_leaf;    // potential at the last leaf
  double prior;     // log-normal prior term of the free parameters at the last gradient
  float eps;        // step size
  float se;         // signed step of the current doubling (0: chain idle)
  int v;            // direction of the current doubling
  int active;       // the tree is still growing
  int sub_active;   // the current subtree is still growing
  int leaf_ok;      // the last leaf was made and did not diverge
  int sel;          // the last leaf became the subtree's candidate
  int merged;       // the last subtree was joined to the tree
  int msel;         // and its candidate became the tree's
  int diverging;
  int depth;
  int n_leaf;
};

// One piece of the NUTS state vectors: chains c0..c0+nc-1, each holding len
// floats at off + (c - c0) * len; the field part (nu) or the free parameters.
struct NutsSeg {
  long long off, len;
  int c0, nc;
  int is_u;
  const float* minv;   // inverse mass of chain c0's first coordinate
  const float* z;      // momentum draws, same layout as minv
};

struct NutsVec {
  float *wq, *wp, *wg;      // working leaf (g: d logL/d nu on the field, dU/du on the parameters)
  float *lq, *lp, *lg;      // backward end of the tree
  float *rq, *rp, *rg;      // forward end
  float *cq, *sq;           // candidates of the tree and of the subtree
  float *rho_t, *rho_s;     // momentum sums of the tree and of the subtree
  float *ckp, *ckr;         // [max_depth][tv]: block-start momenta and prefix sums
  long long tv;             // floats per state vector
  NutsChain* st;
  double* partial;          // [chains][kNutsBlk + 1][nval]
  int nval;
  int has_u;                // the parameter part exists (writes the last partial slot)
};

constexpr int kNutsBlk = 256;
enum { kNutsOpKick = 0, kNutsOpDrift = 1, kNutsOpEnergy = 2, kNutsOpInit = 3, kNutsOpStart = 4, kNutsOpBegin = 5,
       kNutsOpMerge = 6 };

struct NutsLeafPlan {
  int store;        // checkpoint slot written at this leaf, or -1
  int nchk;         // aligned blocks that end at this leaf
  int slot[12];     // their checkpoint slots (max_depth <= 12)
};

// frac scales the chain's signed step for the kick and drift ops
void launch_nuts_vec(const NutsVec& a, const NutsSeg& g, int op, float frac, hipStream_t s);
void launch_nuts_leaf(const NutsVec& a, const NutsSeg& g, const NutsLeafPlan& lp, hipStream_t s);
void launch_nuts_ugrad(const NutsVec& a, const ParamArgs& pa, long long uoff, int chains, hipStream_t s);
struct NutsScalarArgs {
  const float* step;        // [chains]
  const float* uniforms;    // [chains][n_uniforms]
  int n_uniforms, max_depth;
  const double* scal;       // per-chain likelihood scalars (log-likelihood at kScalLogL)
  int* any;                 // one flag: some chain (or subtree) still growing
  double* potential;        // outputs
  double* accept_stat;
  int* stats;               // [chains][3]: depth, leapfrog steps, divergence
};
enum { kNutsInit = 0, kNutsBegin = 1, kNutsLeaf = 2, kNutsChecks = 3, kNutsJoin = 4, kNutsTree = 5, kNutsOut = 6,
       kNutsAnyTree = 7, kNutsAnySub = 8 };
void launch_nuts_scalar(const NutsVec& a, const NutsScalarArgs& sa, int chains, int mode, int j, int k, int nchk,
                        hipStream_t s);
void launch_welford(const float* x, float* mean, float* m2, long long n, int count, hipStream_t s);
void launch_inv_mass(const float* m2, float* minv, long long n, int count, hipStream_t s);

void launch_fill_i32(int* p, long long n, int v, hipStream_t s);
void launch_fill_f32(float* p, long long n, float v, hipStream_t s);
void launch_lpt_fwd(const LptArgs& a, hipStream_t s);
void launch_lpt_bwd(const LptArgs& a, hipStream_t s);
void launch_cic_deposit(const CicArgs& a, int chains, hipStream_t s);
void launch_cic_adjoint(const CicArgs& a, int chains, hipStream_t s);
void launch_cic_deposit_atomic(const CicArgs& a, int chains, hipStream_t s);
void launch_voxel_fwd(int w, const VoxelArgs& a, int chains, int nblk, hipStream_t s);
void launch_voxel_bwd(int w, const VoxelArgs& a, int chains, int nblk, hipStream_t s);
void launch_likelihood(const LikeArgs& a, int chains, int nblk, bool fp64, hipStream_t s);
void launch_finalize(const FinalArgs& a, int chains, hipStream_t s);
void launch_count_consts(const uint16_t* cnt, long long nv, double* partial, int nblk, double* scal, hipStream_t s);
void launch_kick(const LeapArgs& a, int chains, float frac, hipStream_t s);
void launch_drift(const LeapArgs& a, int chains, float frac, hipStream_t s);
void launch_energy(const LeapArgs& a, int chains, int nblk, hipStream_t s);
void launch_params(const ParamArgs& a, int chains, int mode, float frac, int nblk_energy, double* hout, hipStream_t s);
void launch_trace3(const float* a, const float* b, const float* c, float* out, long long n, hipStream_t s);
void launch_wiener_contrast(const uint16_t* counts, const double* scal, int chain0, int chains, long long nv,
                            float* out, hipStream_t s);
void launch_wiener_filter(float2* spec, const float* htab, int n, int pitch, const double* scal, int chain0,
                          int chains, long long per_chain, hipStream_t s);
int stats_blocks();
// The multipoles' fixed partials array of the allocation-free call: its
// device address is resolved once per device (with that device current) by
// scratch_setup; scratch_ptr returns it (nullptr before).  At most
// scratch_max_bins() bins.
hipError_t scratch_setup(int device);
double* scratch_ptr(int device);
int scratch_max_bins();
void launch_multipoles(const float2* a, const float2* b, int n, int pitch, double kf, double k_lo, double dk,
                       int nbins, double pnorm, double* partial, double* out, hipStream_t s);
void launch_shell(const float2* src, float2* dst, int n, int pitch, double kf, double lo, double hi, hipStream_t s);
void launch_triple_sum(const float* a, const float* b, const float* c, long long nv, double* partial, double* dst,
                       hipStream_t s);
void launch_shell_power(const float2* d, int n, int pitch, double kf, double lo, double hi, double* partial,
                        double* dst, hipStream_t s);
void launch_bispectrum_final(const double* sc, const double* p12, const double* k3, int ntheta, int n, double dx,
                             double* out, hipStream_t s);
void launch_spec_repack(const float2* src, float2* dst, int n, int sp, int dp, long long rows, hipStream_t s);

}  // namespace fzw
