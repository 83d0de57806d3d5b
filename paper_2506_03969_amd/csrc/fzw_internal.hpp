// Internal interfaces between the host runtime and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fzw {

// A spectral multiplier m(k) = (re + i im) * K(ax0, ax1) * tab0[|n|^2] * tab1[|n|^2]
// where K is 1 (no axis), k_a (one axis, zero on that axis' Nyquist index),
// k_a k_b (a != b, each zeroed on its Nyquist index) or k_a^2 (a == b).
struct SpecOp {
  float re, im;
  signed char ax[2];
  signed char tb[2];
};

inline SpecOp spec_zero() { return SpecOp{0.f, 0.f, {-1, -1}, {-1, -1}}; }
inline SpecOp spec_const(float re, float im = 0.f) { return SpecOp{re, im, {-1, -1}, {-1, -1}}; }
inline SpecOp spec(float re, float im, int a0, int a1, int t0, int t1) {
  return SpecOp{re, im, {(signed char)a0, (signed char)a1}, {(signed char)t0, (signed char)t1}};
}
inline bool spec_is_zero(const SpecOp& s) { return s.re == 0.f && s.im == 0.f; }

constexpr int kMaxIn = 8;
constexpr int kMaxMid = 3;
constexpr int kMaxOut = 6;

// One strided (x or y) pass over a half spectrum stored [x][y][P] complex.
// Phase 1: each input is transformed forward along the axis (if its bit in
// `in_fft` is set) and mixed: mid[m] = sum_i A[m][i] X_i.
// Phase 2: out[o] = B[o] . mid, inverse-transformed along the axis if its bit
// in `out_fft` is set, then stored.
// Radial multipliers with a closed form in |n|^2 = q, evaluated in registers
// instead of gathered from the tables: kind 0 looks the table up; 1: 1/k^2;
// 2: 2^(-c q); 3: 1 - 2^(-c q); 4: 2^(-c q)/k^2; 5: l 2^(-c q), with
// k^2 = kf^2 q (and 0 for the 1/k^2 forms at q = 0); c holds the Gaussian's
// k^2 r^2 / 2 coefficient divided by ln 2.
constexpr int kRadialTables = 10;
struct RadialForms {
  signed char kind[kRadialTables];
  float c[kRadialTables];
  float l[kRadialTables];
  float inv_kf2;
};

struct PassArgs {
  const float2* in[kMaxIn];
  float2* out[kMaxOut];
  int nin, nmid, nout;
  unsigned in_fft, out_fft;
  SpecOp A[kMaxMid][kMaxIn];
  SpecOp B[kMaxOut][kMaxMid];
  long long chain_stride;     // elements between chains batched on grid.z
  const float* tabs;          // radial tables [ntab][tab_stride]
  int tab_stride;
  float kf;                   // 2 pi / L
  const RadialForms* rf;      // tables evaluated in closed form instead of looked up (device)
};

// The z transforms around the LPT pointwise step, fused with it (see
// lpt_fwd_z4_kernel / lpt_bwd_z4_kernel).  Forward: sin = six phi_ij spectra,
// field = the six phi_ij (written), sout = S2 and d_SC spectra.  Adjoint: sin
// = dS2 and dd_SC spectra, field = phi_ij (read), sout = six d phi_ij spectra.
struct LptZArgs {
  const float2* sin[6];
  float* field[6];
  float2* sout[6];
  long long spec_chain_stride;    // complex elements between chains
  long long field_chain_stride;   // floats between chains
  float d1, tau;
};

// Pure strided transforms of narr arrays (out[i] may equal in[i]).
struct PureArgs {
  const float2* in[8];
  float2* out[8];
  int narr, chains;
  long long chain_stride;   // complex elements between chains
};

// Kernel family of each pass type for one mesh size: the register four-step
// kernels or the LDS Stockham kernels (z passes, mixing x/y passes), and for
// pure x/y transforms the persistent four-step kernel or the mixing kernel.
// Process-wide, so every plan computes with the same kernels; chosen by
// timing when the first plan of a mesh size is created.
enum { kSchedFourStep = 0, kSchedStockham = 1 };
struct FftSchedule {
  int z = kSchedFourStep, xy = kSchedFourStep, pure = kSchedFourStep;
  bool tuned = false;
  double us[3][2] = {};   // measured [z, xy, pure][four-step, alternative] per launch
};
FftSchedule& fft_schedule(int n);

// Launchers (defined next to their kernels).
void launch_zpass_r2c(int n, const float* const* in, float2* const* out, int narr, long long chains,
                      long long in_chain_stride, long long out_chain_stride, const float2* tw_half,
                      const float2* tw_full, hipStream_t s);
// Pure x (axis 0) or y (axis 1) transforms, forward or inverse, of several
// arrays in one persistent launch.  Returns false (nothing launched) for
// meshes without the four-step strided kernels.
bool launch_pure_pass(int n, int axis, bool inverse, const PureArgs& a, const float2* tw, hipStream_t s);
bool has_pure_pass(int n);
// Occupancy queries of the persistent kernels, made once per mesh size
// before any stream capture.
void prime_launch_config(int n);
// Meshes whose z passes use the register four-step kernels (all but 96).
bool has_four_step_z(int n);
// Returns false (and launches nothing) for meshes without the four-step z pass.
bool launch_lpt_z(int n, bool fwd, const LptZArgs& a, int chains, const float2* tw_half, const float2* tw_full,
                  hipStream_t s);
void launch_zpass_c2r(int n, const float2* const* in, float* const* out, int narr, long long chains,
                      long long in_chain_stride, long long out_chain_stride, const float2* tw_half,
                      const float2* tw_full, hipStream_t s);
// axis 0 = x pass, 1 = y pass
void launch_xy_pass(int n, int axis, const PassArgs& a, int chains, const float2* tw, hipStream_t s);

int spectrum_pitch(int n);    // P: padded length of a row of N/2+1 modes

}  // namespace fzw
