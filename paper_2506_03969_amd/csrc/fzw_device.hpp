// Device building blocks shared by the gfx950 kernels of the fuzzy-web
// likelihood: complex arithmetic, small DFT butterflies, an LDS Stockham FFT
// over a tile of lines, spectral multipliers and wave64 reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fzw_internal.hpp"

namespace fzw {

constexpr int kThreads = 256;   // threads per workgroup of the FFT passes
constexpr int kTile = 4096;     // complex elements per FFT tile

// ---------------------------------------------------------------- complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// -------------------------------------------------------------- butterflies
// In-register DFTs of length R; forward uses exp(-2 pi i jk/R), inverse +.
template <bool INV>
__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2* v) {
  const float c = -0.5f;
  const float s = INV ? 0.86602540378443864676f : -0.86602540378443864676f;
  float2 a = v[0], b = v[1], d = v[2];
  float2 t = cadd(b, d);
  float2 u = csub(b, d);
  v[0] = cadd(a, t);
  float2 m = make_float2(a.x + c * t.x, a.y + c * t.y);
  // i*s*u
  float2 r = make_float2(-s * u.y, s * u.x);
  v[1] = cadd(m, r);
  v[2] = csub(m, r);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2* v) {
  float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  float2 b0 = cadd(v[1], v[3]), b1 = rot90<INV>(csub(v[1], v[3]));
  v[0] = cadd(a0, b0);
  v[2] = csub(a0, b0);
  v[1] = cadd(a1, b1);
  v[3] = csub(a1, b1);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  const float h = 0.70710678118654752440f;
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  // twiddles w^k, w = exp(-+2 pi i / 8)
  float2 o1 = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                  : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
  float2 o2 = rot90<INV>(o[2]);
  float2 o3 = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                  : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else if constexpr (R == 8) dft8<INV>(v);
}

// ------------------------------------------------------------ radix plans
// Stockham radix sequence per transform length.
template <int N> struct Radix;
template <> struct Radix<8>   { static constexpr int n = 1; static constexpr int r[3] = {8, 1, 1}; };
template <> struct Radix<16>  { static constexpr int n = 2; static constexpr int r[3] = {4, 4, 1}; };
template <> struct Radix<24>  { static constexpr int n = 2; static constexpr int r[3] = {3, 8, 1}; };
template <> struct Radix<32>  { static constexpr int n = 2; static constexpr int r[3] = {4, 8, 1}; };
template <> struct Radix<48>  { static constexpr int n = 3; static constexpr int r[3] = {3, 4, 4}; };
template <> struct Radix<64>  { static constexpr int n = 2; static constexpr int r[3] = {8, 8, 1}; };
template <> struct Radix<96>  { static constexpr int n = 3; static constexpr int r[3] = {3, 4, 8}; };
template <> struct Radix<128> { static constexpr int n = 3; static constexpr int r[3] = {2, 8, 8}; };
template <> struct Radix<256> { static constexpr int n = 3; static constexpr int r[3] = {4, 8, 8}; };
template <> struct Radix<512> { static constexpr int n = 3; static constexpr int r[3] = {8, 8, 8}; };

// One Stockham stage of radix R on LINES lines of length N stored in LDS with
// line stride LS (in place: every thread reads its butterflies into
// registers, the workgroup synchronises, then writes them back).  `tw` holds
// exp(-2 pi i k / N) for k < N.
template <int N, int LINES, int LS, int R, bool INV, int NT>
__device__ __forceinline__ void stockham_stage(float2* lds, const float2* tw, int ns) {
  constexpr int B = N / R;                         // butterflies per line
  constexpr int TOTAL = LINES * B;
  constexpr int PER = (TOTAL + NT - 1) / NT;
  const int t = threadIdx.x;
  float2 v[PER][R];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int idx = t + p * NT;
    if (TOTAL % NT == 0 || idx < TOTAL) {
      const int line = idx / B;
      const int j = idx - line * B;
      const float2* src = lds + line * LS + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[p][r] = src[r * B];
      const int k = j % ns;
      if (ns > 1) {
        const int step = k * (N / (ns * R));
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[(r * step) % N];
          if (INV) w.y = -w.y;
          v[p][r] = cmul(v[p][r], w);
        }
      }
      dftR<R, INV>(v[p]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int idx = t + p * NT;
    if (TOTAL % NT == 0 || idx < TOTAL) {
      const int line = idx / B;
      const int j = idx - line * B;
      const int k = j % ns;
      float2* dst = lds + line * LS + (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * ns] = v[p][r];
    }
  }
  __syncthreads();
}

// Full length-N transform of LINES lines in LDS (natural order in and out).
// Caller must have synchronised after filling the LDS tile.
template <int N, int LINES, int LS, bool INV, int NT = kThreads>
__device__ __forceinline__ void fft_lines(float2* lds, const float2* tw) {
  using P = Radix<N>;
  int ns = 1;
  stockham_stage<N, LINES, LS, P::r[0], INV, NT>(lds, tw, ns);
  ns *= P::r[0];
  if constexpr (P::n > 1) {
    stockham_stage<N, LINES, LS, P::r[1], INV, NT>(lds, tw, ns);
    ns *= P::r[1];
  }
  if constexpr (P::n > 2) {
    stockham_stage<N, LINES, LS, P::r[2], INV, NT>(lds, tw, ns);
  }
}

// ------------------------------------------------ register (four-step) DFTs
// Compile-time trigonometry for the twiddles inside register DFTs.
constexpr double kPiD = 3.14159265358979323846264338327950288;
constexpr double cx_sin(double x) {
  while (x > kPiD) x -= 2.0 * kPiD;
  while (x < -kPiD) x += 2.0 * kPiD;
  double term = x, sum = x;
  for (int i = 1; i < 40; ++i) {
    term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos(double x) { return cx_sin(x + 0.5 * kPiD); }

template <int N>
struct CTw {   // exp(-2 pi i k / N)
  float re[N], im[N];
  constexpr CTw() : re(), im() {
    for (int k = 0; k < N; ++k) {
      re[k] = (float)cx_cos(2.0 * kPiD * k / N);
      im[k] = (float)(-cx_sin(2.0 * kPiD * k / N));
    }
  }
};

template <int N, bool INV>
__device__ __forceinline__ float2 ctw(int k) {
  constexpr CTw<N> t{};
  return make_float2(t.re[k], INV ? -t.im[k] : t.im[k]);
}

// Natural-order DFT of N values held in registers (N = 2, 4, 8, 16, 32).
template <int N, bool INV>
__device__ __forceinline__ void dft_reg(float2* v) {
  if constexpr (N == 2) dft2<INV>(v);
  else if constexpr (N == 4) dft4<INV>(v);
  else if constexpr (N == 8) dft8<INV>(v);
  else {
    // N = 4 * B: length-B DFTs over stride-4 subsequences, twiddles, length-4 DFTs
    constexpr int B = N / 4;
    float2 s[4][B];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int b = 0; b < B; ++b) s[a][b] = v[a + 4 * b];
      dft_reg<B, INV>(s[a]);
#pragma unroll
      for (int k = 1; k < B; ++k)
        if (a > 0) s[a][k] = cmul(s[a][k], ctw<N, INV>(a * k));
    }
#pragma unroll
    for (int k = 0; k < B; ++k) {
      float2 t[4] = {s[0][k], s[1][k], s[2][k], s[3][k]};
      dft4<INV>(t);
#pragma unroll
      for (int a = 0; a < 4; ++a) v[B * a + k] = t[a];
    }
  }
}

// Factorisation N = N1 * N2 (N2 = m N1) of the register four-step transforms.
template <int N> struct F4;
template <> struct F4<8>   { static constexpr int N1 = 2, N2 = 4; };
template <> struct F4<16>  { static constexpr int N1 = 4, N2 = 4; };
template <> struct F4<32>  { static constexpr int N1 = 4, N2 = 8; };
template <> struct F4<64>  { static constexpr int N1 = 8, N2 = 8; };
template <> struct F4<128> { static constexpr int N1 = 8, N2 = 16; };
template <> struct F4<256> { static constexpr int N1 = 16, N2 = 16; };
template <> struct F4<512> { static constexpr int N1 = 16, N2 = 32; };

// LDS needed per line by the exchanges (rows padded by one element).
template <int N>
__host__ __device__ constexpr int f4_lds() { return N + F4<N>::N2; }

// Layout A: thread j (of N1 per line) holds elements j + N1 q, q < N2.
// Layout B: thread j holds elements N2 k1 + (j + N1 u), at register u N1 + k1.
// Forward transform A -> B through one LDS exchange (`lline` is this line's
// LDS slice of N values, `tw` = exp(-2 pi i k / N)); all threads of the
// workgroup must call it (it synchronises).
template <int N, bool INV_UNUSED = false>
__device__ __forceinline__ void fwd_A_to_B(float2* v, float2* lline, int j, const float2* tw) {
  constexpr int N1 = F4<N>::N1, N2 = F4<N>::N2, M = N2 / N1;
  dft_reg<N2, false>(v);
#pragma unroll
  for (int k2 = 1; k2 < N2; ++k2) v[k2] = cmul(v[k2], tw[j * k2]);
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) lline[j * (N2 + 1) + k2] = v[k2];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < M; ++u) {
    float2 b[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) b[n1] = lline[n1 * (N2 + 1) + j + N1 * u];
    dft_reg<N1, false>(b);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[u * N1 + k1] = b[k1];
  }
  __syncthreads();
}

// Inverse transform B -> A (unnormalised), one LDS exchange.
template <int N>
__device__ __forceinline__ void inv_B_to_A(float2* v, float2* lline, int j, const float2* tw) {
  constexpr int N1 = F4<N>::N1, N2 = F4<N>::N2, M = N2 / N1;
#pragma unroll
  for (int u = 0; u < M; ++u) {
    const int k2 = j + N1 * u;
    float2 z[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) z[k1] = v[u * N1 + k1];
    dft_reg<N1, true>(z);
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      float2 w = tw[k2 * q];
      w.y = -w.y;
      lline[k2 * (N1 + 1) + q] = q ? cmul(z[q], w) : z[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int n = 0; n < N2; ++n) v[n] = lline[n * (N1 + 1) + j];
  dft_reg<N2, true>(v);
  __syncthreads();
}

// ------------------------------------------------------ spectral multipliers
// Signed frequency index of position i on an axis of length n.
__device__ __forceinline__ int freq_index(int i, int n) { return i <= (n - 1) / 2 ? i : i - n; }

struct KVec {
  int n[3];      // signed frequency indices (x may be unknown in the y pass)
  int n2;        // |n|^2 (only valid when all three are known)
};

// Evaluate one multiplier at a mode.  kf = 2 pi / L; nyq = N/2.  (Axis
// selection uses selects, not array indexing, so nothing spills to scratch.)
__device__ __forceinline__ int kv_axis(const KVec& kv, int a) {
  return a == 0 ? kv.n[0] : (a == 1 ? kv.n[1] : kv.n[2]);
}
__device__ __forceinline__ float2 spec_eval(const SpecOp& op, const KVec& kv, float kf, int nyq,
                                            const float* tabs, int tab_stride) {
  float m = 1.0f;
  const int a0 = op.ax[0], a1 = op.ax[1];
  if (a0 >= 0) {
    const int n0 = kv_axis(kv, a0);
    if (a0 == a1) {
      const float k = kf * (float)n0;
      m *= k * k;
    } else {
      // odd factors vanish on the Nyquist index (-N/2 on x and y, +N/2 on z)
      m *= (abs(n0) == nyq) ? 0.0f : kf * (float)n0;
      if (a1 >= 0) {
        const int n1 = kv_axis(kv, a1);
        m *= (abs(n1) == nyq) ? 0.0f : kf * (float)n1;
      }
    }
  }
  const int q = min(kv.n2, tab_stride - 1);   // |n|^2 <= 3 (N/2)^2 for every valid mode
  if (op.tb[0] >= 0) m *= tabs[op.tb[0] * tab_stride + q];
  if (op.tb[1] >= 0) m *= tabs[op.tb[1] * tab_stride + q];
  return make_float2(op.re * m, op.im * m);
}

// Value of radial multiplier t at q = |n|^2: a closed form where one exists
// (the branch is uniform: t comes from the pass arguments), else the table.
__device__ __forceinline__ float radial_value(const RadialForms* __restrict__ rf, int t, int q, const float* tabs,
                                              int tab_stride) {
  // exp(-c q) as 2^(-c log2(e) q): one multiply and the hardware exp2; its
  // relative error, a few ulp times c q, stays below 1e-6 wherever the
  // factor is above 1e-6
  const int kind = rf->kind[t];
  if (kind == 0) return tabs[t * tab_stride + min(q, tab_stride - 1)];
  const float fq = (float)q;
  const float ik2 = q > 0 ? rf->inv_kf2 * __builtin_amdgcn_rcpf(fq) : 0.f;
  if (kind == 1) return ik2;
  const float g = __builtin_amdgcn_exp2f(-rf->c[t] * fq);
  return kind == 2 ? g : kind == 3 ? 1.f - g : kind == 4 ? g * ik2 : rf->l[t] * g;
}

template <bool CF>
__device__ __forceinline__ float2 spec_eval(const SpecOp& op, const KVec& kv, float kf, int nyq,
                                            const float* tabs, int tab_stride, const RadialForms* rf) {
  if constexpr (!CF) return spec_eval(op, kv, kf, nyq, tabs, tab_stride);
  float m = 1.0f;
  const int a0 = op.ax[0], a1 = op.ax[1];
  if (a0 >= 0) {
    const int n0 = kv_axis(kv, a0);
    if (a0 == a1) {
      const float k = kf * (float)n0;
      m *= k * k;
    } else {
      m *= (abs(n0) == nyq) ? 0.0f : kf * (float)n0;
      if (a1 >= 0) {
        const int n1 = kv_axis(kv, a1);
        m *= (abs(n1) == nyq) ? 0.0f : kf * (float)n1;
      }
    }
  }
  if (op.tb[0] >= 0) m *= radial_value(rf, op.tb[0], kv.n2, tabs, tab_stride);
  if (op.tb[1] >= 0) m *= radial_value(rf, op.tb[1], kv.n2, tabs, tab_stride);
  return make_float2(op.re * m, op.im * m);
}

// A multiplier with no wave-number or table factor: a plain constant.
__device__ __forceinline__ bool spec_is_const(const SpecOp& op) {
  return op.ax[0] < 0 && op.tb[0] < 0 && op.tb[1] < 0;
}

// Smooth hinge of the spherical-collapse term: (a + sqrt(a^2 + tau^2)) / 2
// and its derivative; the exact max(a, 0) when tau = 0.
__device__ __forceinline__ void sc_hinge(float a, float tau, float& hv, float& hd) {
  if (tau > 0.f) {
    const float r = sqrtf(a * a + tau * tau);
    hv = 0.5f * (a + r);
    hd = 0.5f * (1.f + a / r);
  } else {
    hv = a > 0.f ? a : 0.f;
    hd = a > 0.f ? 1.f : 0.f;
  }
}

// ------------------------------------------------------------ buffer access
// Raw buffer loads and stores (gfx9 descriptor, 32-bit byte offsets).  A lane
// offset of kBufOff is out of range for every descriptor made here (they span
// less than 1 GiB): its loads return zero and its stores are dropped, so
// masked lanes need no branch.  The per-element row offset goes in the
// scalar offset, so an access costs no address arithmetic.
using BufRsrc = __amdgpu_buffer_rsrc_t;
constexpr int kBufOff = 0x40000000;
__device__ __forceinline__ BufRsrc buf_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ float2 buf_load2(BufRsrc r, int voff, int soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return make_float2(__int_as_float((int)v[0]), __int_as_float((int)v[1]));
}
__device__ __forceinline__ void buf_store2(BufRsrc r, int voff, int soff, float2 x) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  u32x2 v;
  v[0] = (unsigned)__float_as_int(x.x);
  v[1] = (unsigned)__float_as_int(x.y);
  __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
}

// ------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of `v` over the workgroup (blockDim.x threads, multiple of 64); the
// result is valid in thread 0.  `scratch` needs blockDim.x/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) s += scratch[w];
  }
  __syncthreads();
  return s;
}

}  // namespace fzw
