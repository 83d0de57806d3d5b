// Batched 3-D real<->complex FFT passes for gfx950.
//
// A real field is N^3 float in C order [x][y][z].  Its half spectrum is stored
// [x][y][P] complex64 with P = N/2+1 rounded up to a multiple of 16 so that every
// row starts on a 128-byte boundary; only the first N/2+1 entries of a row are
// used.  The same layout holds after each pass: a z pass turns [x][y][z] reals
// into [x][y][kz], a y pass [x][y][kz] into [x][ky][kz], an x pass into
// [kx][ky][kz].  Every pass is one launch that stages a tile of lines through
// LDS, runs a radix-2/3/4/8 Stockham FFT on all lines of the tile and writes
// the tile back; the strided passes also apply spectral multipliers and mix
// several inputs/outputs so that pointwise spectral work costs no extra pass.
// Transforms are unnormalised in both directions (inverse = N^3 x).
#include <algorithm>

#include "fzw_device.hpp"

namespace fzw {

int spectrum_pitch(int n) { return ((n / 2 + 1) + 15) / 16 * 16; }

template <int N>
__host__ __device__ constexpr int pitch_c() { return ((N / 2 + 1) + 15) / 16 * 16; }

template <int N>
__host__ __device__ constexpr int pow2floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
// lines of the z-pass tile: a power of two with at most kTile complex values
template <int N>
__host__ __device__ constexpr int zlines() {
  return pow2floor<N>(kTile / (N / 2)) > N * N ? N * N : pow2floor<N>(kTile / (N / 2));
}
// columns of the strided-pass tile (a power of two; columns past N/2 are masked)
template <int N>
__host__ __device__ constexpr int xycols() {
  return pow2floor<N>(kTile / N) > 256 ? 256 : pow2floor<N>(kTile / N);
}

struct ZArgs {
  const void* in[16];
  void* out[16];
  int narr;
  long long in_chain_stride, out_chain_stride;   // in elements of the array type
};

// --------------------------------------------------------------- z: R2C
template <int N>
__global__ __launch_bounds__(kThreads) void zpass_r2c_kernel(ZArgs a, const float2* __restrict__ tw_half,
                                                             const float2* __restrict__ tw_full) {
  constexpr int M = N / 2;
  constexpr int L = zlines<N>();
  constexpr int P = pitch_c<N>();
  __shared__ float2 lds[L * M];
  __shared__ float2 twh[M];
  __shared__ float2 twf[N];
  const int t = threadIdx.x;
  const int arr = blockIdx.z % a.narr;
  const long long chain = blockIdx.z / a.narr;
  const float2* in = reinterpret_cast<const float2*>(a.in[arr]) + chain * (a.in_chain_stride / 2);
  float2* out = reinterpret_cast<float2*>(a.out[arr]) + chain * a.out_chain_stride;
  const long long line0 = (long long)blockIdx.x * L;
  for (int i = t; i < M; i += kThreads) twh[i] = tw_half[i];
  for (int i = t; i < N; i += kThreads) twf[i] = tw_full[i];
  const float2* src = in + line0 * M;
  for (int e = t; e < L * M; e += kThreads) lds[e] = src[e];
  __syncthreads();
  fft_lines<M, L, M, false>(lds, twh);
  for (int e = t; e < L * (M + 1); e += kThreads) {
    const int line = e / (M + 1);
    const int k = e - line * (M + 1);
    const float2 zk = lds[line * M + (k == M ? 0 : k)];
    const float2 zm = lds[line * M + (k == 0 ? 0 : M - k)];
    const float2 A = cadd(zk, cconj(zm));
    const float2 B = csub(zk, cconj(zm));
    const float2 wB = cmul(twf[k], B);
    out[(line0 + line) * P + k] = make_float2(0.5f * (A.x + wB.y), 0.5f * (A.y - wB.x));
  }
}

// --------------------------------------------------------------- z: C2R
template <int N>
__global__ __launch_bounds__(kThreads) void zpass_c2r_kernel(ZArgs a, const float2* __restrict__ tw_half,
                                                             const float2* __restrict__ tw_full) {
  constexpr int M = N / 2;
  constexpr int L = zlines<N>();
  constexpr int P = pitch_c<N>();
  __shared__ float2 lds[L * M];
  __shared__ float2 twh[M];
  __shared__ float2 twf[N];
  const int t = threadIdx.x;
  const int arr = blockIdx.z % a.narr;
  const long long chain = blockIdx.z / a.narr;
  const float2* in = reinterpret_cast<const float2*>(a.in[arr]) + chain * a.in_chain_stride;
  float2* out = reinterpret_cast<float2*>(a.out[arr]) + chain * (a.out_chain_stride / 2);
  const long long line0 = (long long)blockIdx.x * L;
  for (int i = t; i < M; i += kThreads) twh[i] = tw_half[i];
  for (int i = t; i < N; i += kThreads) twf[i] = tw_full[i];
  __syncthreads();
  for (int e = t; e < L * M; e += kThreads) {
    const int line = e / M;
    const int k = e - line * M;
    const float2* row = in + (line0 + line) * P;
    float2 xk = row[k];
    float2 xm = row[M - k];
    if (k == 0) {
      xk.y = 0.f;
      xm.y = 0.f;
    }
    const float2 A = cadd(xk, cconj(xm));
    const float2 B = csub(xk, cconj(xm));
    const float2 cB = cmul(cconj(twf[k]), B);
    lds[e] = make_float2(A.x - cB.y, A.y + cB.x);
  }
  __syncthreads();
  fft_lines<M, L, M, true>(lds, twh);
  float2* dst = out + line0 * M;
  for (int e = t; e < L * M; e += kThreads) dst[e] = lds[e];
}

// ------------------------------------------------------- strided x / y pass
// Tile: all N rows (the transform axis) x C consecutive kz columns.  Thread t
// owns column t % C and rows t / C + j * (NT / C), so its wave vector along z
// and along the batch axis is fixed and only the row index varies.
constexpr int kThreadsXY = 512;

template <int N, int AXIS, int NMID>
__global__ __launch_bounds__(kThreadsXY) void xy_pass_kernel(PassArgs a, const float2* __restrict__ twg) {
  constexpr int NT = kThreadsXY;
  constexpr int M = N / 2;
  constexpr int P = pitch_c<N>();
  constexpr int C = xycols<N>();
  constexpr int LS = N + 1;
  constexpr int RS = NT / C;          // rows per sweep
  constexpr int E = N / RS;           // elements per thread
  static_assert(NT % C == 0 && N % RS == 0, "tile shape");
  __shared__ float2 lds[C * LS];
  __shared__ float2 tw[N];
  const int t = threadIdx.x;
  const int c = t % C;
  const int r0 = t / C;
  const int c0 = blockIdx.x * C;
  const int b = blockIdx.y;
  const long long chain = blockIdx.z;
  const long long rstride = AXIS == 0 ? (long long)N * P : (long long)P;
  const bool valid = (c0 + c) <= M;
  const long long base = chain * a.chain_stride + (AXIS == 0 ? (long long)b * P : (long long)b * N * P) + c0 + c;
  for (int i = t; i < N; i += NT) tw[i] = twg[i];
  const int nb = freq_index(b, N);
  // masked columns (past N/2) take kz = 0 so that table lookups stay in range
  const int nz = valid ? c0 + c : 0;
  const int nyq = N / 2;
  float2* lcol = lds + c * LS;

  float2 mid[NMID][E];
#pragma unroll
  for (int m = 0; m < NMID; ++m)
#pragma unroll
    for (int j = 0; j < E; ++j) mid[m][j] = make_float2(0.f, 0.f);

  __syncthreads();
  for (int i = 0; i < a.nin; ++i) {
    const float2* src = a.in[i] + base;
    float2 val[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int r = r0 + j * RS;
      val[j] = valid ? src[r * rstride] : make_float2(0.f, 0.f);
    }
    if (a.in_fft & (1u << i)) {
#pragma unroll
      for (int j = 0; j < E; ++j) lcol[r0 + j * RS] = val[j];
      __syncthreads();
      fft_lines<N, C, LS, false, NT>(lds, tw);
#pragma unroll
      for (int j = 0; j < E; ++j) val[j] = lcol[r0 + j * RS];
      __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < NMID; ++m) {
      {
        const SpecOp op = a.A[m][i];
        if (op.re != 0.f || op.im != 0.f) {
#pragma unroll
          for (int j = 0; j < E; ++j) {
            KVec kv;
            const int nr = freq_index(r0 + j * RS, N);
            kv.n[0] = AXIS == 0 ? nr : 0;
            kv.n[1] = AXIS == 0 ? nb : nr;
            kv.n[2] = nz;
            kv.n2 = kv.n[0] * kv.n[0] + kv.n[1] * kv.n[1] + nz * nz;
            const float2 w = spec_eval<true>(op, kv, a.kf, nyq, a.tabs, a.tab_stride, a.rf);
            mid[m][j] = cadd(mid[m][j], cmul(w, val[j]));
          }
        }
      }
    }
  }

  for (int o = 0; o < a.nout; ++o) {
    float2 val[E];
#pragma unroll
    for (int j = 0; j < E; ++j) val[j] = make_float2(0.f, 0.f);
#pragma unroll
    for (int m = 0; m < NMID; ++m) {
      {
        const SpecOp op = a.B[o][m];
        if (op.re != 0.f || op.im != 0.f) {
#pragma unroll
          for (int j = 0; j < E; ++j) {
            KVec kv;
            const int nr = freq_index(r0 + j * RS, N);
            kv.n[0] = AXIS == 0 ? nr : 0;
            kv.n[1] = AXIS == 0 ? nb : nr;
            kv.n[2] = nz;
            kv.n2 = kv.n[0] * kv.n[0] + kv.n[1] * kv.n[1] + nz * nz;
            const float2 w = spec_eval<true>(op, kv, a.kf, nyq, a.tabs, a.tab_stride, a.rf);
            val[j] = cadd(val[j], cmul(w, mid[m][j]));
          }
        }
      }
    }
    if (a.out_fft & (1u << o)) {
#pragma unroll
      for (int j = 0; j < E; ++j) lcol[r0 + j * RS] = val[j];
      __syncthreads();
      fft_lines<N, C, LS, true, NT>(lds, tw);
#pragma unroll
      for (int j = 0; j < E; ++j) val[j] = lcol[r0 + j * RS];
      __syncthreads();
    }
    if (valid) {
      float2* dst = a.out[o] + base;
#pragma unroll
      for (int j = 0; j < E; ++j) dst[(r0 + j * RS) * rstride] = val[j];
    }
  }
}

// ============================================ register four-step variants
// The same passes with the transform done as N = N1 N2: each thread loads its
// N2 strided elements straight into registers, runs a length-N2 DFT there,
// one LDS exchange regroups the data, and a length-N1 DFT finishes it in
// registers (layout B).  The inverse starts from layout B, so a fused
// forward / mix / inverse pass touches LDS only twice.

template <int N>
__host__ __device__ constexpr int z4_lines() {
  return (kTile / (N / 2)) > N * N ? N * N : kTile / (N / 2);
}

// One z line of a four-step tile, thread j of its N1 threads.  Layout A of a
// length-M complex line: register q holds element j + N1 q, i.e. the packed
// reals 2 (j + N1 q) and 2 (j + N1 q) + 1 of the length-N real line.
//
// Half spectrum `row` (N/2 + 1 entries) -> packed reals v (layout A), through
// the real-packing identity and one inverse length-M transform.
template <int N>
__device__ __forceinline__ void z4_c2r_line(const float2* row, float2* v, float2* ll, int j, const float2* twh,
                                            const float2* twf) {
  constexpr int M = N / 2;
  constexpr int N1 = F4<M>::N1, N2 = F4<M>::N2, MU = N2 / N1;
#pragma unroll
  for (int u = 0; u < MU; ++u) {
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      const int k = N2 * k1 + j + N1 * u;
      float2 xk = row[k];
      float2 xm = row[M - k];
      if (k == 0) {
        xk.y = 0.f;
        xm.y = 0.f;
      }
      const float2 A = cadd(xk, cconj(xm));
      const float2 B = csub(xk, cconj(xm));
      const float2 cB = cmul(cconj(twf[k]), B);
      v[u * N1 + k1] = make_float2(A.x - cB.y, A.y + cB.x);
    }
  }
  inv_B_to_A<M>(v, ll, j, twh);
}

// Packed reals v (layout A) -> half spectrum `row` (N/2 + 1 entries).  Ends
// with a barrier, so `ll` may be reused at once.
template <int N>
__device__ __forceinline__ void z4_r2c_line(float2* v, float2* ll, int j, const float2* twh, const float2* twf,
                                            float2* row) {
  constexpr int M = N / 2;
  constexpr int N1 = F4<M>::N1, N2 = F4<M>::N2, MU = N2 / N1;
  fwd_A_to_B<M>(v, ll, j, twh);
  // natural order into LDS for the real-to-complex unpacking
#pragma unroll
  for (int u = 0; u < MU; ++u)
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) ll[N2 * k1 + j + N1 * u] = v[u * N1 + k1];
  __syncthreads();
  for (int k = j; k <= M; k += N1) {
    const float2 zk = ll[k == M ? 0 : k];
    const float2 zm = ll[k == 0 ? 0 : M - k];
    const float2 A = cadd(zk, cconj(zm));
    const float2 B = csub(zk, cconj(zm));
    const float2 wB = cmul(twf[k], B);
    row[k] = make_float2(0.5f * (A.x + wB.y), 0.5f * (A.y - wB.x));
  }
  __syncthreads();
}

template <int N>
__global__ __launch_bounds__(z4_lines<N>() * F4<N / 2>::N1) void zpass4_r2c_kernel(ZArgs a, const float2* __restrict__ tw_half,
                                                                               const float2* __restrict__ tw_full) {
  constexpr int M = N / 2;
  constexpr int N1 = F4<M>::N1, N2 = F4<M>::N2;
  constexpr int L = z4_lines<N>();
  constexpr int NT = L * N1;
  constexpr int LSZ = f4_lds<M>();
  constexpr int P = pitch_c<N>();
  __shared__ float2 lds[L * LSZ];
  __shared__ float2 twh[M];
  __shared__ float2 twf[N];
  const int t = threadIdx.x;
  const int j = t % N1, l = t / N1;
  const int arr = blockIdx.z % a.narr;
  const long long chain = blockIdx.z / a.narr;
  const float2* in = reinterpret_cast<const float2*>(a.in[arr]) + chain * (a.in_chain_stride / 2);
  float2* out = reinterpret_cast<float2*>(a.out[arr]) + chain * a.out_chain_stride;
  const long long line = (long long)blockIdx.x * L + l;
  for (int i = t; i < M; i += NT) twh[i] = tw_half[i];
  for (int i = t; i < N; i += NT) twf[i] = tw_full[i];
  float2 v[N2];
  const float2* src = in + line * M;
#pragma unroll
  for (int q = 0; q < N2; ++q) v[q] = src[j + N1 * q];
  __syncthreads();
  z4_r2c_line<N>(v, lds + l * LSZ, j, twh, twf, out + line * P);
}

template <int N>
__global__ __launch_bounds__(z4_lines<N>() * F4<N / 2>::N1) void zpass4_c2r_kernel(ZArgs a, const float2* __restrict__ tw_half,
                                                                               const float2* __restrict__ tw_full) {
  constexpr int M = N / 2;
  constexpr int N1 = F4<M>::N1, N2 = F4<M>::N2;
  constexpr int L = z4_lines<N>();
  constexpr int NT = L * N1;
  constexpr int LSZ = f4_lds<M>();
  constexpr int P = pitch_c<N>();
  __shared__ float2 lds[L * LSZ];
  __shared__ float2 twh[M];
  __shared__ float2 twf[N];
  const int t = threadIdx.x;
  const int j = t % N1, l = t / N1;
  const int arr = blockIdx.z % a.narr;
  const long long chain = blockIdx.z / a.narr;
  const float2* in = reinterpret_cast<const float2*>(a.in[arr]) + chain * a.in_chain_stride;
  float2* out = reinterpret_cast<float2*>(a.out[arr]) + chain * (a.out_chain_stride / 2);
  const long long line = (long long)blockIdx.x * L + l;
  for (int i = t; i < M; i += NT) twh[i] = tw_half[i];
  for (int i = t; i < N; i += NT) twf[i] = tw_full[i];
  __syncthreads();
  float2 v[N2];
  z4_c2r_line<N>(in + line * P, v, lds + l * LSZ, j, twh, twf);
  float2* dst = out + line * M;
#pragma unroll
  for (int q = 0; q < N2; ++q) dst[j + N1 * q] = v[q];
}

// ------------------------------------------ z transforms fused with the LPT
// Forward: the six Hessian spectra phi_ij of a z line are brought to real
// space (and stored: the adjoint needs them) while S2 = sum_{i<j} (phi_ii
// phi_jj - phi_ij^2) and delta_L = tr phi accumulate in registers; then
// S2 and d_SC = 3 (sqrt(hinge(1 - 2 D1 delta_L / 3)) - 1) are transformed back
// from the same registers (the inverse leaves them in the layout the forward
// transform starts from).  Neither S2 nor d_SC ever exists in real space in
// memory.  Order of the components: xx, yy, zz, xy, xz, yz.
template <int N>
__global__ __launch_bounds__(z4_lines<N>() * F4<N / 2>::N1) void lpt_fwd_z4_kernel(LptZArgs a, const float2* __restrict__ tw_half,
                                                                               const float2* __restrict__ tw_full) {
  constexpr int M = N / 2;
  constexpr int N1 = F4<M>::N1, N2 = F4<M>::N2;
  constexpr int L = z4_lines<N>();
  constexpr int NT = L * N1;
  constexpr int LSZ = f4_lds<M>();
  constexpr int P = pitch_c<N>();
  __shared__ float2 lds[L * LSZ];
  __shared__ float2 twh[M];
  __shared__ float2 twf[N];
  const int t = threadIdx.x;
  const int j = t % N1, l = t / N1;
  const long long chain = blockIdx.z;
  const long long line = (long long)blockIdx.x * L + l;
  const long long soff = chain * a.spec_chain_stride + line * P;
  const long long roff = chain * (a.field_chain_stride / 2) + line * M;
  float2* ll = lds + l * LSZ;
  for (int i = t; i < M; i += NT) twh[i] = tw_half[i];
  for (int i = t; i < N; i += NT) twf[i] = tw_full[i];
  __syncthreads();
  // a.field[0] null: phi is not stored (checkpointed plans recompute it in
  // the adjoint); a.sout[0] null: phi only, no S2 and d_SC (that recompute).
  // Both are kernel arguments, so the branches are uniform and the phi values
  // come from the same instructions either way.
  const bool store = a.field[0] != nullptr;
  const bool lpt = a.sout[0] != nullptr;
  float2 S[N2], D[N2], v[N2];
  for (int c = 0; c < 6; ++c) {
    z4_c2r_line<N>(a.sin[c] + soff, v, ll, j, twh, twf);
    if (store) {
      float2* dst = reinterpret_cast<float2*>(a.field[c]) + roff;
#pragma unroll
      for (int q = 0; q < N2; ++q) dst[j + N1 * q] = v[q];
    }
    if (!lpt) continue;
    if (c == 0) {
#pragma unroll
      for (int q = 0; q < N2; ++q) D[q] = v[q];
    } else if (c == 1) {
#pragma unroll
      for (int q = 0; q < N2; ++q) {
        S[q] = make_float2(D[q].x * v[q].x, D[q].y * v[q].y);
        D[q] = cadd(D[q], v[q]);
      }
    } else if (c == 2) {
#pragma unroll
      for (int q = 0; q < N2; ++q) {
        S[q] = make_float2(S[q].x + D[q].x * v[q].x, S[q].y + D[q].y * v[q].y);
        D[q] = cadd(D[q], v[q]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < N2; ++q) S[q] = make_float2(S[q].x - v[q].x * v[q].x, S[q].y - v[q].y * v[q].y);
    }
  }
  if (!lpt) return;
  z4_r2c_line<N>(S, ll, j, twh, twf, a.sout[0] + soff);
  const float k = (2.f / 3.f) * a.d1;
#pragma unroll
  for (int q = 0; q < N2; ++q) {
    float hv, hd;
    sc_hinge(1.f - k * D[q].x, a.tau, hv, hd);
    v[q].x = 3.f * (sqrtf(hv) - 1.f);
    sc_hinge(1.f - k * D[q].y, a.tau, hv, hd);
    v[q].y = 3.f * (sqrtf(hv) - 1.f);
  }
  z4_r2c_line<N>(v, ll, j, twh, twf, a.sout[1] + soff);
}

// Adjoint: the cotangent spectra of S2 and d_SC come to real space, the
// stored phi give delta_L and the hinge derivative, and each phi_ij cotangent
// is formed in registers and transformed straight to its spectrum:
// d phi_ii = dS2 (delta_L - phi_ii) + d delta_L, d phi_ij = -2 dS2 phi_ij.
template <int N>
__global__ __launch_bounds__(z4_lines<N>() * F4<N / 2>::N1) void lpt_bwd_z4_kernel(LptZArgs a, const float2* __restrict__ tw_half,
                                                                               const float2* __restrict__ tw_full) {
  constexpr int M = N / 2;
  constexpr int N1 = F4<M>::N1, N2 = F4<M>::N2;
  constexpr int L = z4_lines<N>();
  constexpr int NT = L * N1;
  constexpr int LSZ = f4_lds<M>();
  constexpr int P = pitch_c<N>();
  __shared__ float2 lds[L * LSZ];
  __shared__ float2 twh[M];
  __shared__ float2 twf[N];
  const int t = threadIdx.x;
  const int j = t % N1, l = t / N1;
  const long long chain = blockIdx.z;
  const long long line = (long long)blockIdx.x * L + l;
  const long long soff = chain * a.spec_chain_stride + line * P;
  const long long roff = chain * (a.field_chain_stride / 2) + line * M;
  float2* ll = lds + l * LSZ;
  for (int i = t; i < M; i += NT) twh[i] = tw_half[i];
  for (int i = t; i < N; i += NT) twf[i] = tw_full[i];
  __syncthreads();
  float2 G2[N2], GD[N2], D[N2], v[N2];
  z4_c2r_line<N>(a.sin[0] + soff, G2, ll, j, twh, twf);
  z4_c2r_line<N>(a.sin[1] + soff, GD, ll, j, twh, twf);
  auto phi = [&](int c) { return reinterpret_cast<const float2*>(a.field[c]) + roff; };
#pragma unroll
  for (int q = 0; q < N2; ++q) D[q] = cadd(cadd(phi(0)[j + N1 * q], phi(1)[j + N1 * q]), phi(2)[j + N1 * q]);
  const float k = (2.f / 3.f) * a.d1;
#pragma unroll
  for (int q = 0; q < N2; ++q) {
    float hv, hd;
    sc_hinge(1.f - k * D[q].x, a.tau, hv, hd);
    GD[q].x = hv > 0.f ? -GD[q].x * a.d1 * hd * rsqrtf(hv) : 0.f;
    sc_hinge(1.f - k * D[q].y, a.tau, hv, hd);
    GD[q].y = hv > 0.f ? -GD[q].y * a.d1 * hd * rsqrtf(hv) : 0.f;
  }
  for (int c = 0; c < 6; ++c) {
    const float2* src = phi(c);
#pragma unroll
    for (int q = 0; q < N2; ++q) {
      const float2 x = src[j + N1 * q];
      v[q] = c < 3 ? make_float2(G2[q].x * (D[q].x - x.x) + GD[q].x, G2[q].y * (D[q].y - x.y) + GD[q].y)
                   : make_float2(-2.f * G2[q].x * x.x, -2.f * G2[q].y * x.y);
    }
    z4_r2c_line<N>(v, ll, j, twh, twf, a.sout[c] + soff);
  }
}

// Strided x / y pass, four-step variant.  Tile: C columns x N rows; thread t
// owns column t % C and four-step index j = t / C.
template <int N>
__host__ __device__ constexpr int xy4_cols() {
  return N == 96 ? 16 : (kTile / N > 256 ? 256 : kTile / N);
}

// Split of the mixing pass's transform into S sub-lines: a line of N is
// transformed as its S decimated sub-sequences (samples S p + g), S four-step
// transforms of N/S on S groups of threads, joined by one radix-S butterfly
// across the groups (through LDS).  N = 512 (S = 2): a thread holds 16
// elements instead of 32, which keeps the pass at the register budget of
// three workgroups per CU (a 512 four-step in one group needs 256 VGPRs and
// runs one wave per SIMD).  N = 96 (S = 3): three 32-point four-step
// transforms, where 96 has no register four-step of its own.
template <int N>
__host__ __device__ constexpr int xy4_split() {
  return N >= 512 ? 2 : (N == 96 ? 3 : 1);
}
template <int N>
__host__ __device__ constexpr int xy4_threads() {
  return xy4_cols<N>() * xy4_split<N>() * F4<N / xy4_split<N>()>::N1;
}

// Used for single-mix passes (NMID = 1), where three workgroups per CU fit in
// registers without spilling; multi-mix passes use the Stockham kernel.
//
// With a split into S sub-lines, thread (g, j) of a column holds in layout A
// the rows S (j + N1 q) + g (sub-line g), and in layout B the frequencies
// (N/S) g + N2 k1 + j + N1 u; the sub-transforms use the N/S-point twiddles
// (every S-th entry of the N table).
template <int N, int AXIS, int NMID, bool PF>
__global__ __launch_bounds__(xy4_threads<N>(), 3) void xy4_pass_kernel(PassArgs a, const float2* __restrict__ twg) {
  constexpr int S = xy4_split<N>();
  constexpr int NS = N / S;                     // length of a sub-line
  constexpr int N1 = F4<NS>::N1, N2 = F4<NS>::N2;
  constexpr int M = N / 2;
  constexpr int P = pitch_c<N>();
  constexpr int C = xy4_cols<N>();
  constexpr int NT = xy4_threads<N>();
  constexpr int LSZ = f4_lds<NS>() + 1;
  static_assert(S == 1 || S * LSZ >= S * N1 * N2, "a column's LDS holds the butterfly exchange");
  constexpr long long RS = AXIS == 0 ? (long long)N * P : (long long)P;   // row stride (elements)
  constexpr int ROWB = (int)(RS * 8);                                     // row stride (bytes)
  constexpr int RANGE = (int)(((N - 1) * RS + C) * 8);                   // bytes one workgroup spans
  __shared__ float2 lds[C * S * LSZ];
  __shared__ float2 tw[N];
  __shared__ float2 tws[S == 1 ? 1 : NS];       // sub-line twiddles (split only)
  const int t = threadIdx.x;
  const int c = t % C, r = t / C;
  const int g = r / N1, j = r % N1;             // sub-line and four-step index
  // Where a workgroup's C columns cover half of each 128-byte line it reads
  // (C = 8 at N = 512), the workgroup that reads the other halves runs on the
  // same XCD right after it: dispatch goes round-robin over the 8 XCDs by
  // linear workgroup id, so the workgroups 8 ids apart are paired.
  unsigned bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  if constexpr (C * 8 < 128) {
    const unsigned gx = gridDim.x, gy = gridDim.y;
    unsigned lin = bx + gx * (by + gy * bz);
    if (((gx * gy * gridDim.z) & 15u) == 0u) lin = (lin & ~15u) | ((lin & 7u) << 1) | ((lin >> 3) & 1u);
    bx = lin % gx;
    by = (lin / gx) % gy;
    bz = lin / (gx * gy);
  }
  const int c0 = (int)bx * C;
  const int b = (int)by;
  const long long chain = bz;
  const bool valid = (c0 + c) <= M;
  const long long base = chain * a.chain_stride + (AXIS == 0 ? (long long)b * P : (long long)b * N * P) + c0;
  // lane part of every offset; the row part (a compile-time constant per
  // element) goes in the scalar offset.  Layout A rows S (j + N1 q) + g,
  // layout B rows NS g + N2 (e % N1) + j + N1 (e / N1).
  const int voff = valid ? (int)(((S * j + g) * RS + c) * 8) : kBufOff;
  const int voffB = valid ? (int)(((NS * g + j) * RS + c) * 8) : kBufOff;
  for (int i = t; i < N; i += NT) tw[i] = twg[i];
  if constexpr (S > 1)
    for (int i = t; i < NS; i += NT) tws[i] = twg[S * i];
  const float2* twsub = S == 1 ? tw : tws;
  const int nb = freq_index(b, N);
  const int nz = valid ? c0 + c : 0;
  const int nyq = N / 2;
  float2* lcol = lds + (c * S + g) * LSZ;
  auto rowB = [&](int e) { return NS * g + N2 * (e % N1) + j + N1 * (e / N1); };
  auto rowB_off = [&](int e) { return (N2 * (e % N1) + N1 * (e / N1)) * ROWB; };
  // radix-S butterfly across the S sub-lines of a column (split only), in
  // place on the layout B registers (w = exp(-2 pi i / N), k < N/S).  Forward:
  // from the sub-transforms Y_h, group g forms X[k + (N/S) g] = sum_h
  // w^(h k + (N/S) h g) Y_h[k].  Inverse: from X_m[k] = X[k + (N/S) m], held
  // by group m, it forms Z_g[k] = sum_m conj(w^(g k + (N/S) g m)) X_m[k],
  // whose N/S-point inverse is sub-line g.  Synchronises; all threads must
  // call it.
  auto butterfly = [&](float2* v, bool inverse) {
    float2* xc = lds + c * S * LSZ;
#pragma unroll
    for (int e = 0; e < N2; ++e) xc[e * S * N1 + g * N1 + j] = v[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < N2; ++e) {
      const int k = rowB(e) - NS * g;
      if constexpr (S == 2) {
        // X[k] = Y_0 + w^k Y_1, X[k + N/2] = Y_0 - w^k Y_1; Z_0 = X_0 + X_1,
        // Z_1 = conj(w^k) (X_0 - X_1)
        const float2 o = xc[e * 2 * N1 + (1 - g) * N1 + j];
        const float2 x0 = g == 0 ? v[e] : o, x1 = g == 0 ? o : v[e];
        const float2 w = tw[k];
        if (!inverse) {
          const float2 pr = cmul(w, x1);
          v[e] = g == 0 ? cadd(x0, pr) : csub(x0, pr);
        } else {
          v[e] = g == 0 ? cadd(x0, x1) : cmul(cconj(w), csub(x0, x1));
        }
      } else {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int h = 0; h < S; ++h) {
          const float2 y = xc[e * S * N1 + h * N1 + j];
          const int q = inverse ? g * k + NS * ((g * h) % S) : h * k + NS * ((h * g) % S);
          const float2 w = tw[q % N];
          acc = cadd(acc, cmul(inverse ? cconj(w) : w, y));
        }
        v[e] = acc;
        // one element at a time: hoisting every exchange read spills
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();
  };

  float2 mid[NMID][N2];
#pragma unroll
  for (int m = 0; m < NMID; ++m)
#pragma unroll
    for (int e = 0; e < N2; ++e) mid[m][e] = make_float2(0.f, 0.f);
  __syncthreads();

  // input i in registers: layout A rows when it is transformed here, else B
  auto load_input = [&](int i, float2* dst) {
    const BufRsrc src = buf_rsrc(a.in[i] + base, RANGE);
    if (a.in_fft & (1u << i)) {
#pragma unroll
      for (int q = 0; q < N2; ++q) dst[q] = buf_load2(src, voff, S * N1 * q * ROWB);
    } else {
#pragma unroll
      for (int e = 0; e < N2; ++e) dst[e] = buf_load2(src, voffB, rowB_off(e));
    }
  };
  // with several inputs, the loads of input i+1 are in flight during the
  // transform of input i (the single-input variant has no prefetch registers
  // and evaluates the radial multipliers in closed form)
  float2 nxt[PF ? N2 : 1];
  const bool pf = PF && a.nin > 1;
  if constexpr (PF) {
    if (pf) load_input(0, nxt);
  }
  for (int i = 0; i < a.nin; ++i) {
    float2 val[N2];
    if constexpr (PF) {
      if (pf) {
#pragma unroll
        for (int e = 0; e < N2; ++e) val[e] = nxt[e];
        if (i + 1 < a.nin) load_input(i + 1, nxt);
      } else {
        load_input(i, val);
      }
    } else {
      load_input(i, val);
    }
    if (a.in_fft & (1u << i)) {
      fwd_A_to_B<NS>(val, lcol, j, twsub);
      if constexpr (S > 1) butterfly(val, false);
    }
#pragma unroll
    for (int m = 0; m < NMID; ++m) {
      const SpecOp op = a.A[m][i];
      if (op.re == 0.f && op.im == 0.f) continue;
      if (spec_is_const(op)) {
        const float2 k = make_float2(op.re, op.im);
#pragma unroll
        for (int e = 0; e < N2; ++e) mid[m][e] = cadd(mid[m][e], cmul(k, val[e]));
        continue;
      }
#pragma unroll
      for (int e = 0; e < N2; ++e) {
        KVec kv;
        const int nr = freq_index(rowB(e), N);
        kv.n[0] = AXIS == 0 ? nr : 0;
        kv.n[1] = AXIS == 0 ? nb : nr;
        kv.n[2] = nz;
        kv.n2 = kv.n[0] * kv.n[0] + kv.n[1] * kv.n[1] + nz * nz;
        mid[m][e] = cadd(mid[m][e], cmul(spec_eval<!PF>(op, kv, a.kf, nyq, a.tabs, a.tab_stride, a.rf), val[e]));
      }
    }
  }

  for (int o = 0; o < a.nout; ++o) {
    float2 val[N2];
    bool have = false;
#pragma unroll
    for (int m = 0; m < NMID; ++m) {
      const SpecOp op = a.B[o][m];
      if (op.re == 0.f && op.im == 0.f) continue;
      if (spec_is_const(op)) {
        const float2 k = make_float2(op.re, op.im);
        if (!have) {
#pragma unroll
          for (int e = 0; e < N2; ++e) val[e] = (op.re == 1.f && op.im == 0.f) ? mid[m][e] : cmul(k, mid[m][e]);
        } else {
#pragma unroll
          for (int e = 0; e < N2; ++e) val[e] = cadd(val[e], cmul(k, mid[m][e]));
        }
        have = true;
        continue;
      }
      if (!have) {
#pragma unroll
        for (int e = 0; e < N2; ++e) val[e] = make_float2(0.f, 0.f);
        have = true;
      }
#pragma unroll
      for (int e = 0; e < N2; ++e) {
        KVec kv;
        const int nr = freq_index(rowB(e), N);
        kv.n[0] = AXIS == 0 ? nr : 0;
        kv.n[1] = AXIS == 0 ? nb : nr;
        kv.n[2] = nz;
        kv.n2 = kv.n[0] * kv.n[0] + kv.n[1] * kv.n[1] + nz * nz;
        val[e] = cadd(val[e], cmul(spec_eval<!PF>(op, kv, a.kf, nyq, a.tabs, a.tab_stride, a.rf), mid[m][e]));
      }
    }
    if (!have) {
#pragma unroll
      for (int e = 0; e < N2; ++e) val[e] = make_float2(0.f, 0.f);
    }
    const BufRsrc dst = buf_rsrc(a.out[o] + base, RANGE);
    if (a.out_fft & (1u << o)) {
      if constexpr (S > 1) butterfly(val, true);
      inv_B_to_A<NS>(val, lcol, j, twsub);
#pragma unroll
      for (int q = 0; q < N2; ++q) buf_store2(dst, voff, S * N1 * q * ROWB, val[q]);
    } else {
#pragma unroll
      for (int e = 0; e < N2; ++e) buf_store2(dst, voffB, rowB_off(e), val[e]);
    }
  }
}

// Pure strided transforms (no multiplier, one output per input, possibly in
// place): the passes that only carry an array along one axis.  Persistent:
// the grid is sized so that every workgroup walks the same number of column
// groups (group = array, chain, fixed index of the other transverse axis,
// column block), and the loads of the next group are issued before the
// transform of the current one, so each workgroup keeps memory busy while it
// computes.  Registers: the current and the prefetched column (2 x N2
// complex) plus the transform.
template <int N, int AXIS, bool INV>
__global__ __launch_bounds__(xy4_cols<N>() * F4<N>::N1) void xy4_pure_kernel(PureArgs a, const float2* __restrict__ twg,
                                                                           int ngroups) {
  constexpr int N1 = F4<N>::N1, N2 = F4<N>::N2;
  constexpr int M = N / 2;
  constexpr int P = pitch_c<N>();
  constexpr int C = xy4_cols<N>();
  constexpr int NT = C * N1;
  constexpr int NCG = (M + 1 + C - 1) / C;
  constexpr int LSZ = f4_lds<N>() + 1;
  constexpr long long RS = AXIS == 0 ? (long long)N * P : (long long)P;
  constexpr int ROWB = (int)(RS * 8);
  constexpr int RANGE = (int)(((N - 1) * RS + C) * 8);
  __shared__ float2 lds[C * LSZ];
  __shared__ float2 tw[N];
  const int t = threadIdx.x;
  const int c = t % C, j = t / C;
  for (int i = t; i < N; i += NT) tw[i] = twg[i];
  float2* lcol = lds + c * LSZ;
  const int lane_off = (int)((j * RS + c) * 8);
  // the input is in layout A for a forward transform, B for an inverse; the
  // output in the other one
  auto in_off = [&](int e) { return INV ? (N2 * (e % N1) + N1 * (e / N1)) * ROWB : N1 * e * ROWB; };
  auto out_off = [&](int e) { return INV ? N1 * e * ROWB : (N2 * (e % N1) + N1 * (e / N1)) * ROWB; };
  struct Where {
    long long base;
    int arr;
    bool valid;
  };
  auto where = [&](int g) {
    const int cg = g % NCG;
    const int b = (g / NCG) % N;
    const int ac = g / (NCG * N);
    const int arr = ac / a.chains;
    const long long chain = ac % a.chains;
    Where w;
    w.base = chain * a.chain_stride + (AXIS == 0 ? (long long)b * P : (long long)b * N * P) + cg * C;
    w.arr = arr;
    w.valid = cg * C + c <= M;
    return w;
  };
  auto load = [&](int g, float2* dst) {
    const Where w = where(g);
    const BufRsrc r = buf_rsrc(a.in[w.arr] + w.base, RANGE);
    const int voff = w.valid ? lane_off : kBufOff;
#pragma unroll
    for (int e = 0; e < N2; ++e) dst[e] = buf_load2(r, voff, in_off(e));
  };

  int g = blockIdx.x;
  float2 nxt[N2];
  if (g < ngroups) load(g, nxt);
  __syncthreads();
  for (; g < ngroups; g += gridDim.x) {
    float2 v[N2];
#pragma unroll
    for (int e = 0; e < N2; ++e) v[e] = nxt[e];
    const int gn = g + gridDim.x;
    if (gn < ngroups) load(gn, nxt);
    if (INV) inv_B_to_A<N>(v, lcol, j, tw);
    else fwd_A_to_B<N>(v, lcol, j, tw);
    const Where w = where(g);
    const BufRsrc r = buf_rsrc(a.out[w.arr] + w.base, RANGE);
    const int voff = w.valid ? lane_off : kBufOff;
#pragma unroll
    for (int e = 0; e < N2; ++e) buf_store2(r, voff, out_off(e), v[e]);
  }
}

// ------------------------------------------------------------- launchers
// Kernel family per mesh size (process-wide; chosen by the plan's tuner).
FftSchedule& fft_schedule(int n) {
  static FftSchedule table[8];
  switch (n) {
    case 16: return table[0];
    case 32: return table[1];
    case 64: return table[2];
    case 96: return table[3];
    case 128: return table[4];
    case 256: return table[5];
    default: return table[6];
  }
}

template <int N>
static void zr2c(const ZArgs& za, long long chains, const float2* twh, const float2* twf, hipStream_t s) {
  if constexpr (N != 96) {
    if (fft_schedule(N).z == kSchedFourStep) {
      constexpr int L = z4_lines<N>();
      dim3 grid((N * N) / L, 1, (unsigned)(za.narr * chains));
      hipLaunchKernelGGL(zpass4_r2c_kernel<N>, grid, dim3(L * F4<N / 2>::N1), 0, s, za, twh, twf);
      return;
    }
  }
  {
    constexpr int L = zlines<N>();
    dim3 grid((N * N) / L, 1, (unsigned)(za.narr * chains));
    hipLaunchKernelGGL(zpass_r2c_kernel<N>, grid, dim3(kThreads), 0, s, za, twh, twf);
  }
}
template <int N>
static void zc2r(const ZArgs& za, long long chains, const float2* twh, const float2* twf, hipStream_t s) {
  if constexpr (N != 96) {
    if (fft_schedule(N).z == kSchedFourStep) {
      constexpr int L = z4_lines<N>();
      dim3 grid((N * N) / L, 1, (unsigned)(za.narr * chains));
      hipLaunchKernelGGL(zpass4_c2r_kernel<N>, grid, dim3(L * F4<N / 2>::N1), 0, s, za, twh, twf);
      return;
    }
  }
  {
    constexpr int L = zlines<N>();
    dim3 grid((N * N) / L, 1, (unsigned)(za.narr * chains));
    hipLaunchKernelGGL(zpass_c2r_kernel<N>, grid, dim3(kThreads), 0, s, za, twh, twf);
  }
}

#define FZW_DISPATCH_N(n, F, ...)                 \
  switch (n) {                                    \
    case 16: F<16>(__VA_ARGS__); break;           \
    case 32: F<32>(__VA_ARGS__); break;           \
    case 64: F<64>(__VA_ARGS__); break;           \
    case 96: F<96>(__VA_ARGS__); break;           \
    case 128: F<128>(__VA_ARGS__); break;         \
    case 256: F<256>(__VA_ARGS__); break;         \
    case 512: F<512>(__VA_ARGS__); break;         \
    default: break;                               \
  }

void launch_zpass_r2c(int n, const float* const* in, float2* const* out, int narr, long long chains,
                      long long in_chain_stride, long long out_chain_stride, const float2* tw_half,
                      const float2* tw_full, hipStream_t s) {
  ZArgs za{};
  for (int i = 0; i < narr; ++i) {
    za.in[i] = in[i];
    za.out[i] = out[i];
  }
  za.narr = narr;
  za.in_chain_stride = in_chain_stride;
  za.out_chain_stride = out_chain_stride;
  FZW_DISPATCH_N(n, zr2c, za, chains, tw_half, tw_full, s);
}

void launch_zpass_c2r(int n, const float2* const* in, float* const* out, int narr, long long chains,
                      long long in_chain_stride, long long out_chain_stride, const float2* tw_half,
                      const float2* tw_full, hipStream_t s) {
  ZArgs za{};
  for (int i = 0; i < narr; ++i) {
    za.in[i] = in[i];
    za.out[i] = out[i];
  }
  za.narr = narr;
  za.in_chain_stride = in_chain_stride;
  za.out_chain_stride = out_chain_stride;
  FZW_DISPATCH_N(n, zc2r, za, chains, tw_half, tw_full, s);
}

template <int N>
static void lpt_z(bool fwd, const LptZArgs& a, int chains, const float2* twh, const float2* twf, hipStream_t s,
                  bool& done) {
  if constexpr (N != 96) {
    constexpr int L = z4_lines<N>();
    dim3 grid((N * N) / L, 1, (unsigned)chains);
    dim3 block(L * F4<N / 2>::N1);
    if (fwd) hipLaunchKernelGGL(lpt_fwd_z4_kernel<N>, grid, block, 0, s, a, twh, twf);
    else hipLaunchKernelGGL(lpt_bwd_z4_kernel<N>, grid, block, 0, s, a, twh, twf);
    done = true;
  }
}

bool has_four_step_z(int n) { return n != 96; }

bool launch_lpt_z(int n, bool fwd, const LptZArgs& a, int chains, const float2* tw_half, const float2* tw_full,
                  hipStream_t s) {
  bool done = false;
  FZW_DISPATCH_N(n, lpt_z, fwd, a, chains, tw_half, tw_full, s, done);
  return done;
}

// Workgroups of kernel `k` that fit on the device at once.
static int resident_blocks(const void* k, int block) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, 0) != hipSuccess || cus <= 0 || per_cu <= 0) {
    (void)hipGetLastError();
    return 0;
  }
  return cus * per_cu;
}

template <int N, int AX, bool INV>
static int& pure_capacity() {
  static int cap = 0;
  return cap;
}

template <int N, int AX, bool INV>
static void pure_prime() {
  int& cap = pure_capacity<N, AX, INV>();
  if (cap == 0) {
    cap = resident_blocks(reinterpret_cast<const void*>(&xy4_pure_kernel<N, AX, INV>), xy4_cols<N>() * F4<N>::N1);
    if (cap <= 0) cap = 1024;   // a safe default: the kernel walks any number of groups
  }
}

template <int N>
static void pure4(int axis, bool inv, const PureArgs& a, const float2* tw, hipStream_t s, bool& done) {
  if constexpr (N != 96) {
    constexpr int block = xy4_cols<N>() * F4<N>::N1;
    constexpr int NCG = (N / 2 + 1 + xy4_cols<N>() - 1) / xy4_cols<N>();
    const int ngroups = NCG * N * a.chains * a.narr;
    auto go = [&](auto kern, int cap) {
      const int per = (ngroups + cap - 1) / cap;   // equal work per workgroup
      hipLaunchKernelGGL(kern, dim3((ngroups + per - 1) / per), dim3(block), 0, s, a, tw, ngroups);
    };
#define FZW_PURE(AX, INV)                                            \
  do {                                                              \
    pure_prime<N, AX, INV>();                                       \
    go(xy4_pure_kernel<N, AX, INV>, pure_capacity<N, AX, INV>());   \
  } while (0)
    if (axis == 0) {
      if (inv) FZW_PURE(0, true);
      else FZW_PURE(0, false);
    } else {
      if (inv) FZW_PURE(1, true);
      else FZW_PURE(1, false);
    }
#undef FZW_PURE
    done = true;
  }
}

template <int N>
static void pure_prime_all() {
  if constexpr (N != 96) {
    pure_prime<N, 0, false>();
    pure_prime<N, 0, true>();
    pure_prime<N, 1, false>();
    pure_prime<N, 1, true>();
  }
}

bool has_pure_pass(int n) { return n != 96; }

bool launch_pure_pass(int n, int axis, bool inverse, const PureArgs& a, const float2* tw, hipStream_t s) {
  if (fft_schedule(n).pure != kSchedFourStep) return false;
  bool done = false;
  FZW_DISPATCH_N(n, pure4, axis, inverse, a, tw, s, done);
  return done;
}

void prime_launch_config(int n) { FZW_DISPATCH_N(n, pure_prime_all); }

template <int N>
static void xyp4(int axis, const PassArgs& a, int chains, const float2* tw, hipStream_t s) {
  constexpr int C = xy4_cols<N>();
  dim3 grid((N / 2 + 1 + C - 1) / C, N, chains);
  dim3 block(xy4_threads<N>());
  const bool pf = a.nin > 1;
  if (axis == 0) {
    if (pf) hipLaunchKernelGGL((xy4_pass_kernel<N, 0, 1, true>), grid, block, 0, s, a, tw);
    else hipLaunchKernelGGL((xy4_pass_kernel<N, 0, 1, false>), grid, block, 0, s, a, tw);
  } else {
    if (pf) hipLaunchKernelGGL((xy4_pass_kernel<N, 1, 1, true>), grid, block, 0, s, a, tw);
    else hipLaunchKernelGGL((xy4_pass_kernel<N, 1, 1, false>), grid, block, 0, s, a, tw);
  }
}

template <int N>
static void xyp(int axis, const PassArgs& a, int chains, const float2* tw, hipStream_t s) {
  if (a.nmid == 1 && fft_schedule(N).xy == kSchedFourStep) {
    xyp4<N>(axis, a, chains, tw, s);
    return;
  }
  constexpr int C = xycols<N>();
  dim3 grid((N / 2 + 1 + C - 1) / C, N, chains);
#define FZW_XY(AX, NM) hipLaunchKernelGGL((xy_pass_kernel<N, AX, NM>), grid, dim3(kThreadsXY), 0, s, a, tw)
  if (axis == 0) {
    if (a.nmid == 1) FZW_XY(0, 1);
    else if (a.nmid == 2) FZW_XY(0, 2);
    else FZW_XY(0, 3);
  } else {
    if (a.nmid == 1) FZW_XY(1, 1);
    else if (a.nmid == 2) FZW_XY(1, 2);
    else FZW_XY(1, 3);
  }
#undef FZW_XY
}

void launch_xy_pass(int n, int axis, const PassArgs& a, int chains, const float2* tw, hipStream_t s) {
  FZW_DISPATCH_N(n, xyp, axis, a, chains, tw, s);
}

}  // namespace fzw
