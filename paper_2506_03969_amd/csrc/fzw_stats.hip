// Validation statistics of reconstructed fields (Section 4): binned power
// spectrum multipoles of a half spectrum (auto or cross), shell filters for
// the FFT bispectrum estimator, and FP64 sums of triple products.
//
// Every reduction is deterministic: a wave sums its lanes' contributions to
// each bin it touches with register shuffles, each wave keeps its own LDS
// accumulator row, the rows of a workgroup are added in wave order, and the
// workgroups' partials are added in block order by a second kernel.  Bin and
// shell decisions use the same FP64 arithmetic, in the same order, as the
// plain definition (|k| = sqrt(kx^2 + ky^2 + kz^2) with k_a = kf n_a, then
// floor((|k| - k_lo) / dk)); contraction into fma is off there.
#include <mutex>

#include "fzw_device.hpp"
#include "fzw_ops.hpp"

namespace fzw {

namespace {

constexpr int kST = 256;            // threads per workgroup
constexpr int kSW = kST / 64;       // waves per workgroup

__device__ __forceinline__ double mode_k(int x, int y, int z, int n, double kf) {
#pragma clang fp contract(off)
  const int nx = x <= n / 2 ? x : x - n, ny = y <= n / 2 ? y : y - n;
  const double kx = kf * nx, ky = kf * ny, kz = kf * z;
  return sqrt(kx * kx + ky * ky + kz * kz);
}

__device__ __forceinline__ int mode_bin(double k, double k_lo, double dk, int nbins) {
#pragma clang fp contract(off)
  if (!(k > 0.0)) return -1;
  const double t = floor((k - k_lo) / dk);
  return (t >= 0.0 && t < (double)nbins) ? (int)t : -1;
}

// acc[wave][bin][4] += (w, w k, w P, w P L2(mu)) over the half spectrum; one
// partial row [nbins][4] per workgroup.
__global__ void __launch_bounds__(kST) multipole_kernel(const float2* __restrict__ a, const float2* __restrict__ b,
                                                        int n, int pitch, double kf, double k_lo, double dk,
                                                        int nbins, double pnorm, double* __restrict__ partial) {
  extern __shared__ double acc[];   // [kSW][nbins][4]
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < kSW * nbins * 4; i += kST) acc[i] = 0.0;
  __syncthreads();
  double* mine = acc + (size_t)wid * nbins * 4;
  const int m1 = n / 2 + 1;
  const long long total = (long long)n * n * m1;
  const long long stride = (long long)gridDim.x * kST;
  // every wave runs the same number of iterations (wave-uniform loop)
  const long long base0 = (long long)blockIdx.x * kST + wid * 64;
  for (long long base = base0; base < total; base += stride) {
    const long long i = base + lane;
    int bin = -1;
    double w = 0.0, k = 0.0, p = 0.0, pl = 0.0;
    if (i < total) {
      const long long r = i / m1;
      const int z = (int)(i - r * m1);
      const int x = (int)(r / n), y = (int)(r - (long long)x * n);
      k = mode_k(x, y, z, n, kf);
      bin = mode_bin(k, k_lo, dk, nbins);
      if (bin >= 0) {
        w = (z > 0 && 2 * z < n) ? 2.0 : 1.0;
        const float2 va = a[r * pitch + z];
        const float2 vb = b[r * pitch + z];
        p = pnorm * ((double)va.x * vb.x + (double)va.y * vb.y);
        const double mu = (kf * z) / k;
        pl = p * 0.5 * (3.0 * mu * mu - 1.0);
      }
    }
    // bins of this wave: loop from the smallest to the largest
    int lo = bin >= 0 ? bin : 0x7fffffff, hi = bin;
    for (int off = 32; off > 0; off >>= 1) {
      lo = min(lo, __shfl_xor(lo, off, 64));
      hi = max(hi, __shfl_xor(hi, off, 64));
    }
    for (int bb = lo; bb <= hi; ++bb) {
      const bool in = bin == bb;
      const double s0 = wave_sum(in ? w : 0.0);
      const double s1 = wave_sum(in ? w * k : 0.0);
      const double s2 = wave_sum(in ? w * p : 0.0);
      const double s3 = wave_sum(in ? w * pl : 0.0);
      if (lane == 0 && s0 != 0.0) {
        mine[bb * 4 + 0] += s0;
        mine[bb * 4 + 1] += s1;
        mine[bb * 4 + 2] += s2;
        mine[bb * 4 + 3] += s3;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nbins * 4; i += kST) {
    double s = 0.0;
    for (int wv = 0; wv < kSW; ++wv) s += acc[(size_t)wv * nbins * 4 + i];
    partial[(size_t)blockIdx.x * nbins * 4 + i] = s;
  }
}

// out[bin] = (k_mean, modes, P0, P2) from the workgroups' partials.
__global__ void multipole_final_kernel(const double* __restrict__ partial, int nblk, int nbins, double* out) {
  for (int bin = blockIdx.x * blockDim.x + threadIdx.x; bin < nbins; bin += gridDim.x * blockDim.x) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < nblk; ++b)
      for (int j = 0; j < 4; ++j) s[j] += partial[((size_t)b * nbins + bin) * 4 + j];
    const double c = s[0];
    out[bin * 4 + 0] = c > 0 ? s[1] / c : 0.0;
    out[bin * 4 + 1] = c;
    out[bin * 4 + 2] = c > 0 ? s[2] / c : 0.0;
    out[bin * 4 + 3] = c > 0 ? 5.0 * s[3] / c : 0.0;
  }
}

// dst = src on modes with lo <= |k| < hi, else 0 (src null: the indicator);
// the 1/N^3 of the inverse transform is folded in.
__global__ void shell_kernel(const float2* __restrict__ src, float2* __restrict__ dst, int n, int pitch, double kf,
                             double lo, double hi) {
  const int m1 = n / 2 + 1;
  const long long total = (long long)n * n * m1;
  const float inv = 1.0f / ((float)n * (float)n * (float)n);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
    const long long r = i / m1;
    const int z = (int)(i - r * m1);
    const int x = (int)(r / n), y = (int)(r - (long long)x * n);
    const double k = mode_k(x, y, z, n, kf);
    const bool in = k >= lo && k < hi;
    float2 v = make_float2(0.f, 0.f);
    if (in) v = src ? make_float2(src[r * pitch + z].x * inv, src[r * pitch + z].y * inv) : make_float2(inv, 0.f);
    dst[r * pitch + z] = v;
  }
}

// Per-workgroup FP64 partials of sum_x a b c, and of sum w |d_k|^2, sum w over
// a shell of a half spectrum.
__global__ void __launch_bounds__(kST) triple_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                     const float* __restrict__ c, long long nv, double* partial) {
  __shared__ double red[kSW];
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)kST + threadIdx.x; i < nv; i += (long long)gridDim.x * kST)
    s += (double)a[i] * (double)b[i] * (double)c[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kST) shell_power_kernel(const float2* __restrict__ d, int n, int pitch, double kf,
                                                          double lo, double hi, double* partial) {
  __shared__ double red[kSW];
  const int m1 = n / 2 + 1;
  const long long total = (long long)n * n * m1;
  double s = 0.0, c = 0.0;
  for (long long i = blockIdx.x * (long long)kST + threadIdx.x; i < total; i += (long long)gridDim.x * kST) {
    const long long r = i / m1;
    const int z = (int)(i - r * m1);
    const int x = (int)(r / n), y = (int)(r - (long long)x * n);
    const double k = mode_k(x, y, z, n, kf);
    if (k >= lo && k < hi) {
      const double w = (z > 0 && 2 * z < n) ? 2.0 : 1.0;
      const float2 v = d[r * pitch + z];
      s += w * ((double)v.x * v.x + (double)v.y * v.y);
      c += w;
    }
  }
  s = block_sum(s, red);
  c = block_sum(c, red);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s;
    partial[2 * blockIdx.x + 1] = c;
  }
}

// Adds `count` partials of `width` values (fixed order) into dst[0..width).
__global__ void sum_partials_kernel(const double* __restrict__ partial, int count, int width, double* dst) {
  for (int j = threadIdx.x; j < width; j += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < count; ++b) s += partial[(size_t)b * width + j];
    dst[j] = s;
  }
}

// out[t] = (k3, B, Q, triangles) from the reduced sums: sc[t] = (sum I1I2I3,
// sum J1J2J3, P3 power sum, P3 weight); p12 = (P1 sum, w, P2 sum, w).
__global__ void bispectrum_final_kernel(const double* __restrict__ sc, const double* __restrict__ p12,
                                        const double* __restrict__ k3, int ntheta, int n, double dx, double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntheta) return;
  const double n3 = (double)n * n * n;
  const double pn = dx * dx * dx / n3;
  const double p1 = pn * p12[0] / p12[1], p2 = pn * p12[2] / p12[3];
  const double* s = sc + 4 * t;
  const double p3 = pn * s[2] / s[3];
  const double b = (dx * dx * dx * dx * dx * dx / n3) * s[0] / s[1];
  out[4 * t + 0] = k3[t];
  out[4 * t + 1] = b;
  out[4 * t + 2] = b / (p1 * p2 + p2 * p3 + p3 * p1);
  out[4 * t + 3] = s[1] * n3 * n3;
}

}  // namespace

int stats_blocks() { return 512; }

// Block partials of the allocation-free multipoles call
// (fzw_power_multipoles_noalloc): a fixed array per GPU, held until the
// process ends, instead of a buffer allocated at the first call.  Host code
// never uses the array's name as an address (on the host it is only a
// stand-in): scratch_setup resolves the device address once per device, and
// every launch takes that pointer.
constexpr int kScratchBins = 256;
constexpr size_t kScratchDoubles = (size_t)512 * kScratchBins * 4;   // stats_blocks() x bins x 4: 4 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

int scratch_max_bins() { return kScratchBins; }

hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return hipSuccess;
}

double* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

void launch_multipoles(const float2* a, const float2* b, int n, int pitch, double kf, double k_lo, double dk,
                       int nbins, double pnorm, double* partial, double* out, hipStream_t s) {
  const int nblk = stats_blocks();
  const size_t lds = (size_t)kSW * nbins * 4 * sizeof(double);
  hipLaunchKernelGGL(multipole_kernel, dim3(nblk), dim3(kST), lds, s, a, b, n, pitch, kf, k_lo, dk, nbins, pnorm,
                     partial);
  hipLaunchKernelGGL(multipole_final_kernel, dim3((nbins + 255) / 256), dim3(256), 0, s, partial, nblk, nbins, out);
}

void launch_shell(const float2* src, float2* dst, int n, int pitch, double kf, double lo, double hi, hipStream_t s) {
  const long long total = (long long)n * n * (n / 2 + 1);
  long long g = (total + kST - 1) / kST;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(shell_kernel, dim3((unsigned)g), dim3(kST), 0, s, src, dst, n, pitch, kf, lo, hi);
}

void launch_triple_sum(const float* a, const float* b, const float* c, long long nv, double* partial, double* dst,
                       hipStream_t s) {
  const int nblk = stats_blocks();
  hipLaunchKernelGGL(triple_kernel, dim3(nblk), dim3(kST), 0, s, a, b, c, nv, partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, partial, nblk, 1, dst);
}

void launch_shell_power(const float2* d, int n, int pitch, double kf, double lo, double hi, double* partial,
                        double* dst, hipStream_t s) {
  const int nblk = stats_blocks();
  hipLaunchKernelGGL(shell_power_kernel, dim3(nblk), dim3(kST), 0, s, d, n, pitch, kf, lo, hi, partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, partial, nblk, 2, dst);
}

void launch_bispectrum_final(const double* sc, const double* p12, const double* k3, int ntheta, int n, double dx,
                             double* out, hipStream_t s) {
  hipLaunchKernelGGL(bispectrum_final_kernel, dim3((ntheta + 63) / 64), dim3(64), 0, s, sc, p12, k3, ntheta, n, dx,
                     out);
}

}  // namespace fzw
