// Non-FFT kernels of the forward model and its adjoint for gfx950: LPT
// pointwise terms, cloud-in-cell deposit by counting sort with a gather, its
// gather adjoint, the fused per-voxel web/bias kernels, the likelihood pass,
// fixed-order FP64 reductions and the leapfrog updates.
#include <algorithm>

#include "fzw_device.hpp"
#include "fzw_ops.hpp"

namespace fzw {

static inline unsigned grid_for(long long n, int threads, unsigned cap = 1u << 20) {
  long long g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ------------------------------------------------------------------- fill
__global__ void fill_i32_kernel(int* p, long long n, int v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_f32_kernel(float* p, long long n, float v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
void launch_fill_i32(int* p, long long n, int v, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, v);
}
void launch_fill_f32(float* p, long long n, float v, hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, v);
}

// ------------------------------------------------------------ LPT pointwise
// 2LPT source S2 = sum_{i<j} (phi_ii phi_jj - phi_ij^2) and the spherical
// collapse divergence 3 (sqrt(hinge(1 - 2 D1 delta_L / 3)) - 1), delta_L = tr phi.
__global__ void lpt_fwd_kernel(LptArgs a) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.n; i += (long long)gridDim.x * blockDim.x) {
    const float xx = a.phi[0][i], yy = a.phi[1][i], zz = a.phi[2][i];
    const float xy = a.phi[3][i], xz = a.phi[4][i], yz = a.phi[5][i];
    const float dl = xx + yy + zz;
    a.s2[i] = xx * yy + xx * zz + yy * zz - xy * xy - xz * xz - yz * yz;
    float hv, hd;
    sc_hinge(1.f - (2.f / 3.f) * a.d1 * dl, a.tau, hv, hd);
    a.dsc[i] = 3.f * (sqrtf(hv) - 1.f);
  }
}

// Adjoint of lpt_fwd: phi cotangents from the S2 and d_SC cotangents (written
// in place over the phi cotangent buffers, which may alias phi).
__global__ void lpt_bwd_kernel(LptArgs a) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.n; i += (long long)gridDim.x * blockDim.x) {
    const float xx = a.phi[0][i], yy = a.phi[1][i], zz = a.phi[2][i];
    const float xy = a.phi[3][i], xz = a.phi[4][i], yz = a.phi[5][i];
    const float g2 = a.s2[i];
    const float gs = a.dsc[i];
    float hv, hd;
    sc_hinge(1.f - (2.f / 3.f) * a.d1 * (xx + yy + zz), a.tau, hv, hd);
    const float gdl = hv > 0.f ? -gs * a.d1 * hd * rsqrtf(hv) : 0.f;
    a.dphi[0][i] = g2 * (yy + zz) + gdl;
    a.dphi[1][i] = g2 * (xx + zz) + gdl;
    a.dphi[2][i] = g2 * (xx + yy) + gdl;
    a.dphi[3][i] = -2.f * g2 * xy;
    a.dphi[4][i] = -2.f * g2 * xz;
    a.dphi[5][i] = -2.f * g2 * yz;
  }
}

void launch_lpt_fwd(const LptArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(lpt_fwd_kernel, dim3(grid_for(a.n, 256, 16384)), dim3(256), 0, s, a);
}
void launch_lpt_bwd(const LptArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(lpt_bwd_kernel, dim3(grid_for(a.n, 256, 16384)), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------- CIC
// Cell of a particle: lattice node + floor(Psi * scale); the fractional part
// is formed from the displacement alone, never from absolute coordinates.
__device__ __forceinline__ int wrap_index(int c, int n) {
  if (c >= 0 && c < n) return c;
  if (c >= n && c < 2 * n) return c - n;
  if (c < 0 && c >= -n) return c + n;
  const int r = c % n;   // displacements of more than a box length
  return r < 0 ? r + n : r;
}

// Radial redshift-space geometry of one particle (Section 2.9, observer at
// the box centre, cell units): r = node + d - n/2, the ray from the observer to
// the real-space position, and a = f (d.r)/|r|^2, so that the redshift-space
// position is node + d + a r (no shift at r = 0).
struct RadialFrame {
  float rx, ry, rz, r2, a;
};

// Locates a particle in the mesh: node index p, displacement d = psi * scale
// (plus the radial shift when enabled), lower corner (cx, cy, cz) wrapped into
// the box and fractional offsets (tx, ty, tz).  FRAME also returns the radial
// frame and d before the shift, for the adjoint.
// A displacement (after the redshift-space shift) that is not finite or
// reaches 2^30 cells has no cell: it is replaced by zero, so that every index
// stays inside the mesh and every weight is finite, and cic_locate returns
// false; the deposit kernels then flag the chain's state as invalid (its
// log-likelihood becomes NaN).
constexpr float kMaxCells = 1073741824.f;
template <bool FRAME = false>
__device__ __forceinline__ bool cic_locate(const CicArgs& a, int p, int n, int& cx, int& cy, int& cz,
                                           float& tx, float& ty, float& tz, RadialFrame* fr = nullptr,
                                           float* d0 = nullptr) {
  bool ok = true;
  const int q = (int)fast_div((unsigned)p, a.dn);
  const int iz = p - q * n;
  const int ix = (int)fast_div((unsigned)q, a.dn);
  const int iy = q - ix * n;
  {
    // no fma contraction here: fusing psi * scale - floor into one fma is a
    // per-kernel choice of the compiler, and every deposit and its adjoint
    // must see the same fractional offsets bit for bit
#pragma clang fp contract(off)
    float dx = a.psi[0][p] * a.scale[0];
    float dy = a.psi[1][p] * a.scale[1];
    float dz = a.psi[2][p] * a.scale[2];
    if (FRAME) {
      d0[0] = dx;
      d0[1] = dy;
      d0[2] = dz;
    }
    if (a.radial) {
      const int h = n >> 1;
      const float rx = (float)(ix - h) + dx;
      const float ry = (float)(iy - h) + dy;
      const float rz = (float)(iz - h) + dz;
      const float r2 = rx * rx + ry * ry + rz * rz;
      const float ur = dx * rx + dy * ry + dz * rz;
      const float s = r2 > 0.f ? a.f_los * ur / r2 : 0.f;
      dx = dx + s * rx;
      dy = dy + s * ry;
      dz = dz + s * rz;
      if (FRAME) *fr = RadialFrame{rx, ry, rz, r2, s};
    }
    // (comparisons with NaN are false)
    if (!(fabsf(dx) < kMaxCells && fabsf(dy) < kMaxCells && fabsf(dz) < kMaxCells)) {
      dx = dy = dz = 0.f;
      ok = false;
    }
    const float fx = floorf(dx), fy = floorf(dy), fz = floorf(dz);
    tx = dx - fx;
    ty = dy - fy;
    tz = dz - fz;
    cx = ix + (int)fx;
    cy = iy + (int)fy;
    cz = iz + (int)fz;
  }
  cx = wrap_index(cx, n);
  cy = wrap_index(cy, n);
  cz = wrap_index(cz, n);
  return ok;
}

// The count and the scatter take the particles of a tile of kSrcTile x
// kSrcTile source columns (all z) per workgroup.  A particle moves a few cells
// at most, so nearly all of them land in the kWin x kWin destination columns
// around the tile: those are counted in an LDS histogram over that window, and
// the workgroup adds each nonzero bin to the column's global counter with one
// atomic.  A particle that lands outside the window (a displacement above
// kWinR cells across) uses a global atomic of its own.  Global atomics go from
// one per distinct column per wavefront to about one per distinct column per
// tile.
constexpr int kSrcTile = 2;
constexpr int kWinR = 6;
constexpr int kWin = kSrcTile + 2 * kWinR;
constexpr int kTilePmax = 8;   // particles per thread of a tile at n <= 512

// Window bin of destination column (cx, cy) for the tile at (x0, y0), or -1.
__device__ __forceinline__ int win_bin(int cx, int cy, int x0, int y0, int n) {
  int rx = cx - x0 + kWinR, ry = cy - y0 + kWinR;
  rx += rx < 0 ? n : 0;
  rx -= rx >= n ? n : 0;
  ry += ry < 0 ? n : 0;
  ry -= ry >= n ? n : 0;
  return rx < kWin && ry < kWin ? rx * kWin + ry : -1;
}
// Destination column of window bin `bin`.
__device__ __forceinline__ int win_key(int bin, int x0, int y0, int n) {
  int kx = x0 - kWinR + bin / kWin, ky = y0 - kWinR + bin % kWin;
  kx += kx < 0 ? n : 0;
  kx -= kx >= n ? n : 0;
  ky += ky < 0 ? n : 0;
  ky -= ky >= n ? n : 0;
  return kx * n + ky;
}
// Particle index of entry i of the tile at (x0, y0).
__device__ __forceinline__ int tile_particle(int i, int x0, int y0, int n) {
  const int col = i / n, z = i - col * n;
  return ((x0 + col / kSrcTile) * n + (y0 + col % kSrcTile)) * n + z;
}

// Particles per destination column (x, y) of the mesh.
__global__ __launch_bounds__(256) void cic_count_kernel(CicArgs a) {
  __shared__ int hist[kWin * kWin];
  const int n = a.n;
  const long long nv = a.nv;
  const long long c = blockIdx.y;
  CicArgs b = a;
  for (int d = 0; d < 3; ++d) b.psi[d] = a.psi[d] + c * nv;
  int* count = a.count + c * (long long)n * n;
  const int t = threadIdx.x;
  const int tpr = n / kSrcTile, ntile = tpr * tpr;
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    for (int i = t; i < kWin * kWin; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int x0 = (tile / tpr) * kSrcTile, y0 = (tile % tpr) * kSrcTile;
    bool bad = false;
    for (int i = t; i < kSrcTile * kSrcTile * n; i += blockDim.x) {
      int cx, cy, cz;
      float tx, ty, tz;
      bad |= !cic_locate(b, tile_particle(i, x0, y0, n), n, cx, cy, cz, tx, ty, tz);
      const int bin = win_bin(cx, cy, x0, y0, n);
      if (bin >= 0) atomicAdd(hist + bin, 1);
      else atomicAdd(count + cx * n + cy, 1);
    }
    if (__ballot(bad) != 0ull && (t & 63) == 0) atomicOr(a.flags + c, FZW_NF_STATE);
    __syncthreads();
    for (int i = t; i < kWin * kWin; i += blockDim.x) {
      const int h = hist[i];
      if (h) atomicAdd(count + win_key(i, x0, y0, n), h);
    }
    __syncthreads();
  }
}

// Exclusive scan of the column counts: per-block totals, a single-block scan
// of the totals, then per-block local scans.
constexpr int kScanBlock = 4096;
__global__ void scan_reduce_kernel(const int* __restrict__ count, long long nv, int* __restrict__ bsum, int nb) {
  __shared__ int red[256];
  const long long c = blockIdx.y;
  const int* cnt = count + c * nv;
  const long long base = (long long)blockIdx.x * kScanBlock;
  int s = 0;
  for (int i = threadIdx.x; i < kScanBlock; i += 256) {
    const long long g = base + i;
    if (g < nv) s += cnt[g];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[c * nb + blockIdx.x] = red[0];
}

__global__ void scan_blocks_kernel(int* bsum, int nb) {
  // one workgroup of 1024 threads per chain, exclusive scan in place
  __shared__ int tot[1024];
  const long long c = blockIdx.x;
  int* b = bsum + c * nb;
  const int per = (nb + 1023) / 1024;
  const int lo = threadIdx.x * per;
  int s = 0;
  for (int i = 0; i < per; ++i)
    if (lo + i < nb) s += b[lo + i];
  tot[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = threadIdx.x >= off ? tot[threadIdx.x - off] : 0;
    __syncthreads();
    tot[threadIdx.x] += v;
    __syncthreads();
  }
  int run = threadIdx.x > 0 ? tot[threadIdx.x - 1] : 0;
  for (int i = 0; i < per; ++i) {
    if (lo + i < nb) {
      const int v = b[lo + i];
      b[lo + i] = run;
      run += v;
    }
  }
}

__global__ void scan_down_kernel(const int* __restrict__ count, long long nv, const int* __restrict__ bsum, int nb,
                                 int* __restrict__ offset) {
  __shared__ int part[256];
  const long long c = blockIdx.y;
  const int* cnt = count + c * nv;
  int* off = offset + c * (nv + 1);
  const long long base = (long long)blockIdx.x * kScanBlock;
  constexpr int PER = kScanBlock / 256;
  int v[PER];
  int s = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const long long g = base + threadIdx.x * PER + i;
    v[i] = g < nv ? cnt[g] : 0;
    s += v[i];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int x = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  int run = bsum[c * nb + blockIdx.x] + (threadIdx.x > 0 ? part[threadIdx.x - 1] : 0);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const long long g = base + threadIdx.x * PER + i;
    if (g < nv) off[g] = run;
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 255) off[nv] = run;
}

// Scatter the fractional offsets into column order (any order inside a
// column); the bucket's y and z indices travel in the .w lane as by << 16 | bz.
// Per tile (as in the count): the window bins are counted in LDS, each
// nonzero bin reserves its slots in its column with one global atomic, and the
// particles take consecutive slots of their bin's range with LDS atomics;
// particles outside the window take a global slot each.  The located particles
// stay in registers between the two steps.
__global__ __launch_bounds__(256) void cic_scatter_kernel(CicArgs a) {
  __shared__ int hist[kWin * kWin];   // counts, then the bins' first slot
  __shared__ int cur[kWin * kWin];
  const int n = a.n;
  const long long nv = a.nv;
  const long long c = blockIdx.y;
  const long long ncol = (long long)n * n;
  CicArgs b = a;
  for (int d = 0; d < 3; ++d) b.psi[d] = a.psi[d] + c * nv;
  int* cursor = a.count + c * ncol;
  const int* off = a.offset + c * (ncol + 1);
  float4* sorted = a.sorted + c * nv;
  const int t = threadIdx.x;
  const int tpr = n / kSrcTile, ntile = tpr * tpr;
  const int per = kSrcTile * kSrcTile * n;
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    for (int i = t; i < kWin * kWin; i += blockDim.x) {
      hist[i] = 0;
      cur[i] = 0;
    }
    __syncthreads();
    const int x0 = (tile / tpr) * kSrcTile, y0 = (tile % tpr) * kSrcTile;
    int key[kTilePmax], bin[kTilePmax], yz[kTilePmax];
    float fx[kTilePmax], fy[kTilePmax], fz[kTilePmax];
#pragma unroll
    for (int r = 0; r < kTilePmax; ++r) {
      const int i = t + r * (int)blockDim.x;
      bin[r] = -1;
      key[r] = -1;
      if (i < per) {
        int cx, cy, cz;
        cic_locate(b, tile_particle(i, x0, y0, n), n, cx, cy, cz, fx[r], fy[r], fz[r]);
        key[r] = cx * n + cy;
        yz[r] = (cy << 16) | cz;
        bin[r] = win_bin(cx, cy, x0, y0, n);
        if (bin[r] >= 0) atomicAdd(hist + bin[r], 1);
      }
    }
    __syncthreads();
    for (int i = t; i < kWin * kWin; i += blockDim.x) {
      const int h = hist[i];
      if (h) {
        const int k = win_key(i, x0, y0, n);
        hist[i] = off[k] + atomicAdd(cursor + k, h);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTilePmax; ++r) {
      if (key[r] < 0) continue;
      const int dst = bin[r] >= 0 ? hist[bin[r]] + atomicAdd(cur + bin[r], 1)
                                  : off[key[r]] + atomicAdd(cursor + key[r], 1);
      if (dst < off[key[r] + 1]) sorted[dst] = make_float4(fx[r], fy[r], fz[r], __int_as_float(yz[r]));
    }
    __syncthreads();
  }
}

// Gather deposit, tiled: a workgroup owns kLineTile x kLineTile lines of nodes
// along z.  It streams the particles of the (kLineTile+1)^2 source columns
// that touch those lines (contiguous in column order, so the loads coalesce)
// and adds each trilinear weight, in 64-bit fixed point (2^-32 resolution),
// to an LDS copy of its lines with integer atomics.  Integer sums do not
// depend on order, so the density is bitwise reproducible and equal to that of
// the global-atomic deposit below.
constexpr int kLineTile = 4;
// The 4x4-line LDS accumulator (128 KB at N = 256) allows one workgroup per
// CU, so the workgroup is as wide as a CU takes: 16 wavefronts stream the
// particles.
constexpr int kGatherThreads = 1024;
__global__ __launch_bounds__(kGatherThreads) void cic_gather_tiles_kernel(CicArgs a) {
  extern __shared__ unsigned long long acc_lds[];
  constexpr int T = kLineTile;
  const long long nv = a.nv;
  const int n = a.n;
  const long long c = blockIdx.y;
  const int* off = a.offset + c * ((long long)n * n + 1);
  const float4* sorted = a.sorted + c * nv;
  float* rho = a.rho + c * nv;
  const int tiles = n / T;
  const int x0 = (blockIdx.x / tiles) * T, y0 = (blockIdx.x % tiles) * T;
  const int t = threadIdx.x;
  for (int i = t; i < T * T * n; i += blockDim.x) acc_lds[i] = 0ull;
  __syncthreads();
  // the source columns (bx, y0-1 .. y0+T-1) of one bx are consecutive in
  // column order: one range per bx, two where y0-1 wraps to n-1
  for (int seg = 0; seg < 2 * (T + 1); ++seg) {
    const int rx = seg >> 1;
    int bx = x0 - 1 + rx;
    bx += bx < 0 ? n : 0;
    const int* ob = off + bx * n;
    int lo, hi;
    if (y0 > 0) {
      if (seg & 1) continue;
      lo = ob[y0 - 1];
      hi = ob[y0 + T];
    } else if (seg & 1) {
      lo = ob[n - 1];
      hi = ob[n];
    } else {
      lo = ob[0];
      hi = ob[T];
    }
    for (int s = lo + t; s < hi; s += blockDim.x) {
      const float4 q = sorted[s];
      const int yz = __float_as_int(q.w);
      const int bz = yz & 0xffff;
      int ry = (yz >> 16) - y0 + 1;
      ry -= ry > T ? n : 0;
      if ((unsigned)bz >= (unsigned)n || (unsigned)ry > (unsigned)T) continue;   // never taken
      const int bz1 = bz + 1 == n ? 0 : bz + 1;
#pragma unroll
      for (int ox = 0; ox < 2; ++ox) {
        const int lx = rx - 1 + ox;
        if (lx < 0 || lx >= T) continue;
#pragma unroll
        for (int oy = 0; oy < 2; ++oy) {
          const int ly = ry - 1 + oy;
          if (ly < 0 || ly >= T) continue;
          const float wxy = (ox ? q.x : 1.f - q.x) * (oy ? q.y : 1.f - q.y);
          unsigned long long* line = acc_lds + (lx * T + ly) * n;
          atomicAdd(line + bz, (unsigned long long)__float2ll_rn(wxy * (1.f - q.z) * 4294967296.0f));
          atomicAdd(line + bz1, (unsigned long long)__float2ll_rn(wxy * q.z * 4294967296.0f));
        }
      }
    }
  }
  __syncthreads();
  for (int i = t; i < T * T * n; i += blockDim.x) {
    const int l = i / n, z = i % n;
    const int x = x0 + l / T, y = y0 + l % T;
    rho[((long long)x * n + y) * n + z] = (float)((double)(long long)acc_lds[i] * (1.0 / 4294967296.0));
  }
}

// Adjoint: each particle gathers the density cotangent at its 8 nodes and
// writes the displacement cotangent (may alias the displacement buffers).  A
// thread takes two particles, p and p + ceil(nv/2), and issues every load of
// both before its first store: with the output aliasing the input, loads
// after a store could not be moved ahead of it.
__global__ void cic_adjoint_kernel(CicArgs a) {
  const long long nv = a.nv;
  const int n = a.n;
  const long long c = blockIdx.y;
  CicArgs b = a;
  for (int d = 0; d < 3; ++d) b.psi[d] = a.psi[d] + c * nv;
  const float* g = a.drho + c * nv;
  const long long half = (nv + 1) / 2;
  for (long long p0 = blockIdx.x * (long long)blockDim.x + threadIdx.x; p0 < half;
       p0 += (long long)gridDim.x * blockDim.x) {
    float gx[2], gy[2], gz[2];
    RadialFrame fr[2];
    float d0[2][3];
    bool has[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const long long p = p0 + u * half;
      has[u] = p < nv;
      int cx, cy, cz;
      float tx, ty, tz;
      // the second particle of an odd count repeats the first (not stored)
      cic_locate<true>(b, (int)(has[u] ? p : p0), n, cx, cy, cz, tx, ty, tz, &fr[u], d0[u]);
      const int nx = cx + 1 == n ? 0 : cx + 1;
      const int ny = cy + 1 == n ? 0 : cy + 1;
      const int nz = cz + 1 == n ? 0 : cz + 1;
      gx[u] = gy[u] = gz[u] = 0.f;
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const int ox = (o >> 2) & 1, oy = (o >> 1) & 1, oz = o & 1;
        const float v = g[((ox ? nx : cx) * n + (oy ? ny : cy)) * (long long)n + (oz ? nz : cz)];
        const float wx = ox ? tx : 1.f - tx, wy = oy ? ty : 1.f - ty, wz = oz ? tz : 1.f - tz;
        const float sx = ox ? 1.f : -1.f, sy = oy ? 1.f : -1.f, sz = oz ? 1.f : -1.f;
        gx[u] += v * sx * wy * wz;
        gy[u] += v * wx * sy * wz;
        gz[u] += v * wx * wy * sz;
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      float x = gx[u], y = gy[u], z = gz[u];
      if (a.radial) {
        // transpose of ds_i/dd_j = (1+a) delta_ij + r_i (f d_j + (f - 2a) r_j) / |r|^2
        const RadialFrame& f0 = fr[u];
        const float gr = f0.r2 > 0.f ? (x * f0.rx + y * f0.ry + z * f0.rz) / f0.r2 : 0.f;
        const float f = a.f_los, cr = f - 2.f * f0.a, ca = 1.f + f0.a;
        x = ca * x + gr * (f * d0[u][0] + cr * f0.rx);
        y = ca * y + gr * (f * d0[u][1] + cr * f0.ry);
        z = ca * z + gr * (f * d0[u][2] + cr * f0.rz);
      }
      if (!has[u]) continue;
      const long long p = c * nv + p0 + u * half;
      a.dpsi[0][p] = x * a.scale[0];
      a.dpsi[1][p] = y * a.scale[1];
      a.dpsi[2][p] = z * a.scale[2];
    }
  }
}

// Alternative deposit: every particle adds its 8 trilinear weights into a
// 64-bit fixed-point accumulator with integer atomics (no return value); the
// same FP32 weights and the same rounding to 2^-32 as the gather make the
// result bit-identical to it, and integer addition makes it order-free.
__global__ void cic_atomic_kernel(CicArgs a) {
  const long long nv = a.nv;
  const int n = a.n;
  const long long c = blockIdx.y;
  CicArgs b = a;
  for (int d = 0; d < 3; ++d) b.psi[d] = a.psi[d] + c * nv;
  unsigned long long* acc = a.acc + c * nv;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < nv; p += (long long)gridDim.x * blockDim.x) {
    int cx, cy, cz;
    float tx, ty, tz;
    RadialFrame fr;
    float d0[3];
    if (!cic_locate<true>(b, (int)p, n, cx, cy, cz, tx, ty, tz, &fr, d0)) atomicOr(a.flags + c, FZW_NF_STATE);
    const int nx = cx + 1 == n ? 0 : cx + 1;
    const int ny = cy + 1 == n ? 0 : cy + 1;
    const int nz = cz + 1 == n ? 0 : cz + 1;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int ox = (o >> 2) & 1, oy = (o >> 1) & 1, oz = o & 1;
      const float w = (ox ? tx : 1.f - tx) * (oy ? ty : 1.f - ty) * (oz ? tz : 1.f - tz);
      const long long q = ((long long)(ox ? nx : cx) * n + (oy ? ny : cy)) * n + (oz ? nz : cz);
      atomicAdd(acc + q, (unsigned long long)__float2ll_rn(w * 4294967296.0f));
    }
  }
}

// rho from the accumulator; the accumulator is cleared for the next deposit.
__global__ void cic_convert_kernel(CicArgs a, long long total) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long v = a.acc[i];
    a.rho[i] = (float)((double)(long long)v * (1.0 / 4294967296.0));
    a.acc[i] = 0ull;
  }
}

void launch_cic_deposit_atomic(const CicArgs& a0, int chains, hipStream_t s) {
  CicArgs a = a0;
  a.dn = make_fastdiv((unsigned)a.n);
  dim3 gp(grid_for(a.nv, 256, 32768), chains);
  hipLaunchKernelGGL(cic_atomic_kernel, gp, dim3(256), 0, s, a);
  const long long total = a.nv * chains;
  hipLaunchKernelGGL(cic_convert_kernel, dim3(grid_for(total, 256, 32768)), dim3(256), 0, s, a, total);
}

void launch_cic_deposit(const CicArgs& a0, int chains, hipStream_t s) {
  CicArgs a = a0;
  a.dn = make_fastdiv((unsigned)a.n);
  const long long nv = a.nv;
  const long long ncol = (long long)a.n * a.n;
  launch_fill_i32(a.count, ncol * chains, 0, s);
  // one workgroup per source tile (kSrcTile^2 columns)
  const int ntile = (a.n / kSrcTile) * (a.n / kSrcTile);
  dim3 gp((unsigned)std::min(ntile, 65536), chains);
  hipLaunchKernelGGL(cic_count_kernel, gp, dim3(256), 0, s, a);
  const int nb = (int)((ncol + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb, chains), dim3(256), 0, s, a.count, ncol, a.bsum, nb);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(chains), dim3(1024), 0, s, a.bsum, nb);
  hipLaunchKernelGGL(scan_down_kernel, dim3(nb, chains), dim3(256), 0, s, a.count, ncol, a.bsum, nb, a.offset);
  launch_fill_i32(a.count, ncol * chains, 0, s);
  hipLaunchKernelGGL(cic_scatter_kernel, gp, dim3(256), 0, s, a);
  const int tiles = a.n / kLineTile;
  const size_t lds = sizeof(unsigned long long) * kLineTile * kLineTile * a.n;
  if (lds > 32768)
    (void)hipFuncSetAttribute((const void*)cic_gather_tiles_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL(cic_gather_tiles_kernel, dim3(tiles * tiles, chains), dim3(kGatherThreads), lds, s, a);
}

void launch_cic_adjoint(const CicArgs& a0, int chains, hipStream_t s) {
  CicArgs a = a0;
  a.dn = make_fastdiv((unsigned)a.n);
  dim3 gp(grid_for(a.nv, 256, 32768), chains);
  hipLaunchKernelGGL(cic_adjoint_kernel, gp, dim3(256), 0, s, a);
}

// ------------------------------------------------------- symmetric 3x3 eigen
// Eigenvalues of a symmetric 3x3 tensor, descending, by the trigonometric
// solution of the characteristic cubic (Smith 1961).
// Eigenvalues of a symmetric 3x3 tensor from its normalised characteristic
// cubic: with q = tr T / 3, p^2 = tr((T - qI)^2) / 6 and B = (T - qI) / p, the
// eigenvalues are q + p beta where beta^3 - 3 beta = det B = 2r, |r| <= 1.
// The root farthest from the other two is the largest one when r >= 0 and the
// smallest otherwise, and its magnitude lies in [sqrt 3, 2], where the cubic's
// slope is at least 6: two Newton steps from the chord through the end points
// reach float precision, with no trigonometric functions.  Returns that root
// (beta_iso) and whether it is the largest (top); p = 0 flags T = qI.
__device__ __forceinline__ void eig3_cubic(const float t[6], float& q, float& p, float& beta_iso, bool& top) {
  q = (t[0] + t[1] + t[2]) * (1.f / 3.f);
  const float a = t[0] - q, b = t[1] - q, c = t[2] - q;
  const float p2 = (a * a + b * b + c * c + 2.f * (t[3] * t[3] + t[4] * t[4] + t[5] * t[5])) * (1.f / 6.f);
  beta_iso = 0.f;
  top = true;
  if (!(p2 > 0.f)) {
    p = 0.f;
    return;
  }
  p = sqrtf(p2);
  // hardware reciprocals (about 1 ulp): a uniform scale error of B moves r by
  // a few ulp, and the Newton corrections are self-correcting
  const float ip = __builtin_amdgcn_rcpf(p);
  const float ba = a * ip, bb = b * ip, bc = c * ip, bxy = t[3] * ip, bxz = t[4] * ip, byz = t[5] * ip;
  const float det = ba * (bb * bc - byz * byz) - bxy * (bxy * bc - byz * bxz) + bxz * (bxy * byz - bb * bxz);
  const float r = fminf(1.f, fmaxf(-1.f, 0.5f * det));
  top = r >= 0.f;
  const float ra = fabsf(r);
  float x = 1.7320508075688772f + 0.2679491924311228f * ra;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const float x2 = x * x;
    x -= (x * (x2 - 3.f) - 2.f * ra) * __builtin_amdgcn_rcpf(3.f * (x2 - 1.f));
  }
  beta_iso = top ? x : -x;
}

// All three eigenvalues (descending) from the isolated root: the other two
// solve beta^2 + beta_iso beta + beta_iso^2 - 3 = 0.
__device__ __forceinline__ void eig3_all(float q, float p, float beta_iso, bool top, float lam[3]) {
  const float s = sqrtf(fmaxf(0.f, 12.f - 3.f * beta_iso * beta_iso));
  const float hi = 0.5f * (-beta_iso + s), lo = 0.5f * (-beta_iso - s);
  if (top) {
    lam[0] = q + p * beta_iso;
    lam[1] = q + p * hi;
    lam[2] = q + p * lo;
  } else {
    lam[0] = q + p * hi;
    lam[1] = q + p * lo;
    lam[2] = q + p * beta_iso;
  }
}

__device__ __forceinline__ void cross3(const float* a, const float* b, float* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Unit eigenvector of eigenvalue l from the largest cross product of two rows
// of T - l I; returns false when T - l I has rank < 2 numerically.
__device__ __forceinline__ bool eig3_vector(const float t[6], float l, float scale4, float v[3]) {
  const float r0[3] = {t[0] - l, t[3], t[4]};
  const float r1[3] = {t[3], t[1] - l, t[5]};
  const float r2[3] = {t[4], t[5], t[2] - l};
  float c0[3], c1[3], c2[3];
  cross3(r0, r1, c0);
  cross3(r0, r2, c1);
  cross3(r1, r2, c2);
  const float n0 = c0[0] * c0[0] + c0[1] * c0[1] + c0[2] * c0[2];
  const float n1 = c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2];
  const float n2 = c2[0] * c2[0] + c2[1] * c2[1] + c2[2] * c2[2];
  const float* best = c0;
  float nb = n0;
  if (n1 > nb) { best = c1; nb = n1; }
  if (n2 > nb) { best = c2; nb = n2; }
  if (!(nb > 1e-24f * scale4)) return false;
  const float s = rsqrtf(nb);
  v[0] = best[0] * s;
  v[1] = best[1] * s;
  v[2] = best[2] * s;
  return true;
}

__device__ __forceinline__ void any_orthogonal(const float* a, float* v) {
  // unit vector orthogonal to unit a
  float e[3] = {0.f, 0.f, 0.f};
  const float ax = fabsf(a[0]), ay = fabsf(a[1]), az = fabsf(a[2]);
  if (ax <= ay && ax <= az) e[0] = 1.f;
  else if (ay <= az) e[1] = 1.f;
  else e[2] = 1.f;
  float c[3];
  cross3(a, e, c);
  const float s = rsqrtf(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  v[0] = c[0] * s;
  v[1] = c[1] * s;
  v[2] = c[2] * s;
}

__device__ __forceinline__ void sym_mul(const float t[6], const float* x, float* y) {
  y[0] = t[0] * x[0] + t[3] * x[1] + t[4] * x[2];
  y[1] = t[3] * x[0] + t[1] * x[1] + t[5] * x[2];
  y[2] = t[4] * x[0] + t[5] * x[1] + t[2] * x[2];
}
__device__ __forceinline__ float dot3(const float* a, const float* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Eigen-decomposition of a symmetric 3x3 tensor that stays accurate for
// nearly equal eigenvalues: the characteristic cubic only supplies the
// eigenvalue farthest from the other two; its eigenvector (a cross product of
// two rows of T - l I, well conditioned because that eigenvalue is isolated)
// is taken first, and the remaining pair is the exact Jacobi rotation of T
// restricted to the orthogonal plane.  Returns eigenvalues descending and the
// unit eigenvectors v1 (largest) and v3 (smallest).
__device__ __forceinline__ void eig3_robust(const float t[6], float lam[3], float v1[3], float v3[3]) {
  float q, p, beta;
  bool top;
  eig3_cubic(t, q, p, beta, top);
  v1[0] = 1.f; v1[1] = 0.f; v1[2] = 0.f;
  v3[0] = 0.f; v3[1] = 0.f; v3[2] = 1.f;
  if (!(p > 0.f)) {
    lam[0] = lam[1] = lam[2] = q;
    return;
  }
  float v[3];
  if (!eig3_vector(t, q + p * beta, (p * p) * (p * p) * 81.f, v)) {
    eig3_all(q, p, beta, top, lam);
    return;
  }
  float u[3], w[3], tu[3], tw[3], tv[3];
  any_orthogonal(v, u);
  cross3(v, u, w);
  sym_mul(t, u, tu);
  sym_mul(t, w, tw);
  sym_mul(t, v, tv);
  const float a = dot3(u, tu), b = dot3(u, tw), c = dot3(w, tw);
  float cs = 1.f, sn = 0.f, tt = 0.f;
  if (b != 0.f) {
    const float tau = (c - a) / (2.f * b);
    tt = copysignf(1.f, tau) / (fabsf(tau) + sqrtf(1.f + tau * tau));
    cs = rsqrtf(1.f + tt * tt);
    sn = tt * cs;
  }
  // pairs (value, vector): (v.Tv, v), (a - t b, cs u - sn w), (c + t b, sn u + cs w)
  float L[3] = {dot3(v, tv), a - tt * b, c + tt * b};
  float V[3][3] = {{v[0], v[1], v[2]},
                   {cs * u[0] - sn * w[0], cs * u[1] - sn * w[1], cs * u[2] - sn * w[2]},
                   {sn * u[0] + cs * w[0], sn * u[1] + cs * w[1], sn * u[2] + cs * w[2]}};
  int i0 = 0, i1 = 1, i2 = 2;   // sort descending by index
  if (L[i0] < L[i1]) { int x = i0; i0 = i1; i1 = x; }
  if (L[i1] < L[i2]) { int x = i1; i1 = i2; i2 = x; }
  if (L[i0] < L[i1]) { int x = i0; i0 = i1; i1 = x; }
  lam[0] = L[i0]; lam[1] = L[i1]; lam[2] = L[i2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v1[k] = i0 == 0 ? V[0][k] : (i0 == 1 ? V[1][k] : V[2][k]);
    v3[k] = i2 == 0 ? V[0][k] : (i2 == 1 ? V[1][k] : V[2][k]);
  }
}

// Gradient of a function of the eigenvalues with respect to the tensor:
// G = sum_n g_n v_n v_n^T = g2 I + (g1 - g2) v1 v1^T + (g3 - g2) v3 v3^T.
// Returned as cotangents of the 6 stored components (off-diagonals doubled).
__device__ __forceinline__ void eig3_grad(const float v1[3], const float v3[3], const float g[3], float out[6]) {
  const float a1 = g[0] - g[1], a3 = g[2] - g[1];
  out[0] = g[1] + a1 * v1[0] * v1[0] + a3 * v3[0] * v3[0];
  out[1] = g[1] + a1 * v1[1] * v1[1] + a3 * v3[1] * v3[1];
  out[2] = g[1] + a1 * v1[2] * v1[2] + a3 * v3[2] * v3[2];
  out[3] = 2.f * (a1 * v1[0] * v1[1] + a3 * v3[0] * v3[1]);
  out[4] = 2.f * (a1 * v1[0] * v1[2] + a3 * v3[0] * v3[2]);
  out[5] = 2.f * (a1 * v1[1] * v1[2] + a3 * v3[1] * v3[2]);
}

__device__ __forceinline__ float sigmoidf(float x) { return 1.f / (1.f + expf(-x)); }

// Sigmoid weights and memberships of one web (V, S, F, K).
__device__ __forceinline__ void web_memberships(const float lam[3], float s, float th, float w[3], float pm[4]) {
#pragma unroll
  for (int n = 0; n < 3; ++n) w[n] = sigmoidf(s * (lam[n] - th));
  pm[0] = 1.f - w[0];
  pm[1] = w[0] - w[1];
  pm[2] = w[1] - w[2];
  pm[3] = w[2];
}

// ------------------------------------------------ NB constants per voxel
// sum_{m<n} ln(beta+m) = lnGamma(n+beta) - lnGamma(beta), and its beta
// derivative sum_{m<n} 1/(beta+m).
__device__ __forceinline__ double digamma_d(double x) {
  // recurrence up to x >= 8, then the asymptotic series (Abramowitz & Stegun 6.3.18);
  // only x > 0 occurs (x = n + beta with beta > 0): anything else, NaN
  // included, returns NaN before the recurrence, which would not end for
  // x = -inf
  if (!(x > 0.0)) return __builtin_nan("");
  double r = 0.0;
  while (x < 8.0) {
    r -= 1.0 / x;
    x += 1.0;
  }
  const double ix = 1.0 / x, ix2 = ix * ix;
  return r + log(x) - 0.5 * ix -
         ix2 * (1.0 / 12 - ix2 * (1.0 / 120 - ix2 * (1.0 / 252 - ix2 * (1.0 / 240 - ix2 * (1.0 / 132)))));
}

// Counts above 64 are rare: their lnGamma(n+beta) - lnGamma(beta) and
// psi(n+beta) - psi(beta) use float64 special functions out of line (below
// that the finite sums over m < n are used).
__device__ __noinline__ double nb_lgamma_big_d(int n, double beta) {
  return lgamma((double)n + beta) - lgamma(beta);
}
__device__ __noinline__ double nb_digamma_big(int n, double beta) {
  return digamma_d((double)n + beta) - digamma_d(beta);
}

// ---------------------------------------------------------- per-voxel fused
template <int W>
struct VoxelCore {
  static constexpr int R = W == 1 ? 4 : 16;
  float lam[W][3], v1[W][3], v3[W][3], wgt[W][3], pm[W][4], preg[R];
  float theta[4];
  float x, lnx, ellr, u, logf;
  float t6[W][6];

  __device__ __forceinline__ void run(const VoxelArgs& a, const float* tab, long long i, float rho) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
#pragma unroll
      for (int c = 0; c < 6; ++c) t6[w][c] = a.tens[w * 6 + c][i];
      eig3_robust(t6[w], lam[w], v1[w], v3[w]);
      web_memberships(lam[w], a.steep, a.lam_th, wgt[w], pm[w]);
      // one web at a time: interleaving the two solves doubles the live registers
      __builtin_amdgcn_sched_barrier(0);
    }
    if (W == 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) preg[r] = pm[0][r];
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k = 0; k < 4; ++k) preg[4 * j + k] = pm[0][j] * pm[W - 1][k];
    }
    theta[0] = theta[1] = theta[2] = theta[3] = 0.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float4 tr = reinterpret_cast<const float4*>(tab)[r];
      theta[0] += preg[r] * tr.x;
      theta[1] += preg[r] * tr.y;
      theta[2] += preg[r] * tr.z;
      theta[3] += preg[r] * tr.w;
      // four table rows at a time: hoisting every read keeps all 4R entries live
      if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    x = fmaxf(rho, a.x_floor);
    lnx = ::logf(x);
    ellr = lnx - ::logf(theta[2]);
    u = expf(theta[1] * ellr);
    logf = theta[0] * lnx - u;
  }
};

template <int W>
__global__ __launch_bounds__(256) void voxel_fwd_kernel(VoxelArgs a) {
  constexpr int NE = W == 1 ? 16 : 64;
  __shared__ double red[4];
  // the bias table sits in LDS: read from global memory inside the loop it is
  // held in vector registers (the compiler cannot prove it unwritten)
  __shared__ __align__(16) float tab[NE];
  const long long c = blockIdx.y;
  const long long nv = a.nv;
  if (threadIdx.x < NE) tab[threadIdx.x] = a.table[c * NE + threadIdx.x];
  __syncthreads();
  VoxelArgs b = a;
  for (int k = 0; k < 6 * W; ++k) b.tens[k] = a.tens[k] + c * nv;
  double sf = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nv; i += (long long)gridDim.x * blockDim.x) {
    VoxelCore<W> v;
    v.run(b, tab, i, a.rho[c * nv + i]);
    a.logf[c * nv + i] = v.logf;
    a.beta[c * nv + i] = v.theta[3];
    sf += (double)expf(v.logf);
  }
  const double s = block_sum(sf, red);
  if (threadIdx.x == 0) a.partial[c * gridDim.x + blockIdx.x] = s;
}

// Likelihood pass: needs ln C = ln N_tr - ln sum f from the reduced partials.
// Per voxel in float64: nbar = exp(ln C + log f), ln(1 + nbar/beta), and the
// finite sums over m < n of ln(beta + m) (lnGamma(n+beta) - lnGamma(beta))
// and 1/(beta + m) (psi(n+beta) - psi(beta)) from one loop over the count
// with the products of up to 8 factors (one logarithm and one division per 8
// terms; (beta+64)^8 stays inside float64).  Sums in FP64.  With ghat set it
// also writes what the backward needs: g-hat = beta (n - nbar)/(beta + nbar),
// nbar, and d lnP/d beta = psi(n+beta) - psi(beta) - ln(1 + nbar/beta) +
// (nbar - n)/(beta + nbar); G = sum g-hat comes from the same values.
__global__ __launch_bounds__(256) void likelihood_kernel(LikeArgs a) {
  __shared__ double red[4];
  const long long c = blockIdx.y;
  const long long nv = a.nv;
  const double lnc = a.scal[c * kScalStride + kScalLnC];
  const bool grad = a.ghat != nullptr;
  double sl = 0.0, sg = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nv; i += (long long)gridDim.x * blockDim.x) {
    const float lf = a.logf[c * nv + i];
    const double beta = a.beta[c * nv + i];
    const int n = a.counts[c * nv + i];
    const double fn = (double)n;
    const double lnb = lnc + (double)lf;
    const double nb = exp(lnb);
    const double ib = 1.0 / (beta + nb);
    const double l1p = -log1p(-nb * ib);                     // ln(1 + nbar/beta)
    double lg = 0.0, dg = 0.0;
    if (n <= 64) {
      for (int m0 = 0; m0 < n; m0 += 8) {
        double pq = 0.0, qq = 1.0;
        const int m1 = min(n, m0 + 8);
        for (int m = m0; m < m1; ++m) {
          const double bm = beta + (double)m;
          pq = fma(pq, bm, qq);
          qq *= bm;
        }
        lg += log(qq);
        if (grad) dg += pq / qq;
      }
    } else {
      lg = nb_lgamma_big_d(n, beta);
      if (grad) dg = nb_digamma_big(n, beta);
    }
    sl += lg - (beta + fn) * l1p + fn * (lnb - log(beta));
    const double gh = beta * (fn - nb) * ib;
    sg += gh;
    if (a.nbar) a.nbar[c * nv + i] = (float)nb;
    if (grad) {
      a.ghat[c * nv + i] = (float)gh;
      a.nbv[c * nv + i] = (float)nb;
      a.dbeta[c * nv + i] = (float)(dg - l1p + (nb - fn) * ib);
    }
  }
  const double s1 = block_sum(sl, red);
  const double s2 = block_sum(sg, red);
  if (threadIdx.x == 0) {
    a.partial[(c * gridDim.x + blockIdx.x) * 2 + 0] = s1;
    a.partial[(c * gridDim.x + blockIdx.x) * 2 + 1] = s2;
  }
}

// f(x) = x/(1+x) - log1p(x): the part of d lnP/d beta that cancels to
// -x^2/2 for small x = nbar/beta; its alternating series below 0.1
// (truncated after x^9, relative error < 2e-8), the direct form above
// (relative error ~1e-6 at x = 0.1, smaller beyond).
__device__ __forceinline__ float nb_cancel(float x) {
  if (x < 0.1f) {
    const float p = -1.f / 2 + x * (2.f / 3 + x * (-3.f / 4 + x * (4.f / 5 + x * (-5.f / 6 + x * (6.f / 7 +
                    x * (-7.f / 8 + x * (8.f / 9)))))));
    return x * x * p;
  }
  return x / (1.f + x) - log1pf(x);
}

// Running product of factors 1 + m/beta in float64, kept as a mantissa in
// [1/2, 1) and a binary exponent, so that the logarithm of all the factors a
// lane takes is formed once at the end: sum_k ln q_k = ln(prod_k q_k).
struct LogProduct {
  double mant = 1.0;
  int expo = 0;
  // multiply by prod_{1<=m<n} (1 + m/beta), n <= 64: four factors at a time
  // (a factor is below 2^133 for any normal float beta > 0, so four of them
  // times a mantissa below 1 stay finite), renormalised after each four
  __device__ __forceinline__ void rising_tail(int n, float beta) {
    // 1/beta: the float reciprocal (relative error ~1e-7) and two Newton
    // steps, each squaring the error, to float64 rounding
    const double b = (double)beta;
    double rb = (double)__builtin_amdgcn_rcpf(beta);
    rb = rb * fma(-b, rb, 2.0);
    rb = rb * fma(-b, rb, 2.0);
    double q = mant;
    for (int m0 = 1; m0 < n; m0 += 4) {
      const double d0 = (double)m0;
      const double f0 = fma(d0, rb, 1.0);
      const double f1 = m0 + 1 < n ? fma(d0 + 1.0, rb, 1.0) : 1.0;
      const double f2 = m0 + 2 < n ? fma(d0 + 2.0, rb, 1.0) : 1.0;
      const double f3 = m0 + 3 < n ? fma(d0 + 3.0, rb, 1.0) : 1.0;
      int e;
      q = frexp(q * ((f0 * f1) * (f2 * f3)), &e);
      expo += e;
    }
    mant = q;
  }
  __device__ __forceinline__ double log() const {
    return ::log(mant) + fma((double)expo, 0.6931471805599453094, (double)expo * 2.3190468138462996e-17);
  }
};

// Orders the LDS accesses of one wavefront (no cross-wave barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The likelihood pass in float32 arithmetic for what only the gradient uses,
// float64 sums, and float64 wherever a float32 rounding would be the same in
// many voxels.  lnP adds ~N^3 terms up to ~1e8, so a rounding error shared by
// many voxels is multiplied by their number, and it changes at random when
// the state moves (~1 in lnP at 512^3: enough to bias Metropolis decisions).
// Two such sources:
//  * beta and n alone: all voxels of a saturated web region share beta.  With
//      lnGamma(n+beta) - lnGamma(beta) = n ln beta + S,
//      S = sum_{1<=m<n} ln(1 + m/beta),
//    the per-voxel term is S + n ln nbar - (beta + n) ln(1 + nbar/beta) -
//    lnGamma(n+1) (the last depends on the counts alone and is summed once,
//    when they are set): n ln beta cancels, S vanishes for n <= 1 and is
//    taken in float64, and beta + n is formed in float64.
//  * ln nbar = ln C + log f rounded to float32: log f is itself a float32, so
//    in one binade every voxel's ln nbar rounds by the same ln C-dependent
//    amount r.  nbar = expf(float(ln nbar)) is used as it is, and
//    ln(1 + nbar/beta) gets the first-order correction r nbar/(beta + nbar)
//    in float64.
// Every other float32 rounding depends on the voxel's own nbar and averages
// out over voxels.
// S is needed only where n >= 2 and takes a loop over n, so each wavefront
// queues (n, beta) of those voxels in LDS rings of 128 slots and multiplies
// their factors once 64 are queued, one voxel per lane; counts up to 9 and
// counts from 10 to 64 have rings of their own, so that one long loop does
// not hold up a batch of short ones (the voxel loop runs in whole wavefronts
// for this; what is left is drained at the end).  Each lane keeps the product
// of all factors it has taken (LogProduct) and adds its logarithm once, at
// the end: the float64 logarithm per voxel would cost more than the rest of
// the pass.
// The gradient terms:
//   d lnP/d beta = [psi(n+beta) - psi(beta) - n/(beta+nbar)] + f(nbar/beta)
// (the same quantity as psi(n+beta) - psi(beta) - ln(1 + nbar/beta) +
// (nbar - n)/(beta + nbar), with the part that cancels to -x^2/2 for small
// x = nbar/beta evaluated by f) and g-hat in float32.  Counts above 64 take the
// float64 special functions in the lane.
__global__ __launch_bounds__(256) void likelihood32_kernel(LikeArgs a) {
  __shared__ double red[4];
  __shared__ int2 ring[4][2][128];
  const long long c = blockIdx.y;
  const long long nv = a.nv;
  const double lnc = a.scal[c * kScalStride + kScalLnC];
  const bool grad = a.ghat != nullptr;
  const int lane = threadIdx.x & 63;
  int2* qs = ring[threadIdx.x >> 6][0];   // 2 <= n <= 9
  int2* qb = ring[threadIdx.x >> 6][1];   // 10 <= n <= 64
  int hs = 0, ts = 0, hb = 0, tb = 0;     // heads and tails, wave-uniform
  LogProduct prod;
  double sl = 0.0, sg = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long wb = blockIdx.x * (long long)blockDim.x + (threadIdx.x & ~63); wb < nv; wb += stride) {
    const long long i = wb + lane;
    bool queue = false;
    int n = 0;
    float beta = 1.f;
    if (i < nv) {
      const float lf = a.logf[c * nv + i];
      beta = a.beta[c * nv + i];
      n = a.counts[c * nv + i];
      const float fn = (float)n;
      const double lnb = lnc + (double)lf;
      const float lnbf = (float)lnb;
      const float nb = expf(lnbf);
      const float x = nb / beta;
      const float l1p = log1pf(x);
      const float ib = 1.f / (beta + nb);
      const double l1pd = (double)l1p + (lnb - (double)lnbf) * (double)(nb * ib);
      double sv = 0.0;
      if (n > 64) sv = nb_lgamma_big_d(n, (double)beta) - (double)n * log((double)beta);
      else queue = n >= 2;
      sl += sv - ((double)beta + (double)n) * l1pd + (double)n * lnb;
      const float gh = beta * (fn - nb) * ib;
      sg += (double)gh;
      if (a.nbar) a.nbar[c * nv + i] = nb;
      if (grad) {
        // psi(n+beta) - psi(beta) = sum_{m<n} 1/(beta+m): per 8 terms one
        // division of the product's derivative by the product
        float db;
        if (n <= 64) {
          float sr = 0.f;
          for (int m0 = 0; m0 < n; m0 += 8) {
            float pq = 0.f, qq = 1.f;
            const int m1 = min(n, m0 + 8);
            for (int m = m0; m < m1; ++m) {
              const float bm = beta + (float)m;
              pq = fmaf(pq, bm, qq);
              qq *= bm;
            }
            sr += pq / qq;
          }
          // the first two terms are of one size with no more cancellation
          // than ~m/beta; f is the small-x-cancelling part
          db = (sr - fn * ib) + nb_cancel(x);
        } else {
          db = (float)(nb_digamma_big(n, (double)beta) - (double)l1p +
                       ((double)nb - (double)n) / ((double)beta + (double)nb));
        }
        a.ghat[c * nv + i] = gh;
        a.nbv[c * nv + i] = nb;
        a.dbeta[c * nv + i] = db;
      }
    }
    const bool small = queue && n <= 9;
    const unsigned long long ms = __ballot(small);
    const unsigned long long mb = __ballot(queue && !small);
    if (queue) {
      const unsigned long long mm = small ? ms : mb;
      const int rank = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mm, 0u));
      (small ? qs : qb)[((small ? ts : tb) + rank) & 127] = make_int2(n, __float_as_int(beta));
    }
    ts += __popcll(ms);
    tb += __popcll(mb);
    wave_lds_sync();
    if (ts - hs >= 64) {
      const int2 e = qs[(hs + lane) & 127];
      hs += 64;
      prod.rising_tail(e.x, __int_as_float(e.y));
    }
    if (tb - hb >= 64) {
      const int2 e = qb[(hb + lane) & 127];
      hb += 64;
      prod.rising_tail(e.x, __int_as_float(e.y));
    }
    wave_lds_sync();
  }
  if (lane < ts - hs) {
    const int2 e = qs[(hs + lane) & 127];
    prod.rising_tail(e.x, __int_as_float(e.y));
  }
  if (lane < tb - hb) {
    const int2 e = qb[(hb + lane) & 127];
    prod.rising_tail(e.x, __int_as_float(e.y));
  }
  sl += prod.log();
  const double s1 = block_sum(sl, red);
  const double s2 = block_sum(sg, red);
  if (threadIdx.x == 0) {
    a.partial[(c * gridDim.x + blockIdx.x) * 2 + 0] = s1;
    a.partial[(c * gridDim.x + blockIdx.x) * 2 + 1] = s2;
  }
}

// Per-voxel adjoint of bias, memberships and web tensors.  The bias-table
// gradient sum_i p_r,i dtheta_c,i is reduced through LDS: every pass of the
// block stores p (float) and dtheta (float64) of its 256 voxels, then thread t
// sums entry t % NE over a fixed subset of those voxels (fixed order, so the
// result is reproducible).
template <int W>
__global__ __launch_bounds__(256) void voxel_bwd_kernel(VoxelArgs a) {
  constexpr int R = W == 1 ? 4 : 16;
  constexpr int NE = R * 4;
  constexpr int G = 256 / NE;          // voxel groups per entry
  // rows padded to an odd stride: the reduce reads 16 (resp. 4) rows at one
  // column per instruction, which would otherwise fall in one LDS bank
  __shared__ float sp[R][257];
  __shared__ double sd[4][257];
  __shared__ __align__(16) float tab[NE];       // bias table in LDS (see voxel_fwd_kernel)
  const long long c = blockIdx.y;
  const long long nv = a.nv;
  if (threadIdx.x < NE) tab[threadIdx.x] = a.table[c * NE + threadIdx.x];
  __syncthreads();
  VoxelArgs b = a;
  for (int k = 0; k < 6 * W; ++k) b.tens[k] = a.tens[k] + c * nv;
  const double* sc = a.scal + c * kScalStride;
  const double gcoef = sc[kScalG] / sc[kScalNtr];
  const int t = threadIdx.x;
  const int my_e = t % NE, my_g = t / NE;
  double acc = 0.0;
  for (long long i0 = blockIdx.x * (long long)blockDim.x; i0 < nv; i0 += (long long)gridDim.x * blockDim.x) {
    const long long i = i0 + t;
    double dth[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < nv) {
      VoxelCore<W> v;
      const float rho = a.rho[c * nv + i];
      v.run(b, tab, i, rho);
#pragma unroll
      for (int r = 0; r < R; ++r) sp[r][t] = v.preg[r];
      // f dlogL/df = g-hat - (G / N_tr) nbar, in float64 for the sums
      const double af = (double)a.ghat[c * nv + i] - gcoef * (double)a.nbv[c * nv + i];
      dth[0] = af * (double)v.lnx;
      dth[1] = -af * (double)(v.u * v.ellr);
      dth[2] = af * (double)(v.u * v.theta[1] / v.theta[2]);
      dth[3] = (double)a.dbeta[c * nv + i];
      const float dxv = (float)af * ((v.theta[0] - v.theta[1] * v.u) / v.x);
      a.drho[c * nv + i] = rho > a.x_floor ? dxv : 0.f;
      // the membership cotangents only need float precision
      const float dt0 = (float)dth[0], dt1 = (float)dth[1], dt2 = (float)dth[2], dt3 = (float)dth[3];
      float dp[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float4 tr = reinterpret_cast<const float4*>(tab)[r];
        dp[r] = tr.x * dt0 + tr.y * dt1 + tr.z * dt2 + tr.w * dt3;
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
      float dpw[W][4];
      if (W == 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) dpw[0][r] = dp[r];
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float s0 = 0.f, s1 = 0.f;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            s0 += dp[4 * j + k] * v.pm[W - 1][k];
            s1 += dp[4 * k + j] * v.pm[0][k];
          }
          dpw[0][j] = s0;
          dpw[W - 1][j] = s1;
        }
      }
#pragma unroll
      for (int w = 0; w < W; ++w) {
        float gl[3];
        const float dw[3] = {dpw[w][1] - dpw[w][0], dpw[w][2] - dpw[w][1], dpw[w][3] - dpw[w][2]};
#pragma unroll
        for (int m = 0; m < 3; ++m) gl[m] = dw[m] * a.steep * v.wgt[w][m] * (1.f - v.wgt[w][m]);
        float gt[6];
        eig3_grad(v.v1[w], v.v3[w], gl, gt);
#pragma unroll
        for (int k = 0; k < 6; ++k) a.dtens[w * 6 + k][c * nv + i] = gt[k];
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) sp[r][t] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) sd[k][t] = dth[k];
    __syncthreads();
    {
      const int r = my_e >> 2, k = my_e & 3;
      double s = 0.0;
#pragma unroll 8
      for (int q = 0; q < NE; ++q) {
        const int vx = my_g + G * q;
        s += (double)sp[r][vx] * sd[k][vx];
      }
      acc += s;
    }
    __syncthreads();
  }
  double* sacc = &sd[0][0];   // free after the last pass
  sacc[t] = acc;
  __syncthreads();
  if (t < NE) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += sacc[g * NE + t];
    a.partial[(c * gridDim.x + blockIdx.x) * NE + t] = s;
  }
}

// Sum of per-block partials in a fixed order (one workgroup per chain).
// mode 0: sum f -> ln C; mode 1: (logL, G).
__global__ void finalize_kernel(FinalArgs a) {
  __shared__ double red[4];
  const long long c = blockIdx.x;
  double* sc = a.scal + c * kScalStride;
  if (a.mode == 0) {
    double s = 0.0;
    for (int i = threadIdx.x; i < a.nblk; i += blockDim.x) s += a.partial[c * a.nblk + i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
      sc[kScalSumF] = s;
      sc[kScalLnC] = log(sc[kScalNtr]) - log(s);
    }
  } else if (a.mode == 1) {
    double s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < a.nblk; i += blockDim.x) {
      s1 += a.partial[(c * a.nblk + i) * 2];
      s2 += a.partial[(c * a.nblk + i) * 2 + 1];
    }
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
      double logl = s1 - sc[kScalLgConst];
      if (a.flags[c] & FZW_NF_STATE) logl = __builtin_nan("");
      if (!isfinite(logl)) a.flags[c] |= FZW_NF_LOGL;
      sc[kScalLogL] = logl;
      sc[kScalG] = s2;
      if (a.logl) a.logl[c] = logl;
    }
  }
}

// Bias-table gradient: one workgroup per (entry, chain), fixed-order sum of
// the per-block partials.
__global__ void finalize_table_kernel(FinalArgs a) {
  __shared__ double red[4];
  const int e = blockIdx.x;
  const long long c = blockIdx.y;
  const int ne = a.ne;
  double s = 0.0;
  for (int i = threadIdx.x; i < a.nblk; i += blockDim.x) s += a.partial[(c * a.nblk + i) * ne + e];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    a.dtable[c * ne + e] = (float)s;
    if (!isfinite(s)) atomicOr(a.flags + c, FZW_NF_GRAD);
  }
}

void launch_voxel_fwd(int w, const VoxelArgs& a, int chains, int nblk, hipStream_t s) {
  dim3 g(nblk, chains);
  if (w == 1) hipLaunchKernelGGL(voxel_fwd_kernel<1>, g, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(voxel_fwd_kernel<2>, g, dim3(256), 0, s, a);
}
void launch_voxel_bwd(int w, const VoxelArgs& a, int chains, int nblk, hipStream_t s) {
  dim3 g(nblk, chains);
  if (w == 1) hipLaunchKernelGGL(voxel_bwd_kernel<1>, g, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(voxel_bwd_kernel<2>, g, dim3(256), 0, s, a);
}
void launch_likelihood(const LikeArgs& a, int chains, int nblk, bool fp64, hipStream_t s) {
  if (fp64) hipLaunchKernelGGL(likelihood_kernel, dim3(nblk, chains), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(likelihood32_kernel, dim3(nblk, chains), dim3(256), 0, s, a);
}
void launch_finalize(const FinalArgs& a, int chains, hipStream_t s) {
  if (a.mode == 2) hipLaunchKernelGGL(finalize_table_kernel, dim3(a.ne, chains), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(finalize_kernel, dim3(chains), dim3(256), 0, s, a);
}

// ------------------------------------------------------ data-only constants
__global__ void count_consts_kernel(const uint16_t* __restrict__ cnt, long long nv, double* partial) {
  __shared__ double red[4];
  double s0 = 0.0, s1 = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nv; i += (long long)gridDim.x * blockDim.x) {
    const double n = cnt[i];
    s0 += n;
    s1 += lgamma(n + 1.0);
  }
  const double a = block_sum(s0, red);
  const double b = block_sum(s1, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x * 2] = a;
    partial[blockIdx.x * 2 + 1] = b;
  }
}
__global__ void count_consts_final(const double* partial, int nblk, double* sc) {
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nblk; ++i) {
      a += partial[2 * i];
      b += partial[2 * i + 1];
    }
    sc[kScalNtr] = a;
    sc[kScalLgConst] = b;
  }
}
void launch_count_consts(const uint16_t* cnt, long long nv, double* partial, int nblk, double* scal, hipStream_t s) {
  hipLaunchKernelGGL(count_consts_kernel, dim3(nblk), dim3(256), 0, s, cnt, nv, partial);
  hipLaunchKernelGGL(count_consts_final, dim3(1), dim3(64), 0, s, partial, nblk, scal);
}

// ------------------------------------------------------------------ leapfrog
// p -= c (nu - dlogL/dnu)   (gradient of U = -logL + |nu|^2/2)
__global__ void kick_kernel(LeapArgs a, float frac) {
  const long long c = blockIdx.y;
  const float e = a.step[a.chain0 + c] * frac;
  const long long o = c * a.nv;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.nv; i += (long long)gridDim.x * blockDim.x)
    a.p[o + i] -= e * (a.q[o + i] - a.g[o + i]);
}
__global__ void drift_kernel(LeapArgs a, float frac) {
  const long long c = blockIdx.y;
  const float e = a.step[a.chain0 + c] * frac;
  const long long o = c * a.nv;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.nv; i += (long long)gridDim.x * blockDim.x)
    a.q[o + i] += e * a.minv[o + i] * a.p[o + i];
}
// sum nu^2 / 2 + sum minv p^2 / 2 per block
__global__ void energy_kernel(LeapArgs a) {
  __shared__ double red[4];
  const long long c = blockIdx.y;
  const long long o = c * a.nv;
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.nv; i += (long long)gridDim.x * blockDim.x) {
    const double q = a.q[o + i], p = a.p[o + i];
    s += 0.5 * q * q + 0.5 * (double)a.minv[o + i] * p * p;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) a.partial[c * gridDim.x + blockIdx.x] = s;
}
void launch_kick(const LeapArgs& a, int chains, float frac, hipStream_t s) {
  hipLaunchKernelGGL(kick_kernel, dim3(grid_for(a.nv, 256, 4096), chains), dim3(256), 0, s, a, frac);
}
void launch_drift(const LeapArgs& a, int chains, float frac, hipStream_t s) {
  hipLaunchKernelGGL(drift_kernel, dim3(grid_for(a.nv, 256, 4096), chains), dim3(256), 0, s, a, frac);
}
void launch_energy(const LeapArgs& a, int chains, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel, dim3(nblk, chains), dim3(256), 0, s, a);
}

// Free bias parameters: one workgroup per chain.
//   mode 0: table = base with tied entries sign * exp(u)
//   mode 1: half kick of p_u with frac * step
//   mode 2: drift of u with frac * step
//   mode 3: Hamiltonian: H = -logL + field energy partials + prior + kinetic(u)
__global__ void params_kernel(ParamArgs a, int mode, float frac, int nblk_energy, double* hout) {
  const int c = blockIdx.x;
  const int ne = a.ne, nf = a.nfree;
  float* u = a.u + c * nf;
  float* pu = a.pu + c * nf;
  const float* mi = a.minv_u + c * nf;
  if (mode == 0) {
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      const int f = a.tie[e];
      a.table[c * ne + e] = f >= 0 ? a.sign[f] * expf(u[f]) : a.base[c * ne + e];
    }
  } else if (mode == 1) {
    const float e = a.step[c] * frac;
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
      double g = 0.0;
      for (int k = 0; k < ne; ++k)
        if (a.tie[k] == f) g += (double)a.dtable[c * ne + k] * (double)a.table[c * ne + k];
      const double du = -g + ((double)u[f] - a.mu[f]) / (a.sigma[f] * a.sigma[f]);
      pu[f] -= e * (float)du;
    }
  } else if (mode == 2) {
    const float e = a.step[c] * frac;
    for (int f = threadIdx.x; f < nf; f += blockDim.x) u[f] += e * mi[f] * pu[f];
  } else {
    if (threadIdx.x == 0) {
      double h = -a.scal[c * kScalStride + kScalLogL];
      for (int i = 0; i < nblk_energy; ++i) h += a.epartial[c * nblk_energy + i];
      for (int f = 0; f < nf; ++f) {
        const double d = (double)u[f] - a.mu[f];
        h += d * d / (2.0 * a.sigma[f] * a.sigma[f]);
        h += 0.5 * (double)mi[f] * (double)pu[f] * (double)pu[f];
      }
      hout[c] = h;
      if (!isfinite(h)) a.flags[c] |= FZW_NF_HAMILTONIAN;
    }
  }
}
void launch_params(const ParamArgs& a, int chains, int mode, float frac, int nblk_energy, double* hout,
                   hipStream_t s) {
  hipLaunchKernelGGL(params_kernel, dim3(chains), dim3(64), 0, s, a, mode, frac, nblk_energy, hout);
}

__global__ void trace3_kernel(const float* a, const float* b, const float* c, float* out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = a[i] + b[i] + c[i];
}
void launch_trace3(const float* a, const float* b, const float* c, float* out, long long n, hipStream_t s) {
  hipLaunchKernelGGL(trace3_kernel, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, a, b, c, out, n);
}

// Wiener-filter start (Section 2.2 initialisation).  Tracer contrast
// delta_tr = n N^3 / N_tr - 1 per chain (grid.y = chain).
__global__ void wiener_contrast_kernel(const uint16_t* __restrict__ counts, const double* __restrict__ scal,
                                       int chain0, long long nv, float* __restrict__ out) {
  const long long c = blockIdx.y;
  const double scale = (double)nv / scal[(chain0 + c) * kScalStride + kScalNtr];
  const uint16_t* cn = counts + c * nv;
  float* o = out + c * nv;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nv; i += (long long)gridDim.x * blockDim.x)
    o[i] = (float)((double)cn[i] * scale - 1.0);
}
// nu_hat = h / (h^2 + 1/nbar) delta_tr_hat / N^3 on the padded half spectrum
// [n][n][pitch] (the 1/N^3 of the inverse transform folded in); h is the
// white-noise filter tabulated by integer |n|^2.
__global__ void wiener_filter_kernel(float2* __restrict__ spec, const float* __restrict__ htab, int n, int pitch,
                                     const double* __restrict__ scal, int chain0, long long nv, long long per_chain) {
  const long long c = blockIdx.y;
  const double inv_nbar = (double)nv / scal[(chain0 + c) * kScalStride + kScalNtr];
  const int m1 = n / 2 + 1;
  float2* sp = spec + c * per_chain;
  const long long rows = (long long)n * n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < rows * m1; i += (long long)gridDim.x * blockDim.x) {
    const long long r = i / m1;
    const int z = (int)(i - r * m1);
    const int x = (int)(r / n), y = (int)(r - (long long)x * n);
    const int nx = x <= n / 2 ? x : x - n, ny = y <= n / 2 ? y : y - n;
    const float h = htab[nx * nx + ny * ny + z * z];
    const double f = h > 0.f ? (double)h / ((double)h * h + inv_nbar) / (double)nv : 0.0;
    float2& v = sp[r * pitch + z];
    v.x = (float)(v.x * f);
    v.y = (float)(v.y * f);
  }
}
void launch_wiener_contrast(const uint16_t* counts, const double* scal, int chain0, int chains, long long nv,
                            float* out, hipStream_t s) {
  hipLaunchKernelGGL(wiener_contrast_kernel, dim3(grid_for(nv, 256, 4096), chains), dim3(256), 0, s, counts, scal,
                     chain0, nv, out);
}
void launch_wiener_filter(float2* spec, const float* htab, int n, int pitch, const double* scal, int chain0,
                          int chains, long long per_chain, hipStream_t s) {
  const long long nv = (long long)n * n * n;
  hipLaunchKernelGGL(wiener_filter_kernel, dim3(grid_for((long long)n * n * (n / 2 + 1), 256, 4096), chains),
                     dim3(256), 0, s, spec, htab, n, pitch, scal, chain0, nv, per_chain);
}

// Copy of a padded half spectrum into the dense [n][n][n/2+1] layout and back.
__global__ void spec_repack_kernel(const float2* __restrict__ src, float2* __restrict__ dst, int n, int sp, int dp,
                                   long long rows) {
  const int m1 = n / 2 + 1;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < rows * m1; i += (long long)gridDim.x * blockDim.x) {
    const long long r = i / m1;
    const int k = (int)(i - r * m1);
    dst[r * dp + k] = src[r * sp + k];
  }
}
void launch_spec_repack(const float2* src, float2* dst, int n, int sp, int dp, long long rows, hipStream_t s) {
  hipLaunchKernelGGL(spec_repack_kernel, dim3(grid_for(rows * (n / 2 + 1), 256, 16384)), dim3(256), 0, s, src, dst, n,
                     sp, dp, rows);
}

}  // namespace fzw
