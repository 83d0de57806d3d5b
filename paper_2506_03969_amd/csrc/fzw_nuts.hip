// Kernels of the no-U-turn transition (Section 2.2; multinomial NUTS with the
// generalised U-turn criterion of Betancourt 2017) for batches of chains that
// advance in lock step: every doubling and every leaf is one set of launches
// for all chains, and a chain whose trajectory has ended is carried along with
// a zero step.  State vectors hold the field part of every chain (packed like
// nu) followed by the free parameters ([chains][n_free]).
//
// Per leaf: one step of the plan's splitting scheme (kick, drift, gradient,
// ..., kick; kick-drift-kick by default), energy partials, one scalar kernel
// per chain (divergence, multinomial weight, progressive candidate choice),
// then one pass that adds the leaf to the subtree's momentum sum, copies the
// candidate, writes the block-start checkpoints and forms the dot products of
// the U-turn checks of every aligned block that ends at the leaf.
//
// Checkpoints: a leaf k that starts aligned blocks (k even) stores its
// momentum and the subtree's momentum sum before it in slot popcount(k); the
// blocks alive at any leaf start at distinct popcounts, so max_depth slots
// suffice.  The sum over a block [i, k] is then rho(k) - rho_before(i).
#include "fzw_device.hpp"
#include "fzw_ops.hpp"

namespace fzw {

namespace {

constexpr int kNutsThreads = 256;

__device__ __forceinline__ double log_add(double a, double b) {
  if (a == -HUGE_VAL) return b;
  if (b == -HUGE_VAL) return a;
  const double m = fmax(a, b);
  return m + log(exp(a - m) + exp(b - m));
}

// Writes the block's partial sums of `nv` values (fixed order: waves, then
// waves within the block) to partial[c][slot][0..nv).
template <int NV>
__device__ __forceinline__ void put_partials(const NutsVec& a, long long c, int slot, const double* v, double* red) {
  double* dst = a.partial + ((size_t)c * (kNutsBlk + 1) + slot) * a.nval;
  for (int i = 0; i < NV; ++i) {
    const double t = block_sum(v[i], red);
    if (threadIdx.x == 0) dst[i] = t;
  }
}

__global__ void __launch_bounds__(kNutsThreads) nuts_vec_kernel(NutsVec a, NutsSeg g, int op, float frac) {
  __shared__ double red[kNutsThreads / 64];
  const long long c = g.c0 + blockIdx.y;
  const NutsChain& st = a.st[c];
  const long long base = g.off + (long long)blockIdx.y * g.len;
  const float* minv = g.minv + (long long)blockIdx.y * g.len;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int slot = g.is_u ? kNutsBlk : (int)blockIdx.x;
  if (op == kNutsOpKick) {
    const float e = frac * st.se;
    if (e == 0.f) return;
    for (long long i = i0; i < g.len; i += stride) {
      const long long x = base + i;
      const float gr = g.is_u ? a.wg[x] : a.wq[x] - a.wg[x];
      a.wp[x] -= e * gr;
    }
  } else if (op == kNutsOpDrift) {
    const float e = frac * st.se;
    if (e == 0.f) return;
    for (long long i = i0; i < g.len; i += stride) {
      const long long x = base + i;
      a.wq[x] += e * minv[i] * a.wp[x];
    }
  } else if (op == kNutsOpEnergy) {
    double v[2] = {0.0, 0.0};
    for (long long i = i0; i < g.len; i += stride) {
      const long long x = base + i;
      const double q = a.wq[x], p = a.wp[x];
      if (!g.is_u) v[0] += 0.5 * q * q;
      v[1] += 0.5 * (double)minv[i] * p * p;
    }
    put_partials<2>(a, c, slot, v, red);
  } else if (op == kNutsOpInit) {
    const float* z = g.z + (long long)blockIdx.y * g.len;
    for (long long i = i0; i < g.len; i += stride) a.wp[base + i] = z[i] / sqrtf(minv[i]);
  } else if (op == kNutsOpStart) {
    for (long long i = i0; i < g.len; i += stride) {
      const long long x = base + i;
      const float q = a.wq[x], p = a.wp[x], gr = a.wg[x];
      a.lq[x] = q; a.lp[x] = p; a.lg[x] = gr;
      a.rq[x] = q; a.rp[x] = p; a.rg[x] = gr;
      a.cq[x] = q;
      a.rho_t[x] = p;
    }
  } else if (op == kNutsOpBegin) {
    if (!st.active) return;
    const float* eq = st.v > 0 ? a.rq : a.lq;
    const float* ep = st.v > 0 ? a.rp : a.lp;
    const float* eg = st.v > 0 ? a.rg : a.lg;
    for (long long i = i0; i < g.len; i += stride) {
      const long long x = base + i;
      a.wq[x] = eq[x];
      a.wp[x] = ep[x];
      a.wg[x] = eg[x];
      a.rho_s[x] = 0.f;
    }
  } else if (op == kNutsOpMerge) {
    if (!st.merged) return;
    float* eq = st.v > 0 ? a.rq : a.lq;
    float* ep = st.v > 0 ? a.rp : a.lp;
    float* eg = st.v > 0 ? a.rg : a.lg;
    double v[2] = {0.0, 0.0};
    for (long long i = i0; i < g.len; i += stride) {
      const long long x = base + i;
      const float p = a.wp[x];
      eq[x] = a.wq[x];
      ep[x] = p;
      eg[x] = a.wg[x];
      if (st.msel) a.cq[x] = a.sq[x];
      const float rt = a.rho_t[x] + a.rho_s[x];
      a.rho_t[x] = rt;
      const float pl = st.v > 0 ? a.lp[x] : p;
      const float pr = st.v > 0 ? p : a.rp[x];
      v[0] += (double)minv[i] * pl * rt;
      v[1] += (double)minv[i] * pr * rt;
    }
    put_partials<2>(a, c, slot, v, red);
  }
}

template <int NCHK>
__global__ void __launch_bounds__(kNutsThreads) nuts_leaf_kernel(NutsVec a, NutsSeg g, NutsLeafPlan lp) {
  __shared__ double red[kNutsThreads / 64];
  const long long c = g.c0 + blockIdx.y;
  const NutsChain& st = a.st[c];
  if (!st.leaf_ok) return;
  const long long base = g.off + (long long)blockIdx.y * g.len;
  const float* minv = g.minv + (long long)blockIdx.y * g.len;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int slot = g.is_u ? kNutsBlk : (int)blockIdx.x;
  const bool sel = st.sel != 0;
  double v[2 * NCHK + 1];
#pragma unroll
  for (int b = 0; b < 2 * NCHK; ++b) v[b] = 0.0;
  for (long long i = i0; i < g.len; i += stride) {
    const long long x = base + i;
    const float p = a.wp[x];
    const float before = a.rho_s[x];
    if (lp.store >= 0) {
      a.ckp[lp.store * a.tv + x] = p;
      a.ckr[lp.store * a.tv + x] = before;
    }
    const float rs = before + p;
    a.rho_s[x] = rs;
    if (sel) a.sq[x] = a.wq[x];
    const double m = minv[i];
#pragma unroll
    for (int b = 0; b < NCHK; ++b) {
      const long long o = lp.slot[b] * a.tv + x;
      const double rb = (double)(rs - a.ckr[o]);
      v[2 * b] += m * a.ckp[o] * rb;
      v[2 * b + 1] += m * p * rb;
    }
  }
  if (NCHK > 0) put_partials<2 * NCHK>(a, c, slot, v, red);
}

// dU/du of the free parameters (u = ln b) and their log-normal prior term, one
// workgroup per chain, from the bias-table gradient of the last evaluation.
__global__ void nuts_ugrad_kernel(NutsVec a, ParamArgs pa, long long uoff) {
  const int c = blockIdx.x;
  const int ne = pa.ne, nf = pa.nfree;
  const float* u = a.wq + uoff + (long long)c * nf;
  float* gu = a.wg + uoff + (long long)c * nf;
  for (int f = threadIdx.x; f < nf; f += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < ne; ++k)
      if (pa.tie[k] == f) s += (double)pa.dtable[c * ne + k] * (double)pa.table[c * ne + k];
    gu[f] = (float)(-s + ((double)u[f] - pa.mu[f]) / (pa.sigma[f] * pa.sigma[f]));
  }
  if (threadIdx.x == 0) {
    double pr = 0.0;
    for (int f = 0; f < nf; ++f) {
      const double d = (double)u[f] - pa.mu[f];
      pr += d * d / (2.0 * pa.sigma[f] * pa.sigma[f]);
    }
    a.st[c].prior = pr;
  }
}

// Sum of value `i` over a chain's partial slots (kNutsBlk field blocks, then
// the parameter block if any; fixed order); valid in thread 0.
__device__ double chain_sum(const NutsVec& a, int c, int i, double* red) {
  const double* src = a.partial + (size_t)c * (kNutsBlk + 1) * a.nval;
  double s = 0.0;
  const int nslot = kNutsBlk + (a.has_u ? 1 : 0);
  for (int t = threadIdx.x; t < nslot; t += blockDim.x) s += src[(size_t)t * a.nval + i];
  return block_sum(s, red);
}

__global__ void __launch_bounds__(kNutsThreads) nuts_scalar_kernel(NutsVec a, NutsScalarArgs sa, int mode, int j, int k,
                                                              int nchk) {
  __shared__ double red[kNutsThreads / 64];
  const int c = blockIdx.x;
  NutsChain& st = a.st[c];
  const float* uni = sa.uniforms + (size_t)c * sa.n_uniforms;
  if (mode == kNutsInit || mode == kNutsLeaf) {
    const double e0 = chain_sum(a, c, 0, red);
    const double e1 = chain_sum(a, c, 1, red);
    if (threadIdx.x != 0) return;
    const double u = -sa.scal[c * kScalStride + kScalLogL] + e0 + st.prior;
    const double h = u + e1;
    if (mode == kNutsInit) {
      st.h0 = h;
      st.u_cand = u;
      st.log_w = 0.0;
      st.acc_sum = 0.0;
      st.n_leaf = 0;
      st.depth = 0;
      st.diverging = 0;
      st.active = 1;
      st.sub_active = 0;
      st.merged = 0;
      st.msel = 0;
      st.leaf_ok = 0;
      st.sel = 0;
      st.eps = sa.step[c];
      st.se = 0.f;
      return;
    }
    if (!st.sub_active) {
      st.leaf_ok = 0;
      st.sel = 0;
      return;
    }
    st.n_leaf += 1;
    st.acc_sum += exp(fmin(0.0, st.h0 - h));
    if (!(h - st.h0 <= 1000.0)) {      // divergence (NaN included): the tree ends here
      st.diverging = 1;
      st.sub_active = 0;
      st.active = 0;
      st.se = 0.f;
      st.leaf_ok = 0;
      st.sel = 0;
      return;
    }
    st.u_leaf = u;
    st.log_ws = log_add(st.log_ws, st.h0 - h);
    const double r = (double)uni[2 * sa.max_depth + (1 << j) - 1 + k];
    st.sel = r < exp((st.h0 - h) - st.log_ws) ? 1 : 0;
    if (st.sel) st.u_sub = u;
    st.leaf_ok = 1;
    return;
  }
  if (mode == kNutsChecks) {
    if (!st.leaf_ok) return;
    bool turn = false;
    for (int b = 0; b < 2 * nchk; ++b) {
      const double d = chain_sum(a, c, b, red);
      if (threadIdx.x == 0 && !(d > 0.0)) turn = true;
    }
    if (threadIdx.x == 0 && turn) {
      st.sub_active = 0;
      st.active = 0;
      st.se = 0.f;
    }
    return;
  }
  if (mode == kNutsTree) {
    if (!st.merged) return;
    const double d1 = chain_sum(a, c, 0, red);
    const double d2 = chain_sum(a, c, 1, red);
    if (threadIdx.x == 0 && (!(d1 > 0.0) || !(d2 > 0.0) || j + 1 >= sa.max_depth)) st.active = 0;
    return;
  }
  if (threadIdx.x != 0) return;
  if (mode == kNutsBegin) {
    st.merged = 0;
    st.msel = 0;
    if (st.active) {
      st.v = uni[j] >= 0.5f ? 1 : -1;
      st.se = (float)st.v * st.eps;
      st.sub_active = 1;
      st.log_ws = -HUGE_VAL;
    } else {
      st.se = 0.f;
      st.sub_active = 0;
    }
  } else if (mode == kNutsJoin) {
    st.se = 0.f;
    if (st.active) {
      st.merged = 1;
      st.msel = (double)uni[sa.max_depth + j] < exp(fmin(0.0, st.log_ws - st.log_w)) ? 1 : 0;
      if (st.msel) st.u_cand = st.u_sub;
      st.log_w = log_add(st.log_w, st.log_ws);
      st.depth = j + 1;
    }
  } else if (mode == kNutsOut) {
    sa.potential[c] = st.u_cand;
    sa.accept_stat[c] = st.acc_sum / (double)(st.n_leaf > 0 ? st.n_leaf : 1);
    sa.stats[3 * c + 0] = st.depth;
    sa.stats[3 * c + 1] = st.n_leaf;
    sa.stats[3 * c + 2] = st.diverging;
  }
}

// One flag: does any chain still grow its tree (or its current subtree)?
__global__ void nuts_any_kernel(NutsVec a, int chains, int sub, int* out) {
  int any = 0;
  for (int c = threadIdx.x; c < chains; c += blockDim.x) any |= sub ? a.st[c].sub_active : a.st[c].active;
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) *out = any;
}

__global__ void welford_kernel(const float* __restrict__ x, float* mean, float* m2, long long n, float inv_count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float xv = x[i], m0 = mean[i];
    const float d = xv - m0;
    const float m1 = m0 + d * inv_count;
    mean[i] = m1;
    m2[i] += d * (xv - m1);
  }
}

__global__ void inv_mass_kernel(const float* __restrict__ m2, float* minv, long long n, double count) {
  const double w = count / (count + 5.0), sh = 1e-3 * 5.0 / (count + 5.0);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    minv[i] = (float)(w * ((double)m2[i] / (count - 1.0)) + sh);
}

unsigned blocks_for(long long n, unsigned cap) {
  long long b = (n + kNutsThreads - 1) / kNutsThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

void launch_nuts_vec(const NutsVec& a, const NutsSeg& g, int op, float frac, hipStream_t s) {
  // the field part always runs kNutsBlk blocks per chain, so that every
  // partial slot is written; the parameter part one block per chain
  const unsigned bx = g.is_u ? 1u : (unsigned)kNutsBlk;
  hipLaunchKernelGGL(nuts_vec_kernel, dim3(bx, g.nc), dim3(kNutsThreads), 0, s, a, g, op, frac);
}

template <int NCHK>
static void leaf_launch(const NutsVec& a, const NutsSeg& g, const NutsLeafPlan& lp, hipStream_t s) {
  const unsigned bx = g.is_u ? 1u : (unsigned)kNutsBlk;
  hipLaunchKernelGGL(nuts_leaf_kernel<NCHK>, dim3(bx, g.nc), dim3(kNutsThreads), 0, s, a, g, lp);
}

void launch_nuts_leaf(const NutsVec& a, const NutsSeg& g, const NutsLeafPlan& lp, hipStream_t s) {
  switch (lp.nchk) {
    case 0: leaf_launch<0>(a, g, lp, s); break;
    case 1: leaf_launch<1>(a, g, lp, s); break;
    case 2: leaf_launch<2>(a, g, lp, s); break;
    case 3: leaf_launch<3>(a, g, lp, s); break;
    case 4: leaf_launch<4>(a, g, lp, s); break;
    case 5: leaf_launch<5>(a, g, lp, s); break;
    case 6: leaf_launch<6>(a, g, lp, s); break;
    case 7: leaf_launch<7>(a, g, lp, s); break;
    case 8: leaf_launch<8>(a, g, lp, s); break;
    case 9: leaf_launch<9>(a, g, lp, s); break;
    case 10: leaf_launch<10>(a, g, lp, s); break;
    case 11: leaf_launch<11>(a, g, lp, s); break;
    default: leaf_launch<12>(a, g, lp, s); break;
  }
}

void launch_nuts_ugrad(const NutsVec& a, const ParamArgs& pa, long long uoff, int chains, hipStream_t s) {
  hipLaunchKernelGGL(nuts_ugrad_kernel, dim3(chains), dim3(64), 0, s, a, pa, uoff);
}

void launch_nuts_scalar(const NutsVec& a, const NutsScalarArgs& sa, int chains, int mode, int j, int k, int nchk,
                        hipStream_t s) {
  if (mode == kNutsAnyTree || mode == kNutsAnySub) {
    hipLaunchKernelGGL(nuts_any_kernel, dim3(1), dim3(kNutsThreads), 0, s, a, chains, mode == kNutsAnySub ? 1 : 0,
                       sa.any);
    return;
  }
  hipLaunchKernelGGL(nuts_scalar_kernel, dim3(chains), dim3(kNutsThreads), 0, s, a, sa, mode, j, k, nchk);
}

void launch_welford(const float* x, float* mean, float* m2, long long n, int count, hipStream_t s) {
  hipLaunchKernelGGL(welford_kernel, dim3(blocks_for(n, 16384)), dim3(kNutsThreads), 0, s, x, mean, m2, n,
                     1.0f / (float)count);
}

void launch_inv_mass(const float* m2, float* minv, long long n, int count, hipStream_t s) {
  hipLaunchKernelGGL(inv_mass_kernel, dim3(blocks_for(n, 16384)), dim3(kNutsThreads), 0, s, m2, minv, n, (double)count);
}

}  // namespace fzw
