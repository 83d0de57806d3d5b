/*
 * fzw.h: C ABI of the MI355X (gfx950) implementation of the differentiable
 * fuzzy-cosmic-web field-level likelihood (Rossello, Kitaura et al. 2025).
 *
 * Problem statement (Section 2.1): a forward model M maps a white-noise field
 * nu, bias parameters b and fixed cosmology to the expected tracer counts
 * nbar = M_b(M_Psi(M_delta(nu)), b); the data n* enter through the
 * negative-binomial likelihood of Section 2.7; the posterior adds a whitened
 * Gaussian prior on nu and log-normal priors on the bias (Eq. 'posterior',
 * Eq. 'lognormal') and is sampled with Hamiltonian Monte Carlo (Section 2.2).
 *
 * The stages, with the passages that define them:
 *   M_delta : delta_L = irfftn(h(k) rfftn(nu)), h = sqrt(P(k)/dx^3)   (Appendix A)
 *   M_Psi   : ALPT, Psi = K o Psi_2LPT + (1-K) o Psi_SC, Gaussian K of
 *             radius r_s (Section 2.3); particles start on the mesh nodes and
 *             are deposited with cloud-in-cell, optionally after a
 *             plane-parallel redshift-space shift (Section 2.9)
 *   M_b     : tidal tensors (Section 2.8, Appendix B), sorted eigenvalues,
 *             sigmoid weights (Eq. 'sigmoid'), memberships (Eq. 'soft_cweb_p'),
 *             per-voxel parameters interpolated over 4 or 16 regions (boxed
 *             equation of Section 2.8), bias x^alpha exp(-(x/rho)^eps)
 *             (Eq. 'local_bias', signed eps), normalisation sum nbar = N_tr
 *   logL    : sum of negative-binomial log-pmfs, Gamma(beta, nbar/beta) x
 *             Poisson (Section 2.7, Eq. 'log_likelihood'), constants included
 *
 * Conventions for every call:
 *   - Pointers marked (device) are device memory owned by the caller (for
 *     example allocated by PyTorch); the library never frees them and keeps no
 *     reference after the call returns.  (host) pointers are read during the
 *     call only.
 *   - Real fields are float32, C order [x][y][z] (z fastest), one N^3 block per
 *     chain, chains packed back to back in chain order (fzw_chain_offset).
 *   - A bias table is float32 [n_chains][R][4] with columns
 *     (alpha, eps, rho_th, beta_NB); R = 4 (one web) or 16 (two webs, region
 *     4*j + k for class j of web 0 and class k of web 1); classes are ordered
 *     void, sheet, filament, knot.
 *   - Log-likelihoods and Hamiltonians are float64 [n_chains].
 *   - Calls enqueue work on the plan's stream and return without waiting,
 *     except fzw_plan_create and fzw_set_counts, which synchronise.
 *   - A negative status means nothing was enqueued; fzw_last_error() returns a
 *     message (thread-local, valid until the next call on the same thread).
 *     FZW_E_HIP leaves the plan unusable: destroy it.
 *   - Non-finite results are not errors: logL or H = NaN or +-inf is written,
 *     the chain's non-finite flags are set (fzw_nonfinite_flags) and the
 *     caller's Metropolis step rejects.  A state whose displacement field is
 *     not finite (or moves a particle by 2^30 cells or more) is invalid: its
 *     particles are deposited without displacement, so that no index or
 *     weight is undefined, and its logL is NaN.
 */
#ifndef FZW_H_
#define FZW_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FZW_OK = 0,
  FZW_E_ARG = -1,    /* invalid argument (null pointer, out-of-range value) */
  FZW_E_SIZE = -2,   /* unsupported mesh size */
  FZW_E_HIP = -3,    /* a HIP runtime call failed */
  FZW_E_OOM = -4,    /* workspace allocation failed; the plan is not created */
  FZW_E_STATE = -5,  /* call out of order (e.g. counts not set) */
  FZW_W_NONFINITE = 1 /* fzw_check_finite: some chain's last result was not finite */
} fzw_status;

/* Bits of the per-chain non-finite flags. */
enum {
  FZW_NF_STATE = 1,       /* a displacement was not finite or too large: logL set to NaN */
  FZW_NF_LOGL = 2,        /* the log-likelihood was not finite */
  FZW_NF_GRAD = 4,        /* an entry of the bias-table gradient was not finite */
  FZW_NF_HAMILTONIAN = 8  /* H at the start or end of a trajectory was not finite */
};

enum { FZW_WEB_PHI = 0, FZW_WEB_DELTA = 1 };

/* rsd_axis value for radial redshift-space distortions (Section 2.9): each
   particle moves along the ray from an observer at the box centre by the
   line-of-sight component of f Psi, measured from its unwrapped real-space
   position node + Psi; no shift where that position is the centre itself. */
enum { FZW_RSD_RADIAL = 3 };

/* Cosmology and gravity-solver settings, fixed for a plan (Section 2.1). */
typedef struct {
  double omega_m, h, sigma8, n_s; /* BBKS linear spectrum normalised to sigma8 */
  double d1;                      /* linear growth factor at the output time */
  double f_growth;                /* growth rate used by the RSD shift */
  double r_s;                     /* ALPT Gaussian smoothing radius [Mpc/h] */
  int rsd_axis;                   /* -1 real space; 0,1,2 plane-parallel line of sight along
                                     that axis; FZW_RSD_RADIAL radial about an observer at
                                     the box centre (Section 2.9) */
  double tau_sc;                  /* width of a smooth spherical-collapse hinge, 0 = exact */
  double x_floor;                 /* floor applied to 1+delta inside the bias */
} fzw_cosmo;

/* Fuzzy cosmic-web settings (Section 2.8). */
typedef struct {
  int n_webs;        /* 1: Phi-web (4 regions); 2: Phi-web x delta-web (16 regions) */
  int kind[2];       /* FZW_WEB_PHI: tensor of Phi = lap^-1 delta;
                        FZW_WEB_DELTA: -ell^2 times the Hessian of delta */
  double smooth_r[2];/* Gaussian smoothing radius of each web's field [Mpc/h] */
  double ell[2];     /* scale of the delta-web tensor [Mpc/h] */
  double steepness;  /* sigmoid steepness s */
  double lambda_th;  /* eigenvalue threshold */
} fzw_web;

typedef struct fzw_plan fzw_plan;

/* Create a plan for n_chains independent chains.  mesh_n[c] in
 * {16,32,64,96,128,256,512}, box_l[c] > 0 (host arrays).  Chains with equal
 * (mesh_n, box_l) that are adjacent in chain order are batched into single
 * launches.  `stream` is a hipStream_t (NULL = default stream).  Allocates
 * the workspace (fzw_workspace_bytes) and computes the spectral tables. */
fzw_status fzw_plan_create(fzw_plan** out, int n_chains, const int* mesh_n, const double* box_l,
                           const fzw_cosmo* cosmo, const fzw_web* web, void* stream);

/* fzw_plan_create with options (flags = 0 is fzw_plan_create).
 * FZW_PLAN_CHECKPOINT: displacement-field checkpointing for large meshes.
 *   The workspace holds no first-order Hessian phi_ij (6 fields per chain,
 *   and no real-space S2 and d_SC where the LPT step is fused with its z
 *   transforms, i.e. every mesh but 96): the forward model keeps the
 *   displacement Psi, the density and the per-voxel fields, and a gradient
 *   evaluation recomputes phi_ij from nu before the adjoint of the LPT step,
 *   with the forward model's own kernels on the same input, so every result
 *   equals that of a plan without checkpointing bit for bit.  Cost: one more
 *   r2c of nu and the passes that form phi_ij per gradient.  fzw_get_field
 *   field 0 (delta_L, the trace of phi) is then never available.
 * Unknown flags give FZW_E_ARG. */
enum { FZW_PLAN_CHECKPOINT = 1 };
fzw_status fzw_plan_create_ex(fzw_plan** out, int n_chains, const int* mesh_n, const double* box_l,
                              const fzw_cosmo* cosmo, const fzw_web* web, void* stream, unsigned flags);
void fzw_plan_destroy(fzw_plan* plan);

/* Copy the observed counts n* of one chain (device, uint16, N^3, C order)
 * into the plan; also precomputes N_tr and the data-only constant
 * sum_i lnGamma(n*_i + 1) in float64.  Synchronises. */
fzw_status fzw_set_counts(fzw_plan* plan, int chain, const uint16_t* counts);

/* Forward model and log-likelihood for every chain.
 *   nu    (device) float32 white noise, packed chains
 *   bias  (device) float32 [n_chains][R][4]
 *   nbar  (device, may be NULL) float32 expected counts, packed chains
 *   logl  (device) float64 [n_chains]
 * The negative-binomial pass runs in float32 per voxel with float64 sums, and
 * in float64 wherever a rounding would be shared by many voxels (such errors
 * add up coherently and move logl by O(1) at 512^3 between nearby states); the
 * environment variable FZW_LIKELIHOOD_FP64=1, read at fzw_plan_create, runs
 * it in float64 per voxel instead.  fzw_forward and fzw_value_and_grad give
 * the same logl bit for bit. */
fzw_status fzw_forward(fzw_plan* plan, const float* nu, const float* bias, float* nbar, double* logl);

/* Forward model, log-likelihood and its gradient by the hand-written adjoint.
 *   dlogl_dnu   (device) float32, packed chains
 *   dlogl_dbias (device) float32 [n_chains][R][4] */
fzw_status fzw_value_and_grad(fzw_plan* plan, const float* nu, const float* bias, double* logl,
                              float* dlogl_dnu, float* dlogl_dbias);

/* Free bias parameters for HMC: n_free parameters shared by all chains.
 * tie (host, int [R*4]) maps each table entry to a free-parameter index or -1
 * (entry stays at its base value); a free parameter is sampled as u = ln b
 * (u = ln |b| with fzw_set_sampling_signs).
 * prior_mu, prior_sigma (host, double [n_free]) are the log-normal
 * hyper-parameters (Eq. 'lognormal').  n_free <= 64. */
fzw_status fzw_set_sampling(fzw_plan* plan, const int* tie, int n_free, const double* prior_mu,
                            const double* prior_sigma);

/* Signs of the free parameters (host, int [n_free], each +1 or -1; n_free as
 * given to fzw_set_sampling, which resets every sign to +1): a free parameter
 * is sign * exp(u), so a signed entry such as a negative exponential-cut-off
 * exponent (the low-density cut-off of Eq. 'local_bias') can be sampled with a
 * log-normal prior on its magnitude.  Used for the full 64-parameter table of
 * the 16-region model. */
fzw_status fzw_set_sampling_signs(fzw_plan* plan, const int* sign, int n_free);

/* One kick-drift-kick leapfrog trajectory of n_steps steps per chain, on the
 * potential U = -logL + |nu|^2/2 + sum_f (u_f - mu_f)^2/(2 sigma_f^2), with a
 * diagonal inverse mass matrix.  All arrays (device):
 *   nu, p_nu, minv_nu  float32 packed chains (nu and p_nu updated in place)
 *   u, p_u, minv_u     float32 [n_chains][n_free] (updated in place)
 *   bias_base          float32 [n_chains][R][4] (values of the non-free entries)
 *   step               float32 [n_chains]
 *   h_start, h_end     float64 [n_chains]: H = U + p^T M^-1 p / 2
 * The trajectory is captured once as a HIP graph per distinct argument set and
 * replayed.  Accept/reject is left to the caller. */
fzw_status fzw_leapfrog(fzw_plan* plan, float* nu, float* u, float* p_nu, float* p_u,
                        const float* bias_base, const float* minv_nu, const float* minv_u,
                        const float* step, int n_steps, double* h_start, double* h_end);

/* One no-U-turn transition per chain (Section 2.2: the paper samples with
 * NUTS; implemented after Hoffman & Gelman 2014 with multinomial selection and
 * the generalised U-turn criterion of Betancourt 2017) on the potential of
 * fzw_leapfrog.  The trajectory doubles in a drawn direction until the tree
 * or a new subtree turns (a turning or diverging subtree, H - H0 > 1000, is
 * discarded), or max_depth doublings are joined; the new state is drawn from
 * the leaves with weights exp(-H) (uniformly within a subtree, with
 * probability min(1, W_subtree / W_tree) when the subtree is joined).
 * All chains advance in lock step; a chain whose trajectory has ended idles.
 * Each leaf is one step of the plan's splitting scheme (fzw_set_integrator;
 * kick-drift-kick by default).
 * All arrays are device memory:
 *   nu, u              float32 state (packed chains; [n_chains][n_free]),
 *                      replaced by the new state
 *   z_nu, z_u          float32 standard normal draws, same layouts: the
 *                      momentum is p = z / sqrt(minv)
 *   bias_base, minv_nu, minv_u, step   as in fzw_leapfrog
 *   uniforms           float32 [n_chains][2 max_depth + 2^max_depth - 1]
 *                      draws in [0, 1): the direction of each doubling
 *                      (>= 0.5 forward), the join of each doubling, then one
 *                      per leaf in the order the leaves are made
 *   max_depth          1 .. FZW_NUTS_MAX_DEPTH
 *   potential          float64 [n_chains]: U at the new state
 *   accept_stat        float64 [n_chains]: mean of min(1, exp(H0 - H)) over
 *                      the leaves made (the statistic step-size adaptation
 *                      uses)
 *   stats              int32 [n_chains][3]: doublings joined, leapfrog steps
 *                      taken, divergence flag
 * The plan keeps (13 + 2 max_depth) float32 state vectors of the size of
 * nu + u, allocated at the first call.  The caller's stream is synchronised
 * once per doubling (the loop stops when every chain's trajectory has ended),
 * so the call returns with the transition complete. */
#define FZW_NUTS_MAX_DEPTH 12
fzw_status fzw_nuts(fzw_plan* plan, float* nu, float* u, const float* z_nu, const float* z_u,
                    const float* bias_base, const float* minv_nu, const float* minv_u, const float* step,
                    const float* uniforms, int max_depth, double* potential, double* accept_stat,
                    int* stats);

/* Warm-up helpers for a diagonal mass matrix (device arrays of n floats, on
 * the plan's stream).  fzw_welford adds sample number `count` (1-based) x to
 * the running mean and sum of squared deviations m2 (Welford 1962; start from
 * zeros).  fzw_inverse_mass writes the inverse mass from a window of count >= 2
 * samples: (count/(count+5)) m2/(count-1) + 1e-3 * 5/(count+5), the
 * regularised variance of Stan's windowed adaptation. */
fzw_status fzw_welford(fzw_plan* plan, const float* x, float* mean, float* m2, long long n, int count);
fzw_status fzw_inverse_mass(fzw_plan* plan, const float* m2, float* minv, long long n, int count);

/* Step-size adaptation by dual averaging (Hoffman & Gelman 2014, Sec. 3.2),
 * host only: init with the first step size and the target mean acceptance
 * statistic (0.8 in common use), update after every warm-up transition with
 * its accept_stat (returns the next step size), and take the averaged step
 * from fzw_dual_avg_final after warm-up.  gamma 0.05, t0 10, kappa 0.75,
 * mu = log(10 eps0). */
typedef struct {
  double mu, target, gamma, t0, kappa, h_bar, log_eps_bar;
  long long t;
} fzw_dual_avg;
void fzw_dual_avg_init(fzw_dual_avg* state, double eps0, double target);
double fzw_dual_avg_update(fzw_dual_avg* state, double accept_stat);
double fzw_dual_avg_final(const fzw_dual_avg* state);

/* Deterministic starting point of every chain (Section 2.2 initialisation):
 * the tracer contrast delta_tr = n N^3 / N_tr - 1 of the counts set with
 * fzw_set_counts, Wiener-filtered with the plan's linear spectrum and Poisson
 * shot noise 1/nbar per cell (nbar = N_tr / N^3), peculiar motions ignored,
 * and mapped back to white noise: nu_hat = h / (h^2 + 1/nbar) rfft(delta_tr)
 * with h = sqrt(P/dx^3) and nu_hat(0) = 0.  nu: device float32, packed like
 * the state of fzw_value_and_grad (written).  FZW_E_STATE if counts are
 * missing. */
fzw_status fzw_wiener_start(fzw_plan* plan, float* nu);

/* Validation statistics of fields on one of the plan's meshes (Section 4).
 * Both overwrite the plan's intermediate fields of that mesh (fzw_get_field
 * is then stale) and run on the caller's stream.
 *
 * fzw_power_multipoles: monopole and quadrupole of the auto (b = NULL) or
 * cross spectrum of real float32 fields a, b (device, N^3, C order), with
 * respect to a plane-parallel line of sight along z:
 *   P_l(k) = (2l+1) < P(k) L_l(mu) >_shell,  mu = k_z / k,
 *   P(k) = dx^3 / N^3 Re(a_k conj(b_k)) per rfft mode,
 * over shells [k_lo + i dk, k_lo + (i+1) dk), i < nbins <= 256; a half-
 * spectrum mode with 0 < n_z < N/2 counts twice.  out: device float64
 * [nbins][4] = (mean |k|, modes, P0, P2).  Cross-correlation and propagator
 * follow as P_ab / sqrt(P_aa P_bb) and P_ab / P_bb.
 *
 * fzw_bispectrum: bispectrum B and reduced bispectrum
 * Q = B / (P1 P2 + P2 P3 + P3 P1) of a real float32 field (device, N^3) by the
 * FFT estimator over shells of width dk centred on k1, k2 and
 * k3 = sqrt(k1^2 + k2^2 + 2 k1 k2 cos theta) for each opening angle theta
 * (host float64 [ntheta], ntheta <= 256):
 *   B = dx^6 / N^3 * sum_x I1 I2 I3 / sum_x J1 J2 J3,
 * I_i the inverse DFT of the field's spectrum on shell i, J_i that of the
 * shell's indicator.  out: device float64 [ntheta][4] = (k3, B, Q, closed
 * triangles).  Returns after the stream has finished. */
fzw_status fzw_power_multipoles(fzw_plan* plan, int mesh_n, const float* a, const float* b, double k_lo, double dk,
                                int nbins, double* out);
fzw_status fzw_bispectrum(fzw_plan* plan, int mesh_n, const float* delta, double k1, double k2, double dk,
                          int ntheta, const double* theta, double* out);

/* fzw_power_multipoles for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same kernels and the same results bit for bit,
 * but the call allocates nothing.  Its workgroups' partial sums go to a fixed
 * device array of 4 MiB per GPU (512 workgroups x 256 bins x 4 float64),
 * held by the library until the process ends, whose address is resolved when
 * the first plan is created on that GPU; the transforms use the plan's own
 * workspace.  nbins <= 256 (FZW_E_ARG above).  Every call on one GPU shares
 * that array and every partial is written before it is read, so nothing
 * needs clearing; calls that overlap on one GPU (other streams or threads,
 * other plans) race on it and must be serialised by the caller.  No timing
 * records are made (fzw_timing_enable does not apply). */
fzw_status fzw_power_multipoles_noalloc(fzw_plan* plan, int mesh_n, const float* a, const float* b, double k_lo,
                                        double dk, int nbins, double* out);

/* Splitting scheme of fzw_leapfrog's steps (Section 2.2 names second- and
 * fourth-order HMC and the variant of Blanes, Casas & Sanz-Serna 2014).  One
 * step with step size eps is K(a_0) D(b_1) K(a_1) ... D(b_m) K(a_m), K(a) the
 * kick p -= a eps dU/dq, D(b) the drift q += b eps M^-1 p:
 *   FZW_INT_LEAPFROG  a = (1/2, 1/2), b = (1): one gradient per step (default)
 *   FZW_INT_BLANES2   a = (0.21178, 0.57644, 0.21178), b = (1/2, 1/2): two
 *   FZW_INT_YOSHIDA4  three leapfrog steps of w1, w0, w1 eps with
 *                     w1 = 1/(2 - 2^(1/3)), w0 = 1 - 2 w1 (fourth order): three
 * Applies to later fzw_leapfrog calls (each scheme has its own graph) and
 * to the leaves of fzw_nuts (one step of the scheme per leaf). */
enum { FZW_INT_LEAPFROG = 0, FZW_INT_BLANES2 = 1, FZW_INT_YOSHIDA4 = 2 };
fzw_status fzw_set_integrator(fzw_plan* plan, int kind);

/* Per-chain non-finite flags (FZW_NF_* bits) of the last evaluation call:
 * fzw_forward, fzw_value_and_grad, fzw_leapfrog (every gradient of the
 * trajectory and both Hamiltonians) or fzw_nuts (every leaf, rejected ones
 * included).  Each of these calls clears the flags first.
 * fzw_nonfinite_flags enqueues a copy into `flags` (device, int32
 * [n_chains]) on the plan's stream and returns at once.
 * fzw_check_finite synchronises the plan's stream, copies the flags into
 * `flags_host` (host int32 [n_chains], may be NULL) and returns
 * FZW_W_NONFINITE if any chain has a flag set, else FZW_OK. */
fzw_status fzw_nonfinite_flags(fzw_plan* plan, int* flags);
fzw_status fzw_check_finite(fzw_plan* plan, int* flags_host);

/* Copy an intermediate field of the last evaluation (device destination,
 * float32 N^3 of one chain).
 * After fzw_forward: 0 delta_L, 1 Psi_x, 2 Psi_y, 3 Psi_z (displacement,
 * Mpc/h), 4 rho (CIC density, mean 1), 5 log f (log of the unnormalised
 * bias), 6..11 tensor of web 0 (xx,yy,zz,xy,xz,yz), 12..17 web 1.
 * A gradient evaluation (fzw_value_and_grad, fzw_leapfrog, fzw_nuts) reuses
 * the displacement and tensor buffers for their cotangents: afterwards
 * fields 4 and 5 (and 0 on meshes with the fused LPT kernels, all but 96)
 * are still those of its last forward model, 1-3 and 6-17 are not, and the
 * adjoint's cotangents are available instead:
 *   FZW_FIELD_DRHO   d logL / d rho (the density cotangent, both web terms
 *                    and the direct bias term)
 *   FZW_FIELD_DPSI+j d logL / d Psi_j per particle (j = 0, 1, 2; the
 *                    particle of lattice node i at index i)
 * A field that the last call did not leave gives FZW_E_STATE (so does any
 * field before the first evaluation, and field 0 after fzw_bispectrum,
 * which uses its buffers).  FZW_E_ARG for a field the plan does not have. */
enum { FZW_FIELD_DRHO = 18, FZW_FIELD_DPSI = 19 };
fzw_status fzw_get_field(fzw_plan* plan, int chain, int field, float* out);

/* Standalone batched 3-D FFTs on the plan's stream (for testing and reuse).
 * r2c: real (device) [batch][n^3] -> half spectrum (device) complex64
 * [batch][n][n][n/2+1] (unnormalised).  c2r: the inverse, unnormalised
 * (returns n^3 times the input field).  Uses internal scratch of the plan;
 * n must be one of the plan's mesh sizes. */
fzw_status fzw_fft_r2c(fzw_plan* plan, int n, int batch, const float* in, void* out_complex);
fzw_status fzw_fft_c2r(fzw_plan* plan, int n, int batch, const void* in_complex, float* out);

/* Cloud-in-cell deposit method.  Both give bit-identical densities: every
 * weight is rounded to a multiple of 2^-32 and summed exactly in 64-bit
 * integers, so neither depends on the order of particles.
 *   FZW_CIC_SORTED (default): counting sort of the particles by destination
 *     cell, then each node gathers the weights of the particles in its 8
 *     neighbouring buckets (no atomics on the densities).
 *   FZW_CIC_ATOMIC: each particle adds its 8 weights with 64-bit integer
 *     atomics into a fixed-point accumulator. */
enum { FZW_CIC_SORTED = 0, FZW_CIC_ATOMIC = 1 };
fzw_status fzw_set_cic_method(fzw_plan* plan, int method);

/* FFT kernel schedule of a mesh size (process-wide).  The first plan created
 * for a mesh size times, on its own buffers, the two kernel families of each
 * pass type -- register four-step (0) and LDS Stockham (1) for the z passes
 * and the mixing x/y passes; persistent four-step (0) or the mixing kernel (1)
 * for pure x/y transforms -- and keeps the four-step kernels unless the
 * alternative is at least 10% faster.  Every later plan of that size uses the
 * same kernels, so results of plans in one process are comparable bit for
 * bit.  Two processes may choose differently where the two families' times
 * lie within timing noise of the 10% margin (small meshes: 7.7 against
 * 8.3 us for the 16^3 z passes), and their float32 results then differ by
 * rounding.  The environment variable FZW_FFT_TUNE=0 keeps the defaults, and
 * fzw_set_fft_schedule fixes a choice: either makes results reproducible
 * bit for bit across processes.
 *   z, xy, pure: the chosen family per pass type (0 or 1);
 *   us6 (nullable): measured microseconds per launch, [z, xy, pure] x
 *     [four-step, alternative] (0 where a family does not exist for the size).
 * Returns FZW_E_STATE while no plan of that size has been created, FZW_E_ARG
 * for an unsupported size.  Never touches the GPU. */
fzw_status fzw_fft_schedule(int mesh_n, int* z, int* xy, int* pure, double* us6);
/* Set the schedule of a mesh size by hand (each 0 or 1 as above; the tuner
 * then leaves it alone).  Applies to later launches of every plan; a HIP
 * graph captured before keeps the kernels it was captured with.  The 96 mesh
 * has only the Stockham z passes and runs its pure x/y transforms through the
 * mixing kernel, whatever is set; its four-step mixing kernel, like the 512
 * one, transforms a line as decimated sub-lines (3 of 32, 2 of 256) joined by
 * one butterfly.  FZW_E_ARG for an unsupported size or a value other than 0
 * or 1. */
fzw_status fzw_set_fft_schedule(int mesh_n, int z, int xy, int pure);

/* Kernel classes for per-launch timing.  Every class but the CIC deposit is
 * one kernel (at meshes with the four-step kernels; the pure classes are one
 * kernel template with a forward and an inverse instance). */
enum {
  FZW_K_ZR2C = 0,        /* z-axis real-to-complex FFT pass */
  FZW_K_ZC2R = 1,        /* z-axis complex-to-real FFT pass */
  FZW_K_YMIX = 2,        /* strided y pass with spectral multipliers / mixing, one input */
  FZW_K_XMIX = 3,        /* strided x pass with spectral multipliers / mixing, one input */
  FZW_K_YPURE = 4,       /* pure y transforms (persistent kernel) */
  FZW_K_XPURE = 5,       /* pure x transforms (persistent kernel) */
  FZW_K_LPT_FWD = 6,     /* LPT pointwise step with its z transforms, forward */
  FZW_K_LPT_BWD = 7,     /* the same, adjoint */
  FZW_K_CIC_DEP = 8,     /* cloud-in-cell deposit (count, scan, scatter, gather) */
  FZW_K_CIC_ADJ = 9,     /* cloud-in-cell adjoint */
  FZW_K_VOXEL_FWD = 10,  /* per-voxel web memberships and bias */
  FZW_K_LIKE = 11,       /* negative-binomial likelihood pass */
  FZW_K_VOXEL_BWD = 12,  /* per-voxel adjoint of web, bias and likelihood */
  FZW_K_YMIX_MULTI = 13, /* strided y mixing pass with several inputs */
  FZW_K_XMIX_MULTI = 14, /* strided x mixing pass with several inputs */
  FZW_K_COUNT = 15
};
/* Turn per-launch timing on (1) or off (0): every later launch of the plan's
 * kernels (outside HIP graphs) is bracketed by HIP events on the plan's
 * stream.  Resets the records.  Synchronises the plan's stream. */
fzw_status fzw_timing_enable(fzw_plan* plan, int on);
/* Sum over the recorded launches of one kernel class: elapsed milliseconds,
 * number of launches and algorithmic bytes (each stage's distinct inputs and
 * outputs, counted once).  (host) outputs.  Synchronises the plan's stream. */
fzw_status fzw_timing_read(fzw_plan* plan, int klass, double* total_ms, long long* launches, double* bytes);

size_t fzw_chain_offset(const fzw_plan* plan, int chain);   /* voxel offset of chain c */
int fzw_n_regions(const fzw_plan* plan);
size_t fzw_workspace_bytes(const fzw_plan* plan);
const char* fzw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FZW_H_ */
